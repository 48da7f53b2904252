"""GPU parity of the full space charge of Eq. Poisson (holes, Boltzmann and
Fermi-Dirac statistics, incomplete dopant ionization, Sec. II.A.1-3) with
Ohmic contacts (Sec. II.A.4), through the C ABI, against the FP64 oracle on
the same seeded inputs.  Tolerances as in the other parity tests: kernel
outputs to 1e-12 of their scale, converged potentials to 1e-9 relative."""
import numpy as np
import pytest

import synth
from oracle import physics as ph
from oracle import solver
from paper_1403_7561_amd import qe
from tests import gpu_support as gs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CM3 = 1e-21


def dev_tensor(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def pn_block(ionization="complete", stat="mb", T=300.0, nd=1e18 * CM3, na=1e18 * CM3, comp=0.0):
    """Abrupt p-n junction between two Ohmic contacts on a ragged 9 x 10 x 61
    node block (compensation `comp` of the majority dopant added as the other
    species), contacts at the oracle's Ohmic potentials."""
    dev = synth.doped_block("pn", 9, 10, 61, (12.0, 14.0, 120.0),
                            lambda x, y, z: np.where(z > 60.0, nd, comp * na),
                            lambda x, y, z: np.where(z > 60.0, comp * nd, na),
                            [("p", "bottom"), ("n", "top")], stat=stat, T_K=T, holes=True,
                            ionization=ionization)
    st = ph.Statistics(stat, T, dev.m_eff, dev.Ec0_eV, holes=True, ionization=ionization)
    dev.dir_val[:] = [ph.ohmic_potential(st, comp * nd, na), ph.ohmic_potential(st, nd, comp * na)]
    return dev


CASES = {
    "stack_fd4K_incomplete": lambda: gs.full_charge_device("incomplete"),
    "stack_fd4K_complete": lambda: gs.full_charge_device("complete"),
    "pn_mb300K_complete": lambda: pn_block(),
    "pn_mb77K_incomplete_comp": lambda: pn_block("incomplete", "mb", 77.0, 2e17 * CM3, 1e17 * CM3, 0.1),
    "pn_fd300K_incomplete": lambda: pn_block("incomplete", "fd", 300.0, 1e19 * CM3, 1e18 * CM3),
}


def perturbed(po, res_phi, seed, amp=0.02):
    rng = np.random.default_rng(seed)
    return po.with_dirichlet(res_phi + amp * rng.standard_normal(po.mesh.N))


@pytest.fixture(scope="module")
def solved():
    cache = {}

    def get(case):
        if case not in cache:
            dev = CASES[case]()
            po, res = solver.solve(dev, atol=1e-10)
            assert res.status == "ok"
            cache[case] = (dev, po, res)
        return cache[case]
    return get


@pytest.mark.parametrize("case", sorted(CASES))
def test_residual_diag_and_jv(case, solved):
    dev, po, res = solved(case)
    phi = perturbed(po, res.phi, 3)
    P = qe.Problem(dev)
    F, d, n2 = qe.qe_residual(P, dev_tensor(phi))
    Fo, do = po.residual(phi), po.jacobi_diag(phi)
    print(case, "F", rel_max(F.cpu().numpy(), Fo), "diag", rel_max(d.cpu().numpy(), do))
    assert rel_max(F.cpu().numpy(), Fo) < 1e-12
    assert rel_max(d.cpu().numpy(), do) < 1e-12
    assert n2 == pytest.approx(float(Fo @ Fo), rel=1e-11)
    v = np.random.default_rng(4).standard_normal(po.mesh.N)
    y = qe.qe_jv(P, dev_tensor(phi), dev_tensor(v)).cpu().numpy()
    yo = po.jv(phi, v)
    print(case, "jv", rel_max(y, yo))
    assert rel_max(y, yo) < 1e-12
    y32 = qe.qe_jv(P, dev_tensor(phi), dev_tensor(v, torch.float32)).cpu().numpy()
    assert rel_max(y32, yo) < 2e-5


@pytest.mark.parametrize("case", sorted(CASES))
def test_solve_matches_oracle(case, solved):
    dev, po, res = solved(case)
    P = qe.Problem(dev)
    phi, n, rep = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-10))
    print(case, rep)
    phi = phi.cpu().numpy()
    err = rel_max(phi, res.phi)
    print(case, "phi rel err", err)
    assert rep["res_final"] <= 1e-10
    assert err < 1e-9
    n_o = po.nodal_density(res.phi)
    assert np.abs(n.cpu().numpy() - n_o).max() <= 1e-8 * max(n_o.max(), 1e-30)


def test_counts_and_adjoint_with_full_charge(solved):
    dev, po, res = solved("stack_fd4K_incomplete")
    P = qe.Problem(dev)
    boxes = [dev.boxes["D1"], dev.boxes["D2"]]
    c = qe.qe_count_electrons(P, dev_tensor(res.phi), boxes)
    co = np.array([po.count(res.phi, b) for b in boxes])
    print("counts", c, co)
    assert np.allclose(c, co, rtol=1e-12, atol=0) and co.min() > 1.0
    adj_o = solver.adjoint(po, res.phi, boxes[0])
    Q, dV, deps, lam, rep = qe.qe_adjoint(P, dev_tensor(res.phi), boxes[0], want_lam=True)
    assert Q == pytest.approx(adj_o.Q, rel=1e-12)
    assert np.allclose(dV, adj_o.dQ_ddir, rtol=1e-8, atol=1e-10 * np.abs(adj_o.dQ_ddir).max())
    assert rel_max(deps.cpu().numpy(), adj_o.dQ_deps) < 1e-8


def test_net_doping_from_species_when_absent(solved):
    # complete ionization with net_doping NULL takes donors - acceptors
    dev, po, res = solved("pn_mb300K_complete")
    P = qe.Problem(dev)
    P.net_doping = None
    phi, _, rep = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-10))
    assert rel_max(phi.cpu().numpy(), res.phi) < 1e-9


def test_mixed_precision_and_batch_with_full_charge(solved):
    dev, po, res = solved("stack_fd4K_incomplete")
    P = qe.Problem(dev)
    phi64, _, r64 = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-9))
    phi32, _, r32 = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-9, precision=1))
    print("fp64", r64, "\nmixed", r32)
    assert rel_max(phi32.cpu().numpy(), phi64.cpu().numpy()) < 1e-6
    # two instances (the device and a copy with other gate voltages) in one launch
    dev2 = gs.full_charge_device("incomplete", volts=(1.9, 2.2, 1.0, 1.2, 1.0))
    probs = [qe.Problem(dev), qe.Problem(dev2)]
    phis, counts, reps = qe.qe_solve_batch(probs, opts=qe.qe_default_options(newton_atol=1e-10),
                                           boxes=[dev.boxes["D1"]])
    print(reps)
    assert rel_max(phis[0].cpu().numpy(), res.phi) < 1e-9
    po2, res2 = solver.solve(dev2, atol=1e-10)
    assert rel_max(phis[1].cpu().numpy(), res2.phi) < 1e-9
    assert counts[1, 0] == pytest.approx(po2.count(res2.phi, dev.boxes["D1"]), rel=1e-8)


def test_uniform_block_at_ohmic_potential_is_flat():
    # the library's own Ohmic potential on a uniformly doped block makes the
    # solution flat at that value (neutral everywhere, no field)
    for ion in ("complete", "incomplete"):
        nd, na = 5e17 * CM3, 0.0
        dev = synth.doped_block("blk", 5, 6, 9, (20.0, 20.0, 40.0), lambda x, y, z: nd, lambda x, y, z: na,
                                [("bottom", "bottom")], stat="mb", T_K=77.0, holes=True, ionization=ion)
        P = qe.Problem(dev)
        vb = qe.qe_ohmic_potential(P.physics, nd, na)
        dev.dir_val[:] = vb
        P = qe.Problem(dev)
        phi, _, rep = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-12))
        assert np.abs(phi.cpu().numpy() - vb).max() < 1e-10, (ion, rep)


def test_full_size_stack_with_full_charge_sampled():
    """The 129 x 129 x 65 stack with holes, incomplete ionization of the boron
    substrate and the bottom contact at the library's Ohmic potential: the
    converged GPU potential leaves an oracle residual at the FP64 floor on
    sampled nodes, and sampled residual and J.v values at a perturbed
    potential match the oracle."""
    dev = synth.with_species(synth.config2(), ionization="incomplete")
    P = qe.Problem(dev)
    vb = qe.qe_ohmic_potential(P.physics, 0.0, float(dev.acceptors.max()))
    st = ph.Statistics("fd", 4.0, dev.m_eff, dev.Ec0_eV, holes=True, ionization="incomplete")
    assert vb == pytest.approx(ph.ohmic_potential(st, 0.0, float(dev.acceptors.max())), abs=1e-12)
    dev.dir_val[dev.contacts.index("bottom")] = vb
    P = qe.Problem(dev)
    phi, n, rep = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-8))
    print(rep)
    assert rep["status"] == 0 and rep["res_final"] <= 1e-8
    phn = phi.cpu().numpy()
    rng = np.random.default_rng(12)
    nodes = rng.choice(dev.n_nodes, 300, replace=False)
    assert np.abs(gs.sampled_residual(dev, phn, nodes)).max() < 1e-8
    pert = phn + 0.01 * rng.standard_normal(phn.size)
    pert[dev.dir_id >= 0] = dev.dir_val[dev.dir_id[dev.dir_id >= 0]]
    F, _, _ = qe.qe_residual(P, dev_tensor(pert))
    Fo = gs.sampled_residual(dev, pert, nodes)
    assert np.abs(F.cpu().numpy()[nodes] - Fo).max() <= 1e-12 * np.abs(Fo).max()
    v = rng.standard_normal(phn.size)
    y = qe.qe_jv(P, dev_tensor(pert), dev_tensor(v)).cpu().numpy()[nodes]
    yo = gs.sampled_jv(dev, pert, v, nodes)
    assert np.abs(y - yo).max() <= 1e-12 * np.abs(yo).max()
