"""GPU parity of the interface-charge (Eq. NeuBC4fc) and Robin (charged gate)
face terms of Sec. II.A.4 through the C ABI, against the FP64 oracle on the
same seeded inputs: residual, diagonal and J.v at a perturbed potential,
solves, the adjoint's contact terms, mixed precision.  Sheets in all three
plane orientations, partial face ranges, sheets sharing nodes, and Robin
faces next to Dirichlet nodes are covered."""
import numpy as np
import pytest

import synth
from oracle import solver
from paper_1403_7561_amd import qe
from tests import gpu_support as gs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev_tensor(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


VOLTS = (2.2, 2.0, 1.0, 1.3, 0.9)


def interface_stack():
    return synth.with_interface_charge(gs.ragged_device(volts=VOLTS), 1e-3, seed=11, spread=0.5)


def robin_plungers():
    dev = gs.ragged_device(volts=(2.6, 2.4, 1.0, 1.3, 0.9))
    return synth.with_charged_gates(dev, synth.double_dot_gates()[:2], sigma_nm2=-2e-3)


def crossing_sheets():
    # the interface sheet plus a y-plane sheet and an x-plane sheet crossing
    # it (shared nodes on the intersection lines), partial face ranges
    dev = synth.with_interface_charge(gs.ragged_device(volts=VOLTS), -5e-4)
    rng = np.random.default_rng(13)
    sy = synth.Sheet(axis=1, plane=14, a0=3, a1=30, b0=5, b1=17, sigma=rng.uniform(-2e-3, 2e-3, 27 * 12))
    sx = synth.Sheet(axis=0, plane=20, a0=0, a1=28, b0=10, b1=16, sigma=rng.uniform(0, 1e-3, 28 * 6),
                     robin_d=6.0, robin_eps=11.7, phi0=0.2)
    dev.sheets = dev.sheets + [sy, sx]
    return dev


def robin_over_dirichlet():
    # a Robin sheet over the whole top plane, around and over the Dirichlet
    # barrier gates (their rows stay identity, the coupling enters the
    # adjoint's contact terms)
    dev = synth.with_charged_gates(gs.ragged_device(volts=(2.4, 2.2, 1.0, 1.3, 0.9)),
                                   synth.double_dot_gates()[:2])
    top = dev.nz - 1
    dev.sheets = dev.sheets + [synth.Sheet(axis=2, plane=top, a0=0, a1=dev.nx - 1, b0=0, b1=dev.ny - 1,
                                           robin_d=20.0, robin_eps=3.9, phi0=0.5)]
    return dev


def full_charge_with_sheets():
    dev = gs.full_charge_device("incomplete", volts=(2.4, 2.2, 1.1, 1.3, 0.9))
    dev = synth.with_interface_charge(dev, 5e-4)
    return synth.with_charged_gates(dev, synth.double_dot_gates()[1:2], sigma_nm2=1e-3)


CASES = {
    "interface": interface_stack,
    "robin_plungers": robin_plungers,
    "crossing": crossing_sheets,
    "robin_over_dirichlet": robin_over_dirichlet,
    "full_charge": full_charge_with_sheets,
}


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
    rng = np.random.default_rng(5)
    phi = po.with_dirichlet(res.phi + 0.02 * rng.standard_normal(po.mesh.N))
    P = qe.Problem(dev)
    F, d, n2 = qe.qe_residual(P, dev_tensor(phi))
    Fo, do = po.residual(phi), po.jacobi_diag(phi)
    print(case, "F", rel_max(F.cpu().numpy(), Fo), "diag", rel_max(d.cpu().numpy(), do))
    assert rel_max(F.cpu().numpy(), Fo) < 1e-12
    assert rel_max(d.cpu().numpy(), do) < 1e-12
    assert n2 == pytest.approx(float(Fo @ Fo), rel=1e-11)
    v = rng.standard_normal(po.mesh.N)
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
    err = rel_max(phi.cpu().numpy(), res.phi)
    print(case, "phi rel err", err)
    assert rep["res_final"] <= 1e-10 and err < 1e-9
    c = qe.qe_count_electrons(P, phi, [dev.boxes["D1"]])[0]
    assert c == pytest.approx(po.count(res.phi, dev.boxes["D1"]), rel=1e-7, abs=1e-12)


@pytest.mark.parametrize("case", ["robin_over_dirichlet", "crossing"])
def test_adjoint_with_sheets(case, solved):
    dev, po, res = solved(case)
    box = dev.boxes["D1"]
    adj_o = solver.adjoint(po, res.phi, box)
    P = qe.Problem(dev)
    Q, dV, deps, lam, rep = qe.qe_adjoint(P, dev_tensor(res.phi), box, want_lam=True)
    print(case, "Q", Q, adj_o.Q, "dV", dV, adj_o.dQ_ddir)
    assert Q == pytest.approx(adj_o.Q, rel=1e-12)
    assert rel_max(lam.cpu().numpy(), adj_o.lam) < 1e-8
    assert np.allclose(dV, adj_o.dQ_ddir, rtol=1e-8, atol=1e-10 * np.abs(adj_o.dQ_ddir).max())
    assert rel_max(deps.cpu().numpy(), adj_o.dQ_deps) < 1e-8


def test_mixed_precision_with_sheets(solved):
    dev, po, res = solved("crossing")
    P = qe.Problem(dev)
    phi64, _, r64 = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-9))
    phi32, _, r32 = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-9, precision=1))
    print("fp64", r64, "\nmixed", r32)
    assert r32["res_final"] <= 1e-9
    assert rel_max(phi32.cpu().numpy(), phi64.cpu().numpy()) < 1e-6


def test_sheet_sigma_validated_on_device():
    dev = interface_stack()
    dev.sheets[0].sigma = dev.sheets[0].sigma.copy()
    dev.sheets[0].sigma[7] = np.inf
    with pytest.raises(qe.QeError, match="sigma"):
        qe.qe_solve(qe.Problem(dev))


def test_batch_rejects_sheets():
    with pytest.raises(qe.QeError, match="sheets"):
        qe.qe_solve_batch([qe.Problem(interface_stack())], opts=qe.qe_default_options())


def test_full_size_stack_with_sheets():
    """The 129 x 129 x 65 stack with the interface charge and charged plungers
    (the benchmark's sheet workload): the oracle's assembled residual of the
    converged GPU potential is at the FP64 floor, and at a perturbed
    potential the GPU residual and J.v match the oracle's on every node."""
    dev = synth.with_interface_charge(synth.config2(), 1e-3, seed=7563, spread=0.5)
    dev = synth.with_charged_gates(dev, synth.double_dot_gates()[:2], sigma_nm2=-2e-3)
    P = qe.Problem(dev)
    phi, _, rep = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-8))
    print(rep)
    assert rep["status"] == 0 and rep["res_final"] <= 1e-8
    po = gs.oracle_problem(dev)
    ph = phi.cpu().numpy()
    assert np.linalg.norm(po.residual(ph)) < 2e-8
    rng = np.random.default_rng(21)
    pert = po.with_dirichlet(ph + 0.01 * rng.standard_normal(ph.size))
    F, _, _ = qe.qe_residual(P, dev_tensor(pert))
    assert rel_max(F.cpu().numpy(), po.residual(pert)) < 1e-12
    v = rng.standard_normal(ph.size)
    y = qe.qe_jv(P, dev_tensor(pert), dev_tensor(v)).cpu().numpy()
    assert rel_max(y, po.jv(pert, v)) < 1e-12
