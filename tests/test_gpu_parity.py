"""GPU parity: every entry point of the HIP library, called through the C ABI,
against the FP64 CPU oracle on the same seeded inputs.

Tolerances (FP64 paths): kernel outputs agree to 1e-12 of their own scale
(only the summation order differs); converged potentials agree to 1e-9
relative (max|dphi| / max|phi|), the bound the solve is specified to; the
mixed-precision solve agrees with the FP64 GPU solve to 1e-6."""
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


CASES = {
    "c1_tf": lambda: synth.config1(),
    "ragged_fd": lambda: gs.ragged_device(),
    "ragged_tf": lambda: gs.ragged_device(stat="tf", T=0.0),
}


def perturbed_phi(prob_o, seed=0, amp=0.05):
    rng = np.random.default_rng(seed)
    phi = solver.initial_guess(prob_o) + amp * rng.standard_normal(prob_o.mesh.N)
    return prob_o.with_dirichlet(phi)


@pytest.mark.parametrize("case", sorted(CASES))
def test_residual_and_diag(case):
    dev = CASES[case]()
    po = gs.oracle_problem(dev)
    phi = perturbed_phi(po)
    P = qe.Problem(dev)
    F, d, n2 = qe.qe_residual(P, dev_tensor(phi))
    F = F.cpu().numpy()
    d = d.cpu().numpy()
    Fo = po.residual(phi)
    do = po.jacobi_diag(phi)
    print(case, "F", rel_max(F, Fo), "diag", rel_max(d, do))
    assert rel_max(F, Fo) < 1e-12
    assert rel_max(d, do) < 1e-12
    assert n2 == pytest.approx(float(Fo @ Fo), rel=1e-11)
    assert np.all(F[po.dirichlet] == 0.0) and np.all(d[po.dirichlet] == 1.0)


@pytest.mark.parametrize("case", sorted(CASES))
def test_jacobian_vector_product(case):
    dev = CASES[case]()
    po = gs.oracle_problem(dev)
    phi = perturbed_phi(po, seed=1)
    v = np.random.default_rng(2).standard_normal(po.mesh.N)
    P = qe.Problem(dev)
    y = qe.qe_jv(P, dev_tensor(phi), dev_tensor(v)).cpu().numpy()
    yo = po.jv(phi, v)
    print(case, "jv64", rel_max(y, yo))
    assert rel_max(y, yo) < 1e-12
    y32 = qe.qe_jv(P, dev_tensor(phi), dev_tensor(v, torch.float32)).cpu().numpy()
    print(case, "jv32", rel_max(y32, yo))
    assert rel_max(y32, yo) < 2e-5


@pytest.mark.parametrize("case", sorted(CASES))
def test_zero_coefficient_elements_skipped_exactly(case):
    """The J.v reads the Gauss-point coefficients only of elements where they
    are not all exactly zero (depleted silicon, insulators).  The element count
    it reports matches the oracle's coefficients at the same potential, and
    the product at a converged (mostly depleted) potential still matches the
    oracle's assembled Jacobian."""
    dev = CASES[case]()
    po = gs.oracle_problem(dev)
    P = qe.Problem(dev)
    phis = [perturbed_phi(po, seed=4), solver.solve(dev, atol=1e-10)[1].phi]
    v = np.random.default_rng(5).standard_normal(po.mesh.N)
    for phi in phis:
        _, ncoef = qe.qe_time_jv(P, dev_tensor(phi), dev_tensor(v), "fp64", reps=2)
        c = np.asarray(po.coeff(phi)).reshape(po.mesh.E, 8)
        nz_o = int(np.count_nonzero(np.any(c != 0.0, axis=1)))
        print(case, "coef elements gpu", ncoef, "oracle", nz_o, "of", po.mesh.E)
        # FP64 on both sides; only an element whose coefficients sit at the
        # underflow edge of exp could be decided differently
        assert abs(ncoef - nz_o) <= max(2, nz_o // 1000)
        y = qe.qe_jv(P, dev_tensor(phi), dev_tensor(v)).cpu().numpy()
        assert rel_max(y, po.jv(phi, v)) < 1e-12


def solve_gpu(dev, **opt):
    P = qe.Problem(dev)
    o = qe.qe_default_options(**opt)
    phi, n, rep = qe.qe_solve(P, opts=o)
    return P, phi, n, rep


@pytest.mark.parametrize("case,atol", [("c1_tf", 1e-10), ("ragged_fd", 1e-10), ("ragged_tf", 1e-10)])
def test_solve_matches_oracle(case, atol):
    dev = CASES[case]()
    po, res = solver.solve(dev, atol=atol)
    assert res.status == "ok"
    P, phi, n, rep = solve_gpu(dev, newton_atol=atol)
    print(case, rep)
    phi = phi.cpu().numpy()
    assert rep["res_final"] <= atol
    err = rel_max(phi, res.phi)
    print(case, "phi rel err", err)
    assert err < 1e-9
    n_o = po.nodal_density(res.phi)
    assert np.abs(n.cpu().numpy() - n_o).max() <= 1e-8 * max(n_o.max(), 1e-30)
    boxes = [dev.boxes["D1"], dev.boxes["D2"], (0, 200, 0, 200, 0, 100)]
    c = qe.qe_count_electrons(P, dev_tensor(phi), boxes)
    co = np.array([po.count(res.phi, b) for b in boxes])
    print(case, "counts", c, co)
    assert np.allclose(c, co, rtol=1e-8, atol=1e-12 * co.max())


def test_density_and_counts_at_oracle_phi():
    dev = gs.ragged_device()
    po, res = solver.solve(dev, atol=1e-10)
    P = qe.Problem(dev)
    ph = dev_tensor(res.phi)
    n = qe.qe_density(P, ph).cpu().numpy()
    n_o = po.nodal_density(res.phi)
    assert np.abs(n - n_o).max() <= 1e-13 * n_o.max()
    boxes = [dev.boxes["D1"], dev.boxes["D2"], (0, 200, 0, 200, 0, 100), (-9, -1, 0, 1, 0, 1)]
    c = qe.qe_count_electrons(P, ph, boxes)
    co = np.array([po.count(res.phi, b) for b in boxes])
    assert c[3] == 0.0
    assert np.allclose(c, co, rtol=1e-12, atol=0)


def test_mixed_precision_matches_fp64():
    dev = gs.ragged_device()
    _, phi64, _, r64 = solve_gpu(dev, newton_atol=1e-9)
    _, phi32, _, r32 = solve_gpu(dev, newton_atol=1e-9, precision=1)
    print("fp64", r64, "\nmixed", r32)
    err = rel_max(phi32.cpu().numpy(), phi64.cpu().numpy())
    print("mixed vs fp64", err)
    assert r32["res_final"] <= 1e-9
    assert err < 1e-6


def test_adjoint_matches_oracle_and_differences():
    """dQ/dV, dQ/deps and lam against the oracle's adjoint to 1e-10 (both at
    the oracle's converged potential), and central differences of the GPU
    solve on two gates."""
    volts = np.array([1.6, 1.5, 0.5, 0.8, 0.4])
    dev = synth.double_dot_device("adj", 17, 17, 11, volts)
    box = dev.boxes["D1"]
    po, res = solver.solve(dev, atol=1e-11)
    adj_o = solver.adjoint(po, res.phi, box)
    P = qe.Problem(dev)
    Q, dV, deps, lam, rep = qe.qe_adjoint(P, dev_tensor(res.phi), box, want_lam=True)
    print("Q", Q, adj_o.Q, "dV", dV, adj_o.dQ_ddir, rep)
    de = deps.cpu().numpy()
    print("rel dV", rel_max(dV, adj_o.dQ_ddir), "deps", rel_max(de, adj_o.dQ_deps), "lam",
          rel_max(lam.cpu().numpy(), adj_o.lam))
    assert Q == pytest.approx(adj_o.Q, rel=1e-12)
    assert rel_max(dV, adj_o.dQ_ddir) < 1e-10
    assert rel_max(de, adj_o.dQ_deps) < 1e-10
    assert rel_max(lam.cpu().numpy(), adj_o.lam) < 1e-10
    # central differences of the GPU solve (h = 1e-4 V) on two gates
    opts = qe.qe_default_options(newton_atol=1e-11)
    for g in (0, 3):
        vals = []
        for s in (+1, -1):
            d2 = synth.double_dot_device("adj", 17, 17, 11, volts)
            d2.dir_val = d2.dir_val.copy()
            d2.dir_val[g] += s * 1e-4
            P2 = qe.Problem(d2)
            phi2, _, _ = qe.qe_solve(P2, opts=opts)
            vals.append(qe.qe_count_electrons(P2, phi2, [box])[0])
        fd = (vals[0] - vals[1]) / 2e-4
        assert dV[g] == pytest.approx(fd, rel=1e-5)


def test_bulk_neutrality_without_contacts():
    x = np.array([0.0, 3.0, 7.0, 8.0, 12.5])
    dev = synth.Device(name="bulk", x=x, y=x[:4], z=x[:3], eps_r=np.full(24, 11.7),
                       semi=np.ones(24, np.uint8), net_doping=np.full(24, 1e-3),
                       dir_id=np.full(60, -1, np.int32), dir_val=np.zeros(0), stat="fd", T_K=4.0)
    po = gs.oracle_problem(dev)
    target = po.stats.neutral_potential(1e-3)
    P = qe.Problem(dev)
    phi0 = dev_tensor(0.6 + 0.05 * np.random.default_rng(1).random(60))
    phi, _, rep = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-12, init_guess=1), phi=phi0)
    assert np.abs(phi.cpu().numpy() - target).max() < 1e-12


def test_bitwise_reproducible():
    dev = gs.ragged_device()
    _, a, _, ra = solve_gpu(dev, newton_atol=1e-10)
    _, b, _, rb = solve_gpu(dev, newton_atol=1e-10)
    assert torch.equal(a, b) and ra == rb


def test_minimal_and_degenerate_meshes():
    # one element; every node Dirichlet except none free -> F = 0 at once
    x = np.array([0.0, 1.0])
    dev = synth.Device(name="one", x=x, y=x, z=x, eps_r=np.array([11.7]), semi=np.array([1], np.uint8),
                       net_doping=np.array([0.0]), dir_id=np.zeros(8, np.int32), dir_val=np.array([0.3]),
                       stat="tf", T_K=0.0)
    P = qe.Problem(dev)
    phi, n, rep = qe.qe_solve(P)
    assert np.allclose(phi.cpu().numpy(), 0.3) and rep["newton_iters"] == 0
    # thin meshes: one element across x and y, many in z (Thomas-Fermi column)
    z = np.linspace(0, 20, 41)
    dir_id = np.full(4 * 41, -1, np.int32)
    dir_id[:4] = 0
    dev = synth.Device(name="col", x=x, y=x, z=z, eps_r=np.full(40, 11.7), semi=np.ones(40, np.uint8),
                       net_doping=np.zeros(40), dir_id=dir_id, dir_val=np.array([0.2]), stat="tf",
                       T_K=0.0, Ec0_eV=0.0)
    po, res = solver.solve(dev, atol=1e-12)
    P = qe.Problem(dev)
    phi, _, rep = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-12))
    assert rel_max(phi.cpu().numpy(), res.phi) < 1e-10


def test_device_side_validation():
    dev = synth.config1()
    dev.eps_r = dev.eps_r.copy()
    dev.eps_r[100] = -1.0
    with pytest.raises(qe.QeError, match="eps_r"):
        qe.qe_solve(qe.Problem(dev))
    dev = synth.config1()
    dev.dir_id = dev.dir_id.copy()
    dev.dir_id[5] = 7
    with pytest.raises(qe.QeError, match="dir_id"):
        qe.qe_solve(qe.Problem(dev))
    dev = synth.config1()
    dev.net_doping = dev.net_doping.copy()
    dev.net_doping[3] = np.nan
    with pytest.raises(qe.QeError, match="NONFINITE"):
        qe.qe_solve(qe.Problem(dev))
    # mesh coordinates and Dirichlet values, checked on the device as well
    dev = synth.config1()
    dev.x = dev.x.copy()
    dev.x[4] = dev.x[3]
    with pytest.raises(qe.QeError, match="coordinates x"):
        qe.qe_solve(qe.Problem(dev))
    dev = synth.config1()
    dev.z = dev.z.copy()
    dev.z[-1] = np.inf
    with pytest.raises(qe.QeError, match="coordinates z"):
        qe.qe_solve(qe.Problem(dev))
    dev = synth.config1()
    dev.dir_val = np.array(dev.dir_val, dtype=np.float64)
    dev.dir_val[0] = np.nan
    with pytest.raises(qe.QeError, match="dir_val"):
        qe.qe_solve(qe.Problem(dev))


def test_newton_status_codes():
    dev = synth.config1()
    P = qe.Problem(dev)
    phi, _, rep = qe.qe_solve(P, opts=qe.qe_default_options(newton_maxit=2, newton_atol=1e-10), check=False)
    assert rep["status"] == -4 and rep["newton_iters"] == 2
    # an unreachable tolerance below the FP64 floor ends in a line-search failure
    phi, _, rep = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-30, ls_max_halvings=3), check=False)
    assert rep["status"] == -5 and rep["res_final"] < 1e-9


def test_full_size_double_dot_sampled():
    """129 x 129 x 65 five-gate stack at 4 K: the converged GPU potential leaves
    an oracle residual at the FP64 floor on sampled nodes, and sampled J.v and
    residual values at a perturbed potential match the oracle."""
    dev = synth.config2()
    P = qe.Problem(dev)
    phi, n, rep = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-8))
    print(rep)
    assert rep["status"] == 0 and rep["res_final"] <= 1e-8
    ph = phi.cpu().numpy()
    rng = np.random.default_rng(11)
    nodes = rng.choice(dev.n_nodes, 400, replace=False)
    Fs = gs.sampled_residual(dev, ph, nodes)
    assert np.abs(Fs).max() < 1e-8
    pert = ph + 0.01 * rng.standard_normal(ph.size)
    pert[dev.dir_id >= 0] = dev.dir_val[dev.dir_id[dev.dir_id >= 0]]
    F, _, _ = qe.qe_residual(P, dev_tensor(pert))
    Fo = gs.sampled_residual(dev, pert, nodes)
    Fg = F.cpu().numpy()[nodes]
    assert np.abs(Fg - Fo).max() <= 1e-12 * np.abs(Fo).max()
    v = rng.standard_normal(ph.size)
    y = qe.qe_jv(P, dev_tensor(pert), dev_tensor(v)).cpu().numpy()[nodes]
    yo = gs.sampled_jv(dev, pert, v, nodes)
    assert np.abs(y - yo).max() <= 1e-12 * np.abs(yo).max()


@pytest.mark.parametrize("stat,delta,ratio", [("linear", 1e-6, 1e-6), ("fd", 1e-8, 1e-3)])
def test_cg_product_is_the_exact_jacobian(stat, delta, ratio):
    """The CG's own J.v (the loop's sweep, not the qe_jv product) must be the
    exact Jacobian of the residual.  From a start delta off the solution one
    Newton step with a CG solved to 1e-10 multiplies ||F|| by about the
    relative error of the Jacobian used, plus, for Fermi-Dirac electrons,
    the quadratic term (delta / kT ~ 3e-5 here), so ||F_1|| / ||F_0|| <
    ratio bounds that error.  The linear statistics make the residual affine
    in phi (stiffness only); the FD case has Gauss-point coefficients on the
    inversion layers, so it covers the sweep's coefficient path too."""
    dev = gs.ragged_device(stat=stat)
    po, res = solver.solve(dev, atol=1e-11)
    P = qe.Problem(dev)
    rng = np.random.default_rng(5)
    free = dev.dir_id < 0
    phi0 = res.phi.copy()
    phi0[free] += delta * rng.standard_normal(int(free.sum()))
    f0 = float(np.linalg.norm(po.residual(phi0)))
    # one Newton step, an atol it cannot reach (so the CG tolerance is 1e-10)
    opts = qe.qe_default_options(newton_atol=1e-30, newton_maxit=1, krylov_rtol_max=1e-10, init_guess=1)
    phi, _, rep = qe.qe_solve(P, opts=opts, phi=dev_tensor(phi0), check=False)
    print(stat, "||F0||", f0, rep)
    assert rep["newton_iters"] == 1 and rep["ls_halvings"] == 0
    assert rep["res0"] == pytest.approx(f0, rel=1e-6)
    assert rep["res_final"] < ratio * rep["res0"]
    assert rel_max(phi.cpu().numpy(), res.phi) < delta


@pytest.mark.parametrize("k", [1, 2, 7, 25])
def test_cg_iterate_at_the_iteration_limit(k):
    """A Newton step whose CG stops at its iteration limit k takes the k-th
    Jacobi-PCG iterate from x = 0, the last update included (the FP64 loop
    leaves that update to a kernel queued after it): the oracle's Jacobian
    and a library CG run for exactly k iterations give the same vector."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    dev = gs.ragged_device(stat="fd")
    po, res = solver.solve(dev, atol=1e-11)
    rng = np.random.default_rng(11)
    free = po.free
    phi0 = res.phi.copy()
    phi0[free] += 1e-3 * rng.standard_normal(int(free.sum()))
    J = po.jacobian_free(phi0)
    b = -po.residual(phi0)[free]
    xo, info = spla.cg(J, b, rtol=0.0, atol=0.0, maxiter=k, M=sp.diags(1.0 / J.diagonal()))
    assert info == k
    P = qe.Problem(dev)
    opts = qe.qe_default_options(newton_atol=1e-30, newton_maxit=1, krylov_rtol_max=1e-12, krylov_maxit=k,
                                 init_guess=1)
    phi, _, rep = qe.qe_solve(P, opts=opts, phi=dev_tensor(phi0), check=False)
    print(k, rep)
    assert rep["newton_iters"] == 1 and rep["krylov_iters"] == k
    x = (phi.cpu().numpy() - phi0)[free] / 0.5 ** rep["ls_halvings"]
    print(k, "rel diff", rel_max(x, xo))
    assert rel_max(x, xo) < 1e-10
