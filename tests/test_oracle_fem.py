"""Pins of the reference discretisation, Newton solve, outputs and adjoint.

Each test checks the oracle against something other than itself: brute-force
quadrature of the element integrals, closed-form solutions (parallel plate,
bulk neutrality, 1D Thomas-Fermi profile), observed convergence order on a
manufactured solution, finite differences, Gauss's law and uniqueness."""
import numpy as np
import pytest

import synth
from oracle import fem, physics as ph, solver


# ---------------------------------------------------------------- helpers
def box_device(x, y, z, eps, semi, netdop, dir_id, dir_val, stat, T=0.0, Ec0=0.56):
    return synth.Device(name="t", x=np.asarray(x, float), y=np.asarray(y, float),
                        z=np.asarray(z, float), eps_r=np.asarray(eps, float),
                        semi=np.asarray(semi, np.uint8), net_doping=np.asarray(netdop, float),
                        dir_id=np.asarray(dir_id, np.int32), dir_val=np.asarray(dir_val, float),
                        stat=stat, T_K=T, Ec0_eV=Ec0)


def shape(a, xi, eta, zeta):
    """Trilinear shape function of local node a = ia + 2 ib + 4 ic on [0,1]^3."""
    ia, ib, ic = a & 1, (a >> 1) & 1, (a >> 2) & 1
    fx = xi if ia else 1 - xi
    fy = eta if ib else 1 - eta
    fz = zeta if ic else 1 - zeta
    return fx * fy * fz


def shape_grad(a, xi, eta, zeta, h):
    ia, ib, ic = a & 1, (a >> 1) & 1, (a >> 2) & 1
    fx, dx = (xi, 1.0) if ia else (1 - xi, -1.0)
    fy, dy = (eta, 1.0) if ib else (1 - eta, -1.0)
    fz, dz = (zeta, 1.0) if ic else (1 - zeta, -1.0)
    return np.array([dx * fy * fz / h[0], fx * dy * fz / h[1], fx * fy * dz / h[2]])


def gauss3():
    p = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)]) * 0.5 + 0.5
    w = np.array([5.0, 8.0, 5.0]) / 18.0
    return p, w


# ---------------------------------------------------------- element level
def test_element_integrals_brute_force():
    h = (1.3, 0.7, 2.1)
    mesh = fem.Mesh([0, h[0]], [0, h[1]], [0, h[2]])
    Khat = mesh.unit_stiffness()[0]
    p, w = gauss3()
    K = np.zeros((8, 8))
    M = np.zeros((8, 8))
    vol = h[0] * h[1] * h[2]
    for i in range(3):
        for j in range(3):
            for k in range(3):
                wt = w[i] * w[j] * w[k] * vol
                for a in range(8):
                    ga = shape_grad(a, p[i], p[j], p[k], h)
                    na = shape(a, p[i], p[j], p[k])
                    for b in range(8):
                        K[a, b] += wt * ga @ shape_grad(b, p[i], p[j], p[k], h)
                        M[a, b] += wt * na * shape(b, p[i], p[j], p[k])
    assert np.allclose(Khat, K, rtol=0, atol=1e-14 * np.abs(K).max())
    # 2x2x2 Gauss interpolation + weights reproduce the exact consistent mass
    Mq = mesh.W[0] * fem.INTERP.T @ fem.INTERP
    assert np.allclose(Mq, M, rtol=0, atol=1e-15 * np.abs(M).max())
    # Gauss points are where the interpolation matrix says
    g = fem.GAUSS_1D
    for q in range(8):
        pt = (g[q & 1], g[(q >> 1) & 1], g[(q >> 2) & 1])
        for a in range(8):
            assert fem.INTERP[q, a] == pytest.approx(shape(a, *pt), abs=1e-16)
    assert np.abs(Khat.sum(axis=1)).max() < 1e-15        # constants are in the kernel
    assert np.allclose(Khat, Khat.T, atol=0)


# ----------------------------------------------------------- closed forms
@pytest.mark.parametrize("nez", [8, 20, 64])
def test_parallel_plate(nez):
    """Full-top gate, grounded bottom, no charge: phi is linear in each layer
    and the interface sits at V * (90/11.7) / (10/3.9 + 90/11.7) = 0.75 V."""
    x = np.linspace(0, 200, 5)
    z = synth.stack_z(nez)
    dev = synth.make_stack_device("pp", x, x, z, [("G", (0, 200, 0, 200))], [1.0],
                                  stat="linear", T_K=0.0, net_doping_si=0.0)
    prob = solver.make_problem(dev)
    phi = solver.initial_guess(prob, method="direct")
    zz = np.repeat(z, 25)
    exact = np.where(zz <= 90.0, 0.75 * zz / 90.0, 0.75 + 0.25 * (zz - 90.0) / 10.0)
    assert np.abs(phi - exact).max() < 1e-13
    res = solver.newton(prob, atol=1e-9)      # floor ~ 1e-16 * |K| |phi| sqrt(N)
    assert res.status == "ok" and np.abs(res.phi - exact).max() < 1e-13


def _mms_problem(n, stat, T, Ec0, L=20.0):
    x = np.linspace(0.0, L, n + 1)
    mesh = fem.Mesh(x, x, x)
    N, E = mesh.N, mesh.E
    st = ph.Statistics(stat, T, 1.08, Ec0)
    k = np.pi / L

    def ex(X, Y, Z):
        return 0.3 + 0.2 * np.sin(k * X) * np.cos(0.5 * k * Y) + 0.1 * Z / L

    def lap(X, Y, Z):
        return -0.2 * (k ** 2 + 0.25 * k ** 2) * np.sin(k * X) * np.cos(0.5 * k * Y)

    eps, nd = 11.7, 2e-3

    def source(X, Y, Z):
        # -eps lap(phi) - KAPPA (N_net - n(phi)) = f
        return -eps * lap(X, Y, Z) - ph.KAPPA * (nd - st.density(ex(X, Y, Z)))

    # load vector by 3x3x3 Gauss per element (more accurate than the solver's rule)
    p, w = gauss3()
    load = np.zeros((E, 8))
    x0 = mesh.centroid - 0.5 * np.stack([mesh.hx, mesh.hy, mesh.hz], axis=1)
    for i in range(3):
        for j in range(3):
            for kk in range(3):
                X = x0[:, 0] + p[i] * mesh.hx
                Y = x0[:, 1] + p[j] * mesh.hy
                Z = x0[:, 2] + p[kk] * mesh.hz
                fv = source(X, Y, Z) * w[i] * w[j] * w[kk] * mesh.hx * mesh.hy * mesh.hz
                for a in range(8):
                    load[:, a] += fv * shape(a, p[i], p[j], p[kk])
    extra = mesh.scatter(load)
    Z3, Y3, X3 = np.meshgrid(x, x, x, indexing="ij")
    exact = ex(X3, Y3, Z3).ravel()
    bnd = ((X3 == 0) | (X3 == L) | (Y3 == 0) | (Y3 == L) | (Z3 == 0) | (Z3 == L)).ravel()
    dir_id = np.full(N, -1)
    dir_id[bnd] = np.arange(bnd.sum())
    dev = box_device(x, x, x, np.full(E, eps), np.ones(E), np.full(E, nd), dir_id,
                     exact[bnd], stat, T, Ec0)
    prob = fem.Problem(dev, st, extra_load=extra)
    return prob, exact


@pytest.mark.parametrize("stat,T,Ec0", [("tf", 0.0, 0.2), ("fd", 300.0, 0.3)])
def test_manufactured_solution_second_order(stat, T, Ec0):
    errs = []
    for n in (4, 8, 16):
        prob, exact = _mms_problem(n, stat, T, Ec0)
        res = solver.newton(prob, phi0=np.full(prob.mesh.N, 0.4), atol=1e-11)
        assert res.status == "ok"
        errs.append(np.abs(res.phi - exact).max())
    order = np.log2(errs[1] / errs[2])
    assert order > 1.9, errs


@pytest.mark.parametrize("stat,T", [("tf", 0.0), ("fd", 4.0)])
def test_bulk_neutrality(stat, T):
    """Uniform donors, no Dirichlet contact: phi is the neutral potential."""
    x = [0.0, 3.0, 7.0, 8.0, 12.5]
    y = [0.0, 1.0, 4.0, 6.0]
    z = [0.0, 2.5, 5.0]
    E = 4 * 3 * 2
    N = 5 * 4 * 3
    nd = 1e-3
    dev = box_device(x, y, z, np.full(E, 11.7), np.ones(E), np.full(E, nd),
                     np.full(N, -1), [], stat, T, 0.56)
    prob = solver.make_problem(dev)
    rng = np.random.default_rng(1)
    res = solver.newton(prob, phi0=0.6 + 0.05 * rng.random(N), atol=1e-13)
    assert res.status == "ok"
    if stat == "tf":
        ef = ph.HBAR ** 2 * (3 * np.pi ** 2 * nd * 1e27) ** (2 / 3) / (2 * 1.08 * ph.M0) / ph.Q_E
        target = 0.56 + ef
    else:
        target = prob.stats.neutral_potential(nd)
    assert np.abs(res.phi - target).max() < 1e-12


def test_thomas_fermi_column_profile():
    """eps u'' = KAPPA C_TF u^1.5 has u = u0 (1 + z/z0)^-4 with
    z0 = sqrt(20 eps / (KAPPA C_TF)) u0^-1/4; observed order two."""
    eps, u0, Lz = 11.7, 0.2, 20.0
    ctf = ph.thomas_fermi_coeff(1.08)
    z0 = np.sqrt(20.0 * eps / (ph.KAPPA * ctf)) * u0 ** -0.25
    assert z0 == pytest.approx(2.382, abs=1e-3)
    exact_f = lambda zz: u0 * (1.0 + zz / z0) ** -4
    errs = []
    for nz in (41, 81, 161):
        z = np.linspace(0.0, Lz, nz)
        x = [0.0, 1.0]
        E = nz - 1
        dir_id = np.full(4 * nz, -1)
        dir_id[:4] = 0
        dir_id[-4:] = 1
        dev = box_device(x, x, z, np.full(E, eps), np.ones(E), np.zeros(E), dir_id,
                         [u0, exact_f(Lz)], "tf", 0.0, 0.0)
        prob = solver.make_problem(dev)
        res = solver.newton(prob, atol=1e-12, method="direct")
        assert res.status == "ok"
        errs.append(np.abs(res.phi - exact_f(np.repeat(z, 4))).max())
    assert np.log2(errs[0] / errs[1]) > 1.9 and np.log2(errs[1] / errs[2]) > 1.9, errs


# ------------------------------------------------------ Jacobian and solve
@pytest.fixture(scope="module")
def c1_smooth():
    dev = synth.config1()
    dev.stat, dev.T_K = "fd", 300.0       # smooth statistics for difference checks
    prob = solver.make_problem(dev)
    rng = np.random.default_rng(5)
    phi = solver.initial_guess(prob) + 0.05 * rng.standard_normal(prob.mesh.N)
    return prob, prob.with_dirichlet(phi)


def test_jv_matches_residual_difference(c1_smooth):
    prob, phi = c1_smooth
    rng = np.random.default_rng(6)
    v = np.where(prob.free, rng.standard_normal(prob.mesh.N), 0.0)
    h = 1e-6
    fd = (prob.residual(phi + h * v) - prob.residual(phi - h * v)) / (2 * h)
    jv = prob.jv(phi, v)
    f = prob.free
    assert np.linalg.norm(jv[f] - fd[f]) / np.linalg.norm(jv[f]) < 1e-7
    # Dirichlet rows are identity rows of the masked operator
    w = rng.standard_normal(prob.mesh.N)
    assert np.array_equal(prob.jv(phi, w)[~f], w[~f])


def test_jacobian_symmetric_and_diag(c1_smooth):
    prob, phi = c1_smooth
    rng = np.random.default_rng(7)
    f = prob.free
    v = np.where(f, rng.standard_normal(prob.mesh.N), 0.0)
    w = np.where(f, rng.standard_normal(prob.mesh.N), 0.0)
    a, b = v @ prob.jv(phi, w), w @ prob.jv(phi, v)
    assert abs(a - b) <= 1e-13 * abs(a)
    d = prob.jacobi_diag(phi)
    for i in rng.choice(np.nonzero(f)[0], 25, replace=False):
        e = np.zeros(prob.mesh.N)
        e[i] = 1.0
        h = 1e-6
        fd = (prob.residual(phi + h * e)[i] - prob.residual(phi - h * e)[i]) / (2 * h)
        assert d[i] == pytest.approx(fd, rel=1e-7)
    assert np.all(d[~f] == 1.0)


@pytest.fixture(scope="module")
def c1_solution():
    dev = synth.config1()
    prob, res = solver.solve(dev, atol=1e-10)
    assert res.status == "ok"
    return dev, prob, res


def test_uniqueness_from_three_guesses():
    dev = synth.double_dot_device("u", 13, 13, 9, [1.2, 0.9, 0.3, 0.5, 0.2])
    prob = solver.make_problem(dev)
    rng = np.random.default_rng(9)
    sols = []
    for guess in (None, np.zeros(prob.mesh.N), rng.uniform(0.0, 1.0, prob.mesh.N)):
        res = solver.newton(prob, phi0=guess, atol=1e-10)
        assert res.status == "ok"
        sols.append(res.phi)
    scale = np.abs(sols[0]).max()
    assert np.abs(sols[1] - sols[0]).max() / scale < 1e-11
    assert np.abs(sols[2] - sols[0]).max() / scale < 1e-11


def test_gauss_law_and_counts(c1_solution):
    """Rows of K sum to zero, so at F_free = 0 the flux leaving through the
    Dirichlet contacts balances the total charge, which must equal what the
    region count integrates."""
    dev, prob, res = c1_solution
    m = prob.mesh
    Ffull = prob.residual_full(res.phi)
    flux = Ffull[prob.dirichlet].sum()
    everything = (m.x[0], m.x[-1], m.y[0], m.y[-1], m.z[0], m.z[-1])
    n_tot = prob.count(res.phi, everything)
    dop = np.sum(prob.semi * prob.netdop * 8.0 * m.W)
    assert flux == pytest.approx(-ph.KAPPA * (dop - n_tot), rel=1e-9)
    assert n_tot > 1.0
    assert prob.count(res.phi, (-5, -1, 0, 200, 0, 100)) == 0.0
    d1 = prob.count(res.phi, dev.boxes["D1"])
    assert 0.0 < d1 < n_tot


def test_nodal_density(c1_solution):
    dev, prob, res = c1_solution
    n = prob.nodal_density(res.phi)
    top = np.arange(prob.mesh.N) >= prob.mesh.N - 17 * 17     # oxide-only node plane
    assert not np.any(n[top])
    assert np.all(n >= 0) and n.max() > 0


def test_adjoint_matches_finite_differences():
    volts = np.array([1.6, 1.5, 0.5, 0.8, 0.4])
    dev = synth.double_dot_device("a", 17, 17, 11, volts)
    box = dev.boxes["D1"]
    prob, res = solver.solve(dev, atol=1e-11)
    assert res.status == "ok"
    adj = solver.adjoint(prob, res.phi, box)
    assert adj.Q == pytest.approx(prob.count(res.phi, box), rel=1e-14)

    def count_with(dv=None, deps=None):
        d2 = synth.double_dot_device("a", 17, 17, 11, volts)
        if dv is not None:
            d2.dir_val = d2.dir_val + dv
        if deps is not None:
            d2.eps_r = d2.eps_r + deps
        p2, r2 = solver.solve(d2, atol=1e-11, phi0=res.phi)
        assert r2.status == "ok"
        return p2.count(r2.phi, box)

    h = 1e-4
    for g in range(5):
        e = np.zeros(dev.dir_val.size)
        e[g] = h
        fd = (count_with(dv=e) - count_with(dv=-e)) / (2 * h)
        assert adj.dQ_ddir[g] == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(adj.Q))
    # capacitance with the paper's dV = 0.01 V agrees to O(dV^2)
    e = np.zeros(dev.dir_val.size)
    e[0] = 0.01
    fd1 = (count_with(dv=e) - count_with(dv=-e)) / 0.02
    assert adj.dQ_ddir[0] == pytest.approx(fd1, rel=1e-3)
    rng = np.random.default_rng(3)
    elems = rng.choice(prob.mesh.E, 6, replace=False)
    elems[0] = int(np.argmax(np.abs(adj.dQ_deps)))
    for el in elems:
        de = np.zeros(prob.mesh.E)
        de[el] = 1e-4 * dev.eps_r[el]
        fd = (count_with(deps=de) - count_with(deps=-de)) / (2 * de[el])
        assert adj.dQ_deps[el] == pytest.approx(fd, rel=1e-4, abs=1e-7 * np.abs(adj.dQ_deps).max())
    # a random-direction directional derivative in eps
    dirv = rng.standard_normal(prob.mesh.E) * 1e-4 * dev.eps_r
    fd = (count_with(deps=dirv) - count_with(deps=-dirv)) / 2.0
    assert adj.dQ_deps @ dirv == pytest.approx(fd, rel=1e-5)
