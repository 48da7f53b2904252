"""Pins of the oracle's interface-charge (Eq. NeuBC4fc) and Robin face terms
(Sec. II.A.4) against closed forms: Q1 elements reproduce piecewise-linear
potentials exactly at the nodes, so charge-free slabs with a sheet charge or
a Robin condition must match the 1D electrostatics to rounding."""
import numpy as np
import pytest

import synth
from oracle import physics as ph
from oracle import solver

KAPPA = ph.KAPPA


def column(z, eps, dir_nodes, dir_vals, sheets, nxy=2, L=3.0):
    """A charge-free column (insulator) with nxy x nxy nodes per plane,
    per-element permittivity eps[k] along z, Dirichlet planes given by index."""
    xy = np.linspace(0.0, L, nxy)
    nx = ny = nxy
    nz = z.size
    E = (nx - 1) * (ny - 1) * (nz - 1)
    eps_e = np.repeat(np.asarray(eps, float), (nx - 1) * (ny - 1))
    dir_id = np.full(nx * ny * nz, -1, np.int32)
    for c, k in enumerate(dir_nodes):
        dir_id[k * nx * ny:(k + 1) * nx * ny] = c
    return synth.Device(name="col", x=xy, y=xy, z=np.asarray(z, float), eps_r=eps_e,
                        semi=np.zeros(E, np.uint8), net_doping=np.zeros(E), dir_id=dir_id,
                        dir_val=np.asarray(dir_vals, float), stat="linear", T_K=0.0, sheets=sheets)


@pytest.mark.parametrize("sigma", [0.0, 2e-3, -5e-3])
@pytest.mark.parametrize("nxy", [2, 4])
def test_robin_capacitor_closed_form(sigma, nxy):
    # slab [0, L] with phi(0) = 0 and, on top, a plane at phi0 a distance d
    # away through a layer of permittivity eps_g, with a sheet charge on the
    # top face: eps_s a = eps_g (phi0 - a L)/d + KAPPA sigma for phi = a z
    z = np.array([0.0, 1.5, 4.0, 4.5, 7.0, 10.0])
    L, eps_s, eps_g, d, phi0 = z[-1], 11.7, 3.9, 10.0, 0.8
    n = nxy - 1
    sh = synth.Sheet(axis=2, plane=z.size - 1, a0=0, a1=n, b0=0, b1=n, sigma=np.full(n * n, sigma),
                     robin_d=d, robin_eps=eps_g, phi0=phi0)
    dev = column(z, [eps_s] * (z.size - 1), [0], [0.0], [sh], nxy=nxy)
    prob, res = solver.solve(dev, atol=1e-13)
    a = (eps_g * phi0 / d + KAPPA * sigma) / (eps_s + eps_g * L / d)
    Z = np.repeat(z, nxy * nxy)
    assert np.abs(res.phi - a * Z).max() < 1e-12


@pytest.mark.parametrize("sigma", [1e-3, -3e-3])
def test_interface_sheet_between_two_dielectrics(sigma):
    # eps1 below z_i, eps2 above, phi(0) = 0, phi(L) = V, a sheet charge at
    # z_i: Gauss's law eps1 a - eps2 b = KAPPA sigma with slopes a below and
    # b above
    z = np.array([0.0, 2.0, 3.0, 5.0, 6.5, 9.0, 10.0])
    ki = 3
    eps1, eps2, V = 11.7, 3.9, 0.4
    eps = [eps1] * ki + [eps2] * (z.size - 1 - ki)
    sh = synth.Sheet(axis=2, plane=ki, a0=0, a1=2, b0=0, b1=2, sigma=np.full(4, sigma))
    dev = column(z, eps, [0, z.size - 1], [0.0, V], [sh], nxy=3)
    prob, res = solver.solve(dev, atol=1e-13)
    zi, L = z[ki], z[-1]
    # V = a zi + b (L - zi), eps1 a - eps2 b = KAPPA sigma
    A = np.array([[zi, L - zi], [eps1, -eps2]])
    a, b = np.linalg.solve(A, [V, KAPPA * sigma])
    expect = np.where(z <= zi, a * z, a * zi + b * (z - zi))
    assert np.abs(res.phi - np.repeat(expect, 9)).max() < 1e-12


def test_sheet_on_a_side_plane():
    # the same capacitor turned on its side: the sheet lies in an x-plane
    x = np.array([0.0, 2.0, 3.0, 6.0])
    yz = np.array([0.0, 1.0, 2.5])
    nx, ny, nz = 4, 3, 3
    E = 3 * 2 * 2
    dir_id = np.full(nx * ny * nz, -1, np.int32)
    dir_id[np.arange(nx * ny * nz) % nx == 0] = 0
    sh = synth.Sheet(axis=0, plane=nx - 1, a0=0, a1=2, b0=0, b1=2, sigma=np.full(4, 1e-3),
                     robin_d=5.0, robin_eps=3.9, phi0=-0.3)
    dev = synth.Device(name="side", x=x, y=yz, z=yz, eps_r=np.full(E, 7.0), semi=np.zeros(E, np.uint8),
                       net_doping=np.zeros(E), dir_id=dir_id, dir_val=np.zeros(1), stat="linear",
                       T_K=0.0, sheets=[sh])
    prob, res = solver.solve(dev, atol=1e-13)
    a = (3.9 * -0.3 / 5.0 + KAPPA * 1e-3) / (7.0 + 3.9 * x[-1] / 5.0)
    X = np.tile(x, ny * nz)
    assert np.abs(res.phi - a * X).max() < 1e-12


def test_robin_tends_to_dirichlet_as_d_vanishes():
    volts = np.array([1.6, 1.5, 0.5, 0.8, 0.4])
    base = synth.double_dot_device("rb", 11, 11, 9, volts, stat="tf", T_K=0.0)
    _, ref = solver.solve(base, atol=1e-11)
    errs = []
    for d in (1e-2, 1e-3, 1e-4):
        dev = synth.with_charged_gates(base, synth.double_dot_gates(), d_nm=d)
        _, res = solver.solve(dev, atol=1e-11)
        errs.append(np.abs(res.phi - ref.phi).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 2e-3
    assert errs[1] / errs[2] == pytest.approx(10.0, rel=0.2)     # first order in d


def stack_with_sheets():
    volts = np.array([2.3, 2.1, 0.9, 1.2, 0.8])
    dev = synth.double_dot_device("sh", 13, 11, 9, volts)
    dev = synth.with_interface_charge(dev, 1e-3, seed=5, spread=0.5)
    return synth.with_charged_gates(dev, synth.double_dot_gates()[:2], sigma_nm2=-2e-3)


def test_jacobian_with_sheets_matches_differences_and_is_symmetric():
    dev = stack_with_sheets()
    po, res = solver.solve(dev, atol=1e-10)
    assert res.status == "ok" and po.count(res.phi, dev.boxes["D1"]) > 0.1
    rng = np.random.default_rng(3)
    phi = po.with_dirichlet(res.phi + 0.01 * rng.standard_normal(po.mesh.N))
    v = np.where(po.free, rng.standard_normal(po.mesh.N), 0.0)
    h = 1e-6
    fd = (po.residual(phi + h * v) - po.residual(phi - h * v)) / (2 * h)
    jv = po.jv(phi, v)
    f = po.free
    assert np.abs(jv[f] - fd[f]).max() < 1e-6 * np.abs(jv[f]).max()
    J = po.jacobian_free(phi)
    assert abs(J - J.T).max() < 1e-12 * abs(J).max()


def test_solution_with_sheets_is_unique():
    dev = stack_with_sheets()
    po = solver.make_problem(dev)
    a = solver.newton(po, atol=1e-11).phi
    b = solver.newton(po, phi0=po.with_dirichlet(np.full(po.mesh.N, 0.9)), atol=1e-11).phi
    assert np.abs(a - b).max() < 1e-9
