"""Pins of the oracle's Schrodinger eigenproblem (Eqs. SchrodEqn,
SchrodEqnWeakForm and Schrodinger3D): exact discrete eigenvalues of linear
elements for the infinite well and the 3D box, isotropic and with a
diagonal mass tensor (tensor products of the closed-form 1D generalized
eigenvalues, scaled per axis), the harmonic oscillator, and the finite well with
equal and unequal masses against the BenDaniel-Duke transcendental
equations (the paper's 20 nm, 100 meV example)."""
import numpy as np
import pytest
from scipy import optimize

from oracle import schrodinger as sch
from oracle.physics import HBAR, M0, Q_E

HB2M = HBAR ** 2 / (2 * M0) / Q_E * 1e18     # eV nm^2, retyped from CODATA here


def column(z, h_xy=0.5):
    x = np.array([0.0, h_xy])
    return x, x.copy(), np.asarray(z, float)


def lam1d(k, n, h):
    """Generalized eigenvalue k of the 1D linear-element K v = lam M v on n
    uniform elements with both ends fixed (K = tridiag(-1, 2, -1)/h,
    M = h tridiag(1, 4, 1)/6): 6 (1 - cos t) / (h^2 (2 + cos t)), t = k pi / n."""
    t = k * np.pi / n
    return 6.0 * (1.0 - np.cos(t)) / (h * h * (2.0 + np.cos(t)))


def test_constant_of_the_kinetic_term():
    assert HB2M == pytest.approx(0.03809982, rel=1e-7)   # 3.81 eV A^2
    assert sch.HB2M == pytest.approx(HB2M, rel=1e-15)


def test_infinite_well_exact_discrete_levels():
    n, L, m = 40, 20.0, 0.19
    x, y, z = column(np.linspace(0.0, L, n + 1))
    N = 4 * (n + 1)
    fixed = np.zeros(N, bool)
    fixed[:4] = fixed[-4:] = True
    E, psi, (H, M) = sch.solve(x, y, z, np.full(n, 1.0 / m), np.zeros(n), np.zeros(N), fixed, 5)
    expect = HB2M / m * lam1d(np.arange(1, 6), n, L / n)
    assert np.allclose(E, expect, rtol=1e-12)
    # and the continuum levels hbar^2 pi^2 k^2 / (2 m L^2) to O(h^2): the
    # relative error of linear elements is (k pi h / L)^2 / 12 to leading order
    k = np.arange(1, 6)
    cont = HB2M / m * (np.pi * k / L) ** 2
    assert np.all(np.abs(E / cont - 1) < 0.1 * (k * np.pi / n) ** 2)
    # M-orthonormal eigenvectors with small residuals
    G = psi @ (M @ psi.T)
    assert np.allclose(G, np.eye(5), atol=1e-12)
    R = H @ psi.T - (M @ psi.T) * E
    assert np.abs(R[~fixed]).max() < 1e-10 * np.abs(E).max()


def test_three_dimensional_box_levels_are_sums():
    nx, ny, nz = 6, 5, 4
    Lx, Ly, Lz = 12.0, 8.0, 6.0
    x, y, z = np.linspace(0, Lx, nx + 1), np.linspace(0, Ly, ny + 1), np.linspace(0, Lz, nz + 1)
    Z, Y, X = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    fixed = ((X == 0) | (X == nx) | (Y == 0) | (Y == ny) | (Z == 0) | (Z == nz)).ravel()
    E_ = nx * ny * nz
    E, psi, _ = sch.solve(x, y, z, np.full(E_, 1.0), np.zeros(E_), np.zeros(fixed.size), fixed, 6)
    levels = sorted(HB2M * (lam1d(a, nx, Lx / nx) + lam1d(b, ny, Ly / ny) + lam1d(c, nz, Lz / nz))
                    for a in range(1, nx) for b in range(1, ny) for c in range(1, nz))
    assert np.allclose(E, levels[:6], rtol=1e-12)


@pytest.mark.parametrize("masses", [(0.19, 0.19, 0.98), (0.3, 0.5, 0.9)])
def test_anisotropic_box_levels_are_scaled_sums(masses):
    # a diagonal mass tensor (Eq. Schrodinger3D: m_t, m_t, m_l for the Si
    # Delta_2 valleys) separates too: every level is a sum of 1D discrete
    # levels, each scaled by its own axis's 1/m.  Unequal box lengths and
    # masses make any exchange of axes change the levels.
    nx, ny, nz = 6, 5, 4
    Lx, Ly, Lz = 12.0, 8.0, 6.0
    x, y, z = np.linspace(0, Lx, nx + 1), np.linspace(0, Ly, ny + 1), np.linspace(0, Lz, nz + 1)
    Z, Y, X = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    fixed = ((X == 0) | (X == nx) | (Y == 0) | (Y == ny) | (Z == 0) | (Z == nz)).ravel()
    E_ = nx * ny * nz
    mx, my, mz = masses
    im = np.stack([np.full(E_, 1.0 / mx), np.full(E_, 1.0 / my), np.full(E_, 1.0 / mz)])
    E, psi, _ = sch.solve(x, y, z, im, np.zeros(E_), np.zeros(fixed.size), fixed, 8)
    levels = sorted(HB2M * (lam1d(a, nx, Lx / nx) / mx + lam1d(b, ny, Ly / ny) / my + lam1d(c, nz, Lz / nz) / mz)
                    for a in range(1, nx) for b in range(1, ny) for c in range(1, nz))
    assert np.allclose(E, levels[:8], rtol=1e-12)


def test_anisotropic_column_levels_follow_the_axis_mass():
    # a column confined along z only sees m_l (the Sec. II.C 1D-confined
    # case): the z-well levels scale with 1/m_z and not with 1/m_x or 1/m_y
    n, L = 40, 20.0
    x, y, z = column(np.linspace(0.0, L, n + 1))
    N = 4 * (n + 1)
    fixed = np.zeros(N, bool)
    fixed[:4] = fixed[-4:] = True
    im = np.stack([np.full(n, 1.0 / 0.19), np.full(n, 1.0 / 0.19), np.full(n, 1.0 / 0.98)])
    E, _, _ = sch.solve(x, y, z, im, np.zeros(n), np.zeros(N), fixed, 4)
    assert np.allclose(E, HB2M / 0.98 * lam1d(np.arange(1, 5), n, L / n), rtol=1e-12)


def test_isotropic_masses_given_per_axis_or_once():
    nx, ny, nz = 5, 4, 3
    x, y, z = np.linspace(0, 5, nx + 1), np.linspace(0, 4, ny + 1), np.linspace(0, 3, nz + 1)
    Z, Y, X = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    fixed = ((X == 0) | (X == nx) | (Z == nz)).ravel()
    E_ = nx * ny * nz
    rng = np.random.default_rng(4)
    m = rng.uniform(1.0, 5.0, E_)
    v0 = rng.uniform(0.0, 0.3, E_)
    E1, _, _ = sch.solve(x, y, z, m, v0, np.zeros(fixed.size), fixed, 4)
    E3, _, _ = sch.solve(x, y, z, np.stack([m, m, m]), v0, np.zeros(fixed.size), fixed, 4)
    assert np.array_equal(E1, E3)
    with pytest.raises(ValueError, match="inv_mass"):
        sch.solve(x, y, z, np.stack([m, m]), v0, np.zeros(fixed.size), fixed, 4)


def test_harmonic_oscillator():
    # V = (1/2) m w^2 s^2 about the column centre, hbar w = 20 meV: E_n -> hbar w (n + 1/2)
    m, hw = 0.19, 0.02
    n, L = 1200, 60.0          # walls far beyond the classical turning points of n <= 5
    x, y, z = column(np.linspace(-L / 2, L / 2, n + 1))
    N = 4 * (n + 1)
    # (1/2) m w^2 s^2 in eV with s in nm: (hw)^2 s^2 / (4 HB2M / m)
    k = hw * hw / (4.0 * HB2M / m)
    phi = -k * np.repeat(z, 4) ** 2           # V = v0 - phi
    fixed = np.zeros(N, bool)
    fixed[:4] = fixed[-4:] = True
    E, _, _ = sch.solve(x, y, z, np.full(n, 1.0 / m), np.zeros(n), phi, fixed, 6)
    assert np.allclose(E, hw * (np.arange(6) + 0.5), rtol=2e-4)


def bdd_levels(a, V0, mw, mb, count):
    """Bound levels of a finite well of half-width a (BenDaniel-Duke matching:
    psi and psi'/m continuous): even k tan(ka)/mw = kappa/mb, odd
    -k cot(ka)/mw = kappa/mb, k = sqrt(mw E)/sqrt(HB2M), kappa likewise."""
    def f_even(E):
        k, q = np.sqrt(mw * E / HB2M), np.sqrt(mb * (V0 - E) / HB2M)
        return k * np.sin(k * a) / mw - q * np.cos(k * a) / mb

    def f_odd(E):
        k, q = np.sqrt(mw * E / HB2M), np.sqrt(mb * (V0 - E) / HB2M)
        return -k * np.cos(k * a) / mw - q * np.sin(k * a) / mb

    grid = np.linspace(1e-9, V0 * (1 - 1e-9), 20001)
    roots = []
    for f in (f_even, f_odd):
        v = f(grid)
        for i in np.nonzero(np.sign(v[:-1]) != np.sign(v[1:]))[0]:
            roots.append(optimize.brentq(f, grid[i], grid[i + 1], xtol=1e-15))
    return np.sort(roots)[:count]


@pytest.mark.parametrize("mw,mb", [(0.067, 0.067), (0.067, 1.0)])
def test_finite_well_against_bendaniel_duke(mw, mb):
    # the paper's example: 20 nm wide, 100 meV deep
    a, V0, Lb, n = 10.0, 0.1, 30.0, 1600
    z = np.linspace(-(a + Lb), a + Lb, n + 1)
    x, y, z = column(z)
    zc = 0.5 * (z[1:] + z[:-1])
    well = np.abs(zc) < a
    inv_mass = np.where(well, 1.0 / mw, 1.0 / mb)
    v0 = np.where(well, 0.0, V0)
    N = 4 * (n + 1)
    fixed = np.zeros(N, bool)
    fixed[:4] = fixed[-4:] = True
    expect = bdd_levels(a, V0, mw, mb, 3)
    E, _, _ = sch.solve(x, y, z, inv_mass, v0, np.zeros(N), fixed, len(expect))
    assert np.allclose(E, expect, rtol=2e-4)
