"""Carrier statistics (Sec. II.A.1) in plain FP64 NumPy.

Units: potential V, energy eV, length nm, density nm^-3.  With the substrate
grounded the Fermi level is E_F = 0 (Sec. II.A.2, constant Fermi level), the
gate metal work function equals q*phi_ref (so a gate node carries its applied
voltage, Eq. ContOnIns) and the conduction-band edge is
E_C(phi) = Ec0 - phi, i.e. E_F - E_C = phi - Ec0 (Eq. EcEv_phi with the
constant offset folded into Ec0).
"""
from __future__ import annotations

import numpy as np
from scipy import integrate, optimize, special

# CODATA 2018 (SI; q, hbar, k_B exact by definition).
Q_E = 1.602176634e-19          # C
EPS0 = 8.8541878128e-12        # F/m
HBAR = 1.054571817e-34         # J s
M0 = 9.1093837015e-31          # kg
K_B = 1.380649e-23             # J/K

# Poisson divided by eps0 in nm/V units: -div(eps_r grad phi) = KAPPA * rho[nm^-3]
KAPPA = Q_E / EPS0 * 1e9       # V nm

FD_SWITCH = -50.0              # below this F_1/2(x) is replaced by exp(x)
_A_BED = 0.75 * np.sqrt(np.pi)  # 3 sqrt(pi)/4 in Eq. FDIntApprox


def kT_eV(T_K):
    """Thermal energy k_B T in eV."""
    return K_B * T_K / Q_E


def effective_dos(T_K, m_eff):
    """Eq. EffectiveDOS: N_C = 2 (m* k_B T / (2 pi hbar^2))^(3/2), in nm^-3."""
    m = m_eff * M0
    return 2.0 * (m * K_B * T_K / (2.0 * np.pi * HBAR ** 2)) ** 1.5 * 1e-27


def dos_mass(m_l, m_t):
    """Eq. EffectiveMass: conduction DOS mass over six valleys."""
    return 6.0 ** (2.0 / 3.0) * (m_l * m_t * m_t) ** (1.0 / 3.0)


def thomas_fermi_coeff(m_eff):
    """Zero-temperature density prefactor: n = C (E_F - E_C)^(3/2) with the
    energy in eV, from integrating the 3D density of states of Appendix A up to
    E_F at T = 0.  Returns nm^-3 eV^-3/2."""
    m = m_eff * M0
    return (2.0 * m * Q_E) ** 1.5 / (3.0 * np.pi ** 2 * HBAR ** 3) * 1e-27


def fd_half_quadrature(x):
    """Eq. FDIntegral by adaptive quadrature (reference values for the
    approximation).  Uses eps = t^2 to remove the square-root endpoint."""
    def one(xv):
        f = lambda t: 2.0 * t * t * special.expit(xv - t * t)
        upper = np.sqrt(max(xv, 0.0) + 60.0)
        pts = [np.sqrt(xv)] if xv > 0 else None
        val, _ = integrate.quad(f, 0.0, upper, points=pts, limit=400,
                                epsabs=0.0, epsrel=1e-13)
        return 2.0 / np.sqrt(np.pi) * val
    return np.vectorize(one)(np.asarray(x, dtype=np.float64))


def _bed_v(x):
    g = np.exp(-0.17 * (x + 1.0) ** 2)
    v = x ** 4 + 50.0 + 33.6 * x * (1.0 - 0.68 * g)
    dv = 4.0 * x ** 3 + 33.6 * (1.0 - 0.68 * g) + 33.6 * 0.68 * 0.34 * x * (x + 1.0) * g
    return v, dv


def fd_half(x):
    """Eq. FDIntApprox (Bednarczyk), with F = exp(x) for x < -50 as stated
    right after the equation.  The parenthesis the printed equation leaves
    open closes after the Gaussian factor."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lo = x < FD_SWITCH
    out[lo] = np.exp(x[lo])
    xh = x[~lo]
    v, _ = _bed_v(xh)
    out[~lo] = 1.0 / (np.exp(-xh) + _A_BED * v ** -0.375)
    return out


def fd_half_prime(x):
    """Exact derivative of the coded approximation ``fd_half``."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lo = x < FD_SWITCH
    out[lo] = np.exp(x[lo])
    xh = x[~lo]
    v, dv = _bed_v(xh)
    den = np.exp(-xh) + _A_BED * v ** -0.375
    out[~lo] = (np.exp(-xh) + 0.375 * _A_BED * v ** -1.375 * dv) / den ** 2
    return out


def nilsson_inverse(u):
    """Eq. FDintInverse: eta with F_1/2(eta) ~= u (stated error < 0.6%)."""
    u = np.asarray(u, dtype=np.float64)
    nu = (0.75 * np.sqrt(np.pi) * u) ** (2.0 / 3.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        first = np.where(np.abs(u - 1.0) < 1e-8, -0.5, np.log(u) / (1.0 - u * u))
    return first + nu / (1.0 + (0.24 + 1.08 * nu) ** -2)


class Statistics:
    """Electron density n(phi) and dn/dphi for one material set.

    stat: "linear" (no mobile charge), "tf" (Thomas-Fermi, T = 0) or "fd"
    (Fermi-Dirac with the Bednarczyk F_1/2 at temperature T)."""

    def __init__(self, stat, T_K=0.0, m_eff=1.08, Ec0_eV=0.56):
        if stat not in ("linear", "tf", "fd"):
            raise ValueError(stat)
        self.stat = stat
        self.T_K = float(T_K)
        self.m_eff = float(m_eff)
        self.Ec0 = float(Ec0_eV)
        if stat == "fd":
            if not self.T_K > 0:
                raise ValueError("Fermi-Dirac statistics need T > 0")
            self.kT = kT_eV(self.T_K)
            self.Nc = effective_dos(self.T_K, self.m_eff)
        if stat == "tf":
            self.Ctf = thomas_fermi_coeff(self.m_eff)

    def density(self, phi):
        phi = np.asarray(phi, dtype=np.float64)
        u = phi - self.Ec0                      # (E_F - E_C)/q in V
        if self.stat == "linear":
            return np.zeros_like(phi)
        if self.stat == "tf":
            return self.Ctf * np.maximum(u, 0.0) ** 1.5
        return self.Nc * fd_half(u / self.kT)

    def ddensity(self, phi):
        phi = np.asarray(phi, dtype=np.float64)
        u = phi - self.Ec0
        if self.stat == "linear":
            return np.zeros_like(phi)
        if self.stat == "tf":
            return 1.5 * self.Ctf * np.sqrt(np.maximum(u, 0.0))
        return self.Nc * fd_half_prime(u / self.kT) / self.kT

    def neutral_potential(self, n_target):
        """phi with n(phi) = n_target (bulk neutrality against donors), by a
        bracketed scalar root of the coded density."""
        if self.stat == "linear":
            raise ValueError("no mobile charge")
        f = lambda p: self.density(np.array([p]))[0] - n_target
        lo, hi = self.Ec0 - 2.0, self.Ec0 + 2.0
        return optimize.brentq(f, lo, hi, xtol=1e-15, rtol=4 * np.finfo(float).eps,
                               maxiter=500)
