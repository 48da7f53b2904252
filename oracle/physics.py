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


def hole_dos_mass(m_hh, m_lh):
    """Eq. EffectiveMass: valence DOS mass from the heavy and light holes."""
    return (m_hh ** 1.5 + m_lh ** 1.5) ** (2.0 / 3.0)


# Textbook silicon values used as defaults where the paper prints none.
SI_M_HH, SI_M_LH = 0.49, 0.16
SI_M_H = hole_dos_mass(SI_M_HH, SI_M_LH)     # ~0.549 m0
SI_EG_EV = 1.12
SI_ED_EV = 0.046                              # phosphorus (Sec. II.A.3)
SI_EA_EV = 0.044                              # boron
G_D, G_A = 2.0, 4.0


class Statistics:
    """Carrier densities and the space charge of Eq. Poisson for one
    material set.

    stat: "linear" (no mobile charge), "tf" (Thomas-Fermi, T = 0), "mb"
    (Maxwell-Boltzmann, Eq. MBstatistics) or "fd" (Fermi-Dirac with the
    Bednarczyk F_1/2, Eq. FDstatistics) at temperature T.

    Electrons see E_F - E_C = phi - Ec0.  With ``holes`` the valence edge is
    E_V = E_C - Eg, so E_V - E_F = Ec0 - Eg - phi, and holes follow the same
    statistics with the valence DOS mass m_h (Eqs. EffectiveDOS and
    EffectiveMass).  With ``ionization="incomplete"`` the ionised donors and
    acceptors follow Eq. Ionization with E_F - E_D = (phi - Ec0) + E_d and
    E_A - E_F = (Ec0 - Eg - phi) + E_a (Eq. FinalIonization in this
    convention); it needs T > 0."""

    def __init__(self, stat, T_K=0.0, m_eff=1.08, Ec0_eV=0.56, holes=False, m_h=SI_M_H,
                 Eg_eV=SI_EG_EV, ionization="complete", Ed_eV=SI_ED_EV, Ea_eV=SI_EA_EV,
                 gD=G_D, gA=G_A):
        if stat not in ("linear", "tf", "fd", "mb"):
            raise ValueError(stat)
        if ionization not in ("complete", "incomplete"):
            raise ValueError(ionization)
        self.stat = stat
        self.T_K = float(T_K)
        self.m_eff = float(m_eff)
        self.Ec0 = float(Ec0_eV)
        self.holes = bool(holes)
        self.m_h = float(m_h)
        self.Eg = float(Eg_eV)
        self.ionization = ionization
        self.Ed, self.Ea, self.gD, self.gA = float(Ed_eV), float(Ea_eV), float(gD), float(gA)
        if stat in ("fd", "mb") or ionization == "incomplete":
            if not self.T_K > 0:
                raise ValueError("Fermi-Dirac / Boltzmann statistics and incomplete ionization need T > 0")
            self.kT = kT_eV(self.T_K)
        if stat in ("fd", "mb"):
            self.Nc = effective_dos(self.T_K, self.m_eff)
            self.Nv = effective_dos(self.T_K, self.m_h)
        if stat == "tf":
            self.Ctf = thomas_fermi_coeff(self.m_eff)
            self.Ctf_h = thomas_fermi_coeff(self.m_h)

    @property
    def full(self):
        """True when the charge is more than net doping minus electrons."""
        return self.holes or self.ionization == "incomplete"

    def _band(self, u, N, C):
        """N F(u/kT) (or the T = 0 limit) for u = (E_F - E_band edge) in V."""
        if self.stat == "linear":
            return np.zeros_like(u)
        if self.stat == "tf":
            return C * np.maximum(u, 0.0) ** 1.5
        if self.stat == "mb":
            return N * np.exp(u / self.kT)
        return N * fd_half(u / self.kT)

    def _dband(self, u, N, C):
        """d/du of ``_band``."""
        if self.stat == "linear":
            return np.zeros_like(u)
        if self.stat == "tf":
            return 1.5 * C * np.sqrt(np.maximum(u, 0.0))
        if self.stat == "mb":
            return N * np.exp(u / self.kT) / self.kT
        return N * fd_half_prime(u / self.kT) / self.kT

    def density(self, phi):
        """Electron density n(phi)."""
        phi = np.asarray(phi, dtype=np.float64)
        return self._band(phi - self.Ec0, getattr(self, "Nc", 0.0), getattr(self, "Ctf", 0.0))

    def ddensity(self, phi):
        phi = np.asarray(phi, dtype=np.float64)
        return self._dband(phi - self.Ec0, getattr(self, "Nc", 0.0), getattr(self, "Ctf", 0.0))

    def hole_density(self, phi):
        """Hole density p(phi) (0 unless ``holes``)."""
        phi = np.asarray(phi, dtype=np.float64)
        if not self.holes:
            return np.zeros_like(phi)
        return self._band(self.Ec0 - self.Eg - phi, getattr(self, "Nv", 0.0), getattr(self, "Ctf_h", 0.0))

    def dhole_density(self, phi):
        phi = np.asarray(phi, dtype=np.float64)
        if not self.holes:
            return np.zeros_like(phi)
        return -self._dband(self.Ec0 - self.Eg - phi, getattr(self, "Nv", 0.0), getattr(self, "Ctf_h", 0.0))

    def ionized(self, phi, nd, na):
        """(N_D+, N_A-) of Eq. Ionization; complete ionization returns (nd, na)."""
        phi = np.asarray(phi, dtype=np.float64)
        nd = np.broadcast_to(np.asarray(nd, dtype=np.float64), phi.shape)
        na = np.broadcast_to(np.asarray(na, dtype=np.float64), phi.shape)
        if self.ionization == "complete":
            return nd.copy(), na.copy()
        a = (phi - self.Ec0 + self.Ed) / self.kT          # (E_F - E_D)/kT
        b = (self.Ec0 - self.Eg - phi + self.Ea) / self.kT  # (E_A - E_F)/kT
        return nd * special.expit(-(a + np.log(self.gD))), na * special.expit(-(b + np.log(self.gA)))

    def dionized(self, phi, nd, na):
        """(d N_D+/dphi, d N_A-/dphi)."""
        phi = np.asarray(phi, dtype=np.float64)
        nd = np.broadcast_to(np.asarray(nd, dtype=np.float64), phi.shape)
        na = np.broadcast_to(np.asarray(na, dtype=np.float64), phi.shape)
        if self.ionization == "complete":
            return np.zeros_like(phi), np.zeros_like(phi)
        a = (phi - self.Ec0 + self.Ed) / self.kT + np.log(self.gD)
        b = (self.Ec0 - self.Eg - phi + self.Ea) / self.kT + np.log(self.gA)
        # d/dx of 1/(1 + e^x) = -s(1 - s) with s = 1/(1 + e^-x) ... written with expit
        sa = special.expit(a)
        sb = special.expit(b)
        return -nd * sa * (1.0 - sa) / self.kT, na * sb * (1.0 - sb) / self.kT

    def rho(self, phi, netdop, nd=None, na=None, electrons=None):
        """Space charge p - n + N_D+ - N_A- in nm^-3 (Eq. Poisson).  With
        complete ionization the dopants enter through netdop = N_D - N_A.
        ``electrons`` replaces n(phi) (the predictor-corrector density)."""
        phi = np.asarray(phi, dtype=np.float64)
        n = self.density(phi) if electrons is None else electrons
        r = self.hole_density(phi) - n
        if self.ionization == "complete":
            return r + np.asarray(netdop, dtype=np.float64)
        dp, am = self.ionized(phi, nd, na)
        return r + dp - am

    def drho(self, phi, nd=None, na=None, delectrons=None):
        phi = np.asarray(phi, dtype=np.float64)
        dn = self.ddensity(phi) if delectrons is None else delectrons
        r = self.dhole_density(phi) - dn
        if self.ionization == "complete":
            return r
        ddp, dam = self.dionized(phi, nd, na)
        return r + ddp - dam

    def neutral_potential(self, n_target):
        """phi with n(phi) = n_target (bulk neutrality against donors), by a
        bracketed scalar root of the coded density."""
        if self.stat == "linear":
            raise ValueError("no mobile charge")
        f = lambda p: self.density(np.array([p]))[0] - n_target
        lo, hi = self.Ec0 - 2.0, self.Ec0 + 2.0
        return optimize.brentq(f, lo, hi, xtol=1e-15, rtol=4 * np.finfo(float).eps,
                               maxiter=500)


def ohmic_potential(st, nd, na, Va=0.0, low_T_log_min=None):
    """Dirichlet value of an Ohmic contact (Sec. II.A.4, second case):
    thermal equilibrium and charge neutrality at the contact, majority
    carriers only.  n-type when nd >= na, else p-type; with complete
    ionization the net doping |nd - na| sets the majority density, with
    incomplete ionization the majority dopant alone (as printed).

    * MB, complete ionization: Eq. PotBC4MBCompIon.
    * MB, incomplete ionization: Eqs. Yval4MBIncompIon and PotBC4MBIncompIon,
      with ln y from Eq. ApproxLogTerms once the exponential in y would not be
      representable (the argument of the square root exceeds 1e300, or
      ``low_T_log_min`` if given).  The p-type potential carries +E_a: that is
      what the definitions of y_p and E_a give (the printed equation shows
      -E_a).
    * FD, complete ionization: Eq. PotBC4FDCompIon with the Nilsson inverse of
      Eq. FDintInverse.  FD with incomplete ionization uses the MB form, as
      the paper does.
    Potentials in V with our convention E_C(phi) = Ec0 - phi at E_F = 0."""
    kT = st.kT
    ntype = nd >= na
    if st.ionization == "complete":
        # majority carriers balance the net doping (the printed forms take a
        # single dopant species; with compensation n = N_D - N_A)
        net = abs(nd - na)
        if st.stat == "mb":
            if ntype:
                return st.Ec0 + kT * np.log(net / st.Nc) + Va
            return st.Ec0 - st.Eg - kT * np.log(net / st.Nv) + Va
        if st.stat == "fd":
            if ntype:
                return st.Ec0 + kT * float(nilsson_inverse(net / st.Nc)) + Va
            return st.Ec0 - st.Eg - kT * float(nilsson_inverse(net / st.Nv)) + Va
        raise ValueError("Ohmic contacts need MB or FD statistics")
    lim = 1e300 if low_T_log_min is None else low_T_log_min
    if ntype:
        ln_arg = np.log(8.0 * nd / st.Nc) + st.Ed / kT
        if ln_arg < np.log(lim):
            ln_y = np.log(-0.25 + 0.25 * np.sqrt(1.0 + np.exp(ln_arg)))
        else:
            ln_y = 0.5 * np.log(nd / (2.0 * st.Nc)) + st.Ed / (2.0 * kT)
        return st.Ec0 - st.Ed + kT * ln_y + Va
    ln_arg = np.log(16.0 * na / st.Nv) + st.Ea / kT
    if ln_arg < np.log(lim):
        ln_y = np.log(-0.125 + 0.125 * np.sqrt(1.0 + np.exp(ln_arg)))
    else:
        ln_y = 0.5 * np.log(na / (4.0 * st.Nv)) + st.Ea / (2.0 * kT)
    return st.Ec0 - st.Eg + st.Ea - kT * ln_y + Va


def neutral_root(st, netdop, nd=None, na=None, lo=-3.0, hi=3.0):
    """phi with rho(phi) = 0 for a uniform material, by a bracketed root of
    the coded space charge (a check for the closed forms above).  At low
    temperature a Boltzmann density at the bracket ends exceeds the double
    range; +inf or -inf there still gives the sign the bracket needs."""
    def f(p):
        with np.errstate(over="ignore"):
            return float(st.rho(np.array([p]), netdop, nd, na)[0])
    return optimize.brentq(f, lo, hi, xtol=1e-15, rtol=4 * np.finfo(float).eps, maxiter=1000)
