"""Approximate quantum electron density of the predictor-corrector Poisson
step (Eq. pcPoisson with Eqs. ApproxEDens3DConfined and
ApproxEDens1DConfined).  Test infrastructure: the checker of the GPU path.

Given eigenstates of a previous outer iteration k -- nodal |psi_i|^2, levels
E_i (eV, relative to E_F = 0) and the potential phi^(k) they were computed
in -- the electron density at a point is

    n~(phi) = sum_i P |psi_i|^2 G(x_i),   x_i = (E_F - E_i + (phi - phi^(k))) / kT

(a potential rise lowers every level by the same amount to first order).
3D confinement: P = 4 (two spins, two valleys), G(x) = 1 / (1 + exp(-x)),
which is the printed denominator exp((E_i - E_F - q(phi - phi^(k)))/kT).
1D confinement: P = 2 m_t kT / (pi hbar^2), G(x) = ln(1 + exp(x)).
In the discretisation |psi_i|^2 and phi^(k) are trilinear nodal fields
evaluated at the Gauss points like phi.
"""
from __future__ import annotations

import numpy as np
from scipy import special

from .physics import HBAR, K_B, M0, kT_eV


class QuantumDensity:
    def __init__(self, psi2, phi_k, E_i, T_K, confinement=3, m_t=0.19):
        self.psi2 = np.atleast_2d(np.asarray(psi2, dtype=np.float64))
        self.phi_k = np.asarray(phi_k, dtype=np.float64)
        self.E = np.asarray(E_i, dtype=np.float64).ravel()
        if self.psi2.shape[0] != self.E.size:
            raise ValueError("one level per state")
        if confinement not in (1, 3):
            raise ValueError("confinement must be 1 or 3")
        if not T_K > 0:
            raise ValueError("the predictor-corrector density needs T > 0")
        self.conf = confinement
        self.T_K = float(T_K)
        self.kT = kT_eV(self.T_K)
        if confinement == 3:
            self.P = 4.0
        else:
            # 2 m_t kT / (pi hbar^2) in nm^-2
            self.P = 2.0 * m_t * M0 * K_B * self.T_K / (np.pi * HBAR ** 2) * 1e-18

    def occupation(self, x):
        if self.conf == 3:
            return special.expit(x)
        return np.logaddexp(0.0, x)

    def doccupation(self, x):
        s = special.expit(x)
        return s * (1.0 - s) if self.conf == 3 else s

    def _sum(self, dphi, psi2_at):
        n = np.zeros_like(dphi)
        dn = np.zeros_like(dphi)
        for i, Ei in enumerate(self.E):
            s2 = psi2_at(i)
            x = (dphi - Ei) / self.kT
            n += self.P * s2 * self.occupation(x)
            dn += self.P * s2 * self.doccupation(x) / self.kT
        return n, dn

    def at_gauss(self, mesh, phi):
        """(n~, dn~/dphi) at the Gauss points, [E, 8] each."""
        dphi = mesh.at_gauss(np.asarray(phi, dtype=np.float64) - self.phi_k)
        return self._sum(dphi, lambda i: mesh.at_gauss(self.psi2[i]))

    def at_nodes(self, phi):
        dphi = np.asarray(phi, dtype=np.float64) - self.phi_k
        return self._sum(dphi, lambda i: self.psi2[i])
