"""Newton solve, outputs and adjoint of the discrete nonlinear Poisson system.

The paper solves the discretised weak form with Trilinos' Newton method and
an exact (automatically differentiated) Jacobian (Sec. II.A.3 and II.C); it
does not state the initial guess or the globalisation.  This reference uses:

* initial guess: the charge-free linear problem (n = 0, doping kept) with the
  Dirichlet values imposed;
* Newton steps J_ff delta = -F_f with the exact Jacobian of the coded
  residual, solved directly (SuperLU) or by Jacobi-preconditioned CG;
* backtracking on ||F||_2: lambda = 1, halved until
  ||F(phi + lambda delta)|| is finite and <= (1 - 1e-4 lambda) ||F(phi)||;
* stop when ||F_free||_2 <= atol.

The discrete solution is unique (F is the gradient of a strictly convex
energy because K is SPD and n is nondecreasing), so none of these choices
changes the converged potential.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import INTERP, Problem  # noqa: F401
from .physics import Statistics

DIRECT_MAX = 3_000


def linear_solve(A, b, rtol=1e-12, method="auto", maxiter=None):
    """Solve the SPD system A x = b (library primitive: SuperLU or CG)."""
    if b.size == 0:
        return b.copy()
    if method == "direct" or (method == "auto" and A.shape[0] <= DIRECT_MAX):
        return spla.spsolve(A.tocsc(), b, permc_spec="MMD_AT_PLUS_A")
    d = A.diagonal()
    M = sp.diags(1.0 / d)
    x, info = spla.cg(A, b, rtol=rtol, atol=0.0, M=M,
                      maxiter=maxiter or 20 * A.shape[0])
    if info != 0:
        raise RuntimeError(f"CG did not converge (info={info})")
    return x


def initial_guess(prob, method="auto"):
    """Charge-free linear Poisson solve with the Dirichlet data imposed."""
    phi = prob.with_dirichlet(np.zeros(prob.mesh.N))
    lin = Statistics("linear")
    F = prob.residual(phi, stats=lin)
    f = prob.free
    K_ff = prob.K_lin[np.nonzero(f)[0]][:, np.nonzero(f)[0]]
    phi[f] -= linear_solve(K_ff, F[f], rtol=1e-13, method=method)
    return phi


@dataclass
class NewtonResult:
    phi: np.ndarray
    status: str
    iters: int
    res_history: list = field(default_factory=list)
    halvings: int = 0


def newton(prob, phi0=None, atol=1e-10, maxit=200, ls_max=30, method="auto",
           sufficient=1e-4):
    """Damped Newton on F(phi) = 0 over the free nodes."""
    phi = initial_guess(prob, method) if phi0 is None else prob.with_dirichlet(phi0)
    f = prob.free
    fidx = np.nonzero(f)[0]
    F = prob.residual(phi)
    nrm = float(np.linalg.norm(F[f]))
    hist = [nrm]
    halv = 0
    prev = None
    for it in range(maxit):
        if nrm <= atol:
            return NewtonResult(phi, "ok", it, hist, halv)
        J = prob.jacobian_full(phi)[fidx][:, fidx]
        eta = 1e-2 if prev is None else min(1e-2, 0.1 * (nrm / prev) ** 2)
        eta = max(eta, 0.5 * atol / nrm)
        delta = np.zeros_like(phi)
        delta[f] = linear_solve(J, -F[f], rtol=min(eta, 1e-2), method=method)
        lam = 1.0
        for h in range(ls_max + 1):
            trial = phi + lam * delta
            # a full step can put a Boltzmann exponent beyond the double range
            # (the density is then +inf and the residual not finite): such a
            # trial is rejected like any other that does not decrease ||F||
            with np.errstate(over="ignore", invalid="ignore"):
                Ft = prob.residual(trial)
                nt = float(np.linalg.norm(Ft[f]))
            if np.isfinite(nt) and nt <= (1.0 - sufficient * lam) * nrm:
                break
            lam *= 0.5
            halv += 1
        else:
            return NewtonResult(phi, "linesearch", it, hist, halv)
        prev = nrm
        phi, F, nrm = trial, Ft, nt
        hist.append(nrm)
    return NewtonResult(phi, "ok" if nrm <= atol else "not_converged", maxit, hist, halv)


def make_problem(dev, extra_load=None):
    """Problem from a device description (see synth.devices.Device)."""
    st = Statistics(dev.stat, dev.T_K, dev.m_eff, dev.Ec0_eV, holes=getattr(dev, "holes", False),
                    ionization=getattr(dev, "ionization", "complete"))
    return Problem(dev, st, extra_load=extra_load)


def solve(dev, **kw):
    prob = make_problem(dev)
    res = newton(prob, **kw)
    return prob, res


@dataclass
class AdjointResult:
    Q: float
    dQ_ddir: np.ndarray       # [n_dir] electrons per volt
    dQ_deps: np.ndarray       # [E] electrons per unit relative permittivity
    lam: np.ndarray           # [N] adjoint state (zero on Dirichlet nodes)


def adjoint(prob, phi, box, method="auto"):
    """Gradient of the electron count in ``box`` at a converged phi.

    With F_f(phi_f; V, eps) = 0, dQ/dp = dQ/dp|_explicit - lam_f^T dF_f/dp where
    J_ff lam_f = dQ/dphi_f (J is symmetric).  For a contact value V_g the
    explicit part is dQ/dphi summed over that contact's nodes and
    dF_f/dV_g = J_{f,D_g} 1; for eps_e, dF/deps_e = Khat_e phi_e."""
    m = prob.mesh
    sel = prob.box_elements(box).astype(np.float64)
    nq = prob.stats.density(m.at_gauss(phi))
    Q = float(np.sum((m.W * sel)[:, None] * nq))
    gq = (m.W * sel)[:, None] * prob.stats.ddensity(m.at_gauss(phi))
    g = m.scatter(gq @ INTERP)
    J = prob.jacobian_full(phi)
    fidx = np.nonzero(prob.free)[0]
    lam = np.zeros(m.N)
    lam[fidx] = linear_solve(J[fidx][:, fidx], g[fidx], rtol=1e-13, method=method)
    s = J.T @ lam
    dQdV = np.zeros(prob.dir_val.size)
    didx = np.nonzero(prob.dirichlet)[0]
    np.add.at(dQdV, prob.dir_id[didx], g[didx] - s[didx])
    le = lam[m.conn]
    pe = phi[m.conn]
    dQde = -np.einsum("ea,eab,eb->e", le, prob.Khat, pe)
    return AdjointResult(Q, dQdV, dQde, lam)
