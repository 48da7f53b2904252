"""Effective-mass Schrodinger eigenproblem on the Q1 mesh (Eqs. SchrodEqn and
SchrodEqnWeakForm, Sec. II.B).  Test infrastructure: the checker of the GPU
eigensolver.

With w_i the trilinear basis, the weak form gives the generalized symmetric
eigenproblem H psi = E M psi with

    H_ij = sum_e (hbar^2 / (2 m0)) sum_a (m0 / m*_e,a) int_e d_a w_i d_a w_j
           + sum_e int_e V w_i w_j,        V = v0_e - phi   (eV)
    M_ij = sum_e int_e w_i w_j

where a runs over x, y, z: a diagonal mass tensor per element, as Eq.
Schrodinger3D writes for the Delta_2 valleys of a Si dot (m_t along x and y,
m_l along z, Sec. II.C); equal masses give the isotropic operator of Eq.
SchrodEqn.

(the element integrals exact under 2x2x2 Gauss quadrature, V evaluated at
the Gauss points from the interpolated phi).  Nodes listed as fixed carry
psi = 0 (Dirichlet) and are removed; every other boundary is the natural
Neumann condition.  Energies in eV, lengths in nm; eigenvectors are
M-orthonormal with their largest-magnitude entry positive.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as la
import scipy.sparse.linalg as spla

from .fem import INTERP, Mesh
from .physics import HBAR, M0, Q_E

HB2M = HBAR ** 2 / (2.0 * M0) / Q_E * 1e18      # hbar^2 / (2 m0) in eV nm^2
DENSE_MAX = 2500


def axis_inverse_masses(inv_mass, E):
    """m0 / m* per element and axis, [3, E] (x, y, z), from [E] (isotropic)
    or [3, E]."""
    im = np.asarray(inv_mass, float)
    if im.shape == (E,):
        return np.stack([im, im, im])
    if im.shape != (3, E):
        raise ValueError(f"inv_mass: shape {im.shape}, expected ({E},) or (3, {E})")
    return im


def assemble(mesh, inv_mass, v0, phi):
    """H and M as CSR matrices over all nodes."""
    im = axis_inverse_masses(inv_mass, mesh.E)
    K = mesh.axis_stiffness()
    H = mesh.assemble(sum((HB2M * im[a])[:, None, None] * K[a] for a in range(3)))
    Vq = np.asarray(v0, float)[:, None] - mesh.at_gauss(np.asarray(phi, float))   # [E, q]
    Mv = np.einsum("eq,qa,qb->eab", mesh.W[:, None] * Vq, INTERP, INTERP)
    Mm = np.einsum("e,qa,qb->eab", mesh.W, INTERP, INTERP)
    return H + mesh.assemble(Mv), mesh.assemble(Mm)


def solve(x, y, z, inv_mass, v0, phi, fixed, n_states):
    """Lowest n_states eigenpairs: (E [n], psi [n, N] with zeros on fixed
    nodes).  inv_mass: [E] or [3, E] (see axis_inverse_masses)."""
    mesh = Mesh(x, y, z)
    H, M = assemble(mesh, inv_mass, v0, phi)
    free = np.nonzero(~np.asarray(fixed, bool))[0]
    Hf = H[free][:, free]
    Mf = M[free][:, free]
    if free.size <= DENSE_MAX:
        E, V = la.eigh(Hf.toarray(), Mf.toarray(), subset_by_index=[0, n_states - 1])
    else:
        # shift-invert about a point below the spectrum (the smallest V)
        sigma = float(np.min(np.asarray(v0, float)[:, None] - mesh.at_gauss(np.asarray(phi, float)))) - 1.0
        E, V = spla.eigsh(Hf.tocsc(), k=n_states, M=Mf.tocsc(), sigma=sigma, which="LM", tol=1e-14)
        order = np.argsort(E)
        E, V = E[order], V[:, order]
    psi = np.zeros((n_states, mesh.N))
    for i in range(n_states):
        v = V[:, i] / np.sqrt(V[:, i] @ (Mf @ V[:, i]))
        if v[np.argmax(np.abs(v))] < 0:
            v = -v
        psi[i, free] = v
    return E, psi, (H, M)
