"""Galerkin discretisation of Eq. PoissonWeakForm on a rectilinear Q1 mesh.

Divided by eps0 and written in nm/V units the weak form reads, for every
basis function w_i of a free node,

    F_i(phi) = sum_e [ eps_e (Khat_e phi_e)_i
                       - KAPPA semi_e sum_q W_q (N_net,e - n(phi_q)) w_i(q) ] = 0

with the boundary integral dropped on every non-Dirichlet face (the default
flux-conserving Neumann condition, Sec. II.A.4) except on the faces of the
device's sheets, which carry a surface charge and / or a Robin condition
(``sheet_terms``).  Khat_e is the unit-
permittivity trilinear stiffness of a box element, exact under 2x2x2 Gauss
quadrature; phi_q is the trilinear interpolant at the Gauss points and
W_q = hx*hy*hz/8.  Everything is assembled into scipy.sparse matrices.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .physics import KAPPA
from .quantum import QuantumDensity

# 1D linear-element pieces on a unit interval: stiffness and mass.
_A1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
_M1 = np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0
# Two-point Gauss-Legendre abscissae on [0, 1] and the 1D shape values there.
GAUSS_1D = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
_B1 = np.stack([1.0 - GAUSS_1D, GAUSS_1D], axis=1)   # [q, a] = w_a(xi_q)


def _kron3(z, y, x):
    # local index a + 2 b + 4 c  (x fastest) <-> kron(z, kron(y, x))
    return np.kron(z, np.kron(y, x))


KHAT_X = _kron3(_M1, _M1, _A1)
KHAT_Y = _kron3(_M1, _A1, _M1)
KHAT_Z = _kron3(_A1, _M1, _M1)
INTERP = _kron3(_B1, _B1, _B1)          # [q, a]: shape function a at Gauss point q


class Mesh:
    """Connectivity and element sizes of a rectilinear hexahedral mesh."""

    def __init__(self, x, y, z):
        self.x = np.asarray(x, dtype=np.float64)
        self.y = np.asarray(y, dtype=np.float64)
        self.z = np.asarray(z, dtype=np.float64)
        for c in (self.x, self.y, self.z):
            if c.size < 2 or np.any(np.diff(c) <= 0):
                raise ValueError("coordinates must be strictly increasing, >= 2 nodes")
        nx, ny, nz = self.x.size, self.y.size, self.z.size
        self.nx, self.ny, self.nz = nx, ny, nz
        self.N = nx * ny * nz
        ex, ey, ez = nx - 1, ny - 1, nz - 1
        self.E = ex * ey * ez
        k, j, i = np.meshgrid(np.arange(ez), np.arange(ey), np.arange(ex), indexing="ij")
        i, j, k = i.ravel(), j.ravel(), k.ravel()
        conn = np.empty((self.E, 8), dtype=np.int64)
        for c in range(2):
            for b in range(2):
                for a in range(2):
                    conn[:, a + 2 * b + 4 * c] = (i + a) + nx * ((j + b) + ny * (k + c))
        self.conn = conn
        self.hx = np.diff(self.x)[i]
        self.hy = np.diff(self.y)[j]
        self.hz = np.diff(self.z)[k]
        self.W = self.hx * self.hy * self.hz / 8.0          # per Gauss point
        self.centroid = np.stack([0.5 * (self.x[i] + self.x[i + 1]),
                                  0.5 * (self.y[j] + self.y[j + 1]),
                                  0.5 * (self.z[k] + self.z[k + 1])], axis=1)

    def unit_stiffness(self):
        """Khat_e for every element, [E, 8, 8]."""
        return ((self.hy * self.hz / self.hx)[:, None, None] * KHAT_X
                + (self.hx * self.hz / self.hy)[:, None, None] * KHAT_Y
                + (self.hx * self.hy / self.hz)[:, None, None] * KHAT_Z)

    def axis_stiffness(self):
        """The three parts of Khat_e, int_e d_a w_i d_a w_j for a = x, y, z,
        each [E, 8, 8] (their sum is unit_stiffness())."""
        return ((self.hy * self.hz / self.hx)[:, None, None] * KHAT_X,
                (self.hx * self.hz / self.hy)[:, None, None] * KHAT_Y,
                (self.hx * self.hy / self.hz)[:, None, None] * KHAT_Z)

    def assemble(self, elem_mats):
        """Sum element matrices [E, 8, 8] into an N x N CSR matrix."""
        rows = np.broadcast_to(self.conn[:, :, None], elem_mats.shape).ravel()
        cols = np.broadcast_to(self.conn[:, None, :], elem_mats.shape).ravel()
        return sp.coo_matrix((elem_mats.ravel(), (rows, cols)), shape=(self.N, self.N)).tocsr()

    def scatter(self, elem_vecs):
        """Sum element vectors [E, 8] into a nodal vector [N]."""
        return np.bincount(self.conn.ravel(), weights=elem_vecs.ravel(), minlength=self.N)

    def at_gauss(self, nodal):
        """Trilinear interpolant at the 8 Gauss points of every element, [E, 8]."""
        return nodal[self.conn] @ INTERP.T


def sheet_nodes(mesh, sh):
    """Global node indices [nb+1, na+1] of a sheet's face range (a fastest)."""
    a = np.arange(sh.a0, sh.a1 + 1)
    b = np.arange(sh.b0, sh.b1 + 1)
    B, A = np.meshgrid(b, a, indexing="ij")
    nx, ny = mesh.nx, mesh.ny
    if sh.axis == 2:
        i, j, k = A, B, np.full_like(A, sh.plane)
    elif sh.axis == 1:
        i, j, k = A, np.full_like(A, sh.plane), B
    elif sh.axis == 0:
        i, j, k = np.full_like(A, sh.plane), A, B
    else:
        raise ValueError("sheet axis must be 0, 1 or 2")
    return i + nx * (j + ny * k)


def sheet_coords(mesh, sh):
    """Coordinates along the sheet's first and second in-plane axes."""
    xs = {0: (mesh.y, mesh.z), 1: (mesh.x, mesh.z), 2: (mesh.x, mesh.y)}[sh.axis]
    return xs


def sheet_terms(mesh, sheets):
    """Face integrals of the interface and Robin conditions (Sec. II.A.4).

    For every face f of a sheet (a rectangle of the plane x_axis = const):

    * surface charge (Eq. NeuBC4fc): the flux jump across the face equals
      q sigma_f, so the weak form gains the load KAPPA sigma_f int_f w_i, the
      same sign as a volume charge;
    * Robin (a pinned plane at potential phi0 a distance d beyond the face,
      with the layer's permittivity eps): the outward flux is
      eps (phi0 - phi)/d, so the weak form gains (eps/d) int_f (phi - phi0) w_i.

    Returns the face-mass matrix R (N x N CSR, (eps/d) int_f w_i w_j) and the
    constant load s (KAPPA sigma int_f w_i + (eps/d) phi0 int_f w_i); the
    residual is then K phi + R phi - s - b(phi)."""
    N = mesh.N
    rows, cols, vals = [], [], []
    load = np.zeros(N)
    for sh in sheets:
        ca, cb = sheet_coords(mesh, sh)
        if not (0 <= sh.a0 < sh.a1 <= ca.size - 1 and 0 <= sh.b0 < sh.b1 <= cb.size - 1):
            raise ValueError("sheet face range outside the mesh")
        nodes = sheet_nodes(mesh, sh)                 # [nb+1, na+1]
        ha = np.diff(ca)[sh.a0:sh.a1]
        hb = np.diff(cb)[sh.b0:sh.b1]
        na, nb = sh.a1 - sh.a0, sh.b1 - sh.b0
        sigma = np.zeros((nb, na)) if sh.sigma is None else np.asarray(sh.sigma, float).reshape(nb, na)
        alpha = sh.robin_eps / sh.robin_d if sh.robin_d > 0 else 0.0
        for jb in range(nb):
            for ia in range(na):
                corners = [nodes[jb, ia], nodes[jb, ia + 1], nodes[jb + 1, ia], nodes[jb + 1, ia + 1]]
                area = ha[ia] * hb[jb]
                # int_f w_i w_j = (int X_i X_j da)(int Y_i Y_j db), 1D linear mass [[2,1],[1,2]]/6
                Mf = np.kron(_M1 * hb[jb], _M1 * ha[ia])
                if alpha > 0:
                    for r in range(4):
                        for c in range(4):
                            rows.append(corners[r])
                            cols.append(corners[c])
                            vals.append(alpha * Mf[r, c])
                for r in range(4):
                    load[corners[r]] += (KAPPA * sigma[jb, ia] + alpha * sh.phi0) * area / 4.0
    R = sp.coo_matrix((vals, (rows, cols)), shape=(N, N)).tocsr()
    return R, load


class Problem:
    """One device: mesh, materials, Dirichlet data, statistics.

    dev: an object with x, y, z, eps_r, semi, net_doping, dir_id, dir_val
    stats: physics.Statistics
    extra_load: optional nodal load vector added to the right-hand side (used
        for manufactured solutions only)."""

    def __init__(self, dev, stats, extra_load=None):
        self.mesh = Mesh(dev.x, dev.y, dev.z)
        m = self.mesh
        self.eps = np.asarray(dev.eps_r, dtype=np.float64)
        self.semi = np.asarray(dev.semi).astype(np.float64)
        self.netdop = np.asarray(dev.net_doping, dtype=np.float64)
        # separate donor / acceptor densities (needed for incomplete ionization)
        nd = getattr(dev, "donors", None)
        na = getattr(dev, "acceptors", None)
        self.nd = None if nd is None else np.asarray(nd, dtype=np.float64)
        self.na = None if na is None else np.asarray(na, dtype=np.float64)
        self.dir_id = np.asarray(dev.dir_id, dtype=np.int64)
        self.dir_val = np.asarray(dev.dir_val, dtype=np.float64)
        if self.eps.shape != (m.E,) or self.semi.shape != (m.E,) or self.netdop.shape != (m.E,):
            raise ValueError("per-element arrays have the wrong length")
        if self.dir_id.shape != (m.N,):
            raise ValueError("dir_id must have one entry per node")
        self.stats = stats
        if stats.ionization == "incomplete" and (self.nd is None or self.na is None):
            raise ValueError("incomplete ionization needs donors and acceptors per element")
        self.dirichlet = self.dir_id >= 0
        self.free = ~self.dirichlet
        self.extra_load = extra_load
        self.Khat = m.unit_stiffness()
        self.K = m.assemble(self.eps[:, None, None] * self.Khat)
        # interface charge and Robin faces (Sec. II.A.4)
        self.sheets = list(getattr(dev, "sheets", None) or [])
        self.R, self.sheet_load = sheet_terms(m, self.sheets)
        self.K_lin = self.K + self.R      # the phi-linear part of F
        # predictor-corrector electrons from given eigenstates (replace n(phi))
        q = getattr(dev, "quantum", None)
        self.quantum = None if q is None else QuantumDensity(q.psi2, q.phi_k, q.E_i, stats.T_K, q.confinement,
                                                             q.m_t)
        # elements whose electrons come from the states (all when no region is given)
        reg = None if q is None else getattr(q, "region", None)
        self.qregion = None if reg is None else np.asarray(reg).astype(bool)

    def electrons_at_gauss(self, phi):
        """(n, dn/dphi) at the Gauss points, [E, 8]: the statistics, or the
        predictor-corrector density inside the quantum region."""
        m = self.mesh
        phq = m.at_gauss(phi)
        n, dn = self.stats.density(phq), self.stats.ddensity(phq)
        if self.quantum is None:
            return n, dn
        nq, dnq = self.quantum.at_gauss(m, phi)
        if self.qregion is None:
            return nq, dnq
        r = self.qregion[:, None]
        return np.where(r, nq, n), np.where(r, dnq, dn)

    # --- nodal vectors -------------------------------------------------
    def with_dirichlet(self, phi):
        out = np.array(phi, dtype=np.float64, copy=True)
        out[self.dirichlet] = self.dir_val[self.dir_id[self.dirichlet]]
        return out

    def charge_load(self, phi, stats=None):
        """b_i = KAPPA sum_e semi_e sum_q W_q rho(phi_q) w_i(q) with the space
        charge rho = p - n + N_D+ - N_A- (= N_net - n without holes and with
        complete ionization)."""
        m = self.mesh
        st = self.stats if stats is None else stats
        phq = m.at_gauss(phi)
        nd = None if self.nd is None else self.nd[:, None]
        na = None if self.na is None else self.na[:, None]
        nq = None
        if self.quantum is not None and stats is None:
            nq, _ = self.electrons_at_gauss(phi)
        rho = st.rho(phq, self.netdop[:, None], nd, na, electrons=nq)
        qv = KAPPA * (self.semi * m.W)[:, None] * rho          # [E, q]
        b = m.scatter(qv @ INTERP)                               # project: sum_q qv_q w_a(q)
        if self.extra_load is not None:
            b = b + self.extra_load
        return b

    def residual_full(self, phi, stats=None):
        """K phi - b(phi) on every node (Dirichlet rows included)."""
        return self.K_lin @ phi - self.sheet_load - self.charge_load(phi, stats)

    def residual(self, phi, stats=None):
        """Eq. PoissonWeakForm residual on free nodes, zero on Dirichlet rows."""
        F = self.residual_full(phi, stats)
        F[self.dirichlet] = 0.0
        return F

    def coeff(self, phi):
        """c_{e,q} = -KAPPA semi_e W_q rho'(phi_q) (= KAPPA semi_e W_q n'(phi_q)
        for electrons alone): the linearised charge weights, >= 0."""
        m = self.mesh
        nd = None if self.nd is None else self.nd[:, None]
        na = None if self.na is None else self.na[:, None]
        dnq = None if self.quantum is None else self.electrons_at_gauss(phi)[1]
        return -KAPPA * (self.semi * m.W)[:, None] * self.stats.drho(m.at_gauss(phi), nd, na, delectrons=dnq)

    def jacobian_full(self, phi):
        """dF/dphi on all nodes: eps K + sum_q c_q w(q) w(q)^T (N x N CSR)."""
        c = self.coeff(phi)
        Me = np.einsum("eq,qa,qb->eab", c, INTERP, INTERP)
        return self.K_lin + self.mesh.assemble(Me)

    def jacobian_free(self, phi):
        J = self.jacobian_full(phi)
        f = np.nonzero(self.free)[0]
        return J[f][:, f]

    def jv(self, phi, v):
        """Masked Jacobian product: v is zeroed on Dirichlet nodes, free rows get
        (J v)_i, Dirichlet rows return v_i (identity rows)."""
        vm = np.where(self.free, v, 0.0)
        y = self.jacobian_full(phi) @ vm
        return np.where(self.free, y, v)

    def jacobi_diag(self, phi):
        d = self.jacobian_full(phi).diagonal().copy()
        d[self.dirichlet] = 1.0
        return d

    def nodal_density(self, phi):
        """n(phi_i) at nodes that touch a semiconductor element, else 0."""
        touch = np.zeros(self.mesh.N, dtype=bool)
        touch[self.mesh.conn[self.semi > 0].ravel()] = True
        n = self.stats.density(phi)
        if self.quantum is not None:
            # nodes touching a quantum-region element take the states' density
            qn = np.ones(self.mesh.N, dtype=bool)
            if self.qregion is not None:
                qn[:] = False
                qn[self.mesh.conn[self.qregion].ravel()] = True
            n = np.where(qn, self.quantum.at_nodes(phi)[0], n)
        return np.where(touch, n, 0.0)

    def box_elements(self, box):
        """Semiconductor elements whose centroid lies in the closed box
        (x0, x1, y0, y1, z0, z1)."""
        c = self.mesh.centroid
        x0, x1, y0, y1, z0, z1 = box
        inside = ((c[:, 0] >= x0) & (c[:, 0] <= x1) & (c[:, 1] >= y0) & (c[:, 1] <= y1)
                  & (c[:, 2] >= z0) & (c[:, 2] <= z1))
        return inside & (self.semi > 0)

    def count(self, phi, box):
        """Electrons in a region: sum_e sum_q W_q n(phi_q) over its elements
        (the integral of n that enters C = q dN/dV in Sec. III)."""
        sel = self.box_elements(box)
        m = self.mesh
        nq = self.electrons_at_gauss(phi)[0]
        return float(np.sum(m.W[sel][:, None] * nq[sel]))
