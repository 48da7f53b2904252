"""Seeded Si/SiO2 gate-stack devices on rectilinear Q1 hexahedral meshes.

Layout conventions shared by every consumer:

* nodes are numbered ``i + nx*(j + ny*k)`` (x fastest), elements
  ``i + (nx-1)*(j + (ny-1)*k)``; coordinates are in nm;
* z = 0 is the bottom (grounded substrate contact), z = z_max the top face
  where the metal gates sit on the oxide;
* per element: relative permittivity, a semiconductor flag and the net doping
  N_D - N_A in nm^-3 (1 cm^-3 = 1e-21 nm^-3);
* Dirichlet data: ``dir_id[node]`` is -1 for a free node, otherwise an index
  into ``dir_val`` (volts); gates come first, the bottom contact last.

The workloads mirror the paper's devices (a Si substrate under a 10 nm gate
oxide with top depletion gates, Sec. III and IV); the real device layouts are
not available, so every geometry here is synthetic and drawn from a seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

EPS_SI = 11.7
EPS_OX = 3.9
BOX_XY_NM = 200.0
SI_NM = 90.0
OX_NM = 10.0
NA_BULK_NM3 = 1e15 * 1e-21          # 1e15 cm^-3 acceptors, fully ionised
SEED_BASE = 7561

# Dot regions of the double-dot stack (x0, x1, y0, y1, z0, z1) in nm.
DOT_BOX_D1 = (0.0, 60.0, 70.0, 130.0, 70.0, 90.0)
DOT_BOX_D2 = (140.0, 200.0, 70.0, 130.0, 70.0, 90.0)


@dataclass
class Sheet:
    """A rectangle of mesh faces in the plane x_axis = coordinate[plane]
    (axis 0: x, 1: y, 2: z) covering faces a0..a1-1 along its first in-plane
    axis and b0..b1-1 along its second (axis 2: x then y; axis 1: x then z;
    axis 0: y then z).  sigma: per-face surface charge density in nm^-2
    (a fastest) or None; a Robin condition pins the potential phi0 (V) on a
    plane robin_d nm beyond the faces through a layer of relative permittivity
    robin_eps (robin_d = 0: no Robin term)."""
    axis: int
    plane: int
    a0: int
    a1: int
    b0: int
    b1: int
    sigma: np.ndarray = None
    robin_d: float = 0.0
    robin_eps: float = 0.0
    phi0: float = 0.0


@dataclass
class QuantumStates:
    """Eigenstates of an earlier outer iteration for the predictor-corrector
    density: psi2 [n_states, N] nodal |psi_i|^2 (nm^-3 for 3D confinement,
    nm^-1 for 1D), phi_k [N] the potential they were computed in (V), E_i
    [n_states] levels relative to E_F (eV), confinement 3 or 1, m_t the
    transverse mass (1D form), region the elements whose electrons come from
    the states (the semiclassical statistics elsewhere; None: everywhere)."""
    psi2: np.ndarray
    phi_k: np.ndarray
    E_i: np.ndarray
    confinement: int = 3
    m_t: float = 0.19
    region: np.ndarray = None      # [E] quantum-region elements (None: all)


@dataclass
class Device:
    name: str
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    eps_r: np.ndarray          # [E] float64
    semi: np.ndarray           # [E] uint8
    net_doping: np.ndarray     # [E] float64, nm^-3
    dir_id: np.ndarray         # [N] int32
    dir_val: np.ndarray        # [G] float64, V
    contacts: list = field(default_factory=list)
    stat: str = "fd"           # "linear" | "tf" | "fd" | "mb"
    T_K: float = 4.0
    m_eff: float = 1.08
    Ec0_eV: float = 0.56
    boxes: dict = field(default_factory=dict)
    # the full space charge of Eq. Poisson: holes and dopant ionization
    holes: bool = False
    ionization: str = "complete"   # "complete" | "incomplete"
    donors: np.ndarray = None      # [E] float64, nm^-3 (incomplete ionization)
    acceptors: np.ndarray = None   # [E] float64, nm^-3
    # interface-charge and Robin faces (list of Sheet)
    sheets: list = field(default_factory=list)
    # predictor-corrector electrons (QuantumStates) instead of n(phi)
    quantum: object = None

    @property
    def nx(self):
        return int(self.x.size)

    @property
    def ny(self):
        return int(self.y.size)

    @property
    def nz(self):
        return int(self.z.size)

    @property
    def n_nodes(self):
        return self.nx * self.ny * self.nz

    @property
    def n_elems(self):
        return (self.nx - 1) * (self.ny - 1) * (self.nz - 1)

    def contact_index(self, name):
        return self.contacts.index(name)


def stack_z(n_ez, si_nm=SI_NM, ox_nm=OX_NM):
    """Node z coordinates for ``n_ez`` element layers that put a node plane
    exactly on the Si/SiO2 interface: the oxide gets max(1, round(n_ez*ox/total))
    uniform layers, the silicon the rest."""
    n_ox = max(1, int(round(n_ez * ox_nm / (si_nm + ox_nm))))
    n_si = n_ez - n_ox
    if n_si < 1:
        raise ValueError("need at least two element layers")
    z_si = np.linspace(0.0, si_nm, n_si + 1)
    z_ox = np.linspace(si_nm, si_nm + ox_nm, n_ox + 1)[1:]
    return np.concatenate([z_si, z_ox])


def _bilinear(ctrl, pitch, xq, yq):
    """Bilinear interpolation of a control grid with uniform pitch starting at 0."""
    n = ctrl.shape[0]
    fx = np.clip(xq / pitch, 0.0, n - 1 - 1e-12)
    fy = np.clip(yq / pitch, 0.0, n - 1 - 1e-12)
    i = np.floor(fx).astype(np.int64)
    j = np.floor(fy).astype(np.int64)
    tx = fx - i
    ty = fy - j
    # ctrl indexed [ix, iy]
    return ((1 - tx) * (1 - ty) * ctrl[i, j] + tx * (1 - ty) * ctrl[i + 1, j]
            + (1 - tx) * ty * ctrl[i, j + 1] + tx * ty * ctrl[i + 1, j + 1])


def make_stack_device(name, x, y, z, gates, volts, stat="fd", T_K=4.0,
                      m_eff=1.08, Ec0_eV=0.56, interface=None,
                      net_doping_si=-NA_BULK_NM3, boxes=None,
                      bottom_contact=True, gate_tol=1e-9):
    """Lay out a Si substrate under an oxide with rectangular top gates.

    gates:  list of (name, (x0, x1, y0, y1)) on the top face (closed rectangles)
    volts:  gate voltages in the same order
    interface: None for a flat interface at z = 90 nm, else a callable
        (xc, yc) -> z_int; an element is oxide iff its centroid lies above it.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    nx, ny, nz = x.size, y.size, z.size
    xc = 0.5 * (x[1:] + x[:-1])
    yc = 0.5 * (y[1:] + y[:-1])
    zc = 0.5 * (z[1:] + z[:-1])
    ZC, YC, XC = np.meshgrid(zc, yc, xc, indexing="ij")     # [ez, ey, ex]
    if interface is None:
        zint = np.full_like(XC, SI_NM)
    else:
        zint = interface(XC, YC)
    oxide = ZC > zint
    semi = (~oxide).astype(np.uint8).ravel()
    eps_r = np.where(oxide, EPS_OX, EPS_SI).ravel().astype(np.float64)
    net = np.where(oxide, 0.0, net_doping_si).ravel().astype(np.float64)

    dir_id = np.full(nx * ny * nz, -1, dtype=np.int32)
    contacts = []
    dir_val = []
    top = nz - 1
    Y2, X2 = np.meshgrid(y, x, indexing="ij")           # [j, i]
    for g, (gname, (x0, x1, y0, y1)) in enumerate(gates):
        inside = ((X2 >= x0 - gate_tol) & (X2 <= x1 + gate_tol)
                  & (Y2 >= y0 - gate_tol) & (Y2 <= y1 + gate_tol))
        jj, ii = np.nonzero(inside)
        dir_id[ii + nx * (jj + ny * top)] = len(contacts)
        contacts.append(gname)
        dir_val.append(float(volts[g]))
    if bottom_contact:
        dir_id[: nx * ny] = len(contacts)
        contacts.append("bottom")
        dir_val.append(0.0)
    return Device(name=name, x=x, y=y, z=z, eps_r=eps_r, semi=semi,
                  net_doping=net, dir_id=dir_id,
                  dir_val=np.asarray(dir_val, dtype=np.float64),
                  contacts=contacts, stat=stat, T_K=T_K, m_eff=m_eff,
                  Ec0_eV=Ec0_eV, boxes=dict(boxes or {}))


def double_dot_gates():
    """Five 40 nm wide gates with 30 nm gaps in a 200x200 nm footprint:
    two plungers (P1, P2), a middle barrier (B2) between them and two long
    barriers (B1 above, B3 below).  Voltages are drawn in the order
    P1, P2, B1, B2, B3."""
    return [
        ("P1", (10.0, 50.0, 80.0, 120.0)),
        ("P2", (150.0, 190.0, 80.0, 120.0)),
        ("B1", (10.0, 190.0, 150.0, 190.0)),
        ("B2", (80.0, 120.0, 80.0, 120.0)),
        ("B3", (10.0, 190.0, 10.0, 50.0)),
    ]


def _uniform_xy(n):
    return np.linspace(0.0, BOX_XY_NM, n)


def config1():
    """17x17x9 nodes, two top gates, Thomas-Fermi electrons at 0 K."""
    rng = np.random.default_rng(SEED_BASE + 1)
    volts = rng.uniform(0.5, 1.5, 2)
    gates = [("G1", (30.0, 90.0, 50.0, 150.0)), ("G2", (110.0, 170.0, 50.0, 150.0))]
    return make_stack_device("c1", _uniform_xy(17), _uniform_xy(17), stack_z(8),
                             gates, volts, stat="tf", T_K=0.0,
                             boxes={"D1": DOT_BOX_D1, "D2": DOT_BOX_D2})


def double_dot_device(name, nx, ny, nz, volts, stat="fd", T_K=4.0):
    """The five-gate double-dot stack at an arbitrary node count."""
    return make_stack_device(name, _uniform_xy(nx), _uniform_xy(ny), stack_z(nz - 1),
                             double_dot_gates(), volts, stat=stat, T_K=T_K,
                             boxes={"D1": DOT_BOX_D1, "D2": DOT_BOX_D2})


def config2(nx=129, ny=129, nz=65):
    """Five-gate double-dot stack, Fermi-Dirac electrons at 4 K."""
    rng = np.random.default_rng(SEED_BASE + 2)
    volts = rng.uniform(0.0, 2.0, 5)
    return double_dot_device("c2", nx, ny, nz, volts)


PLUNGER_GRID = np.linspace(0.8, 1.6, 16)


def config3_spec(n_inst=256):
    """Mesh sizes and gate voltages of the batched plunger sweep.

    Returns (m[n_inst], volts[n_inst][5]); instance k has
    (m+1) x (m+1) x (m//2 + 1) nodes and plunger voltages on the 16x16 grid."""
    rng = np.random.default_rng(SEED_BASE + 3)
    ms = rng.integers(32, 65, size=n_inst)
    vb = rng.uniform(0.0, 2.0, 3)            # B1, B2, B3, shared by the sweep
    volts = np.empty((n_inst, 5))
    for k in range(n_inst):
        vp1 = PLUNGER_GRID[(k // 16) % 16]
        vp2 = PLUNGER_GRID[k % 16]
        volts[k] = (vp1, vp2, vb[0], vb[1], vb[2])
    return ms, volts


def config3_instance(k, spec=None):
    ms, volts = spec if spec is not None else config3_spec()
    m = int(ms[k])
    return double_dot_device(f"c3[{k}]", m + 1, m + 1, m // 2 + 1, volts[k])


def config4(nx=129, ny=129, nz=65):
    """The five-gate stack used for dot-charge gradients."""
    rng = np.random.default_rng(SEED_BASE + 4)
    volts = rng.uniform(0.0, 2.0, 5)
    return double_dot_device("c4", nx, ny, nz, volts)


def _random_gates(rng, n=8, min_gap=10.0, max_tries=10000):
    acc = []
    tries = 0
    while len(acc) < n and tries < max_tries:
        tries += 1
        w = rng.uniform(20.0, 60.0)
        l = rng.uniform(20.0, 60.0)
        x0 = rng.uniform(0.0, BOX_XY_NM - w)
        y0 = rng.uniform(0.0, BOX_XY_NM - l)
        r = (x0, x0 + w, y0, y0 + l)
        ok = True
        for a in acc:
            gx = max(0.0, max(r[0] - a[1], a[0] - r[1]))
            gy = max(0.0, max(r[2] - a[3], a[2] - r[3]))
            if max(gx, gy) < min_gap:
                ok = False
                break
        if ok:
            acc.append(r)
    return acc


def config5(nx=257, ny=257, nz=129):
    """Eight random top gates over an oxide with +-1 nm thickness roughness."""
    rng = np.random.default_rng(SEED_BASE + 5)
    ctrl = rng.uniform(-1.0, 1.0, (11, 11))
    rects = _random_gates(rng)
    volts = rng.uniform(0.0, 2.0, len(rects))
    gates = [(f"G{g + 1}", r) for g, r in enumerate(rects)]

    def interface(xq, yq):
        return SI_NM + _bilinear(ctrl, 20.0, xq, yq)

    return make_stack_device("c5", _uniform_xy(nx), _uniform_xy(ny), stack_z(nz - 1),
                             gates, volts, stat="fd", T_K=4.0, interface=interface,
                             boxes={"D1": DOT_BOX_D1, "D2": DOT_BOX_D2})


def doped_block(name, nx, ny, nz, size_nm, donors_fn, acceptors_fn, contacts, stat="mb", T_K=300.0,
                holes=True, ionization="complete"):
    """A silicon block with position-dependent doping and Ohmic contacts.

    size_nm: (Lx, Ly, Lz); donors_fn / acceptors_fn: callables of the element
    centroid (x, y, z) returning nm^-3; contacts: list of (name, face) with
    face one of "bottom", "top" -- every node of that face gets the contact's
    Dirichlet value, which the caller fills into ``dir_val`` (zeros here)."""
    Lx, Ly, Lz = size_nm
    x = np.linspace(0.0, Lx, nx)
    y = np.linspace(0.0, Ly, ny)
    z = np.linspace(0.0, Lz, nz)
    xc = 0.5 * (x[1:] + x[:-1])
    yc = 0.5 * (y[1:] + y[:-1])
    zc = 0.5 * (z[1:] + z[:-1])
    ZC, YC, XC = np.meshgrid(zc, yc, xc, indexing="ij")
    nd = np.asarray(donors_fn(XC, YC, ZC), dtype=np.float64).ravel() * np.ones(XC.size)
    na = np.asarray(acceptors_fn(XC, YC, ZC), dtype=np.float64).ravel() * np.ones(XC.size)
    E = XC.size
    dir_id = np.full(nx * ny * nz, -1, dtype=np.int32)
    names = []
    for c, (cname, face) in enumerate(contacts):
        k = 0 if face == "bottom" else nz - 1
        dir_id[k * nx * ny:(k + 1) * nx * ny] = c
        names.append(cname)
    return Device(name=name, x=x, y=y, z=z, eps_r=np.full(E, EPS_SI), semi=np.ones(E, dtype=np.uint8),
                  net_doping=nd - na, dir_id=dir_id, dir_val=np.zeros(len(contacts)), contacts=names,
                  stat=stat, T_K=T_K, holes=holes, ionization=ionization, donors=nd, acceptors=na)


def with_species(dev, donors_si=0.0, acceptors_si=NA_BULK_NM3, holes=True, ionization="incomplete"):
    """A copy of a gate-stack device with the full space charge switched on:
    holes, the chosen ionization model, and per-element donor / acceptor
    densities (nm^-3) in the silicon (zero in the oxide); net_doping becomes
    donors - acceptors.  Contact values are left as they are: the caller sets
    the Ohmic potential of the substrate contact."""
    from dataclasses import replace
    semi = np.asarray(dev.semi).astype(bool)
    nd = np.where(semi, donors_si, 0.0).astype(np.float64)
    na = np.where(semi, acceptors_si, 0.0).astype(np.float64)
    return replace(dev, holes=holes, ionization=ionization, donors=nd, acceptors=na,
                   net_doping=nd - na, dir_val=np.array(dev.dir_val, dtype=np.float64, copy=True))


def with_interface_charge(dev, sigma_nm2, z_nm=SI_NM, seed=None, spread=0.0):
    """A copy of a flat-interface stack with a surface charge on the Si/SiO2
    interface plane z = z_nm: sigma_nm2 per face, optionally varied by a
    seeded factor U[1 - spread, 1 + spread] per face."""
    from dataclasses import replace
    k = int(np.argmin(np.abs(dev.z - z_nm)))
    if abs(dev.z[k] - z_nm) > 1e-9:
        raise ValueError("the interface is not a mesh plane")
    na, nb = dev.nx - 1, dev.ny - 1
    sig = np.full(na * nb, float(sigma_nm2))
    if spread:
        sig *= np.random.default_rng(seed).uniform(1.0 - spread, 1.0 + spread, sig.size)
    sh = Sheet(axis=2, plane=k, a0=0, a1=na, b0=0, b1=nb, sigma=sig)
    return replace(dev, sheets=list(dev.sheets) + [sh])


def with_charged_gates(dev, gates, sigma_nm2=0.0, d_nm=10.0, eps_r=EPS_OX, gate_tol=1e-9):
    """A copy of a stack whose top gates are Robin faces instead of Dirichlet
    nodes: each gate rectangle becomes a sheet on the top plane with its
    voltage as phi0, a charge sigma_nm2 per face and the pinned plane d_nm
    away through a layer of relative permittivity eps_r; its nodes become
    free.  gates: the (name, (x0, x1, y0, y1)) list the device was built with."""
    from dataclasses import replace
    dir_id = dev.dir_id.copy()
    sheets = list(dev.sheets)
    top = dev.nz - 1
    for gname, (x0, x1, y0, y1) in gates:
        ii = np.nonzero((dev.x >= x0 - gate_tol) & (dev.x <= x1 + gate_tol))[0]
        jj = np.nonzero((dev.y >= y0 - gate_tol) & (dev.y <= y1 + gate_tol))[0]
        c = dev.contacts.index(gname)
        J, I = np.meshgrid(jj, ii, indexing="ij")
        dir_id[(I + dev.nx * (J + dev.ny * top)).ravel()] = -1
        na, nb = ii[-1] - ii[0], jj[-1] - jj[0]
        sheets.append(Sheet(axis=2, plane=top, a0=int(ii[0]), a1=int(ii[-1]), b0=int(jj[0]), b1=int(jj[-1]),
                            sigma=np.full(na * nb, float(sigma_nm2)), robin_d=d_nm, robin_eps=eps_r,
                            phi0=float(dev.dir_val[c])))
    return replace(dev, dir_id=dir_id, sheets=sheets)


def box_states(dev, box, n_states, phi_k, seed=None, e0=-0.004, spacing=0.002):
    """Synthetic 3D-confined states in a box (x0, x1, y0, y1, z0, z1) nm: the
    standing waves of a hard-walled box, |psi|^2 = (8/V) prod sin^2(pi m (s -
    s0)/L) (normalised in the continuum), zero outside; modes taken in order
    of m_x^2/Lx^2 + m_y^2/Ly^2 + m_z^2/Lz^2.  Levels: e0, then seeded steps
    of spacing * U[0.5, 1.5] (eV relative to E_F)."""
    x0, x1, y0, y1, z0, z1 = box
    L = np.array([x1 - x0, y1 - y0, z1 - z0])
    modes = sorted(((mx, my, mz) for mx in range(1, 6) for my in range(1, 6) for mz in range(1, 4)),
                   key=lambda m: (m[0] / L[0]) ** 2 + (m[1] / L[1]) ** 2 + (m[2] / L[2]) ** 2)[:n_states]
    Z, Y, X = np.meshgrid(dev.z, dev.y, dev.x, indexing="ij")
    X, Y, Z = X.ravel(), Y.ravel(), Z.ravel()
    inside = (X >= x0) & (X <= x1) & (Y >= y0) & (Y <= y1) & (Z >= z0) & (Z <= z1)
    psi2 = np.zeros((n_states, X.size))
    for i, (mx, my, mz) in enumerate(modes):
        f = (np.sin(np.pi * mx * (X - x0) / L[0]) * np.sin(np.pi * my * (Y - y0) / L[1])
             * np.sin(np.pi * mz * (Z - z0) / L[2])) ** 2 * 8.0 / np.prod(L)
        psi2[i] = np.where(inside, f, 0.0)
    rng = np.random.default_rng(seed)
    E = e0 + np.concatenate([[0.0], np.cumsum(spacing * rng.uniform(0.5, 1.5, n_states - 1))])
    return QuantumStates(psi2=psi2, phi_k=np.asarray(phi_k, dtype=np.float64).copy(), E_i=E)


def with_quantum(dev, states):
    """A copy of a device whose electrons come from the given states."""
    from dataclasses import replace
    return replace(dev, quantum=states)


SIO2_CB_OFFSET_EV = 3.1          # Si/SiO2 conduction-band offset
M_SI_T, M_SI_L, M_OX = 0.19, 0.98, 0.5   # effective masses (m0): Si transverse and longitudinal, SiO2


def quantum_region(dev, box, isotropic=False):
    """Inputs of the Schrodinger step for a quantum region `box` (x0, x1, y0,
    y1, z0, z1) nm of a gate stack: per-element m0/m* along x, y, z ([3, E]:
    the Delta_2 valleys' m_t, m_t, m_l in Si with the interface normal to z,
    isotropic in the oxide), the conduction-band edge at phi = 0 (Ec0 in Si,
    Ec0 + the band offset in the oxide), the fixed nodes (psi = 0: every
    node not strictly inside the box) and the region's elements (centroid
    strictly inside).  isotropic=True gives m_t along every axis."""
    x0, x1, y0, y1, z0, z1 = box
    ox = np.asarray(dev.semi) == 0
    v0 = np.where(ox, dev.Ec0_eV + SIO2_CB_OFFSET_EV, dev.Ec0_eV).astype(np.float64)
    m_z = M_SI_T if isotropic else M_SI_L
    inv_mass = np.stack([np.where(ox, 1.0 / M_OX, 1.0 / M_SI_T), np.where(ox, 1.0 / M_OX, 1.0 / M_SI_T),
                         np.where(ox, 1.0 / M_OX, 1.0 / m_z)]).astype(np.float64)
    Z, Y, X = np.meshgrid(dev.z, dev.y, dev.x, indexing="ij")
    inside = (X > x0) & (X < x1) & (Y > y0) & (Y < y1) & (Z > z0) & (Z < z1)
    xc, yc, zc = [0.5 * (c[1:] + c[:-1]) for c in (dev.x, dev.y, dev.z)]
    Zc, Yc, Xc = np.meshgrid(zc, yc, xc, indexing="ij")
    region = (Xc > x0) & (Xc < x1) & (Yc > y0) & (Yc < y1) & (Zc > z0) & (Zc < z1)
    return inv_mass, v0, ~inside.ravel(), region.ravel()
