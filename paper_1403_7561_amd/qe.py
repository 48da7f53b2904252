"""Thin ctypes binding of the C ABI in include/qe.h.

Each ``qe_*`` function here marshals torch device tensors into the C structs
and calls the function of the same name in ``libqe.so``; every step of the
computation runs in the HIP kernels behind it.  PyTorch only provides device
memory and the current stream.  There is no fallback: if the library or a
GPU is missing, the call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("QE_LIB_PATH") or os.path.join(HERE, "libqe.so")

QE_OK = 0
STATUS_NAMES = {
    0: "OK", -1: "INVALID_ARG", -2: "HIP", -3: "WORKSPACE", -4: "NOT_CONVERGED",
    -5: "LINESEARCH", -6: "KRYLOV_BREAKDOWN", -7: "NONFINITE", -8: "KRYLOV_MAXIT",
}
STAT = {"linear": 0, "tf": 1, "fd": 2, "mb": 3}
IONIZATION = {"complete": 0, "incomplete": 1}
PREC = {"fp64": 0, "mixed": 1}

EXPORTED = [
    "qe_default_options", "qe_workspace_bytes", "qe_solve", "qe_solve_static", "qe_residual", "qe_jv",
    "qe_jv_f32", "qe_count_electrons", "qe_density", "qe_adjoint",
    "qe_batch_workspace_bytes", "qe_solve_batch", "qe_time_jv", "qe_ohmic_potential",
    "qe_schrodinger_workspace_bytes", "qe_schrodinger_solve", "qe_last_error",
]

# Silicon parameters of Sec. II.A.3: band gap, phosphorus / boron ionization
# energies, ground-state degeneracies, and the valence DOS mass from the heavy
# and light holes (Eq. EffectiveMass: m_h^(3/2) = m_hh^(3/2) + m_lh^(3/2)).
SI_EG_EV, SI_ED_EV, SI_EA_EV, SI_GD, SI_GA = 1.12, 0.046, 0.044, 2.0, 4.0
SI_M_H = (0.49 ** 1.5 + 0.16 ** 1.5) ** (2.0 / 3.0)


class QeError(RuntimeError):
    def __init__(self, status, msg, report=None):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
        self.report = report


class CSheet(ctypes.Structure):
    _fields_ = [("axis", ctypes.c_int32), ("plane", ctypes.c_int32), ("a0", ctypes.c_int32),
                ("a1", ctypes.c_int32), ("b0", ctypes.c_int32), ("b1", ctypes.c_int32),
                ("sigma", ctypes.c_void_p), ("robin_d", ctypes.c_double), ("robin_eps", ctypes.c_double),
                ("phi0", ctypes.c_double)]


class CQuantum(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_int32), ("confinement", ctypes.c_int32), ("psi2", ctypes.c_void_p),
                ("phi_k", ctypes.c_void_p), ("E_i", ctypes.POINTER(ctypes.c_double)), ("m_t", ctypes.c_double),
                ("region", ctypes.c_void_p)]


class CSchrodinger(ctypes.Structure):
    _fields_ = [("inv_mass", ctypes.c_void_p), ("v0", ctypes.c_void_p), ("fixed", ctypes.c_void_p)]


class CProblem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("eps_r", ctypes.c_void_p), ("semi", ctypes.c_void_p),
                ("net_doping", ctypes.c_void_p), ("dir_id", ctypes.c_void_p),
                ("dir_val", ctypes.c_void_p), ("n_dir", ctypes.c_int32),
                ("donors", ctypes.c_void_p), ("acceptors", ctypes.c_void_p),
                ("n_sheets", ctypes.c_int32), ("sheets", ctypes.POINTER(CSheet)),
                ("quantum", ctypes.POINTER(CQuantum))]


class CPhysics(ctypes.Structure):
    _fields_ = [("stat", ctypes.c_int32), ("T_K", ctypes.c_double),
                ("m_eff", ctypes.c_double), ("Ec0_eV", ctypes.c_double),
                ("holes", ctypes.c_int32), ("m_h", ctypes.c_double), ("Eg_eV", ctypes.c_double),
                ("ionization", ctypes.c_int32), ("Ed_eV", ctypes.c_double), ("Ea_eV", ctypes.c_double),
                ("gD", ctypes.c_double), ("gA", ctypes.c_double)]


class COptions(ctypes.Structure):
    _fields_ = [("newton_atol", ctypes.c_double), ("newton_maxit", ctypes.c_int32),
                ("ls_max_halvings", ctypes.c_int32), ("krylov_rtol_max", ctypes.c_double),
                ("krylov_maxit", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("init_guess", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("precond", ctypes.c_int32)]


class CReport(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("newton_iters", ctypes.c_int32),
                ("krylov_iters", ctypes.c_int32), ("ls_halvings", ctypes.c_int32),
                ("init_krylov_iters", ctypes.c_int32), ("n_residual_evals", ctypes.c_int32),
                ("res0", ctypes.c_double), ("res_final", ctypes.c_double), ("seq_levels", ctypes.c_int32),
                ("mg_levels", ctypes.c_int32), ("mg_krylov_iters", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path=LIB_PATH):
    """Load libqe.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1403_7561_amd.build`")
    lib = ctypes.CDLL(path)
    P, V, S, D, I32 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_double, ctypes.c_int32
    pp, pph, po, pr = P(CProblem), P(CPhysics), P(COptions), P(CReport)
    sig = {
        "qe_default_options": (None, [po]),
        "qe_workspace_bytes": (S, [pp, po]),
        "qe_solve": (I32, [pp, pph, po, V, V, V, S, V, pr]),
        "qe_solve_static": (I32, [pp, pph, po, V, V, V, pr]),
        "qe_residual": (I32, [pp, pph, V, V, V, P(D), V, S, V]),
        "qe_jv": (I32, [pp, pph, V, V, V, V, S, V]),
        "qe_jv_f32": (I32, [pp, pph, V, V, V, V, S, V]),
        "qe_count_electrons": (I32, [pp, pph, V, I32, P(D), P(D), V, S, V]),
        "qe_density": (I32, [pp, pph, V, V, V, S, V]),
        "qe_adjoint": (I32, [pp, pph, po, V, P(D), P(D), P(D), V, V, V, S, V, pr]),
        "qe_batch_workspace_bytes": (S, [I32, pp, po]),
        "qe_solve_batch": (I32, [I32, pp, pph, po, P(V), I32, P(D), P(D), ctypes.c_char_p,
                                 V, S, V, pr]),
        "qe_time_jv": (I32, [pp, pph, V, V, I32, I32, P(D), P(ctypes.c_int64), V, S, V]),
        "qe_ohmic_potential": (I32, [pph, D, D, D, P(D)]),
        "qe_schrodinger_workspace_bytes": (S, [pp, I32]),
        "qe_schrodinger_solve": (I32, [pp, P(CSchrodinger), V, I32, D, I32, ctypes.c_uint64, I32, P(D), V, V,
                                       P(I32), V, S, V]),
        "qe_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def qe_last_error():
    return load_library().qe_last_error().decode()


def _check(status, report=None):
    if status != QE_OK:
        raise QeError(status, qe_last_error(), report)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the HIP library needs a GPU (torch.cuda.is_available() is False)")
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _device(device):
    """torch.device with the index resolved (a bare "cuda" is the current one)."""
    import torch
    d = torch.device(device)
    if d.type == "cuda" and d.index is None:
        d = torch.device("cuda", torch.cuda.current_device())
    return d


def _dev(t, dtype, n, device, name):
    """t itself if it is a contiguous tensor of exactly ``dtype`` with ``n``
    entries on ``device``; anything else raises ValueError before the library
    is called (the kernels trust every pointer and length they are given)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    d = _device(device)
    if t.device.type != d.type or (d.index is not None and t.device.index != d.index):
        raise ValueError(f"{name}: tensor on {t.device}, the problem is on {d}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if t.numel() != n:
        raise ValueError(f"{name}: {t.numel()} entries, expected {n}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: not contiguous")
    return t


@dataclass
class Physics:
    stat: str = "fd"
    T_K: float = 4.0
    m_eff: float = 1.08
    Ec0_eV: float = 0.56
    holes: bool = False
    m_h: float = SI_M_H
    Eg_eV: float = SI_EG_EV
    ionization: str = "complete"
    Ed_eV: float = SI_ED_EV
    Ea_eV: float = SI_EA_EV
    gD: float = SI_GD
    gA: float = SI_GA

    def c(self):
        return CPhysics(STAT[self.stat], float(self.T_K), float(self.m_eff), float(self.Ec0_eV),
                        int(bool(self.holes)), float(self.m_h), float(self.Eg_eV),
                        IONIZATION[self.ionization], float(self.Ed_eV), float(self.Ea_eV),
                        float(self.gD), float(self.gA))

    @classmethod
    def of(cls, dev):
        return cls(dev.stat, dev.T_K, dev.m_eff, dev.Ec0_eV, holes=bool(getattr(dev, "holes", False)),
                   ionization=getattr(dev, "ionization", "complete"))


def qe_default_options(**over):
    o = COptions()
    load_library().qe_default_options(ctypes.byref(o))
    for k, v in over.items():
        if k == "precision" and isinstance(v, str):
            v = PREC[v]
        setattr(o, k, v)
    return o


class Problem:
    """Device copies of one device's arrays plus the C struct pointing at them."""

    def __init__(self, dev, device="cuda"):
        torch = _torch()
        f64 = dict(dtype=torch.float64, device=device)
        self.nx, self.ny, self.nz = dev.nx, dev.ny, dev.nz
        self.N, self.E = dev.n_nodes, dev.n_elems
        self.x = torch.as_tensor(np.ascontiguousarray(dev.x), **f64)
        self.y = torch.as_tensor(np.ascontiguousarray(dev.y), **f64)
        self.z = torch.as_tensor(np.ascontiguousarray(dev.z), **f64)
        self.eps_r = torch.as_tensor(np.ascontiguousarray(dev.eps_r), **f64)
        self.semi = torch.as_tensor(np.ascontiguousarray(dev.semi, dtype=np.uint8), device=device)
        self.net_doping = torch.as_tensor(np.ascontiguousarray(dev.net_doping), **f64)
        self.dir_id = torch.as_tensor(np.ascontiguousarray(dev.dir_id, dtype=np.int32), device=device)
        dv = np.ascontiguousarray(dev.dir_val, dtype=np.float64)
        self.dir_val = torch.as_tensor(dv if dv.size else np.zeros(1), **f64)
        self.n_dir = int(dv.size)
        nd, na = getattr(dev, "donors", None), getattr(dev, "acceptors", None)
        self.donors = None if nd is None else torch.as_tensor(np.ascontiguousarray(nd, dtype=np.float64), **f64)
        self.acceptors = None if na is None else torch.as_tensor(np.ascontiguousarray(na, dtype=np.float64), **f64)
        self.physics = Physics.of(dev) if hasattr(dev, "stat") else Physics()
        # interface-charge / Robin sheets: host descriptors, sigma on the device
        sheets = list(getattr(dev, "sheets", None) or [])
        self.sheet_sigma = [None if sh.sigma is None else
                            torch.as_tensor(np.ascontiguousarray(sh.sigma, dtype=np.float64), **f64)
                            for sh in sheets]
        self.c_sheets = (CSheet * max(len(sheets), 1))()
        for i, sh in enumerate(sheets):
            sg = self.sheet_sigma[i]
            self.c_sheets[i] = CSheet(int(sh.axis), int(sh.plane), int(sh.a0), int(sh.a1), int(sh.b0), int(sh.b1),
                                      sg.data_ptr() if sg is not None else None, float(sh.robin_d),
                                      float(sh.robin_eps), float(sh.phi0))
        self.n_sheets = len(sheets)
        self.device = _device(device)
        self._set_quantum(getattr(dev, "quantum", None))

    def _set_quantum(self, q):
        """Predictor-corrector states: |psi|^2 and phi^(k) on the device (a
        float64 device tensor is used as it is, arrays are copied), levels on
        the host."""
        torch = _torch()
        f64 = dict(dtype=torch.float64, device=self.device)

        def dev64(a):
            if hasattr(a, "data_ptr"):
                return a.to(**f64).contiguous()
            return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), **f64)

        self.c_quantum = None
        if q is None:
            return
        self.q_psi2 = dev64(q.psi2)
        self.q_phik = dev64(q.phi_k)
        E = np.ascontiguousarray(q.E_i, dtype=np.float64)
        _dev(self.q_psi2, torch.float64, E.size * self.N, self.device, "quantum psi2 [n_states, N]")
        _dev(self.q_phik, torch.float64, self.N, self.device, "quantum phi_k")
        self.q_E = (ctypes.c_double * E.size)(*E.tolist())
        reg = getattr(q, "region", None)
        if reg is None:
            self.q_region = None
        elif hasattr(reg, "data_ptr"):
            self.q_region = reg.to(dtype=torch.uint8, device=self.device).contiguous()
        else:
            self.q_region = torch.as_tensor(np.ascontiguousarray(reg, dtype=np.uint8), device=self.device)
        if self.q_region is not None:
            _dev(self.q_region, torch.uint8, self.E, self.device, "quantum region")
        self.c_quantum = CQuantum(int(E.size), int(q.confinement), self.q_psi2.data_ptr(),
                                  self.q_phik.data_ptr(), self.q_E, float(q.m_t),
                                  self.q_region.data_ptr() if self.q_region is not None else None)

    def with_quantum(self, q):
        """The same problem (its device arrays shared, not copied) with the
        electrons of the quantum region taken from the states q."""
        import copy
        o = copy.copy(self)
        o._set_quantum(q)
        return o

    def c(self):
        return CProblem(self.nx, self.ny, self.nz, self.x.data_ptr(), self.y.data_ptr(),
                        self.z.data_ptr(), self.eps_r.data_ptr(), self.semi.data_ptr(),
                        self.net_doping.data_ptr() if self.net_doping is not None else None,
                        self.dir_id.data_ptr(),
                        self.dir_val.data_ptr(), self.n_dir,
                        self.donors.data_ptr() if self.donors is not None else None,
                        self.acceptors.data_ptr() if self.acceptors is not None else None,
                        self.n_sheets, self.c_sheets if self.n_sheets else None,
                        ctypes.pointer(self.c_quantum) if self.c_quantum is not None else None)


class Workspace:
    """Caller-owned device scratch sized by qe_workspace_bytes."""

    def __init__(self, nbytes, device="cuda"):
        torch = _torch()
        self.t = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)
        base = self.t.data_ptr()
        self.off = (-base) % 256
        self.ptr = ctypes.c_void_p(base + self.off)
        self.nbytes = int(nbytes)


def qe_workspace_bytes(prob, opts=None):
    o = opts if opts is not None else qe_default_options()
    cp = prob.c()
    return int(load_library().qe_workspace_bytes(ctypes.byref(cp), ctypes.byref(o)))


def workspace_for(prob, opts=None):
    return Workspace(qe_workspace_bytes(prob, opts), prob.device)


def qe_solve(prob, phys=None, opts=None, phi=None, want_density=True, ws=None, check=True):
    """Solve; returns (phi, n_nodal or None, report dict)."""
    torch = _torch()
    lib = load_library()
    phys = phys or prob.physics
    o = opts if opts is not None else qe_default_options()
    if phi is None:
        phi = torch.zeros(prob.N, dtype=torch.float64, device=prob.device)
    _dev(phi, torch.float64, prob.N, prob.device, "phi")
    n = torch.empty(prob.N, dtype=torch.float64, device=prob.device) if want_density else None
    ws = ws or workspace_for(prob, o)
    cp, cph, rep = prob.c(), phys.c(), CReport()
    st = lib.qe_solve(ctypes.byref(cp), ctypes.byref(cph), ctypes.byref(o), _ptr(phi), _ptr(n),
                      ws.ptr, ws.nbytes, _stream(), ctypes.byref(rep))
    if check:
        _check(st, rep.as_dict())
    return phi, n, rep.as_dict()


def qe_solve_static(prob, phi, n=None, phys=None, opts=None, check=True):
    """qe_solve on the library's static workspace, for callers that cannot
    allocate: phi (device, float64 [N]) holds the guess when opts.init_guess
    = 1 and receives the solution; n (device [N] or None) the nodal density.
    The call itself allocates nothing; returns the report dict."""
    torch = _torch()
    lib = load_library()
    phys = phys or prob.physics
    o = opts if opts is not None else qe_default_options()
    _dev(phi, torch.float64, prob.N, prob.device, "phi")
    if n is not None:
        _dev(n, torch.float64, prob.N, prob.device, "n")
    cp, cph, rep = prob.c(), phys.c(), CReport()
    st = lib.qe_solve_static(ctypes.byref(cp), ctypes.byref(cph), ctypes.byref(o), _ptr(phi), _ptr(n), _stream(),
                             ctypes.byref(rep))
    if check:
        _check(st, rep.as_dict())
    return rep.as_dict()


def qe_residual(prob, phi, phys=None, ws=None, want_diag=True):
    torch = _torch()
    lib = load_library()
    phys = phys or prob.physics
    _dev(phi, torch.float64, prob.N, prob.device, "phi")
    F = torch.empty(prob.N, dtype=torch.float64, device=prob.device)
    d = torch.empty_like(F) if want_diag else None
    n2 = ctypes.c_double(0.0)
    ws = ws or workspace_for(prob)
    cp, cph = prob.c(), phys.c()
    _check(lib.qe_residual(ctypes.byref(cp), ctypes.byref(cph), _ptr(phi), _ptr(F), _ptr(d),
                           ctypes.byref(n2), ws.ptr, ws.nbytes, _stream()))
    return F, d, n2.value


def qe_jv(prob, phi, v, phys=None, ws=None):
    torch = _torch()
    lib = load_library()
    phys = phys or prob.physics
    _dev(phi, torch.float64, prob.N, prob.device, "phi")
    if getattr(v, "dtype", None) not in (torch.float64, torch.float32):
        raise ValueError(f"v: dtype {getattr(v, 'dtype', type(v).__name__)}, expected torch.float64 (qe_jv) "
                         "or torch.float32 (qe_jv_f32)")
    _dev(v, v.dtype, prob.N, prob.device, "v")
    y = torch.empty_like(v)
    ws = ws or workspace_for(prob)
    cp, cph = prob.c(), phys.c()
    fn = lib.qe_jv if v.dtype == torch.float64 else lib.qe_jv_f32
    _check(fn(ctypes.byref(cp), ctypes.byref(cph), _ptr(phi), _ptr(v), _ptr(y), ws.ptr,
              ws.nbytes, _stream()))
    return y


def qe_jv_f32(prob, phi, v32, phys=None, ws=None):
    return qe_jv(prob, phi, v32, phys, ws)


def qe_count_electrons(prob, phi, boxes, phys=None, ws=None):
    torch = _torch()
    lib = load_library()
    phys = phys or prob.physics
    _dev(phi, torch.float64, prob.N, prob.device, "phi")
    b = np.ascontiguousarray(np.asarray(boxes, dtype=np.float64).reshape(-1, 6))
    out = np.zeros(b.shape[0])
    ws = ws or workspace_for(prob)
    cp, cph = prob.c(), phys.c()
    P = ctypes.POINTER(ctypes.c_double)
    _check(lib.qe_count_electrons(ctypes.byref(cp), ctypes.byref(cph), _ptr(phi), b.shape[0],
                                  b.ctypes.data_as(P), out.ctypes.data_as(P), ws.ptr, ws.nbytes,
                                  _stream()))
    return out


def qe_density(prob, phi, phys=None, ws=None):
    torch = _torch()
    lib = load_library()
    phys = phys or prob.physics
    _dev(phi, torch.float64, prob.N, prob.device, "phi")
    n = torch.empty(prob.N, dtype=torch.float64, device=prob.device)
    ws = ws or workspace_for(prob)
    cp, cph = prob.c(), phys.c()
    _check(lib.qe_density(ctypes.byref(cp), ctypes.byref(cph), _ptr(phi), _ptr(n), ws.ptr,
                          ws.nbytes, _stream()))
    return n


def qe_adjoint(prob, phi, box, phys=None, opts=None, ws=None, want_eps=True, want_lam=False,
               check=True):
    """Returns (Q, dQ/dV per Dirichlet value [numpy], dQ/deps [device] or None,
    lam [device] or None, report)."""
    torch = _torch()
    lib = load_library()
    phys = phys or prob.physics
    o = opts if opts is not None else qe_default_options()
    _dev(phi, torch.float64, prob.N, prob.device, "phi")
    b = np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(6))
    dV = np.zeros(max(prob.n_dir, 1))
    Q = ctypes.c_double(0.0)
    deps = torch.empty(prob.E, dtype=torch.float64, device=prob.device) if want_eps else None
    lam = torch.empty(prob.N, dtype=torch.float64, device=prob.device) if want_lam else None
    ws = ws or workspace_for(prob, o)
    cp, cph, rep = prob.c(), phys.c(), CReport()
    P = ctypes.POINTER(ctypes.c_double)
    st = lib.qe_adjoint(ctypes.byref(cp), ctypes.byref(cph), ctypes.byref(o), _ptr(phi),
                        b.ctypes.data_as(P), ctypes.byref(Q), dV.ctypes.data_as(P), _ptr(deps),
                        _ptr(lam), ws.ptr, ws.nbytes, _stream(), ctypes.byref(rep))
    if check:
        _check(st, rep.as_dict())
    return Q.value, dV[:prob.n_dir], deps, lam, rep.as_dict()


def qe_time_jv(prob, phi, v, precision="fp64", reps=200, phys=None, ws=None):
    """Mean time (ms) of one CG J.v kernel launch, measured with HIP events,
    and the number of elements whose Gauss-point coefficients it reads."""
    torch = _torch()
    lib = load_library()
    phys = phys or prob.physics
    _dev(phi, torch.float64, prob.N, prob.device, "phi")
    _dev(v, torch.float64, prob.N, prob.device, "v")
    ms = ctypes.c_double(0.0)
    ncoef = ctypes.c_int64(0)
    ws = ws or workspace_for(prob)
    cp, cph = prob.c(), phys.c()
    _check(lib.qe_time_jv(ctypes.byref(cp), ctypes.byref(cph), _ptr(phi), _ptr(v), PREC[precision],
                          int(reps), ctypes.byref(ms), ctypes.byref(ncoef), ws.ptr, ws.nbytes, _stream()))
    return ms.value, int(ncoef.value)


def qe_batch_workspace_bytes(probs, opts=None):
    o = opts if opts is not None else qe_default_options()
    arr = (CProblem * len(probs))(*[p.c() for p in probs])
    return int(load_library().qe_batch_workspace_bytes(len(probs), arr, ctypes.byref(o)))


def qe_solve_batch(probs, phys=None, opts=None, phis=None, boxes=(), tune_cache=None, ws=None,
                   check=True):
    """Solve many devices in one persistent launch.  Returns (phis, counts
    [n_inst, n_boxes], reports)."""
    torch = _torch()
    lib = load_library()
    phys = phys or probs[0].physics
    o = opts if opts is not None else qe_default_options()
    n = len(probs)
    if phis is None:
        phis = [torch.zeros(p.N, dtype=torch.float64, device=p.device) for p in probs]
    if len(phis) != n:
        raise ValueError(f"phis: {len(phis)} tensors for {n} problems")
    for k, (p, ph) in enumerate(zip(probs, phis)):
        _dev(ph, torch.float64, p.N, p.device, f"phis[{k}]")
    arr = (CProblem * n)(*[p.c() for p in probs])
    ptrs = (ctypes.c_void_p * n)(*[ph.data_ptr() for ph in phis])
    b = np.ascontiguousarray(np.asarray(boxes, dtype=np.float64).reshape(-1, 6))
    counts = np.zeros((n, max(b.shape[0], 1)))
    reps = (CReport * n)()
    if ws is None:
        ws = Workspace(qe_batch_workspace_bytes(probs, o), probs[0].device)
    P = ctypes.POINTER(ctypes.c_double)
    cph = phys.c()
    path = tune_cache.encode() if tune_cache else None
    st = lib.qe_solve_batch(n, arr, ctypes.byref(cph), ctypes.byref(o), ptrs, b.shape[0],
                            b.ctypes.data_as(P), counts.ctypes.data_as(P), path, ws.ptr,
                            ws.nbytes, _stream(), reps)
    rlist = [reps[i].as_dict() for i in range(n)]
    if check:
        _check(st, rlist)
    return phis, counts[:, : b.shape[0]], rlist


def qe_ohmic_potential(phys, N_D, N_A, V_a=0.0):
    """Dirichlet potential (V) of an Ohmic contact with donor / acceptor
    densities N_D, N_A (nm^-3) at applied voltage V_a (host computation)."""
    out = ctypes.c_double()
    _check(load_library().qe_ohmic_potential(ctypes.byref(phys.c()), float(N_D), float(N_A), float(V_a),
                                              ctypes.byref(out)))
    return out.value


def qe_schrodinger_solve(prob, inv_mass, v0, phi, n_states, fixed=None, tol=1e-8, maxit=500, seed=1,
                         want_psi2=True, ws=None, check=True, guess=None):
    """Lowest eigenpairs of the effective-mass Schrodinger problem on the
    problem's mesh: V = v0_e - phi.  inv_mass: m0/m* per element, [E]
    (isotropic) or [3, E] (along x, y, z: a diagonal mass tensor); v0: per
    element (eV); fixed: per node booleans (psi = 0) or None; guess: device
    [n, N] starting vectors or None.  Returns (E [n] eV, psi [n, N], psi2
    [n, N] or None, iterations)."""
    im_h = np.asarray(inv_mass, dtype=np.float64)
    if im_h.shape == (prob.E,):
        im_h = np.stack([im_h, im_h, im_h])
    if im_h.shape != (3, prob.E):
        raise ValueError(f"inv_mass: shape {im_h.shape}, expected ({prob.E},) or (3, {prob.E})")
    torch = _torch()
    lib = load_library()
    f64 = dict(dtype=torch.float64, device=prob.device)
    im = torch.as_tensor(np.ascontiguousarray(im_h), **f64)
    vv = torch.as_tensor(np.ascontiguousarray(v0, dtype=np.float64), **f64)
    fx = None if fixed is None else torch.as_tensor(np.ascontiguousarray(fixed, dtype=np.uint8), device=prob.device)
    ph = phi if hasattr(phi, "data_ptr") else torch.as_tensor(np.ascontiguousarray(phi, dtype=np.float64), **f64)
    _dev(ph, torch.float64, prob.N, prob.device, "phi")
    _dev(im, torch.float64, 3 * prob.E, prob.device, "inv_mass [3, E]")
    _dev(vv, torch.float64, prob.E, prob.device, "v0")
    if fx is not None:
        _dev(fx, torch.uint8, prob.N, prob.device, "fixed")
    if guess is not None:
        _dev(guess, torch.float64, int(n_states) * prob.N, prob.device, "guess [n_states, N]")
    cp = prob.c()
    cs = CSchrodinger(im.data_ptr(), vv.data_ptr(), fx.data_ptr() if fx is not None else None)
    if ws is None:
        ws = Workspace(lib.qe_schrodinger_workspace_bytes(ctypes.byref(cp), int(n_states)), prob.device)
    E = np.zeros(int(n_states))
    psi = torch.empty((int(n_states), prob.N), **f64) if guess is None else guess.clone()
    psi2 = torch.empty((int(n_states), prob.N), **f64) if want_psi2 else None
    it = ctypes.c_int32(0)
    st = lib.qe_schrodinger_solve(ctypes.byref(cp), ctypes.byref(cs), _ptr(ph), int(n_states), float(tol),
                                  int(maxit), ctypes.c_uint64(int(seed)), int(guess is not None),
                                  E.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(psi), _ptr(psi2),
                                  ctypes.byref(it), ws.ptr, ws.nbytes, _stream())
    if check:
        _check(st)
    return E, psi, psi2, it.value
