"""Host-side checks of the C ABI (no kernel is launched): the library loads,
exports every function include/qe.h declares, and rejects bad arguments with
the documented status codes before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1403_7561_amd import qe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "qe.h")) as fh:
        src = fh.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qe_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = qe.load_library()
    names = declared_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(qe.EXPORTED) == names


def test_default_options():
    o = qe.qe_default_options()
    assert o.newton_atol == 1e-8 and o.newton_maxit == 100 and o.ls_max_halvings == 30
    assert o.precision == 0 and o.init_guess == 2
    assert o.precond == 0          # QE_PC_AUTO


def test_report_layout_matches_the_header():
    """The binding's report struct ends with the fields include/qe.h declares
    last (the multigrid counts after the sequence's level count)."""
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "qe.h")).read()

    def fields(struct):
        body = hdr[:hdr.index("} %s;" % struct)]
        body = body[body.rindex("typedef struct {"):]
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        return re.findall(r"\b(\w+)\s*;", body)

    assert [f for f, _ in qe.CReport._fields_] == fields("qe_report")
    assert [f for f, _ in qe.COptions._fields_] == fields("qe_options")
    assert fields("qe_report")[-2:] == ["mg_levels", "mg_krylov_iters"]


def fake_problem(nx=4, ny=3, nz=2, n_dir=1):
    # pointers are never dereferenced: every call below fails host-side validation first
    return qe.CProblem(nx, ny, nz, 16, 16, 16, 16, 16, 16, 16, 16 if n_dir else 0, n_dir)


@pytest.mark.parametrize("mut,needle", [
    (dict(nx=1), "nx, ny, nz >= 2"),
    (dict(nz=0), "nx, ny, nz >= 2"),
    (dict(eps_r=0), "NULL array"),
    (dict(dir_id=0), "NULL array"),
    (dict(n_dir=-1), "n_dir < 0"),
    (dict(dir_val=0), "dir_val is NULL"),
])
def test_invalid_problem_rejected(mut, needle):
    lib = qe.load_library()
    p = fake_problem()
    for k, v in mut.items():
        setattr(p, k, v)
    o = qe.qe_default_options()
    ph = qe.CPhysics(2, 4.0, 1.08, 0.56)
    rep = qe.CReport()
    st = lib.qe_solve(ctypes.byref(p), ctypes.byref(ph), ctypes.byref(o), ctypes.c_void_p(16),
                      None, ctypes.c_void_p(256), 1 << 40, None, ctypes.byref(rep))
    assert st == -1 and rep.status == -1
    assert needle in qe.qe_last_error()
    assert lib.qe_workspace_bytes(ctypes.byref(p), ctypes.byref(o)) == 0


@pytest.mark.parametrize("field,val,needle", [
    ("newton_atol", 0.0, "newton_atol"),
    ("newton_atol", float("nan"), "newton_atol"),
    ("newton_maxit", -1, "newton_maxit"),
    ("ls_max_halvings", 99, "ls_max_halvings"),
    ("krylov_rtol_max", 1.5, "krylov_rtol_max"),
    ("krylov_maxit", 0, "krylov_maxit"),
    ("precision", 7, "precision"),
    ("init_guess", 3, "init_guess"),
    ("precond", 3, "precond"),
    ("precond", -1, "precond"),
])
def test_invalid_options_rejected(field, val, needle):
    lib = qe.load_library()
    p = fake_problem()
    o = qe.qe_default_options()
    setattr(o, field, val)
    ph = qe.CPhysics(2, 4.0, 1.08, 0.56)
    st = lib.qe_solve(ctypes.byref(p), ctypes.byref(ph), ctypes.byref(o), ctypes.c_void_p(16),
                      None, ctypes.c_void_p(256), 1 << 40, None, None)
    assert st == -1 and needle in qe.qe_last_error()


@pytest.mark.parametrize("phys,needle", [
    ((2, 0.0, 1.08, 0.56), "T_K > 0"),
    ((2, float("inf"), 1.08, 0.56), "T_K > 0"),
    ((1, 0.0, -1.0, 0.56), "m_eff"),
    ((9, 4.0, 1.08, 0.56), "unknown statistics"),
    ((1, 0.0, 1.08, float("nan")), "Ec0_eV"),
])
def test_invalid_physics_rejected(phys, needle):
    lib = qe.load_library()
    p = fake_problem()
    o = qe.qe_default_options()
    ph = qe.CPhysics(*phys)
    st = lib.qe_solve(ctypes.byref(p), ctypes.byref(ph), ctypes.byref(o), ctypes.c_void_p(16),
                      None, ctypes.c_void_p(256), 1 << 40, None, None)
    assert st == -1 and needle in qe.qe_last_error()


def test_workspace_checks():
    lib = qe.load_library()
    p = fake_problem()
    o = qe.qe_default_options()
    ph = qe.CPhysics(2, 4.0, 1.08, 0.56)
    need = lib.qe_workspace_bytes(ctypes.byref(p), ctypes.byref(o))
    assert need > 0 and need % 256 == 0
    # NULL, misaligned and short workspaces are rejected before any device work
    for ws, nb, msg in ((None, need, "NULL"), (ctypes.c_void_p(257), need, "aligned"),
                        (ctypes.c_void_p(256), need - 1, "too small")):
        st = lib.qe_solve(ctypes.byref(p), ctypes.byref(ph), ctypes.byref(o), ctypes.c_void_p(16),
                          None, ws, nb, None, None)
        assert st == -3 and msg in qe.qe_last_error()


def test_workspace_scales_with_mesh(monkeypatch):
    lib = qe.load_library()
    o = qe.qe_default_options()
    small = lib.qe_workspace_bytes(ctypes.byref(fake_problem(17, 17, 9)), ctypes.byref(o))
    big = lib.qe_workspace_bytes(ctypes.byref(fake_problem(129, 129, 65)), ctypes.byref(o))
    N = 129 * 129 * 65
    assert big > small
    def size(seq, mg):
        monkeypatch.setenv("QE_SEQ_MIN_NODES", "1" if seq else str(10 ** 12))
        monkeypatch.setenv("QE_MG_MIN_NODES", "1" if mg else str(10 ** 12))
        return lib.qe_workspace_bytes(ctypes.byref(fake_problem(129, 129, 65)), ctypes.byref(o))
    # without the coarse-mesh sequence and multigrid: about 7 FP64 + 5 FP32
    # nodal vectors, FP64 + FP32 Gauss-point coefficients
    fine = size(False, False)
    assert 150 * N < fine < 230 * N
    # the sequence's coarse level (65 x 65 x 33, an eighth of the nodes) adds
    # its arrays and its own layout
    assert fine / 10 < size(True, False) - fine < fine / 6
    # multigrid: the fine level's smoother weights and J x in FP64 and FP32
    # (24 B per node) plus three coarse levels (an eighth, a 64th, a 512th of
    # the nodes)
    mg = size(False, True) - fine
    assert 24 * N + fine / 10 < mg < 24 * N + fine / 5
    # both share one region after the fine layout
    assert size(True, True) - fine == max(size(True, False) - fine, mg) == big - fine


def test_count_and_adjoint_argument_checks():
    lib = qe.load_library()
    p = fake_problem()
    ph = qe.CPhysics(1, 0.0, 1.08, 0.56)
    P = ctypes.POINTER(ctypes.c_double)
    boxes = np.zeros(6 * 17)
    out = np.zeros(17)
    st = lib.qe_count_electrons(ctypes.byref(p), ctypes.byref(ph), ctypes.c_void_p(16), 17,
                                boxes.ctypes.data_as(P), out.ctypes.data_as(P),
                                ctypes.c_void_p(256), 1 << 40, None)
    assert st == -1 and "n_boxes" in qe.qe_last_error()
    o = qe.qe_default_options(precision=1)
    st = lib.qe_adjoint(ctypes.byref(p), ctypes.byref(ph), ctypes.byref(o), ctypes.c_void_p(16),
                        boxes.ctypes.data_as(P), None, out.ctypes.data_as(P), None, None,
                        ctypes.c_void_p(256), 1 << 40, None, None)
    assert st == -1 and "FP64" in qe.qe_last_error()


def full_physics(**kw):
    f = dict(stat="fd", T_K=4.0, holes=True, ionization="incomplete")
    f.update(kw)
    return qe.Physics(**f).c()


@pytest.mark.parametrize("over,needle", [
    (dict(holes=2), "holes must be 0 or 1"),
    (dict(ionization=5), "unknown ionization"),
    (dict(m_h=0.0), "m_h"),
    (dict(Eg_eV=-0.1), "Eg_eV"),
    (dict(Ed_eV=float("nan")), "Ed_eV"),
    (dict(gA=0.0), "gD and gA"),
    (dict(stat=1, T_K=0.0), "incomplete ionization needs"),
    (dict(stat=3, T_K=0.0), "T_K > 0"),
])
def test_invalid_full_charge_physics_rejected(over, needle):
    lib = qe.load_library()
    p = fake_problem()
    p.donors = p.acceptors = 16
    o = qe.qe_default_options()
    ph = full_physics()
    for k, v in over.items():
        setattr(ph, k, v)
    st = lib.qe_solve(ctypes.byref(p), ctypes.byref(ph), ctypes.byref(o), ctypes.c_void_p(16),
                      None, ctypes.c_void_p(256), 1 << 40, None, None)
    assert st == -1 and needle in qe.qe_last_error()


def test_dopant_species_arguments_checked_before_device_work():
    lib = qe.load_library()
    o = qe.qe_default_options()
    ph = full_physics()
    p = fake_problem()
    p.donors = 16                       # acceptors missing
    st = lib.qe_solve(ctypes.byref(p), ctypes.byref(ph), ctypes.byref(o), ctypes.c_void_p(16),
                      None, ctypes.c_void_p(256), 1 << 40, None, None)
    assert st == -1 and "together" in qe.qe_last_error()
    p = fake_problem()                  # neither: fine for complete ionization, not for incomplete
    st = lib.qe_solve(ctypes.byref(p), ctypes.byref(ph), ctypes.byref(o), ctypes.c_void_p(16),
                      None, ctypes.c_void_p(256), 1 << 40, None, None)
    assert st == -1 and "needs donors and acceptors" in qe.qe_last_error()


def test_ohmic_potential_argument_checks():
    lib = qe.load_library()
    out = ctypes.c_double()
    for ph, nd, na, needle in [
        (qe.Physics(stat="tf", T_K=0.0).c(), 1e-3, 0.0, "Boltzmann or Fermi-Dirac"),
        (qe.Physics(stat="mb", T_K=0.0).c(), 1e-3, 0.0, "T_K"),
        (qe.Physics(stat="mb", T_K=300.0).c(), -1e-3, 0.0, "N_D and N_A"),
        (qe.Physics(stat="mb", T_K=300.0).c(), 1e-3, 1e-3, "net doping"),
        (qe.Physics(stat="mb", T_K=300.0, ionization="incomplete").c(), 0.0, 0.0, "majority dopant"),
        (qe.Physics(stat="fd", T_K=300.0, m_h=0.0).c(), 0.0, 1e-3, "m_h"),
    ]:
        st = lib.qe_ohmic_potential(ctypes.byref(ph), nd, na, 0.0, ctypes.byref(out))
        assert st == -1 and needle in qe.qe_last_error(), (needle, qe.qe_last_error())
    assert lib.qe_ohmic_potential(None, 1e-3, 0.0, 0.0, ctypes.byref(out)) == -1


@pytest.mark.parametrize("sheet,needle", [
    (dict(axis=3), "axis"),
    (dict(plane=2), "plane out of range"),          # nz = 2 for axis 2
    (dict(a0=1, a1=1), "face range"),
    (dict(a1=4), "face range"),                      # nx - 1 = 3 faces
    (dict(b1=3), "face range"),                      # ny - 1 = 2 faces
    (dict(robin_d=-1.0), "robin_d"),
    (dict(robin_d=10.0, robin_eps=0.0), "robin_eps"),
    (dict(phi0=float("nan")), "phi0"),
])
def test_invalid_sheet_rejected(sheet, needle):
    lib = qe.load_library()
    p = fake_problem()
    f = dict(axis=2, plane=1, a0=0, a1=3, b0=0, b1=2, sigma=None, robin_d=0.0, robin_eps=0.0, phi0=0.0)
    f.update(sheet)
    arr = (qe.CSheet * 1)(qe.CSheet(**f))
    p.n_sheets = 1
    p.sheets = arr
    o = qe.qe_default_options()
    ph = qe.CPhysics(2, 4.0, 1.08, 0.56)
    st = lib.qe_solve(ctypes.byref(p), ctypes.byref(ph), ctypes.byref(o), ctypes.c_void_p(16),
                      None, ctypes.c_void_p(256), 1 << 40, None, None)
    assert st == -1 and needle in qe.qe_last_error(), qe.qe_last_error()


def test_sheet_count_checks():
    lib = qe.load_library()
    o = qe.qe_default_options()
    ph = qe.CPhysics(2, 4.0, 1.08, 0.56)
    for n, needle in ((17, "n_sheets"), (-1, "n_sheets"), (1, "sheets is NULL")):
        p = fake_problem()
        p.n_sheets = n
        st = lib.qe_solve(ctypes.byref(p), ctypes.byref(ph), ctypes.byref(o), ctypes.c_void_p(16),
                          None, ctypes.c_void_p(256), 1 << 40, None, None)
        assert st == -1 and needle in qe.qe_last_error()


@pytest.mark.parametrize("over,needle", [
    (dict(n_states=0), "n_states"),
    (dict(n_states=33), "n_states"),
    (dict(confinement=2), "confinement"),
    (dict(psi2=None), "NULL array"),
    (dict(confinement=1, m_t=0.0), "m_t"),
    (dict(E_nan=True), "E_i[1]"),
    (dict(T=0.0), "T_K > 0"),
])
def test_invalid_quantum_rejected(over, needle):
    lib = qe.load_library()
    p = fake_problem()
    E = (ctypes.c_double * 2)(-0.01, float("nan") if over.pop("E_nan", False) else 0.01)
    T = over.pop("T", 4.0)
    f = dict(n_states=2, confinement=3, psi2=16, phi_k=16, E_i=E, m_t=0.19)
    f.update(over)
    q = qe.CQuantum(**f)
    p.quantum = ctypes.pointer(q)
    o = qe.qe_default_options()
    ph = qe.Physics(stat="tf", T_K=T).c()
    st = lib.qe_solve(ctypes.byref(p), ctypes.byref(ph), ctypes.byref(o), ctypes.c_void_p(16),
                      None, ctypes.c_void_p(256), 1 << 40, None, None)
    assert st in (-1, -3) and needle in qe.qe_last_error(), qe.qe_last_error()


def test_schrodinger_argument_checks():
    lib = qe.load_library()
    p = fake_problem(6, 5, 4)
    P = ctypes.POINTER(ctypes.c_double)
    E = np.zeros(20)
    assert lib.qe_schrodinger_workspace_bytes(ctypes.byref(p), 17) == 0
    assert lib.qe_schrodinger_workspace_bytes(ctypes.byref(p), 3) > 0
    s = qe.CSchrodinger(16, 16, None)
    cases = [(dict(n=0), "n_states"), (dict(n=17), "n_states"), (dict(tol=0.0), "tol"), (dict(tol=1.5), "tol"),
             (dict(maxit=0), "maxit"), (dict(inv=None), "inv_mass"), (dict(ws=None), "workspace is NULL")]
    for over, needle in cases:
        a = dict(n=3, tol=1e-8, maxit=10, inv=16, ws=256)
        a.update(over)
        s.inv_mass = a["inv"]
        st = lib.qe_schrodinger_solve(ctypes.byref(p), ctypes.byref(s), ctypes.c_void_p(16), a["n"], a["tol"],
                                      a["maxit"], ctypes.c_uint64(1), 0, E.ctypes.data_as(P), ctypes.c_void_p(16),
                                      None, None, ctypes.c_void_p(a["ws"]) if a["ws"] else None, 1 << 40, None)
        assert st in (-1, -3) and needle in qe.qe_last_error(), (needle, qe.qe_last_error())


def test_tensor_arguments_checked_before_the_library():
    """The binding rejects a tensor on the wrong device, of the wrong dtype or
    length, or not contiguous, before any pointer reaches the library."""
    import numpy as np
    import torch
    from paper_1403_7561_amd.qe import _dev
    cpu = torch.device("cpu")
    t = torch.zeros(10, dtype=torch.float64)
    assert _dev(t, torch.float64, 10, cpu, "phi") is t
    with pytest.raises(ValueError, match="tensor on cpu"):
        _dev(t, torch.float64, 10, torch.device("cuda", 0), "phi")
    with pytest.raises(ValueError, match="dtype"):
        _dev(t.to(torch.float32), torch.float64, 10, cpu, "phi")
    with pytest.raises(ValueError, match="dtype"):
        _dev(t.to(torch.int16), torch.float64, 10, cpu, "phi")
    with pytest.raises(ValueError, match="11"):
        _dev(t, torch.float64, 11, cpu, "phi")
    with pytest.raises(ValueError, match="contiguous"):
        _dev(torch.zeros(20, dtype=torch.float64)[::2], torch.float64, 10, cpu, "phi")
    with pytest.raises(ValueError, match="torch tensor"):
        _dev(np.zeros(10), torch.float64, 10, cpu, "phi")


def test_static_solve_rejects_a_problem_too_large_before_device_work():
    """qe_solve_static checks the workspace a problem needs against its static
    array before any device work (so this runs without a GPU)."""
    lib = qe.load_library()
    p = fake_problem(400, 400, 200)
    o = qe.qe_default_options()
    assert lib.qe_workspace_bytes(ctypes.byref(p), ctypes.byref(o)) > (256 << 20)
    rep = qe.CReport()
    st = lib.qe_solve_static(ctypes.byref(p), ctypes.byref(qe.Physics().c()), ctypes.byref(o),
                             ctypes.c_void_p(8), None, None, ctypes.byref(rep))
    assert st == -3 and rep.status == -3 and "static workspace" in qe.qe_last_error()


def test_schrodinger_masses_take_one_or_three_axes():
    """qe_schrodinger_solve takes m0/m* as [E] (isotropic) or [3, E] (per
    axis) and rejects any other shape before the library is called."""
    import numpy as np
    import torch
    from types import SimpleNamespace
    P = SimpleNamespace(E=10, N=30, device=torch.device("cpu"))
    for bad in (np.ones((2, 10)), np.ones(30), np.ones((10, 3))):
        with pytest.raises(ValueError, match="inv_mass"):
            qe.qe_schrodinger_solve(P, bad, np.zeros(10), np.zeros(30), 2)
