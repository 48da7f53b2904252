"""The solve that allocates nothing (qe_solve_static: the library's static
device workspace, no caller workspace, no events) against qe_solve with a
caller workspace, on two calls in a row, the second on a smaller mesh."""
import ctypes

import numpy as np
import pytest

import synth
from paper_1403_7561_amd import qe
from tests import gpu_support as gs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_static_workspace_solve_matches_qe_solve():
    # the larger mesh first, so that the second call finds the array holding
    # the first call's data (Fermi-Dirac 37x29x19, then Thomas-Fermi 17x17x9)
    for dev in (gs.ragged_device(), synth.config1()):
        P = qe.Problem(dev)
        opts = qe.qe_default_options(newton_atol=1e-10)
        phi_ref, n_ref, rep_ref = qe.qe_solve(P, opts=opts, want_density=True)
        phi = torch.zeros(P.N, dtype=torch.float64, device=P.device)
        n = torch.empty(P.N, dtype=torch.float64, device=P.device)
        rep = qe.qe_solve_static(P, phi, n, opts=opts)
        torch.cuda.synchronize()
        err = rel_max(phi.cpu().numpy(), phi_ref.cpu().numpy())
        errn = rel_max(n.cpu().numpy(), n_ref.cpu().numpy())
        print(dev.name, dev.nx, dev.ny, dev.nz, "static", rep, "workspace", rep_ref, "rel phi", err, "rel n", errn)
        assert rep["status"] == 0 and rep["res_final"] <= 1e-10
        assert rep["newton_iters"] == rep_ref["newton_iters"]
        assert err <= 1e-12 and errn <= 1e-12


def test_static_workspace_rejects_problems_that_need_more():
    lib = qe.load_library()
    N = 400 * 400 * 200
    arrs = [torch.zeros(400, dtype=torch.float64, device="cuda") for _ in range(3)]
    big = torch.zeros(1, dtype=torch.float64, device="cuda")
    prob = qe.CProblem(400, 400, 200, arrs[0].data_ptr(), arrs[1].data_ptr(), arrs[2].data_ptr(),
                       big.data_ptr(), big.data_ptr(), big.data_ptr(), big.data_ptr(), big.data_ptr(), 0,
                       None, None, 0, None, None)
    o = qe.qe_default_options()
    assert lib.qe_workspace_bytes(ctypes.byref(prob), ctypes.byref(o)) > (256 << 20)
    rep = qe.CReport()
    st = lib.qe_solve_static(ctypes.byref(prob), ctypes.byref(qe.Physics().c()), ctypes.byref(o),
                             ctypes.c_void_p(big.data_ptr()), None, None, ctypes.byref(rep))
    assert st == -3 and "static workspace" in qe.qe_last_error() and rep.status == -3
    assert N > 0


def test_static_workspace_sequenced_solve_at_the_benchmark_size():
    """129x129x65: the static array also holds the coarse level of the
    default coarse-mesh sequence, which then runs without allocating; the
    solve matches qe_solve's (with the Jacobi preconditioner, the only one
    the static entry point runs)."""
    dev = synth.config2()
    P = qe.Problem(dev)
    opts = qe.qe_default_options(newton_atol=1e-10, precond=1)
    phi_ref, _, rep_ref = qe.qe_solve(P, opts=opts, want_density=False)
    phi = torch.zeros(P.N, dtype=torch.float64, device=P.device)
    rep = qe.qe_solve_static(P, phi, None, opts=opts)
    torch.cuda.synchronize()
    print("static", rep, "workspace", rep_ref)
    assert rep["status"] == 0 and rep["res_final"] <= 1e-10
    assert rep["seq_levels"] == 1 and rep_ref["seq_levels"] == 1
    assert rep["newton_iters"] == rep_ref["newton_iters"]
    assert rel_max(phi.cpu().numpy(), phi_ref.cpu().numpy()) <= 1e-12
