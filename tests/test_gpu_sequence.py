"""The coarse-mesh sequence that starts Newton by default (init_guess = 2):
the problem coarsened by taking every other node (the last kept) is solved,
its potential interpolated, and Newton continues on the given mesh.  The
discrete problem has one solution, so the sequenced solve must equal the
oracle and the linear-guess solve; these tests lower the size threshold
(QE_SEQ_MIN_NODES) so that meshes the oracle solves quickly are sequenced,
with odd and even node counts, one coarse level (the default) and two,
the full space
charge (donor and acceptor arrays coarsened) and mixed precision, and check
the fallbacks to the linear guess."""
import numpy as np
import pytest

import synth
from oracle import solver
from paper_1403_7561_amd import qe
from tests import gpu_support as gs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def double_dot(nx, ny, nz, volts=(1.5, 1.4, 0.5, 0.7, 0.3)):
    return synth.double_dot_device(f"seq{nx}x{ny}x{nz}", nx, ny, nz, np.array(volts))


@pytest.mark.parametrize("dims,min_nodes,levels", [
    ((33, 33, 17), 1000, 1),      # odd counts: nested halving, 17x17x9
    ((36, 30, 20), 1000, 1),      # even counts (19x16x11): the last coarse element spans one fine element
    ((41, 41, 21), 3000, 2),      # two levels (QE_SEQ_LEVELS): 41x41x21 -> 21x21x11 -> 11x11x6
])
def test_sequenced_solve_matches_oracle_and_linear_guess(monkeypatch, dims, min_nodes, levels):
    monkeypatch.setenv("QE_SEQ_MIN_NODES", str(min_nodes))
    monkeypatch.setenv("QE_SEQ_LEVELS", str(levels))
    dev = double_dot(*dims)
    P = qe.Problem(dev)
    opts = qe.qe_default_options(newton_atol=1e-10)
    phi_s, _, rep_s = qe.qe_solve(P, opts=opts)
    assert rep_s["status"] == 0 and rep_s["seq_levels"] == levels
    assert rep_s["init_krylov_iters"] > 0 and rep_s["res_final"] <= 1e-10
    phi_l, _, rep_l = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-10, init_guess=0))
    assert rep_l["seq_levels"] == 0
    print(dims, "sequenced", rep_s, "linear", rep_l)
    assert rel_max(phi_s.cpu().numpy(), phi_l.cpu().numpy()) <= 1e-12
    _, res = solver.solve(dev, atol=1e-10)
    assert rel_max(phi_s.cpu().numpy(), res.phi) <= 1e-9


def test_sequenced_full_charge_and_mixed_precision(monkeypatch):
    monkeypatch.setenv("QE_SEQ_MIN_NODES", "5000")
    dev = gs.full_charge_device("incomplete")
    P = qe.Problem(dev)
    phi, _, rep = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-10))
    assert rep["seq_levels"] == 1
    _, res = solver.solve(dev, atol=1e-10)
    assert rel_max(phi.cpu().numpy(), res.phi) <= 1e-9
    phim, _, repm = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-10, precision="mixed"))
    assert repm["seq_levels"] == 1
    assert rel_max(phim.cpu().numpy(), res.phi) <= 1e-6


def test_fallbacks_to_the_linear_guess(monkeypatch):
    dev = double_dot(33, 33, 17)
    P = qe.Problem(dev)
    opts = qe.qe_default_options(newton_atol=1e-10)
    # below the size threshold (the library's own, 250000 nodes)
    _, _, rep = qe.qe_solve(P, opts=opts)
    assert rep["seq_levels"] == 0
    # a workspace without room for the coarse level
    monkeypatch.setenv("QE_SEQ_MIN_NODES", str(10 ** 12))
    fine_only = qe.qe_workspace_bytes(P, opts)
    monkeypatch.setenv("QE_SEQ_MIN_NODES", "5000")
    assert qe.qe_workspace_bytes(P, opts) > fine_only
    phi_w, _, rep = qe.qe_solve(P, opts=opts, ws=qe.Workspace(fine_only, P.device))
    assert rep["status"] == 0 and rep["seq_levels"] == 0
    # sheets and eigenstates
    sdev = synth.with_interface_charge(dev, 1e-3, seed=5, spread=0.5)
    _, _, rep = qe.qe_solve(qe.Problem(sdev), opts=opts)
    assert rep["status"] == 0 and rep["seq_levels"] == 0
    _, res = solver.solve(dev, atol=1e-10)
    st = synth.box_states(dev, (10.0, 60.0, 80.0, 120.0, 75.0, 90.0), 4, res.phi, seed=3, e0=-0.003, spacing=0.0006)
    _, _, rep = qe.qe_solve(qe.Problem(synth.with_quantum(dev, st)), opts=opts)
    assert rep["status"] == 0 and rep["seq_levels"] == 0


def test_benchmark_mesh_sequenced_by_default():
    """129x129x65: the default options sequence once (65x65x33), take fewer
    Newton steps on the fine mesh than the linear guess, and reach the same
    potential."""
    dev = synth.config2()
    P = qe.Problem(dev)
    phi_s, _, rep_s = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-10))
    phi_l, _, rep_l = qe.qe_solve(P, opts=qe.qe_default_options(newton_atol=1e-10, init_guess=0))
    print("sequenced", rep_s, "linear", rep_l)
    assert rep_s["seq_levels"] == 1 and rep_l["seq_levels"] == 0
    assert rep_s["newton_iters"] < rep_l["newton_iters"]
    assert rel_max(phi_s.cpu().numpy(), phi_l.cpu().numpy()) <= 1e-12
