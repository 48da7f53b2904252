"""Batched persistent sweep: every instance of one launch agrees with the
single-instance GPU solve and with the CPU oracle; the autotuner's cache is
written once and reused; invalid instances are rejected."""
import os

import numpy as np
import pytest

import synth
from oracle import solver
from paper_1403_7561_amd import qe

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def small_sweep(n=6, seed=3):
    """Uneven double-dot meshes with a plunger sweep (sizes kept small so the
    oracle can solve every instance)."""
    rng = np.random.default_rng(seed)
    devs = []
    for k in range(n):
        m = int(rng.integers(12, 25))
        volts = np.array([0.9 + 0.15 * k, 1.6 - 0.1 * k, 0.4, 0.7, 0.3])
        devs.append(synth.double_dot_device(f"b{k}", m + 1, m + 1, m // 2 + 1, volts))
    return devs


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_batch_matches_single_and_oracle(tmp_path):
    devs = small_sweep()
    probs = [qe.Problem(d) for d in devs]
    # solved to near the FP64 floor of ||F||, so that two paths with different
    # summation orders must agree to 1e-12
    opts = qe.qe_default_options(newton_atol=2e-12)
    boxes = [synth.DOT_BOX_D1, synth.DOT_BOX_D2]
    cache = str(tmp_path / "tune.txt")
    phis, counts, reps = qe.qe_solve_batch(probs, opts=opts, boxes=boxes, tune_cache=cache)
    assert os.path.exists(cache) and open(cache).read().count("\n") == 1
    for k, (d, P) in enumerate(zip(devs, probs)):
        assert reps[k]["status"] == 0 and reps[k]["res_final"] <= 2e-12
        phi1, _, rep1 = qe.qe_solve(P, opts=opts, want_density=False)
        err = rel_max(phis[k].cpu().numpy(), phi1.cpu().numpy())
        print(k, d.nx, d.ny, d.nz, reps[k], "vs single", err)
        assert err <= 1e-12
        c1 = qe.qe_count_electrons(P, phi1, boxes)
        assert np.allclose(counts[k], c1, rtol=1e-10, atol=1e-12 * max(c1.max(), 1e-30))
    for k in (0, len(devs) - 1):
        po, res = solver.solve(devs[k], atol=1e-10)
        assert rel_max(phis[k].cpu().numpy(), res.phi) < 1e-9
        co = [po.count(res.phi, b) for b in boxes]
        assert np.allclose(counts[k], co, rtol=1e-8, atol=1e-12 * max(max(co), 1e-30))
    # second call: the cache is read, not extended, and the answer is the same
    phis2, counts2, _ = qe.qe_solve_batch(probs, opts=opts, boxes=boxes, tune_cache=cache)
    assert open(cache).read().count("\n") == 1
    for a, b in zip(phis, phis2):
        assert torch.equal(a, b)
    assert np.array_equal(counts, counts2)


def test_batch_rejects_invalid_instance():
    devs = small_sweep(3)
    devs[1].eps_r = devs[1].eps_r.copy()
    devs[1].eps_r[7] = 0.0
    probs = [qe.Problem(d) for d in devs]
    with pytest.raises(qe.QeError, match="eps_r"):
        qe.qe_solve_batch(probs, opts=qe.qe_default_options())
    with pytest.raises(qe.QeError, match="FP64"):
        qe.qe_solve_batch(probs[:1], opts=qe.qe_default_options(precision=1))


def test_batch_reports_nonconvergence_per_instance():
    devs = small_sweep(2)
    probs = [qe.Problem(d) for d in devs]
    phis, counts, reps = qe.qe_solve_batch(probs, opts=qe.qe_default_options(newton_maxit=1, newton_atol=1e-10),
                                           check=False)
    assert all(r["status"] == -4 and r["newton_iters"] == 1 for r in reps)


def test_autograd_dot_charge_matches_differences():
    """torch.autograd through DotCharge (backward = qe_adjoint) against
    central differences of the forward solve, and the capacitance formula."""
    from paper_1403_7561_amd import autograd as ag
    volts = np.array([1.6, 1.5, 0.5, 0.8, 0.4])
    dev = synth.double_dot_device("ad", 17, 17, 11, volts)
    P = qe.Problem(dev)
    opts = qe.qe_default_options(newton_atol=1e-11)
    V = torch.tensor(dev.dir_val, dtype=torch.float64, device="cuda", requires_grad=True)
    eps = torch.tensor(dev.eps_r, dtype=torch.float64, device="cuda", requires_grad=True)
    Q = ag.DotCharge.apply(V, eps, P, dev.boxes["D1"], opts)
    Q.backward()
    gV = V.grad.cpu().numpy()
    ge = eps.grad.cpu().numpy()
    h = 1e-4
    for g in (0, 1, 3):
        e = torch.zeros_like(V)
        e[g] = h
        qp = ag.DotCharge.apply(V.detach() + e, eps.detach(), P, dev.boxes["D1"], opts).item()
        qm = ag.DotCharge.apply(V.detach() - e, eps.detach(), P, dev.boxes["D1"], opts).item()
        assert gV[g] == pytest.approx((qp - qm) / (2 * h), rel=1e-5, abs=1e-10)
    el = int(np.argmax(np.abs(ge)))
    de = torch.zeros_like(eps)
    de[el] = 1e-4 * dev.eps_r[el]
    qp = ag.DotCharge.apply(V.detach(), eps.detach() + de, P, dev.boxes["D1"], opts).item()
    qm = ag.DotCharge.apply(V.detach(), eps.detach() - de, P, dev.boxes["D1"], opts).item()
    assert ge[el] == pytest.approx((qp - qm) / (2 * de[el].item()), rel=1e-4)
    assert ag.capacitance_aF(gV[0]) == pytest.approx(1.602176634e-19 * gV[0] * 1e18)
