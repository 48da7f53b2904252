"""GPU tests of the benchmark workloads at their own sizes: the dot-charge
gradient of the 129 x 129 x 65 five-gate stack (Sec. III, C = q dN/dV)
against central differences of the GPU solve, and the 256-instance plunger
sweep, whose smallest and largest meshes must equal their single-instance
solves, and the 257 x 257 x 129 stack's FP64 and mixed-precision solves.
(The oracle cannot solve these sizes in a test's time; the gradient is
pinned by differences, the sweep by the single-instance path, which the
oracle pins at smaller sizes, and the large solves by the oracle's residual
and Jacobian on sampled nodes.)"""
import numpy as np
import pytest

import synth
from paper_1403_7561_amd import qe

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

H_V = 1e-4          # central-difference step in the gate voltages (V)
# Relative permittivity steps: one element moves the dot charge by ~1e-6 of
# itself per 1e-3 change, so central differences at 1e-4 would sit at the
# solve's floor (||F|| ~ 1e-11); a 1 % step with Richardson extrapolation
# from steps h and 2h keeps the truncation error O(h^4) and the noise ~100x
# smaller.
H_EPS = 1e-2


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_c4_gradient_matches_differences_at_full_size():
    dev = synth.config4()
    box = dev.boxes["D1"] if dev.dir_val[0] >= dev.dir_val[1] else dev.boxes["D2"]
    P = qe.Problem(dev)
    opts = qe.qe_default_options(newton_atol=2e-11)
    ws = qe.workspace_for(P, opts)
    phi, _, rep = qe.qe_solve(P, opts=opts, ws=ws)
    Q, dV, deps, _, arep = qe.qe_adjoint(P, phi, box, opts=opts, ws=ws)
    deps = deps.cpu().numpy()
    print("solve", rep, "adjoint", arep, "Q", Q)
    assert Q > 1.0                     # the dot holds electrons

    # every difference restarts Newton from the solution, so both sides of a
    # difference follow the same path to the same floor
    warm = qe.qe_default_options(newton_atol=2e-11, init_guess=1)

    def charge(d):
        Pd = qe.Problem(d)
        ph, _, r = qe.qe_solve(Pd, opts=warm, phi=phi.clone(), ws=ws, want_density=False)
        return qe.qe_count_electrons(Pd, ph, [box], ws=ws)[0]

    # the five gates and the grounded bottom contact
    nd = len(dev.dir_val)
    assert nd == 6 and len(dV) == nd
    fdV = np.empty(nd)
    for g in range(nd):
        qs = []
        for s in (+1, -1):
            d = synth.config4()
            d.dir_val = d.dir_val.copy()
            d.dir_val[g] += s * H_V
            qs.append(charge(d))
        fdV[g] = (qs[0] - qs[1]) / (2 * H_V)
    print("dQ/dV adjoint", dV, "\n      differences", fdV, "\n      rel", np.abs(dV - fdV) / np.abs(fdV))
    assert np.all(np.abs(dV - fdV) <= 1e-6 * np.abs(fdV))

    # 32 seeded elements around the dot, and one random direction
    x, y, z = dev.x, dev.y, dev.z
    ex, ey, ez = dev.nx - 1, dev.ny - 1, dev.nz - 1
    cx = 0.5 * (x[:-1] + x[1:])
    cy = 0.5 * (y[:-1] + y[1:])
    cz = 0.5 * (z[:-1] + z[1:])
    CZ, CY, CX = np.meshgrid(cz, cy, cx, indexing="ij")
    near = ((CX >= box[0] - 15) & (CX <= box[1] + 15) & (CY >= box[2] - 15) & (CY <= box[3] + 15)
            & (CZ >= box[4] - 10) & (CZ <= box[5] + 12)).ravel()
    cand = np.nonzero(near)[0]
    rng = np.random.default_rng(7564)
    els = rng.choice(cand, size=32, replace=False)
    def richardson(scaled_eps, h=H_EPS):
        """d/dt Q(eps (1 + t w)) at t = 0 from central differences at steps
        h and 2h, combined to cancel the O(h^2) term."""
        def central(h):
            qs = []
            for s in (+1, -1):
                d = synth.config4()
                d.eps_r = scaled_eps(s * h)
                qs.append(charge(d))
            return (qs[0] - qs[1]) / (2 * h)
        return (4.0 * central(h) - central(2 * h)) / 3.0

    fde = np.empty(32)
    for t, e in enumerate(els):
        def one(h, e=e):
            a = dev.eps_r.copy()
            a[e] *= 1.0 + h
            return a
        fde[t] = richardson(one) / dev.eps_r[e]
    ad = deps[els]
    scale = np.abs(fde).max()
    print("dQ/deps max", scale, "max abs diff", np.abs(ad - fde).max(), "rel to max",
          np.abs(ad - fde).max() / scale, "rel", np.abs(ad - fde) / np.abs(fde))
    assert np.abs(ad - fde).max() <= 1e-6 * scale
    dirn = rng.standard_normal(dev.n_elems)
    # every element moves at once here, and the derivative is a sum of
    # contributions of both signs: a 0.1 % step keeps the higher-order terms
    # out while the charge still moves ~1e-4 of itself
    fd_dir = richardson(lambda h: dev.eps_r * (1.0 + h * dirn), h=1e-3)
    ad_dir = float(np.sum(dirn * dev.eps_r * deps))
    print("random direction: adjoint", ad_dir, "differences", fd_dir, "rel", abs(ad_dir - fd_dir) / abs(fd_dir))
    assert ad_dir == pytest.approx(fd_dir, rel=1e-6)


def test_c3_smallest_and_largest_instances_match_single_solves(tmp_path):
    spec = synth.config3_spec()
    devs = [synth.config3_instance(k, spec) for k in range(len(spec[0]))]
    probs = [qe.Problem(d) for d in devs]
    opts = qe.qe_default_options(newton_atol=5e-11)
    boxes = [synth.DOT_BOX_D1, synth.DOT_BOX_D2]
    phis, counts, reps = qe.qe_solve_batch(probs, opts=opts, boxes=boxes, tune_cache=str(tmp_path / "t.txt"))
    assert all(r["status"] == 0 for r in reps)
    sizes = [p.N for p in probs]
    for k in (int(np.argmin(sizes)), int(np.argmax(sizes))):
        phi1, _, rep1 = qe.qe_solve(probs[k], opts=opts, want_density=False)
        err = rel_max(phis[k].cpu().numpy(), phi1.cpu().numpy())
        c1 = qe.qe_count_electrons(probs[k], phi1, boxes)
        print(k, devs[k].nx, devs[k].ny, devs[k].nz, "batch", reps[k], "single", rep1, "rel", err,
              "counts", counts[k], c1)
        assert err <= 1e-12
        assert np.allclose(counts[k], c1, rtol=1e-10, atol=1e-12 * max(c1.max(), 1e-30))


def test_c5_fp64_and_mixed_solves_at_full_size():
    """257 x 257 x 129 stack with eight random gates over a rough oxide, in the
    launch configuration the benchmark times (coarse-mesh start, default
    options): the FP64 and mixed-precision solves both reach ||F|| < 1e-8;
    the oracle's residual at the returned potentials is at the FP64 floor on
    sampled nodes (half of them where the electron density is largest, so the
    charge terms are exercised); the mixed potential and dot counts agree with
    the FP64 ones to 1e-6; sampled J.v values (FP64 and FP32 operands) at a
    perturbed potential match the oracle's element-by-element Jacobian."""
    from tests import gpu_support as gs
    dev = synth.config5()
    P = qe.Problem(dev)
    boxes = [dev.boxes["D1"], dev.boxes["D2"]]
    opts64 = qe.qe_default_options(newton_atol=1e-8)
    optsm = qe.qe_default_options(newton_atol=1e-8, precision=1)
    ws = qe.workspace_for(P, opts64)
    phi64, n64, rep64 = qe.qe_solve(P, opts=opts64, ws=ws, want_density=True)
    phim, _, repm = qe.qe_solve(P, opts=optsm, ws=ws, want_density=False)
    print("fp64", rep64, "\nmixed", repm)
    assert rep64["status"] == 0 and rep64["res_final"] <= 1e-8 and rep64["seq_levels"] == 1
    assert repm["status"] == 0 and repm["res_final"] <= 1e-8
    ph64, phm = phi64.cpu().numpy(), phim.cpu().numpy()
    err = rel_max(phm, ph64)
    c64 = qe.qe_count_electrons(P, phi64, boxes, ws=ws)
    cm = qe.qe_count_electrons(P, phim, boxes, ws=ws)
    print("mixed vs fp64", err, "counts", c64, cm)
    assert err <= 1e-6
    assert np.allclose(cm, c64, rtol=1e-6, atol=1e-6 * max(c64.max(), 1e-30))
    rng = np.random.default_rng(55)
    dens = n64.cpu().numpy()
    nodes = np.concatenate([rng.choice(dev.n_nodes, 150, replace=False), np.argsort(dens)[-150:]])
    for name, ph in (("fp64", ph64), ("mixed", phm)):
        Fs = gs.sampled_residual(dev, ph, nodes)
        print(name, "sampled oracle |F| max", np.abs(Fs).max())
        assert np.abs(Fs).max() < 1e-8
    pert = ph64 + 0.01 * rng.standard_normal(ph64.size)
    pert[dev.dir_id >= 0] = dev.dir_val[dev.dir_id[dev.dir_id >= 0]]
    v = rng.standard_normal(ph64.size)
    pt = torch.as_tensor(pert, device="cuda")
    yo = gs.sampled_jv(dev, pert, v, nodes)
    y = qe.qe_jv(P, pt, torch.as_tensor(v, device="cuda"), ws=ws).cpu().numpy()[nodes]
    y32 = qe.qe_jv(P, pt, torch.as_tensor(v, dtype=torch.float32, device="cuda"), ws=ws).cpu().numpy()[nodes]
    print("jv64", np.abs(y - yo).max() / np.abs(yo).max(), "jv32", np.abs(y32 - yo).max() / np.abs(yo).max())
    assert np.abs(y - yo).max() <= 1e-12 * np.abs(yo).max()
    assert np.abs(y32 - yo).max() <= 2e-5 * np.abs(yo).max()
