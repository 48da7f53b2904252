"""Benchmark of the nonlinear-Poisson Newton-Krylov path on one MI355X.

A step is one full FP64 solve of the five-gate double-dot stack
(129 x 129 x 65 nodes, Fermi-Dirac electrons at 4 K) from the default
initial guess (the coarse-mesh sequence: the 65 x 65 x 33 problem solved from
its charge-free guess, interpolated) to ||F|| < 1e-8, plus the electron counts
in the two dot boxes.  ``value`` is solves per second over the timed steps.  Also
reported: the J.v kernel rate (GDOF/s, FP64 and FP32) with its HBM roofline,
the adjoint/forward time ratio, and the CPU oracle timed on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1403_7561_amd/csrc/qe_device.h", "paper_1403_7561_amd/csrc/qe_tiles.h",
                  "paper_1403_7561_amd/csrc/qe_kernels.hip"]
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "cg_loop_traffic.md")
METRIC = "GDOF/s of nonlinear-Poisson J·v; solves/s at ‖F‖<1e-8; adjoint/forward time"


def jv_bytes(dev, val_bytes, n_coef):
    """Algorithmic bytes of one launch of the CG loop's J.v kernel: per node
    read z, y, p and write y, p (y = J z + beta y, p = z + beta p) and, in
    FP64, read and write x (the previous iteration's x += alpha p); per
    element read the permittivity and the coefficient flag; the 8 Gauss-point
    coefficients of the n_coef elements where they are not all exactly zero."""
    per_node = 7 if val_bytes == 8 else 5
    return dev.n_nodes * per_node * val_bytes + dev.n_elems * (val_bytes + 1) + n_coef * 8 * val_bytes


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key):
    """Counter-measured bytes per launch of a CG-loop kernel (key such as
    "k_cg_jv<double>.c5") from the committed summary, or None if the kernel
    sources changed since the counters were taken."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    fields = dict((a.strip(), b.strip()) for a, b in
                  (ln.split(":", 1) for ln in text.splitlines() if ln.startswith(("source_hash:", "traffic."))))
    if fields.get("source_hash") != kernel_source_hash() or "traffic." + key not in fields:
        return None
    return float(fields["traffic." + key])


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_count": os.cpu_count(), "cpu_model": model}


def _oracle_c3(k):
    """One instance of the batched sweep solved by the oracle, single-threaded
    (a pool worker)."""
    from threadpoolctl import threadpool_limits
    import synth
    from oracle import solver
    with threadpool_limits(1):
        dev = synth.config3_instance(k)
        t0 = time.perf_counter()
        _, res = solver.solve(dev, atol=1e-8, method="cg")
        return k, time.perf_counter() - t0, res.status, dev.n_nodes


def cpu_measure(budget_s=25.0, full=False, c3_workers=None):
    """The oracle on the host, before the GPU is initialised (the sweep's pool
    forks): single-threaded c2 solve (a bounded sample unless full), its CSR
    J.v, the small c1 solve, and a 16-instance subset of the c3 sweep over a
    pool of worker processes."""
    import multiprocessing as mp
    import numpy as np
    from threadpoolctl import threadpool_limits
    import synth
    from oracle import solver
    out = cpu_info()
    with threadpool_limits(1):
        dev1 = synth.config1()
        t0 = time.perf_counter()
        _, r1 = solver.solve(dev1, atol=1e-10)
        out["c1_solve_s"] = time.perf_counter() - t0
        dev = synth.config2()
        t0 = time.perf_counter()
        prob = solver.make_problem(dev)
        t_setup = time.perf_counter() - t0
        if full:
            t0 = time.perf_counter()
            r = solver.newton(prob, atol=1e-8, method="cg")
            out.update(c2_setup_s=t_setup, c2_solve_s=time.perf_counter() - t0, c2_newton_steps=r.iters,
                       c2_full=True)
            phi_k = r.phi
        else:
            t0 = time.perf_counter()
            phi_k = solver.initial_guess(prob, method="cg")
            t_init = time.perf_counter() - t0
            steps, t_steps = 0, 0.0
            while True:
                t0 = time.perf_counter()
                r = solver.newton(prob, phi0=phi_k, atol=1e-8, maxit=1, method="cg")
                dt = time.perf_counter() - t0
                log(f"oracle Newton step {steps + 1}: {dt:.1f} s")
                t_steps += dt
                phi_k = r.phi
                steps += 1
                if r.status == "ok" or t_setup + t_init + t_steps > budget_s:
                    break
            out.update(c2_setup_s=t_setup, c2_init_s=t_init, c2_step_s=t_steps / steps, c2_steps_timed=steps,
                       c2_full=False)
        # the assembled Jacobian's CSR product (scipy), median of three
        J = prob.jacobian_full(phi_k)
        v = np.random.default_rng(0).standard_normal(J.shape[0])
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            J @ v
            ts.append(time.perf_counter() - t0)
        out["jv_csr_ms"] = [t * 1e3 for t in ts]
        out["jv_csr_gdof_s"] = J.shape[0] / sorted(ts)[1] / 1e9
        out["jv_csr_nnz"] = int(J.nnz)
        del J, prob
    workers = c3_workers or min(16, os.cpu_count() or 1)
    ks = [17 * j for j in range(16)]          # the sweep's diagonal: P1 = P2 on the 16 grid points
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        done = pool.map(_oracle_c3, ks, chunksize=1)
    wall = time.perf_counter() - t0
    out["c3_subset"] = {"instances": ks, "workers": workers, "wall_s": wall, "solves_per_s": len(ks) / wall,
                        "instance_s": [d[1] for d in done], "nodes": [d[3] for d in done],
                        "all_ok": all(d[2] == "ok" for d in done)}
    return out


def cpu_baseline(m, gpu_newton):
    """The c2 rate from the host measurement: a full solve, or the sample's
    setup + initial guess + per-step time scaled to the Newton steps of the
    same solve from the linear guess on the GPU (the oracle's start)."""
    if m["c2_full"]:
        est = m["c2_setup_s"] + m["c2_solve_s"]
        sample = (f"c2 device: full oracle solve, assembly {m['c2_setup_s']:.1f} s + {m['c2_newton_steps']} "
                  f"Newton steps {m['c2_solve_s']:.1f} s")
    else:
        est = m["c2_setup_s"] + m["c2_init_s"] + m["c2_step_s"] * max(gpu_newton, 1)
        sample = (f"c2 device: assembly {m['c2_setup_s']:.1f} s + linear initial guess {m['c2_init_s']:.1f} s + "
                  f"{m['c2_steps_timed']} Newton step(s) timed at {m['c2_step_s']:.1f} s each, scaled to the "
                  f"{gpu_newton} Newton steps the GPU takes from the same linear guess = {est:.1f} s "
                  f"(scipy CSR / Jacobi-CG)")
    out = {"value": 1.0 / est, "unit": "solves/s", "cores": 1, "kind": "oracle", "sample": sample}
    out.update({k: m[k] for k in ("cpu_count", "cpu_model", "c1_solve_s", "jv_csr_gdof_s", "jv_csr_ms",
                                  "jv_csr_nnz", "c3_subset")})
    return out


def full_charge_run(synth, qe, torch, dev, opts, boxes, jv_reps):
    """The same stack with the full space charge: holes, a 1e15 cm^-3 boron
    substrate with incomplete ionization, the bottom contact at the library's
    Ohmic potential of that substrate.  One warm-up and two timed solves,
    then the CG loop's J.v kernel at the solution."""
    fdev = synth.with_species(dev, ionization="incomplete")
    phys = qe.Physics(stat=fdev.stat, T_K=fdev.T_K, m_eff=fdev.m_eff, Ec0_eV=fdev.Ec0_eV, holes=True,
                      ionization="incomplete")
    vb = qe.qe_ohmic_potential(phys, 0.0, float(fdev.acceptors.max()))
    fdev.dir_val[fdev.contacts.index("bottom")] = vb
    P = qe.Problem(fdev)
    # its own workspace: the coarse levels carry the donor and acceptor arrays
    ws = qe.workspace_for(P, opts)
    qe.qe_solve(P, opts=opts, ws=ws, want_density=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        ph, _, rep = qe.qe_solve(P, opts=opts, ws=ws, want_density=True)
        c = qe.qe_count_electrons(P, ph, boxes, ws=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 2
    v = torch.randn(P.N, dtype=torch.float64, device="cuda")
    ms64, ncoef = qe.qe_time_jv(P, ph, v, "fp64", jv_reps, ws=ws)
    b64 = jv_bytes(fdev, 8, ncoef)
    ach = b64 / (ms64 * 1e-3) / 1e9
    return {"solves_per_s": 1.0 / dt, "ms": dt * 1e3, "ohmic_bottom_V": vb,
            "newton_iters": rep["newton_iters"], "krylov_iters": rep["krylov_iters"],
            "mg_krylov_iters": rep["mg_krylov_iters"],
            "res_final": rep["res_final"], "dot_electrons": [float(x) for x in c],
            "jv": {"ms": ms64, "coef_elems": ncoef, "achieved_GBs": ach, "frac": ach / HBM_PEAK_GBS}}


def sheets_run(synth, qe, torch, dev, opts, ws, boxes):
    """The same stack with a fixed charge of 1e11 cm^-2 (+-50 %, seeded) on the
    Si/SiO2 interface and the two plungers as charged gates (Robin faces,
    d = 10 nm through oxide, -2e11 cm^-2 trapped charge).  One warm-up and two
    timed solves."""
    sdev = synth.with_interface_charge(dev, 1e-3, seed=7563, spread=0.5)
    sdev = synth.with_charged_gates(sdev, synth.double_dot_gates()[:2], sigma_nm2=-2e-3)
    P = qe.Problem(sdev)
    wsz = qe.workspace_for(P, opts)
    qe.qe_solve(P, opts=opts, ws=wsz, want_density=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        ph, _, rep = qe.qe_solve(P, opts=opts, ws=wsz, want_density=True)
        c = qe.qe_count_electrons(P, ph, boxes, ws=wsz)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 2
    return {"solves_per_s": 1.0 / dt, "ms": dt * 1e3, "newton_iters": rep["newton_iters"],
            "krylov_iters": rep["krylov_iters"], "mg_krylov_iters": rep["mg_krylov_iters"],
            "res_final": rep["res_final"], "dot_electrons": [float(x) for x in c], "n_sheets": len(sdev.sheets)}


def predictor_run(synth, qe, torch, dev, P, opts, boxes, phi_sc):
    """The predictor step of the predictor-corrector loop on the same stack:
    16 synthetic 3D-confined states in the D1 dot (hard-wall box modes,
    seeded levels from -3 meV around E_F) computed in the semiclassical
    solution phi_sc, which is also phi^(k).  One warm-up and two timed
    solves from the default guess."""
    st = synth.box_states(dev, (10.0, 60.0, 80.0, 120.0, 75.0, 90.0), 16, phi_sc.cpu().numpy(), seed=7564,
                          e0=-0.003, spacing=0.0006)
    Pq = qe.Problem(synth.with_quantum(dev, st))
    # its own workspace: the V-cycle's coarse levels carry the states
    ws = qe.workspace_for(Pq, opts)
    qe.qe_solve(Pq, opts=opts, ws=ws, want_density=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        ph, _, rep = qe.qe_solve(Pq, opts=opts, ws=ws, want_density=True)
        c = qe.qe_count_electrons(Pq, ph, boxes, ws=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 2
    return {"solves_per_s": 1.0 / dt, "ms": dt * 1e3, "n_states": 16, "newton_iters": rep["newton_iters"],
            "krylov_iters": rep["krylov_iters"], "mg_krylov_iters": rep["mg_krylov_iters"], "res_final": rep["res_final"],
            "dot_electrons": [float(x) for x in c],
            "max_dphi_vs_phi_k": float((ph - phi_sc).abs().max())}


def schrodinger_run(synth, qe, torch, dev, P, opts, phi_sc):
    """The Schrodinger step on the same stack: the 8 lowest states of a
    quantum region around the plunger P1 (x 0..70, y 60..140, z 40..100 nm)
    in V = E_C(phi_sc), from a random start to a relative residual of 1e-8;
    then the predictor-corrector loop with 16 states (the eigensolver warm
    started from the previous states, the predictor's Newton from phi^(k))
    until max |phi^(k) - phi^(k-1)| < 1e-5 V or 60 outer iterations."""
    inv_mass, v0, fixed, region = synth.quantum_region(dev, (0.0, 70.0, 60.0, 140.0, 40.0, 100.0))
    ws = qe.Workspace(qe.load_library().qe_schrodinger_workspace_bytes(qe.ctypes.byref(P.c()), 16), P.device)
    qe.qe_schrodinger_solve(P, inv_mass, v0, phi_sc, 8, fixed=fixed, tol=1e-8, maxit=3000, ws=ws)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E, psi, _, it = qe.qe_schrodinger_solve(P, inv_mass, v0, phi_sc, 8, fixed=fixed, tol=1e-8, maxit=3000, ws=ws)
    torch.cuda.synchronize()
    t_eig = time.perf_counter() - t0
    box = (0.0, 70.0, 60.0, 140.0, 40.0, 100.0)
    region_t = torch.as_tensor(region.astype("uint8"), device=P.device)
    t0 = time.perf_counter()
    phi_k, guess, hist, lob = phi_sc.clone(), None, [], []
    # each predictor solve starts from phi^(k), the previous outer step's potential
    opts_warm = qe.qe_default_options(newton_atol=opts.newton_atol, init_guess=1)
    newton = []
    for _ in range(60):
        E16, psi16, psi2, it16 = qe.qe_schrodinger_solve(P, inv_mass, v0, phi_k, 16, fixed=fixed, tol=1e-8,
                                                         maxit=3000, ws=ws, guess=guess)
        guess = psi16
        lob.append(it16)
        # the states stay on the device; the problem's other arrays are shared
        Pq = P.with_quantum(synth.QuantumStates(psi2=psi2, phi_k=phi_k, E_i=E16, region=region_t))
        new, _, rep = qe.qe_solve(Pq, opts=opts_warm, phi=phi_k.clone(), want_density=False)
        newton.append(rep["newton_iters"])
        hist.append(float((new - phi_k).abs().max()))
        phi_k = new
        if hist[-1] < 1e-5:
            break
    n_dot = qe.qe_count_electrons(Pq, phi_k, [box])[0]
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    # the loop's end state: converged, or settled into a two-cycle (every
    # other outer step repeats: successive max |dphi| equal to 1e-3 over the
    # last ten steps), or neither
    tail = hist[-10:]
    two_cycle = (hist[-1] >= 1e-5 and len(tail) == 10 and
                 all(abs(tail[i] - tail[i + 2]) <= 1e-3 * tail[i] for i in range(8)))
    state = "converged" if hist[-1] < 1e-5 else ("two-cycle" if two_cycle else "not converged")
    return {"eig8_ms": t_eig * 1e3, "eig8_lobpcg_iters": it, "E8_meV": [float(e * 1e3) for e in E],
            "sp_loop_s": t_loop, "sp_outer_iters": len(hist), "sp_final_dphi_V": hist[-1], "sp_state": state,
            "sp_dphi_history_V": hist,
            "sp_lobpcg_iters": lob, "sp_newton_iters": newton, "sp_dot_electrons": float(n_dot),
            "sp_levels_meV": [float(e * 1e3) for e in E16[:4]]}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--jv-reps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full", action="store_true", help="time the whole c2 oracle solve (minutes)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-full-charge", action="store_true")
    ap.add_argument("--no-sheets", action="store_true")
    ap.add_argument("--no-predictor", action="store_true")
    ap.add_argument("--no-schrodinger", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "slab decomposition is a design, not a build", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (before the GPU is initialised)")
        cpu = cpu_measure(full=args.cpu_full)

    import torch

    import synth
    from paper_1403_7561_amd import qe

    torch.cuda.set_device(0)
    dev = synth.config2()
    P = qe.Problem(dev)
    opts = qe.qe_default_options(newton_atol=1e-8)
    ws = qe.workspace_for(P, opts)
    boxes = [dev.boxes["D1"], dev.boxes["D2"]]
    phi = torch.zeros(P.N, dtype=torch.float64, device="cuda")

    def step():
        ph, _, rep = qe.qe_solve(P, opts=opts, phi=phi, want_density=True, ws=ws)
        c = qe.qe_count_electrons(P, ph, boxes, ws=ws)
        return rep, c

    log("warmup")
    for _ in range(args.warmup):
        step()
    log("timed steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for _ in range(args.steps):
        rep, counts = step()
        reps.append(rep)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = args.steps / (t1 - t0)

    # the same solve from the linear (charge-free) guess instead of the default
    # coarse-mesh sequence: the Newton count the oracle's sample is scaled to
    # (the oracle starts from the linear guess) and the sequence's gain
    opts_lin = qe.qe_default_options(newton_atol=1e-8, init_guess=0)
    qe.qe_solve(P, opts=opts_lin, phi=phi, want_density=False, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, rep_lin = qe.qe_solve(P, opts=opts_lin, phi=phi, want_density=False, ws=ws)
    torch.cuda.synchronize()
    t_lin = time.perf_counter() - t0
    # and with the Jacobi preconditioner on every CG (no multigrid)
    opts_jac = qe.qe_default_options(newton_atol=1e-8, precond=1)
    qe.qe_solve(P, opts=opts_jac, phi=phi, want_density=False, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, rep_jac = qe.qe_solve(P, opts=opts_jac, phi=phi, want_density=False, ws=ws)
    torch.cuda.synchronize()
    t_jac = time.perf_counter() - t0
    log(f"{value:.3f} solves/s; timing J.v")
    # J.v kernel alone (HIP events on the library's stream)
    v = torch.randn(P.N, dtype=torch.float64, device="cuda")
    ms64, ncoef = qe.qe_time_jv(P, phi, v, "fp64", args.jv_reps, ws=ws)
    ms32, ncoef32 = qe.qe_time_jv(P, phi, v, "mixed", args.jv_reps, ws=ws)
    b64 = jv_bytes(dev, 8, ncoef)
    b32 = jv_bytes(dev, 4, ncoef32)
    ach = b64 / (ms64 * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "double-dot Si/SiO2 stack 129x129x65 nodes (1081665 DOF), 5 gates, "
                               "Fermi-Dirac 4 K, FP64 Newton + PCG (Jacobi; multigrid V-cycle on the steps with CG "
                               "tolerance <= 3e-2) to ||F||<1e-8 from the default start (65x65x33 "
                               "coarse-mesh sequence, its inner CG in FP32)",
                   "global_batch": 1, "parallelism": "single GPU"},
        "newton_iters": reps[-1]["newton_iters"],
        "krylov_iters": reps[-1]["krylov_iters"],
        "init_krylov_iters": reps[-1]["init_krylov_iters"],
        "seq_levels": reps[-1]["seq_levels"],
        "mg_levels": reps[-1]["mg_levels"],
        "mg_krylov_iters": reps[-1]["mg_krylov_iters"],
        "linear_guess": {"ms": t_lin * 1e3, "newton_iters": rep_lin["newton_iters"],
                         "krylov_iters": rep_lin["krylov_iters"]},
        "jacobi_only": {"ms": t_jac * 1e3, "newton_iters": rep_jac["newton_iters"],
                        "krylov_iters": rep_jac["krylov_iters"]},
        "res_final": reps[-1]["res_final"],
        "dot_electrons": [float(c) for c in counts],
        "jv_gdof_s": {"fp64": P.N / (ms64 * 1e-3) / 1e9, "fp32": P.N / (ms32 * 1e-3) / 1e9,
                      "ms_fp64": ms64, "ms_fp32": ms32},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic("k_cg_jv<double>.c2"),
                     "cache_assisted": True,
                     "note": "the 129x129x65 CG working set (~74 MB) fits in the 256 MB Infinity Cache; "
                             "roofline_c5 (257x257x129, ~700 MB) is the HBM-bound figure",
                     "kernel": "k_cg_jv<double> (FP64 J.v of the CG loop with the direction update and the solution step)",
                     "bytes_per_launch": b64, "ms_per_launch": ms64,
                     "coef_elems": ncoef, "elems": dev.n_elems},
        "roofline_fp32": {"achieved": b32 / (ms32 * 1e-3) / 1e9, "bytes_per_launch": b32},
    }
    log("adjoint")
    if not args.no_adjoint:
        dev4 = synth.config4()
        P4 = qe.Problem(dev4)
        ws4 = qe.workspace_for(P4, opts)
        # differentiate the dot under the more positive plunger (the other is empty)
        box_name = "D1" if dev4.dir_val[0] >= dev4.dir_val[1] else "D2"
        ph4, _, _ = qe.qe_solve(P4, opts=opts, ws=ws4, want_density=False)      # warm-up
        qe.qe_adjoint(P4, ph4, dev4.boxes[box_name], opts=opts, ws=ws4)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        ph4, _, rep4 = qe.qe_solve(P4, opts=opts, ws=ws4, want_density=False)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        Q, dV, deps, _, arep = qe.qe_adjoint(P4, ph4, dev4.boxes[box_name], opts=opts, ws=ws4)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        # the adjoint CG with Jacobi instead of the V-cycle, for comparison
        _, dVj, _, _, arepj = qe.qe_adjoint(P4, ph4, dev4.boxes[box_name], opts=opts_jac, ws=ws4)
        torch.cuda.synchronize()
        td = time.perf_counter()
        out["adjoint"] = {"forward_ms": (tb - ta) * 1e3, "adjoint_ms": (tc - tb) * 1e3,
                          "ratio": (tc - tb) / (tb - ta), "box": box_name, "Q": Q,
                          "dQ_dV": [float(x) for x in dV],
                          "C_aF": [float(1.602176634e-19 * x * 1e18) for x in dV],
                          "forward_cg_iters": rep4["krylov_iters"], "adjoint_cg_iters": arep["krylov_iters"],
                          "adjoint_mg_levels": arep["mg_levels"],
                          "jacobi": {"adjoint_ms": (td - tc) * 1e3, "cg_iters": arepj["krylov_iters"],
                                     "dQ_dV_max_rel_diff": float(np.abs(np.asarray(dV) - np.asarray(dVj)).max()
                                                                 / np.abs(np.asarray(dVj)).max())}}
    if not args.no_batch:
        log("batched sweep (256 instances)")
        spec = synth.config3_spec()
        devs3 = [synth.config3_instance(k, spec) for k in range(len(spec[0]))]
        P3 = [qe.Problem(d) for d in devs3]
        cache = os.path.join("/tmp", "qe_batch_tune.txt")
        qe.qe_solve_batch(P3, opts=opts, boxes=boxes, tune_cache=cache)      # tunes once, cached
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, cnt3, reps3 = qe.qe_solve_batch(P3, opts=opts, boxes=boxes, tune_cache=cache)
        torch.cuda.synchronize()
        tb3 = time.perf_counter() - t0
        # the same 256 instances by the single-instance FP64 path, one after
        # another (one workspace sized for the largest)
        wsb = qe.Workspace(max(qe.qe_workspace_bytes(p, opts) for p in P3), P3[0].device)
        qe.qe_solve(P3[0], opts=opts, ws=wsb, want_density=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cnt_seq = []
        for p in P3:
            ph, _, _ = qe.qe_solve(p, opts=opts, ws=wsb, want_density=False)
            cnt_seq.append(qe.qe_count_electrons(p, ph, boxes, ws=wsb))
        torch.cuda.synchronize()
        ts3 = time.perf_counter() - t0
        cnt3 = np.asarray(cnt3, dtype=np.float64)
        cnt_seq = np.asarray(cnt_seq, dtype=np.float64)
        grid = cnt3.reshape(16, 16, 2)            # [P1 index, P2 index, dot]
        out["batch_c3"] = {"solves_per_s": len(P3) / tb3, "ms": tb3 * 1e3, "n_inst": len(P3),
                           "dof_total": int(sum(p.N for p in P3)),
                           "all_converged": all(r["status"] == 0 for r in reps3),
                           "max_res_final": max(r["res_final"] for r in reps3),
                           "sequential_solves_per_s": len(P3) / ts3, "sequential_ms": ts3 * 1e3,
                           "speedup_vs_sequential": ts3 / tb3,
                           "counts_max_rel_diff_vs_sequential":
                               float(np.abs(cnt3 - cnt_seq).max() / max(np.abs(cnt_seq).max(), 1e-300)),
                           "dot_electrons": {
                               "plunger_grid_V": [float(v) for v in synth.PLUNGER_GRID],
                               "D1_by_P1": [float(x) for x in grid[:, :, 0].mean(axis=1)],
                               "D2_by_P2": [float(x) for x in grid[:, :, 1].mean(axis=0)],
                               "max": [float(cnt3[:, 0].max()), float(cnt3[:, 1].max())],
                               "instances_with_an_electron": [int((cnt3[:, 0] > 0.5).sum()),
                                                              int((cnt3[:, 1] > 0.5).sum())]}}
        del P3, devs3, wsb
    if not args.no_mixed:
        log("mixed precision at 257x257x129")
        dev5 = synth.config5()
        P5 = qe.Problem(dev5)
        ws5 = qe.workspace_for(P5, opts)
        res = {}
        for prec in ("fp64", "mixed"):
            o5 = qe.qe_default_options(newton_atol=1e-8, precision=prec)
            qe.qe_solve(P5, opts=o5, ws=ws5, want_density=False)            # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ph5, _, r5 = qe.qe_solve(P5, opts=o5, ws=ws5, want_density=False)
            torch.cuda.synchronize()
            res[prec] = (time.perf_counter() - t0, ph5.clone(), r5)
        # the CG loop's kernel at the FP64 solution: vectors and coefficients
        # exceed the 256 MB Infinity Cache here, so this rate is HBM-bound
        v5 = torch.randn(P5.N, dtype=torch.float64, device="cuda")
        ms5_64, nc5_64 = qe.qe_time_jv(P5, res["fp64"][1], v5, "fp64", args.jv_reps, ws=ws5)
        ms5_32, nc5_32 = qe.qe_time_jv(P5, res["fp64"][1], v5, "mixed", args.jv_reps, ws=ws5)
        b5_64, b5_32 = jv_bytes(dev5, 8, nc5_64), jv_bytes(dev5, 4, nc5_32)
        t5_64, t5_32 = measured_traffic("k_cg_jv<double>.c5"), measured_traffic("k_cg_jv<float>.c5")
        out["roofline_c5"] = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "achieved": b5_64 / (ms5_64 * 1e-3) / 1e9,
                              "frac": b5_64 / (ms5_64 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "traffic": t5_64,
                              "traffic_frac": None if t5_64 is None else t5_64 / (ms5_64 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "kernel": "k_cg_jv<double>", "bytes_per_launch": b5_64, "ms_per_launch": ms5_64,
                              "coef_elems": nc5_64,
                              "fp32": {"kernel": "k_cg_jv<float>", "achieved": b5_32 / (ms5_32 * 1e-3) / 1e9,
                                       "frac": b5_32 / (ms5_32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                       "traffic": t5_32,
                                       "traffic_frac": None if t5_32 is None else
                                       t5_32 / (ms5_32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                       "bytes_per_launch": b5_32, "ms_per_launch": ms5_32},
                              "gdof_s": {"fp64": P5.N / (ms5_64 * 1e-3) / 1e9, "fp32": P5.N / (ms5_32 * 1e-3) / 1e9}}
        d = (res["mixed"][1] - res["fp64"][1]).abs().max().item() / res["fp64"][1].abs().max().item()
        out["mixed_c5"] = {"fp64_s": res["fp64"][0], "mixed_s": res["mixed"][0],
                           "speedup": res["fp64"][0] / res["mixed"][0],
                           "max_rel_diff_phi": d,
                           "fp64_cg_iters": res["fp64"][2]["krylov_iters"],
                           "mixed_cg_iters": res["mixed"][2]["krylov_iters"],
                           "res_final": [res["fp64"][2]["res_final"], res["mixed"][2]["res_final"]]}
        del P5, ws5, res
    if not args.no_full_charge:
        log("full space charge on the same stack")
        out["full_charge_c2"] = full_charge_run(synth, qe, torch, dev, opts, boxes, args.jv_reps)
    if not args.no_sheets:
        log("interface charge and charged plunger gates on the same stack")
        out["sheets_c2"] = sheets_run(synth, qe, torch, dev, opts, ws, boxes)
    if not args.no_predictor:
        log("predictor step with 16 synthetic dot states")
        out["predictor_c2"] = predictor_run(synth, qe, torch, dev, P, opts, boxes, phi)
    if not args.no_schrodinger:
        log("Schrodinger states and the predictor-corrector loop")
        out["schrodinger_c2"] = schrodinger_run(synth, qe, torch, dev, P, opts, phi)
    if cpu is not None:
        out["cpu_baseline"] = cpu_baseline(cpu, rep_lin["newton_iters"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
