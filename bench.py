"""Benchmark: the STFAS keyframe smoke-control solve on one MI355X.

One step = one full solve (the ADMM loop of Alg:outter with the density and
velocity subproblems, run to its visual-difference stop, then the
re-simulated outputs) of the 128x128, 40-step 2D workload (a blurred disk to a
union of strokes at t = 40, r = 1e-4) in the mixed-precision form (FP32 bulk,
FP64 coarsest projection level and reductions), with the paper's upwind
exponential density operator (eq:Adv).  Inputs are synthetic and seeded and
already resident on the device.

Prints one JSON line: the solve rate (spacetime cell-updates per second of
the fine V-cycles), the solve time to the stop and the keyframe error of the
mixed solve against the FP64 solve of the same workload on the GPU (the
"1e-4 keyframe error" of the metric), the roofline of the dominant kernel
(launches timed with HIP events on the solver's stream; the method's bytes
per launch; counter-measured HBM bytes from the committed profile), the same
workload with the semi-Lagrangian density operator, the L-BFGS and
augmented-Lagrangian-fallback comparisons, the 3D precision form, the
64-request serving run against a FIFO loop, and the oracle's CPU rate on one
thread and on all host cores."""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = ("2D 128x128 MAC grid, 40 steps, r=1e-4, disk to stroke keyframe at t=40, upwind exponential density "
            "operator, mixed precision, ADMM to the visual-difference stop max(rho0)/100")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-admm", type=int, default=100)
    ap.add_argument("--density", default="upwind", choices=["upwind", "sl"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-check", action="store_true")
    ap.add_argument("--trace-kernel", default="kkt_split",
                    help="kernel family of the roofline: its launches on the finest level are timed with HIP events "
                         "in an extra (untimed) solve")
    ap.add_argument("--calibrate", action="store_true",
                    help="start with the 256 MiB device copy the counter passes are scaled by")
    ap.add_argument("--lbfgs-iters", type=int, default=200,
                    help="iteration cap of the L-BFGS comparison (0 skips it)")
    ap.add_argument("--no-sl", action="store_true", help="skip the solve with the semi-Lagrangian density operator")
    ap.add_argument("--al-admm", type=int, default=10,
                    help="ADMM cap of the solves with and without the augmented-Lagrangian fallback (0 skips them)")
    ap.add_argument("--al-tol", type=float, default=0.05,
                    help="relative objective decrease below which the fallback updates the multipliers")
    ap.add_argument("--no-3d", action="store_true", help="skip the 64^3 x 60 precision-form comparison")
    ap.add_argument("--no-rotational", action="store_true",
                    help="skip the solves with the paper's rotational velocity operator")
    ap.add_argument("--serve-requests", type=int, default=64, help="0 skips the serving run")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-budget-gb", type=float, default=24.0)
    return ap.parse_args()


def progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def solve_once(S, w, precision, density, **kw):
    """One solve on a fresh context; returns (stats, u as float64 numpy)."""
    import numpy as np
    import torch
    dt = torch.float64 if precision == "fp64" else torch.float32
    prob = S.make_problem(w["n"], w["num_steps"], w["r"], dt=w["dt"], precision=precision, density=density, **kw)
    ctx = S.stfas_create(prob)
    ks = sorted(w["keys"])
    rho0 = torch.tensor(w["rho0"], dtype=dt, device="cuda")
    keys = torch.tensor(np.stack([w["keys"][k] for k in ks]), dtype=dt, device="cuda")
    u = torch.zeros(w["num_steps"] * ctx.faces, dtype=dt, device="cuda")
    st = S.stfas_solve(ctx, rho0, ks, keys, u)
    ctx.destroy()
    return st, u.double().cpu().numpy()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: measures one GPU only (the solve is not sharded across GPUs); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synthetic
    from paper_1608_01102_amd import stfas as S

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate:
        from paper_1608_01102_amd.profiling import calibration_copy
        calibration_copy()
    w = synthetic.c2_plain_2d_128(args.seed)
    n, N = w["n"], w["num_steps"]
    kw = dict(max_admm=args.max_admm)
    prob = S.make_problem(n, N, w["r"], dt=w["dt"], precision="mixed", density=args.density, **kw)
    ctx = S.stfas_create(prob)
    ks = sorted(w["keys"])
    rho0 = torch.tensor(w["rho0"], dtype=torch.float32, device=dev)
    keys = torch.tensor(np.stack([w["keys"][k] for k in ks]), dtype=torch.float32, device=dev)
    u = torch.zeros(N * ctx.faces, dtype=torch.float32, device=dev)

    for _ in range(args.warmup):
        S.stfas_solve(ctx, rho0, ks, keys, u)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats.append(S.stfas_solve(ctx, rho0, ks, keys, u))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    progress(f"{args.steps} timed solves done, {ms:.1f} ms each")
    vcycles = sum(s["vcycles"] for s in stats) / len(stats)
    cells = n[0] * n[1]
    value = cells * N * vcycles / (ms * 1e-3)
    last = stats[-1]
    u_mixed = u.double().cpu().numpy()
    out = {
        "metric": "KKT solve s to 1e-4 keyframe err; spacetime cell-upd/s; serve p50/p99",
        "value": value,
        "unit": "spacetime cell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": WORKLOAD if args.density == "upwind" else WORKLOAD.replace(
                       "upwind exponential", "semi-Lagrangian"),
                   "grid": list(n), "num_steps": N, "precision": "mixed", "density_op": args.density,
                   "eps_admm": "max(rho0)/100", "max_admm": args.max_admm, "parallelism": "single GPU"},
        "solve_s": ms * 1e-3,
        "admm_iters": last["admm_iters"], "vcycles": last["vcycles"], "converged": bool(last["converged"]),
        "objective": last["objective"], "kkt_res_inf": last["kkt_res_inf"], "visual_diff": last["visual_diff"],
    }
    # rooflines: one more solve per kernel family with its finest-level launches timed by HIP events
    out["roofline"] = roofline(S, ctx, rho0, ks, keys, u, args.trace_kernel)
    if args.density == "upwind" and args.trace_kernel != "up_term":
        # the upwind series term: most kernel time in total, but each launch is a 16384-cell dispatch of a
        # few microseconds, which a per-launch event pair cannot resolve (it adds the dispatch gap)
        out["roofline_density_op"] = roofline(S, ctx, rho0, ks, keys, u, "up_term")
    ctx.destroy()
    progress("rooflines done")
    if not args.no_fp64_check:
        # the same solve in FP64 on the GPU (untimed): the mixed form's keyframe error against it
        s64, u64 = solve_once(S, w, "fp64", args.density, **kw)
        kf = keyframe_error(S, w, args.density, u_mixed, u64)
        out["kf_err_vs_fp64_gpu"] = kf
        out["meets_1e-4_kf_err"] = bool(kf <= 1e-4 and last["converged"] and s64["converged"])
        out["fp64_gpu"] = {"objective": s64["objective"], "admm_iters": s64["admm_iters"],
                           "vcycles": s64["vcycles"], "converged": bool(s64["converged"]),
                           "seconds": s64["seconds"]}
        progress("fp64 solve done")
    if not args.no_sl:
        out["sl_density"] = sl_run(S, w, kw, args.no_fp64_check)
        progress("semi-Lagrangian solves done")
    if args.lbfgs_iters > 0:
        out["lbfgs_baseline"] = lbfgs_run(S, w, args.density, args.lbfgs_iters, last)
        progress("L-BFGS done")
    if args.al_admm > 0:
        out["al_fallback"] = al_run(S, w, args.density, args.al_admm, args.al_tol)
        progress("augmented-Lagrangian solves done")
    if not args.no_rotational:
        out["rotational_velocity"] = rotational_run(S, w, args.density, kw)
        progress("rotational-operator solves done")
        if args.lbfgs_iters > 0:
            out["rotational_velocity"]["lbfgs"] = lbfgs_run(
                S, w, args.density, min(args.lbfgs_iters, ROT_LBFGS_CAP), out["rotational_velocity"]["mixed"],
                velocity="rotational")
            progress("rotational-operator L-BFGS done")
    if not args.no_3d:
        out["precision_3d"] = precision_3d_run(S)
        progress("3D solves done")
        if not args.no_rotational:
            out["rotational_velocity_3d"] = precision_3d_run(S, velocity="rotational")
            progress("3D rotational-operator solves done")
    if args.serve_requests > 0:
        out["serving"] = serving_run(args)
        progress("serving done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
        progress("cpu baseline done")
    print(json.dumps(out), flush=True)


def roofline(S, ctx, rho0, ks, keys, u, kernel):
    """Achieved HBM rate of one kernel family over one solve: the method's
    bytes of its launches / their summed duration (HIP events on the solver's
    stream), against 8 TB/s; `traffic` is the counter-measured HBM bytes per
    launch from the committed profile (None when there is none or the kernel
    sources changed since)."""
    import torch
    S.stfas_trace_enable(ctx, kernel, 1 << 17)
    S.stfas_solve(ctx, rho0, ks, keys, u)
    torch.cuda.synchronize()
    n, tms, tbytes, timpl = S.stfas_trace_read(ctx)
    S.stfas_trace_enable(ctx, 0, 0)
    if not n:
        return None
    achieved = tbytes / (tms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
            "frac": achieved / 8000.0, "traffic": measured_traffic(kernel),
            "avg_launch_us": tms * 1e3 / n, "launches_timed": n, "alg_bytes_per_launch": tbytes / n,
            "impl_bytes_per_launch": timpl / n, "alg_bytes_rule": alg_rule(kernel)}


def alg_rule(kernel):
    rules = {"kkt_split": "the rows of one colour's cells per SCGS colour pass (and every cell for a whole-level "
                          "residual): 80 B per spacetime cell in 2D, 108 B in 3D (v, u, pbar, p, w, res in, r out; "
                          "FP32)",
             "self_advect_T": "v, y in and J_S^T y out: 24 B per spacetime cell in 2D, 36 B in 3D (FP32)",
             "up_term": "per working term of the upwind series (launches past the series' stop credited 0): "
                        "T_(j-1) in, T_j out, the running sum read and written per cell and v per face "
                        "(16 B per cell + 4 B per face, FP32); the first launch (j = 0) reads rho and copies it "
                        "into the sum (8 B per cell)"}
    return rules.get(kernel, "the kernel family's inputs and outputs once")


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter summary of this kernel
    on this workload, or None when there is none or the kernel sources
    changed since it was taken."""
    from paper_1608_01102_amd.profiling import kernel_source_hash
    path = os.path.join(ROOT, "profiles", f"{kernel}_128x128x40_pmc.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        key = line.split(":")[0]
        if ":" in line and key in ("traffic_bytes_per_launch", "kernel_source_hash"):
            vals[key] = line.split(":", 1)[1].strip()
    if vals.get("kernel_source_hash") != kernel_source_hash() or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def sl_run(S, w, kw, no_fp64):
    """The same workload with the semi-Lagrangian density operator (outside
    the step clock): iterations, seconds and, against its FP64 solve, the
    keyframe error of the mixed form."""
    s, u = solve_once(S, w, "mixed", "sl", **kw)          # warm-up
    s, u = solve_once(S, w, "mixed", "sl", **kw)
    res = {"admm_iters": s["admm_iters"], "vcycles": s["vcycles"], "converged": bool(s["converged"]),
           "objective": s["objective"], "seconds": s["seconds"],
           "cell_updates_per_s": w["n"][0] * w["n"][1] * w["num_steps"] * s["vcycles"] / s["seconds"]}
    if not no_fp64:
        s64, u64 = solve_once(S, w, "fp64", "sl", **kw)
        res["kf_err_vs_fp64_gpu"] = keyframe_error(S, w, "sl", u, u64)
        res["fp64_admm_iters"] = s64["admm_iters"]
    return res


def lbfgs_run(S, w, density, iters, admm_stats, velocity="sl"):
    """The gradient-based baseline of the paper's comparison (Sec. 5, outside
    the step clock): L-BFGS from u = 0 on the same problem, precision and
    objective, stopped by the same visual-difference rule as the ADMM loop
    (or the iteration cap); its time, its objective and the first iteration
    (if any) at which it reaches the ADMM solve's objective.  velocity:
    the velocity operator of both (the rotational one's gradient is the
    adjoint of its fixed-point steps)."""
    import numpy as np
    import torch
    prob = S.make_problem(w["n"], w["num_steps"], w["r"], dt=w["dt"], precision="mixed", density=density,
                          velocity=velocity)
    ctx = S.stfas_create(prob)
    ks = sorted(w["keys"])
    rho0 = torch.tensor(w["rho0"], dtype=torch.float32, device="cuda")
    keys = torch.tensor(np.stack([w["keys"][k] for k in ks]), dtype=torch.float32, device="cuda")
    eps = float(np.max(w["rho0"])) / 100.0
    u = torch.zeros(w["num_steps"] * ctx.faces, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist, done = S.stfas_lbfgs(ctx, rho0, ks, keys, u, iters, eps)
    sec = time.perf_counter() - t0
    ctx.destroy()
    target = admm_stats["objective"]
    reach = next((i for i, j in enumerate(hist) if j <= target), None)
    return {"iters": done, "iter_cap": iters, "eps_stop": eps, "stopped_before_cap": done < iters, "seconds": sec,
            "objective_start": hist[0], "objective": hist[-1], "admm_objective": target,
            "admm_seconds": admm_stats["seconds"], "reaches_admm_at_iter": reach}


def al_run(S, w, density, max_admm, al_tol):
    """The augmented-Lagrangian fallback of the ADMM loop (outside the step
    clock): the same workload and ADMM cap solved with plain ADMM and with
    the multiplier update held while the density subproblem's objective still
    falls by more than al_tol; ADMM iterations, multiplier updates, objective,
    visual difference and seconds of each (one warm-up solve first)."""
    res = {"admm_cap": max_admm, "al_tol": al_tol}
    for name, tol in (("plain", 0.0), ("fallback", al_tol)):
        solve_once(S, w, "mixed", density, al_tol=tol, max_admm=max_admm)
        st, _ = solve_once(S, w, "mixed", density, al_tol=tol, max_admm=max_admm)
        res[name] = {"admm_iters": st["admm_iters"], "multiplier_updates": st["multiplier_updates"],
                     "vcycles": st["vcycles"], "objective": st["objective"], "visual_diff": st["visual_diff"],
                     "seconds": st["seconds"]}
    return res


def rotational_run(S, w, density, kw):
    """The same workload with the paper's own velocity operator (eq:NSA: the
    implicit rotational form, 2D), outside the step clock: the mixed solve
    (after a warm-up solve) and the FP64 solve to the ADMM stop, their
    iterations, seconds and objective, and the mixed form's keyframe error
    against the FP64 run."""
    solve_once(S, w, "mixed", density, velocity="rotational", **kw)
    res, us, conv = {}, {}, []
    for prec in ("mixed", "fp64"):
        st, us[prec] = solve_once(S, w, prec, density, velocity="rotational", **kw)
        res[prec] = {"admm_iters": st["admm_iters"], "vcycles": st["vcycles"], "converged": bool(st["converged"]),
                     "seconds": st["seconds"], "objective": st["objective"], "visual_diff": st["visual_diff"]}
        conv.append(bool(st["converged"]))
    kf = keyframe_error(S, w, density, us["mixed"], us["fp64"], velocity="rotational")
    res["kf_err_mixed_vs_fp64"] = kf
    res["meets_1e-4_kf_err"] = bool(kf <= 1e-4 and all(conv))
    res["cell_updates_per_s"] = (w["n"][0] * w["n"][1] * w["num_steps"] * res["mixed"]["vcycles"]
                                 / res["mixed"]["seconds"])
    # the smoother's other local matrices (mixed): eq:HESS's block on every
    # level, and on none (which needs the perturbation mu dt^2 = 1 to stay finite)
    res["smoother"] = {"default": "local block of dAdv/dv on the finest level, omega 1, no perturbation"}
    for name, extra in (("block_every_level", dict(scgs_local="exact")),
                        ("no_block_mu1", dict(scgs_local="collapsed", scgs_lm=1.0))):
        st, _ = solve_once(S, w, "mixed", density, velocity="rotational", **extra, **kw)
        res["smoother"][name] = {"admm_iters": st["admm_iters"], "vcycles": st["vcycles"],
                                 "converged": bool(st["converged"]), "seconds": st["seconds"]}
    return res


EQUAL_COUNTS = (20, 3)   # ADMM iterations, V-cycles per iteration
ROT_LBFGS_CAP = 150       # L-BFGS iterations with the rotational operator


def precision_3d_run(S, velocity="sl"):
    """The 3D precision form (outside the step clock): the 64^3, 60-step
    workload (sphere to ellipsoid unions at t = 30 and 60, SL density) solved
    to the ADMM stop in the mixed form and in FP64 on the GPU, with
    K dt^2 / r = 4 and four density-subproblem iterations per ADMM iteration
    (with the defaults the solve does not reach the stop within 100
    iterations; at K dt^2 / r = 2 the mixed form's stop comes at 74 to over
    100 iterations from run to run), cap 150; iterations, seconds, seconds
    per V-cycle, final visual difference, and the mixed
    form's keyframe error against the FP64 run after re-simulating both
    controls with the FP64 step; then both forms again with equal fixed
    iteration counts (EQUAL_COUNTS), whose keyframe error is that of the
    arithmetic alone, for the SL and for the upwind density operator.
    velocity="rotational" runs the same with the paper's rotational operator
    (vorticity on edges; its smoother without the local block in 3D)."""
    import torch
    import synthetic
    w = synthetic.c3_precision_3d(0)
    opts = dict(K=4.0 * w["r"] / w["dt"] ** 2, ao_iters=4, max_admm=150)
    res, us, conv = {}, {}, []
    for prec in ("mixed", "fp64"):
        st, us[prec] = solve_once(S, w, prec, "sl", velocity=velocity, **opts)
        res[prec] = {"seconds": st["seconds"], "admm_iters": st["admm_iters"], "vcycles": st["vcycles"],
                     "converged": bool(st["converged"]),
                     "ms_per_vcycle_incl_ao": st["seconds"] * 1e3 / max(st["vcycles"], 1),
                     "objective": st["objective"], "visual_diff": st["visual_diff"]}
        conv.append(bool(st["converged"]))
        torch.cuda.empty_cache()
    kf = keyframe_error(S, w, "sl", us["mixed"], us["fp64"], velocity=velocity)
    res["kf_err_mixed_vs_fp64"] = kf
    res["meets_1e-4_kf_err"] = bool(kf <= 1e-4 and all(conv))
    # the same solves with equal iteration counts in both forms: the difference
    # left is that of the arithmetic, not of the iteration where the stop fires
    # (with the SL velocity operator also with the upwind density operator,
    # smooth in v where the SL backtrace's cell choice is not)
    fc = dict(opts, max_admm=EQUAL_COUNTS[0], max_vcycles=EQUAL_COUNTS[1], fixed_counts=True)
    eq = {"admm_iters": EQUAL_COUNTS[0], "vcycles_per_admm": EQUAL_COUNTS[1]}
    for density in ("sl", "upwind") if velocity == "sl" else ("sl",):
        d = eq if density == "sl" else eq.setdefault("upwind_density", {})
        for prec in ("mixed", "fp64"):
            st, us[prec] = solve_once(S, w, prec, density, velocity=velocity, **fc)
            d[prec + "_seconds"] = st["seconds"]
            torch.cuda.empty_cache()
        d["kf_err_mixed_vs_fp64"] = keyframe_error(S, w, density, us["mixed"], us["fp64"], velocity=velocity)
    res["equal_counts"] = eq
    res["workload"] = ("3D 64^3 MAC grid, 60 steps, r=1e-3, SL density, K dt^2/r = 4, 4 density-subproblem "
                       "iterations, ADMM to the visual-difference stop max(rho0)/100"
                       + (", rotational velocity operator" if velocity != "sl" else ""))
    return res


def keyframe_error(S, w, density, u_a, u_b, velocity="sl"):
    """max over keyframes of |rho_a - rho_b| / |rho_b| after re-simulating both
    control sequences with the FP64 step of the library (with the velocity
    operator the controls were solved for)."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    N = w["num_steps"]
    p64 = S.make_problem(w["n"], 1, w["r"], dt=w["dt"], precision="fp64", density=density, velocity=velocity)
    cells, faces = S.counts(p64)
    work = torch.empty(S.stfas_step_work_bytes(p64), dtype=torch.uint8, device=dev)

    def run(u):
        ut = torch.tensor(u.reshape(N, faces), dtype=torch.float64, device=dev)
        rho = torch.tensor(w["rho0"], dtype=torch.float64, device=dev)
        v = torch.zeros(faces, dtype=torch.float64, device=dev)
        out = {}
        for i in range(N):
            rn, vn = torch.empty_like(rho), torch.empty_like(v)
            S.stfas_step_forward(p64, rho, v, ut[i], rn, vn, work=work)
            rho, v = rn, vn
            if i + 1 in w["keys"]:
                out[i + 1] = rho.cpu().numpy()
        return out
    a, b = run(u_a), run(u_b)
    return max(float(np.linalg.norm(a[t] - b[t]) / np.linalg.norm(b[t])) for t in b)


SERVE_CAP = dict(max_admm=2, max_vcycles=3, fixed_counts=True)


def serving_run(args):
    """Continuous batching of the 64-request mixed 2D/3D stream against a
    FIFO loop, both in real time on the same Poisson arrivals (rate 0.8 x the
    FIFO loop's closed-loop throughput, measured first).  Each request is
    capped at 2 ADMM iterations of 3 V-cycles (fixed counts): with full solves
    the 96^3 x 60 requests alone would take minutes."""
    import synthetic
    from paper_1608_01102_amd import serving
    raw = synthetic.c5_requests(args.seed, args.serve_requests, rate=1.0)
    reqs = [serving.Request(q["rid"], q["arrival"], q["n"], q["num_steps"], q["r"], q["rho0"], q["key_steps"],
                            q["key_rho"], dict(dt=q["dt"], **SERVE_CAP)) for q in raw]
    _, closed_span = serving.run_sequential(reqs, realtime=False)
    rate = 0.8 * len(reqs) / closed_span
    for q, r0 in zip(reqs, raw):
        q.arrival = r0["arrival"] / rate
    fifo, fifo_span = serving.run_sequential(reqs, realtime=True)
    srv = serving.Server(budget_bytes=int(args.serve_budget_gb * 2 ** 30), max_slots=args.serve_slots,
                         precision="mixed")
    res, span = srv.run(reqs, realtime=True)
    cont = serving.summary(res, span)
    seq = serving.summary(fifo, fifo_span)
    return {"requests": len(reqs), "arrival_rate_per_s": rate, "slots": args.serve_slots,
            "budget_gb": args.serve_budget_gb, "max_bypass": srv.max_bypass,
            "mix": {"2d": sum(len(q.n) == 2 for q in reqs), "3d": sum(len(q.n) == 3 for q in reqs)},
            "continuous": {k: cont[k] for k in ("p50_s", "p99_s", "mean_s", "solves_per_hour", "makespan_s")},
            "fifo": {k: seq[k] for k in ("p50_s", "p99_s", "mean_s", "solves_per_hour", "makespan_s")},
            "fifo_closed_loop_solves_per_hour": 3600.0 * len(reqs) / closed_span,
            "per_request": "2 ADMM iterations x 3 V-cycles (fixed counts), mixed precision, SL density",
            "latency": "arrival to result, both measured in real time"}


def _oracle_vcycles(sample):
    """The timed oracle work (one process): `cycles` FAS V-cycles of the
    velocity subproblem on the 128x128 x 40 problem with the BLAS and OpenMP
    pools held to one thread; returns the seconds."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import synthetic
    from oracle import kkt, stfas
    from oracle.grid import Grid
    n, N, dt, cycles = sample
    g = Grid(n)
    H = stfas.Hierarchy(g, N, dt, 1.0 / dt ** 2, omega=0.7, lm=1.0)
    rng = np.random.default_rng(0)
    tw = np.stack([synthetic.curl_noise_velocity(n, rng, 4.0, 0.5) for _ in range(N)])
    x = kkt.zeros_state(H.levels[0])
    ws = H.targets(tw)
    res = [np.zeros_like(a) for a in x]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for _ in range(cycles):
            stfas.vcycle(H, 0, x, ws, res)
        return time.perf_counter() - t0


def cpu_baseline(w):
    """The FP64 oracle timed on this host: two FAS V-cycles of the velocity
    subproblem on the benchmark's own 128x128 x 40-step problem (same
    operators, levels and smoother settings as the GPU solve's V-cycles),
    once on one thread and once in as many independent processes as the host
    has cores (up to 16), each on one thread; `cores` is what the all-core
    leg used."""
    import multiprocessing as mp
    n, N = w["n"], w["num_steps"]
    cycles = 2
    sample = (n, N, w["dt"], cycles)
    work = n[0] * n[1] * N * cycles
    t1 = _oracle_vcycles(sample)
    procs = max(1, min(16, os.cpu_count() or 1))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        times = pool.map(_oracle_vcycles, [sample] * procs)
    wall = time.perf_counter() - t0
    return {"value": procs * work / wall, "unit": "spacetime cell-updates/s", "cores": procs, "kind": "oracle",
            "sample": f"{cycles} FP64 oracle V-cycles of the velocity subproblem on the 128x128 x {N}-step problem "
                      f"in each of {procs} processes (NumPy, one thread each; {wall:.1f} s wall including process "
                      f"start, {max(times):.1f} s the slowest process's V-cycles)",
            "one_thread": {"value": work / t1, "cores": 1, "seconds": t1},
            "host_cpus": os.cpu_count()}


if __name__ == "__main__":
    main()
