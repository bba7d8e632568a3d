"""Benchmark: the STFAS keyframe smoke-control solve on one MI355X.

One step = one full solve (ADMM with density and velocity subproblems,
then the re-simulated outputs) of the 128x128, 40-step 2D workload in the
mixed-precision form (FP32 bulk, FP64 coarsest projection level and
reductions), regularisation 1e-4, ADMM stopped at 1e-4 * max(rho_0)
visual difference or 50 iterations.  Inputs are synthetic and seeded
(a blurred disk to a union of strokes), already resident on the device.

Prints one JSON line: the solve rate with its roofline (the finest residual
launch, timed with HIP events on the solver's stream, and its counter-
measured HBM bytes), the FP64 solve beside the mixed one, the L-BFGS,
upwind-operator and augmented-Lagrangian-fallback comparisons, the 3D
precision form, the serving run and the oracle's CPU rate."""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-admm", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-check", action="store_true")
    ap.add_argument("--trace-kernel", default="kkt_split",
                    help="kernel family whose launches on the finest level are timed with HIP events")
    ap.add_argument("--lbfgs-iters", type=int, default=200,
                    help="iteration cap of the L-BFGS comparison (0 skips it)")
    ap.add_argument("--upwind-admm", type=int, default=10,
                    help="ADMM cap of the solve with the upwind exponential density operator (0 skips it)")
    ap.add_argument("--al-admm", type=int, default=10,
                    help="ADMM cap of the solves with and without the augmented-Lagrangian fallback (0 skips them)")
    ap.add_argument("--al-tol", type=float, default=0.05,
                    help="relative objective decrease below which the fallback updates the multipliers")
    ap.add_argument("--no-3d", action="store_true", help="skip the 64^3 x 60 precision-form comparison")
    ap.add_argument("--serve-requests", type=int, default=16, help="0 skips the serving run")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-budget-gb", type=float, default=24.0)
    return ap.parse_args()


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
    w = synthetic.c2_plain_2d_128(args.seed)
    n, N = w["n"], w["num_steps"]
    rho_max = float(np.max(w["rho0"]))
    kw = dict(dt=w["dt"], eps_admm=1e-4 * rho_max, max_admm=args.max_admm)
    prob = S.make_problem(n, N, w["r"], precision="mixed", **kw)
    ctx = S.stfas_create(prob)
    ks = sorted(w["keys"])
    rho0 = torch.tensor(w["rho0"], dtype=torch.float32, device=dev)
    keys = torch.tensor(np.stack([w["keys"][k] for k in ks]), dtype=torch.float32, device=dev)
    u = torch.zeros(N * ctx.faces, dtype=torch.float32, device=dev)

    for _ in range(args.warmup):
        S.stfas_solve(ctx, rho0, ks, keys, u)
    torch.cuda.synchronize()
    S.stfas_trace_enable(ctx, args.trace_kernel, 8192)
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats.append(S.stfas_solve(ctx, rho0, ks, keys, u))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    nlaunch, tms, tbytes, _impl = S.stfas_trace_read(ctx)
    S.stfas_trace_enable(ctx, 0, 0)
    vcycles = sum(s["vcycles"] for s in stats) / len(stats)
    cells = n[0] * n[1]
    value = cells * N * vcycles / (ms * 1e-3)
    last = stats[-1]
    out = {
        "metric": "KKT solve s to 1e-4 keyframe err; spacetime cell-upd/s; serve p50/p99",
        "value": value,
        "unit": "spacetime cell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "2D 128x128 MAC grid, 40 steps, r=1e-4, stroke keyframe at t=40 (mixed precision)",
                   "grid": list(n), "num_steps": N, "precision": "mixed", "parallelism": "single GPU"},
        "solve_s": ms * 1e-3,
        "admm_iters": last["admm_iters"], "vcycles": last["vcycles"], "converged": bool(last["converged"]),
        "objective": last["objective"], "kkt_res_inf": last["kkt_res_inf"], "visual_diff": last["visual_diff"],
    }
    if nlaunch:
        avg_us = tms * 1e3 / nlaunch
        achieved = tbytes / (tms * 1e-3) / 1e9
        traffic, valu_us = measured_counters(args.trace_kernel)
        out["roofline"] = {"bound": "hbm", "kernel": args.trace_kernel, "achieved": achieved, "peak": 8000.0,
                           "unit": "GB/s", "frac": achieved / 8000.0,
                           "traffic": traffic,
                           "avg_launch_us": avg_us, "launches_timed": nlaunch,
                           "alg_bytes_per_launch": tbytes / nlaunch,
                           # VALU-busy share of the launch from the committed counters (instruction issue,
                           # not HBM, is what limits this launch; see the counter summary)
                           "valu_busy_frac": (valu_us / avg_us) if valu_us else None}
    u_mixed = u.double().cpu().numpy()
    if not args.no_fp64_check:
        # same solve in FP64 on the GPU (untimed): the mixed form's keyframe error against it
        p64 = S.make_problem(n, N, w["r"], precision="fp64", **kw)
        c64 = S.stfas_create(p64)
        u64 = torch.zeros(N * ctx.faces, dtype=torch.float64, device=dev)
        s64 = S.stfas_solve(c64, rho0.double(), ks, keys.double(), u64)
        kf = keyframe_error(S, p64, w, u_mixed, u64.cpu().numpy())
        out["fp64_gpu"] = {"objective": s64["objective"], "admm_iters": s64["admm_iters"],
                           "seconds": s64["seconds"], "kf_err_mixed_vs_fp64": kf}
        c64.destroy()
    if args.lbfgs_iters > 0:
        out["lbfgs_baseline"] = lbfgs_run(S, ctx, rho0, ks, keys, args.lbfgs_iters, kw["eps_admm"], last)
    ctx.destroy()
    if args.upwind_admm > 0:
        out["upwind_solve"] = upwind_run(S, w, kw, rho0, ks, keys, args.upwind_admm, last)
    if args.al_admm > 0:
        out["al_fallback"] = al_run(S, w, kw, rho0, ks, keys, args.al_admm, args.al_tol)
    if not args.no_3d:
        out["precision_3d"] = precision_3d_run(S)
    if args.serve_requests > 0:
        out["serving"] = serving_run(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


def measured_counters(kernel):
    """HBM bytes per launch and the VALU-busy time per launch from the
    committed counter summary of this kernel, or None for each when there is
    none or the kernel sources changed since."""
    from paper_1608_01102_amd.profiling import kernel_source_hash
    path = os.path.join(ROOT, "profiles", f"{kernel}_128x128x40_pmc.md")
    if not os.path.exists(path):
        return None, None
    vals = {}
    for line in open(path):
        key = line.split(":")[0]
        if ":" in line and key in ("traffic_bytes_per_launch", "valu_busy_us_per_launch", "kernel_source_hash"):
            vals[key] = line.split(":", 1)[1].strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None, None
    t = float(vals["traffic_bytes_per_launch"]) if "traffic_bytes_per_launch" in vals else None
    u = float(vals["valu_busy_us_per_launch"]) if "valu_busy_us_per_launch" in vals else None
    return t, u


def lbfgs_run(S, ctx, rho0, ks, keys, iters, eps, admm_stats):
    """The gradient-based baseline of the paper's comparison (outside the
    step clock): L-BFGS from u = 0 on the same problem, precision and
    objective, stopped by the same visual-difference rule as the ADMM loop
    (or the iteration cap); reports its time, its objective and the first
    iteration (if any) at which it reaches the ADMM solve's objective."""
    import torch
    u = torch.zeros(ctx.N * ctx.faces, dtype=torch.float32, device=rho0.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist, done = S.stfas_lbfgs(ctx, rho0, ks, keys, u, iters, eps)
    sec = time.perf_counter() - t0
    target = admm_stats["objective"]
    reach = next((i for i, j in enumerate(hist) if j <= target), None)
    return {"iters": done, "iter_cap": iters, "eps_stop": eps, "stopped_before_cap": done < iters, "seconds": sec, "objective_start": hist[0], "objective": hist[-1],
            "admm_objective": target, "admm_seconds": admm_stats["seconds"], "reaches_admm_at_iter": reach}


def upwind_run(S, w, kw, rho0, ks, keys, max_admm, sl_stats):
    """The same workload with the paper's upwind exponential density operator
    (outside the step clock): seconds per ADMM iteration beside the
    semi-Lagrangian solve's."""
    import torch
    n, N = w["n"], w["num_steps"]
    kwu = dict(kw, max_admm=max_admm)
    prob = S.make_problem(n, N, w["r"], precision="mixed", density="upwind", **kwu)
    ctx = S.stfas_create(prob)
    u = torch.zeros(N * ctx.faces, dtype=torch.float32, device=rho0.device)
    S.stfas_solve(ctx, rho0, ks, keys, u)          # warm-up
    torch.cuda.synchronize()
    st = S.stfas_solve(ctx, rho0, ks, keys, u)
    ctx.destroy()
    return {"admm_cap": max_admm, "admm_iters": st["admm_iters"], "vcycles": st["vcycles"],
            "seconds": st["seconds"], "objective": st["objective"], "visual_diff": st["visual_diff"],
            "s_per_admm_iter": st["seconds"] / max(st["admm_iters"], 1),
            "sl_s_per_admm_iter": sl_stats["seconds"] / max(sl_stats["admm_iters"], 1)}


def al_run(S, w, kw, rho0, ks, keys, max_admm, al_tol):
    """The augmented-Lagrangian fallback of the ADMM loop (outside the step
    clock): the same workload and ADMM cap solved with plain ADMM and with
    the multiplier update held while the density subproblem's objective still
    falls by more than al_tol; ADMM iterations, multiplier updates, objective,
    visual difference and seconds of each (one warm-up solve first)."""
    import torch
    n, N = w["n"], w["num_steps"]
    res = {"admm_cap": max_admm, "al_tol": al_tol}
    for name, tol in (("plain", 0.0), ("fallback", al_tol)):
        prob = S.make_problem(n, N, w["r"], precision="mixed", al_tol=tol, **dict(kw, max_admm=max_admm))
        ctx = S.stfas_create(prob)
        u = torch.zeros(N * ctx.faces, dtype=torch.float32, device=rho0.device)
        S.stfas_solve(ctx, rho0, ks, keys, u)          # warm-up
        torch.cuda.synchronize()
        st = S.stfas_solve(ctx, rho0, ks, keys, u)
        ctx.destroy()
        res[name] = {"admm_iters": st["admm_iters"], "multiplier_updates": st["multiplier_updates"],
                     "vcycles": st["vcycles"], "objective": st["objective"], "visual_diff": st["visual_diff"],
                     "seconds": st["seconds"]}
    return res


def precision_3d_run(S):
    """The 3D precision form (outside the step clock): the 64^3, 60-step
    workload (sphere to ellipsoid unions at t = 30 and 60), 2 ADMM iterations
    of 4 V-cycles each (fixed counts), mixed and FP64 on the GPU; seconds,
    seconds per V-cycle, and the mixed form's keyframe error against the
    FP64 run after re-simulating both controls with the FP64 step."""
    import numpy as np
    import torch
    import synthetic
    w = synthetic.c3_precision_3d(0)
    n, N = w["n"], w["num_steps"]
    ks = sorted(w["keys"])
    res, us = {}, {}
    for prec, dt in (("mixed", torch.float32), ("fp64", torch.float64)):
        p = S.make_problem(n, N, w["r"], dt=w["dt"], precision=prec, max_admm=2, max_vcycles=4, fixed_counts=True)
        ctx = S.stfas_create(p)
        rho0 = torch.tensor(w["rho0"], dtype=dt, device="cuda")
        keys = torch.tensor(np.stack([w["keys"][k] for k in ks]), dtype=dt, device="cuda")
        u = torch.zeros(N * ctx.faces, dtype=dt, device="cuda")
        st = S.stfas_solve(ctx, rho0, ks, keys, u)
        ctx.destroy()
        us[prec] = u.double().cpu().numpy()
        res[prec] = {"seconds": st["seconds"], "vcycles": st["vcycles"],
                     "ms_per_vcycle_incl_ao": st["seconds"] * 1e3 / max(st["vcycles"], 1),
                     "objective": st["objective"]}
        torch.cuda.empty_cache()
    p64 = S.make_problem(n, N, w["r"], dt=w["dt"], precision="fp64")
    res["kf_err_mixed_vs_fp64"] = keyframe_error(S, p64, w, us["mixed"], us["fp64"])
    res["workload"] = "3D 64^3 MAC grid, 60 steps, r=1e-3, 2 ADMM x 4 V-cycles (fixed counts)"
    return res


def keyframe_error(S, p64, w, u_a, u_b):
    """max over keyframes of |rho_a - rho_b| / |rho_b| after re-simulating both
    control sequences with the FP64 step of the library."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    N = w["num_steps"]
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


def serving_run(args):
    """Continuous batching of the mixed 2D/3D request stream against a FIFO
    loop.  Each request runs 2 ADMM iterations of 4 V-cycles (fixed counts)
    so that the stream finishes within a minute; arrivals are a Poisson
    process at 0.8 x the FIFO loop's measured throughput."""
    import numpy as np
    import synthetic
    from paper_1608_01102_amd import serving
    raw = synthetic.c5_requests(args.seed, args.serve_requests, rate=1.0)
    reqs = [serving.Request(q["rid"], q["arrival"], q["n"], q["num_steps"], q["r"], q["rho0"], q["key_steps"],
                            q["key_rho"], dict(dt=q["dt"], max_admm=2, max_vcycles=4, fixed_counts=True))
            for q in raw]
    # FIFO loop, closed (back to back): service times and throughput
    seq, seq_span = serving.run_sequential(reqs, realtime=False)
    service = {r.rid: r.finished - r.admitted for r in seq}
    rate = 0.8 * len(reqs) / seq_span
    for q, r0 in zip(reqs, raw):
        q.arrival = r0["arrival"] / rate
    # FIFO latencies under these arrivals: finish_i = max(arrival_i, finish_{i-1}) + service_i
    fin = 0.0
    fifo_lat = []
    for q in sorted(reqs, key=lambda x: x.arrival):
        fin = max(q.arrival, fin) + service[q.rid]
        fifo_lat.append(fin - q.arrival)
    fifo_span = fin
    srv = serving.Server(budget_bytes=int(args.serve_budget_gb * 2 ** 30), max_slots=args.serve_slots,
                         precision="mixed")
    res, span = srv.run(reqs, realtime=True)
    summ = serving.summary(res, span)
    lat = np.array(fifo_lat)
    return {"requests": len(reqs), "arrival_rate_per_s": rate, "slots": args.serve_slots,
            "budget_gb": args.serve_budget_gb,
            "mix": {"2d": sum(len(q.n) == 2 for q in reqs), "3d": sum(len(q.n) == 3 for q in reqs)},
            "continuous": {"p50_s": summ["p50_s"], "p99_s": summ["p99_s"], "solves_per_hour": summ["solves_per_hour"],
                           "makespan_s": summ["makespan_s"]},
            "fifo": {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                     "solves_per_hour": 3600.0 * len(reqs) / fifo_span, "makespan_s": fifo_span,
                     "closed_loop_solves_per_hour": 3600.0 * len(reqs) / seq_span},
            "per_request": "2 ADMM iterations x 4 V-cycles, fixed counts, mixed precision"}


def cpu_baseline(w):
    """The FP64 oracle timed on this host: two FAS V-cycles of the velocity
    subproblem on the benchmark's own 128x128 x 40-step problem (same
    operators and levels as the GPU solve's V-cycles), with the BLAS and
    OpenMP pools held to one thread, so `cores` is what it used."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import synthetic
    from oracle import kkt, stfas
    from oracle.grid import Grid
    n, N = w["n"], w["num_steps"]
    cycles = 2
    g = Grid(n)
    dt, r = w["dt"], w["r"]
    K = r / dt ** 2
    H = stfas.Hierarchy(g, N, dt, K / r)
    rng = np.random.default_rng(0)
    tw = np.stack([synthetic.curl_noise_velocity(n, rng, 4.0, 0.5) for _ in range(N)])
    x = kkt.zeros_state(H.levels[0])
    ws = H.targets(tw)
    res = [np.zeros_like(a) for a in x]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for _ in range(cycles):
            stfas.vcycle(H, 0, x, ws, res)
        t = time.perf_counter() - t0
    return {"value": n[0] * n[1] * N * cycles / t, "unit": "spacetime cell-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{cycles} FP64 oracle V-cycles on the 128x128 x {N}-step problem ({t:.1f} s, NumPy, "
                      "one thread)",
            "host_cpus": os.cpu_count()}


if __name__ == "__main__":
    main()
