"""Profiling helpers: summaries of rocprofv3 output and the counter workload.

  python -m paper_1608_01102_amd.profiling stats RESULTS.db [KERNEL GRID_X]
      per-kernel calls / total / average from a rocprofv3 --kernel-trace
      --stats SQLite output, and the average of one kernel's launches with
      a given grid size.
  python -m paper_1608_01102_amd.profiling workload
      the program run under rocprofv3 --pmc: a plain device copy of known
      size, then SCGS sweeps on the finest level of the 128x128, 40-step
      mixed-precision problem (the launches the benchmark's roofline covers).
  python -m paper_1608_01102_amd.profiling pmc DIR COUNTER KERNEL GRID_X
      mean counter value per dispatch (KiB) of KERNEL at GRID_X and of the
      copy kernel, from a rocprofv3 --pmc CSV directory.
  python -m paper_1608_01102_amd.profiling ops
      the per-operator workload: the calibration copy, then every operator
      of the path once per repetition on the 64^3 grid, batched over the 60
      time slices of the 3D precision workload (mixed precision).
  python -m paper_1608_01102_amd.profiling opstable RESULTS.db [FETCH_DIR WRITE_DIR]
      achieved GB/s of each operator kernel of that workload: algorithmic
      bytes per launch / average launch time, and, with the two counter
      directories, the measured HBM bytes per launch.
"""
import csv
import glob
import hashlib
import os
import sqlite3
import sys

COPY_BYTES = 256 << 20          # the calibration copy moves this many bytes each way
HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash():
    """Hash of the kernel sources (a counter summary is valid only for these)."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stats(db, kernel=None, grid_x=None):
    con = sqlite3.connect(db)
    cur = con.cursor()
    rows = cur.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    lines = [f"{'kernel':60s} {'calls':>8s} {'total_ms':>10s} {'avg_us':>9s} {'pct':>6s}"]
    for name, calls, tot, avg, pct in rows[:20]:
        short = name.split("(")[0].replace("void ", "")
        lines.append(f"{short[:60]:60s} {calls:8d} {tot / 1e3:10.2f} {avg:9.2f} {pct:6.2f}")
    if kernel:
        r = cur.execute("select count(*), avg(duration), min(duration), max(duration) from kernels "
                        "where name like ? and grid_x = ?", (f"%{kernel}%", int(grid_x))).fetchone()
        lines.append(f"\n{kernel} launches with grid_x={grid_x}: count={r[0]} avg_us={r[1] / 1e3:.2f} "
                     f"min_us={r[2] / 1e3:.2f} max_us={r[3] / 1e3:.2f}")
    return "\n".join(lines)


def calibration_copy():
    """Four plain device copies of COPY_BYTES each (the reference the counter
    readings are scaled by)."""
    import torch
    dev = torch.device("cuda:0")
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()


def workload(reps=20):
    import numpy as np
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    import synthetic
    from paper_1608_01102_amd import stfas as S
    dev = torch.device("cuda:0")
    calibration_copy()
    w = synthetic.c2_plain_2d_128(0)
    n, N = w["n"], w["num_steps"]
    prob = S.make_problem(n, N, w["r"], dt=w["dt"], precision="mixed")
    ctx = S.stfas_create(prob)
    rng = np.random.default_rng(0)
    F, C = ctx.faces, ctx.cells
    x = tuple(torch.tensor(a, dtype=torch.float32, device=dev) for a in (
        np.stack([synthetic.curl_noise_velocity(n, rng, 4.0, 0.5, 1.0) for _ in range(N)]),
        rng.standard_normal((N, C)) * 1e-3,
        np.stack([synthetic.random_faces(n, rng, 0.1) for _ in range(N)]),
        rng.standard_normal((N, C)) * 1e-3))
    tgt = torch.tensor(np.stack([synthetic.curl_noise_velocity(n, rng, 4.0, 0.5, 1.0) for _ in range(N)]),
                       dtype=torch.float32, device=dev)
    for _ in range(reps):
        S.stfas_op_scgs_sweep(ctx, 0, x, tgt)
    torch.cuda.synchronize()
    ctx.destroy()
    print("workload done", flush=True)


def pmc(directory, counter, kernel, grid_x, min_frac=0.0):
    """Mean counter reading per dispatch of `kernel` with this grid size,
    scaled by the calibration copy's reading.  min_frac > 0 drops dispatches
    reading below that fraction of the largest (launches that return at once,
    such as the upwind series terms past the series' stop)."""
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    vals, copy = [], []
    for f in files:
        with open(f) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                name = row.get("Kernel_Name", "")
                v = float(row["Counter_Value"])
                if kernel in name and int(row.get("Grid_Size", row.get("Grid_Size_X", "0"))) == int(grid_x):
                    vals.append(v)
                elif "copy" in name.lower() and v > 0.25 * COPY_BYTES / 1024.0:
                    copy.append(v)      # the calibration copy (smaller copies are ignored)
    dropped = 0
    if vals and float(min_frac) > 0:
        keep = [v for v in vals if v >= float(min_frac) * max(vals)]
        dropped, vals = len(vals) - len(keep), keep
    out = {"counter": counter, "kernel": kernel, "grid_x": int(grid_x), "dispatches": len(vals),
           "dropped_below_min_frac": dropped,
           "mean_kib": sum(vals) / len(vals) if vals else None,
           "copy_dispatches": len(copy), "copy_mean_kib": sum(copy) / len(copy) if copy else None,
           "copy_expected_kib": COPY_BYTES / 1024.0}
    if vals and copy:
        scale = out["copy_expected_kib"] / out["copy_mean_kib"]
        out["scale"] = scale
        out["bytes_per_dispatch"] = out["mean_kib"] * 1024.0 * scale
    return out


# ---------------------------------------------------------------- per-operator roofline
OPS_N = (64, 64, 64)
OPS_SLICES = 60


def ops_workload(reps=5):
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    import synthetic
    from paper_1608_01102_amd import stfas as S
    dev = torch.device("cuda:0")
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(4):
        b.copy_(a)
    del a, b
    n, N = OPS_N, OPS_SLICES
    prob = S.make_problem(n, N, 1e-3, precision="mixed")
    ctx = S.stfas_create(prob)
    C, F = ctx.cells, ctx.faces
    import numpy as np
    rng = np.random.default_rng(0)
    v1 = torch.tensor(synthetic.curl_noise_velocity(n, rng, 4.0, 2.0, 1.0), dtype=torch.float32, device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(0)
    v = v1.repeat(N)
    rho = torch.rand(N * C, generator=g, device=dev)
    mu = torch.randn(N * C, generator=g, device=dev)
    y = torch.randn(N * F, generator=g, device=dev) * (v != 0)
    out_c = torch.empty(N * C, device=dev)
    out_f = torch.empty(N * F, device=dev)
    st = tuple(torch.randn(N * m, generator=g, device=dev) * 1e-3 for m in (F, C, F, C))
    res = tuple(torch.zeros(N * m, device=dev) for m in (F, C, F, C))
    rout = tuple(torch.empty(N * m, device=dev) for m in (F, C, F, C))
    w = v.clone()
    lc, lf = ctx.level_counts(1)
    coarse = tuple(torch.empty(N * m, device=dev) for m in (lf, lc, lf, lc))
    for _ in range(reps):
        S.stfas_op_advect(ctx, N, rho, v, out_c)
        S.stfas_op_advect_T(ctx, N, mu, v, None, out_c)
        S.stfas_op_advect_dv_T(ctx, N, mu, rho, v, None, 1.0, out_f)
        S.stfas_op_self_advect(ctx, 0, N, v, y, out_f)
        S.stfas_op_self_advect_T(ctx, 0, N, v, y, 1.0, out_f)
        S.stfas_op_project(ctx, N, y, out_f)
        S.stfas_op_metric(ctx, rho[:C], out_c[:C])
        S.stfas_op_kkt_residual(ctx, 0, st, w, res, rout)
        S.stfas_op_scgs_sweep(ctx, 0, st, w)
        S.stfas_op_restrict(ctx, 0, st, coarse)
        S.stfas_op_prolong(ctx, 0, coarse, 1.0, st)
    torch.cuda.synchronize()
    ctx.destroy()
    # the upwind exponential density operator on one field of the same grid
    # (its series is launched term by term; the table needs its k)
    pu = S.make_problem(n, 1, 1e-3, precision="mixed", density="upwind")
    cu = S.stfas_create(pu)
    ks = [S.stfas_op_upwind(cu, rho[:C], v1, out_c[:C]) for _ in range(reps)]
    torch.cuda.synchronize()
    cu.destroy()
    print(f"upwind series k = {ks[0]} (all calls: {ks})", flush=True)
    print("ops workload done", flush=True)


def _ceil256(x):
    return -(-x // 256) * 256


def ops_expectations():
    """(label, kernel name part, grid x, grid y, algorithmic bytes per launch,
    what they are) of the operator kernels of the ops workload, FP32."""
    n0, n1, n2 = OPS_N
    N = OPS_SLICES
    C = n0 * n1 * n2
    F = (n0 + 1) * n1 * n2 + n0 * (n1 + 1) * n2 + n0 * n1 * (n2 + 1)
    half = (n0 + 1) // 2 * n1 * n2
    return [
        ("SL density advection", "k_advect<", _ceil256(C), N, N * C * 20, "rho, 3 face velocities, rho' per cell"),
        ("its rho adjoint", "k_advect_T_tiled<", ((n0 + 7) // 8) * ((n1 + 7) // 8) * ((n2 + 3) // 4) * 256, N,
         N * C * 24, "mu, 3 face velocities, out read+write"),
        ("its v adjoint", "k_advect_dv_T<", _ceil256(F), N, N * F * 16, "mu, rho, v, out per face"),
        ("SL self-advection", "k_self_advect<", _ceil256(F), N, N * F * 12, "v, u, out per face"),
        ("its adjoint (tiled)", "k_self_advect_T_tiled<", None, N, N * F * 16, "v, y, out read+write per face"),
        ("divergence", "k_divergence<", _ceil256(C), N, N * C * 16, "3 faces, b per cell"),
        ("red-black GS, one colour, finest", "k_rbgs<", _ceil256(half), N, N * C * 6,
         "phi of the other colour, b and phi of this one"),
        ("projection apply", "k_project_apply<", _ceil256(F), N, N * (F * 12 + C * 4), "w, v per face; phi"),
        ("Gaussian, one axis", "k_blur_axis<", _ceil256(C), 1, C * 8, "in, out per cell"),
    ] + _stfas_expectations(n0, n1, n2, N, C, F)


def _stfas_expectations(n0, n1, n2, N, C, F):
    """The velocity-subproblem kernels of the ops workload (level 0 and the
    transfers to level 1): the KKT residual, one colour pass's residual, the
    SCGS colour pass and the four FAS transfers."""
    nb = lambda x: -(-x // 256)
    # colour 0 of the SCGS sweep (every colour of an even grid has the same counts)
    cnt = [(m + 1) // 2 for m in (n0, n1, n2)]
    cc = cnt[0] * cnt[1] * cnt[2]
    fc = sum((m + 1) * (cnt[0] * cnt[1] * cnt[2] // cnt[a]) for a, m in enumerate((n0, n1, n2)))
    inner = 3 * (2 * cnt[0] - 1) * cnt[1] * cnt[2]          # interior faces of colour 0's cells
    Cc = (n0 // 2) * (n1 // 2) * (n2 // 2)
    Fc = 3 * (n0 // 2) * (n0 // 2) * (n0 // 2 + 1)
    full = (nb(F) + nb(C)) * N * 256
    tiles = (-(-(n0 + 1) // 8)) * (-(-n1 // 8)) * (-(-n2 // 4))
    rows = (nb(fc) + nb(cc)) * N * 256
    transpose = (tiles * (N - 1) * 3 + min(nb(N * F), 2048)) * 256
    return [
        ("KKT residual rows (whole level)", "k_kkt_split<", full, 1, N * C * 108,
         "the method's bytes: v, u, w, res in and r out per face (3 per cell), p-bar, p in per cell"),
        ("colour-pass rows (one colour)", "k_kkt_split<", rows, 1, N * cc * 108,
         "the method's bytes of the colour's cells (108 B per spacetime cell)"),
        ("sweep transpose J_S^T u (once per sweep)", "k_kkt_split<", transpose, 1, (N - 1) * C * 36,
         "the method's bytes: v, y in, J_S^T y out, 3 faces per cell"),
        ("SCGS colour pass", "k_scgs_colour_rows<", None, 1, 4 * 2 * N * (inner * 3.5 + cc * 3),
         "r1, t1, r3 read and u/v read+written per face block pair; 3 per cell block"),
        ("FAS restriction, faces", "k_restrict_faces<", _ceil256(Fc), N, N * (F + Fc) * 4, "fine in, coarse out"),
        ("FAS restriction, cells", "k_restrict_cells<", _ceil256(Cc), N, N * (C + Cc) * 4, "fine in, coarse out"),
        ("FAS prolongation, faces", "k_prolong_faces<", _ceil256(F), N, N * (2 * F + Fc) * 4,
         "fine read+written, coarse in"),
        ("FAS prolongation, cells", "k_prolong_cells<", _ceil256(C), N, N * (2 * C + Cc) * 4,
         "fine read+written, coarse in"),
    ]


def upwind_term_row(rows, k, C, F):
    """Table row of the upwind series' working terms: the k_up_term
    launches of each series in launch order (terms 0 .. UP_KMAX), of which
    terms 1..k compute a term (0 copies rho into the sum, terms after k
    return at once).  Algorithmic bytes per term: prev, next and the sum's
    read and write per cell, the velocity once per face."""
    per = 49                                  # terms 0..48 launched per call of the operator
    ds = [r[4] for r in rows if "k_up_term<" in r[0]]
    if not ds or len(ds) % per:
        return None
    work = [d for s0 in range(0, len(ds), per) for d in ds[s0 + 1:s0 + 1 + k]]
    avg = sum(work) / len(work)
    nbytes = C * 16 + F * 4
    gbs = nbytes / avg
    return (f"| upwind exponential, one term (k = {k}) | `k_up_term` | {len(work)} | {avg / 1e3:.1f} | "
            f"{nbytes / 1e6:.1f} | {gbs:.0f} | {100 * gbs / 8000:.0f}% |")


def ops_table(db, fetch_dir=None, write_dir=None, upwind_k=None):
    con = sqlite3.connect(db)
    rows = con.execute("select name, grid_x, grid_y, grid_z, duration from kernels order by start").fetchall()
    lines = ["| Operator | Kernel | Launches | Avg µs | Alg. MB/launch | Alg. GB/s | % of 8000 |"
             + (" HBM MB/launch | HBM GB/s |" if fetch_dir else ""),
             "|---|---|---|---|---|---|---|" + ("---|---|" if fetch_dir else "")]
    for label, part, gx, gy, nbytes, what in ops_expectations():
        ds = [r[4] for r in rows if part in r[0] and (gx is None or int(r[1]) == gx) and int(r[2]) == gy]
        if not ds:
            lines.append(f"| {label} | `{part[:-1]}` | 0 | | | | |")
            continue
        avg = sum(ds) / len(ds)       # ns
        gbs = nbytes / avg
        line = (f"| {label} | `{part[:-1]}` | {len(ds)} | {avg / 1e3:.1f} | {nbytes / 1e6:.1f} | {gbs:.0f} | "
                f"{100 * gbs / 8000:.0f}% |")
        if fetch_dir:
            gsz = None
            m = [r for r in rows if part in r[0] and (gx is None or int(r[1]) == gx) and int(r[2]) == gy]
            gsz = int(m[0][1]) * int(m[0][2]) * int(m[0][3])
            fb = pmc(fetch_dir, "FETCH_SIZE", part, gsz).get("bytes_per_dispatch")
            wb = pmc(write_dir, "WRITE_SIZE", part, gsz).get("bytes_per_dispatch")
            if fb is not None and wb is not None:
                line += f" {(fb + wb) / 1e6:.1f} | {(fb + wb) / avg:.0f} |"
            else:
                line += " | |"
        lines.append(line)
    if upwind_k is not None:
        n0, n1, n2 = OPS_N
        C = n0 * n1 * n2
        F = (n0 + 1) * n1 * n2 + n0 * (n1 + 1) * n2 + n0 * n1 * (n2 + 1)
        row = upwind_term_row(rows, int(upwind_k), C, F)
        if row:
            lines.append(row + (" | |" if fetch_dir else ""))
    return "\n".join(lines)


def sq_valu(directory, kernel, grid_x, simds=1024, clock_hz=2.4e9):
    """Mean SQ_ACTIVE_INST_VALU per dispatch of KERNEL at GRID_X and the
    VALU-busy time it stands for (4 cycles per wavefront instruction over all
    SIMDs), from a rocprofv3 --pmc CSV directory."""
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    vals = []
    for f in files:
        with open(f) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") == "SQ_ACTIVE_INST_VALU" and kernel in row.get("Kernel_Name", "") and \
                        int(row.get("Grid_Size", row.get("Grid_Size_X", "0"))) == int(grid_x):
                    vals.append(float(row["Counter_Value"]))
    if not vals:
        return {"dispatches": 0}
    mean = sum(vals) / len(vals)
    return {"dispatches": len(vals), "sq_active_inst_valu": mean, "valu_busy_us": mean * 4 / simds / clock_hz * 1e6}


def main(argv):
    if argv[0] == "stats":
        print(stats(argv[1], *(argv[2:4] if len(argv) >= 4 else [])))
    elif argv[0] == "workload":
        workload()
    elif argv[0] == "pmc":
        import json
        print(json.dumps(pmc(*argv[1:6])))
    elif argv[0] == "ops":
        ops_workload()
    elif argv[0] == "opstable":
        print(ops_table(*argv[1:5]))
    elif argv[0] == "valu":
        import json
        print(json.dumps(sq_valu(argv[1], argv[2], argv[3])))
    elif argv[0] == "hash":
        print(kernel_source_hash())


if __name__ == "__main__":
    main(sys.argv[1:])
