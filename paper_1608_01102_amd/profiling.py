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


def workload(reps=20):
    import numpy as np
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    import synthetic
    from paper_1608_01102_amd import stfas as S
    dev = torch.device("cuda:0")
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()
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


def pmc(directory, counter, kernel, grid_x):
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
    out = {"counter": counter, "kernel": kernel, "grid_x": int(grid_x), "dispatches": len(vals),
           "mean_kib": sum(vals) / len(vals) if vals else None,
           "copy_dispatches": len(copy), "copy_mean_kib": sum(copy) / len(copy) if copy else None,
           "copy_expected_kib": COPY_BYTES / 1024.0}
    if vals and copy:
        scale = out["copy_expected_kib"] / out["copy_mean_kib"]
        out["scale"] = scale
        out["bytes_per_dispatch"] = out["mean_kib"] * 1024.0 * scale
    return out


def main(argv):
    if argv[0] == "stats":
        print(stats(argv[1], *(argv[2:4] if len(argv) >= 4 else [])))
    elif argv[0] == "workload":
        workload()
    elif argv[0] == "pmc":
        import json
        print(json.dumps(pmc(argv[1], argv[2], argv[3], argv[4])))
    elif argv[0] == "hash":
        print(kernel_source_hash())


if __name__ == "__main__":
    main(sys.argv[1:])
