"""Writes oracle_tiny_solves.json: a regression record of the oracle's ADMM
solve (Alg:outter with the STFAS velocity subproblem, Sec. 4) on tiny seeded
problems, for each density operator (SL, and the upwind exponential of
eq:Adv) and velocity operator (SL, and the rotational form of eq:NSA), in
2D and 3D.  It calls only the oracle and the seeded input generators.

This is not an independent pin (the paper prints no worked example of a
solve): it records what the oracle computes so that any change to its
arithmetic shows up as a failing test and has to be regenerated here,
in a commit that names the passage justifying the change.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synthetic  # noqa: E402
from oracle import admm  # noqa: E402

OUT = os.path.join(HERE, "oracle_tiny_solves.json")

# name: (grid, steps, seed, Problem options)
CASES = {
    "sl_2d_fixed": ((8, 8), 3, 0, dict(max_admm=2, max_vcycles=3, fixed_counts=True)),
    "upwind_2d_fixed": ((8, 8), 3, 1, dict(max_admm=2, max_vcycles=3, fixed_counts=True, density="upwind")),
    "rotational_2d_fixed": ((8, 8), 3, 2, dict(max_admm=2, max_vcycles=3, fixed_counts=True,
                                               velocity="vorticity")),
    "sl_3d_fixed": ((4, 4, 4), 2, 3, dict(max_admm=2, max_vcycles=2, fixed_counts=True)),
    "sl_2d_stopped": ((8, 8), 3, 4, dict(max_admm=6, max_vcycles=8)),
}
SAMPLE = 7   # every SAMPLE-th control entry is stored


def run(name):
    n, N, seed, opts = CASES[name]
    w = synthetic.small_problem(n, N, seed=seed, r=1e-2)
    res = admm.solve(admm.Problem(n=w["n"], num_steps=N, r=w["r"], dt=w["dt"], **opts), w["rho0"], w["keys"])
    u = np.asarray(res.u).ravel()
    return {"objective": float(res.objective), "objective_l2": float(res.objective_l2),
            "reg_term": float(res.reg_term), "admm_iters": int(res.admm_iters), "vcycles": int(res.vcycles),
            "u_norm": float(np.linalg.norm(u)), "u_sample": [float(x) for x in u[::SAMPLE]]}


def main():
    rec = {"about": "regression record of the oracle's solve; written by tests/golden/make_golden.py",
           "sample_stride": SAMPLE, "cases": {k: run(k) for k in CASES}}
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
