"""Parity of a converged, tolerance-driven solve (fixed_counts = 0): the
32x32 x 10 workload with the paper's upwind exponential density operator and
the default solver settings runs to the ADMM stop of Alg:outter (visual
difference below max(rho_0)/100) in a few dozen iterations, each velocity
subproblem to its relative KKT residual 1e-5.  The GPU in FP64 takes the
same stop decisions as the FP64 oracle (same ADMM iterations and V-cycles)
and returns the same controls; the oracle's run is checked to keep every
decision away from its threshold first."""
import numpy as np
import pytest

import synthetic
from gpu_common import TOL, empty, flag, rel, to_dev, to_np
from oracle import admm
from oracle.grid import Grid

pytestmark = pytest.mark.gpu

ARGS = dict(max_admm=100, density="upwind")


@pytest.fixture(scope="module")
def c1_oracle():
    w = synthetic.c1_plain_2d_32(0)
    flag("oracle: 32x32 x 10 upwind, to the ADMM stop (about a minute)")
    prob = admm.Problem(n=w["n"], num_steps=w["num_steps"], r=w["r"], dt=w["dt"], **ARGS)
    ref = admm.solve(prob, w["rho0"], w["keys"])
    return w, ref, prob.resolved(w["rho0"])


def _gpu_solve(w, prec):
    from paper_1608_01102_amd import stfas as S
    g = Grid(w["n"])
    N = w["num_steps"]
    prob = S.make_problem(w["n"], N, w["r"], dt=w["dt"], precision=prec, **ARGS)
    ctx = S.stfas_create(prob)
    ks = sorted(w["keys"])
    u = empty(N * g.nface, prec)
    flag(f"solve 32x32 x 10 upwind {prec} to the ADMM stop")
    st = S.stfas_solve(ctx, to_dev(w["rho0"], prec), ks, to_dev(np.stack([w["keys"][k] for k in ks]), prec), u)
    ctx.destroy()
    return st, to_np(u).reshape(N, -1)


@pytest.mark.timeout(900)
def test_converged_solve_fp64(c1_oracle):
    w, ref, p = c1_oracle
    assert ref.converged and ref.admm_iters < ARGS["max_admm"]
    h = ref.history
    # every stop decision of the oracle's run is clear of its threshold (FP64 rounding cannot flip it)
    for d in h["visual_diff"]:
        assert abs(d - p.eps_admm) > 1e-3 * p.eps_admm, d
    for res, f0 in zip(h["nso_res"], h["nso_f0"]):
        for x in res:
            assert abs(x - p.eps_stfas * f0) > 1e-3 * p.eps_stfas * f0
    st, u = _gpu_solve(w, "fp64")
    print(f"32x32x10 upwind fp64: {st['admm_iters']} ADMM iterations ({ref.admm_iters} oracle), "
          f"{st['vcycles']} V-cycles ({ref.vcycles}), |u - u_oracle|/|u_oracle| = {rel(u, ref.u):.2e}")
    assert st["converged"] == 1
    assert st["admm_iters"] == ref.admm_iters and st["vcycles"] == ref.vcycles
    assert rel(u, ref.u) <= TOL["fp64"]
    assert abs(st["objective"] - ref.objective) <= TOL["fp64"] * ref.objective
