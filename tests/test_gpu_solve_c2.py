"""Full-solve parity on the 128x128 x 40-step stroke workload (the shape the
benchmark times): one ADMM iteration of two V-cycles, FP64 and mixed, against
the FP64 oracle run once on the same inputs."""
import numpy as np
import pytest

import synthetic
from gpu_common import TOL, empty, flag, rel, to_dev, to_np
from oracle import admm
from oracle.grid import Grid

pytestmark = pytest.mark.gpu

ARGS = dict(max_admm=1, max_vcycles=2, fixed_counts=True)


@pytest.fixture(scope="module")
def c2_oracle():
    w = synthetic.c2_plain_2d_128(0)
    flag("oracle: 128x128 x 40, 1 ADMM x 2 V-cycles (about two minutes)")
    ref = admm.solve(admm.Problem(n=w["n"], num_steps=w["num_steps"], r=w["r"], dt=w["dt"], **ARGS), w["rho0"],
                     w["keys"])
    return w, ref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_c2_shape(c2_oracle, prec):
    from paper_1608_01102_amd import stfas as S
    w, ref = c2_oracle
    g = Grid(w["n"])
    N = w["num_steps"]
    prob = S.make_problem(w["n"], N, w["r"], dt=w["dt"], precision=prec, **ARGS)
    ctx = S.stfas_create(prob)
    ks = sorted(w["keys"])
    u = empty(N * g.nface, prec)
    flag(f"solve 128x128 x 40 {prec}, 1 ADMM x 2 V-cycles")
    st = S.stfas_solve(ctx, to_dev(w["rho0"], prec), ks, to_dev(np.stack([w["keys"][k] for k in ks]), prec), u)
    ctx.destroy()
    ug = to_np(u).reshape(N, -1)
    e_u = rel(ug, ref.u)
    e_j = abs(st["objective"] - ref.objective) / ref.objective
    print(f"128x128x40 {prec}: |u - u_oracle|/|u_oracle| = {e_u:.2e}, objective {e_j:.2e}")
    assert st["admm_iters"] == ref.admm_iters == 1 and st["vcycles"] == ref.vcycles == 2
    assert e_u <= TOL[prec]
    assert e_j <= TOL[prec]
