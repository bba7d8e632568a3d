"""Operator parity at the full 3D size in the launch configuration the
per-operator roofline times: the 64^3 grid, each operator batched over all
60 time slices in one launch.  The oracle recomputes three sampled slices
(first, middle, last) of every batched result; the other slices are checked
by a property that holds at any size (the batch slices are independent, so
equal inputs give bit-identical outputs)."""
import numpy as np
import pytest

import synthetic
from gpu_common import TOL, empty, flag, rel, to_dev, to_np
from oracle import advect, poisson, upwind
from oracle.grid import Grid

pytestmark = pytest.mark.gpu

N3 = (64, 64, 64)
SLICES = 60
SAMPLE = (0, 29, 59)


def _q(x, prec):
    return np.asarray(x, dtype=np.float32).astype(np.float64) if prec == "mixed" else np.asarray(x)


@pytest.fixture(scope="module")
def fields():
    g = Grid(N3)
    rng = np.random.default_rng(71)
    # three distinct velocity / density fields, laid out over the 60 slices in turn
    v = [synthetic.curl_noise_velocity(N3, rng, 4.0, 2.0, 1.0) for _ in range(3)]
    rho = [synthetic.smooth_noise_density(N3, rng, 2.0) for _ in range(3)]
    mu = [rng.standard_normal(g.ncell) for _ in range(3)]
    y = [synthetic.random_faces(N3, rng) for _ in range(3)]
    return g, v, rho, mu, y


def _batch(parts, prec):
    """[SLICES][n] with slice s = parts[s % 3]."""
    return np.stack([_q(parts[s % 3], prec) for s in range(SLICES)])


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_batched_operators_64cubed_60_slices(fields, prec):
    import torch
    from paper_1608_01102_amd import stfas as S
    g, v, rho, mu, y = fields
    dt = g.h
    prob = S.make_problem(N3, SLICES, 1e-3, dt=dt, precision=prec)
    ctx = S.stfas_create(prob)
    C, F = g.ncell, g.nface
    vb, rb, mb, yb = (to_dev(_batch(a, prec), prec) for a in (v, rho, mu, y))
    tol = TOL[prec]

    def check(out, per_slice, what):
        o = to_np(out).reshape(SLICES, -1)
        for s in SAMPLE:
            k = s % 3
            assert rel(o[s], per_slice(k)) <= tol, (what, s)
        for s in range(3, SLICES):       # equal inputs, equal outputs, bit for bit
            assert np.array_equal(o[s], o[s % 3]), (what, s)

    vq = [_q(a, prec) for a in v]
    rq = [_q(a, prec) for a in rho]
    mq = [_q(a, prec) for a in mu]
    yq = [_q(a, prec) for a in y]
    flag(f"fullsize advect {prec}")
    out_c = empty(SLICES * C, prec)
    S.stfas_op_advect(ctx, SLICES, rb, vb, out_c)
    check(out_c, lambda k: advect.advect_scalar(g, rq[k], vq[k], dt), "advect")
    flag(f"fullsize advect_dv_T {prec}")
    out_f = empty(SLICES * F, prec)
    S.stfas_op_advect_dv_T(ctx, SLICES, mb, rb, vb, None, 1.0, out_f)
    check(out_f, lambda k: advect.advect_scalar_dv_T(g, mq[k], rq[k], vq[k], dt), "advect_dv_T")
    flag(f"fullsize self_advect {prec}")
    S.stfas_op_self_advect(ctx, 0, SLICES, vb, yb, out_f)
    check(out_f, lambda k: advect.self_advect(g, vq[k], dt) + dt * yq[k] * g.interior_mask(), "self_advect")
    flag(f"fullsize advect_T {prec}")
    # the transposes scatter with atomics (summation order not fixed): sampled slices only
    S.stfas_op_advect_T(ctx, SLICES, mb, vb, None, out_c)
    o = to_np(out_c).reshape(SLICES, -1)
    for s in SAMPLE:
        assert rel(o[s], advect.advect_scalar_T(g, mq[s % 3], vq[s % 3], dt)) <= tol, ("advect_T", s)
    flag(f"fullsize self_advect_T {prec}")
    out_f.zero_()                        # the operator accumulates into out
    S.stfas_op_self_advect_T(ctx, 0, SLICES, vb, yb, 1.0, out_f)
    o = to_np(out_f).reshape(SLICES, -1)
    for s in SAMPLE:
        assert rel(o[s], advect.self_advect_T(g, vq[s % 3], yq[s % 3], dt)) <= tol, ("self_advect_T", s)
    flag(f"fullsize project {prec}")
    wb = to_dev(_batch([a * 3.0 for a in y], prec), prec)
    S.stfas_op_project(ctx, SLICES, wb, out_f)
    o = to_np(out_f).reshape(SLICES, -1)
    # the projection is iterative: the oracle's exact projection of one slice,
    # within the multigrid tolerance of the precision
    ref, _ = poisson.project(g, _q(y[0] * 3.0, prec), rtol=1e-12)
    assert rel(o[0], ref) <= (1e-9 if prec == "fp64" else 1e-5)
    ctx.destroy()
    torch.cuda.empty_cache()


def test_upwind_64cubed():
    """The upwind exponential operator on one full-size 3D field."""
    from paper_1608_01102_amd import stfas as S
    g = Grid(N3)
    rng = np.random.default_rng(72)
    rho = synthetic.smooth_noise_density(N3, rng, 2.0)
    v = synthetic.curl_noise_velocity(N3, rng, 4.0, 1.5, 1.0)
    prob = S.make_problem(N3, 1, 1e-3, dt=g.h, precision="fp64", density="upwind")
    ctx = S.stfas_create(prob)
    out = empty(g.ncell, "fp64")
    flag("fullsize upwind")
    k = S.stfas_op_upwind(ctx, to_dev(rho, "fp64"), to_dev(v, "fp64"), out)
    assert k == upwind.advect_up_k(g, rho, v, g.h)
    assert rel(to_np(out), upwind.advect_up(g, rho, v, g.h)) <= 1e-10
    ctx.destroy()
