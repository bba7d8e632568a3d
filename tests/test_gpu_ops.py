"""Operator-level parity of the HIP library with the FP64 oracle, through the
C interface.  Bar: relative L2 error <= 1e-10 (FP64) / 1e-4 (mixed)."""
import numpy as np
import pytest

import synthetic
from gpu_common import TOL, empty, flag, rel, to_dev, to_np, zeros
from oracle import advect, kkt, metric, poisson, scgs, transfer
from oracle.grid import Grid

pytestmark = pytest.mark.gpu

CASES = [((16, 12), 4), ((8, 8, 8), 3), ((20, 12), 5), ((16, 16), 3), ((12, 8, 16), 2)]
PRECS = ["fp64", "mixed"]


def _ctx(n, N, prec, dt=None, K=None, r=1e-2, **kw):
    from paper_1608_01102_amd import stfas as S
    g = Grid(n)
    dt = 0.7 * g.h if dt is None else dt
    K = 3.0 * r / dt ** 2 if K is None else K
    kw.setdefault("scgs_omega", 1.0)
    kw.setdefault("scgs_lm", -1.0)          # the oracle Level's default: no perturbation
    prob = S.make_problem(n, N, r, dt=dt, K=K, precision=prec, **kw)
    return S, S.stfas_create(prob), g, dt, K


def _q(x, prec):
    """Round inputs to the device precision so both sides see the same data."""
    return np.asarray(x, dtype=np.float32).astype(np.float64) if prec == "mixed" else np.asarray(x)


def _faces(g, rng, B, s=1.0):
    return np.stack([synthetic.random_faces(g.n, rng, s) for _ in range(B)])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,N", CASES)
def test_advect_and_transposes(n, N, prec):
    S, ctx, g, dt, K = _ctx(n, N, prec)
    rng = np.random.default_rng(11)
    B = N
    rho = _q(rng.standard_normal((B, g.ncell)), prec)
    v = _q(_faces(g, rng, B, 2.0), prec)
    mu = _q(rng.standard_normal((B, g.ncell)), prec)
    vt = _q(_faces(g, rng, B), prec)
    flag(f"advect n={n} N={N} {prec}")
    out = empty(B * g.ncell, prec)
    S.stfas_op_advect(ctx, B, to_dev(rho, prec), to_dev(v, prec), out)
    ref = advect.advect_scalar(g, rho, v, dt)
    assert rel(to_np(out), ref) <= TOL[prec]
    add = _q(rng.standard_normal((B, g.ncell)), prec)
    S.stfas_op_advect_T(ctx, B, to_dev(mu, prec), to_dev(v, prec), to_dev(add, prec), out)
    ref = advect.advect_scalar_T(g, mu, v, dt) + add
    assert rel(to_np(out), ref) <= TOL[prec]
    gv = empty(B * g.nface, prec)
    S.stfas_op_advect_dv_T(ctx, B, to_dev(mu, prec), to_dev(rho, prec), to_dev(v, prec), to_dev(vt, prec), 0.3, gv)
    ref = vt * g.interior_mask() + 0.3 * advect.advect_scalar_dv_T(g, mu, rho, v, dt)
    assert rel(to_np(gv), ref) <= TOL[prec]
    ctx.destroy()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,N", CASES)
def test_self_advect_and_transpose(n, N, prec):
    S, ctx, g, dt, K = _ctx(n, N, prec)
    rng = np.random.default_rng(12)
    B = N
    for level in range(ctx.num_levels()):
        gl = Grid(tuple(x >> level for x in n), g.h * 2 ** level)
        v = _q(_faces(gl, rng, B, 1.5), prec)
        u = _q(_faces(gl, rng, B), prec)
        y = _q(_faces(gl, rng, B), prec)
        flag(f"self_advect n={n} level={level} {prec}")
        out = empty(B * gl.nface, prec)
        S.stfas_op_self_advect(ctx, level, B, to_dev(v, prec), to_dev(u, prec), out)
        ref = advect.self_advect(gl, v, dt) + dt * u * gl.interior_mask()
        assert rel(to_np(out), ref) <= TOL[prec]
        base = _q(_faces(gl, rng, B), prec)
        acc = to_dev(base, prec)
        S.stfas_op_self_advect_T(ctx, level, B, to_dev(v, prec), to_dev(y, prec), -2.5, acc)
        ref = base - 2.5 * advect.self_advect_T(gl, v, y, dt)
        assert rel(to_np(acc), ref) <= TOL[prec]
    ctx.destroy()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,B", [((96, 80), 20), ((40, 32, 24), 3), ((33, 17), 300)])
def test_self_advect_T_tiled_sizes(n, B, prec):
    """The tiled transpose (LDS window, merged corners, foot-point slots) at
    sizes above the untiled threshold, with ragged tiles at the lattice
    edges, and velocities up to 3 cells per step (backtraces past the halo
    take the global-atomic path)."""
    S, ctx, g, dt, K = _ctx(n, 2, prec, dt=1.0 / n[0])
    rng = np.random.default_rng(24)
    v = _q(np.stack([synthetic.curl_noise_velocity(n, rng, 2.0, 3.0, dt / g.h) for _ in range(B)]), prec)
    y = _q(_faces(g, rng, B), prec)
    base = _q(_faces(g, rng, B), prec)
    acc = to_dev(base, prec)
    flag(f"self_advect_T tiled n={n} B={B} {prec}")
    S.stfas_op_self_advect_T(ctx, 0, B, to_dev(v, prec), to_dev(y, prec), 0.75, acc)
    ref = base + 0.75 * advect.self_advect_T(g, v, y, dt)
    assert rel(to_np(acc), ref) <= TOL[prec]
    ctx.destroy()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,B", [((96, 80), 20), ((40, 32, 24), 6), ((33, 17), 300)])
def test_advect_T_tiled_sizes(n, B, prec):
    """The tiled density adjoint (LDS window in fixed point, one flush per
    node) at launch sizes above its threshold, with ragged tiles at the grid
    edges and backtraces of up to 3 cells (beyond the halo: the global-atomic
    path)."""
    S, ctx, g, dt, K = _ctx(n, 2, prec, dt=1.0 / n[0])
    rng = np.random.default_rng(25)
    assert g.ncell * B >= 131072
    v = _q(np.stack([synthetic.curl_noise_velocity(n, rng, 2.0, 3.0, dt / g.h) for _ in range(B)]), prec)
    mu = _q(rng.standard_normal((B, g.ncell)), prec)
    add = _q(rng.standard_normal((B, g.ncell)), prec)
    out = empty(B * g.ncell, prec)
    flag(f"advect_T tiled n={n} B={B} {prec}")
    S.stfas_op_advect_T(ctx, B, to_dev(mu, prec), to_dev(v, prec), to_dev(add, prec), out)
    ref = advect.advect_scalar_T(g, mu, v, dt) + add
    assert rel(to_np(out), ref) <= TOL[prec]
    ctx.destroy()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,N", CASES)
def test_projection_batched(n, N, prec):
    S, ctx, g, dt, K = _ctx(n, N, prec)
    rng = np.random.default_rng(13)
    w = _q(_faces(g, rng, N), prec)
    out = empty(N * g.nface, prec)
    phi = empty(N * g.ncell, prec)
    flag(f"project n={n} N={N} {prec}")
    cycles = S.stfas_op_project(ctx, N, to_dev(w, prec), out, phi)
    ref = np.stack([poisson.project(g, w[b])[0] for b in range(N)])
    refphi = np.stack([poisson.project(g, w[b])[1] for b in range(N)])
    tol = TOL[prec] if prec == "fp64" else 2e-5
    assert rel(to_np(out), ref) <= tol
    assert rel(to_np(phi), refphi) <= 10 * tol
    assert 1 <= cycles <= 60
    ctx.destroy()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,N", [((128, 128), 8), ((64, 64), 3), ((16, 16, 16), 2), ((40, 24), 2)])
def test_projection_benchmark_sizes(n, N, prec):
    """Projection at the sizes the solver runs: 128x128 with 8 slices (the
    single-launch LDS form in FP32; the multi-kernel form in FP64, whose
    hierarchy does not fit in LDS), 64x64, 16^3, and a grid whose hierarchy
    stops at an odd size."""
    S, ctx, g, dt, K = _ctx(n, N, prec)
    rng = np.random.default_rng(14)
    w = _q(_faces(g, rng, N, 3.0), prec)
    out = empty(N * g.nface, prec)
    phi = empty(N * g.ncell, prec)
    flag(f"project sizes n={n} N={N} {prec}")
    cycles = S.stfas_op_project(ctx, N, to_dev(w, prec), out, phi)
    refs = [poisson.project(g, w[b]) for b in range(N)]
    ref = np.stack([r[0] for r in refs])
    refphi = np.stack([r[1] for r in refs])
    tol = TOL[prec] if prec == "fp64" else 2e-5
    assert rel(to_np(out), ref) <= tol
    assert rel(to_np(phi), refphi) <= 10 * tol
    assert 1 <= cycles <= 60
    ctx.destroy()


@pytest.mark.parametrize("prec", PRECS)
def test_metric(prec):
    S, ctx, g, dt, K = _ctx((24, 20), 2, prec, metric_levels=2)
    rng = np.random.default_rng(14)
    e = _q(rng.standard_normal(g.ncell), prec)
    out = empty(g.ncell, prec)
    S.stfas_op_metric(ctx, to_dev(e, prec), out)
    assert rel(to_np(out), metric.apply_metric(g, e, 2)) <= TOL[prec]
    ctx.destroy()


def _state(gl, N, rng, s, prec):
    return [_q(_faces(gl, rng, N, s), prec), _q(rng.standard_normal((N, gl.ncell)) * s, prec),
            _q(_faces(gl, rng, N, s), prec), _q(rng.standard_normal((N, gl.ncell)) * s, prec)]


def _dev_state(x, prec):
    return tuple(to_dev(a, prec) for a in x)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,N", CASES)
def test_kkt_residual_all_levels(n, N, prec):
    S, ctx, g, dt, K = _ctx(n, N, prec)
    kr = K / 1e-2
    rng = np.random.default_rng(15)
    for level in range(ctx.num_levels()):
        gl = Grid(tuple(x >> level for x in n), g.h * 2 ** level)
        L = kkt.Level(gl, N, dt, kr)
        x = _state(gl, N, rng, 0.5, prec)
        w = _q(_faces(gl, rng, N), prec)
        res = _state(gl, N, rng, 1.0, prec)
        out = tuple(empty(a.size, prec) for a in res)
        flag(f"kkt n={n} level={level} {prec}")
        S.stfas_op_kkt_residual(ctx, level, _dev_state(x, prec), to_dev(w, prec), _dev_state(res, prec), out)
        ref = kkt.residual(L, x, w, res)
        for k in range(4):
            assert rel(to_np(out[k]), ref[k]) <= TOL[prec], (level, k)
    ctx.destroy()


@pytest.mark.parametrize("omega,lm", [(1.0, -1.0), (0.7, -1.0), (0.7, 1.0), (1.0, 2.5)])
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,N", CASES)
def test_scgs_sweep(n, N, prec, omega, lm):
    """One SCGS sweep per level, with and without the Levenberg-Marquardt
    perturbation of the local matrix."""
    S, ctx, g, dt, K = _ctx(n, N, prec, scgs_omega=omega, scgs_lm=lm)
    kr = K / 1e-2
    rng = np.random.default_rng(16)
    for level in (0, ctx.num_levels() - 1):
        gl = Grid(tuple(x >> level for x in n), g.h * 2 ** level)
        L = kkt.Level(gl, N, dt, kr, omega=omega, lm=max(lm, 0.0))
        x = _state(gl, N, rng, 0.3, prec)
        w = _q(_faces(gl, rng, N), prec)
        res = _state(gl, N, rng, 1.0, prec) if level > 0 else None
        xd = _dev_state(x, prec)
        flag(f"scgs n={n} level={level} {prec}")
        S.stfas_op_scgs_sweep(ctx, level, xd, to_dev(w, prec), _dev_state(res, prec) if res else None)
        ref = [a.copy() for a in x]
        scgs.sweep(L, ref, w, res if res else [np.zeros_like(a) for a in x])
        for k in range(4):
            assert rel(to_np(xd[k]), ref[k]) <= TOL[prec], (level, k)
    ctx.destroy()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,N", [((8, 8), 9), ((12, 8), 37), ((8, 8), 300), ((4, 4, 4), 70), ((8, 4), 512), ((4, 4, 4), 200),
                                 ((4, 4, 4), 300)])
def test_scgs_sweep_long_horizon(n, N, prec):
    """Horizons whose 2N blocks split over 2..64 lanes per column, with a
    ragged last chunk (the face solve runs as a chunked scan in time)."""
    S, ctx, g, dt, K = _ctx(n, N, prec, scgs_omega=0.7)
    kr = K / 1e-2
    rng = np.random.default_rng(18)
    L = kkt.Level(g, N, dt, kr, omega=0.7)
    x = _state(g, N, rng, 0.3, prec)
    w = _q(_faces(g, rng, N), prec)
    xd = _dev_state(x, prec)
    flag(f"scgs long n={n} N={N} {prec}")
    S.stfas_op_scgs_sweep(ctx, 0, xd, to_dev(w, prec), None)
    ref = [a.copy() for a in x]
    scgs.sweep(L, ref, w, [np.zeros_like(a) for a in x])
    for k in range(4):
        assert rel(to_np(xd[k]), ref[k]) <= TOL[prec], k
    ctx.destroy()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,N", [((128, 128), 40), ((128, 128), 20), ((32, 32, 32), 10)])
def test_scgs_sweep_benchmark_shapes(n, N, prec):
    """Colours of at least 4096 cells take the row layout of the colour pass
    (chunks across the waves of a workgroup, chunk maps joined in LDS):
    128x128 x 40 is the shape the benchmark times (16 chunks of 6 blocks in
    FP32), 128x128 x 20 and 32^3 x 10 reach it in FP64 and in 3D; with the
    solver's default smoother (omega 0.7, Levenberg-Marquardt perturbation on)."""
    S, ctx, g, dt, K = _ctx(n, N, prec, scgs_omega=0.7, scgs_lm=1.0)
    kr = K / 1e-2
    rng = np.random.default_rng(19)
    L = kkt.Level(g, N, dt, kr, omega=0.7, lm=1.0)
    x = _state(g, N, rng, 0.3, prec)
    w = _q(_faces(g, rng, N), prec)
    xd = _dev_state(x, prec)
    flag(f"scgs shapes n={n} N={N} {prec}")
    S.stfas_op_scgs_sweep(ctx, 0, xd, to_dev(w, prec), None)
    ref = [a.copy() for a in x]
    scgs.sweep(L, ref, w, [np.zeros_like(a) for a in x])
    for k in range(4):
        assert rel(to_np(xd[k]), ref[k]) <= TOL[prec], k
    ctx.destroy()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,N", [((16, 12), 3), ((8, 8, 8), 2)])
def test_transfers(n, N, prec):
    S, ctx, g, dt, K = _ctx(n, N, prec)
    rng = np.random.default_rng(17)
    T = transfer.Transfer(g)
    gc = T.coarse
    xf = _state(g, N, rng, 1.0, prec)
    xc = tuple(empty(a.size // g.nface * gc.nface if k % 2 == 0 else a.size // g.ncell * gc.ncell, prec)
               for k, a in enumerate(xf))
    flag(f"transfers n={n} {prec}")
    S.stfas_op_restrict(ctx, 0, _dev_state(xf, prec), xc)
    ref = T.restrict_state([a.copy() for a in xf])
    for k in range(4):
        assert rel(to_np(xc[k]), ref[k]) <= TOL[prec]
    cs = _state(gc, N, rng, 1.0, prec)
    fd = _dev_state(xf, prec)
    S.stfas_op_prolong(ctx, 0, _dev_state(cs, prec), -1.0, fd)
    pr = T.prolong_state(cs)
    for k in range(4):
        assert rel(to_np(fd[k]), xf[k] - pr[k]) <= TOL[prec]
    ctx.destroy()


@pytest.mark.parametrize("prec", PRECS)
def test_invalid_arguments_rejected(prec):
    from paper_1608_01102_amd import stfas as S
    from paper_1608_01102_amd._lib import StfasError
    S_, ctx, g, dt, K = _ctx((16, 12), 3, prec)
    with pytest.raises(StfasError):
        S.stfas_op_kkt_residual(ctx, 5, tuple(zeros(1 << 12, prec) for _ in range(4)), zeros(1 << 12, prec),
                                None, tuple(zeros(1 << 12, prec) for _ in range(4)))
    rho0 = zeros(g.ncell, prec)
    u = zeros(3 * g.nface, prec)
    for bad in ([0], [4], [2, 2], [3, 1]):
        with pytest.raises(StfasError):
            S.stfas_solve(ctx, rho0, bad, zeros(len(bad) * g.ncell, prec), u)
    ctx.destroy()


@pytest.mark.parametrize("prec", PRECS)
def test_tiled_adjoints_propagate_nonfinite(prec):
    """A NaN in the cotangent of the tiled density adjoint and of the tiled
    velocity-advection transpose (both sum their windows in fixed point)
    reaches the output at the affected nodes instead of turning into an
    arbitrary integer; every other node keeps the oracle's value."""
    n, B = (64, 64), 40
    S, ctx, g, dt, K = _ctx(n, 2, prec, dt=1.0 / n[0])
    rng = np.random.default_rng(26)
    assert g.ncell * B >= 131072
    v = _q(np.stack([synthetic.curl_noise_velocity(n, rng, 2.0, 1.0, dt / g.h) for _ in range(B)]), prec)
    mu = _q(rng.standard_normal((B, g.ncell)), prec)
    bad = (3, 2000)
    mu[bad] = np.nan
    out = empty(B * g.ncell, prec)
    flag(f"advect_T tiled with a NaN {prec}")
    S.stfas_op_advect_T(ctx, B, to_dev(mu, prec), to_dev(v, prec), None, out)
    got = to_np(out).reshape(B, -1)
    mu_ok = mu.copy()
    mu_ok[bad] = 0.0
    ref = advect.advect_scalar_T(g, mu_ok, v, dt)
    nan = ~np.isfinite(got)
    assert nan[3].any() and not nan[np.arange(B) != 3].any() and nan[3].sum() <= 4
    assert rel(got[~nan], ref[~nan]) <= TOL[prec]
    # the velocity-advection transpose, tiled (one slice covers more than the untiled limit per launch)
    y = _q(np.stack([synthetic.random_faces(n, rng) for _ in range(B)]), prec)
    badf = (5, g.face_offsets[0] + 40 * (n[0] + 1) + 30)        # an interior x-face
    y[badf] = np.nan
    outf = zeros(B * g.nface, prec)
    flag(f"self_advect_T tiled with a NaN {prec}")
    S.stfas_op_self_advect_T(ctx, 0, B, to_dev(v, prec), to_dev(y, prec), 1.0, outf)
    gotf = to_np(outf).reshape(B, -1)
    y_ok = y.copy()
    y_ok[badf] = 0.0
    reff = advect.self_advect_T(g, v, y_ok, dt)
    nanf = ~np.isfinite(gotf)
    assert nanf[5].any() and not nanf[np.arange(B) != 5].any()
    assert rel(gotf[~nanf], reff[~nanf]) <= TOL[prec]
