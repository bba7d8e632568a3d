"""Parity of the composite stages (velocity subproblem, density subproblem,
full ADMM solve, simulation step and its adjoint) with the FP64 oracle,
through the C interface, with identical control flow (fixed counts)."""
import numpy as np
import pytest

import synthetic
from gpu_common import TOL, empty, flag, rel, to_dev, to_np, zeros
from oracle import admm, ao, step, stfas
from oracle.grid import Grid

pytestmark = pytest.mark.gpu


def _q(x, prec):
    return np.asarray(x, dtype=np.float32).astype(np.float64) if prec == "mixed" else np.asarray(x)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n,N", [((16, 16), 4), ((8, 8, 8), 3)])
def test_nso_vcycles(n, N, prec):
    from paper_1608_01102_amd import stfas as S
    g = Grid(n)
    dt, r = g.h, 1e-2
    K = r / dt ** 2
    prob = S.make_problem(n, N, r, dt=dt, K=K, max_vcycles=3, fixed_counts=True, precision=prec, scgs_omega=0.7)
    ctx = S.stfas_create(prob)
    rng = np.random.default_rng(21)
    w = _q(np.stack([synthetic.curl_noise_velocity(n, rng, 1.0, 0.8) for _ in range(N)]), prec)
    x = [np.zeros((N, g.nface)), np.zeros((N, g.ncell)), np.zeros((N, g.nface)), np.zeros((N, g.ncell))]
    xd = tuple(to_dev(a, prec) for a in x)
    flag(f"nso n={n} N={N} {prec}")
    nv, hist = S.stfas_op_nso(ctx, xd, to_dev(w, prec))
    H = stfas.Hierarchy(g, N, dt, K / r, omega=0.7, lm=1.0)
    nv_ref, hist_ref = stfas.nso(H, x, w, max_vcycles=3, fixed_counts=True)
    assert nv == nv_ref == 3
    for k in range(4):
        assert rel(to_np(xd[k]), x[k]) <= TOL[prec], k
    assert np.allclose(hist, hist_ref, rtol=1e-8 if prec == "fp64" else 1e-2)
    ctx.destroy()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_density_subproblem(prec):
    from paper_1608_01102_amd import stfas as S
    w = synthetic.c1_plain_2d_32(3)
    g = Grid(w["n"])
    N, dt, r = w["num_steps"], w["dt"], w["r"]
    K = r / dt ** 2
    prob = S.make_problem(w["n"], N, r, dt=dt, K=K, ao_iters=2, metric_levels=3, precision=prec)
    ctx = S.stfas_create(prob)
    rng = np.random.default_rng(22)
    vt = _q(np.stack([synthetic.curl_noise_velocity(w["n"], rng, 2.0, 0.5) for _ in range(N)]), prec)
    rho0 = _q(w["rho0"], prec)
    keys = {t: _q(v, prec) for t, v in w["keys"].items()}
    ks = sorted(keys)
    vs = empty(N * g.nface, prec)
    rho = empty((N + 1) * g.ncell, prec)
    flag(f"ao c1-shape {prec}")
    hist = S.stfas_op_ao(ctx, to_dev(rho0, prec), ks, to_dev(np.stack([keys[k] for k in ks]), prec),
                         to_dev(vt, prec), vs, rho)
    vs_ref, rho_ref, hist_ref = ao.solve(g, rho0, keys, vt, K, dt, 3, iters=2)
    tol = TOL[prec]
    assert rel(to_np(vs), vs_ref) <= tol
    assert rel(to_np(rho), rho_ref) <= tol
    assert np.allclose(hist, hist_ref, rtol=1e-9 if prec == "fp64" else 1e-4)
    assert all(hist[i + 1] <= hist[i] for i in range(len(hist) - 1))
    ctx.destroy()


def _solve_pair(w, prec, max_admm, max_vcycles, **kw):
    from paper_1608_01102_amd import stfas as S
    g = Grid(w["n"])
    N = w["num_steps"]
    args = dict(n=w["n"], num_steps=N, r=w["r"], dt=w["dt"], max_admm=max_admm, max_vcycles=max_vcycles,
                fixed_counts=True, **kw)
    prob = S.make_problem(precision=prec, **args)
    ctx = S.stfas_create(prob)
    rho0 = _q(w["rho0"], prec)
    keys = {t: _q(v, prec) for t, v in w["keys"].items()}
    ks = sorted(keys)
    u = empty(N * g.nface, prec)
    flag(f"solve n={w['n']} N={N} {prec} admm={max_admm} vc={max_vcycles}")
    st = S.stfas_solve(ctx, to_dev(rho0, prec), ks, to_dev(np.stack([keys[k] for k in ks]), prec), u)
    ref = admm.solve(admm.Problem(**args), rho0, keys)
    ctx.destroy()
    return to_np(u).reshape(N, -1), st, ref


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_small(prec):
    w = synthetic.small_problem((8, 8), 4, seed=0, r=1e-2)
    u, st, ref = _solve_pair(w, prec, 3, 3)
    tol = TOL[prec]
    assert rel(u, ref.u) <= tol
    assert abs(st["objective"] - ref.objective) <= tol * ref.objective
    assert st["admm_iters"] == ref.admm_iters and st["vcycles"] == ref.vcycles


def test_solve_c1_fp64():
    """The 32x32x10 workload (FP64), two ADMM iterations of four V-cycles."""
    w = synthetic.c1_plain_2d_32(0)
    u, st, ref = _solve_pair(w, "fp64", 2, 4)
    assert rel(u, ref.u) <= 1e-10
    assert abs(st["objective"] - ref.objective) <= 1e-10 * ref.objective
    assert abs(st["reg_term"] - ref.reg_term) <= 1e-10 * ref.reg_term


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n", [(16, 12), (8, 8, 8)])
def test_step_forward_backward(n, prec):
    from paper_1608_01102_amd import stfas as S
    g = Grid(n)
    dt = 0.9 * g.h
    prob = S.make_problem(n, 1, 1.0, dt=dt, precision=prec)
    rng = np.random.default_rng(23)
    rho = _q(synthetic.smooth_noise_density(n, rng, 1.0), prec)
    v = _q(synthetic.curl_noise_velocity(n, rng, 1.0, 1.5, dt / g.h), prec)
    u = _q(synthetic.random_faces(n, rng, 2.0), prec)
    ro, vo, po = empty(g.ncell, prec), empty(g.nface, prec), empty(g.ncell, prec)
    flag(f"step n={n} {prec}")
    S.stfas_step_forward(prob, to_dev(rho, prec), to_dev(v, prec), to_dev(u, prec), ro, vo, po)
    rr, vr, pr = step.step_forward(g, rho, v, u, dt)
    tol = TOL[prec] if prec == "fp64" else 2e-5
    assert rel(to_np(ro), rr) <= tol and rel(to_np(vo), vr) <= tol and rel(to_np(po), pr) <= 10 * tol
    grn = _q(rng.standard_normal(g.ncell), prec)
    gvn = _q(synthetic.random_faces(n, rng), prec)
    gr, gv, gu = empty(g.ncell, prec), empty(g.nface, prec), empty(g.nface, prec)
    S.stfas_step_backward(prob, to_dev(rho, prec), to_dev(v, prec), to_dev(grn, prec), to_dev(gvn, prec), gr, gv, gu)
    a, b, c = step.step_backward(g, rho, v, grn, gvn, dt)
    assert rel(to_np(gr), a) <= tol and rel(to_np(gv), b) <= tol and rel(to_np(gu), c) <= tol


def _edge_case(name):
    """Degenerate and boundary instances of the full solve."""
    rng = np.random.default_rng(31)
    if name == "one_step":                     # N = 1: the keyframe is the first step
        return synthetic.small_problem((8, 8), 1, seed=3, r=1e-2)
    if name == "two_keys_3d":                  # keyframes in the middle and at the end
        w = synthetic.small_problem((8, 8, 8), 4, seed=4, r=1e-2)
        w["keys"] = {2: synthetic.smooth_noise_density((8, 8, 8), rng, 1.0), 4: w["keys"][4]}
        return w
    if name == "odd_coarse":                   # 12 x 10: the hierarchy stops at 6 x 5
        return synthetic.small_problem((12, 10), 3, seed=5, r=1e-2)
    if name == "zero":                         # no density anywhere: the control stays zero
        w = synthetic.small_problem((8, 8), 3, seed=6, r=1e-2)
        w["rho0"] = np.zeros_like(w["rho0"])
        w["keys"] = {3: np.zeros_like(w["keys"][3])}
        return w
    raise ValueError(name)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["one_step", "two_keys_3d", "odd_coarse", "zero"])
def test_solve_edge_cases(name, prec):
    w = _edge_case(name)
    u, st, ref = _solve_pair(w, prec, 2, 2, eps_admm=1.0)
    tol = TOL[prec]
    scale = max(float(np.abs(ref.u).max()), 1e-30)
    if name == "zero":
        assert np.abs(u).max() == 0.0 and np.abs(ref.u).max() == 0.0
        assert st["objective"] == 0.0
    elif name == "one_step":
        # with one step the control acts only after the last density: it stays zero,
        # and the objective is the keyframe mismatch of the uncontrolled density
        assert np.abs(u).max() == 0.0 and np.abs(ref.u).max() == 0.0
        assert abs(st["objective"] - ref.objective) <= tol * ref.objective
    else:
        assert rel(u, ref.u) <= tol
        assert abs(st["objective"] - ref.objective) <= tol * max(ref.objective, 1e-30)
    assert np.isfinite(u).all() and np.abs(u).max() <= 10 * scale
    assert st["admm_iters"] == ref.admm_iters and st["vcycles"] == ref.vcycles


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("al_tol", [1e-300, 0.05])
def test_solve_al_fallback(al_tol, prec):
    """The augmented-Lagrangian fallback of the ADMM loop: same controls,
    objective and number of multiplier updates as the oracle."""
    w = synthetic.small_problem((8, 8), 3, seed=4, r=1e-2)
    u, st, ref = _solve_pair(w, prec, 4, 3, al_tol=al_tol)
    tol = TOL[prec]
    assert st["multiplier_updates"] == ref.history["updates"]
    assert rel(u, ref.u) <= tol
    assert abs(st["objective"] - ref.objective) <= tol * ref.objective


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_repeatable(prec):
    """Two solves of the 32x32x10 workload on fresh contexts.  The
    transposes add their tile windows into the output with floating-point
    atomics, so the order of those additions varies between runs: FP64 agrees
    to rounding, the mixed form within its parity tolerance."""
    from paper_1608_01102_amd import stfas as S
    w = synthetic.c1_plain_2d_32(0)
    g = Grid(w["n"])
    N = w["num_steps"]
    ks = sorted(w["keys"])
    out = []
    for rep in range(2):
        prob = S.make_problem(w["n"], N, w["r"], dt=w["dt"], max_admm=2, max_vcycles=4, fixed_counts=True,
                              precision=prec)
        ctx = S.stfas_create(prob)
        u = zeros(N * g.nface, prec)
        flag(f"repeatable solve {prec} run {rep}")
        st = S.stfas_solve(ctx, to_dev(_q(w["rho0"], prec), prec), ks,
                           to_dev(np.stack([_q(w["keys"][k], prec) for k in ks]), prec), u)
        ctx.destroy()
        out.append((to_np(u), st["objective"]))
    (u0, j0), (u1, j1) = out
    tol = 1e-12 if prec == "fp64" else TOL[prec]
    assert rel(u1, u0) <= tol
    assert abs(j1 - j0) <= tol * abs(j0)


def _stop_margins(ref, eps_admm, eps_stfas, margin=0.05):
    """Every stop decision of the oracle's run is at least `margin` (relative)
    away from its threshold, so that rounding cannot flip it."""
    h = ref.history
    for d in h["visual_diff"]:
        assert abs(d - eps_admm) > margin * eps_admm, d
    for res, f0 in zip(h["nso_res"], h["nso_f0"]):
        for x in res:
            assert abs(x - eps_stfas * f0) > margin * eps_stfas * f0, (x, f0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_stop_tests(prec):
    """Tolerance-driven solve (fixed_counts = 0): the velocity subproblem stops
    on its relative KKT residual (eps_stfas) before the V-cycle cap and the ADMM
    loop on its visual difference (eps_admm) before the iteration cap; the
    GPU takes the same decisions as the oracle (same ADMM iterations and
    V-cycles) and returns the same controls."""
    from paper_1608_01102_amd import stfas as S
    w = synthetic.small_problem((16, 16), 6, seed=1, r=1e-2)
    g = Grid(w["n"])
    N = w["num_steps"]
    args = dict(n=w["n"], num_steps=N, r=w["r"], dt=w["dt"], max_admm=12, max_vcycles=30, eps_stfas=1e-4,
                eps_admm=0.011, fixed_counts=False)
    ref = admm.solve(admm.Problem(**args), w["rho0"], w["keys"])
    assert ref.converged and ref.admm_iters < 12
    nso_counts = [len(x) - 1 for x in ref.history["nso_res"]]
    assert all(0 < c < 30 for c in nso_counts), nso_counts
    _stop_margins(ref, 0.011, 1e-4)
    prob = S.make_problem(precision=prec, **args)
    ctx = S.stfas_create(prob)
    ks = sorted(w["keys"])
    u = empty(N * g.nface, prec)
    flag(f"solve with stop tests {prec}")
    st = S.stfas_solve(ctx, to_dev(_q(w["rho0"], prec), prec), ks,
                       to_dev(np.stack([_q(w["keys"][k], prec) for k in ks]), prec), u)
    ctx.destroy()
    assert st["converged"] == 1
    assert st["admm_iters"] == ref.admm_iters and st["vcycles"] == ref.vcycles
    assert rel(to_np(u).reshape(N, -1), ref.u) <= TOL[prec]
    assert abs(st["objective"] - ref.objective) <= TOL[prec] * ref.objective
