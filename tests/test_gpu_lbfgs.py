"""Parity of the L-BFGS baseline (the gradient-based optimiser the paper
compares against in Sec. 5) with the FP64 oracle, through the C interface:
same objective history, same iteration count, same controls."""
import numpy as np
import pytest

import synthetic
from gpu_common import TOL, flag, rel, to_dev, to_np
from oracle import lbfgs, metric
from oracle.admm import resimulate
from oracle.grid import Grid

pytestmark = pytest.mark.gpu


def _q(x, prec):
    return np.asarray(x, dtype=np.float32).astype(np.float64) if prec == "mixed" else np.asarray(x)


def _pair(w, prec, iters, u0=None, eps_stop=0.0):
    from paper_1608_01102_amd import stfas as S
    g = Grid(w["n"])
    N, dt, r = w["num_steps"], w["dt"], w["r"]
    prob = S.make_problem(w["n"], N, r, dt=dt, precision=prec)
    ctx = S.stfas_create(prob)
    rho0 = _q(w["rho0"], prec)
    keys = {t: _q(v, prec) for t, v in w["keys"].items()}
    ks = sorted(keys)
    u0 = np.zeros((N, g.nface)) if u0 is None else _q(u0, prec)
    u = to_dev(u0, prec)
    flag(f"lbfgs n={w['n']} N={N} {prec} iters={iters}")
    hist, done = S.stfas_lbfgs(ctx, to_dev(rho0, prec), ks, to_dev(np.stack([keys[k] for k in ks]), prec), u,
                               iters, eps_stop)
    ctx.destroy()
    u_ref, hist_ref, done_ref = lbfgs.solve(g, rho0, keys, N, r, dt, metric.default_levels(w["n"]), iters, u0=u0,
                                            eps_stop=eps_stop)
    return to_np(u).reshape(N, -1), hist, done, u_ref, hist_ref, done_ref


@pytest.mark.parametrize("n,N,iters", [((8, 8), 4, 6), ((8, 8, 8), 3, 4), ((12, 10), 3, 5)])
def test_lbfgs_fp64(n, N, iters):
    w = synthetic.small_problem(n, N, seed=7, r=1e-2)
    u, hist, done, u_ref, hist_ref, done_ref = _pair(w, "fp64", iters)
    assert done == done_ref
    assert np.allclose(hist, hist_ref, rtol=1e-9, atol=0)
    assert rel(u, u_ref) <= 1e-9
    assert all(hist[i + 1] < hist[i] for i in range(len(hist) - 1))


def test_lbfgs_mixed():
    w = synthetic.small_problem((8, 8), 4, seed=8, r=1e-2)
    u, hist, done, u_ref, hist_ref, done_ref = _pair(w, "mixed", 3)
    assert done == done_ref
    assert np.allclose(hist, hist_ref, rtol=1e-4, atol=0)
    assert rel(u, u_ref) <= TOL["mixed"]


def test_lbfgs_warm_start_and_zero_iterations():
    """iters = 0 evaluates J at the start only; a nonzero start is honoured."""
    w = synthetic.small_problem((8, 8), 3, seed=9, r=1e-2)
    g = Grid(w["n"])
    rng = np.random.default_rng(41)
    u0 = 0.1 * np.stack([synthetic.random_faces(w["n"], rng) for _ in range(3)])
    u, hist, done, u_ref, hist_ref, done_ref = _pair(w, "fp64", 0, u0=u0)
    assert done == done_ref == 0 and len(hist) == 1
    assert abs(hist[0] - hist_ref[0]) <= 1e-10 * hist_ref[0]
    assert np.array_equal(u, u0)
    u, hist, done, u_ref, hist_ref, done_ref = _pair(w, "fp64", 3, u0=u0)
    assert done == done_ref and np.allclose(hist, hist_ref, rtol=1e-9, atol=0)
    assert rel(u, u_ref) <= 1e-9
    assert g.nface == u.shape[1]


def test_lbfgs_visual_difference_stop():
    """The stop rule shared with the ADMM loop: the oracle's iterates give a
    threshold that fires before the iteration cap, away from every change."""
    w = synthetic.small_problem((8, 8), 4, seed=11, r=1e-2)
    g = Grid(w["n"])
    N, dt, r = w["num_steps"], w["dt"], w["r"]
    lev = metric.default_levels(w["n"])
    K = 8
    xs = [lbfgs.solve(g, w["rho0"], w["keys"], N, r, dt, lev, k)[0] for k in range(K + 1)]
    traj = [resimulate(g, w["rho0"], x, dt)[0] for x in xs]
    diffs = np.array([np.max(np.abs(traj[k] - traj[k - 1])) for k in range(1, K + 1)])
    eps = float(np.sqrt(diffs.min() * diffs.max()))
    assert np.min(np.abs(diffs - eps)) > 1e-3 * eps
    u, hist, done, u_ref, hist_ref, done_ref = _pair(w, "fp64", K, eps_stop=eps)
    assert done == done_ref < K
    assert np.allclose(hist, hist_ref, rtol=1e-9, atol=0)
    assert rel(u, u_ref) <= 1e-9


def test_lbfgs_rejects_caller_workspace():
    """A context on caller memory makes no allocation, so L-BFGS is refused."""
    import torch
    from paper_1608_01102_amd import stfas as S
    w = synthetic.small_problem((8, 8), 2, seed=10, r=1e-2)
    g = Grid(w["n"])
    prob = S.make_problem(w["n"], 2, w["r"], dt=w["dt"], precision="fp64")
    ws = torch.empty(S.stfas_workspace_bytes(prob) + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    ctx = S.stfas_create_in(prob, ws[off:])
    u = to_dev(np.zeros((2, g.nface)), "fp64")
    with pytest.raises(RuntimeError):
        S.stfas_lbfgs(ctx, to_dev(w["rho0"], "fp64"), [2], to_dev(w["keys"][2][None], "fp64"), u, 2)
    ctx.destroy()


def test_lbfgs_invalid_arguments():
    """Rejected before anything runs: negative iterations, a negative or NaN
    stop threshold, keyframe steps outside 1..N."""
    from paper_1608_01102_amd import stfas as S
    w = synthetic.small_problem((8, 8), 2, seed=12, r=1e-2)
    g = Grid(w["n"])
    prob = S.make_problem(w["n"], 2, w["r"], dt=w["dt"], precision="fp64")
    ctx = S.stfas_create(prob)
    rho0 = to_dev(w["rho0"], "fp64")
    key = to_dev(w["keys"][2][None], "fp64")
    u = to_dev(np.zeros((2, g.nface)), "fp64")
    flag("lbfgs invalid arguments")
    for args in ([2], key, -1, 0.0), ([2], key, 2, -1.0), ([2], key, 2, float("nan")), ([3], key, 2, 0.0), \
            ([0], key, 2, 0.0):
        with pytest.raises(RuntimeError):
            S.stfas_lbfgs(ctx, rho0, args[0], args[1], u, args[2], args[3])
    assert not np.any(to_np(u))                  # nothing ran
    ctx.destroy()
