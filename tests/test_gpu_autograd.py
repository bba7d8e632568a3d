"""Differentiation form: the autograd step against the oracle's adjoint, FP64
central finite differences and the dot-product test at 128^3, and the
checkpointed 60-step trajectory against the fully stored one."""
import numpy as np
import pytest
import torch

import synthetic
from gpu_common import flag, rel
from oracle import step as ostep
from oracle.grid import Grid

pytestmark = pytest.mark.gpu


def _t(x, dt):
    return torch.tensor(np.ascontiguousarray(x).ravel(), dtype=dt, device="cuda:0")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_autograd_step_matches_oracle_adjoint(prec):
    from paper_1608_01102_amd import autograd, stfas as S
    n = (16, 12, 10)
    g = Grid(n)
    dt = 0.8 * g.h
    prob = S.make_problem(n, 1, 1.0, dt=dt, precision=prec)
    tdt = torch.float64 if prec == "fp64" else torch.float32
    rng = np.random.default_rng(31)
    q = (lambda x: x) if prec == "fp64" else (lambda x: np.float32(x).astype(np.float64))
    rho = q(synthetic.smooth_noise_density(n, rng, 1.0))
    v = q(synthetic.curl_noise_velocity(n, rng, 1.0, 1.5, dt / g.h))
    u = q(synthetic.random_faces(n, rng, 1.0))
    grn = q(rng.standard_normal(g.ncell))
    gvn = q(synthetic.random_faces(n, rng))
    rt, vt_, ut = [_t(a, tdt).requires_grad_() for a in (rho, v, u)]
    flag(f"autograd step {n} {prec}")
    ro, vo = autograd.step(rt, vt_, ut, prob)
    loss = (ro * _t(grn, tdt)).sum() + (vo * _t(gvn, tdt)).sum()
    loss.backward()
    a, b, c = ostep.step_backward(g, rho, v, grn, gvn, dt)
    tol = 1e-10 if prec == "fp64" else 2e-5
    assert rel(rt.grad.double().cpu().numpy(), a) <= tol
    assert rel(vt_.grad.double().cpu().numpy(), b) <= tol
    assert rel(ut.grad.double().cpu().numpy(), c) <= tol


def _c4_inputs(n, rng, dt_over_h):
    rho = synthetic.smooth_noise_density(n, rng, 2.0)
    v = synthetic.curl_noise_velocity(n, rng, 4.0, 2.0, dt_over_h)
    return rho, v


def test_c4_step_fd_and_dot_product():
    """128^3 single step: FP32 backward vs FP64 backward, and the FP64 backward
    vs central differences of the FP64 forward in 16 seeded directions."""
    from paper_1608_01102_amd import autograd, stfas as S
    n = (128, 128, 128)
    g = Grid(n)
    dt = g.h
    rng = np.random.default_rng(32)
    rho, v = _c4_inputs(n, rng, dt / g.h)
    u = synthetic.curl_noise_velocity(n, rng, 4.0, 0.3, dt / g.h) / dt
    grn = rng.standard_normal(g.ncell)
    gvn = synthetic.random_faces(n, rng)
    p64 = S.make_problem(n, 1, 1.0, dt=dt, precision="fp64")
    p32 = S.make_problem(n, 1, 1.0, dt=dt, precision="mixed")
    grads = {}
    for prec, prob, tdt in (("fp64", p64, torch.float64), ("mixed", p32, torch.float32)):
        flag(f"c4 step 128^3 {prec}")
        xs = [_t(a, tdt).requires_grad_() for a in (rho, v, u)]
        ro, vo = autograd.step(*xs, prob)
        if prec == "mixed":
            # the projected velocity is divergence free to FP32 precision
            vv = vo.detach().double().cpu().numpy()
            from oracle.grid import div
            assert np.max(np.abs(div(g, vv))) * g.h / np.max(np.abs(vv)) < 1e-5
        loss = (ro * _t(grn, tdt)).sum() + (vo * _t(gvn, tdt)).sum()
        loss.backward()
        grads[prec] = [x.grad.double().cpu().numpy() for x in xs]
    for k in range(3):
        assert rel(grads["mixed"][k], grads["fp64"][k]) <= 1e-4, k
    # FP64 central differences in 16 seeded directions
    x64 = [_t(a, torch.float64) for a in (rho, v, u)]
    gr64, gv64 = _t(grn, torch.float64), _t(gvn, torch.float64)

    def L(xs):
        with torch.no_grad():
            ro, vo = autograd.step(*xs, p64)
        return float((ro * gr64).sum() + (vo * gv64).sum())
    bad = 0
    for d in range(16):
        dirs = [rng.standard_normal(g.ncell), synthetic.random_faces(n, rng), synthetic.random_faces(n, rng)]
        scale = [np.linalg.norm(a) / np.linalg.norm(b) for a, b in zip((rho, v, u), dirs)]
        dirs = [b * s for b, s in zip(dirs, scale)]
        eps = 1e-7
        xp = [a + eps * _t(b, torch.float64) for a, b in zip(x64, dirs)]
        xm = [a - eps * _t(b, torch.float64) for a, b in zip(x64, dirs)]
        fd = (L(xp) - L(xm)) / (2 * eps)
        ad = sum(float(np.dot(gk, dk)) for gk, dk in zip(grads["fp64"], dirs))
        if abs(fd - ad) > 1e-5 * abs(ad):
            bad += 1
    # a direction may cross a kink of the piecewise-linear interpolation
    assert bad <= 1
    # dot-product test <J dx, y> = <dx, J^T y> with J dx from the linearised FD
    dirs = [rng.standard_normal(g.ncell) * 1e-3, synthetic.random_faces(n, rng) * 1e-3, synthetic.random_faces(n, rng)]
    eps = 1e-6
    with torch.no_grad():
        rp, vp = autograd.step(*[a + eps * _t(b, torch.float64) for a, b in zip(x64, dirs)], p64)
        rm, vm = autograd.step(*[a - eps * _t(b, torch.float64) for a, b in zip(x64, dirs)], p64)
    jdx = float(((rp - rm) * gr64).sum() + ((vp - vm) * gv64).sum()) / (2 * eps)
    jty = sum(float(np.dot(gk, dk)) for gk, dk in zip(grads["fp64"], dirs))
    assert abs(jdx - jty) <= 1e-6 * (abs(jty) + 1e-30)


def test_c4_trajectory_checkpointing():
    """128^3 x 60 steps (FP32): gradients with every-8th-state checkpointing
    equal the fully stored ones, with far less memory held."""
    from paper_1608_01102_amd import autograd, stfas as S
    n = (128, 128, 128)
    g = Grid(n)
    dt = g.h
    N = 60
    rng = np.random.default_rng(33)
    rho, v = _c4_inputs(n, rng, 1.0)
    base = [synthetic.curl_noise_velocity(n, rng, 6.0, 0.2, 1.0) / dt for _ in range(2)]
    coef = rng.uniform(-1, 1, size=(N, 2))
    target = synthetic.smooth_noise_density(n, rng, 3.0)
    prob = S.make_problem(n, 1, 1.0, dt=dt, precision="mixed")
    f32 = torch.float32
    B = [_t(b, f32) for b in base]
    tgt = _t(target, f32)
    res = {}
    for k in (0, 8):
        flag(f"trajectory checkpoint_every={k}")
        # one leaf per step with a preallocated gradient, so that gradients
        # accumulate in place and the peak measures the stored states
        us = [(float(c[0]) * B[0] + float(c[1]) * B[1]).requires_grad_() for c in coef]
        for x in us:
            x.grad = torch.zeros_like(x)
        r0 = _t(rho, f32).requires_grad_()
        r0.grad = torch.zeros_like(r0)
        v0 = torch.zeros(g.nface, dtype=f32, device="cuda:0")
        # memory the rollout and its backward add on top of inputs and gradients
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        torch.cuda.reset_peak_memory_stats()
        rN, vN, _ = autograd.rollout(prob, r0, v0, us, checkpoint_every=k)
        loss = 0.5 * ((rN - tgt) ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        extra = torch.cuda.max_memory_allocated() - base
        ug = torch.stack([x.grad for x in us]).double().cpu().numpy()
        res[k] = (float(loss.detach()), ug, r0.grad.double().cpu().numpy(), extra)
        del us, r0, v0, rN, vN, loss
        torch.cuda.empty_cache()
    assert abs(res[8][0] - res[0][0]) <= 1e-6 * abs(res[0][0])
    assert rel(res[8][1], res[0][1]) <= 1e-4
    assert rel(res[8][2], res[0][2]) <= 1e-4
    # 60 stored states of 128^3 (rho and v, FP32) are about 2 GB; every 8th is about 0.3 GB
    assert res[0][3] > 1.5e9
    assert res[8][3] < 0.5 * res[0][3]
