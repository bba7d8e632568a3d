"""Pins of the upwind Taylor-exponential density operator (Sec. 3.1 eq:Adv)
against what fixes it independently: the derivative of linear data, second
order convergence on smooth data, mass conservation, constants carried by a
divergence-free field, the matrix exponential of a library routine, dense
matrix powers for the truncation rule, finite differences and the
dot-product test for the two adjoints."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import upwind
from oracle.grid import Grid
from oracle.poisson import project


def _cell_coords(g):
    """Cell-centre coordinates (x, y[, z]) in units of h, C-ordered."""
    idx = np.indices(g.cell_shape)
    return [idx[g.npax(a)].ravel() + 0.5 for a in range(g.dim)]


def _uniform_faces(g, a, val):
    v = np.zeros(g.nface)
    parts = g.split(v)
    parts[a][...] = val
    return g.join(parts) * g.interior_mask()


@pytest.mark.parametrize("n", [(12, 9), (7, 6, 8)])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_linear_data_gives_the_exact_derivative(n, sign):
    g = Grid(n)
    X = _cell_coords(g)
    for a in range(g.dim):
        rho = 0.3 + 0.7 * X[a] * g.h + 0.2 * X[(a + 1) % g.dim] * g.h
        v = _uniform_faces(g, a, sign * 1.3)
        out = upwind.matrix(g, v) @ rho
        ia = np.rint(X[a] - 0.5).astype(int)
        inner = (ia >= 2) & (ia <= g.n[a] - 3)           # both faces interior with a full stencil
        assert np.allclose(out[inner], -sign * 1.3 * 0.7, rtol=0, atol=1e-12)


def test_second_order_on_smooth_data():
    errs = []
    for m in (32, 64, 128):
        g = Grid((m, 4))
        X = _cell_coords(g)
        x = X[0] * g.h
        rho = np.sin(2 * np.pi * x)
        v = _uniform_faces(g, 0, 1.0)
        out = upwind.matrix(g, v) @ rho
        ia = np.rint(X[0] - 0.5).astype(int)
        inner = (ia >= 2) & (ia <= m - 3)
        errs.append(np.max(np.abs(out[inner] + 2 * np.pi * np.cos(2 * np.pi * x[inner]))))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.9, rates


def test_upwind_side_only():
    """For v_x > 0 the x-stencil of a cell uses only itself and upstream cells."""
    g = Grid((10, 6))
    A = upwind.matrix(g, _uniform_faces(g, 0, 0.8)).toarray()
    X = _cell_coords(g)
    ix = np.rint(X[0] - 0.5).astype(int)
    iy = np.rint(X[1] - 0.5).astype(int)
    for c in range(g.ncell):
        for c2 in np.nonzero(A[c])[0]:
            assert iy[c2] == iy[c] and ix[c] - 2 <= ix[c2] <= ix[c]


@pytest.mark.parametrize("n", [(9, 7), (5, 6, 4)])
def test_mass_conservation_and_constants(n):
    g = Grid(n)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(g.nface) * g.interior_mask() * 0.5
    A = upwind.matrix(g, v)
    assert np.allclose(np.asarray(A.sum(axis=0)).ravel(), 0.0, atol=1e-9)
    rho = rng.random(g.ncell)
    out = upwind.advect_up(g, rho, v, g.h)
    assert abs(out.sum() - rho.sum()) <= 1e-12 * rho.sum()
    vd, _ = project(g, v, rtol=1e-14)                       # discretely divergence-free
    one = np.ones(g.ncell)
    assert np.allclose(upwind.advect_up(g, one, vd, g.h), 1.0, rtol=0, atol=1e-11)


def test_series_against_library_exponential():
    g = Grid((10, 8))
    rng = np.random.default_rng(4)
    v, _ = project(g, rng.standard_normal(g.nface) * g.interior_mask(), rtol=1e-14)
    v *= 1.5 / np.max(np.abs(v))                            # 1.5 cells per step at dt = h
    rho = rng.random(g.ncell)
    dt = g.h
    exact = spla.expm_multiply(dt * upwind.matrix(g, v), rho)
    terms, k = upwind.series(g, rho, v, dt, tol=1e-15, kmax=200)
    assert np.max(np.abs(np.sum(terms, axis=0) - exact)) <= 1e-11
    terms, k = upwind.series(g, rho, v, dt)
    assert np.max(np.abs(np.sum(terms, axis=0) - exact)) <= 1e-4
    assert 0 < k < upwind.KMAX


def test_truncation_rule_by_dense_powers():
    g = Grid((6, 5))
    rng = np.random.default_rng(5)
    v = rng.standard_normal(g.nface) * g.interior_mask()
    rho = rng.random(g.ncell)
    dt = 0.7 * g.h
    A = upwind.matrix(g, v).toarray()
    k_ref, acc = None, np.zeros(g.ncell)
    for j in range(0, 60):
        t = dt ** j / math.factorial(j) * (np.linalg.matrix_power(A, j) @ rho)
        acc += t
        if np.max(np.abs(t)) < upwind.TOL:
            k_ref = j
            break
    out = upwind.advect_up(g, rho, v, dt)
    assert upwind.advect_up_k(g, rho, v, dt) == k_ref
    assert np.allclose(out, acc, rtol=1e-12, atol=1e-14)


def test_zero_velocity_and_zero_density():
    g = Grid((6, 6))
    rho = np.linspace(0, 1, g.ncell)
    assert np.array_equal(upwind.advect_up(g, rho, np.zeros(g.nface), g.h), rho)
    assert upwind.advect_up_k(g, rho, np.zeros(g.nface), g.h) == 1
    assert upwind.advect_up_k(g, np.zeros(g.ncell), np.ones(g.nface), g.h) == 0


def _away_from_zero(g, rng, scale):
    s = rng.choice([-1.0, 1.0], g.nface)
    return s * (0.2 + rng.random(g.nface)) * scale * g.interior_mask()


@pytest.mark.parametrize("n", [(6, 5), (4, 5, 3)])
def test_dA_dv_T_by_finite_differences(n):
    g = Grid(n)
    rng = np.random.default_rng(6)
    v = _away_from_zero(g, rng, 1.0)
    x, z = rng.standard_normal(g.ncell), rng.standard_normal(g.ncell)
    d = rng.standard_normal(g.nface) * g.interior_mask()
    eps = 1e-6
    fd = (z @ (upwind.matrix(g, v + eps * d) @ x) - z @ (upwind.matrix(g, v - eps * d) @ x)) / (2 * eps)
    an = upwind.dA_dv_T(g, v, x, z) @ d
    assert abs(fd - an) <= 1e-8 * abs(fd)


@pytest.mark.parametrize("n", [(8, 6), (4, 5, 3)])
def test_adjoints_dot_product_and_finite_differences(n):
    g = Grid(n)
    rng = np.random.default_rng(7)
    v = _away_from_zero(g, rng, 0.6)
    dt = g.h
    rho = rng.random(g.ncell)
    mu = rng.standard_normal(g.ncell)
    k = upwind.advect_up_k(g, rho, v, dt)
    assert k >= 3
    x = rng.standard_normal(g.ncell)
    lhs = mu @ upwind.apply_fixed_k(g, x, v, dt, k)
    rhs = x @ upwind.advect_up_T(g, mu, rho, v, dt)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
    d = rng.standard_normal(g.nface) * g.interior_mask()
    eps = 1e-7
    fd = (mu @ upwind.apply_fixed_k(g, rho, v + eps * d, dt, k)
          - mu @ upwind.apply_fixed_k(g, rho, v - eps * d, dt, k)) / (2 * eps)
    an = upwind.advect_up_dv_T(g, mu, rho, v, dt) @ d
    assert abs(fd - an) <= 1e-7 * abs(fd)


# ------------------------------------------------------------ composites with the upwind operator
import synthetic  # noqa: E402
from oracle import ao, lbfgs, metric, step  # noqa: E402
from oracle.admm import objectives, resimulate  # noqa: E402


@pytest.mark.parametrize("n", [(8, 7), (5, 4, 6)])
def test_step_adjoint_fd_upwind(n):
    g = Grid(n)
    rng = np.random.default_rng(8)
    dt = g.h
    rho = synthetic.smooth_noise_density(n, rng, 1.0)
    v = synthetic.curl_noise_velocity(n, rng, 1.5, 1.2, 1.0)
    u = synthetic.random_faces(n, rng, 2.0)
    grn = rng.standard_normal(g.ncell)
    gvn = rng.standard_normal(g.nface) * g.interior_mask()
    g_rho, g_v, g_u = step.step_backward(g, rho, v, grn, gvn, dt, kind="upwind")

    def loss(r, vv, uu):
        rn, vn, _ = step.step_forward(g, r, vv, uu, dt, kind="upwind")
        return rn @ grn + vn @ gvn
    for _ in range(3):
        dr = rng.standard_normal(g.ncell)
        dv = rng.standard_normal(g.nface) * g.interior_mask()
        du = rng.standard_normal(g.nface) * g.interior_mask()
        e = 1e-7
        fd = (loss(rho + e * dr, v + e * dv, u + e * du) - loss(rho - e * dr, v - e * dv, u - e * du)) / (2 * e)
        ad = dr @ g_rho + dv @ g_v + du @ g_u
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1.0)


def test_ao_gradient_fd_and_monotone_upwind():
    w = synthetic.small_problem((8, 8), 4, seed=3)
    g = Grid(w["n"])
    rng = np.random.default_rng(9)
    N, dt, K = w["num_steps"], w["dt"], 2.0
    vt = np.stack([project(g, 0.4 * rng.standard_normal(g.nface) * g.interior_mask())[0] for _ in range(N)])
    vs = vt + 0.1 * np.stack([rng.standard_normal(g.nface) * g.interior_mask() for _ in range(N)])
    rho = ao.forward(g, w["rho0"], vs, dt, "upwind")
    grad_ad = ao.gradient(g, rho, w["keys"], vt, vs, K, dt, 1, kind="upwind")

    def phi(x):
        return ao.objective(g, ao.forward(g, w["rho0"], x, dt, "upwind"), w["keys"], vt, x, K, 1)
    for _ in range(3):
        d = np.stack([rng.standard_normal(g.nface) * g.interior_mask() for _ in range(N)])
        fd = (phi(vs + 1e-7 * d) - phi(vs - 1e-7 * d)) / 2e-7
        assert abs(fd - np.sum(d * grad_ad)) <= 1e-6 * max(abs(fd), 1.0)
    _, _, hist = ao.solve(g, w["rho0"], w["keys"], vt, K, dt, 1, iters=4, kind="upwind")
    assert all(hist[k + 1] <= hist[k] for k in range(len(hist) - 1))
    assert hist[-1] < hist[0]


def test_reduced_gradient_fd_upwind():
    w = synthetic.small_problem((8, 8), 3, seed=12, r=1e-2)
    g = Grid(w["n"])
    N, dt, r = w["num_steps"], w["dt"], w["r"]
    levels = metric.default_levels(w["n"])
    rng = np.random.default_rng(13)
    u = 0.05 * np.stack([synthetic.random_faces(w["n"], rng) for _ in range(N)])

    def J(x):
        rho, _ = resimulate(g, w["rho0"], x, dt, "upwind")
        return objectives(g, rho, w["keys"], x, r, levels)[0]
    rho, v = resimulate(g, w["rho0"], u, dt, "upwind")
    gr = lbfgs.gradient(g, rho, v, u, w["keys"], r, dt, levels, "upwind")
    for _ in range(3):
        d = np.stack([synthetic.random_faces(w["n"], rng) for _ in range(N)])
        fd = (J(u + 1e-6 * d) - J(u - 1e-6 * d)) / 2e-6
        assert abs(fd - np.sum(gr * d)) <= 1e-6 * max(abs(fd), 1e-12)
