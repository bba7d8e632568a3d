"""Pins of the FP64 oracle against things other than itself: closed forms,
library routines, special cases, adjoint/finite-difference identities and
brute force on tiny grids.  CPU only."""
import numpy as np
import pytest
import scipy.fft
from scipy import ndimage

import synthetic
from oracle import advect, ao, kkt, metric, poisson, scgs, stfas, step, transfer
from oracle.grid import Grid, div, grad

GRIDS = [(8, 6), (6, 4, 5)]


def rand_faces(g, rng, s=1.0):
    return synthetic.random_faces(g.n, rng, s)


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


# ---------------------------------------------------------------- grid, Q
@pytest.mark.parametrize("n", GRIDS)
def test_grad_is_minus_div_transpose(n):
    g = Grid(n)
    D = np.stack([div(g, e) for e in np.eye(g.nface)], axis=1)         # ncell x nface
    G = np.stack([grad(g, e) for e in np.eye(g.ncell)], axis=1)        # nface x ncell
    m = g.interior_mask().astype(bool)
    assert np.allclose(G[m], -D.T[m], atol=0, rtol=0)
    assert np.all(G[~m] == 0)
    # Neumann Laplacian rows sum to zero (constants are its null space)
    L = D @ G
    assert np.allclose(L.sum(axis=1), 0.0, atol=1e-9)


@pytest.mark.parametrize("n", [(16, 12), (8, 6, 10)])
def test_poisson_matches_dct_closed_form(n, rng):
    """The DCT-II diagonalises the Neumann Laplacian, eigenvalues
    -(4/h^2) sum_a sin^2(pi k_a / (2 n_a))."""
    g = Grid(n)
    b = rng.standard_normal(g.ncell)
    b -= b.mean()
    bh = scipy.fft.dctn(b.reshape(g.cell_shape), type=2, norm="ortho")
    lam = np.zeros(g.cell_shape)
    for a in range(g.dim):
        k = np.arange(g.n[a])
        shape = [1] * g.dim
        shape[g.npax(a)] = g.n[a]
        lam = lam + np.sin(np.pi * k / (2.0 * g.n[a])).reshape(shape) ** 2
    lam = -(4.0 / g.h ** 2) * lam
    lam.flat[0] = 1.0
    ph = bh / lam
    ph.flat[0] = 0.0
    phi_ref = scipy.fft.idctn(ph, type=2, norm="ortho").ravel()
    phi = poisson.solve_neumann(g, b)
    assert rel(phi, phi_ref) < 1e-11
    assert abs(phi.mean()) < 1e-12 * np.abs(phi).max()


@pytest.mark.parametrize("n", GRIDS + [(32, 32)])
def test_projection_invariants(n, rng):
    g = Grid(n)
    w = rand_faces(g, rng)
    v, phi = poisson.project(g, w)
    assert np.max(np.abs(div(g, v))) * g.h / np.max(np.abs(w)) <= 1e-12
    assert np.all(v[g.interior_mask() == 0] == 0)
    v2, _ = poisson.project(g, v)
    assert rel(v2, v) < 1e-12                                           # Q^2 = Q
    y = rand_faces(g, rng)
    qy, _ = poisson.project(g, y)
    assert abs(v @ y - w @ qy) <= 1e-12 * np.linalg.norm(w) * np.linalg.norm(y)   # Q^T = Q
    gp = grad(g, rng.standard_normal(g.ncell))
    qg, _ = poisson.project(g, gp)
    assert np.linalg.norm(qg) <= 1e-11 * np.linalg.norm(gp)             # Q G = 0
    c = synthetic.curl_noise_velocity(g.n, rng, sigma=1.0)
    qc, _ = poisson.project(g, c)
    assert rel(qc, c) < 1e-12                                           # Q curl = curl


# ---------------------------------------------------------------- SL scalar
@pytest.mark.parametrize("n", GRIDS)
def test_sl_zero_velocity_is_identity(n, rng):
    g = Grid(n)
    rho = rng.standard_normal(g.ncell)
    assert np.array_equal(advect.advect_scalar(g, rho, np.zeros(g.nface), 0.1), rho)
    assert np.array_equal(advect.self_advect(g, rand_faces(g, rng) * 0, 0.1), np.zeros(g.nface))
    v = rand_faces(g, rng)
    assert rel(advect.self_advect(g, v, 0.0), v) == 0.0


def _uniform_x(g, value):
    v = np.zeros(g.nface)
    parts = g.split(v)
    parts[0][g.sl_along(0, 1, g.n[0])] = value
    return v


@pytest.mark.parametrize("shift", [1.0, 2.0, 0.3, 1.75])
def test_sl_uniform_shift_closed_form(shift, rng):
    """Uniform interior velocity: interior cells read rho at X - shift exactly
    (integer shift) or its linear mix (fractional shift)."""
    g = Grid((12, 7))
    dt = 0.05
    rho = rng.standard_normal(g.cell_shape)
    v = _uniform_x(g, shift * g.h / dt)
    out = advect.advect_scalar(g, rho.ravel(), v, dt).reshape(g.cell_shape)
    k = int(np.floor(shift))
    t = shift - k
    for x in range(int(np.ceil(shift)) + 1, g.n[0] - 1):
        ref = (1 - t) * rho[:, x - k] + (t * rho[:, x - k - 1] if t > 0 else 0.0)
        assert np.allclose(out[:, x], ref, rtol=0, atol=1e-13)


def test_sl_is_convex_combination(rng):
    for n in GRIDS:
        g = Grid(n)
        rho = rng.standard_normal(g.ncell)
        out = advect.advect_scalar(g, rho, rand_faces(g, rng, 3.0), 0.7)
        assert out.min() >= rho.min() - 1e-14 and out.max() <= rho.max() + 1e-14


def _fd(f, x, dx, eps):
    return (f(x + eps * dx) - f(x - eps * dx)) / (2 * eps)


@pytest.mark.parametrize("n", GRIDS)
def test_sl_adjoints_dot_product_and_fd(n, rng):
    g = Grid(n)
    dt = 0.37 * g.h
    rho = rng.standard_normal(g.ncell)
    v = rand_faces(g, rng, 1.3)
    mu = rng.standard_normal(g.ncell)
    # W is linear in rho: <W x, y> = <x, W^T y>
    x = rng.standard_normal(g.ncell)
    lhs = advect.advect_scalar(g, x, v, dt) @ mu
    rhs = x @ advect.advect_scalar_T(g, mu, v, dt)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(x) * np.linalg.norm(mu) * 4
    # dA/dv against central differences (foot points away from grid lines)
    for _ in range(4):
        dv = rand_faces(g, rng)
        fd = _fd(lambda vv: advect.advect_scalar(g, rho, vv, dt), v, dv, 1e-7) @ mu
        ad = dv @ advect.advect_scalar_dv_T(g, mu, rho, v, dt)
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1.0)


@pytest.mark.parametrize("n", GRIDS)
def test_self_advection_jacobian_transpose_fd(n, rng):
    g = Grid(n)
    dt = 0.41 * g.h
    v = rand_faces(g, rng, 1.1)
    y = rand_faces(g, rng)
    jty = advect.self_advect_T(g, v, y, dt)
    assert np.all(jty[g.interior_mask() == 0] == 0)
    for _ in range(4):
        dv = rand_faces(g, rng)
        fd = _fd(lambda vv: advect.self_advect(g, vv, dt), v, dv, 1e-7) @ y
        assert abs(fd - dv @ jty) <= 1e-6 * max(abs(fd), 1.0)


def _torch_sl_2d(rho, vx, vy, cfl):
    """Independent plain-torch bilinear semi-Lagrangian step (floor/clamp)."""
    import torch
    n1, n0 = rho.shape
    vbx = 0.5 * (vx[:, :-1] + vx[:, 1:])
    vby = 0.5 * (vy[:-1, :] + vy[1:, :])
    X = torch.arange(n0, dtype=torch.float64).expand(n1, n0)
    Yy = torch.arange(n1, dtype=torch.float64).unsqueeze(1).expand(n1, n0)
    px = torch.clamp(X - cfl * vbx, 0.0, n0 - 1.0)
    py = torch.clamp(Yy - cfl * vby, 0.0, n1 - 1.0)
    ix = torch.clamp(torch.floor(px).detach(), max=n0 - 2).long()
    iy = torch.clamp(torch.floor(py).detach(), max=n1 - 2).long()
    tx = px - ix
    ty = py - iy
    flat = rho.reshape(-1)

    def at(j, i):
        return flat[j * n0 + i]
    return ((1 - tx) * (1 - ty) * at(iy, ix) + tx * (1 - ty) * at(iy, ix + 1)
            + (1 - tx) * ty * at(iy + 1, ix) + tx * ty * at(iy + 1, ix + 1))


@pytest.mark.parametrize("zero_v", [True, False])
def test_sl_derivative_convention_matches_autograd(zero_v, rng):
    import torch
    g = Grid((7, 5))
    dt = 0.6 * g.h
    rho = rng.standard_normal(g.ncell)
    v = np.zeros(g.nface) if zero_v else rand_faces(g, rng, 1.7)
    mu = rng.standard_normal(g.ncell)
    vx, vy = [torch.tensor(p.copy(), requires_grad=True) for p in g.split(v)]
    rt = torch.tensor(rho.reshape(g.cell_shape), requires_grad=True)
    out = _torch_sl_2d(rt, vx, vy, dt / g.h)
    assert np.allclose(out.detach().numpy().ravel(), advect.advect_scalar(g, rho, v, dt), atol=1e-14)
    (out.reshape(-1) @ torch.tensor(mu)).backward()
    gv = g.join([vx.grad.numpy(), vy.grad.numpy()]) * g.interior_mask()
    assert np.allclose(gv, advect.advect_scalar_dv_T(g, mu, rho, v, dt), atol=1e-13)
    assert np.allclose(rt.grad.numpy().ravel(), advect.advect_scalar_T(g, mu, v, dt), atol=1e-13)


# ---------------------------------------------------------------- metric
@pytest.mark.parametrize("sigma", [1.0, 2.0, 4.0])
def test_blur_matches_scipy_gaussian(sigma, rng):
    g = Grid((24, 20))
    e = rng.standard_normal(g.ncell)
    ref = ndimage.gaussian_filter(e.reshape(g.cell_shape), sigma, mode="constant", truncate=3.0)
    assert rel(metric.blur(g, e, sigma), ref) < 1e-13
    assert abs(metric.gauss_taps(sigma).sum() - 1.0) < 1e-15


def test_metric_spd_and_identity(rng):
    g = Grid((10, 8))
    C = np.stack([metric.apply_metric(g, e, 3) for e in np.eye(g.ncell)], axis=1)
    assert np.allclose(C, C.T, atol=1e-14)
    assert np.linalg.eigvalsh(C).min() >= 1.0 - 1e-12
    e = rng.standard_normal(g.ncell)
    assert np.array_equal(metric.apply_metric(g, e, 0), e)
    assert metric.default_levels((32, 32)) == 3 and metric.default_levels((128, 128)) == 5


# ---------------------------------------------------------------- step
@pytest.mark.parametrize("n", GRIDS)
def test_step_adjoint_matches_fd(n, rng):
    g = Grid(n)
    dt = 0.5 * g.h
    rho = rng.standard_normal(g.ncell)
    v, _ = poisson.project(g, rand_faces(g, rng, 1.2))
    u = rand_faces(g, rng, 3.0)
    grn = rng.standard_normal(g.ncell)
    gvn = rand_faces(g, rng)

    def loss(r, vv, uu):
        rn, vn, _ = step.step_forward(g, r, vv, uu, dt)
        return rn @ grn + vn @ gvn
    g_rho, g_v, g_u = step.step_backward(g, rho, v, grn, gvn, dt)
    for _ in range(3):
        dr = rng.standard_normal(g.ncell)
        dv = rand_faces(g, rng)
        du = rand_faces(g, rng)
        e = 1e-6
        fd = (loss(rho + e * dr, v + e * dv, u + e * du) - loss(rho - e * dr, v - e * dv, u - e * du)) / (2 * e)
        ad = dr @ g_rho + dv @ g_v + du @ g_u
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1.0)


@pytest.mark.parametrize("n", [(12, 10), (8, 6, 7)])
def test_step_adjoint_fd_large_cfl(n, rng):
    """Smooth divergence-free velocity moving up to 2 cells per step (foot
    points leave the cell and the domain)."""
    g = Grid(n)
    dt = g.h
    rho = synthetic.smooth_noise_density(n, rng, 1.0)
    v = synthetic.curl_noise_velocity(n, rng, 1.5, 2.0, 1.0)
    u = synthetic.random_faces(n, rng, 2.0)
    grn = rng.standard_normal(g.ncell)
    gvn = rand_faces(g, rng)
    g_rho, g_v, g_u = step.step_backward(g, rho, v, grn, gvn, dt)

    def loss(vv):
        rn, vn, _ = step.step_forward(g, rho, vv, u, dt)
        return rn @ grn + vn @ gvn
    for _ in range(4):
        dv = rand_faces(g, rng)
        fd = (loss(v + 1e-7 * dv) - loss(v - 1e-7 * dv)) / 2e-7
        assert abs(fd - dv @ g_v) <= 1e-6 * abs(fd)


# ---------------------------------------------------------------- AO
def test_ao_gradient_fd_and_monotone(rng):
    w = synthetic.small_problem((8, 8), 4, seed=3)
    g = Grid(w["n"])
    N, dt, K = w["num_steps"], w["dt"], 2.0
    vt = np.stack([poisson.project(g, rand_faces(g, rng, 0.4))[0] for _ in range(N)])
    vs = vt + 0.1 * np.stack([rand_faces(g, rng) for _ in range(N)])
    rho = ao.forward(g, w["rho0"], vs, dt)
    grad_ad = ao.gradient(g, rho, w["keys"], vt, vs, K, dt, 1)

    def phi(x):
        return ao.objective(g, ao.forward(g, w["rho0"], x, dt), w["keys"], vt, x, K, 1)
    for _ in range(3):
        d = np.stack([rand_faces(g, rng) for _ in range(N)])
        fd = (phi(vs + 1e-7 * d) - phi(vs - 1e-7 * d)) / 2e-7
        assert abs(fd - np.sum(d * grad_ad)) <= 1e-6 * max(abs(fd), 1.0)
    _, _, hist = ao.solve(g, w["rho0"], w["keys"], vt, K, dt, 1, iters=4)
    assert all(hist[k + 1] <= hist[k] for k in range(len(hist) - 1))
    assert hist[-1] < hist[0]


# ---------------------------------------------------------------- KKT
@pytest.mark.parametrize("n", [(8, 8), (4, 6, 4)])
def test_kkt_feasible_trajectory_and_f1_gradient(n, rng):
    g = Grid(n)
    N, dt, kr = 4, 0.5 * g.h, 3.0
    L = kkt.Level(g, N, dt, kr)
    vs = [np.zeros(g.nface)] + [poisson.project(g, rand_faces(g, rng, 0.8))[0] for _ in range(N)]
    w = np.stack([rand_faces(g, rng, 0.5) for _ in range(N)])

    def build(vlist):
        u = np.zeros((N, g.nface))
        p = np.zeros((N, g.ncell))
        for i in range(N):
            s = advect.self_advect(g, vlist[i], dt) if i > 0 else np.zeros(g.nface)
            q = (vlist[i + 1] - s) / dt
            u[i], phi = poisson.project(g, q)
            p[i] = -phi                    # F3: (v'-S)/dt - u + G p = G phi + G p = 0
        return [np.stack(vlist[1:]), np.zeros((N, g.ncell)), u, p]

    x = build(vs)
    f = kkt.residual_f(L, x, w)
    scale = np.max(np.abs(x[2]))
    assert np.max(np.abs(f[1])) < 1e-11 * scale and np.max(np.abs(f[3])) < 1e-11 * scale
    assert np.max(np.abs(f[2])) < 1e-10 * scale

    def jred(vlist):
        xx = build(vlist)
        val = 0.5 * np.sum(xx[2] ** 2)
        for i in range(1, N):
            val += 0.5 * kr * np.sum((vlist[i] - w[i]) ** 2)
        return val
    for _ in range(3):
        dvs = [np.zeros(g.nface)] + [synthetic.curl_noise_velocity(g.n, rng, 1.0) for _ in range(N)]
        e = 1e-6
        fd = (jred([a + e * b for a, b in zip(vs, dvs)]) - jred([a - e * b for a, b in zip(vs, dvs)])) / (2 * e)
        ad = sum(f[0][j] @ dvs[j + 1] for j in range(N))
        assert abs(fd - ad) <= 1e-5 * max(abs(fd), 1.0)


def _random_state(g, N, rng, s=0.3):
    return [np.stack([rand_faces(g, rng, s) for _ in range(N)]), rng.standard_normal((N, g.ncell)) * s,
            np.stack([rand_faces(g, rng, s) for _ in range(N)]), rng.standard_normal((N, g.ncell)) * s]


def _colour_rows(g, colour):
    cells = scgs.colour_cells(g, colour)
    faces = set()
    for a in range(g.dim):
        for off in (0, 1):
            idx = cells.copy()
            idx[:, a] += off
            faces.update(scgs._face_flat(g, a, idx).tolist())
    return np.array(sorted(faces)), scgs._cell_flat(g, cells)


@pytest.mark.parametrize("n", [(8, 8), (4, 6, 4)])
def test_scgs_local_solve_is_exact_without_advection(n, rng):
    """With S = I the local Jacobian is exact: after a colour pass the
    residual vanishes on every row owned by that colour's cells."""
    g = Grid(n)
    N = 5
    L = kkt.Level(g, N, 0.3 * g.h, 7.0, advect=False)
    x = _random_state(g, N, rng)
    w = np.stack([rand_faces(g, rng) for _ in range(N)])
    res = _random_state(g, N, rng, 1.0)
    m = g.interior_mask().astype(bool)
    for colour in range(2 ** g.dim):
        scgs.smooth_colour(L, x, w, res, colour)
        r = kkt.residual(L, x, w, res)
        fr, cr = _colour_rows(g, colour)
        fr = fr[m[fr]]
        scale = max(np.max(np.abs(a)) for a in res)
        for k, rows in ((0, fr), (2, fr), (1, cr), (3, cr)):
            assert np.max(np.abs(r[k][:, rows])) < 1e-9 * scale, (colour, k)


@pytest.mark.parametrize("lm", [0.0, 1.0, 3.0])
def test_stfas_linear_case_matches_dense_solve(rng, lm):
    """S = I makes f affine; V-cycles converge to the dense solution, also
    with the Levenberg-Marquardt perturbation of the smoother's local matrix
    (it changes the smoother, not the equations being solved)."""
    g = Grid((8, 8))
    N, dt, kr = 3, 0.5 * g.h, 4.0
    H = stfas.Hierarchy(g, N, dt, kr, advect=False, lm=lm)
    L = H.levels[0]
    w = np.stack([poisson.project(g, rand_faces(g, rng))[0] for _ in range(N)])
    sizes = [N * g.nface, N * g.ncell, N * g.nface, N * g.ncell]
    m = g.interior_mask().astype(bool)
    keep = np.concatenate([np.tile(m, N), np.ones(N * g.ncell, bool), np.tile(m, N), np.ones(N * g.ncell, bool)])

    def unpack(z):
        out, o = [], 0
        for k, s in enumerate(sizes):
            out.append(z[o:o + s].reshape(N, -1))
            o += s
        return out

    def fvec(z):
        return np.concatenate([a.ravel() for a in kkt.residual_f(L, unpack(z), w)])
    tot = sum(sizes)
    b = fvec(np.zeros(tot))
    cols = np.flatnonzero(keep)
    A = np.stack([fvec(np.eye(tot)[c]) - b for c in cols], axis=1)[keep]
    # pressures are defined up to a constant per slab: least squares picks one
    z = np.zeros(tot)
    z[cols] = np.linalg.lstsq(A, -b[keep], rcond=None)[0]
    xref = unpack(z)
    x = kkt.zeros_state(L)
    # the perturbation damps the smoother: more cycles to the same solution
    n_vc, hist = stfas.nso(H, x, w, eps=1e-13, max_vcycles=60 if lm <= 1 else 200)
    assert hist[-1] <= 1e-12 * hist[0]
    assert rel(x[0], xref[0]) < 1e-9 and rel(x[2], xref[2]) < 1e-9
    # at a fixed N the velocities satisfy the closed-form recurrence in time:
    # (K/r)(v_i - w_i) + (2 v_i - v_{i-1} - v_{i+1})/dt^2 = 0 for solenoidal w
    v = np.vstack([np.zeros(g.nface), x[0]])
    for i in range(1, N):
        lhs = kr * (v[i] - w[i]) + (2 * v[i] - v[i - 1] - v[i + 1]) / dt ** 2
        assert np.max(np.abs(lhs[m])) < 1e-8 * np.max(np.abs(kr * w))


# ---------------------------------------------------------------- transfers
@pytest.mark.parametrize("n", [(8, 12), (8, 4, 8)])
def test_transfers(n, rng):
    g = Grid(n)
    T = transfer.Transfer(g)
    c = T.coarse
    # P reproduces linear functions of the sample position in the interior
    coef = rng.standard_normal(g.dim)
    pc = c.cell_positions() @ coef
    pf = T.prolong_cells(pc)
    expect = ((g.cell_positions() + 0.5) / 2.0 - 0.5) @ coef
    inner = np.all((g.cell_positions() >= 1) & (g.cell_positions() <= np.array(g.n) - 2), axis=1)
    assert np.allclose(pf[inner], expect[inner], atol=1e-12)
    # R = 2^-d P^T (dot product) and R 1 = 1
    xf = rng.standard_normal(g.ncell)
    yc = rng.standard_normal(c.ncell)
    assert abs(T.restrict_cells(xf) @ yc - 2.0 ** -g.dim * (xf @ T.prolong_cells(yc))) < 1e-12 * 10
    assert np.allclose(T.restrict_cells(np.ones(g.ncell)), 1.0, atol=1e-14)
    xf = rand_faces(g, rng)
    yc = rand_faces(c, rng)
    assert abs(T.restrict_faces(xf) @ yc - 2.0 ** -g.dim * (xf @ T.prolong_faces(yc))) < 1e-12 * 10
    rf = T.restrict_faces(g.interior_mask())
    assert np.allclose(rf[c.interior_mask() == 1], 1.0, atol=1e-14)
    assert np.all(T.prolong_faces(yc)[g.interior_mask() == 0] == 0)


# ---------------------------------------------------------------- FAS with advection on
def _kkt_state(g, N, rng, s):
    m = g.interior_mask()
    return [np.stack([s * m * rand_faces(g, rng) for _ in range(N)]),
            s * rng.standard_normal((N, g.ncell)),
            np.stack([s * m * rand_faces(g, rng) for _ in range(N)]),
            s * rng.standard_normal((N, g.ncell))]


@pytest.mark.parametrize("n", [(8, 8), (8, 8, 8)])
def test_fas_vcycle_fixed_point_with_advection(n, rng):
    """Alg:STFAS on the nonlinear (advecting) system: with res = f(x*) the
    state x* solves f(x) = res exactly, so a consistent FAS cycle returns it
    unchanged: every local SCGS correction sees a zero residual, and the
    coarse problem f_2h(x_2h) = f_2h(R x*) + R 0 is solved by R x*, whose
    prolonged correction cancels.  A smoother whose local residual differs
    from f, or a coarse right-hand side without f_2h(R x), moves x."""
    g = Grid(n)
    N, dt, kr = 3, g.h, 4.0
    H = stfas.Hierarchy(g, N, dt, kr, advect=True, omega=0.7)
    assert len(H.levels) == 2
    L = H.levels[0]
    xs = _kkt_state(g, N, rng, 0.5)
    w = np.stack([rand_faces(g, rng) for _ in range(N)])
    res = kkt.residual_f(L, xs, w)
    x = [a.copy() for a in xs]
    stfas.vcycle(H, 0, x, H.targets(w), res)
    for k in range(4):
        assert rel(x[k], xs[k]) < 1e-12, k


def test_fas_vcycle_contracts_near_solution():
    """Near an exact solution of f(x) = res (a perturbation small enough that
    no backtrace crosses a lattice line) the cycle converges linearly
    (Sec. 4.3): each of three V-cycles reduces |f(x) - res| at least 2x, the
    three together at least 20x.  On this rough random state (CFL 1) the
    per-cycle factors over twelve seeds lie between 0.12 and 0.43."""
    rng = np.random.default_rng(3)
    g = Grid((8, 8))
    N, dt, kr = 3, g.h, 4.0
    H = stfas.Hierarchy(g, N, dt, kr, advect=True, omega=0.7)
    L = H.levels[0]
    xs = _kkt_state(g, N, rng, 0.5)
    w = np.stack([rand_faces(g, rng) for _ in range(N)])
    res = kkt.residual_f(L, xs, w)
    dx = _kkt_state(g, N, rng, 1e-7)
    x = [xs[k] + dx[k] for k in range(4)]
    hist = [kkt.inf_norm(kkt.residual(L, x, w, res))]
    for _ in range(3):
        stfas.vcycle(H, 0, x, H.targets(w), res)
        hist.append(kkt.inf_norm(kkt.residual(L, x, w, res)))
    assert all(hist[i + 1] <= 0.5 * hist[i] for i in range(3)), hist
    assert hist[3] <= 0.05 * hist[0], hist
