"""Pins of the oracle's rotational velocity operator (Sec. 3.1 eq:NSA, the
vorticity form (curl v) x v) and of the KKT residual of eq:KKTAO built on it
(CPU): the operator does no work, its Jacobian transpose passes the
dot-product test, an irrotational field has none, solid-body rotation gives
the closed form, and F1 is the gradient of the reduced objective."""
import numpy as np
import pytest

import synthetic
from oracle import kkt, poisson, step, vorticity
from oracle.grid import Grid, grad


@pytest.fixture
def rng():
    return np.random.default_rng(61)


def _faces(g, rng, s=1.0):
    return rng.standard_normal(g.nface) * s * g.interior_mask()


@pytest.mark.parametrize("n", [(8, 6), (13, 9), (16, 16)])
def test_rotational_operator_does_no_work(n, rng):
    g = Grid(n)
    for _ in range(3):
        v = _faces(g, rng)
        a = vorticity.adv(g, v)
        assert abs(v @ a) <= 1e-13 * np.linalg.norm(v) * np.linalg.norm(a)
        assert np.all(a[g.interior_mask() == 0] == 0)


@pytest.mark.parametrize("n", [(8, 6), (13, 9)])
def test_rotational_operator_is_quadratic_and_its_transpose_is_exact(n, rng):
    g = Grid(n)
    v, y, d = _faces(g, rng), _faces(g, rng), _faces(g, rng)
    assert np.allclose(vorticity.adv(g, 2.5 * v), 6.25 * vorticity.adv(g, v), rtol=1e-13, atol=0)
    # central differences are exact for a quadratic map (up to rounding)
    e = 1e-3
    jd = (vorticity.adv(g, v + e * d) - vorticity.adv(g, v - e * d)) / (2 * e)
    assert abs(y @ jd - vorticity.adv_T(g, v, y) @ d) <= 1e-11 * abs(y @ jd)
    # the gradient of <y, Adv[v]> by central differences of the scalar
    f = lambda x: y @ vorticity.adv(g, x)
    fd = (f(v + e * d) - f(v - e * d)) / (2 * e)
    assert abs(fd - vorticity.adv_T(g, v, y) @ d) <= 1e-11 * abs(fd)


def test_irrotational_field_has_no_rotational_term(rng):
    g = Grid((12, 10))
    v = grad(g, rng.standard_normal(g.ncell), g.h) * g.interior_mask()
    assert np.max(np.abs(vorticity.node_vorticity(g, v))) <= 1e-12 * np.max(np.abs(v)) / g.h
    assert np.max(np.abs(vorticity.adv(g, v))) <= 1e-12 * np.max(np.abs(v)) ** 2 / g.h


def test_solid_rotation_closed_form():
    """v = (y - 1/2, -(x - 1/2)) on the unit square: vorticity -2 at every
    interior node and Adv_x = -2 (x - 1/2), Adv_y = -2 (y - 1/2) (that is
    (curl v) x v) at faces whose end nodes are interior."""
    n = 16
    g = Grid((n, n))
    h = g.h
    vx = np.tile(((np.arange(n) + 0.5) * h - 0.5)[:, None], (1, n + 1))
    vy = np.tile(-((np.arange(n) + 0.5) * h - 0.5)[None, :], (n + 1, 1))
    v = g.join([vx, vy]) * g.interior_mask()
    w = vorticity.node_vorticity(g, v)
    assert np.allclose(w[1:n, 1:n], -2.0, rtol=0, atol=1e-12)
    ax, ay = g.split(vorticity.adv(g, v))
    nodes = np.arange(n + 1) * h
    assert np.allclose(ax[1:n - 1, 1:n], -2 * (nodes[None, 1:n] - 0.5), rtol=0, atol=1e-12)
    assert np.allclose(ay[1:n, 1:n - 1], -2 * (nodes[1:n, None] - 0.5), rtol=0, atol=1e-12)


def test_implicit_step_satisfies_its_update():
    """The re-simulation step (fixed-point steps from Q(v + dt u)) leaves a
    residual of the implicit update far below its terms on a slow flow, and
    that residual shrinks with every extra step."""
    g = Grid((16, 16))
    rng = np.random.default_rng(62)
    dt = 0.5 * g.h
    v = synthetic.curl_noise_velocity(g.n, rng, 2.0, 0.5, dt / g.h)
    u = poisson.project(g, _faces(g, rng, 0.5))[0]
    rho = np.zeros(g.ncell)
    res = []
    for m in (1, 2, 4):
        old = step.PICARD
        step.PICARD = m
        try:
            _, vn, p = step.step_forward(g, rho, v, u, dt, velocity="vorticity")
        finally:
            step.PICARD = old
        r = ((vn - v) / dt + vorticity.adv(g, vn) - u + grad(g, p, g.h)) * g.interior_mask()
        # the projection absorbs the gradient part; what is left is the fixed-point error
        res.append(np.linalg.norm(poisson.project(g, r)[0]))
    assert res[2] < res[1] < res[0]
    assert res[2] <= 1e-3 * np.linalg.norm(vorticity.adv(g, v))


def test_kkt_rotational_f1_is_the_reduced_gradient(rng):
    """For a state whose u and p satisfy F3 = F4 = 0 given v (u the solenoidal
    part of (v_{i+1} - v_i)/dt + Adv[v_{i+1}]), F2 = F4 = 0 and <F1, dv>
    equals the directional derivative of 1/2 sum |u_i|^2 + (K/r)/2 sum |v_i - w_i|^2
    for solenoidal dv (eq:KKTAO as printed)."""
    g = Grid((8, 8))
    N, dt, kr = 4, 0.5 * g.h, 3.0
    L = kkt.Level(g, N, dt, kr, velocity="vorticity")
    vs = [np.zeros(g.nface)] + [poisson.project(g, _faces(g, rng, 0.8))[0] for _ in range(N)]
    w = np.stack([_faces(g, rng, 0.5) for _ in range(N)])

    def build(vlist):
        u = np.zeros((N, g.nface))
        p = np.zeros((N, g.ncell))
        for i in range(N):
            q = (vlist[i + 1] - vlist[i]) / dt + vorticity.adv(g, vlist[i + 1])
            u[i], phi = poisson.project(g, q)
            p[i] = -phi
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


def _colour_rows(g, colour):
    from oracle import scgs
    cells = scgs.colour_cells(g, colour)
    faces = set()
    for a in range(g.dim):
        for off in (0, 1):
            idx = cells.copy()
            idx[:, a] += off
            faces.update(scgs._face_flat(g, a, idx).tolist())
    faces = np.array(sorted(faces))
    return faces[g.interior_mask()[faces] > 0], scgs._cell_flat(g, cells)


@pytest.mark.parametrize("n", [(8, 8), (9, 6), (6, 4, 4)])
def test_local_block_is_the_exact_jacobian_at_zero_u(n, rng):
    """eq:HESS with the cell's block of dAdv/dv: at u = 0 (where the second
    derivative of Adv that eq:HESS leaves out is multiplied by zero) it is
    the exact Jacobian of the colour's rows in the colour's unknowns, so one
    pass with omega = 1 is a Newton step on those rows: what is left there
    falls with the square of the right-hand side's defect.  Without the
    block (the collapsed local matrix) it falls only linearly."""
    from oracle import scgs
    g = Grid(n)
    N, dt, kr = 4, 0.6 * g.h, 5.0
    x0 = [np.stack([_faces(g, rng, 0.8) for _ in range(N)]), rng.standard_normal((N, g.ncell)) * 0.3,
          np.zeros((N, g.nface)), rng.standard_normal((N, g.ncell)) * 0.3]
    w = np.stack([_faces(g, rng, 0.5) for _ in range(N)])
    z = [np.stack([_faces(g, rng) for _ in range(N)]), rng.standard_normal((N, g.ncell)),
         np.stack([_faces(g, rng) for _ in range(N)]), rng.standard_normal((N, g.ncell))]
    for colour in range(2 ** g.dim):
        fr, cr = _colour_rows(g, colour)
        for local_adv, order in ((True, 2.0), (False, 1.0)):
            L = kkt.Level(g, N, dt, kr, velocity="vorticity", local_adv=local_adv)
            f0 = kkt.residual_f(L, x0, w)
            left = []
            for eps in (1e-3, 1e-4):
                x = [a.copy() for a in x0]
                res = [a + eps * b for a, b in zip(f0, z)]
                scgs.smooth_colour(L, x, w, res, colour)
                r = kkt.residual(L, x, w, res)
                left.append(max(np.max(np.abs(r[0][:, fr])), np.max(np.abs(r[2][:, fr])),
                                np.max(np.abs(r[1][:, cr])), np.max(np.abs(r[3][:, cr]))))
            assert 10 ** (order - 0.15) <= left[0] / left[1] <= 10 ** (order + 0.15), (colour, local_adv, left)


# ---------------------------------------------------------------- 3D (vorticity on edges)
def test_edge_form_equals_node_form_in_2d(rng):
    """The any-dimension form (edges) and the 2D form (nodes) are two
    separate codes for the same 2D operator."""
    for n in ((9, 7), (8, 8)):
        g = Grid(n)
        v, y = _faces(g, rng), rng.standard_normal(g.nface)
        assert np.max(np.abs(vorticity.adv_nd(g, v) - vorticity._adv_2d(g, v))) <= 1e-13 * np.max(np.abs(v)) ** 2 / g.h
        assert np.max(np.abs(vorticity.adv_nd_T(g, v, y) - vorticity._adv_T_2d(g, v, y))) <= 1e-12 / g.h


@pytest.mark.parametrize("n", [(6, 5, 4), (8, 8, 8)])
def test_3d_operator_does_no_work_and_its_transpose_is_exact(n, rng):
    g = Grid(n)
    for _ in range(2):
        v, y, d = _faces(g, rng), _faces(g, rng), _faces(g, rng)
        a = vorticity.adv(g, v)
        assert abs(v @ a) <= 1e-13 * np.linalg.norm(v) * np.linalg.norm(a)
        assert np.all(a[g.interior_mask() == 0] == 0)
        assert np.allclose(vorticity.adv(g, -1.5 * v), 2.25 * a, rtol=1e-13, atol=1e-13 * np.max(np.abs(a)))
        e = 1e-3
        jd = (vorticity.adv(g, v + e * d) - vorticity.adv(g, v - e * d)) / (2 * e)
        assert abs(y @ jd - vorticity.adv_T(g, v, y) @ d) <= 1e-11 * abs(y @ jd)


def _embed(g3, c, v2x, v2y):
    """A 3D face field invariant along axis c whose components in the plane
    (p, q) of the triple (c, p, q) are the 2D field (x-role p, y-role q); the
    c component is zero."""
    n0, n1, n2 = g3.n
    parts = [np.zeros(s) for s in g3.face_shapes]
    if c == 2:                                   # p = x, q = y
        parts[0][:] = v2x[None, :, :]
        parts[1][:] = v2y[None, :, :]
    elif c == 0:                                 # p = y, q = z
        parts[1][:] = v2x[:, :, None]
        parts[2][:] = v2y[:, :, None]
    else:                                        # c = y: p = z, q = x
        parts[2][:] = v2x.T[:, None, :]
        parts[0][:] = v2y.T[:, None, :]
    return g3.join(parts)


@pytest.mark.parametrize("c", [2, 0, 1])
def test_3d_operator_on_planar_fields_is_the_2d_operator(c, rng):
    """A field that does not vary along axis c and has no c component is a 2D
    flow in every layer: the 3D operator (vorticity on edges, all three
    pairings) returns the 2D operator of each layer and nothing along c.
    Run for the three axes, this fixes the sign and orientation of every
    pairing against the 2D form and its closed forms."""
    n = (6, 5, 7)
    g3 = Grid(n)
    p, q = {2: (0, 1), 0: (1, 2), 1: (2, 0)}[c]
    g2 = Grid((n[p], n[q]), g3.h)
    v2 = _faces(g2, rng)
    v2x, v2y = g2.split(v2)
    v3 = _embed(g3, c, v2x, v2y)
    a2x, a2y = g2.split(vorticity._adv_2d(g2, v2))
    assert np.max(np.abs(vorticity.adv(g3, v3) - _embed(g3, c, a2x, a2y))) <= 1e-12 * np.max(np.abs(a2x))
    y2 = rng.standard_normal(g2.nface) * g2.interior_mask()
    y3 = _embed(g3, c, *g2.split(y2))
    t2x, t2y = g2.split(vorticity._adv_T_2d(g2, v2, y2))
    got = vorticity.adv_T(g3, v3, y3)
    # the transpose also has no c part: the c faces enter no pairing with a nonzero partner here
    assert np.max(np.abs(got - _embed(g3, c, t2x, t2y))) <= 1e-12 * np.max(np.abs(t2x))


@pytest.mark.parametrize("n", [(12, 10), (8, 6, 6)])
def test_rotational_step_adjoint_matches_fd(n, rng):
    """The adjoint of the rotational step (its fixed-point steps as computed)
    against central differences of the forward step, in rho, v and u."""
    g = Grid(n)
    dt = 0.5 * g.h
    rho = rng.standard_normal(g.ncell)
    v, _ = poisson.project(g, _faces(g, rng, 1.0))
    u = _faces(g, rng, 2.0)
    grn = rng.standard_normal(g.ncell)
    gvn = _faces(g, rng)

    def loss(r, vv, uu):
        rn, vn, _ = step.step_forward(g, r, vv, uu, dt, velocity="vorticity")
        return rn @ grn + vn @ gvn
    g_rho, g_v, g_u = step.step_backward(g, rho, v, grn, gvn, dt, velocity="vorticity", u=u)
    for _ in range(3):
        dr = rng.standard_normal(g.ncell)
        dv, du = _faces(g, rng), _faces(g, rng)
        e = 1e-6
        fd = (loss(rho + e * dr, v + e * dv, u + e * du) - loss(rho - e * dr, v - e * dv, u - e * du)) / (2 * e)
        ad = dr @ g_rho + dv @ g_v + du @ g_u
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1.0)


def _rigid_rotation(g, c, omega):
    """Solid-body rotation about axis c at rate omega, sampled on the faces:
    v_p = -omega (x_q - x_q0), v_q = omega (x_p - x_p0) for the cyclic
    triple (c, p, q); its curl is 2 omega along c and 0 along the others."""
    p, q = [(a, b) for (cc, a, b) in [(2, 0, 1), (0, 1, 2), (1, 2, 0)] if cc == c][0]
    centre = [0.37 * n for n in g.n]
    parts = []
    for a in range(g.dim):
        pos = g.face_positions(a) + 0.5                 # cell-centre offset on the axes other than a
        pos[:, a] -= 0.5                                # a-faces sit on the cell boundary along a
        f = np.zeros(len(pos))
        if a == p:
            f = -omega * g.h * (pos[:, q] - centre[q])
        elif a == q:
            f = omega * g.h * (pos[:, p] - centre[p])
        parts.append(f.reshape(g.face_shapes[a]))
    return g.join(parts)


@pytest.mark.parametrize("n,c", [((10, 8), 2), ((7, 6, 5), 0), ((7, 6, 5), 1), ((7, 6, 5), 2)])
def test_edge_vorticity_of_rigid_rotation_and_gradients(n, c, rng):
    """The edge vorticity against closed forms: a solid-body rotation at rate
    omega has curl 2 omega along its axis and none across it (every interior
    edge, exactly for a linear field), and a discrete gradient has none."""
    g = Grid(n)
    omega = 1.7
    v = _rigid_rotation(g, c, omega)
    for cc in ((2,) if g.dim == 2 else (0, 1, 2)):
        w = vorticity.edge_vorticity(g, v, cc)
        inner = w[:, 1:-1, 1:-1]
        want = 2 * omega if cc == c else 0.0
        assert np.max(np.abs(inner - want)) <= 1e-12 * 2 * omega, cc
        assert np.all(w[:, 0, :] == 0) and np.all(w[:, -1, :] == 0)
        assert np.all(w[:, :, 0] == 0) and np.all(w[:, :, -1] == 0)
        gphi = grad(g, rng.standard_normal(g.ncell))
        assert np.max(np.abs(vorticity.edge_vorticity(g, gphi, cc))) <= 1e-12 * np.max(np.abs(gphi)) / g.h
