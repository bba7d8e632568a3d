"""The paper's velocity self-advection in rotational form (Sec. 3.1 eq:NSA:
Adv[v] discretises the quadratic operator (curl v) x v, the gradient part of
(v . grad) v going into the kinetic pressure), on the 2D MAC grid and, with
the vorticity on the grid's edges, on the 3D one (adv_nd below).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.

Reading (the paper cites a structure-preserving discretisation, whose
defining property is that the operator does no work, but does not print the
stencil):

  * vorticity at the grid nodes (cell corners), the circulation around the
    node's dual cell:  w_n = (v_y right - v_y left - v_x above + v_x below)/h
    at interior nodes, w_n = 0 on the walls;
  * at node n the sums of the two incident x-faces and of the two incident
    y-faces, Sx_n and Sy_n (wall faces hold zero);
  * A_x(f) = -1/4 sum over the two end nodes n of the x-face f of w_n Sy_n,
    A_y(g) = +1/4 sum over the two end nodes n of the y-face g of w_n Sx_n,
    zero on wall faces.

Every (x-face, y-face) pair meeting at a node enters A_x and A_y with the
same weight and opposite sign, so sum_f v_f A_f(v) = 0 for every v: the
discrete operator does no work, as (curl v) x v does not.  A is bilinear in
(w(v), v); its Jacobian transpose is formed from the same node sums.
"""
import numpy as np

from .grid import Grid


def _split2(g: Grid, f):
    assert g.dim == 2, "the rotational operator is built for 2D grids"
    vx, vy = g.split(np.asarray(f, dtype=np.float64))
    return vx, vy          # vx[j, I]: x-face I of row j; vy[J, i]: y-face J of column i


def node_vorticity(g: Grid, v):
    """w_n at the (n1 + 1, n0 + 1) nodes; zero on the walls."""
    vx, vy = _split2(g, v)
    n0, n1 = g.n
    w = np.zeros((n1 + 1, n0 + 1))
    w[1:n1, 1:n0] = (vy[1:n1, 1:n0] - vy[1:n1, 0:n0 - 1] - vx[1:n1, 1:n0] + vx[0:n1 - 1, 1:n0]) / g.h
    return w


def node_sums(g: Grid, f):
    """(Sx, Sy): per node the sum of its two incident x-faces and of its two
    incident y-faces."""
    fx, fy = _split2(g, f)
    n0, n1 = g.n
    sx = np.zeros((n1 + 1, n0 + 1))
    sx[:n1, :] += fx
    sx[1:, :] += fx
    sy = np.zeros((n1 + 1, n0 + 1))
    sy[:, :n0] += fy
    sy[:, 1:] += fy
    return sx, sy


def adv(g: Grid, v):
    """Adv[v] on the faces (zero on walls); 3D grids take adv_nd."""
    return adv_nd(g, v) if g.dim == 3 else _adv_2d(g, v)


def adv_T(g: Grid, v, y):
    """J_Adv(v)^T y: the gradient in v of <y, Adv[v]>; 3D grids take adv_nd_T."""
    return adv_nd_T(g, v, y) if g.dim == 3 else _adv_T_2d(g, v, y)


def _adv_2d(g: Grid, v):
    """Adv[v] on a 2D grid, from the node quantities."""
    n0, n1 = g.n
    w = node_vorticity(g, v)
    sx, sy = node_sums(g, v)
    ax = -0.25 * ((w * sy)[0:n1, :] + (w * sy)[1:n1 + 1, :])
    ay = 0.25 * ((w * sx)[:, 0:n0] + (w * sx)[:, 1:n0 + 1])
    return g.join([ax, ay]) * g.interior_mask()


def _adv_T_2d(g: Grid, v, y):
    """J_Adv(v)^T y on a 2D grid, from the node quantities."""
    n0, n1 = g.n
    h = g.h
    y = np.asarray(y, dtype=np.float64) * g.interior_mask()
    w = node_vorticity(g, v)
    sx, sy = node_sums(g, v)
    yx, yy = node_sums(g, y)
    # <y, Adv[v]> = 1/4 sum_n w_n (Sx_n Yy_n - Sy_n Yx_n)
    P = np.zeros((n1 + 1, n0 + 1))
    P[1:n1, 1:n0] = 0.25 * (sx * yy - sy * yx)[1:n1, 1:n0]
    # through w_n (interior nodes): dw/dvx[j, I] = -1/h at node (I, j), +1/h at (I, j + 1);
    # dw/dvy[J, i] = +1/h at node (i, J), -1/h at (i + 1, J)
    gx = (P[1:n1 + 1, :] - P[0:n1, :]) / h
    gy = (P[:, 0:n0] - P[:, 1:n0 + 1]) / h
    # through the node sums: Sx_n gains v_f for the x-faces at n, Sy_n the y-faces
    gx = gx + 0.25 * ((w * yy)[0:n1, :] + (w * yy)[1:n1 + 1, :])
    gy = gy - 0.25 * ((w * yx)[:, 0:n0] + (w * yx)[:, 1:n0 + 1])
    return g.join([gx, gy]) * g.interior_mask()


# ---------------------------------------------------------------- any dimension
# The same operator on the edges of a 2D or 3D grid.  For each cyclic triple of
# axes (c, a, b) = (z, x, y), (x, y, z), (y, z, x) (in 2D only the first, with
# c a single layer) the c-directed edges sit at a-nodes, b-nodes and c-cells
# and carry
#   w_c = (D_a v_b - D_b v_a)/h    (the circulation around the edge; zero on walls),
#   S_a, S_b = the sums of the two a-faces and of the two b-faces at the edge,
# and add -1/4 w_c S_b to each of the two a-faces and +1/4 w_c S_a to each of the
# two b-faces at the edge.  This is (curl v) x v: its x part is w_y v_z - w_z v_y.
# Every pair of faces meeting at an edge enters both components with the same
# weight and opposite signs, so sum_f v_f Adv_f(v) = 0 in 3D as in 2D.  In 2D the
# z-edges are the grid nodes and the result is adv() above.

_TRIPLES = {2: [(2, 0, 1)], 3: [(2, 0, 1), (0, 1, 2), (1, 2, 0)]}


_NPAX = {0: 2, 1: 1, 2: 0}                # spatial axis -> NumPy axis of a 3-axis array


def _canon(g: Grid, arr, a, b, c):
    """A face or edge array with NumPy axes (c, b, a); a 2D array gains a
    single c layer."""
    if g.dim == 2:
        arr = arr[None]
    return np.transpose(arr, (_NPAX[c], _NPAX[b], _NPAX[a]))


def _uncanon(g: Grid, arr, a, b, c):
    """Inverse of _canon."""
    out = np.transpose(arr, np.argsort((_NPAX[c], _NPAX[b], _NPAX[a])))
    return out[0] if g.dim == 2 else out


def _edge_terms(g: Grid, f, a, b, c):
    """(Sa, Sb, Da f_b - Db f_a) on the c-edges, axes (c, b-node, a-node)."""
    parts = g.split(np.asarray(f, dtype=np.float64))
    fa = _canon(g, parts[a], a, b, c)            # (c, b-cells, a-nodes)
    fb = _canon(g, parts[b], a, b, c)            # (c, b-nodes, a-cells)
    pa = np.pad(fa, ((0, 0), (1, 1), (0, 0)))
    pb = np.pad(fb, ((0, 0), (0, 0), (1, 1)))
    sa = pa[:, :-1, :] + pa[:, 1:, :]
    sb = pb[:, :, :-1] + pb[:, :, 1:]
    curl = (pb[:, :, 1:] - pb[:, :, :-1]) - (pa[:, 1:, :] - pa[:, :-1, :])
    return sa, sb, curl


def _interior_edges(shape):
    m = np.zeros(shape)
    m[:, 1:-1, 1:-1] = 1.0
    return m


def edge_vorticity(g: Grid, v, c):
    """w_c on the c-edges, axes (c-cells, b-nodes, a-nodes) of its triple."""
    a, b = [(x, y) for (cc, x, y) in _TRIPLES[3] if cc == c][0]
    _, _, curl = _edge_terms(g, v, a, b, c)
    return curl / g.h * _interior_edges(curl.shape)


def adv_nd(g: Grid, v):
    """Adv[v] on the faces (zero on walls), 2D or 3D."""
    parts = [np.zeros(s) for s in g.face_shapes]
    for (c, a, b) in _TRIPLES[g.dim]:
        sa, sb, curl = _edge_terms(g, v, a, b, c)
        w = curl / g.h * _interior_edges(curl.shape)
        ea, eb = w * sb, w * sa
        parts[a] += _uncanon(g, -0.25 * (ea[:, :-1, :] + ea[:, 1:, :]), a, b, c)
        parts[b] += _uncanon(g, 0.25 * (eb[:, :, :-1] + eb[:, :, 1:]), a, b, c)
    return g.join(parts) * g.interior_mask()


def adv_nd_T(g: Grid, v, y):
    """J_Adv(v)^T y, 2D or 3D: the gradient in v of
    <y, Adv[v]> = sum over edges of w_c (S_a Y_b - S_b Y_a)/4."""
    y = np.asarray(y, dtype=np.float64) * g.interior_mask()
    parts = [np.zeros(s) for s in g.face_shapes]
    for (c, a, b) in _TRIPLES[g.dim]:
        sa, sb, curl = _edge_terms(g, v, a, b, c)
        ya, yb, _ = _edge_terms(g, y, a, b, c)
        m = _interior_edges(curl.shape)
        w = curl / g.h * m
        P = 0.25 * (sa * yb - sb * ya) * m / g.h       # d<y, Adv>/d(curl) on interior edges
        # through the curl (D_a f_b - D_b f_a): the b-face of a-cell A enters
        # D_a f_b at the edges A (+1) and A + 1 (-1); the a-face of b-cell B
        # enters D_b f_a at the edges B (+1) and B + 1 (-1), with a minus sign
        ga = -(P[:, :-1, :] - P[:, 1:, :])
        gb = P[:, :, :-1] - P[:, :, 1:]
        # through the sums: dP/dS_a = Y_b / 4 and dP/dS_b = -Y_a / 4, times w
        qa = 0.25 * w * yb
        qb = -0.25 * w * ya
        ga = ga + qa[:, :-1, :] + qa[:, 1:, :]
        gb = gb + qb[:, :, :-1] + qb[:, :, 1:]
        parts[a] += _uncanon(g, ga, a, b, c)
        parts[b] += _uncanon(g, gb, a, b, c)
    return g.join(parts) * g.interior_mask()
