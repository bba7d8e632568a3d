"""The paper's velocity self-advection in rotational form (Sec. 3.1 eq:NSA:
Adv[v] discretises the quadratic operator (curl v) x v, the gradient part of
(v . grad) v going into the kinetic pressure), on the 2D MAC grid.

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
    """Adv[v] on the faces (zero on walls)."""
    n0, n1 = g.n
    w = node_vorticity(g, v)
    sx, sy = node_sums(g, v)
    ax = -0.25 * ((w * sy)[0:n1, :] + (w * sy)[1:n1 + 1, :])
    ay = 0.25 * ((w * sx)[:, 0:n0] + (w * sx)[:, 1:n0 + 1])
    return g.join([ax, ay]) * g.interior_mask()


def adv_T(g: Grid, v, y):
    """J_Adv(v)^T y: the gradient in v of <y, Adv[v]>."""
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
