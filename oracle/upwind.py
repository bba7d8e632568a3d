"""Upwind Taylor-exponential density advection: the paper's own density
operator (Sec. 3.1 eq:Adv), with the partial derivatives in rho and v that
the density subproblem needs (Sec. 4.1, Alg:Passive).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.

  A(rho, v) = sum_{j=0..k} (dt^j / j!) A(v)^j rho

A(v) is a flux-form upwind stencil on the MAC grid: across an interior
a-face f between cells L = I - e_a and R = I with normal velocity v_f, the
flux is v_f times an upwind face value of the scalar; L loses flux/h and R
gains it.  Walls carry no flux.  The face value is second order: with U the
upstream cell and UU the next cell upstream (U = L, UU = L - e_a for
v_f >= 0; U = R, UU = R + e_a for v_f < 0), x_f = (3 x_U - x_UU) / 2, and
x_f = x_U where UU lies outside the grid.

The series is truncated adaptively: T_0 = rho, T_j = (dt / j) A(v) T_{j-1};
k is the first j with max|T_j| < tol (tol = 1e-5), at most KMAX; the terms
T_0..T_k are summed.

Readings (the paper names the operator, a second-order upwind stencil, and
the truncation test, but not the stencil's form or the norm):
  * flux form with second-order upwind face values, first order next to a
    wall; this conserves mass (every column of A sums to zero) but is not
    skew-symmetric, so the norm-preservation argument of Sec. 3.1 holds only
    for its central part;
  * the truncation test uses the max norm and includes the term that
    passes it; KMAX = 48 bounds the work;
  * at v_f = 0 the v_f >= 0 branch is taken, for the value and the
    derivative;
  * the derivative in rho of the truncated series is taken at fixed k (the
    series is linear in rho for fixed k), and so is the derivative in v.
"""
import math

import numpy as np
import scipy.sparse as sp

from .grid import Grid

TOL = 1e-5
KMAX = 48


def _cell_ids(g: Grid):
    return np.arange(g.ncell).reshape(g.cell_shape)


def _interior_faces(g: Grid, a):
    """For every interior a-face: its flat index in the face vector and the
    (numpy-ordered) multi-index of cell R = I (cell L = I - e_a)."""
    ax = g.npax(a)
    shape = g.face_shapes[a]
    idx = np.indices(shape).reshape(g.dim, -1)
    flat = g.face_offsets[a] + np.arange(int(np.prod(shape)))
    keep = (idx[ax] >= 1) & (idx[ax] <= g.n[a] - 1)
    return flat[keep], idx[:, keep]


def _upwind_weights(g: Grid, a, idx, vf):
    """Cells and weights of the upwind face value at each face: a list of
    (cell ids, weights) pairs, weights 0 where an entry does not apply."""
    ax = g.npax(a)
    ids = _cell_ids(g)
    Ia = idx[ax]
    pos = vf >= 0
    U = np.where(pos, Ia - 1, Ia)
    UU = np.where(pos, Ia - 2, Ia + 1)
    has_uu = (UU >= 0) & (UU <= g.n[a] - 1)
    UUc = np.clip(UU, 0, g.n[a] - 1)

    def cell(along):
        m = idx.copy()
        m[ax] = along
        return ids[tuple(m)]

    wU = np.where(has_uu, 1.5, 1.0)
    wUU = np.where(has_uu, -0.5, 0.0)
    return [(cell(U), wU), (cell(UUc), wUU)]


def matrix(g: Grid, v, h=None):
    """The stencil A(v) as a sparse ncell x ncell matrix."""
    h = g.h if h is None else h
    v = np.asarray(v, dtype=np.float64)
    rows, cols, vals = [], [], []
    ids = _cell_ids(g)
    for a in range(g.dim):
        ax = g.npax(a)
        flat, idx = _interior_faces(g, a)
        vf = v[flat]
        R = ids[tuple(idx)]
        m = idx.copy()
        m[ax] = idx[ax] - 1
        L = ids[tuple(m)]
        for c, w in _upwind_weights(g, a, idx, vf):
            # flux = v_f * w * x_c through the face: L loses flux/h, R gains it
            rows += [L, R]
            cols += [c, c]
            vals += [-vf * w / h, vf * w / h]
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(g.ncell, g.ncell))


def face_values(g: Grid, v, x):
    """Upwind face values x_f on every face (zero on walls)."""
    v = np.asarray(v, dtype=np.float64)
    out = np.zeros(g.nface)
    for a in range(g.dim):
        flat, idx = _interior_faces(g, a)
        acc = np.zeros(flat.size)
        for c, w in _upwind_weights(g, a, idx, v[flat]):
            acc += w * x[c]
        out[flat] = acc
    return out


def dA_dv_T(g: Grid, v, x, z, h=None):
    """(d(A(v) x)/dv)^T z on the faces: at an interior face between L and R,
    (z_R - z_L) x_f / h; zero on walls."""
    h = g.h if h is None else h
    xf = face_values(g, v, x)
    out = np.zeros(g.nface)
    ids = _cell_ids(g)
    for a in range(g.dim):
        ax = g.npax(a)
        flat, idx = _interior_faces(g, a)
        R = ids[tuple(idx)]
        m = idx.copy()
        m[ax] = idx[ax] - 1
        L = ids[tuple(m)]
        out[flat] = (z[R] - z[L]) * xf[flat] / h
    return out


def series(g: Grid, rho, v, dt, tol=TOL, kmax=KMAX, h=None):
    """The summed terms T_0..T_k of eq:Adv and k."""
    A = matrix(g, v, h)
    terms = [np.asarray(rho, dtype=np.float64)]
    k = 0
    while np.max(np.abs(terms[-1])) >= tol and k < kmax:
        k += 1
        terms.append((dt / k) * (A @ terms[-1]))
    return terms, k


def advect_up(g: Grid, rho, v, dt, h=None):
    terms, _ = series(g, rho, v, dt, h=h)
    return np.sum(terms, axis=0)


def advect_up_k(g: Grid, rho, v, dt, h=None):
    return series(g, rho, v, dt, h=h)[1]


def apply_fixed_k(g: Grid, x, v, dt, k, h=None):
    """sum_{j=0..k} (dt^j / j!) A(v)^j x for a given k (the linear map the
    series applies to rho)."""
    A = matrix(g, v, h)
    t = np.asarray(x, dtype=np.float64)
    out = t.copy()
    for j in range(1, k + 1):
        t = (dt / j) * (A @ t)
        out = out + t
    return out


def advect_up_T(g: Grid, mu, rho, v, dt, h=None):
    """(dA/drho)^T mu = sum_{j=0..k} (dt^j / j!) (A^T)^j mu, k from rho."""
    k = advect_up_k(g, rho, v, dt, h)
    At = matrix(g, v, h).T.tocsr()
    t = np.asarray(mu, dtype=np.float64)
    out = t.copy()
    for j in range(1, k + 1):
        t = (dt / j) * (At @ t)
        out = out + t
    return out


def advect_up_dv_T(g: Grid, mu, rho, v, dt, h=None):
    """(dA(rho, v)/dv)^T mu at fixed k.  By the product rule,
      d/dv [(dt^j/j!) A^j rho] = (dt^j/j!) sum_{a+b=j-1} A^a (dA) A^b rho,
    so the transpose is sum_j sum_{a+b=j-1} (dt^j/j!) D(A^b rho)^T (A^T)^a mu
    with D(x)^T z = dA_dv_T(x, z).  With the scaled powers
    T_b = (dt^b/b!) A^b rho and M_a = (dt^a/a!) (A^T)^a mu each pair carries
    dt * a! b! / j!."""
    terms, k = series(g, rho, v, dt, h=h)
    At = matrix(g, v, h).T.tocsr()
    M = [np.asarray(mu, dtype=np.float64)]
    for a in range(1, k):
        M.append((dt / a) * (At @ M[-1]))
    out = np.zeros(g.nface)
    for j in range(1, k + 1):
        for a in range(j):
            b = j - 1 - a
            coef = dt * math.factorial(a) * math.factorial(b) / math.factorial(j)
            out += coef * dA_dv_T(g, v, terms[b], M[a], h)
    return out
