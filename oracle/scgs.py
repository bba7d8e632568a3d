"""Spacetime SCGS smoother (Sec. 4.3, eq:HESS).

SCGS (Vanka) visits one cell at a time and solves together for the face
unknowns around it and the pressure at its centre; the spacetime version
takes those unknowns for all time steps at once.  The local matrix is block
tridiagonal in time with (2d+1)x(2d+1) blocks and is solved by block
elimination in O(N).  Cells are processed by 2^d colours (parity of each
coordinate) so that cells of one colour share no unknowns; within a colour
every cell first forms its local residual from the state at the start of the
colour, then all cells apply their corrections (Jacobi within a colour,
colours in lexicographic order).

One term of the residual is not local: J_S(v_i)^T u_i / dt in F1 gathers
from every face whose foot point lands near the row's face.  In 3D a sweep
evaluates it once, from the state at its start, and holds it while its
eight colours pass (Jacobi in that coupling, Gauss-Seidel in the local
ones): that costs about a third more V-cycles and saves seven of every
eight evaluations of the term, which is most of a colour pass in 3D.  In 2D
(four colours, a cheaper term) it is evaluated per colour.  The residual the
V-cycle restricts is exact either way, so the solution is unchanged.

The correction is relaxed by the weight omega of the level (1 unless set).

Levenberg-Marquardt safeguard (Sec. 5, convergence analysis: a perturbation
of the penalty K in the Hessian eq:HESS makes the cycle the inner solver of
a Levenberg-Marquardt method): with lm > 0 the local matrix has
K/r + lm/dt^2 on every v block (v_N included, which has no K term).  Only
the local matrix changes; the residual, and hence the solution the cycles
converge to, is the unperturbed one.  With the semi-Lagrangian operator the
local matrix leaves out the advection derivative (du_i/dv_i = -I/dt below),
which is far from J_S once the flow moves about a cell per step; the
perturbation keeps the smoother contracting there.

Local unknown blocks, in time order k = 0..2N-1:
  k = 2i     (u_i, p_{i+1})        row F3_i (faces), F4_i (centre)
  k = 2i + 1 (v_{i+1}, pbar_{i+1}) row F1_{i+1},     F2_{i+1}
Within a block: face slots 2a (low a-face of the cell), 2a+1 (high a-face),
then the pressure.  Wall faces are not unknowns: their slot is an identity
row with zero right-hand side.

Local Jacobian (reading of the smoother for the semi-Lagrangian operator:
the derivative of the advection is left out of the local matrix, i.e.
du_i/dv_i = -I/dt exactly as eq:KKTAO states; the residual stays exact):
  face rows   T_kk x_k + T_k,k-1 x_{k-1} + T_k,k+1 x_{k+1} - g pi_k
  centre row  g^T x_k
  T_kk  = -1 (u blocks),  K/r (v_i, i<N),  0 (v_N)   [+ lm/dt^2 on v blocks]
  T(u_{i-1}, v_i) = +1/dt,   T(v_i, u_i) = -1/dt   (symmetric)
  g = divergence coefficients of the cell's faces (-1/h low, +1/h high).

With the rotational operator (level.local_adv) the local matrix is eq:HESS
itself: the coupling of u_i and v_{i+1} is the cell's block of
du_i/dv_{i+1} = I/dt + dAdv/dv at v_{i+1} (rows: F3_i at the cell's faces,
columns: v_{i+1} at the cell's faces), and its transpose couples v_{i+1}
and u_i in F1_{i+1}.  The v blocks keep K/r (+ the perturbation) as printed:
the second derivative of Adv, which F1_{i+1} carries through
J_Adv(v_{i+1})^T u_i, is not in eq:HESS.  The blocks are no longer scalar
multiples of the identity, so the elimination below takes them as full
(2d+1)x(2d+1) matrices.
"""
import numpy as np

from .grid import Grid
from .kkt import Level, residual, transpose_term
from . import vorticity


def colour_cells(g: Grid, colour):
    """Multi-indices (x, y[, z] columns) of the cells of one colour."""
    pos = g.cell_positions().astype(np.int64)
    par = np.zeros(g.ncell, dtype=np.int64)
    for a in range(g.dim):
        par += (pos[:, a] % 2) << a
    return pos[par == colour]


def _face_flat(g: Grid, a, idx):
    """Flat face index of the a-faces with multi-index idx (x first)."""
    ext = g.face_lattice_extent(a)
    flat = np.zeros(idx.shape[0], dtype=np.int64)
    stride = 1
    for b in range(g.dim):
        flat += idx[:, b] * stride
        stride *= ext[b]
    return g.face_offsets[a] + flat


def _cell_flat(g: Grid, idx):
    flat = np.zeros(idx.shape[0], dtype=np.int64)
    stride = 1
    for b in range(g.dim):
        flat += idx[:, b] * stride
        stride *= g.n[b]
    return flat


def _tmatrix(N, dt, kr, mu=0.0):
    """Diagonal and the coupling T_{k,k+1} of the temporal matrix; mu is the
    Levenberg-Marquardt perturbation added to K/r on every v block."""
    diag = np.zeros(2 * N)
    off = np.zeros(2 * N - 1)
    for k in range(2 * N):
        if k % 2 == 0:
            diag[k] = -1.0
        else:
            i = (k + 1) // 2
            diag[k] = (kr if i < N else 0.0) + mu
        if k + 1 < 2 * N:
            off[k] = (1.0 / dt) if k % 2 == 0 else (-1.0 / dt)
    return diag, off


def adv_local_blocks(L: Level, v, fidx, inner):
    """Per slot i (v[i] = v_{i+1}) and cell of the colour, the block of
    I/dt + dAdv/dv at v_{i+1} on the cell's face slots: out[i, c, t, s] =
    d(F3_i at slot t) / d(v_{i+1} at slot s), zero where a slot is a wall.

    Adv is a homogeneous quadratic, so (Adv(v + d) - Adv(v - d)) / 2 is its
    Jacobian times d exactly (up to rounding).  d is taken as the indicator
    of slot s of every cell of the colour at once: Adv at a face reads only
    the faces that share one of its end nodes, and two cells of one colour
    differ by an even, nonzero offset, so no face of one of them shares a
    node with a face of the other: each cell's slots see only its own d."""
    g, N, dt = L.g, L.N, L.dt
    nc, ns = fidx.shape
    out = np.zeros((N, nc, ns, ns))
    for s in range(ns):
        d = np.zeros(g.nface)
        sel = inner[:, s]
        d[fidx[sel, s]] = 1.0
        for i in range(N):
            jd = 0.5 * (vorticity.adv(g, v[i] + d) - vorticity.adv(g, v[i] - d))
            out[i, :, :, s] = jd[fidx] * inner * inner[:, s:s + 1]
    for s in range(ns):
        out[:, :, s, s] += inner[:, s] / dt
    return out


def smooth_colour(L: Level, x, w, res, colour, jst=None):
    """One colour: local residuals from the current state (with the transpose
    term jst of F1 if given), local solves, corrections."""
    g, N, h = L.g, L.N, L.g.h
    d = g.dim
    B = 2 * d + 1
    cells = colour_cells(g, colour)
    nc = cells.shape[0]
    if nc == 0:
        return
    r = residual(L, x, w, res, jst)
    v, pb, u, p = x
    # face slots of each cell
    fidx = np.zeros((nc, 2 * d), dtype=np.int64)
    coef = np.zeros((nc, 2 * d))
    inner = np.zeros((nc, 2 * d), dtype=bool)
    for a in range(d):
        lo = cells.copy()
        hi = cells.copy()
        hi[:, a] += 1
        fidx[:, 2 * a] = _face_flat(g, a, lo)
        fidx[:, 2 * a + 1] = _face_flat(g, a, hi)
        inner[:, 2 * a] = lo[:, a] >= 1
        inner[:, 2 * a + 1] = hi[:, a] <= g.n[a] - 1
        coef[:, 2 * a] = -1.0 / h
        coef[:, 2 * a + 1] = 1.0 / h
    coef = coef * inner
    cidx = _cell_flat(g, cells)
    E = np.zeros((nc, B, B))
    for s in range(2 * d):
        E[:, s, s] = inner[:, s]
    diag, off = _tmatrix(N, L.dt, L.kr, L.lm / (L.dt * L.dt))

    def block(k):
        A = np.zeros((nc, B, B))
        for s in range(2 * d):
            A[:, s, s] = np.where(inner[:, s], diag[k], 1.0)
            A[:, s, B - 1] = -coef[:, s]
            A[:, B - 1, s] = coef[:, s]
        return A

    def rhs(k):
        j = k // 2
        fr, cr = (r[2], r[3]) if k % 2 == 0 else (r[0], r[1])
        dk = np.zeros((nc, B))
        dk[:, :2 * d] = fr[j][fidx] * inner
        dk[:, B - 1] = cr[j][cidx]
        return dk

    Bl = adv_local_blocks(L, v, fidx, inner) if L.local_adv else None

    def upper(k):
        """Coupling of block k (rows) with block k + 1 (columns)."""
        if Bl is not None and k % 2 == 0:
            A = np.zeros((nc, B, B))
            A[:, :2 * d, :2 * d] = Bl[k // 2]          # dF3_i / dv_{i+1}, i = k / 2
            return A
        return off[k] * E

    # block elimination forward (the matrix is symmetric: the coupling of
    # block k with block k - 1 is upper(k - 1) transposed)
    Ahat = [None] * (2 * N)
    dhat = [None] * (2 * N)
    Ahat[0], dhat[0] = block(0), rhs(0)
    for k in range(1, 2 * N):
        Uk1 = upper(k - 1)
        Lk = np.transpose(Uk1, (0, 2, 1))
        M = np.linalg.solve(np.transpose(Ahat[k - 1], (0, 2, 1)), np.transpose(Lk, (0, 2, 1)))
        M = np.transpose(M, (0, 2, 1))                      # M = Lk Ahat_{k-1}^{-1}
        Ahat[k] = block(k) - M @ Uk1
        dhat[k] = rhs(k) - np.einsum("cij,cj->ci", M, dhat[k - 1])
    # back substitution
    xs = [None] * (2 * N)
    xs[2 * N - 1] = np.linalg.solve(Ahat[2 * N - 1], dhat[2 * N - 1][..., None])[..., 0]
    for k in range(2 * N - 2, -1, -1):
        Uk = upper(k)
        t = dhat[k] - np.einsum("cij,cj->ci", Uk, xs[k + 1])
        xs[k] = np.linalg.solve(Ahat[k], t[..., None])[..., 0]
    # apply the corrections (disjoint unknowns within a colour), relaxed by omega
    xs = [L.omega * xk for xk in xs]
    for k in range(2 * N):
        j = k // 2
        fx, cx = (u, p) if k % 2 == 0 else (v, pb)
        for s in range(2 * d):
            sel = inner[:, s]
            fx[j][fidx[sel, s]] += xs[k][sel, s]
        cx[j][cidx] += xs[k][:, B - 1]


def sweep(L: Level, x, w, res):
    """All colours in order.  In 3D the transpose term J_S(v_i)^T u_i/dt of F1
    is evaluated once, from the state at the start of the sweep, and held
    while the colours pass; every other row, and in 2D that term too, is
    evaluated per colour from the current state."""
    jst = transpose_term(L, x) if L.g.dim == 3 else None
    for colour in range(2 ** L.g.dim):
        smooth_colour(L, x, w, res, colour, jst)
