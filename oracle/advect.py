"""Semi-Lagrangian advection of density and velocity, and the partial
derivatives the optimality conditions need.

Density (Sec. 3.1 eq:Conv: rho_{i+1} = A(rho_i, v_i)): one Euler backtrace
from each cell centre with the cell-centred velocity, then clamped
multilinear interpolation of rho at the foot point.  The paper's own
operator is an upwind matrix exponential (eq:Adv); Sec. 4.1 states that any
advection operator with available partials in rho and v may replace it, and
the semi-Lagrangian one is used here.

Velocity self-advection: S(v) on every interior a-face backtraces with the
face velocity (own component, plus the 4-face average of each other
component) and interpolates v_a on the a-face lattice.  It replaces the
implicit velocity-vorticity term of eq:NSA, giving the explicit step
v_{i+1} = Q(S(v_i) + dt u_i).  The interpolation of S is the C1 variant of
the multilinear one (smoothstep of each fraction, see interp.Stencil): the
KKT residual of the velocity subproblem contains J_S(v)^T u, whose foot-point
term is the interpolant's gradient, and with plain multilinear weights that
gradient jumps where a foot point crosses a lattice line, so eq:KKTAO has no
continuous residual for the FAS cycle of Alg:STFAS to drive to zero (it
settles into a limit cycle); the paper's own velocity operator is a smooth
finite-difference one.  The density keeps plain multilinear weights.

All backtraces are computed in index space as  Y = X - (dt/h) * velocity.
Every function accepts one field (1-D) or a batch of independent fields
(2-D, one per row) and returns the same rank.
"""
import numpy as np

from .grid import Grid
from .interp import Stencil, interp, interp_grad, interp_transpose


def _batch(x):
    x = np.asarray(x, dtype=np.float64)
    return (x[None, :], True) if x.ndim == 1 else (x, False)


def _unbatch(x, single):
    return x[0] if single else x


def _faces(g: Grid, v):
    """Per-axis arrays of a batch of face fields: shape (B,) + face_shape."""
    B = v.shape[0]
    return [v[:, g.face_offsets[a]:g.face_offsets[a + 1]].reshape((B,) + g.face_shapes[a])
            for a in range(g.dim)]


def _sl(g: Grid, a, start, stop):
    """Batched slice along spatial axis a."""
    return (slice(None),) + g.sl_along(a, start, stop)


def cell_velocity(g: Grid, v):
    """vbar_{c,a} = (v_a[c] + v_a[c + e_a]) / 2, shape (B, ncell, d)."""
    parts = _faces(g, v)
    B = v.shape[0]
    out = np.zeros((B, g.ncell, g.dim))
    for a in range(g.dim):
        lo = parts[a][_sl(g, a, 0, g.n[a])]
        hi = parts[a][_sl(g, a, 1, g.n[a] + 1)]
        out[:, :, a] = (0.5 * (lo + hi)).reshape(B, -1)
    return out


def _cell_backtrace(g, v, dt, h):
    return g.cell_positions()[None] - (dt / h) * cell_velocity(g, v)


def advect_scalar(g: Grid, rho, v, dt, h=None):
    """A(rho, v) = W(v) rho."""
    h = g.h if h is None else h
    rho, single = _batch(rho)
    v, _ = _batch(v)
    return _unbatch(interp(rho, _cell_backtrace(g, v, dt, h), g.n), single)


def advect_scalar_T(g: Grid, mu, v, dt, h=None):
    """(dA/drho)^T mu = W(v)^T mu."""
    h = g.h if h is None else h
    mu, single = _batch(mu)
    v, _ = _batch(v)
    return _unbatch(interp_transpose(mu, _cell_backtrace(g, v, dt, h), g.n), single)


def advect_scalar_dv_T(g: Grid, mu, rho, v, dt, h=None):
    """(dA(rho, v)/dv)^T mu on the faces.  A_c depends on the two a-faces of
    cell c through vbar_{c,a}; each carries half of  mu_c * (-dt/h) * d_a I[rho](Y_c)."""
    h = g.h if h is None else h
    mu, single = _batch(mu)
    rho, _ = _batch(rho)
    v, _ = _batch(v)
    B = v.shape[0]
    dI = interp_grad(rho, _cell_backtrace(g, v, dt, h), g.n)          # (B, ncell, d)
    out = np.zeros((B, g.nface))
    parts = _faces(g, out)
    for a in range(g.dim):
        t = (0.5 * (-dt / h) * mu * dI[:, :, a]).reshape((B,) + g.cell_shape)
        # interior face I gets the contributions of cells I - e_a and I
        parts[a][_sl(g, a, 1, g.n[a])] = t[_sl(g, a, 0, g.n[a] - 1)] + t[_sl(g, a, 1, g.n[a])]
    return _unbatch(out, single)


def face_velocity(g: Grid, v, a):
    """Velocity at every interior a-face, shape (B, count_interior, d): own
    component v_a[I]; component b != a is the mean of v_b at I - e_a,
    I - e_a + e_b, I and I + e_b."""
    parts = _faces(g, v)
    B = v.shape[0]
    n = g.n
    cols = []
    for b in range(g.dim):
        if b == a:
            cols.append(parts[a][_sl(g, a, 1, n[a])].reshape(B, -1))
            continue
        acc = 0.0
        for a_lo in (0, 1):
            for b_lo in (0, 1):
                acc = acc + parts[b][_quad(g, a, b, a_lo, b_lo)]
        cols.append((0.25 * acc).reshape(B, -1))
    return np.stack(cols, axis=2)


def _quad(g, a, b, a_lo, b_lo):
    """Batched slice of the b-faces around the interior a-faces:
    a_lo = 0 -> I - e_a, 1 -> I;  b_lo = 0 -> I, 1 -> I + e_b."""
    sl = [slice(None)] * (g.dim + 1)
    sl[1 + g.npax(a)] = slice(a_lo, a_lo + g.n[a] - 1)
    sl[1 + g.npax(b)] = slice(b_lo, b_lo + g.n[b])
    return tuple(sl)


def _interior_positions(g: Grid, a):
    pos = g.face_positions(a).reshape(g.face_shapes[a] + (g.dim,))
    return pos[g.sl_along(a, 1, g.n[a])].reshape(-1, g.dim)


def self_advect(g: Grid, v, dt, h=None):
    """S(v): semi-Lagrangian self-advection on interior faces, zero on walls."""
    h = g.h if h is None else h
    v, single = _batch(v)
    B = v.shape[0]
    vparts = _faces(g, v)
    out = np.zeros((B, g.nface))
    oparts = _faces(g, out)
    for a in range(g.dim):
        Y = _interior_positions(g, a)[None] - (dt / h) * face_velocity(g, v, a)
        ext = g.face_lattice_extent(a)
        val = interp(vparts[a].reshape(B, -1), Y, ext, Stencil(Y, ext, c1=True))
        dst = oparts[a][_sl(g, a, 1, g.n[a])]
        oparts[a][_sl(g, a, 1, g.n[a])] = val.reshape(dst.shape)
    return _unbatch(out, single)


def self_advect_T(g: Grid, v, y, dt, h=None):
    """J_S(v)^T y: the transpose of the Jacobian of S at v applied to y.

    Two parts per interior a-face I: the interpolation weights scatter y_I onto
    the a-face lattice, and the foot-point term y_I * (-dt/h) * grad_Y I[v_a]
    flows back to the sampled velocities (component a to v_a[I]; component
    b != a by quarters to the four v_b faces averaged at I).  Wall faces are
    fixed, so whatever lands on them is dropped."""
    h = g.h if h is None else h
    v, single = _batch(v)
    y, _ = _batch(y)
    B = v.shape[0]
    n = g.n
    vparts = _faces(g, v)
    yparts = _faces(g, y)
    out = np.zeros((B, g.nface))
    acc = _faces(g, out)
    for a in range(g.dim):
        ext = g.face_lattice_extent(a)
        Y = _interior_positions(g, a)[None] - (dt / h) * face_velocity(g, v, a)
        yin = yparts[a][_sl(g, a, 1, n[a])]
        ya = yin.reshape(B, -1)
        st = Stencil(Y, ext, c1=True)
        acc[a] += interp_transpose(ya, Y, ext, st).reshape(acc[a].shape)
        gp = ya[..., None] * (-dt / h) * interp_grad(vparts[a].reshape(B, -1), Y, ext, st)
        for b in range(g.dim):
            comp = gp[..., b].reshape(yin.shape)
            if b == a:
                acc[a][_sl(g, a, 1, n[a])] += comp
                continue
            for a_lo in (0, 1):
                for b_lo in (0, 1):
                    acc[b][_quad(g, a, b, a_lo, b_lo)] += 0.25 * comp
    out *= g.interior_mask()[None]
    return _unbatch(out, single)
