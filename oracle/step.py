"""One simulation step (Sec. 3.1, eq:NSA-eq:Conv with the semi-Lagrangian
velocity operator; the density operator is semi-Lagrangian or the upwind
exponential of eq:Adv, `kind`) and its exact adjoint.

  rho' = A(rho, v)            (density is carried by the old velocity, eq:Conv)
  w    = S(v) + dt u          (advect, then add the control force)
  v'   = Q(w),  p' = phi / dt (projection; the pressure is the multiplier of
                               the divergence constraint, eq:NSB)

With the paper's rotational operator (velocity = "vorticity", 2D or 3D) the
velocity update of eq:NSA is implicit, (v' - v)/dt + Adv[v'] = u - G p'.
Reading: it is solved by a fixed number of fixed-point (Picard) steps from
v'_0 = Q(v + dt u):  v'_{m+1} = Q(v + dt u - dt Adv[v'_m]), m < PICARD;
the density is carried by the old velocity as before.  The step's adjoint
(step_backward with u) is the exact adjoint of those fixed-point steps as
computed, not of the implicit equation they approach.
"""
import numpy as np

from .grid import Grid
from . import advect, density, vorticity
from .poisson import project

PICARD = 4


def step_forward(g: Grid, rho, v, u, dt, rtol=1e-14, kind="sl", velocity="sl"):
    rho_n = density.fwd(g, rho, v, dt, kind)
    if velocity == "vorticity":
        base = (v + dt * u) * g.interior_mask()
        v_n, phi = project(g, base, rtol=rtol)
        for _ in range(PICARD):
            v_n, phi = project(g, base - dt * vorticity.adv(g, v_n), rtol=rtol)
        return rho_n, v_n, phi / dt
    w = advect.self_advect(g, v, dt) + dt * u * g.interior_mask()
    v_n, phi = project(g, w, rtol=rtol)
    return rho_n, v_n, phi / dt


def step_backward(g: Grid, rho, v, g_rho_n, g_v_n, dt, rtol=1e-14, kind="sl", velocity="sl", u=None):
    """Gradients (g_rho, g_v, g_u) of <g_rho_n, rho'> + <g_v_n, v'>.
    Q is symmetric, so the cotangent of w is Q g_v'.  The rotational form
    needs u (its fixed-point iterates depend on it)."""
    mask = g.interior_mask()
    if velocity == "vorticity":
        # forward again, keeping the iterates y_0 .. y_{PICARD-1}
        base = (v + dt * u) * mask
        ys = [project(g, base, rtol=rtol)[0]]
        for _ in range(PICARD - 1):
            ys.append(project(g, base - dt * vorticity.adv(g, ys[-1]), rtol=rtol)[0])
        # backward: y_m = Q(base - dt Adv[y_{m-1}]) for m = PICARD .. 1, then y_0 = Q(base)
        g_y = g_v_n * mask
        g_base = np.zeros(g.nface)
        for m in range(PICARD, 0, -1):
            g_w = project(g, g_y * mask, rtol=rtol)[0] * mask
            g_base += g_w
            g_y = -dt * vorticity.adv_T(g, ys[m - 1], g_w)
        g_w = project(g, g_y * mask, rtol=rtol)[0] * mask
        g_base += g_w
        g_v = g_base + density.adj_v(g, g_rho_n, rho, v, dt, kind)
        g_rho = density.adj_rho(g, g_rho_n, rho, v, dt, kind)
        return g_rho, g_v * mask, dt * g_base
    g_w, _ = project(g, g_v_n * mask, rtol=rtol)
    g_w = g_w * mask
    g_u = dt * g_w
    g_v = advect.self_advect_T(g, v, g_w, dt) + density.adj_v(g, g_rho_n, rho, v, dt, kind)
    g_rho = density.adj_rho(g, g_rho_n, rho, v, dt, kind)
    return g_rho, g_v * mask, g_u
