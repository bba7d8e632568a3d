"""KKT residual of the velocity subproblem (Sec. 4.2 eq:KKTAO, derived in
App. A), with the semi-Lagrangian step v_{i+1} = Q(S(v_i) + dt u_i).

Unknowns on one level: v_i, pbar_i for i = 1..N and u_i, p_{i+1} for
i = 0..N-1; v_0 = 0 is the fixed initial state.  Storage uses N slots per
field:  v[j] = v_{j+1},  pbar[j] = pbar_{j+1},  u[j] = u_j,  p[j] = p_{j+1}.
The residual f = (F1, F2, F3, F4) uses the same slots as (v, pbar, u, p):

  F1_i = (K/r)[i<N](v_i - w_i) - [i<N] J_S(v_i)^T u_i / dt + u_{i-1} / dt + G pbar_i
  F2_i = D v_i
  F3_i = (v_{i+1} - S(v_i)) / dt - u_i + G p_{i+1},     S(v_0) = 0
  F4_i = D u_i

F1 is the gradient of the reduced objective r/2 sum|u_i|^2 + K/2 sum|v_i - w_i|^2
(divided by r) with u_i = (v_{i+1} - S(v_i))/dt + G p_{i+1}:
du_i/dv_i = -J_S(v_i)/dt and du_{i-1}/dv_i = I/dt.  This moves the
advection derivative from the u_{i-1} coupling of eq:KKTAO (implicit
operator) to the u_i coupling (explicit operator).  As in App. A, Q is
dropped from these partials because u_i is solenoidal at the optimum.
F1 and F3 are zero on wall faces.

With the paper's own velocity operator (velocity = "vorticity", 2D or 3D; Adv of
eq:NSA in the rotational form of vorticity.py, implicit in v_{i+1}):

  F1_i = (K/r)[i<N](v_i - w_i) - [i<N] u_i / dt + u_{i-1} / dt + J_Adv(v_i)^T u_{i-1} + G pbar_i
  F3_i = (v_{i+1} - v_i) / dt + Adv[v_{i+1}] - u_i + G p_{i+1},     v_0 = 0

which is eq:KKTAO as printed: du_i/dv_i = -I/dt and
du_{i-1}/dv_i = I/dt + dAdv/dv_i.  Every term is a local stencil, so F1 has
no non-local part.
"""
import numpy as np

from .grid import Grid, div, grad
from . import advect, vorticity


class Level:
    """Grid plus the constants of eq:KKTAO on that level (h doubles per level).
    advect=False replaces S by the identity (the linear-quadratic special
    case used by the brute-force checks)."""

    def __init__(self, g: Grid, N, dt, K_over_r, advect=True, omega=1.0, lm=0.0, velocity="sl",
                 local_adv=True):
        self.g, self.N, self.dt, self.kr = g, N, dt, K_over_r
        self.mask = g.interior_mask()
        self.advect = advect
        assert velocity in ("sl", "vorticity")
        self.velocity = velocity    # "sl": v_{i+1} = Q(S(v_i) + dt u_i); "vorticity": eq:NSA with Adv
        self.omega = omega          # relaxation weight of the smoother
        self.lm = lm                # Levenberg-Marquardt perturbation of the smoother's K/r, times dt^2
        # rotational operator: the smoother's local matrix holds the cell's block of dAdv/dv (eq:HESS);
        # False leaves it out (du_{i-1}/dv_i = I/dt, the collapsed form of the SL operator)
        self.local_adv = bool(local_adv) and velocity == "vorticity"

    def S(self, v):
        return advect.self_advect(self.g, v, self.dt, self.g.h) if self.advect else v * self.mask

    def JST(self, v, y):
        return advect.self_advect_T(self.g, v, y, self.dt, self.g.h) if self.advect else y * self.mask


def zeros_state(L: Level):
    g, N = L.g, L.N
    return [np.zeros((N, g.nface)), np.zeros((N, g.ncell)), np.zeros((N, g.nface)), np.zeros((N, g.ncell))]


def transpose_term(L: Level, x):
    """J_S(v_i)^T u_i / dt for i = 1..N-1 (slots 0..N-2), the non-local part of
    F1; None when N = 1 or with the rotational operator (no non-local part)."""
    if L.velocity == "vorticity":
        return None
    v, u = x[0], x[2]
    return L.JST(v[:L.N - 1], u[1:L.N]) / L.dt if L.N > 1 else None


def residual_f_vorticity(L: Level, x, w):
    """f(x) with the rotational operator (the module docstring's second form)."""
    g, N, dt, kr, h = L.g, L.N, L.dt, L.kr, L.g.h
    v, pb, u, p = x
    F1 = u / dt + grad(g, pb, h)
    for j in range(N):
        F1[j] += vorticity.adv_T(g, v[j], u[j])
    if N > 1:
        F1[:N - 1] += kr * (v[:N - 1] - w[1:N]) - u[1:N] / dt
    F1 *= L.mask
    F2 = div(g, v, h)
    vprev = np.zeros_like(v)
    vprev[1:] = v[:N - 1]
    A = np.stack([vorticity.adv(g, v[j]) for j in range(N)])
    F3 = ((v - vprev) / dt + A - u + grad(g, p, h)) * L.mask
    F4 = div(g, u, h)
    return [F1, F2, F3, F4]


def residual_f(L: Level, x, w, jst=None):
    """f(x) for the state x = [v, pbar, u, p] and targets w (slot i = w_i).
    The N time slices are independent given x, so they are evaluated as one
    batch.  jst, if given, replaces the transpose term of F1 (the smoother
    holds it over a sweep)."""
    if L.velocity == "vorticity":
        return residual_f_vorticity(L, x, w)
    g, N, dt, kr, h = L.g, L.N, L.dt, L.kr, L.g.h
    v, pb, u, p = x
    # F1_i, i = j + 1:  u_{i-1}/dt + G pbar_i  [+ (K/r)(v_i - w_i) - J_S(v_i)^T u_i / dt  if i < N]
    F1 = u / dt + grad(g, pb, h)
    if N > 1:
        F1[:N - 1] += kr * (v[:N - 1] - w[1:N]) - (transpose_term(L, x) if jst is None else jst)
    F1 *= L.mask
    F2 = div(g, v, h)
    # F3_i, i = j:  (v_{i+1} - S(v_i))/dt - u_i + G p_{i+1},  S(v_0) = 0
    S = np.zeros_like(v)
    if N > 1:
        S[1:] = L.S(v[:N - 1])
    F3 = ((v - S) / dt - u + grad(g, p, h)) * L.mask
    F4 = div(g, u, h)
    return [F1, F2, F3, F4]


def residual(L: Level, x, w, res, jst=None):
    """r = res - f(x)."""
    f = residual_f(L, x, w, jst)
    return [res[k] - f[k] for k in range(4)]


def inf_norm(parts):
    return max(float(np.max(np.abs(a))) if a.size else 0.0 for a in parts)
