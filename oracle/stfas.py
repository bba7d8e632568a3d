"""STFAS: the FAS V-cycle of Alg:STFAS and the NSO loop of Alg:outter.

V-cycle(2,2) on level l (coarsest: 10 smoothing sweeps):
  two pre-sweeps
  x_s = x;   r = res - f(x_s)
  x^{2h} = R x_s;   x = x_s - P x^{2h}
  res^{2h} = f^{2h}(x^{2h}) + R r
  V-cycle on level l+1
  x = x + P x^{2h};   two post-sweeps
Reading: the fine residual is evaluated on the smoothed iterate before the
subtraction (as in a standard FAS cycle); the algorithm as printed
overwrites the iterate first.  The subtract-then-add form of the correction
is kept.  Levels coarsen every axis by 2 while every n_a / 2^l >= 4; the
coarse operator re-discretises with h_l = 2^l h and the same N, dt, K/r,
and the coarse targets are w^{2h} = R w.

NSO: warm start; V-cycles until |f|_inf <= eps |f(0)|_inf (f(0) is the
residual of the zero iterate) or a cap (reading of the absolute test of
Alg:outter, whose 1e-5 is out of reach when F1 scales with K/r).
"""
import numpy as np

from .grid import Grid
from .kkt import Level, residual, residual_f, inf_norm
from .scgs import sweep
from .transfer import Transfer


def level_grids(g: Grid):
    gs = [g]
    while all(x % 2 == 0 and x // 2 >= 4 for x in gs[-1].n):
        gs.append(gs[-1].coarse())
    return gs


class Hierarchy:
    def __init__(self, g: Grid, N, dt, K_over_r, advect=True, omega=1.0, lm=0.0, velocity="sl", local_adv=True):
        self.grids = level_grids(g)
        # local_adv: True on every level, False on none, "finest" on level 0 only
        self.levels = [Level(gl, N, dt, K_over_r, advect, omega, lm, velocity,
                             local_adv if local_adv != "finest" else l == 0) for l, gl in enumerate(self.grids)]
        self.transfers = [Transfer(gl) for gl in self.grids[:-1]]

    def targets(self, w):
        ws = [w]
        for t in self.transfers:
            ws.append(t.restrict_faces_seq(ws[-1]))
        return ws


def vcycle(H: Hierarchy, l, x, ws, res, pre=2, post=2, coarse_sweeps=10):
    L = H.levels[l]
    if l == len(H.levels) - 1:
        for _ in range(coarse_sweeps):
            sweep(L, x, ws[l], res)
        return
    for _ in range(pre):
        sweep(L, x, ws[l], res)
    T = H.transfers[l]
    r = residual(L, x, ws[l], res)
    xc = T.restrict_state(x)
    px = T.prolong_state(xc)
    for k in range(4):
        x[k] -= px[k]
    Lc = H.levels[l + 1]
    fc = residual_f(Lc, xc, ws[l + 1])
    rr = T.restrict_state(r)
    resc = [fc[k] + rr[k] for k in range(4)]
    vcycle(H, l + 1, xc, ws, resc, pre, post, coarse_sweeps)
    px = T.prolong_state(xc)
    for k in range(4):
        x[k] += px[k]
    for _ in range(post):
        sweep(L, x, ws[l], res)


def nso(H: Hierarchy, x, w, eps=1e-5, max_vcycles=30, fixed_counts=False, info=None):
    """Returns (vcycles run, |f|_inf history); info (a dict), if given,
    receives f0 = |f(0)|_inf, the scale of the relative stop."""
    L = H.levels[0]
    ws = H.targets(w)
    zero = [np.zeros_like(a) for a in x]
    f0 = inf_norm(residual_f(L, zero, w))
    if info is not None:
        info["f0"] = f0
    res = [np.zeros_like(a) for a in x]
    hist = [inf_norm(residual_f(L, x, w))]
    n = 0
    while n < max_vcycles:
        if not fixed_counts and hist[-1] <= eps * f0:
            break
        vcycle(H, 0, x, ws, res)
        n += 1
        hist.append(inf_norm(residual_f(L, x, w)))
    return n, hist
