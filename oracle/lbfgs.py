"""L-BFGS on the reduced objective: the gradient-based baseline the paper
compares against (Sec. 5, "Comparison with LBFGS"; Sec. 3.2 for the approach
it stands for: eliminate the simulation and minimise over u directly).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.

Reduced objective (Sec. 3.2 eq:opt with the simulation eliminated):
  J(u) = 1/2 sum_k <e_k, C e_k> + r/2 sum_i |u_i|^2,  e_k = rho_k - rho*_k,
with (rho_i, v_i) from the simulation started at (rho_0, v_0 = 0).  Its
gradient is the adjoint of the step chain (each evaluation costs a forward
and a backward pass, as the paper notes).  With the rotational velocity
operator (velocity = "vorticity") the simulation is that of its fixed-point
steps and the gradient is their exact adjoint.

Optimiser (Nocedal & Wright, two-loop recursion): history m = 8 (the
paper's), initial Hessian gamma I with gamma = s^T y / y^T y of the newest
pair, and 1 / |g| on the first iteration; a backtracking line search on
the Armijo condition (c1 = 1e-4, first trial step 1, halved up to 20
times); a pair with y^T s <= 1e-12 |s| |y| is not stored.  The paper does
not state its line search: this is the reading.  Stopping (Sec. 5 uses the
same criterion for both optimisers, the ADMM one of Sec. 5): after an
accepted iterate, stop when the largest change of the density over all
steps between it and the previous iterate is at most eps_stop.
"""
import numpy as np

from .grid import Grid
from . import metric
from .admm import objectives, resimulate
from .step import step_backward


def gradient(g: Grid, rho, v, u, keys, r, dt, levels, kind="sl", velocity="sl"):
    """dJ/du by the adjoint of the step chain; rho, v from resimulate."""
    N = u.shape[0]
    gu = np.zeros_like(u)
    g_rho = np.zeros(g.ncell)
    g_v = np.zeros(g.nface)
    for i in range(N, 0, -1):
        if i in keys:
            e = rho[i] - keys[i]
            g_rho = g_rho + metric.apply_metric(g, e, levels)
        g_rho, g_v, gu[i - 1] = step_backward(g, rho[i - 1], v[i - 1], g_rho, g_v, dt, kind=kind,
                                              velocity=velocity, u=u[i - 1])
    return gu + r * u


def minimize(fg, x0, iters, m=8, c1=1e-4, max_halvings=20, stop=None):
    """Generic L-BFGS: fg(x) -> (f, grad).  Returns x, the f history (one
    entry per accepted iterate, starting with f(x0)) and the iterations done
    (fewer than iters when the line search finds no decrease, or when
    stop(x_previous, x_accepted) is true after an accepted iterate)."""
    x = np.array(x0, dtype=np.float64)
    f, gr = fg(x)
    hist = [f]
    S, Y = [], []
    done = 0
    for _ in range(iters):
        # two-loop recursion
        q = gr.copy()
        al = []
        for s, y in zip(reversed(S), reversed(Y)):
            a = (s @ q) / (y @ s)
            al.append(a)
            q = q - a * y
        if S:
            gamma = (S[-1] @ Y[-1]) / (Y[-1] @ Y[-1])
        else:
            gamma = 1.0 / max(np.linalg.norm(gr), 1e-300)
        z = gamma * q
        for (s, y), a in zip(zip(S, Y), reversed(al)):
            b = (y @ z) / (y @ s)
            z = z + s * (a - b)
        d = -z
        slope = gr @ d
        if not slope < 0:
            break
        # backtracking on the Armijo condition
        alpha = 1.0
        accepted = False
        for _ in range(max_halvings + 1):
            xt = x + alpha * d
            ft, gt = fg(xt)
            if ft <= f + c1 * alpha * slope:
                accepted = True
                break
            alpha *= 0.5
        if not accepted:
            break
        s = xt - x
        y = gt - gr
        if y @ s > 1e-12 * np.linalg.norm(s) * np.linalg.norm(y):
            S.append(s)
            Y.append(y)
            if len(S) > m:
                S.pop(0)
                Y.pop(0)
        x_prev = x
        x, f, gr = xt, ft, gt
        hist.append(f)
        done += 1
        if stop is not None and stop(x_prev, x):
            break
    return x, hist, done


def solve(g: Grid, rho0, keys, N, r, dt, levels, iters, u0=None, m=8, eps_stop=0.0, kind="sl", velocity="sl"):
    """L-BFGS on J(u) over N steps from u0 (zero by default), at most iters
    iterations; eps_stop > 0 adds the visual-difference stop.  Returns u,
    the J history and the iterations done."""
    shape = (N, g.nface)
    u0 = np.zeros(shape) if u0 is None else np.asarray(u0, dtype=np.float64).reshape(shape)

    def fg(x):
        u = x.reshape(shape)
        rho, v = resimulate(g, rho0, u, dt, kind, velocity)
        f = objectives(g, rho, keys, u, r, levels)[0]
        return f, gradient(g, rho, v, u, keys, r, dt, levels, kind, velocity).ravel()

    def visual_stop(xa, xb):
        ra, _ = resimulate(g, rho0, xa.reshape(shape), dt, kind, velocity)
        rb, _ = resimulate(g, rho0, xb.reshape(shape), dt, kind, velocity)
        return float(np.max(np.abs(rb - ra))) <= eps_stop

    x, hist, done = minimize(fg, u0.ravel(), iters, m=m, stop=visual_stop if eps_stop > 0 else None)
    return x.reshape(shape), hist, done
