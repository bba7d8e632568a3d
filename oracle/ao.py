"""Density subproblem (Sec. 4.1 eq:PO; the paper's "passive"/advection
optimisation): find slack velocities v*_i that carry rho_0 onto the
keyframes while staying close to  vt_i = v_i + lambda_i / K.

  Phi(v*) = 1/2 sum_i c_i <rho_i - rho*_i, C (rho_i - rho*_i)>
            + K/2 sum_{i<N} |vt_i - v*_i|^2,   rho_{i+1} = A(rho_i, v*_i),  div v*_i = 0.

One call runs the fixed-point iteration of Alg:Passive (its KKT form is
eq:KKTPO) a fixed number of times:
  forward   rho_{i+1} = A(rho_i, v*_i)
  backward  mu_{i-1} = W(v*_i)^T mu_i - c_i C (rho_i - rho*_i),  mu_N = 0
  update    v*_i <- Q(vt_i + (dA(rho_i, v*_i)/dv*)^T mu_i / K)
with the blending safeguard of the convergence analysis in Sec. 5: the new
v* is mixed with the old one, v* + alpha (new - old), and the first alpha in
1, 1/2, ..., 2^-10 that does not increase Phi is taken (no re-projection is
needed: a blend of solenoidal fields is solenoidal).  If none qualifies, v*
is kept.

The density operator A is the semi-Lagrangian one or the paper's upwind
exponential (`density` = "sl" or "upwind").

Readings: the backward sweep uses the v* of the forward sweep for every i
(all projections are then independent); the initialisation v* <- vt runs once
per call; alpha = 0 when no trial decreases Phi.
"""
import numpy as np

from .grid import Grid
from . import density
from .metric import apply_metric
from .poisson import project


def forward(g, rho0, vstar, dt, kind="sl"):
    N = vstar.shape[0]
    rho = np.zeros((N + 1, g.ncell))
    rho[0] = rho0
    for i in range(N):
        rho[i + 1] = density.fwd(g, rho[i], vstar[i], dt, kind)
    return rho


def objective(g, rho, keys, vt, vstar, K, levels):
    phi = 0.0
    for t, target in keys.items():
        e = rho[t] - target
        phi += 0.5 * float(e @ apply_metric(g, e, levels))
    diff = vt - vstar
    return phi + 0.5 * K * float(np.sum(diff * diff))


def backward(g, rho, keys, vstar, dt, levels, kind="sl"):
    """mu_i for i = 0..N-1 (mu_N = 0)."""
    N = vstar.shape[0]
    mu = np.zeros((N + 1, g.ncell))
    for i in range(N, 0, -1):
        m = density.adj_rho(g, mu[i], rho[i], vstar[i], dt, kind) if i < N else np.zeros(g.ncell)
        if i in keys:
            e = rho[i] - keys[i]
            m = m - apply_metric(g, e, levels)
        mu[i - 1] = m
    return mu[:N]


def candidate(g, rho, mu, vt, vstar, K, dt, rtol=1e-14, kind="sl"):
    N = vstar.shape[0]
    out = np.zeros_like(vstar)
    for i in range(N):
        gi = density.adj_v(g, mu[i], rho[i], vstar[i], dt, kind)
        out[i], _ = project(g, vt[i] + gi / K, rtol=rtol)
    return out


def gradient(g, rho, keys, vt, vstar, K, dt, levels, kind="sl"):
    """dPhi/dv* = -K (vt - v*) - (dA/dv*)^T mu  (used by the finite-difference pin)."""
    mu = backward(g, rho, keys, vstar, dt, levels, kind)
    N = vstar.shape[0]
    out = np.zeros_like(vstar)
    for i in range(N):
        out[i] = -K * (vt[i] - vstar[i]) - density.adj_v(g, mu[i], rho[i], vstar[i], dt, kind)
    return out * g.interior_mask()


def solve(g: Grid, rho0, keys, vt, K, dt, levels, iters=2, max_halvings=10, rtol=1e-14, kind="sl"):
    """Returns (v*, rho, history of Phi after each iteration)."""
    vstar = vt.copy()
    rho = forward(g, rho0, vstar, dt, kind)
    phi = objective(g, rho, keys, vt, vstar, K, levels)
    hist = [phi]
    for _ in range(iters):
        mu = backward(g, rho, keys, vstar, dt, levels, kind)
        cand = candidate(g, rho, mu, vt, vstar, K, dt, rtol, kind)
        alpha = 1.0
        for _ in range(max_halvings + 1):
            trial = vstar + alpha * (cand - vstar)
            rho_t = forward(g, rho0, trial, dt, kind)
            phi_t = objective(g, rho_t, keys, vt, trial, K, levels)
            if phi_t <= phi:
                vstar, rho, phi = trial, rho_t, phi_t
                break
            alpha *= 0.5
        hist.append(phi)
    return vstar, rho, hist
