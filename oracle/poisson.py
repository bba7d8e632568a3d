"""Solenoidal projection Q (Sec. 4.1: Q replaces the multiplier of the
divergence constraint; the paper evaluates it with a conventional Poisson
solver).

  Q(w) = w - G phi,  where  L phi = D w,  L = D G (Neumann),  mean(phi) = 0.

The oracle solves the singular Neumann system with plain conjugate
gradients on -L (symmetric positive definite on mean-zero vectors) to a
relative residual of 1e-14; the device path uses multigrid instead.
"""
import numpy as np

from .grid import Grid, div, grad, laplacian


def solve_neumann(g: Grid, b, h=None, rtol=1e-14, maxiter=100000):
    """Mean-zero phi with L phi = b - mean(b)."""
    h = g.h if h is None else h
    b = np.asarray(b, dtype=np.float64).ravel()
    b = b - b.mean()
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    if nb == 0.0:
        return x
    r = -b.copy()                 # residual of (-L) x = -b at x = 0
    p = r.copy()
    rs = r @ r
    for _ in range(maxiter):
        if np.sqrt(rs) <= rtol * nb:
            break
        Ap = -laplacian(g, p, h)
        alpha = rs / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        rs_new = r @ r
        p = r + (rs_new / rs) * p
        rs = rs_new
    return x - x.mean()


def project(g: Grid, w, h=None, rtol=1e-14):
    """Q(w) and the potential phi (so that the step pressure is phi / dt)."""
    h = g.h if h is None else h
    phi = solve_neumann(g, div(g, w, h), h, rtol)
    return w - grad(g, phi, h), phi
