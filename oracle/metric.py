"""Keyframe metric C (Sec. 4.1): a sum of Gaussian filters with doubling
standard deviation ("receding support") that spreads the keyframe mismatch
over the domain.

Reading used (the paper fixes neither the first sigma, the number of
filters, the normalisation nor the boundary treatment):
  C e = e + sum_{l=1..L} G_l (G_l e),
  G_l separable, sigma_l = 2^(l-1) cells, taps -R..R with R = ceil(3 sigma_l),
  weights exp(-j^2 / (2 sigma_l^2)) normalised to sum 1, zero outside the grid.
G_l is symmetric, so G_l^T G_l = G_l G_l and C is symmetric positive definite.
"""
import math
import numpy as np

from .grid import Grid


def default_levels(n):
    """Largest L with sigma_L = 2^(L-1) <= min(n) / 8."""
    m = min(n)
    L = 0
    while 2 ** L <= m / 8.0:
        L += 1
    return L


def gauss_taps(sigma):
    R = int(math.ceil(3.0 * sigma))
    j = np.arange(-R, R + 1, dtype=np.float64)
    k = np.exp(-j * j / (2.0 * sigma * sigma))
    return k / k.sum()


def blur(g: Grid, e, sigma):
    """G e: the separable Gaussian with zero padding, one axis at a time."""
    x = np.asarray(e, dtype=np.float64).reshape(g.cell_shape)
    taps = gauss_taps(sigma)
    R = (len(taps) - 1) // 2
    for a in range(g.dim):
        ax = g.npax(a)
        n = x.shape[ax]
        out = np.zeros_like(x)
        for j in range(-R, R + 1):
            # out[c] += taps[j] * x[c + j]  (zero outside the grid)
            lo, hi = max(0, -j), min(n, n - j)
            if lo >= hi:
                continue
            dst = [slice(None)] * g.dim
            src = [slice(None)] * g.dim
            dst[ax] = slice(lo, hi)
            src[ax] = slice(lo + j, hi + j)
            out[tuple(dst)] += taps[j + R] * x[tuple(src)]
        x = out
    return x.ravel()


def apply_metric(g: Grid, e, levels):
    out = np.array(e, dtype=np.float64).ravel().copy()
    for l in range(1, levels + 1):
        s = 2.0 ** (l - 1)
        out += blur(g, blur(g, e, s), s)
    return out
