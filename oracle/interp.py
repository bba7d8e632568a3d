"""Clamped multilinear interpolation on a lattice, with its position
derivative and its transpose (needed because the semi-Lagrangian operator is
used in place of the paper's upwind exponential, Sec. 4.1: any advection
operator with partials in density and velocity is admissible).

Convention for a lattice with M_a nodes along axis a (index coordinates):
  clamp:     Yc_a = clamp(Y_a, 0, M_a - 1)
  base cell: i0_a = min(floor(Yc_a), M_a - 2),  t_a = Yc_a - i0_a in [0, 1]
  value:     sum over the 2^d corners of prod_a (t_a or 1 - t_a) * q[corner]
  dvalue/dY_a: the derivative of that multilinear function in cell i0, times
             the clamp derivative, which is 1 on the closed box [0, M_a - 1]
             and 0 outside it.

Every function takes a batch: q has shape (B, M) (B independent lattice
functions, flattened with x fastest) and Y has shape (B, P, d); point p of
batch b is evaluated on q[b].
"""
import itertools
import numpy as np


def stencil(Y, extent):
    """Corner indices (flat, within one lattice) and weights for points Y of
    shape (..., d), x first.  Returns a list of (flat_index, weight, dweight)
    with dweight of shape (..., d)."""
    d = Y.shape[-1]
    i0, t, inside = [], [], []
    for a in range(d):
        M = extent[a]
        y = Y[..., a]
        yc = np.clip(y, 0.0, M - 1.0)
        i = np.minimum(np.floor(yc), M - 2).astype(np.int64)
        i0.append(i)
        t.append(yc - i)
        inside.append(((y >= 0.0) & (y <= M - 1.0)).astype(np.float64))
    stride = [1] * d
    for a in range(1, d):
        stride[a] = stride[a - 1] * extent[a - 1]
    out = []
    for bits in itertools.product((0, 1), repeat=d):
        idx = np.zeros(Y.shape[:-1], dtype=np.int64)
        w = np.ones(Y.shape[:-1])
        for a in range(d):
            idx += (i0[a] + bits[a]) * stride[a]
            w = w * (t[a] if bits[a] else 1.0 - t[a])
        dw = np.zeros(Y.shape)
        for a in range(d):
            prod = (1.0 if bits[a] else -1.0) * inside[a]
            for b in range(d):
                if b != a:
                    prod = prod * (t[b] if bits[b] else 1.0 - t[b])
            dw[..., a] = prod
        out.append((idx, w, dw))
    return out


def interp(q, Y, extent):
    """Values, shape (B, P)."""
    val = np.zeros(Y.shape[:-1])
    for idx, w, _ in stencil(Y, extent):
        val += w * np.take_along_axis(q, idx, axis=1)
    return val


def interp_grad(q, Y, extent):
    """Derivative of the interpolant with respect to the position, (B, P, d)."""
    g = np.zeros(Y.shape)
    for idx, _, dw in stencil(Y, extent):
        g += dw * np.take_along_axis(q, idx, axis=1)[..., None]
    return g


def interp_transpose(mu, Y, extent):
    """Transpose of q -> interp(q, Y) applied to mu (shape (B, P)); (B, M)."""
    B = Y.shape[0]
    M = int(np.prod(extent))
    out = np.zeros(B * M)
    base = (np.arange(B, dtype=np.int64) * M)[:, None]
    for idx, w, _ in stencil(Y, extent):
        out += np.bincount((idx + base).ravel(), weights=(w * mu).ravel(), minlength=B * M)
    return out.reshape(B, M)
