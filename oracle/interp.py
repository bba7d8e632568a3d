"""Clamped multilinear interpolation on a lattice, with its position
derivative and its transpose (needed because the semi-Lagrangian operator is
used in place of the paper's upwind exponential, Sec. 4.1: any advection
operator with partials in density and velocity is admissible).

Convention for a lattice with M_a nodes along axis a (index coordinates;
the C1 variant of Stencil replaces t_a below by its smoothstep):
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


class Stencil:
    """Corner indices, weights and (on demand) position-derivative weights of
    the interpolation at points Y (shape (..., d), x first).

    c1=True gives the C1 variant: every fraction t is replaced by the
    smoothstep s(t) = t^2 (3 - 2 t) before the multilinear weights are
    formed, so the weights stay convex and interpolate the nodes, and the
    position derivative picks up the factor s'(t) = 6 t (1 - t), which
    vanishes at every lattice line: the interpolant is continuously
    differentiable in Y (the plain multilinear one has a gradient that jumps
    across lattice lines)."""

    def __init__(self, Y, extent, c1=False):
        d = Y.shape[-1]
        self.d = d
        self.i0, self.t, self.inside = [], [], []
        for a in range(d):
            M = extent[a]
            y = Y[..., a]
            yc = np.clip(y, 0.0, M - 1.0)
            i = np.minimum(np.floor(yc), M - 2).astype(np.int64)
            t = yc - i
            inside = ((y >= 0.0) & (y <= M - 1.0)).astype(np.float64)
            if c1:
                inside = inside * 6.0 * t * (1.0 - t)
                t = t * t * (3.0 - 2.0 * t)
            self.i0.append(i)
            self.t.append(t)
            self.inside.append(inside)
        self.stride = [1] * d
        for a in range(1, d):
            self.stride[a] = self.stride[a - 1] * extent[a - 1]
        self.bits = list(itertools.product((0, 1), repeat=d))
        self.idx, self.w = [], []
        fac = [(1.0 - self.t[a], self.t[a]) for a in range(d)]
        for bits in self.bits:
            idx = sum((self.i0[a] + bits[a]) * self.stride[a] for a in range(d))
            w = fac[0][bits[0]]
            for a in range(1, d):
                w = w * fac[a][bits[a]]
            self.idx.append(idx)
            self.w.append(w)
        self._fac = fac

    def dweights(self):
        """d weight / d Y_a for every corner: list of d arrays per corner."""
        out = []
        for bits in self.bits:
            per = []
            for a in range(self.d):
                prod = self.inside[a] if bits[a] else -self.inside[a]
                for b in range(self.d):
                    if b != a:
                        prod = prod * self._fac[b][bits[b]]
                per.append(prod)
            out.append(per)
        return out


def stencil(Y, extent):
    """List of (flat_index, weight, dweight) per corner, dweight of shape (..., d)."""
    st = Stencil(Y, extent)
    return [(i, w, np.stack(dw, axis=-1)) for i, w, dw in zip(st.idx, st.w, st.dweights())]


def interp(q, Y, extent, st=None):
    """Values, shape (B, P)."""
    st = Stencil(Y, extent) if st is None else st
    val = np.zeros(Y.shape[:-1])
    for idx, w in zip(st.idx, st.w):
        val += w * np.take_along_axis(q, idx, axis=1)
    return val


def interp_grad(q, Y, extent, st=None):
    """Derivative of the interpolant with respect to the position, (B, P, d)."""
    st = Stencil(Y, extent) if st is None else st
    g = np.zeros(Y.shape)
    for idx, dw in zip(st.idx, st.dweights()):
        qv = np.take_along_axis(q, idx, axis=1)
        for a in range(st.d):
            g[..., a] += dw[a] * qv
    return g


def interp_transpose(mu, Y, extent, st=None):
    """Transpose of q -> interp(q, Y) applied to mu (shape (B, P)); (B, M)."""
    st = Stencil(Y, extent) if st is None else st
    B = Y.shape[0]
    M = int(np.prod(extent))
    out = np.zeros(B * M)
    base = (np.arange(B, dtype=np.int64) * M)[:, None]
    for idx, w in zip(st.idx, st.w):
        out += np.bincount((idx + base).ravel(), weights=(w * mu).ravel(), minlength=B * M)
    return out.reshape(B, M)
