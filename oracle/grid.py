"""Staggered MAC grid (Sec. 3.1: velocity and forces on faces, density and
pressures at cell centres) with zero-Neumann walls.

Layout (shared with the device path only as a data convention):
  * cells: C-order array of shape (n2, n1, n0) in 3D, (n1, n0) in 2D; axis
    a = 0 is x (the last NumPy axis).
  * a-faces: the cell shape with one extra entry along axis a.  Face index I
    sits between cells I - e_a and I; I_a in {0, n_a} are wall faces, which
    are identically zero in every face field (no flow through walls).
  * a face field is one flat vector: x-faces, then y-faces, then z-faces.
"""
import numpy as np


class Grid:
    def __init__(self, n, h=None):
        self.n = tuple(int(x) for x in n)          # (n0, n1[, n2]), x first
        self.dim = len(self.n)
        assert self.dim in (2, 3)
        self.h = 1.0 / self.n[0] if h is None else float(h)
        self.cell_shape = tuple(reversed(self.n))
        self.ncell = int(np.prod(self.n))
        self.face_shapes = []
        for a in range(self.dim):
            s = list(self.cell_shape)
            s[self.npax(a)] += 1
            self.face_shapes.append(tuple(s))
        self.face_counts = [int(np.prod(s)) for s in self.face_shapes]
        self.nface = int(sum(self.face_counts))
        self.face_offsets = np.cumsum([0] + self.face_counts)

    def npax(self, a):
        """NumPy axis of spatial axis a (x is the last NumPy axis)."""
        return self.dim - 1 - a

    def coarse(self):
        return Grid(tuple(x // 2 for x in self.n), 2.0 * self.h)

    # ----- face-field helpers -------------------------------------------
    def split(self, f):
        """Views of a flat face vector as the d per-axis arrays."""
        return [f[self.face_offsets[a]:self.face_offsets[a + 1]].reshape(self.face_shapes[a])
                for a in range(self.dim)]

    def join(self, parts):
        return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])

    def zeros_faces(self):
        return np.zeros(self.nface)

    def zeros_cells(self):
        return np.zeros(self.ncell)

    def interior_mask(self):
        """1 on interior faces, 0 on wall faces (flat face vector)."""
        if getattr(self, "_imask", None) is None:
            self._imask = self._interior_mask()
        return self._imask

    def _interior_mask(self):
        parts = []
        for a in range(self.dim):
            m = np.ones(self.face_shapes[a])
            ax = self.npax(a)
            sl = [slice(None)] * self.dim
            sl[ax] = 0
            m[tuple(sl)] = 0
            sl[ax] = self.n[a]
            m[tuple(sl)] = 0
            parts.append(m)
        return self.join(parts)

    def sl_along(self, a, start, stop):
        """Index tuple selecting [start:stop] along spatial axis a."""
        sl = [slice(None)] * self.dim
        sl[self.npax(a)] = slice(start, stop)
        return tuple(sl)

    def cell_positions(self):
        """Index-space position of each cell centre, shape (ncell, d), columns x, y[, z]."""
        if getattr(self, "_cpos", None) is None:
            self._cpos = self._cell_positions()
        return self._cpos

    def _cell_positions(self):
        grids = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in self.cell_shape], indexing="ij")
        return np.stack([grids[self.npax(a)].ravel() for a in range(self.dim)], axis=1)

    def face_positions(self, a):
        """Index-space position of every a-face in the a-face lattice, shape (count, d)."""
        cache = self.__dict__.setdefault("_fpos", {})
        if a not in cache:
            cache[a] = self._face_positions(a)
        return cache[a]

    def _face_positions(self, a):
        shape = self.face_shapes[a]
        grids = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
        return np.stack([grids[self.npax(b)].ravel() for b in range(self.dim)], axis=1)

    def face_lattice_extent(self, a):
        """Lattice extent (x, y[, z] order) of the a-face lattice."""
        return tuple(self.n[b] + (1 if b == a else 0) for b in range(self.dim))


def div(g, w, h=None):
    """(D w)_c = sum_a (w_a[c + e_a] - w_a[c]) / h  (wall faces hold zero).
    w may be one face field or a batch (one per row)."""
    h = g.h if h is None else h
    w = np.asarray(w, dtype=np.float64)
    single = w.ndim == 1
    w = w[None] if single else w
    B = w.shape[0]
    out = np.zeros((B,) + g.cell_shape)
    for a in range(g.dim):
        wa = w[:, g.face_offsets[a]:g.face_offsets[a + 1]].reshape((B,) + g.face_shapes[a])
        out += np.diff(wa, axis=1 + g.npax(a)) / h
    out = out.reshape(B, -1)
    return out[0] if single else out


def grad(g, phi, h=None):
    """(G phi)_I = (phi[I] - phi[I - e_a]) / h on interior faces, 0 on walls.
    phi may be one cell field or a batch (one per row)."""
    h = g.h if h is None else h
    phi = np.asarray(phi, dtype=np.float64)
    single = phi.ndim == 1
    phi = phi[None] if single else phi
    B = phi.shape[0]
    phi = phi.reshape((B,) + g.cell_shape)
    out = np.zeros((B, g.nface))
    for a in range(g.dim):
        ga = out[:, g.face_offsets[a]:g.face_offsets[a + 1]].reshape((B,) + g.face_shapes[a])
        ga[(slice(None),) + g.sl_along(a, 1, g.n[a])] = np.diff(phi, axis=1 + g.npax(a)) / h
    return out[0] if single else out


def laplacian(g, phi, h=None):
    """Neumann 5/7-point Laplacian L = D G."""
    return div(g, grad(g, phi, h), h)
