"""Spacetime restriction R and prolongation P (Sec. 4.3: plain multilinear
interpolation on scalar and vector fields; semi-coarsening in space only, so
every level keeps all N time steps).

P interpolates the coarse lattice at the fine sample positions, written in
coarse index coordinates:
  cell lattice:           fine cell i   -> (i + 1/2)/2 - 1/2
  a-face lattice, axis a: fine face I   -> I/2
  a-face lattice, b != a: fine index j  -> (j + 1/2)/2 - 1/2
with the clamp of the interpolation (constant extrapolation at the walls of
the cell-centred directions).  Coarse wall faces hold zero, so P gives zero
on fine wall faces.  R = 2^-d P^T, with the coarse wall rows set to zero.
"""
import numpy as np
import scipy.sparse as sp

from .grid import Grid
from .interp import stencil


def _sample_positions(fine_ext, axis_kind):
    """axis_kind[b] is 'node' (face normal axis) or 'cell' for each axis b."""
    d = len(fine_ext)
    grids = np.meshgrid(*[np.arange(fine_ext[b], dtype=np.float64) for b in reversed(range(d))],
                        indexing="ij")
    cols = []
    for b in range(d):
        idx = grids[d - 1 - b].ravel()
        cols.append(idx / 2.0 if axis_kind[b] == "node" else (idx + 0.5) / 2.0 - 0.5)
    return np.stack(cols, axis=1)


def _interp_matrix(fine_ext, coarse_ext, axis_kind):
    Y = _sample_positions(fine_ext, axis_kind)
    rows, cols, vals = [], [], []
    P = Y.shape[0]
    for idx, w, _ in stencil(Y, coarse_ext):
        rows.append(np.arange(P))
        cols.append(idx)
        vals.append(w)
    m = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(P, int(np.prod(coarse_ext))))
    return m.tocsr()


class Transfer:
    def __init__(self, fine: Grid):
        self.fine = fine
        self.coarse = fine.coarse()
        d = fine.dim
        self.Pc = _interp_matrix(fine.n, self.coarse.n, ["cell"] * d)
        self.Pf = []
        for a in range(d):
            kind = ["node" if b == a else "cell" for b in range(d)]
            self.Pf.append(_interp_matrix(fine.face_lattice_extent(a), self.coarse.face_lattice_extent(a), kind))
        self.scale = 2.0 ** (-d)
        self.cmask = self.coarse.interior_mask()

    def prolong_cells(self, xc):
        return self.Pc @ xc

    def restrict_cells(self, xf):
        return self.scale * (self.Pc.T @ xf)

    def prolong_faces(self, xc):
        parts = self.coarse.split(xc)
        return self.fine.join([self.Pf[a] @ parts[a].ravel() for a in range(self.fine.dim)])

    def restrict_faces(self, xf):
        parts = self.fine.split(xf)
        out = self.coarse.join([self.scale * (self.Pf[a].T @ parts[a].ravel()) for a in range(self.fine.dim)])
        return out * self.cmask

    def restrict_state(self, x):
        """x = [faces, cells, faces, cells] with a leading time axis."""
        out = []
        for k, a in enumerate(x):
            f = self.restrict_faces if k % 2 == 0 else self.restrict_cells
            out.append(np.stack([f(a[j]) for j in range(a.shape[0])]))
        return out

    def prolong_state(self, x):
        out = []
        for k, a in enumerate(x):
            f = self.prolong_faces if k % 2 == 0 else self.prolong_cells
            out.append(np.stack([f(a[j]) for j in range(a.shape[0])]))
        return out

    def restrict_faces_seq(self, a):
        return np.stack([self.restrict_faces(a[j]) for j in range(a.shape[0])])
