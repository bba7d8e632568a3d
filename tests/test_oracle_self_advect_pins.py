"""Pins of the oracle's semi-Lagrangian velocity self-advection S and of its
transpose J_S^T against things other than the oracle itself.  CPU only.

S interpolates with the C1 variant of multilinear weights: each fraction t
of the foot point's lattice coordinate is replaced by s(t) = t^2 (3 - 2t).

1. Closed form.  For a linear, divergence-free velocity field V(x) sampled
   at the face centres, the four-face average of component b at an a-face
   equals V_b at that face's centre (the four b-faces sit symmetrically
   around it).  The backtrace from lattice index I is then exactly
   Y = I - (dt/h) V(X), and multilinear weights built on s(t) applied to a
   linear function q give q at the lattice point floor(Y) + s(Y - floor(Y))
   (the weights of each axis sum to one and the function separates by
   axis).  So, away from the walls, S(v) at an a-face is V_a at the
   position of that lattice point.  A wrong neighbour set in the average, a
   wrong axis, a sign error in the backtrace, a misplaced face centre or a
   plain (non-smoothstep) weight each change the value.
2. An independent implementation in plain torch: one loop over faces, the
   neighbours named explicitly, floor/clamp interpolation on the face
   lattice with smoothstep fractions.  Its values must equal the oracle's,
   and torch autograd through it gives J_S(v)^T y, which must equal the
   oracle's hand-written transpose (the derivative convention at the clamp
   is the one autograd gives for floor/clamp: clamp slope 1 on the closed
   box; at lattice nodes s'(t) vanishes on both sides).
"""
import itertools

import numpy as np
import pytest

import synthetic
from oracle import advect
from oracle.grid import Grid


def _face_centre(g, a, idx):
    """Cell-centre coordinates of the a-face with lattice index idx (x first):
    the face between cells idx - e_a and idx sits half a cell below idx along a."""
    return np.array([idx[b] - (0.5 if b == a else 0.0) for b in range(g.dim)])


def _sample(g, V):
    """Face field holding V at every interior face centre, zero on walls."""
    parts = [np.zeros(s) for s in g.face_shapes]
    for a in range(g.dim):
        ext = g.face_lattice_extent(a)
        for idx in itertools.product(*[range(e) for e in ext]):
            if idx[a] in (0, g.n[a]):
                continue
            parts[a][tuple(reversed(idx))] = V(_face_centre(g, a, idx))[a]
    return g.join(parts)


def _linear_field(dim, rng):
    """A linear field whose component a does not depend on x_a, so it is
    divergence free; magnitudes keep backtraces under one cell."""
    if dim == 2:
        al, be, ga, de = rng.uniform(-0.3, 0.3, 4)
        sl = rng.uniform(-0.04, 0.04, 2)
        return lambda X: np.array([al + sl[0] * (X[1] - 5.0), ga + sl[1] * (X[0] - 5.0)])
    c = rng.uniform(-0.25, 0.25, 3)
    s = rng.uniform(-0.03, 0.03, 6)
    return lambda X: np.array([c[0] + s[0] * (X[1] - 4.0) + s[1] * (X[2] - 4.0),
                               c[1] + s[2] * (X[2] - 4.0) + s[3] * (X[0] - 4.0),
                               c[2] + s[4] * (X[0] - 4.0) + s[5] * (X[1] - 4.0)])


@pytest.mark.parametrize("n", [(10, 9), (9, 8, 10)])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_self_advect_linear_field_closed_form(n, seed):
    rng = np.random.default_rng(100 + seed)
    g = Grid(n)
    V = _linear_field(g.dim, rng)
    cfl = 0.9                                   # dt / h
    v = _sample(g, V)
    S = g.split(advect.self_advect(g, v, cfl * g.h))
    checked = 0
    for a in range(g.dim):
        ext = g.face_lattice_extent(a)
        for idx in itertools.product(*[range(e) for e in ext]):
            # at least two lattice steps from every wall: the four averaged
            # b-faces are interior, and the backtrace (under one cell) stays
            # among interior a-faces without clamping
            if any(idx[b] < 2 or idx[b] > ext[b] - 3 for b in range(g.dim)):
                continue
            X = _face_centre(g, a, idx)
            Y = np.array(idx, dtype=np.float64) - cfl * V(X)        # lattice index of the foot point
            base = np.floor(Y)
            t = Y - base
            Ys = base + t * t * (3.0 - 2.0 * t)
            want = V(_face_centre(g, a, Ys))[a]
            got = S[a][tuple(reversed(idx))]
            assert abs(got - want) < 1e-13, (a, idx, got, want)
            checked += 1
    assert checked > 20


def _torch_self_advect(n, v_parts, cfl):
    """S(v) written independently: loop over interior faces; the velocity at
    an a-face is v_a there and, for b != a, the mean of the four b-faces of
    the two cells that share the face; one Euler backtrace in lattice index
    space; floor/clamp multilinear interpolation on the a-face lattice with
    each fraction passed through the smoothstep t^2 (3 - 2t)."""
    import torch
    dim = len(n)

    def get(a, idx):                              # v_a at lattice index idx (x first)
        return v_parts[a][tuple(reversed(idx))]

    out = [torch.zeros_like(p) for p in v_parts]
    for a in range(dim):
        ext = [n[b] + (1 if b == a else 0) for b in range(dim)]
        for idx in itertools.product(*[range(e) for e in ext]):
            if idx[a] in (0, n[a]):
                continue
            vel = []
            for b in range(dim):
                if b == a:
                    vel.append(get(a, idx))
                    continue
                lo_cell = list(idx)
                lo_cell[a] -= 1                      # the cell below the face along a
                hi_cell = list(idx)                  # the cell above it
                quad = []
                for cell in (lo_cell, hi_cell):
                    low_b = list(cell)               # that cell's low b-face
                    high_b = list(cell)
                    high_b[b] += 1                   # and its high b-face
                    quad += [get(b, low_b), get(b, high_b)]
                vel.append(0.25 * (quad[0] + quad[1] + quad[2] + quad[3]))
            pos = [torch.clamp(idx[b] - cfl * vel[b], 0.0, ext[b] - 1.0) for b in range(dim)]
            base = [int(min(np.floor(float(pos[b].detach())), ext[b] - 2)) for b in range(dim)]
            frac = [pos[b] - base[b] for b in range(dim)]
            frac = [f * f * (3.0 - 2.0 * f) for f in frac]          # smoothstep
            val = 0.0
            for bits in itertools.product((0, 1), repeat=dim):
                wgt = 1.0
                for b in range(dim):
                    wgt = wgt * (frac[b] if bits[b] else 1.0 - frac[b])
                node = [base[b] + bits[b] for b in range(dim)]
                val = val + wgt * get(a, node)
            o = out[a].clone()
            o[tuple(reversed(idx))] = val
            out[a] = o
    return out


@pytest.mark.parametrize("n,cfl,scale", [((6, 5), 0.7, 1.0), ((6, 5), 1.3, 2.5), ((4, 5, 3), 0.8, 1.5)])
def test_self_advect_and_transpose_against_torch(n, cfl, scale):
    import torch
    rng = np.random.default_rng(7 + len(n))
    g = Grid(n)
    v = synthetic.random_faces(n, rng, scale)
    y = synthetic.random_faces(n, rng, 1.0)
    vt = [torch.tensor(p.copy(), requires_grad=True) for p in g.split(v)]
    out = _torch_self_advect(g.n, vt, cfl)
    s_ref = g.join([o.detach().numpy() for o in out])
    assert np.allclose(s_ref, advect.self_advect(g, v, cfl * g.h), rtol=0, atol=1e-14)
    loss = sum((o * torch.tensor(yp)).sum() for o, yp in zip(out, g.split(y)))
    loss.backward()
    jt = g.join([p.grad.numpy() for p in vt]) * g.interior_mask()
    assert np.allclose(jt, advect.self_advect_T(g, v, y, cfl * g.h), rtol=0, atol=1e-13)
