// Semi-Lagrangian advection kernels and their transposes.
//
// Density (Sec. 3.1 eq:Conv; Sec. 4.1 admits any advection operator whose
// partials are available): one Euler backtrace per cell centre with the
// cell-centred velocity, Y = X - (dt/h) vbar, then clamped multilinear
// interpolation.  Velocity (replaces the implicit self-advection of eq:NSA):
// every interior a-face backtraces with its own component and the 4-face
// averages of the others and interpolates v_a on the a-face lattice.
//
// Launch shape: one thread per cell or face, blockIdx.y = batch slice.
// The transposes scatter with global atomics (the foot point of a
// backtrace is data dependent), so their summation order is not fixed.
#pragma once
#include "common.hpp"

namespace stfas {

// Cell-centred velocity component a of cell (i, j, k).
template <typename T>
__device__ inline T vbar(const Grid& g, const T* v, int a, int i, int j, int k) {
    const int lo = face_index(g, a, i, j, k);
    const int hi = face_index(g, a, i + (a == 0), j + (a == 1), k + (a == 2));
    return (T)0.5 * (v[lo] + v[hi]);
}

// Velocity sampled at interior a-face (i, j, k): own component, and for
// b != a the mean of v_b at I - e_a, I - e_a + e_b, I and I + e_b.
template <typename T, int D>
__device__ inline void face_velocity(const Grid& g, const T* v, int a, int i, int j, int k, T* vh) {
    for (int b = 0; b < D; ++b) {
        if (b == a) {
            vh[b] = v[face_index(g, a, i, j, k)];
            continue;
        }
        const int ia = i - (a == 0), ja = j - (a == 1), ka = k - (a == 2);
        const int db0 = (b == 0), db1 = (b == 1), db2 = (b == 2);
        const T s = v[face_index(g, b, ia, ja, ka)] + v[face_index(g, b, ia + db0, ja + db1, ka + db2)] +
                    v[face_index(g, b, i, j, k)] + v[face_index(g, b, i + db0, j + db1, k + db2)];
        vh[b] = (T)0.25 * s;
    }
}

// ---------------------------------------------------------------- density
template <typename T, int D>
__global__ void k_advect(Grid g, T cfl, const T* __restrict__ rho, const T* __restrict__ v, T* __restrict__ out,
                         long rs, long vs) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    rho += blockIdx.y * rs;
    v += blockIdx.y * vs;
    out += blockIdx.y * rs;
    const int i = c % g.n[0], j = (c / g.n[0]) % g.n[1], k = c / (g.n[0] * g.n[1]);
    const int idx[3] = {i, j, k};
    T y[3];
    for (int a = 0; a < D; ++a) y[a] = -cfl * vbar(g, v, a, i, j, k);
    Interp<T, D> it;
    it.setup_disp(idx, y, g.n[0], g.n[1], g.n[2]);
    out[c] = it.value(rho);
}

// out += W(v)^T mu  (out must be initialised by the caller).
template <typename T, int D>
__global__ void k_advect_T(Grid g, T cfl, const T* __restrict__ mu, const T* __restrict__ v, T* out, long rs,
                           long vs) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    mu += blockIdx.y * rs;
    v += blockIdx.y * vs;
    out += blockIdx.y * rs;
    const T m = mu[c];
    if (m == (T)0) return;
    const int i = c % g.n[0], j = (c / g.n[0]) % g.n[1], k = c / (g.n[0] * g.n[1]);
    const int idx[3] = {i, j, k};
    T y[3];
    for (int a = 0; a < D; ++a) y[a] = -cfl * vbar(g, v, a, i, j, k);
    Interp<T, D> it;
    it.setup_disp(idx, y, g.n[0], g.n[1], g.n[2]);
#pragma unroll
    for (int q = 0; q < (1 << D); ++q) {
        const T w = it.weight(q) * m;
        if (w != (T)0) atomic_add(out + it.corner(q), w);
    }
}

// gv = vt + scale * (dA(rho, v)/dv)^T mu on interior faces, 0 on walls.
// Face I collects half of  mu_c (-dt/h) d_a I[rho](Y_c)  from the two cells
// c = I - e_a and I that average it into their centre velocity.
template <typename T, int D>
__global__ void k_advect_dv_T(Grid g, T cfl, const T* __restrict__ mu, const T* __restrict__ rho,
                              const T* __restrict__ v, const T* __restrict__ vt, T scale, T* __restrict__ gv,
                              long rs, long vs) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= g.nface) return;
    mu += blockIdx.y * rs;
    rho += blockIdx.y * rs;
    v += blockIdx.y * vs;
    gv += blockIdx.y * vs;
    if (vt) vt += blockIdx.y * vs;
    int a, i, j, k;
    face_decode(g, f, a, i, j, k);
    if (!face_interior(g, a, i, j, k)) {
        gv[f] = (T)0;
        return;
    }
    T acc = 0;
    for (int side = 0; side < 2; ++side) {
        const int ci = i - (side == 0 && a == 0), cj = j - (side == 0 && a == 1), ck = k - (side == 0 && a == 2);
        const int c = cell_index(g, ci, cj, ck);
        const T m = mu[c];
        if (m == (T)0) continue;
        const int idx[3] = {ci, cj, ck};
        T y[3];
        for (int b = 0; b < D; ++b) y[b] = -cfl * vbar(g, v, b, ci, cj, ck);
        Interp<T, D> it;
        it.setup_disp(idx, y, g.n[0], g.n[1], g.n[2]);
        T gr[3];
        it.grad(rho, gr);
        acc += (T)0.5 * (-cfl) * m * (a == 0 ? gr[0] : (a == 1 ? gr[1] : gr[D - 1]));
    }
    gv[f] = (vt ? vt[f] : (T)0) + scale * acc;
}

// ---------------------------------------------------------------- velocity
// out = S(v) + dt u on interior faces (u may be null), 0 on walls.
template <typename T, int D>
__global__ void k_self_advect(Grid g, T cfl, T dt, const T* __restrict__ v, const T* __restrict__ u,
                              T* __restrict__ out, long vs) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= g.nface) return;
    v += blockIdx.y * vs;
    out += blockIdx.y * vs;
    if (u) u += blockIdx.y * vs;
    int a, i, j, k;
    face_decode(g, f, a, i, j, k);
    if (!face_interior(g, a, i, j, k)) {
        out[f] = (T)0;
        return;
    }
    T vh[3];
    face_velocity<T, D>(g, v, a, i, j, k, vh);
    const int idx[3] = {i, j, k};
    T y[3];
    for (int b = 0; b < D; ++b) y[b] = -cfl * vh[b];
    Interp<T, D> it;
    it.setup_disp(idx, y, face_ext(g, a, 0), face_ext(g, a, 1), face_ext(g, a, 2));
    T s = it.value(v + g.foff[a]);
    if (u) s += dt * u[f];
    out[f] = s;
}

// out += scale * J_S(v)^T y.  Per interior a-face I: the interpolation
// weights scatter y_I onto the a-face lattice, and the foot-point term
// y_I (-dt/h) grad_Y I[v_a] returns to the sampled velocities (component a
// to v_a[I], component b != a by quarters to the four v_b faces averaged at
// I).  Contributions that land on wall faces are dropped.
template <typename T, int D>
__global__ void k_self_advect_T(Grid g, T cfl, const T* __restrict__ v, const T* __restrict__ y, T scale, T* out,
                                long vs) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= g.nface) return;
    v += blockIdx.y * vs;
    y += blockIdx.y * vs;
    out += blockIdx.y * vs;
    int a, i, j, k;
    face_decode(g, f, a, i, j, k);
    if (!face_interior(g, a, i, j, k)) return;
    const T yv = y[f] * scale;
    if (yv == (T)0) return;
    T vh[3];
    face_velocity<T, D>(g, v, a, i, j, k, vh);
    const int idx[3] = {i, j, k};
    T yy[3];
    for (int b = 0; b < D; ++b) yy[b] = -cfl * vh[b];
    const int ex = face_ext(g, a, 0), ey = face_ext(g, a, 1), ez = face_ext(g, a, 2);
    Interp<T, D> it;
    it.setup_disp(idx, yy, ex, ey, ez);
    const T* va = v + g.foff[a];
    T* oa = out + g.foff[a];
    T gr[3];
    it.grad(va, gr);
#pragma unroll
    for (int q = 0; q < (1 << D); ++q) {
        const T w = it.weight(q) * yv;
        if (w == (T)0) continue;
        // corner lattice coordinate along a decides whether it is a wall
        const int ia0 = a == 0 ? it.ax[0].i0 : (a == 1 ? it.ax[1].i0 : it.ax[D - 1].i0);
        const int ca = ia0 + ((q >> a) & 1);
        if (ca == 0 || ca == g.n[a]) continue;
        atomic_add(oa + it.corner(q), w);
    }
    for (int b = 0; b < D; ++b) {
        const T gb = yv * (-cfl) * gr[b];
        if (gb == (T)0) continue;
        if (b == a) {
            atomic_add(out + f, gb);
            continue;
        }
        const T qv = (T)0.25 * gb;
        const int ia = i - (a == 0), ja = j - (a == 1), ka = k - (a == 2);
        const int db0 = (b == 0), db1 = (b == 1), db2 = (b == 2);
        const int bi = b == 0 ? i : (b == 1 ? j : k);   // b-coordinate of I (and of I - e_a)
        // faces at b-coordinate bi (I, I - e_a) are walls when bi == 0; at bi + 1 when bi + 1 == n_b
        if (bi != 0) {
            atomic_add(out + face_index(g, b, ia, ja, ka), qv);
            atomic_add(out + face_index(g, b, i, j, k), qv);
        }
        if (bi + 1 != g.n[b]) {
            atomic_add(out + face_index(g, b, ia + db0, ja + db1, ka + db2), qv);
            atomic_add(out + face_index(g, b, i + db0, j + db1, k + db2), qv);
        }
    }
}

}  // namespace stfas
