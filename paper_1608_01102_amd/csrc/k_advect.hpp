// Semi-Lagrangian advection kernels and their transposes.
//
// Density (Sec. 3.1 eq:Conv; Sec. 4.1 admits any advection operator whose
// partials are available): one Euler backtrace per cell centre with the
// cell-centred velocity, Y = X - (dt/h) vbar, then clamped multilinear
// interpolation.  Velocity (replaces the implicit self-advection of eq:NSA):
// every interior a-face backtraces with its own component and the 4-face
// averages of the others and interpolates v_a on the a-face lattice with the
// C1 (smoothstep) weights of Interp::c1, so that the foot-point term of its
// transpose, and with it the KKT residual of the velocity subproblem, is
// continuous in v.
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
    it.c1();
    T s = it.value(v + g.foff[a]);
    if (u) s += dt * u[f];
    out[f] = s;
}

// J_S(v)^T y for one source, a-face (i, j, k) of one slice, straight into
// out with global atomics: the same contributions as the tiled kernel below,
// without its LDS window and barriers.  Used on small levels, where a launch
// is a chain of dependent memory steps and the atomics are few.
template <typename T, int D>
__device__ inline void self_advect_T_source(const Grid& g, T cfl, const T* __restrict__ v, const T* __restrict__ y,
                                            T scale, T* out, int a, int i, int j, int k) {
    if (!face_interior(g, a, i, j, k)) return;
    const int f = face_index(g, a, i, j, k);
    const T yv = y[f] * scale;
    const int ex = face_ext(g, a, 0), ey = face_ext(g, a, 1), ez = face_ext(g, a, 2);
    T vh[3];
    face_velocity<T, D>(g, v, a, i, j, k, vh);
    const int idx[3] = {i, j, k};
    T dl[3];
    for (int b = 0; b < D; ++b) dl[b] = -cfl * vh[b];
    Interp<T, D> it;
    it.setup_disp(idx, dl, ex, ey, ez);
    it.c1();
    T gr[3];
    it.grad(v + g.foff[a], gr);
    if (yv == (T)0) return;
    const int c0[3] = {it.ax[0].i0, it.ax[1].i0, D == 3 ? it.ax[D - 1].i0 : 0};
#pragma unroll
    for (int q = 0; q < (1 << D); ++q) {
        const T w = it.weight(q) * yv;
        if (w == (T)0) continue;
        const int ci = c0[0] + (q & 1), cj = c0[1] + ((q >> 1) & 1), ck = D == 3 ? c0[2] + ((q >> 2) & 1) : 0;
        const int ca = a == 0 ? ci : (a == 1 ? cj : ck);
        if (ca == 0 || ca == g.n[a]) continue;          // wall node of the a-lattice
        atomic_add(out + face_index(g, a, ci, cj, ck), w);
    }
#pragma unroll
    for (int b = 0; b < D; ++b) {
        const T gb = yv * (-cfl) * gr[b];
        if (gb == (T)0) continue;
        if (b == a) {
            atomic_add(out + f, gb);
            continue;
        }
        // a quarter to each of the four b-faces averaged at I (walls dropped)
        const T qv = (T)0.25 * gb;
        const int ia = i - (a == 0), ja = j - (a == 1), ka = k - (a == 2);
        const int db0 = (b == 0), db1 = (b == 1), db2 = (b == 2);
        const int bi = b == 0 ? i : (b == 1 ? j : k);
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

// out += scale * J_S(v)^T y.  Per interior a-face I: the interpolation
// weights scatter y_I onto the a-face lattice, and the foot-point term
// g_I = y_I (-dt/h) grad_Y I[v_a] returns to the sampled velocities
// (component a to v_a[I], component b != a by quarters to the four v_b
// faces averaged at I).  Contributions that land on wall faces are dropped.
// Tiled: each workgroup takes a tile of a-faces of one time slice
// (blockIdx.y = slice, blockIdx.z = axis a).
//  * weights: accumulated with LDS atomics into a window that covers the
//    tile plus a halo of H nodes; a weight outside the window (a backtrace
//    longer than the halo) goes straight to global memory;
//  * foot-point term: each source stores its d components g_I in an LDS slot
//    of its own (no atomics), and the flush gathers them: an a-node takes
//    the slot of the source at the same node, a b-node J (b != a) a quarter
//    of the b-components of the sources J, J + e_a (when J_b != 0) and
//    J - e_b, J - e_b + e_a (when J_b != n_b) that lie in the tile;
//  * flush: every touched a-window node and every b-node next to the tile
//    is added to global memory once (neighbouring tiles overlap there).
template <int D>
struct TileShape;
template <>
struct TileShape<2> {
    static constexpr int X = 32, Y = 8, Z = 1, H = 3;
};
template <>
struct TileShape<3> {
    static constexpr int X = 8, Y = 8, Z = 4, H = 2;
};

// out += W(v)^T mu with an LDS window per tile of cells (the shape and halo
// of TileShape): each cell scatters its eight (2D: four) weights into the
// window in 64-bit fixed point (scale from the tile's largest weight, so the
// window sums are exact and independent of order; a node takes at most one
// weight per cell of the tile), a weight beyond the halo goes straight to
// global memory, and the window is flushed with one global atomic per
// nonzero node.  blockIdx.x = tile, blockIdx.y = slice.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_advect_T_tiled(Grid g, T cfl, const T* __restrict__ mu,
                                                        const T* __restrict__ v, T* out, long rs, long vs) {
    using TS = TileShape<D>;
    constexpr int H = TS::H;
    constexpr int HZ = D == 3 ? H : 0;
    constexpr int WX = TS::X + 2 * H, WY = TS::Y + 2 * H, WZ = TS::Z + 2 * HZ;
    constexpr int WN = WX * WY * WZ;
    __shared__ unsigned long long win[WN];
    __shared__ T wmax[4];
    mu += blockIdx.y * rs;
    v += blockIdx.y * vs;
    out += blockIdx.y * rs;
    const int ntx = (g.n[0] + TS::X - 1) / TS::X, nty = (g.n[1] + TS::Y - 1) / TS::Y;
    const int tile = blockIdx.x;
    const int tx0 = (tile % ntx) * TS::X, ty0 = ((tile / ntx) % nty) * TS::Y, tz0 = (tile / (ntx * nty)) * TS::Z;
    const int ox = tx0 - H, oy = ty0 - H, oz = tz0 - HZ;
    for (int e = threadIdx.x; e < WN; e += blockDim.x) win[e] = 0ull;
    __syncthreads();
    const int i = tx0 + (int)threadIdx.x % TS::X, j = ty0 + ((int)threadIdx.x / TS::X) % TS::Y;
    const int k = tz0 + (int)threadIdx.x / (TS::X * TS::Y);
    T wq[1 << D];
    int c0[3] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < (1 << D); ++q) wq[q] = 0;
    if (i < g.n[0] && j < g.n[1] && k < g.n[2]) {
        const T m = mu[cell_index(g, i, j, k)];
        if (m != (T)0) {
            const int idx[3] = {i, j, k};
            T y[3];
            for (int a = 0; a < D; ++a) y[a] = -cfl * vbar(g, v, a, i, j, k);
            Interp<T, D> it;
            it.setup_disp(idx, y, g.n[0], g.n[1], g.n[2]);
            c0[0] = it.ax[0].i0;
            c0[1] = it.ax[1].i0;
            c0[2] = D == 3 ? it.ax[D - 1].i0 : 0;
#pragma unroll
            for (int q = 0; q < (1 << D); ++q) wq[q] = it.weight(q) * m;
        }
    }
    T my = 0;
#pragma unroll
    for (int q = 0; q < (1 << D); ++q) my = fmax(my, fabs(wq[q]));
    for (int o = 32; o > 0; o >>= 1) my = fmax(my, __shfl_xor(my, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = my;
    __syncthreads();
    my = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
    // a non-finite weight anywhere in the tile (fmax drops NaNs, so it is
    // tested apart): every weight goes straight to out with float atomics, so
    // that the NaN or Inf reaches the result instead of an undefined integer
    bool nf = false;
#pragma unroll
    for (int q = 0; q < (1 << D); ++q) nf = nf || !isfinite(wq[q]);
    const bool direct = __syncthreads_or(nf) != 0 || !isfinite(my);
    int e2 = 0;
    (void)frexp((double)(direct ? (T)1 : my), &e2);
    const double fx = ldexp(1.0, 52 - e2), ifx = ldexp(1.0, e2 - 52);
#pragma unroll
    for (int q = 0; q < (1 << D); ++q) {
        const T w = wq[q];
        if (w == (T)0) continue;
        const int ci = c0[0] + (q & 1), cj = c0[1] + ((q >> 1) & 1), ck = D == 3 ? c0[2] + ((q >> 2) & 1) : 0;
        const int wx = ci - ox, wy = cj - oy, wz = ck - oz;
        if (!direct && wx >= 0 && wx < WX && wy >= 0 && wy < WY && wz >= 0 && wz < WZ)
            atomicAdd(&win[(wz * WY + wy) * WX + wx], (unsigned long long)llrint((double)w * fx));
        else
            atomic_add(out + cell_index(g, ci, cj, ck), w);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < WN; e += blockDim.x) {
        const int ci = ox + e % WX, cj = oy + (e / WX) % WY, ck = oz + e / (WX * WY);
        if (ci < 0 || cj < 0 || ck < 0 || ci >= g.n[0] || cj >= g.n[1] || ck >= g.n[2]) continue;
        const long long s = (long long)win[e];
        if (s != 0) atomic_add(out + cell_index(g, ci, cj, ck), (T)((double)s * ifx));
    }
}

// Tiled from 131072 cells per launch (at 64^3 x 60: 1506 -> 271 us); below,
// a launch is a short chain of dependent steps and the window's clear and
// flush cost more than the global atomics it saves (128^2, one slice: 2.9
// against 4.2 us), so each cell adds its weights straight into out.
template <typename T, int D>
inline void launch_advect_T(const Grid& g, T cfl, const T* mu, const T* v, T* out, int batch, hipStream_t st) {
    if ((long)g.ncell * batch < 131072) {
        k_advect_T<T, D><<<dim3((g.ncell + 255) / 256, batch), 256, 0, st>>>(g, cfl, mu, v, out, g.ncell, g.nface);
        return;
    }
    using TS = TileShape<D>;
    const int tiles = ((g.n[0] + TS::X - 1) / TS::X) * ((g.n[1] + TS::Y - 1) / TS::Y) *
                      ((g.n[2] + TS::Z - 1) / TS::Z);
    k_advect_T_tiled<T, D><<<dim3(tiles, batch), 256, 0, st>>>(g, cfl, mu, v, out, g.ncell, g.nface);
}

// gq != nullptr: the quarters of the foot-point term that go to the faces of
// the other axes are not added here; instead every a-face of the tile stores
// its components b != a in gq (slice s, k-th axis other than a at
// gq[(2 s + k) F + f]), and k_quarter_gather adds them afterwards as a
// gather (no atomics).
template <typename T, int D>
__device__ inline void self_advect_T_tile(const Grid& g, T cfl, const T* __restrict__ v, const T* __restrict__ y,
                                          T scale, T* out, long vs, int tile, int slice, int a, T* gq = nullptr) {
    using TS = TileShape<D>;
    constexpr int H = TS::H;
    constexpr int WX = TS::X + 2 * H, WY = TS::Y + 2 * H, WZ = (D == 3) ? TS::Z + 2 * H : 1;
    constexpr int WN = WX * WY * WZ;
    constexpr int TN = TS::X * TS::Y * TS::Z;
    // b-nodes next to the tile: the tile grown by one node on each side
    constexpr int BX = TS::X + 2, BY = TS::Y + 2, BZ = (D == 3) ? TS::Z + 2 : 1;
    constexpr int BN = BX * BY * BZ;
    // the window accumulates in 64-bit fixed point (integer LDS atomics are
    // much cheaper than float ones); the scale puts the tile's largest |y|
    // at 2^52, so up to 1024 contributions per node fit and every value
    // keeps 2^-52 of that maximum
    __shared__ unsigned long long win[WN];
    __shared__ T slot[D][TN];
    __shared__ T wmax[4];
    v += slice * vs;
    y += slice * vs;
    out += slice * vs;
    // tile origin in a-lattice coordinates
    const int ex = face_ext(g, a, 0), ey = face_ext(g, a, 1), ez = face_ext(g, a, 2);
    const int ntx = (ex + TS::X - 1) / TS::X, nty = (ey + TS::Y - 1) / TS::Y;
    const int ntz = (D == 3) ? (ez + TS::Z - 1) / TS::Z : 1;
    // the launch covers the axis with the most tiles; the others' extra
    // workgroups have nothing to do (uniform exit before any barrier)
    if (tile >= ntx * nty * ntz) return;
    const int tx0 = (tile % ntx) * TS::X;
    const int ty0 = ((tile / ntx) % nty) * TS::Y;
    const int tz0 = (D == 3) ? (tile / (ntx * nty)) * TS::Z : 0;
    const int ox = tx0 - H, oy = ty0 - H, oz = (D == 3) ? tz0 - H : 0;
    for (int e = threadIdx.x; e < WN; e += blockDim.x) win[e] = 0ull;
    __syncthreads();
    const int lx = threadIdx.x % TS::X, ly = (threadIdx.x / TS::X) % TS::Y, lz = threadIdx.x / (TS::X * TS::Y);
    const int i = tx0 + lx, j = ty0 + ly, k = tz0 + lz;
    T gs[3] = {0, 0, 0};
    T wq[1 << D];
    int c0[3] = {-4, 0, 0};            // x corner far from any real one when the lane has nothing to add
#pragma unroll
    for (int q = 0; q < (1 << D); ++q) wq[q] = 0;
    const bool valid = i < ex && j < ey && (D == 2 || k < ez);
    if (valid && face_interior(g, a, i, j, k)) {
        // y and the velocities are loaded together; a zero y then drops
        // the source (its results are not used, whatever they are)
        const int f = face_index(g, a, i, j, k);
        const T yv = y[f] * scale;
        T vh[3];
        face_velocity<T, D>(g, v, a, i, j, k, vh);
        const int idx[3] = {i, j, k};
        T dl[3];
        for (int b = 0; b < D; ++b) dl[b] = -cfl * vh[b];
        Interp<T, D> it;
        it.setup_disp(idx, dl, ex, ey, ez);
        it.c1();
        T gr[3];
        it.grad(v + g.foff[a], gr);
        if (yv != (T)0) {
#pragma unroll
            for (int b = 0; b < D; ++b) gs[b] = yv * (-cfl) * gr[b];
            c0[0] = it.ax[0].i0;
            c0[1] = it.ax[1].i0;
            c0[2] = D == 3 ? it.ax[D - 1].i0 : 0;
#pragma unroll
            for (int q = 0; q < (1 << D); ++q) wq[q] = it.weight(q) * yv;
        }
    }
    // fixed-point scale from the largest |y| of the tile
    T my = 0;
#pragma unroll
    for (int q = 0; q < (1 << D); ++q) my = fmax(my, fabs(wq[q]));
    for (int o = 32; o > 0; o >>= 1) my = fmax(my, __shfl_xor(my, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = my;
    __syncthreads();
    my = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
    // a non-finite weight anywhere in the tile: every weight goes straight to
    // out with float atomics (as in the density adjoint above)
    bool nf = false;
#pragma unroll
    for (int q = 0; q < (1 << D); ++q) nf = nf || !isfinite(wq[q]);
    const bool direct = __syncthreads_or(nf) != 0 || !isfinite(my);
    int e2 = 0;
    (void)frexp((double)(direct ? (T)1 : my), &e2);
    const double fx = ldexp(1.0, 52 - e2), ifx = ldexp(1.0, e2 - 52);
    // Weights.  Neighbouring lanes of a row usually backtrace into
    // neighbouring cells, so the +x corner of lane l is the 0 corner of lane
    // l+1: that lane adds both (one LDS atomic instead of two).  The match
    // compares the target nodes themselves, so any pairing it makes is exact.
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < (1 << (D - 1)); ++r) {
        const int q0 = r << 1, q1 = q0 | 1;
        const int pi = __shfl_up(c0[0], 1, 64), pj = __shfl_up(c0[1], 1, 64), pk = __shfl_up(c0[2], 1, 64);
        const T pw = __shfl_up(wq[q1], 1, 64);
        const bool match = lane > 0 && pi == c0[0] - 1 && pj == c0[1] && pk == c0[2];
        const bool taken = __shfl_down(match ? 1 : 0, 1, 64) != 0 && lane < 63;
        const int cj = c0[1] + (r & 1), ck = D == 3 ? c0[2] + ((r >> 1) & 1) : 0;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const T w = e == 0 ? wq[q0] + (match ? pw : (T)0) : (taken ? (T)0 : wq[q1]);
            if (w == (T)0) continue;
            const int ci = c0[0] + e;
            const int ca = a == 0 ? ci : (a == 1 ? cj : ck);
            if (ca == 0 || ca == g.n[a]) continue;          // wall node of the a-lattice
            const int wx = ci - ox, wy = cj - oy, wz = ck - oz;
            if (!direct && wx >= 0 && wx < WX && wy >= 0 && wy < WY && wz >= 0 && wz < WZ)
                atomicAdd(&win[(wz * WY + wy) * WX + wx], (unsigned long long)llrint((double)w * fx));
            else
                atomic_add(out + face_index(g, a, ci, cj, ck), w);
        }
    }
#pragma unroll
    for (int b = 0; b < D; ++b) slot[b][threadIdx.x] = gs[b];
    if (gq && valid) {
        const long f = face_index(g, a, i, j, k);
#pragma unroll
        for (int b = 0; b < D; ++b)
            if (b != a) gq[(2L * slice + (b < a ? b : b - 1)) * vs + f] = gs[b];
    }
    __syncthreads();
    // foot-point component b of the tile's source at a-lattice node (si, sj, sk), 0 outside the tile
    auto src = [&](int b, int si, int sj, int sk) -> T {
        const int px = si - tx0, py = sj - ty0, pz = sk - tz0;
        if (px < 0 || px >= TS::X || py < 0 || py >= TS::Y || pz < 0 || pz >= TS::Z) return (T)0;
        return slot[b][(pz * TS::Y + py) * TS::X + px];
    };
    // flush the a-window: weights plus the foot-point term of the source at the node
    for (int e = threadIdx.x; e < WN; e += blockDim.x) {
        const int ci = ox + e % WX, cj = oy + (e / WX) % WY, ck = oz + e / (WX * WY);
        T val = (T)((double)(long long)win[e] * ifx) + src(a, ci, cj, ck);
        if (val == (T)0) continue;
        if (ci < 0 || cj < 0 || ck < 0 || ci >= ex || cj >= ey || (D == 3 && ck >= ez)) continue;
        atomic_add(out + face_index(g, a, ci, cj, ck), val);
    }
    if (gq) return;
    // b-nodes next to the tile: gather the quarters of the b-components
#pragma unroll
    for (int b = 0; b < D; ++b) {
        if (b == a) continue;
        const int da0 = a == 0, da1 = a == 1, da2 = a == 2;
        const int db0 = b == 0, db1 = b == 1, db2 = b == 2;
        const int bx = face_ext(g, b, 0), by = face_ext(g, b, 1), bz = face_ext(g, b, 2);
        for (int e = threadIdx.x; e < BN; e += blockDim.x) {
            const int ci = tx0 - 1 + e % BX, cj = ty0 - 1 + (e / BX) % BY, ck = (D == 3) ? tz0 - 1 + e / (BX * BY) : 0;
            if (ci < 0 || cj < 0 || ck < 0 || ci >= bx || cj >= by || (D == 3 && ck >= bz)) continue;
            const int Jb = b == 0 ? ci : (b == 1 ? cj : ck);
            T s = 0;
            if (Jb != 0) s += src(b, ci, cj, ck) + src(b, ci + da0, cj + da1, ck + da2);
            if (Jb != g.n[b])
                s += src(b, ci - db0, cj - db1, ck - db2) + src(b, ci - db0 + da0, cj - db1 + da1, ck - db2 + da2);
            if (s == (T)0) continue;
            atomic_add(out + face_index(g, b, ci, cj, ck), (T)0.25 * s);
        }
    }
}

// out += the quarters of the foot-point term stored in gq by the tiles: a
// b-face J takes, from each other axis a, a quarter of the b-component of
// the a-faces J, J + e_a, J - e_b and J + e_a - e_b (the four whose averaged
// b-velocity includes J); wall b-faces take nothing.  blockIdx.y = slice.
template <typename T, int D>
__global__ void k_quarter_gather(Grid g, const T* __restrict__ gq, T* __restrict__ out, long vs) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= g.nface) return;
    int b, i, j, k;
    face_decode(g, f, b, i, j, k);
    if (!face_interior(g, b, i, j, k)) return;
    const long s = blockIdx.y;
    T acc = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        if (a == b) continue;
        const T* q = gq + (2 * s + (b < a ? b : b - 1)) * vs;
        const int da0 = a == 0, da1 = a == 1, da2 = a == 2;
        const int db0 = b == 0, db1 = b == 1, db2 = b == 2;
        acc += q[face_index(g, a, i, j, k)] + q[face_index(g, a, i + da0, j + da1, k + da2)] +
               q[face_index(g, a, i - db0, j - db1, k - db2)] +
               q[face_index(g, a, i + da0 - db0, j + da1 - db1, k + da2 - db2)];
    }
    out[s * vs + f] += (T)0.25 * acc;
}

template <typename T, int D>
__global__ void __launch_bounds__(256) k_self_advect_T_tiled(Grid g, T cfl, const T* __restrict__ v,
                                                             const T* __restrict__ y, T scale, T* out, long vs) {
    self_advect_T_tile<T, D>(g, cfl, v, y, scale, out, vs, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Untiled form: one thread per (face, slice), blockIdx.y = slice.
template <typename T, int D>
__global__ void k_self_advect_T_direct(Grid g, T cfl, const T* __restrict__ v, const T* __restrict__ y, T scale,
                                       T* out, long vs) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= g.nface) return;
    int a, i, j, k;
    face_decode(g, f, a, i, j, k);
    const long o = (long)blockIdx.y * vs;
    self_advect_T_source<T, D>(g, cfl, v + o, y + o, scale, out + o, a, i, j, k);
}

}  // namespace stfas
