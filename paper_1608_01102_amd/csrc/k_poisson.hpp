// Multigrid Poisson kernels for the projection Q (Sec. 4.1: Q(w) = w - G phi
// with L phi = D w, L = D G the Neumann 5/7-point Laplacian, mean(phi) = 0;
// the paper evaluates Q with a conventional multigrid Poisson solver).
//
// Cell-centred V(2,2) cycles: red-black Gauss-Seidel, restriction of the
// residual by the 2^d-average of the children, prolongation by clamped
// multilinear interpolation at (i + 1/2)/2 - 1/2, and an exact solve on the
// coarsest level with the pseudo-inverse (double precision).  Every kernel
// is batched over independent slices (blockIdx.y or blockIdx.x).
#pragma once
#include "common.hpp"

namespace stfas {

// A projection stops early when a V-cycle reduces the relative residual by
// less than this factor: the cycles have reached the rounding floor of the
// working precision (a healthy cycle reduces it by about 0.13).
constexpr double PROJECT_STALL = 0.5;

// b = D w  (per cell; wall faces hold zero).
template <typename T, int D>
__global__ void k_divergence(Grid g, const T* __restrict__ w, T* __restrict__ b, long ws, long bs) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    w += blockIdx.y * ws;
    b += blockIdx.y * bs;
    const int i = c % g.n[0], j = (c / g.n[0]) % g.n[1], k = c / (g.n[0] * g.n[1]);
    const int idx[3] = {i, j, k};
    T s = 0;
    for (int a = 0; a < D; ++a) {
        // wall faces count as zero whatever the buffer holds
        if (idx[a] + 1 < g.n[a]) s += w[face_index(g, a, i + (a == 0), j + (a == 1), k + (a == 2))];
        if (idx[a] > 0) s -= w[face_index(g, a, i, j, k)];
    }
    b[c] = s / (T)g.h;
}

// One colour of a red-black Gauss-Seidel sweep for L phi = b.
template <typename T, int D>
__global__ void k_rbgs(Grid g, T* __restrict__ phi, const T* __restrict__ b, int colour, long cs) {
    // thread q covers cells of one parity; x index reconstructed from the row parity
    const int half = (g.n[0] + 1) / 2;
    const int rows = g.n[1] * g.n[2];
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= half * rows) return;
    phi += blockIdx.y * cs;
    b += blockIdx.y * cs;
    const int r = q / half;
    const int j = r % g.n[1], k = r / g.n[1];
    const int i = 2 * (q % half) + ((j + k + colour) & 1);
    if (i >= g.n[0]) return;
    const int c = cell_index(g, i, j, k);
    T s = 0;
    int cnt = 0;
    if (i > 0) { s += phi[c - 1]; ++cnt; }
    if (i < g.n[0] - 1) { s += phi[c + 1]; ++cnt; }
    if (j > 0) { s += phi[c - g.n[0]]; ++cnt; }
    if (j < g.n[1] - 1) { s += phi[c + g.n[0]]; ++cnt; }
    if (D == 3) {
        const int sz = g.n[0] * g.n[1];
        if (k > 0) { s += phi[c - sz]; ++cnt; }
        if (k < g.n[2] - 1) { s += phi[c + sz]; ++cnt; }
    }
    const T h2 = (T)(g.h * g.h);
    phi[c] = (s - h2 * b[c]) / (T)cnt;
}

// (L phi)_c for the Neumann Laplacian.
template <typename T, int D>
__device__ inline T lap(const Grid& g, const T* phi, int i, int j, int k) {
    const int c = cell_index(g, i, j, k);
    const T pc = phi[c];
    T s = 0;
    if (i > 0) s += phi[c - 1] - pc;
    if (i < g.n[0] - 1) s += phi[c + 1] - pc;
    if (j > 0) s += phi[c - g.n[0]] - pc;
    if (j < g.n[1] - 1) s += phi[c + g.n[0]] - pc;
    if (D == 3) {
        const int sz = g.n[0] * g.n[1];
        if (k > 0) s += phi[c - sz] - pc;
        if (k < g.n[2] - 1) s += phi[c + sz] - pc;
    }
    return s / (T)(g.h * g.h);
}

// bc = 2^-d sum over the 2^d children of (b - L phi).
template <typename T, int D>
__global__ void k_resid_restrict(Grid gf, Grid gc, const T* __restrict__ phi, const T* __restrict__ b,
                                 T* __restrict__ bc, long fs, long cs) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= gc.ncell) return;
    phi += blockIdx.y * fs;
    b += blockIdx.y * fs;
    bc += blockIdx.y * cs;
    const int I = c % gc.n[0], J = (c / gc.n[0]) % gc.n[1], Kk = c / (gc.n[0] * gc.n[1]);
    T s = 0;
    for (int q = 0; q < (1 << D); ++q) {
        const int i = 2 * I + (q & 1), j = 2 * J + ((q >> 1) & 1), k = D == 3 ? 2 * Kk + ((q >> 2) & 1) : 0;
        s += b[cell_index(gf, i, j, k)] - lap<T, D>(gf, phi, i, j, k);
    }
    bc[c] = s * (T)(D == 3 ? 0.125 : 0.25);
}

// phi += P phic (clamped multilinear interpolation at (i + 1/2)/2 - 1/2).
template <typename T, int D>
__global__ void k_prolong_add(Grid gf, Grid gc, const T* __restrict__ phic, T* __restrict__ phi, long fs,
                              long cs) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= gf.ncell) return;
    phi += blockIdx.y * fs;
    phic += blockIdx.y * cs;
    const int i = c % gf.n[0], j = (c / gf.n[0]) % gf.n[1], k = c / (gf.n[0] * gf.n[1]);
    const int idx[3] = {i, j, k};
    T y[3];
    for (int a = 0; a < D; ++a) y[a] = ((T)idx[a] + (T)0.5) * (T)0.5 - (T)0.5;
    Interp<T, D> it;
    it.setup(y, gc.n[0], gc.n[1], gc.n[2]);
    phi[c] += it.value(phic);
}

// Exact coarsest solve: phic = pinv(L) bc in double, one block per slice.
// pinv is m x m row-major; the dynamic LDS holds bc as double.
template <typename T>
__global__ void k_coarse_solve(int m, const double* __restrict__ pinv, const T* __restrict__ bc,
                               T* __restrict__ phic, long cs) {
    extern __shared__ double sb[];
    bc += blockIdx.x * cs;
    phic += blockIdx.x * cs;
    for (int i = threadIdx.x; i < m; i += blockDim.x) sb[i] = (double)bc[i];
    __syncthreads();
    for (int r = threadIdx.x; r < m; r += blockDim.x) {
        const double* row = pinv + (long)r * m;
        double s = 0;
        for (int q = 0; q < m; ++q) s += row[q] * sb[q];
        phic[r] = (T)s;
    }
}

// v = w - G phi on interior faces, 0 on walls.
template <typename T, int D>
__global__ void k_project_apply(Grid g, const T* __restrict__ w, const T* __restrict__ phi, T* __restrict__ v,
                                long ws, long cs) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= g.nface) return;
    w += blockIdx.y * ws;
    v += blockIdx.y * ws;
    phi += blockIdx.y * cs;
    int a, i, j, k;
    face_decode(g, f, a, i, j, k);
    if (!face_interior(g, a, i, j, k)) {
        v[f] = (T)0;
        return;
    }
    const int c = cell_index(g, i, j, k);
    const int cm = cell_index(g, i - (a == 0), j - (a == 1), k - (a == 2));
    v[f] = w[f] - (phi[c] - phi[cm]) / (T)g.h;
}

// Per-slice sums of (b - L phi)^2 and b^2 into part[slice][block][2] (double).
template <typename T, int D>
__global__ void k_poisson_resid_norm(Grid g, const T* __restrict__ phi, const T* __restrict__ b,
                                     double* __restrict__ part, long cs) {
    __shared__ double s0[256], s1[256];
    phi += blockIdx.y * cs;
    b += blockIdx.y * cs;
    double r2 = 0, b2 = 0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.ncell; c += gridDim.x * blockDim.x) {
        const int i = c % g.n[0], j = (c / g.n[0]) % g.n[1], k = c / (g.n[0] * g.n[1]);
        const double bb = (double)b[c];
        const double rr = bb - (double)lap<T, D>(g, phi, i, j, k);
        r2 += rr * rr;
        b2 += bb * bb;
    }
    s0[threadIdx.x] = r2;
    s1[threadIdx.x] = b2;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            s0[threadIdx.x] += s0[threadIdx.x + s];
            s1[threadIdx.x] += s1[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* o = part + ((long)blockIdx.y * gridDim.x + blockIdx.x) * 2;
        o[0] = s0[0];
        o[1] = s1[0];
    }
}

// Subtract the per-slice mean (computed into mean[slice]) from phi.
template <typename T>
__global__ void k_sub_mean(int n, T* phi, const double* __restrict__ sums, long cs) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    phi += blockIdx.y * cs;
    phi[c] -= (T)(sums[blockIdx.y] / (double)n);
}

// ---------------------------------------------------------------- in LDS
// The whole projection of one slice in one workgroup, for grids whose
// multigrid hierarchy fits in a CU's LDS: the same V(2,2) cycle as the
// kernels above (same smoother, transfers and coarsest pseudo-inverse), with
// every level's phi and every coarse level's right-hand side in LDS and the
// finest right-hand side in registers.  The cycle count is decided in the
// kernel from the slice's own residual ratio, so a projection is a single
// launch with no host synchronisation.
//
// Finest-level ownership: thread t holds the x-pairs of cells (2p, 2p+1),
// p = t + 1024 q, q < CPT/2 (n_x is even whenever the grid coarsens) and
// their packed coordinates; the finest right-hand side goes to a global
// buffer (b0, one slice per workgroup) that only the owning thread touches,
// so it stays in the CU's cache.  A pair has one cell of each colour, so a
// half-sweep updates exactly one cell per pair.
constexpr int PL_MAX = 12;

// x / d for 0 <= x < 2^31 by multiply and shift (d >= 1).
struct FastDiv {
    unsigned mul, shift, d;
};
inline FastDiv make_fastdiv(unsigned d) {
    unsigned l = 0;
    while ((1ull << l) < d) ++l;
    const unsigned long long m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
    return FastDiv{(unsigned)m, l, d};
}
__device__ inline unsigned fdiv(unsigned x, const FastDiv& f) {
    const unsigned long long t = (unsigned long long)__umulhi(x, f.mul) + x;
    return (unsigned)(t >> f.shift);
}

struct PLevels {
    Grid g[PL_MAX];
    FastDiv dx[PL_MAX];      // divide by n_x
    FastDiv dy[PL_MAX];      // divide by n_y
    FastDiv dh[PL_MAX];      // divide by ceil(n_x / 2)
    int off_phi[PL_MAX];     // element offsets in the LDS block
    int off_b[PL_MAX];       // (level 0 keeps b in registers)
    int n;
    int coarse_m;            // cells of the coarsest level (pinv is coarse_m^2)
};

__device__ inline double block_sum_1024(double x, double* red) {
    // red: 16 doubles of LDS; all 1024 threads call this
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = x;
    __syncthreads();
    double s = 0;
    for (int q = 0; q < 16; ++q) s += red[q];
    return s;
}

// Neighbour sum and count of cell c = (i, j, k) (Neumann: missing
// neighbours are dropped), and (L phi)_c in the order of lap().
template <typename T, int D>
__device__ inline T pl_nbsum(const Grid& g, const T* phi, int c, int i, int j, int k, int& cnt) {
    T s = 0;
    cnt = 0;
    if (i > 0) { s += phi[c - 1]; ++cnt; }
    if (i < g.n[0] - 1) { s += phi[c + 1]; ++cnt; }
    if (j > 0) { s += phi[c - g.n[0]]; ++cnt; }
    if (j < g.n[1] - 1) { s += phi[c + g.n[0]]; ++cnt; }
    if (D == 3) {
        const int sz = g.n[0] * g.n[1];
        if (k > 0) { s += phi[c - sz]; ++cnt; }
        if (k < g.n[2] - 1) { s += phi[c + sz]; ++cnt; }
    }
    return s;
}
template <typename T, int D>
__device__ inline T pl_lap(const Grid& g, const T* phi, int c, int i, int j, int k) {
    const T pc = phi[c];
    T s = 0;
    if (i > 0) s += phi[c - 1] - pc;
    if (i < g.n[0] - 1) s += phi[c + 1] - pc;
    if (j > 0) s += phi[c - g.n[0]] - pc;
    if (j < g.n[1] - 1) s += phi[c + g.n[0]] - pc;
    if (D == 3) {
        const int sz = g.n[0] * g.n[1];
        if (k > 0) s += phi[c - sz] - pc;
        if (k < g.n[2] - 1) s += phi[c + sz] - pc;
    }
    return s / (T)(g.h * g.h);
}

// One axis of the 2:1 cell-centred prolongation (clamped linear
// interpolation at (i + 1/2)/2 - 1/2 on M coarse cells).
__device__ inline void pl_axis(int i, int M, int& lo, int& hi, float& wlo) {
    const int I = i >> 1;
    if ((i & 1) == 0) {
        if (I == 0) { lo = hi = 0; wlo = 1.f; }
        else { lo = I - 1; hi = I; wlo = 0.25f; }
    } else {
        if (I == M - 1) { lo = hi = M - 1; wlo = 1.f; }
        else { lo = I; hi = I + 1; wlo = 0.75f; }
    }
}

template <typename T, int D, int CPT>
__global__ void __launch_bounds__(1024) k_project_lds(PLevels pl_arg, const double* __restrict__ pinv,
                                                      const T* w, T* o, T* phi_out, T* b0, double rtol,
                                                      int fixed, int max_cycles, int* cycles_max, long ws,
                                                      long cs) {
    constexpr int NP = CPT / 2;
    // the level table goes to LDS once, so that indexing it by a run-time
    // level reads LDS rather than a private copy of the argument
    __shared__ PLevels pl;
    if (threadIdx.x == 0) pl = pl_arg;
    __syncthreads();
    extern __shared__ unsigned char smem_raw[];
    double* red = reinterpret_cast<double*>(smem_raw);          // 16 doubles
    T* sm = reinterpret_cast<T*>(smem_raw + 256);
    const int tid = threadIdx.x;
    w += blockIdx.x * ws;
    o += blockIdx.x * ws;
    b0 += blockIdx.x * cs;
    const Grid& g0 = pl.g[0];
    const int C0 = g0.ncell;
    T* phi0 = sm + pl.off_phi[0];
    const T h20 = (T)(g0.h * g0.h);
    // ---- finest pairs: coordinates (i of the even cell, j, k) of pair q
    auto pair = [&](int q, int& i, int& j, int& k) -> bool {
        const int c = 2 * (tid + 1024 * q);
        if (c >= C0) return false;
        const unsigned r = fdiv((unsigned)c, pl.dx[0]);
        i = c - (int)r * g0.n[0];
        k = D == 3 ? (int)fdiv(r, pl.dy[0]) : 0;
        j = (int)r - k * g0.n[1];
        return true;
    };
    // ---- right-hand side b0 = D w (wall faces count as zero), phi = 0
    double bb = 0;
    for (int q = 0; q < NP; ++q) {
        int i0, j, k;
        if (!pair(q, i0, j, k)) break;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int i = i0 + e;
            const int idx[3] = {i, j, k};
            T s = 0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                if (idx[a] + 1 < g0.n[a]) s += w[face_index(g0, a, i + (a == 0), j + (a == 1), k + (a == 2))];
                if (idx[a] > 0) s -= w[face_index(g0, a, i, j, k)];
            }
            s = s / (T)g0.h;
            b0[cell_index(g0, i, j, k)] = s;
            bb += (double)s * (double)s;
        }
    }
    for (int c = tid; c < C0; c += 1024) phi0[c] = (T)0;
    bb = block_sum_1024(bb, red);
    // ---- smoothing: one colour of red-black Gauss-Seidel
    auto smooth0 = [&](int colour) {
        for (int q = 0; q < NP; ++q) {
            int i, j, k;
            if (!pair(q, i, j, k)) break;
            const int e = (colour + j + k) & 1;         // i is even
            i += e;
            const int c = cell_index(g0, i, j, k);
            int cnt;
            const T s = pl_nbsum<T, D>(g0, phi0, c, i, j, k, cnt);
            phi0[c] = (s - h20 * b0[c]) / (T)cnt;
        }
        __syncthreads();
    };
    auto smooth = [&](int l, int colour) {
        const Grid& g = pl.g[l];
        T* phi = sm + pl.off_phi[l];
        const T* b = sm + pl.off_b[l];
        const T h2 = (T)(g.h * g.h);
        const int half = (g.n[0] + 1) >> 1;
        const int tot = half * g.n[1] * g.n[2];
        for (int q = tid; q < tot; q += 1024) {
            const unsigned r = fdiv((unsigned)q, pl.dh[l]);
            const unsigned k = D == 3 ? fdiv(r, pl.dy[l]) : 0u;
            const int j = (int)r - (int)k * g.n[1];
            const int i = 2 * (q - (int)r * half) + ((j + (int)k + colour) & 1);
            if (i >= g.n[0]) continue;
            const int c = cell_index(g, i, j, (int)k);
            int cnt;
            const T s = pl_nbsum<T, D>(g, phi, c, i, j, (int)k, cnt);
            phi[c] = (s - h2 * b[c]) / (T)cnt;
        }
        __syncthreads();
    };
    // residual of the finest level restricted to level 1: the two cells of
    // a pair share a coarse cell; the 2^(d-1) pairs of a coarse cell add in
    // turn (one phase per row/slab parity), and the last phase scales
    auto restrict0 = [&]() {
        const Grid& gc = pl.g[1];
        T* bc = sm + pl.off_b[1];
        constexpr int NPH = D == 3 ? 4 : 2;
        const T scale = (T)(D == 3 ? 0.125 : 0.25);
        for (int phase = 0; phase < NPH; ++phase) {
            for (int q = 0; q < NP; ++q) {
                int i, j, k;
                if (!pair(q, i, j, k)) break;
                if ((j & 1) + 2 * (k & 1) != phase) continue;
                const int c = cell_index(g0, i, j, k);
                const T part = (b0[c] - pl_lap<T, D>(g0, phi0, c, i, j, k)) +
                               (b0[c + 1] - pl_lap<T, D>(g0, phi0, c + 1, i + 1, j, k));
                const int cc = cell_index(gc, i >> 1, j >> 1, k >> 1);
                const T acc = (phase == 0 ? (T)0 : bc[cc]) + part;
                bc[cc] = phase == NPH - 1 ? acc * scale : acc;
            }
            __syncthreads();
        }
    };
    auto restrict_l = [&](int l) {
        const Grid& gf = pl.g[l];
        const Grid& gc = pl.g[l + 1];
        const T* phi = sm + pl.off_phi[l];
        const T* b = sm + pl.off_b[l];
        T* bc = sm + pl.off_b[l + 1];
        for (int c = tid; c < gc.ncell; c += 1024) {
            const unsigned r = fdiv((unsigned)c, pl.dx[l + 1]);
            const unsigned K = D == 3 ? fdiv(r, pl.dy[l + 1]) : 0u;
            const int I = c - (int)r * gc.n[0], J = (int)r - (int)K * gc.n[1];
            T s = 0;
            for (int q = 0; q < (1 << D); ++q) {
                const int i = 2 * I + (q & 1), j = 2 * J + ((q >> 1) & 1), k = D == 3 ? 2 * (int)K + ((q >> 2) & 1) : 0;
                const int f = cell_index(gf, i, j, k);
                s += b[f] - pl_lap<T, D>(gf, phi, f, i, j, k);
            }
            bc[c] = s * (T)(D == 3 ? 0.125 : 0.25);
        }
        __syncthreads();
    };
    // phi_l += P phi_{l+1}
    auto prolong_cell = [&](const Grid& gc, const T* phic, int i, int j, int k) -> T {
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        float wl[3] = {1.f, 1.f, 1.f};
        pl_axis(i, gc.n[0], lo[0], hi[0], wl[0]);
        pl_axis(j, gc.n[1], lo[1], hi[1], wl[1]);
        if (D == 3) pl_axis(k, gc.n[2], lo[2], hi[2], wl[2]);
        T v = 0;
#pragma unroll
        for (int q = 0; q < (1 << D); ++q) {
            const int ci = (q & 1) ? hi[0] : lo[0], cj = (q & 2) ? hi[1] : lo[1], ck = (q & 4) ? hi[2] : lo[2];
            const T wt = (T)((q & 1) ? 1.f - wl[0] : wl[0]) * (T)((q & 2) ? 1.f - wl[1] : wl[1]) *
                         (T)(D == 3 ? ((q & 4) ? 1.f - wl[2] : wl[2]) : 1.f);
            v += wt * phic[cell_index(gc, ci, cj, ck)];
        }
        return v;
    };
    auto prolong = [&](int l) {
        const Grid& gf = pl.g[l];
        const Grid& gc = pl.g[l + 1];
        T* phi = sm + pl.off_phi[l];
        const T* phic = sm + pl.off_phi[l + 1];
        if (l == 0) {
            for (int q = 0; q < NP; ++q) {
                int i, j, k;
                if (!pair(q, i, j, k)) break;
                const int c = cell_index(g0, i, j, k);
                phi[c] += prolong_cell(gc, phic, i, j, k);
                phi[c + 1] += prolong_cell(gc, phic, i + 1, j, k);
            }
        } else {
            for (int c = tid; c < gf.ncell; c += 1024) {
                const unsigned r = fdiv((unsigned)c, pl.dx[l]);
                const unsigned k = D == 3 ? fdiv(r, pl.dy[l]) : 0u;
                const int i = c - (int)r * gf.n[0], j = (int)r - (int)k * gf.n[1];
                phi[c] += prolong_cell(gc, phic, i, j, (int)k);
            }
        }
        __syncthreads();
    };
    const int nl = pl.n;
    int cyc = 0;
    double prev = 0;
    for (;;) {
        // ---- one V(2,2) cycle
        for (int l = 0; l < nl - 1; ++l) {
            for (int s2 = 0; s2 < 2; ++s2) {
                if (l == 0) {
                    smooth0(0);
                    smooth0(1);
                } else {
                    smooth(l, 0);
                    smooth(l, 1);
                }
            }
            if (l == 0)
                restrict0();
            else
                restrict_l(l);
            T* phic = sm + pl.off_phi[l + 1];
            for (int c = tid; c < pl.g[l + 1].ncell; c += 1024) phic[c] = (T)0;
            __syncthreads();
        }
        {   // coarsest: phi = pinv b in double
            const int m = pl.coarse_m;
            T* phic = sm + pl.off_phi[nl - 1];
            const T* bcst = sm + pl.off_b[nl - 1];
            for (int r = tid; r < m; r += 1024) {
                double s = 0;
                for (int q = 0; q < m; ++q) s += pinv[(long)r * m + q] * (double)bcst[q];
                phic[r] = (T)s;
            }
            __syncthreads();
        }
        for (int l = nl - 2; l >= 0; --l) {
            prolong(l);
            for (int s2 = 0; s2 < 2; ++s2) {
                if (l == 0) {
                    smooth0(1);
                    smooth0(0);
                } else {
                    smooth(l, 1);
                    smooth(l, 0);
                }
            }
        }
        ++cyc;
        if (fixed > 0) {
            if (cyc >= fixed) break;
            continue;
        }
        if (cyc >= max_cycles) break;
        // ---- relative residual of this slice
        double rr = 0;
        for (int q = 0; q < NP; ++q) {
            int i, j, k;
            if (!pair(q, i, j, k)) break;
            const int c = cell_index(g0, i, j, k);
            const double r0 = (double)b0[c] - (double)pl_lap<T, D>(g0, phi0, c, i, j, k);
            const double r1 = (double)b0[c + 1] - (double)pl_lap<T, D>(g0, phi0, c + 1, i + 1, j, k);
            rr += r0 * r0 + r1 * r1;
        }
        rr = block_sum_1024(rr, red);
        const double ratio = bb > 0 ? sqrt(rr / bb) : 0.0;
        if (!(ratio > rtol)) break;                          // converged, or not finite
        if (cyc >= 2 && ratio > PROJECT_STALL * prev) break; // at the rounding floor
        prev = ratio;
    }
    if (tid == 0 && cycles_max) atomicMax(cycles_max, cyc);
    // ---- o = w - G phi on interior faces, 0 on walls (o may alias w)
    for (int f = tid; f < g0.nface; f += 1024) {
        int a, i, j, k;
        face_decode(g0, f, a, i, j, k);
        if (!face_interior(g0, a, i, j, k)) {
            o[f] = (T)0;
            continue;
        }
        const int c = cell_index(g0, i, j, k);
        const int cm = cell_index(g0, i - (a == 0), j - (a == 1), k - (a == 2));
        o[f] = w[f] - (phi0[c] - phi0[cm]) / (T)g0.h;
    }
    if (phi_out) {
        double sp = 0;
        for (int c = tid; c < C0; c += 1024) sp += (double)phi0[c];
        sp = block_sum_1024(sp, red);
        const T mean = (T)(sp / (double)C0);
        phi_out += blockIdx.x * cs;
        for (int c = tid; c < C0; c += 1024) phi_out[c] = phi0[c] - mean;
    }
}

}  // namespace stfas
