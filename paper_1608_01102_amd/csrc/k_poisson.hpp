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

}  // namespace stfas
