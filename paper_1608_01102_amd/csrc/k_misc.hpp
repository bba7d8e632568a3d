// Elementwise kernels of the ADMM / density-subproblem drivers, the
// separable Gaussian of the keyframe metric (Sec. 4.1) and deterministic
// two-stage reductions accumulated in double.
#pragma once
#include "common.hpp"

namespace stfas {

template <typename T>
__global__ void k_fill(long n, T* x, T val) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) x[e] = val;
}

// out = a x + b y   (y may be null)
template <typename T>
__global__ void k_axpby(long n, T a, const T* __restrict__ x, T b, const T* __restrict__ y, T* __restrict__ out) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    T s = a * x[e];
    if (y) s += b * y[e];
    out[e] = s;
}

// Time-shifted combine used by the ADMM driver: for slot i = 0..N-1 of a
// face sequence, vi = (i == 0 ? 0 : vshift[i-1]) (v_0 = 0 is fixed), then
//   out[i] = ca * vi + cb * x[i] + cc * y[i]   (y may be null)
template <typename T>
__global__ void k_shift_combine(long F, int N, T ca, const T* __restrict__ vshift, T cb, const T* __restrict__ x,
                                T cc, const T* __restrict__ y, T* __restrict__ out) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= F * N) return;
    const long i = e / F;
    const T vi = i == 0 ? (T)0 : vshift[e - F];
    T s = ca * vi + cb * x[e];
    if (y) s += cc * y[e];
    out[e] = s;
}

// One axis of the separable Gaussian with zero padding:
// out[c] = sum_{t=-R..R} taps[t+R] in[c + t e_axis].
template <typename T>
__global__ void k_blur_axis(Grid g, int axis, int R, const T* __restrict__ taps, const T* __restrict__ in,
                            T* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    const int idx[3] = {c % g.n[0], (c / g.n[0]) % g.n[1], c / (g.n[0] * g.n[1])};
    const int stride = axis == 0 ? 1 : (axis == 1 ? g.n[0] : g.n[0] * g.n[1]);
    const int pos = idx[axis], n = g.n[axis];
    const int lo = pos - R < 0 ? R - pos : 0;
    const int hi = pos + R >= n ? R + (n - 1 - pos) : 2 * R;
    T s = 0;
    for (int t = lo; t <= hi; ++t) s += taps[t] * in[c + (t - R) * stride];
    out[c] = s;
}

// ---------------------------------------------------------------- reductions
enum RedOp { RED_DOT = 0, RED_SUMSQ_DIFF = 1, RED_MAXABS_DIFF = 2 };
constexpr int RED_BS = 256;     // threads per block of the reduction kernels

template <typename T>
__device__ inline double red_elem(int op, const T* x, const T* y, long e) {
    const double a = (double)x[e];
    if (op == RED_DOT) return a * (double)y[e];
    const double d = y ? a - (double)y[e] : a;
    return op == RED_SUMSQ_DIFF ? d * d : fabs(d);
}

__device__ inline double red_combine(int op, double a, double b) { return op == RED_MAXABS_DIFF ? fmax(a, b) : a + b; }

// Combine over a wave64 by cross-lane shuffles (after it, lane 0 holds the
// wave's value), then over the block's waves through a few LDS words; the
// order is fixed, so the result is deterministic.  Thread 0 of the block
// gets the block's value.
__device__ inline double wave_combine(int op, double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = red_combine(op, v, __shfl_down(v, off, 64));
    return v;
}

__device__ inline double block_combine(int op, double v) {
    __shared__ double per_wave[RED_BS / 64];
    v = wave_combine(op, v);
    if ((threadIdx.x & 63) == 0) per_wave[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        v = per_wave[0];
#pragma unroll
        for (int w = 1; w < RED_BS / 64; ++w) v = red_combine(op, v, per_wave[w]);
    }
    return v;
}

// Block partials of a reduction over n elements (grid-stride, fixed order).
// Launched with RED_BS threads per block.
template <typename T>
__global__ void __launch_bounds__(RED_BS) k_reduce_part(long n, int op, const T* __restrict__ x,
                                                        const T* __restrict__ y, double* __restrict__ part) {
    double acc = 0;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        acc = red_combine(op, acc, red_elem(op, x, y, e));
    acc = block_combine(op, acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Block partials of max |x| over up to four arrays at once (the four parts
// of a KKT residual): one launch instead of one per array.
template <typename T>
__global__ void __launch_bounds__(RED_BS) k_maxabs4_part(long n0, const T* __restrict__ x0, long n1,
                                                         const T* __restrict__ x1, long n2, const T* __restrict__ x2,
                                                         long n3, const T* __restrict__ x3,
                                                         double* __restrict__ part) {
    const long step = (long)gridDim.x * blockDim.x, first = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0;
    for (long e = first; e < n0; e += step) acc = fmax(acc, fabs((double)x0[e]));
    for (long e = first; e < n1; e += step) acc = fmax(acc, fabs((double)x1[e]));
    for (long e = first; e < n2; e += step) acc = fmax(acc, fabs((double)x2[e]));
    for (long e = first; e < n3; e += step) acc = fmax(acc, fabs((double)x3[e]));
    acc = block_combine(RED_MAXABS_DIFF, acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Block partials of max |x| over the interior faces of `slices` consecutive
// face fields (wall entries are left out, whatever they hold).
template <typename T>
__global__ void __launch_bounds__(RED_BS) k_maxabs_interior_part(Grid g, long slices, const T* __restrict__ x,
                                                                 double* __restrict__ part) {
    const long n = slices * g.nface;
    double acc = 0;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        int a, i, j, k;
        face_decode(g, (int)(e % g.nface), a, i, j, k);
        if (face_interior(g, a, i, j, k)) acc = fmax(acc, fabs((double)x[e]));
    }
    acc = block_combine(RED_MAXABS_DIFF, acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// out[slot] = (accumulate ? out[slot] op : ) combine of the partials.
__global__ void __launch_bounds__(RED_BS) k_reduce_final(int nparts, int op, const double* __restrict__ part,
                                                         double* out, int slot, int accumulate) {
    double acc = 0;
    for (int e = threadIdx.x; e < nparts; e += blockDim.x) acc = red_combine(op, acc, part[e]);
    acc = block_combine(op, acc);
    if (threadIdx.x == 0) out[slot] = accumulate ? red_combine(op, out[slot], acc) : acc;
}

// Per-slice sums of a cell field (for mean removal).
template <typename T>
__global__ void k_slice_sum(int n, const T* __restrict__ x, double* __restrict__ out, long cs) {
    __shared__ double sm[256];
    x += blockIdx.x * cs;
    double acc = 0;
    for (int e = threadIdx.x; e < n; e += blockDim.x) acc += (double)x[e];
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}

// Per-slice Poisson residual ratios |r|/|b| from block partials; the max over
// slices goes to out[slot].
__global__ void k_poisson_ratio(int nslice, int nblk, const double* __restrict__ part, double* out, int slot) {
    // one wavefront per slice: its lanes stride over the slice's block
    // partials and fold them with shuffles; then the largest ratio of all
    // slices (one launch of 256 threads)
    __shared__ double sm[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    double worst = 0;
    for (int s = wave; s < nslice; s += nw) {
        double r2 = 0, b2 = 0;
        for (int q = lane; q < nblk; q += 64) {
            r2 += part[((long)s * nblk + q) * 2];
            b2 += part[((long)s * nblk + q) * 2 + 1];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            r2 += __shfl_xor(r2, o);
            b2 += __shfl_xor(b2, o);
        }
        worst = fmax(worst, b2 > 0 ? sqrt(r2 / b2) : 0.0);
    }
    if (lane == 0) sm[wave] = worst;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0;
        for (int w = 0; w < nw; ++w) m = fmax(m, sm[w]);
        out[slot] = m;
    }
}

}  // namespace stfas
