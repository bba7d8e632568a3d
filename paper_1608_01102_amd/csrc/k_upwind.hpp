// Upwind Taylor-exponential density advection (Sec. 3.1 eq:Adv) and its two
// adjoints, on one grid, one field at a time.
//
//   A(rho, v) = sum_{j=0..k} T_j,  T_0 = rho,  T_j = (dt / j) A(v) T_{j-1}
//
// A(v) is a flux-form upwind stencil: across an interior a-face with cells
// L (below) and R (above) and normal velocity v_f the flux is v_f x_f, L
// loses flux / h and R gains it; walls carry no flux.  The face value x_f is
// second order, (3 x_U - x_UU) / 2 with U the upstream cell and UU the next
// one upstream (first order, x_U, when UU is outside the grid); v_f = 0
// counts as v_f >= 0.  k is the first j with max|T_j| < 1e-5, at most 48.
//
// The truncated series is linear in rho for fixed k, so its adjoints are
// taken at that k.  With Z_k = 0 and, for b = k-1 .. 0,
//   Z_b = (dt / (b+1)) (mu + A^T Z_{b+1}),
// the rho adjoint is mu + A^T Z_0 and the v adjoint is
// sum_{b<k} D(T_b)^T Z_b, where D(x)^T z on an interior face is
// (z_R - z_L) x_f / h: expanding the powers, each pair of (scaled) powers
// of A and A^T carries dt a! b! / (a+b+1)!, which is what the recursion
// accumulates.
//
// Device form: one launch per term.  Each block folds max|T_j| into a
// per-term word with atomicMax on the bit pattern (non-negative floats order
// like their bits); launch j + 1 reads that word and returns at once when
// the series has already stopped, so a fixed sequence of launches needs no
// host synchronisation.  Every active launch records its j, so the last one
// leaves k.  The adjoint launches read k and are empty for b >= k.
#pragma once

#include "common.hpp"
#include "k_misc.hpp"

namespace stfas {

constexpr int UP_KMAX = 48;
constexpr double UP_TOL = 1e-5;

template <typename T>
struct UpBits;
template <>
struct UpBits<float> {
    using U = unsigned int;
    static __host__ __device__ U of(float x) { return __builtin_bit_cast(U, x); }
};
template <>
struct UpBits<double> {
    using U = unsigned long long;
    static __host__ __device__ U of(double x) { return __builtin_bit_cast(U, x); }
};

template <typename T>
struct UpCtl {
    typename UpBits<T>::U* maxb;   // [UP_KMAX + 1]: bits of max|T_j|
    int* k;                        // index of the last summed term
};

__device__ inline void cell_decode(const Grid& g, int c, int (&x)[3]) {
    x[0] = c % g.n[0];
    const int r = c / g.n[0];
    x[1] = r % g.n[1];
    x[2] = r / g.n[1];
}

__device__ inline int cell_stride(const Grid& g, int a) { return a == 0 ? 1 : (a == 1 ? g.n[0] : g.n[0] * g.n[1]); }

// a-face whose upper cell has coordinates x with x[a] replaced by I
__device__ inline int face_at(const Grid& g, int a, const int (&x)[3], int I) {
    return face_index(g, a, a == 0 ? I : x[0], a == 1 ? I : x[1], a == 2 ? I : x[2]);
}

// Upwind face value at the interior a-face I (cells cR - s and cR).
template <typename T>
__device__ inline T up_face(const T* __restrict__ x, T vf, int cR, int s, int I, int n) {
    if (vf >= (T)0) {
        const T xu = x[cR - s];
        return I >= 2 ? (T)1.5 * xu - (T)0.5 * x[cR - 2 * s] : xu;
    }
    const T xu = x[cR];
    return I + 1 <= n - 1 ? (T)1.5 * xu - (T)0.5 * x[cR + s] : xu;
}

// Block maximum of a non-negative value (256 threads, four waves) folded
// into *out by its bit pattern.  Atomics on one word serialise, so a block
// first reads the word (at device scope) and folds only when it would raise
// it: the word only grows after its reset, so a value at or below what was
// read can never be the maximum's last word, and the result is unchanged.
template <typename T>
__device__ inline void block_max_fold(T m, typename UpBits<T>::U* out) {
    __shared__ T wm[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        const T b = fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]));
        const typename UpBits<T>::U bb = UpBits<T>::of(b);
        if (bb > __hip_atomic_load(out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(out, bb);
    }
}

// Term j of the series: next = (dt / (j h)) h A(v) prev, sum += next (sum may
// be null); j = 0 only measures prev (= rho) and copies it into sum.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_up_term(Grid g, T coef, int j, const T* __restrict__ prev,
                                                 const T* __restrict__ v, T* __restrict__ next, T* __restrict__ sum,
                                                 UpCtl<T> ctl, typename UpBits<T>::U tolb) {
    if (j > 0 && ctl.maxb[j - 1] < tolb) return;     // stopped (the same decision in every block)
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    T val = 0;
    if (c < g.ncell) {
        if (j == 0) {
            val = prev[c];
            if (sum) sum[c] = val;
        } else {
            int x[3];
            cell_decode(g, c, x);
            T acc = 0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const int s = cell_stride(g, a), I = x[a], n = g.n[a];
                if (I >= 1) {                                    // inflow through the lower face
                    const T vf = v[face_at(g, a, x, I)];
                    acc += vf * up_face(prev, vf, c, s, I, n);
                }
                if (I + 1 <= n - 1) {                            // outflow through the upper face
                    const T vf = v[face_at(g, a, x, I + 1)];
                    acc -= vf * up_face(prev, vf, c + s, s, I + 1, n);
                }
            }
            val = coef * acc;
            next[c] = val;
            if (sum) sum[c] += val;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *ctl.k = j;
    block_max_fold<T>(fabs(val), ctl.maxb + j);
}

// (A^T z) at cell c (gather over the faces whose upwind value uses c), times h.
template <typename T, int D>
__device__ inline T up_AT(const Grid& g, const T* __restrict__ z, const T* __restrict__ v, int c, const int (&x)[3]) {
    T acc = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int s = cell_stride(g, a), I = x[a], n = g.n[a];
        if (I + 1 <= n - 1) {                 // face I+1: c is U when v >= 0
            const T vf = v[face_at(g, a, x, I + 1)];
            if (vf >= (T)0) acc += (I >= 1 ? (T)1.5 : (T)1) * vf * (z[c + s] - z[c]);
        }
        if (I + 2 <= n - 1) {                 // face I+2: c is UU when v >= 0
            const T vf = v[face_at(g, a, x, I + 2)];
            if (vf >= (T)0) acc -= (T)0.5 * vf * (z[c + 2 * s] - z[c + s]);
        }
        if (I >= 1) {                         // face I: c is U when v < 0
            const T vf = v[face_at(g, a, x, I)];
            if (vf < (T)0) acc += (I + 1 <= n - 1 ? (T)1.5 : (T)1) * vf * (z[c] - z[c - s]);
        }
        if (I >= 2) {                         // face I-1: c is UU when v < 0
            const T vf = v[face_at(g, a, x, I - 1)];
            if (vf < (T)0) acc -= (T)0.5 * vf * (z[c - s] - z[c - 2 * s]);
        }
    }
    return acc;
}

// One step of the adjoint recursion, b = k-1 .. 0, and the closing step b = -1.
//   b >= 0:  zout = dtb (mu + A^T zin)          (zin = Z_{b+1}, zero when b+1 = k)
//   b = -1:  grho += mu + A^T zin               (grho may be null)
// and, when b+1 < k, gv += scale D(xb1)^T zin on the lower face of every
// cell (xb1 = T_{b+1}; each interior face belongs to exactly one cell).
template <typename T, int D>
__global__ void __launch_bounds__(256) k_up_adj(Grid g, T dtb, T inv_h, int b, const T* __restrict__ mu,
                                                const T* __restrict__ zin, T* __restrict__ zout,
                                                const T* __restrict__ xb1, const T* __restrict__ v,
                                                T* __restrict__ grho, T* __restrict__ gv, T scale,
                                                const int* __restrict__ kp) {
    const int k = *kp;
    if (b >= k) return;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    int x[3];
    cell_decode(g, c, x);
    const bool has_z = b + 1 < k;
    const T atz = has_z ? up_AT<T, D>(g, zin, v, c, x) * inv_h : (T)0;
    if (b >= 0)
        zout[c] = dtb * (mu[c] + atz);
    else if (grho)
        grho[c] += mu[c] + atz;
    if (has_z) {
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int I = x[a];
            if (I < 1) continue;
            const int s = cell_stride(g, a);
            const int f = face_at(g, a, x, I);
            const T xf = up_face(xb1, v[f], c, s, I, g.n[a]);
            gv[f] += scale * (zin[c] - zin[c - s]) * xf * inv_h;
        }
    }
}

// The series after launches 0..nl: its k, and whether it stopped (the last
// launched term passed the test, or the cap was reached).
template <typename T>
__global__ void k_up_record(UpCtl<T> ctl, int nl, typename UpBits<T>::U tolb, int* __restrict__ k_out,
                            int* __restrict__ ok_out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    *k_out = *ctl.k;
    *ok_out = (nl >= UP_KMAX || ctl.maxb[nl] < tolb) ? 1 : 0;
}

// gv = base (or 0) on interior faces, 0 on walls.
template <typename T>
__global__ void k_up_gv_init(Grid g, const T* __restrict__ base, T* __restrict__ gv) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= g.nface) return;
    int a, i, j, k;
    face_decode(g, f, a, i, j, k);
    gv[f] = face_interior(g, a, i, j, k) && base ? base[f] : (T)0;
}

// Buffers and launch sequences of the operator on one grid.
template <typename T, int D>
struct UpwindExp {
    using U = typename UpBits<T>::U;
    T* terms = nullptr;   // [UP_KMAX][ncell]: T_1 .. T_KMAX
    T* z[2] = {nullptr, nullptr};
    UpCtl<T> ctl{};
    Tracer* tr = nullptr;   // records the working term launches (j >= 1) when tracing is on

    template <typename Ar>
    void layout(Ar& A, long ncell) {
        terms = A.template take<T>((size_t)UP_KMAX * ncell);
        z[0] = A.template take<T>(ncell);
        z[1] = A.template take<T>(ncell);
        ctl.maxb = A.template take<U>(UP_KMAX + 1);
        ctl.k = A.template take<int>(1);
    }
    const T* term(const T* rho, int j, long C) const { return j == 0 ? rho : terms + (long)(j - 1) * C; }

    // terms T_1..T_k of rho (and their sum into out, unless null); k on the
    // device.  Launches terms 0..nl only: when the series has not stopped by
    // then (record() tells), the result is truncated and the caller runs it
    // again with a larger nl.
    void series(const Grid& g, double dt, const T* rho, const T* v, T* out, hipStream_t st, int nl = UP_KMAX) {
        const long C = g.ncell;
        k_fill<U><<<1, 64, 0, st>>>(UP_KMAX + 1, ctl.maxb, (U)0);
        const U tolb = UpBits<T>::of((T)UP_TOL);
        const int nb = blocks_for(C, 256);
        nl = nl < 0 ? 0 : (nl > UP_KMAX ? UP_KMAX : nl);
        for (int j = 0; j <= nl; ++j) {
            auto launch = [&] {
                k_up_term<T, D><<<nb, 256, 0, st>>>(g, j ? (T)(dt / (j * g.h)) : (T)0, j,
                                                     j ? term(rho, j - 1, C) : rho, v,
                                                     j ? terms + (long)(j - 1) * C : nullptr, out, ctl, tolb);
            };
            // every launch is recorded and credited as working; the caller takes back the credit of
            // launches past the stop (term_bytes each) once it knows k
            if (tr)
                traced(*tr, st, TR_UP_TERM, j ? term_bytes(g) : copy_bytes(g, out != nullptr), launch);
            else
                launch();
        }
    }
    // The method's bytes of one working term: T_{j-1} in, T_j out, the sum read and written per cell, v
    // per face; of the first launch (j = 0): rho in, and copied into the sum when there is one.
    static double term_bytes(const Grid& g) { return (double)sizeof(T) * (4.0 * g.ncell + (double)g.nface); }
    static double copy_bytes(const Grid& g, bool sum) { return (double)sizeof(T) * g.ncell * (sum ? 2.0 : 1.0); }
    // record = false: the call's launches are not recorded by the tracer (the caller will not learn k)
    void forward(const Grid& g, double dt, const T* rho, const T* v, T* out, hipStream_t st, int nl = UP_KMAX,
                 bool record = false) {
        Tracer* keep = tr;
        if (!record) tr = nullptr;
        series(g, dt, rho, v, out, st, nl);
        tr = keep;
    }
    // k and the stopped flag of the last series (launched to nl) into device ints
    void record(int nl, int* k_out, int* ok_out, hipStream_t st) {
        k_up_record<T><<<1, 64, 0, st>>>(ctl, nl, UpBits<T>::of((T)UP_TOL), k_out, ok_out);
    }
    // grho += (dA/drho)^T mu (grho may be null); gv = base + scale (dA/dv)^T mu
    // on interior faces, 0 on walls (base may be null).  k_known >= 0: the
    // series of (rho, v) is known to stop at that k (the forward sweep of the
    // same trajectory measured it), so exactly the needed launches are made.
    void adjoint(const Grid& g, double dt, const T* mu, const T* rho, const T* v, T* grho, T* gv, const T* base,
                 T scale, hipStream_t st, int k_known = -1) {
        const long C = g.ncell;
        const int nl = k_known >= 0 ? k_known : UP_KMAX;
        // with k unknown the launches past the stop cannot be told apart: such calls are not recorded
        Tracer* keep = tr;
        if (k_known < 0) tr = nullptr;
        series(g, dt, rho, v, nullptr, st, nl);
        tr = keep;
        k_up_gv_init<T><<<blocks_for(g.nface, 256), 256, 0, st>>>(g, base, gv);
        const int nb = blocks_for(C, 256);
        const T inv_h = (T)(1.0 / g.h);
        for (int b = (nl < UP_KMAX ? nl : UP_KMAX) - 1; b >= -1; --b)
            k_up_adj<T, D><<<nb, 256, 0, st>>>(g, (T)(dt / (b + 1 > 0 ? b + 1 : 1)), inv_h, b, mu, z[(b + 1) & 1],
                                                b >= 0 ? z[b & 1] : nullptr, term(rho, b + 1, C), v, grho, gv,
                                                scale, ctl.k);
    }
};

}  // namespace stfas
