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
// Device form: each block folds max|T_j| into a per-term word with atomicMax
// on the bit pattern (non-negative floats order like their bits); a launch
// reads the words of the terms before it and returns at once when the series
// has already stopped, so a fixed sequence of launches needs no host
// synchronisation.  A closing launch finds k from the words.  The adjoint
// launches read k and are empty for b >= k.  In 3D a launch is one term (or
// one adjoint step) of the whole grid; in 2D a launch is several terms of
// one tile (below).
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
    int* stopped;                  // 1 when the series stopped within the launched terms (or at the cap)
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

// ---------------------------------------------------------------- 2D: several terms per launch
//
// On a 2D grid one term is a few microseconds of work behind a launch, so a
// launch here takes UP_M consecutive terms (or adjoint steps) of one TS x TS
// tile of cells.  Term j at a cell reads term j-1 within two cells along each
// axis (the second-order upstream value), so after t terms only the cells at
// least 2t from the edge of the loaded region are exact: the tile is loaded
// with a halo of 2 UP_M cells and each term is computed on the region shrunk
// by two more cells, in LDS.  Every term at every cell is the same expression
// of the same values as in the one-term launch; the halo cells are computed
// again by the neighbouring tiles.  A launch block has one thread per cell
// of the loaded 32 x 32 region.
//
// A launch cannot know whether one of its own terms ends the series (that is
// a maximum over all tiles), so it computes all of its terms and the sum is
// formed after the last launch (k_up_close), in the order of the one-term
// launches: rho, then T_1, T_2, ... T_k.

constexpr int UP_M = 4;                          // terms (adjoint steps) per launch
constexpr int UP_TS = 16;                        // tile edge in cells
constexpr int UP_R = UP_TS + 4 * UP_M;           // edge of the loaded region (tile + halo)
constexpr int UP_NT = UP_R * UP_R;               // one thread per region cell
static_assert(UP_NT <= 1024, "one thread per cell of the loaded region");

// Fold the per-wave maxima of nt terms (wm[t][wave]) into ctl words j0 .. j0+nt-1.
template <typename T>
__device__ inline void fold_term_maxima(T (*wm)[UP_NT / 64], int nt, int j0, typename UpBits<T>::U* maxb) {
    const int t = threadIdx.x;
    if (t >= nt) return;
    T b = wm[t][0];
#pragma unroll
    for (int w = 1; w < UP_NT / 64; ++w) b = fmax(b, wm[t][w]);
    const typename UpBits<T>::U bb = UpBits<T>::of(b);
    if (bb > __hip_atomic_load(maxb + j0 + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(maxb + j0 + t, bb);
}

// dst[q] = value(q) for q < n (n <= NMAX), q = threadIdx.x + i UP_NT: a
// thread issues all of its loads before its first LDS store, so the load
// latencies overlap.
template <int NMAX, typename T, typename F>
__device__ inline void stage_lds(T* dst, int n, F value) {
    constexpr int K = (NMAX + UP_NT - 1) / UP_NT;
    T r[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int q = threadIdx.x + i * UP_NT;
        r[i] = q < n ? value(q) : (T)0;
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int q = threadIdx.x + i * UP_NT;
        if (q < n) dst[q] = r[i];
    }
}

template <typename T>
__device__ inline T wave_max(T m) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    return m;
}

// Upwind face value from an LDS row: cells at offsets -2 .. +1 around the face
// (lo2 = x[cL - s], lo1 = x[cL], hi1 = x[cR], hi2 = x[cR + s]); I is the face's
// index along the axis, n the cell count.
template <typename T>
__device__ inline T up_face_lds(T vf, T lo2, T lo1, T hi1, T hi2, int I, int n) {
    if (vf >= (T)0) return I >= 2 ? (T)1.5 * lo1 - (T)0.5 * lo2 : lo1;
    return I + 1 <= n - 1 ? (T)1.5 * hi1 - (T)0.5 * hi2 : hi1;
}

// Terms j0 .. j0+nt-1 of the series of one tile (2D).  prev = T_{j0-1} on
// the whole grid (rho when j0 = 1, whose maximum this launch also measures);
// T_j goes to terms + (j-1) C.  Returns at once when an earlier term has
// already passed the test.
template <typename T>
__global__ void __launch_bounds__(UP_NT) k_up_fwd_block(Grid g, double dt, int j0, int nt, const T* __restrict__ prev,
                                                        const T* __restrict__ v, T* __restrict__ terms, UpCtl<T> ctl,
                                                        typename UpBits<T>::U tolb) {
    constexpr int H = 2 * UP_M, R = UP_R;
    __shared__ T buf[2][R * R];
    __shared__ T vx[R * (R + 1)];     // x-face at (rx, ry): vx[ry (R+1) + rx], rx in [0, R]
    __shared__ T vy[(R + 1) * R];     // y-face at (rx, ry): vy[ry R + rx], ry in [0, R]
    __shared__ T wm[UP_M + 1][UP_NT / 64];
    int stop = 0;   // an earlier launch's term (T_0 .. T_{j0-1}) passed the test
    for (int j = threadIdx.x; j0 > 1 && j < j0; j += UP_NT) stop |= ctl.maxb[j] < tolb;
    if (__syncthreads_or(stop)) return;
    const int nx = g.n[0], ny = g.n[1];
    const long C = g.ncell;
    const int ox = blockIdx.x * UP_TS - H, oy = blockIdx.y * UP_TS - H;
    stage_lds<R * R>(buf[0], R * R, [&](int q) {
        const int x = ox + q % R, y = oy + q / R;
        return (x >= 0 && x < nx && y >= 0 && y < ny) ? prev[x + (long)y * nx] : (T)0;
    });
    stage_lds<R * (R + 1)>(vx, R * (R + 1), [&](int q) {
        const int x = ox + q % (R + 1), y = oy + q / (R + 1);
        return (x >= 0 && x <= nx && y >= 0 && y < ny) ? v[face_index(g, 0, x, y, 0)] : (T)0;
    });
    stage_lds<(R + 1) * R>(vy, (R + 1) * R, [&](int q) {
        const int x = ox + q % R, y = oy + q / R;
        return (x >= 0 && x < nx && y >= 0 && y <= ny) ? v[face_index(g, 1, x, y, 0)] : (T)0;
    });
    __syncthreads();
    // this thread's region cell; its maxima of |T_j| when it is a tile cell
    // (mt[0]: T_0, measured by the first launch), reduced after the last term
    const int rx = threadIdx.x % R, ry = threadIdx.x / R, x = ox + rx, y = oy + ry, c = threadIdx.x;
    const bool in = x >= 0 && x < nx && y >= 0 && y < ny;
    const bool mine = in && rx >= H && rx < H + UP_TS && ry >= H && ry < H + UP_TS;
    T mt[UP_M + 1];
#pragma unroll
    for (int t = 0; t <= UP_M; ++t) mt[t] = 0;
    if (j0 == 1 && mine) mt[0] = fabs(buf[0][c]);
    int cur = 0;
#pragma unroll
    for (int t = 1; t <= UP_M; ++t) {
        if (t > nt) break;
        const int j = j0 - 1 + t;
        const T coef = (T)(dt / (j * g.h));
        const T* p = buf[cur];
        T* o = buf[cur ^ 1];
        // exact on the region shrunk by 2t (each term reads two cells along each axis)
        if (in && rx >= 2 * t && rx < R - 2 * t && ry >= 2 * t && ry < R - 2 * t) {
            T acc = 0;
            if (x >= 1) {                          // x: lower face x
                const T vf = vx[ry * (R + 1) + rx];
                acc += vf * up_face_lds(vf, p[c - 2], p[c - 1], p[c], p[c + 1], x, nx);
            }
            if (x + 1 <= nx - 1) {                 // x: upper face x + 1
                const T vf = vx[ry * (R + 1) + rx + 1];
                acc -= vf * up_face_lds(vf, p[c - 1], p[c], p[c + 1], p[c + 2], x + 1, nx);
            }
            if (y >= 1) {                          // y: lower face y
                const T vf = vy[ry * R + rx];
                acc += vf * up_face_lds(vf, p[c - 2 * R], p[c - R], p[c], p[c + R], y, ny);
            }
            if (y + 1 <= ny - 1) {                 // y: upper face y + 1
                const T vf = vy[(ry + 1) * R + rx];
                acc -= vf * up_face_lds(vf, p[c - R], p[c], p[c + R], p[c + 2 * R], y + 1, ny);
            }
            const T val = coef * acc;
            o[c] = val;
            if (mine) {
                terms[(long)(j - 1) * C + x + (long)y * nx] = val;
                mt[t] = fabs(val);
            }
        }
        __syncthreads();
        cur ^= 1;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int t = 0; t <= UP_M; ++t) {
        const T m = wave_max(mt[t]);
        if (lane == 0) wm[t][wave] = m;
    }
    __syncthreads();
    if (j0 == 1) fold_term_maxima<T>(wm, nt + 1, 0, ctl.maxb);
    else fold_term_maxima<T>(wm + 1, nt, j0, ctl.maxb);
}

// acc + (A^T z) h at an LDS cell c for one axis, cell stride s: vf0 points
// at the cell's lower face of that axis (index I along it, n cells), the
// faces I-1 .. I+2 are at face offsets -1 .. +2 (pitch sv).  The terms are
// added in the order of the one-step kernel.
template <typename T>
__device__ inline T up_AT_axis(T acc, const T* __restrict__ z, int c, int s, const T* __restrict__ vf0, int sv, int I,
                               int n) {
    if (I + 1 <= n - 1) {
        const T vf = vf0[sv];
        if (vf >= (T)0) acc += (I >= 1 ? (T)1.5 : (T)1) * vf * (z[c + s] - z[c]);
    }
    if (I + 2 <= n - 1) {
        const T vf = vf0[2 * sv];
        if (vf >= (T)0) acc -= (T)0.5 * vf * (z[c + 2 * s] - z[c + s]);
    }
    if (I >= 1) {
        const T vf = vf0[0];
        if (vf < (T)0) acc += (I + 1 <= n - 1 ? (T)1.5 : (T)1) * vf * (z[c] - z[c - s]);
    }
    if (I >= 2) {
        const T vf = vf0[-sv];
        if (vf < (T)0) acc -= (T)0.5 * vf * (z[c - s] - z[c - 2 * s]);
    }
    return acc;
}

// Adjoint steps b = b0 .. max(b0 - UP_M + 1, -1) of one tile (2D); steps
// with b >= k are skipped.  zin = Z_{b0+1} (read only when the first active
// step needs it), zout = Z of the last step when that step is >= 0; grho at
// b = -1; gv of the tile's cells' lower faces gathered in registers over the
// steps, in the order of the one-step launches.
template <typename T>
__global__ void __launch_bounds__(UP_NT) k_up_adj_block(Grid g, double dt, int b0, const T* __restrict__ mu,
                                                        const T* __restrict__ zin, T* __restrict__ zout,
                                                        const T* __restrict__ rho, const T* __restrict__ terms,
                                                        const T* __restrict__ v, T* __restrict__ grho,
                                                        T* __restrict__ gv, T scale, const int* __restrict__ kp) {
    constexpr int H = 2 * UP_M, R = UP_R, X = UP_TS + 4;
    __shared__ T zb[2][R * R];
    __shared__ T mus[R * R];
    __shared__ T vx[R * (R + 1)];
    __shared__ T vy[(R + 1) * R];
    __shared__ T xb[X * X];          // T_{b+1} on the tile and two cells around it
    const int k = *kp;
    const int blo = b0 - UP_M + 1 < -1 ? -1 : b0 - UP_M + 1;
    const int bs = b0 < k - 1 ? b0 : k - 1;
    if (bs < blo) return;            // every step of this launch is past the series
    const int nx = g.n[0], ny = g.n[1];
    const long C = g.ncell;
    const int ox = blockIdx.x * UP_TS - H, oy = blockIdx.y * UP_TS - H;
    const bool zin_used = bs + 1 < k;
    stage_lds<R * R>(mus, R * R, [&](int q) {
        const int x = ox + q % R, y = oy + q / R;
        return (x >= 0 && x < nx && y >= 0 && y < ny) ? mu[x + (long)y * nx] : (T)0;
    });
    stage_lds<R * R>(zb[0], R * R, [&](int q) {
        const int x = ox + q % R, y = oy + q / R;
        return (zin_used && x >= 0 && x < nx && y >= 0 && y < ny) ? zin[x + (long)y * nx] : (T)0;
    });
    stage_lds<R * (R + 1)>(vx, R * (R + 1), [&](int q) {
        const int x = ox + q % (R + 1), y = oy + q / (R + 1);
        return (x >= 0 && x <= nx && y >= 0 && y < ny) ? v[face_index(g, 0, x, y, 0)] : (T)0;
    });
    stage_lds<(R + 1) * R>(vy, (R + 1) * R, [&](int q) {
        const int x = ox + q % R, y = oy + q / R;
        return (x >= 0 && x < nx && y >= 0 && y <= ny) ? v[face_index(g, 1, x, y, 0)] : (T)0;
    });
    // this thread's region cell; a tile cell also owns its lower faces' gv,
    // gathered in registers over the steps
    const int rx = threadIdx.x % R, ry = threadIdx.x / R, x = ox + rx, y = oy + ry, c = threadIdx.x;
    const bool in = x >= 0 && x < nx && y >= 0 && y < ny;
    const bool mine = in && rx >= H && rx < H + UP_TS && ry >= H && ry < H + UP_TS;
    const int fx = mine && x >= 1 ? face_index(g, 0, x, y, 0) : -1;
    const int fy = mine && y >= 1 ? face_index(g, 1, x, y, 0) : -1;
    T gx = fx >= 0 ? gv[fx] : (T)0, gy = fy >= 0 ? gv[fy] : (T)0;
    const int e = (ry - H + 2) * X + (rx - H + 2);     // the cell in xb (tile cells only)
    const T inv_h = (T)(1.0 / g.h);
    int cur = 0;
    for (int b = bs, t = 0; b >= blo; --b, ++t) {
        const bool has_z = b + 1 < k;
        if (has_z) {
            const T* xs = b + 1 == 0 ? rho : terms + (long)b * C;      // T_{b+1}
            stage_lds<X * X>(xb, X * X, [&](int q) {
                const int xx = ox + H - 2 + q % X, yy = oy + H - 2 + q / X;
                return (xx >= 0 && xx < nx && yy >= 0 && yy < ny) ? xs[xx + (long)yy * nx] : (T)0;
            });
        }
        __syncthreads();
        const T* z = zb[cur];
        T* zo = zb[cur ^ 1];
        const T dtb = (T)(dt / (b + 1 > 0 ? b + 1 : 1));
        // Z_b is exact on the region shrunk by 2 (t + 1); at b = -1 only the tile's grho is formed
        const int lo = 2 * (t + 1);
        const bool act = b >= 0 ? in && rx >= lo && rx < R - lo && ry >= lo && ry < R - lo : mine;
        if (act) {
            T atz = 0;
            if (has_z)
                atz = up_AT_axis<T>(up_AT_axis<T>((T)0, z, c, 1, vx + ry * (R + 1) + rx, 1, x, nx), z, c, R,
                                    vy + ry * R + rx, R, y, ny) * inv_h;
            if (b >= 0)
                zo[c] = dtb * (mus[c] + atz);
            else if (grho)
                grho[x + (long)y * nx] += mus[c] + atz;
        }
        if (has_z && mine) {
            if (fx >= 0) {
                const T vf = vx[ry * (R + 1) + rx];
                const T xf = up_face_lds(vf, xb[e - 2], xb[e - 1], xb[e], xb[e + 1], x, nx);
                gx += scale * (z[c] - z[c - 1]) * xf * inv_h;
            }
            if (fy >= 0) {
                const T vf = vy[ry * R + rx];
                const T xf = up_face_lds(vf, xb[e - 2 * X], xb[e - X], xb[e], xb[e + X], y, ny);
                gy += scale * (z[c] - z[c - R]) * xf * inv_h;
            }
        }
        __syncthreads();
        cur ^= 1;
    }
    if (blo >= 0 && mine) zout[x + (long)y * nx] = zb[cur][c];
    if (fx >= 0) gv[fx] = gx;
    if (fy >= 0) gv[fy] = gy;
}

// What the closing launch of a series also does: the caller's copies of k
// and of the stop flag (either may be null), and gv = base (or 0) on interior
// faces and 0 on walls when gv is given (the start of an adjoint).
template <typename T>
struct UpClose {
    int* k_out = nullptr;
    int* ok_out = nullptr;
    const T* gv_base = nullptr;
    T* gv = nullptr;
    int k_set = -1;   // >= 0: no series was launched; k is this (known) value
};

// After a series launched to nl: k = the first j <= nl with max|T_j| below
// the threshold (nl when there is none), whether the series stopped, and,
// when out is given, out = rho + T_1 + ... + T_k in that order.  It also
// clears `next`, the threshold words of the following series (the words
// alternate between two sets, so no launch clears the set in use), and does
// the extras of `x`.  next may be null (nothing to clear).
template <typename T>
__global__ void __launch_bounds__(256) k_up_close(Grid g, UpCtl<T> ctl, typename UpBits<T>::U* __restrict__ next,
                                                  int nl, typename UpBits<T>::U tolb, const T* __restrict__ rho,
                                                  const T* __restrict__ terms, T* __restrict__ out, UpClose<T> x) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (next && id <= UP_KMAX) next[id] = 0;
    if (x.gv && id < g.nface) {
        int a, i, j, kk;
        face_decode(g, (int)id, a, i, j, kk);
        x.gv[id] = face_interior(g, a, i, j, kk) && x.gv_base ? x.gv_base[id] : (T)0;
    }
    // k: the lowest word below the threshold, one word per lane (nl <= 48 < 64)
    const int lane = threadIdx.x & 63;
    const bool below = x.k_set < 0 && lane <= nl && ctl.maxb[lane] < tolb;
    const unsigned long long mask = __ballot(below);
    const int found = x.k_set >= 0 || mask != 0;
    const int k = x.k_set >= 0 ? x.k_set : (mask ? __builtin_ctzll(mask) : nl);
    if (id == 0) {
        const int stopped = found || nl >= UP_KMAX;
        *ctl.k = k;
        *ctl.stopped = stopped;
        if (x.k_out) *x.k_out = k;
        if (x.ok_out) *x.ok_out = stopped;
    }
    const long C = g.ncell;
    if (!out || id >= C) return;
    // added in the order j = 1 .. k; four terms' loads issued together
    T s = rho[id];
    int j = 1;
    for (; j + 3 <= k; j += 4) {
        const T* t = terms + (long)(j - 1) * C + id;
        const T a0 = t[0], a1 = t[C], a2 = t[2 * C], a3 = t[3 * C];
        s += a0;
        s += a1;
        s += a2;
        s += a3;
    }
    for (; j <= k; ++j) s += terms[(long)(j - 1) * C + id];
    out[id] = s;
}

// Buffers and launch sequences of the operator on one grid.
template <typename T, int D>
struct UpwindExp {
    using U = typename UpBits<T>::U;
    T* terms = nullptr;   // [UP_KMAX][ncell]: T_1 .. T_KMAX
    T* z[2] = {nullptr, nullptr};
    // 2D: the terms of every step of two density trajectories, [steps][UP_KMAX][ncell] each, so that an
    // adjoint sweep over a trajectory whose forward sweep stored its terms launches no series
    T* hist[2] = {nullptr, nullptr};
    UpCtl<T> ctl{};
    U* maxb_set[2] = {nullptr, nullptr};   // the threshold words of alternate series
    int par = 0;
    bool primed = false;                   // both sets cleared once
    Tracer* tr = nullptr;   // records the working term launches (j >= 1) when tracing is on

    template <typename Ar>
    void layout(Ar& A, long ncell, int hist_steps = 0) {
        terms = A.template take<T>((size_t)UP_KMAX * ncell);
        if (D == 2 && hist_steps > 0) {
            hist[0] = A.template take<T>((size_t)hist_steps * UP_KMAX * ncell);
            hist[1] = A.template take<T>((size_t)hist_steps * UP_KMAX * ncell);
        }
        z[0] = A.template take<T>(ncell);
        z[1] = A.template take<T>(ncell);
        maxb_set[0] = A.template take<U>(UP_KMAX + 1);
        maxb_set[1] = A.template take<U>(UP_KMAX + 1);
        ctl.maxb = maxb_set[0];
        ctl.k = A.template take<int>(1);
        ctl.stopped = A.template take<int>(1);
    }
    const T* term(const T* rho, int j, long C) const { return j == 0 ? rho : terms + (long)(j - 1) * C; }
    // where step i of trajectory `set` keeps its terms (null without stored trajectories)
    T* hist_step(int set, int i, long C) const { return hist[set] ? hist[set] + (size_t)i * UP_KMAX * C : nullptr; }

    // terms T_1..T_k of rho (and their sum into out, unless null); k on the
    // device.  Launches terms 0..nl only: when the series has not stopped by
    // then (record() tells), the result is truncated and the caller runs it
    // again with a larger nl.
    // tb (2D, may be null): where the terms go instead of the operator's own buffer
    void series(const Grid& g, double dt, const T* rho, const T* v, T* out, hipStream_t st, int nl = UP_KMAX,
                UpClose<T> x = {}, T* tb = nullptr) {
        const long C = g.ncell;
        T* tt = tb ? tb : terms;
        if (!primed) {
            k_fill<U><<<1, 64, 0, st>>>(UP_KMAX + 1, maxb_set[0], (U)0);
            k_fill<U><<<1, 64, 0, st>>>(UP_KMAX + 1, maxb_set[1], (U)0);
            primed = true;
        }
        ctl.maxb = maxb_set[par];
        U* next = maxb_set[par ^ 1];
        par ^= 1;
        const long nclose = std::max<long>(std::max<long>(out ? C : 0, UP_KMAX + 1), x.gv ? g.nface : 0);
        const U tolb = UpBits<T>::of((T)UP_TOL);
        nl = nl < 0 ? 0 : (nl > UP_KMAX ? UP_KMAX : nl);
        if constexpr (D == 2) {
            const dim3 tiles(blocks_for(g.n[0], UP_TS), blocks_for(g.n[1], UP_TS));
            for (int j0 = 1; j0 == 1 || j0 <= nl; j0 += UP_M) {
                const int nt = nl - j0 + 1 < UP_M ? nl - j0 + 1 : UP_M;   // 0 only when nl = 0
                auto launch = [&] {
                    k_up_fwd_block<T><<<tiles, UP_NT, 0, st>>>(g, dt, j0, nt,
                                                               j0 == 1 ? rho : tt + (long)(j0 - 2) * C, v, tt,
                                                               ctl, tolb);
                };
                if (tr)
                    traced(*tr, st, TR_UP_TERM,
                           nt * term_bytes(g) + (j0 == 1 ? copy_bytes(g, out != nullptr) : 0.0), launch);
                else
                    launch();
            }
            k_up_close<T><<<blocks_for(nclose, 256), 256, 0, st>>>(g, ctl, next, nl, tolb, rho, tt, out, x);
        } else {
            series_terms(g, dt, rho, v, out, st, nl, tolb);
            k_up_close<T><<<blocks_for(nclose, 256), 256, 0, st>>>(g, ctl, next, nl, tolb, rho, terms, nullptr, x);
        }
    }
    // 3D: one launch per term over the whole grid, the sum added in each
    void series_terms(const Grid& g, double dt, const T* rho, const T* v, T* out, hipStream_t st, int nl, U tolb) {
        const long C = g.ncell;
        const int nb = blocks_for(C, 256);
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
    // k_out, ok_out (device ints, may be null): the series' k and whether it stopped within the nl terms
    // tb (2D, may be null): keep the terms there (a stored trajectory's step)
    void forward(const Grid& g, double dt, const T* rho, const T* v, T* out, hipStream_t st, int nl = UP_KMAX,
                 bool record = false, int* k_out = nullptr, int* ok_out = nullptr, T* tb = nullptr) {
        Tracer* keep = tr;
        if (!record) tr = nullptr;
        UpClose<T> x;
        x.k_out = k_out;
        x.ok_out = ok_out;
        series(g, dt, rho, v, out, st, nl, x, tb);
        tr = keep;
    }
    // grho += (dA/drho)^T mu (grho may be null); gv = base + scale (dA/dv)^T mu
    // on interior faces, 0 on walls (base may be null).  k_known >= 0: the
    // series of (rho, v) is known to stop at that k (the forward sweep of the
    // same trajectory measured it), so exactly the needed launches are made.
    // stored (2D, with k_known): the terms of this series as its forward sweep kept them; no series is
    // launched then
    void adjoint(const Grid& g, double dt, const T* mu, const T* rho, const T* v, T* grho, T* gv, const T* base,
                 T scale, hipStream_t st, int k_known = -1, const T* stored = nullptr) {
        const int nl = k_known >= 0 ? k_known : UP_KMAX;
        if constexpr (D == 2) {
            if (stored && k_known >= 0) {
                UpClose<T> x;
                x.gv_base = base;
                x.gv = gv;
                x.k_set = k_known;
                const long nclose = std::max<long>(UP_KMAX + 1, g.nface);
                k_up_close<T><<<blocks_for(nclose, 256), 256, 0, st>>>(g, ctl, nullptr, nl, (U)0, rho, stored,
                                                                       nullptr, x);
                adjoint_tiles(g, dt, mu, rho, v, grho, gv, scale, st, nl - 1, stored);
                return;
            }
        }
        // with k unknown the launches past the stop cannot be told apart: such calls are not recorded
        Tracer* keep = tr;
        if (k_known < 0) tr = nullptr;
        UpClose<T> x;
        x.gv_base = base;
        x.gv = gv;
        series(g, dt, rho, v, nullptr, st, nl, x);
        tr = keep;
        const int top = (nl < UP_KMAX ? nl : UP_KMAX) - 1;
        if constexpr (D == 2)
            adjoint_tiles(g, dt, mu, rho, v, grho, gv, scale, st, top, terms);
        else
            adjoint_steps(g, dt, mu, rho, v, grho, gv, scale, st, top);
    }
    // 2D: UP_M steps of the recursion per launch, from b = top down to -1 (k on the device)
    void adjoint_tiles(const Grid& g, double dt, const T* mu, const T* rho, const T* v, T* grho, T* gv, T scale,
                       hipStream_t st, int top, const T* tt) {
        const dim3 tiles(blocks_for(g.n[0], UP_TS), blocks_for(g.n[1], UP_TS));
        int p = 0;
        for (int b0 = top; b0 >= -1; b0 -= UP_M, p ^= 1)
            k_up_adj_block<T><<<tiles, UP_NT, 0, st>>>(g, dt, b0, mu, z[p], z[p ^ 1], rho, tt, v, grho, gv, scale,
                                                       ctl.k);
    }
    // 3D: one launch per step of the recursion over the whole grid
    void adjoint_steps(const Grid& g, double dt, const T* mu, const T* rho, const T* v, T* grho, T* gv, T scale,
                       hipStream_t st, int top) {
        const long C = g.ncell;
        const int nb = blocks_for(C, 256);
        const T inv_h = (T)(1.0 / g.h);
        for (int b = top; b >= -1; --b)
            k_up_adj<T, D><<<nb, 256, 0, st>>>(g, (T)(dt / (b + 1 > 0 ? b + 1 : 1)), inv_h, b, mu, z[(b + 1) & 1],
                                                b >= 0 ? z[b & 1] : nullptr, term(rho, b + 1, C), v, grho, gv,
                                                scale, ctl.k);
    }
};

}  // namespace stfas
