// Device-side grid description, index maps and the clamped multilinear
// interpolation shared by every kernel of the solver.
//
// MAC grid (Sec. 3.1): cells [n2][n1][n0], faces x | y | z with shapes
// [n2][n1][n0+1], [n2][n1+1][n0], [n2+1][n1][n0]; wall faces are stored and
// held at zero.  2D problems use n2 = 1 and have no z block.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>
#include <stdint.h>

namespace stfas {

// A failed HIP call on the host side throws; the C interface turns it into
// STFAS_E_DEVICE.
struct HipError {
    hipError_t e;
};
#define HCK(x)                                   \
    do {                                         \
        hipError_t _e = (x);                     \
        if (_e != hipSuccess) throw HipError{_e}; \
    } while (0)
#define LAUNCH_CHECK() HCK(hipPeekAtLastError())

// Event tracing of one kernel family: when enabled, launches of that
// family on the finest level are bracketed by events on the context's
// stream (up to `cap` launches per enable) and their algorithmic bytes are
// summed on the host.
enum TraceKernel {
    TR_NONE = 0,
    TR_SCGS_THOMAS = 1,
    TR_SCGS_PROJECT = 2,
    TR_KKT_FACES = 3,
    TR_SELF_ADVECT_T = 4,
    TR_RBGS = 5,
    TR_ADVECT = 6,
    TR_KKT_CELLS = 7,
    TR_SCGS_CELLS = 8,
    TR_SCGS_COLOUR = 9,
    TR_KKT_SPLIT = 10,
    TR_UP_TERM = 11
};

struct Tracer {
    int id = TR_NONE;
    int cap = 0, used = 0;
    long launches = 0;
    double bytes = 0;        // the method's bytes of the recorded launches
    double impl_bytes = 0;   // every buffer the launches read or write once (with the implementation's scratch)
    std::vector<hipEvent_t> ev;
    bool on(int k) const { return id == k && used < cap; }
    // correction of the bytes credited to launches already recorded (a launch
    // that turned out to have no work, known only once the host has synchronised)
    void credit(int k, double b) {
        if (id == k) bytes += b;
    }
    void reset() {
        for (auto e : ev) (void)hipEventDestroy(e);
        ev.clear();
        id = TR_NONE;
        cap = used = 0;
        launches = 0;
        bytes = 0;
        impl_bytes = 0;
    }
};

// impl < 0: the launch moves exactly the method's bytes.
template <typename Launch>
inline void traced(Tracer& tr, hipStream_t st, int kind, double bytes, Launch&& launch, double impl = -1) {
    if (!tr.on(kind)) {
        launch();
        return;
    }
    HCK(hipEventRecord(tr.ev[2 * tr.used], st));
    launch();
    HCK(hipEventRecord(tr.ev[2 * tr.used + 1], st));
    ++tr.used;
    ++tr.launches;
    tr.bytes += bytes;
    tr.impl_bytes += impl < 0 ? bytes : impl;
}



struct Grid {
    int n[3];        // n0, n1, n2 (n2 = 1 in 2D)
    int dim;
    int ncell;
    int fcount[3];   // faces per axis (0 for z in 2D)
    int foff[3];     // offset of each axis block
    int nface;
    double h;        // cell size on this level
};

inline Grid make_grid(int dim, const int n[3], double h) {
    Grid g{};
    g.dim = dim;
    g.n[0] = n[0];
    g.n[1] = n[1];
    g.n[2] = dim == 3 ? n[2] : 1;
    g.ncell = g.n[0] * g.n[1] * g.n[2];
    g.fcount[0] = g.n[2] * g.n[1] * (g.n[0] + 1);
    g.fcount[1] = g.n[2] * (g.n[1] + 1) * g.n[0];
    g.fcount[2] = dim == 3 ? (g.n[2] + 1) * g.n[1] * g.n[0] : 0;
    g.foff[0] = 0;
    g.foff[1] = g.fcount[0];
    g.foff[2] = g.fcount[0] + g.fcount[1];
    g.nface = g.fcount[0] + g.fcount[1] + g.fcount[2];
    g.h = h;
    return g;
}

inline Grid coarse_grid(const Grid& f) {
    int n[3] = {f.n[0] / 2, f.n[1] / 2, f.dim == 3 ? f.n[2] / 2 : 1};
    return make_grid(f.dim, n, 2.0 * f.h);
}

// Extent of the a-face lattice along axis b.
__host__ __device__ inline int face_ext(const Grid& g, int a, int b) { return g.n[b] + (a == b ? 1 : 0); }

__host__ __device__ inline int cell_index(const Grid& g, int i, int j, int k) {
    return (k * g.n[1] + j) * g.n[0] + i;
}

// Flat index of a-face (i, j, k) (lattice coordinates of that axis).
__host__ __device__ inline int face_index(const Grid& g, int a, int i, int j, int k) {
    const int ex = face_ext(g, a, 0), ey = face_ext(g, a, 1);
    return g.foff[a] + (k * ey + j) * ex + i;
}

// Decode a flat face index into (axis, i, j, k).
__device__ inline void face_decode(const Grid& g, int f, int& a, int& i, int& j, int& k) {
    a = (f >= g.foff[1]) + (g.dim == 3 && f >= g.foff[2]);
    int r = f - g.foff[a];
    const int ex = face_ext(g, a, 0), ey = face_ext(g, a, 1);
    i = r % ex;
    r /= ex;
    j = r % ey;
    k = r / ey;
}

__device__ inline bool face_interior(const Grid& g, int a, int i, int j, int k) {
    const int c = a == 0 ? i : (a == 1 ? j : k);
    return c >= 1 && c <= g.n[a] - 1;
}

// One axis of the clamped multilinear interpolation on a lattice with M
// nodes:  yc = clamp(y, 0, M-1),  i0 = min(floor(yc), M-2),  t = yc - i0;
// the derivative of the interpolant along this axis is multiplied by 1 on
// the closed box [0, M-1] and 0 outside.
template <typename T>
struct Axis {
    int i0;
    T t;
    T in;
};

template <typename T>
__device__ inline Axis<T> locate(T y, int M) {
    Axis<T> s;
    const T top = (T)(M - 1);
    // fmax/fmin return the non-NaN operand, so a NaN foot point is clamped
    // to node 0 and every corner index stays inside the lattice.
    const T yc = fmin(fmax(y, (T)0), top);
    int i = (int)floor(yc);
    if (i < 0) i = 0;
    if (i > M - 2) i = M - 2;
    s.i0 = i;
    s.t = yc - (T)i;
    s.in = (y >= (T)0 && y <= top) ? (T)1 : (T)0;
    return s;
}

// The same axis for a backtrace Y = X + delta from an integer node X.  The
// base cell and the fraction come from delta alone (floor(X + delta) =
// X + floor(delta)), which keeps the fraction accurate in FP32 where X is
// large and delta small.  Identical to locate(X + delta, M) in exact
// arithmetic, including the clamp and its derivative on the closed box.
template <typename T>
__device__ inline Axis<T> locate_disp(int X, T delta, int M) {
    Axis<T> s;
    const T lim = (T)(2 * M + 2);
    const T d = fmin(fmax(delta, -lim), lim);      // also maps NaN to -lim
    const T fl = floor(d);
    int i = X + (int)fl;
    T t = d - fl;
    if (i < 0) {                                    // Y < 0: clamped to node 0
        s.i0 = 0;
        s.t = (T)0;
        s.in = (T)0;
    } else if (i >= M - 1) {                        // Y >= M-1: clamped to the top node
        s.i0 = M - 2;
        s.t = (T)1;
        s.in = (i == M - 1 && t == (T)0) ? (T)1 : (T)0;
    } else {
        s.i0 = i;
        s.t = t;
        s.in = (T)1;
    }
    return s;
}

// Lattice with extents ex, ey (ez implied) and x-fastest strides.
template <typename T, int D>
struct Interp {
    Axis<T> ax[3];
    int base;   // flat index of corner (i0, j0, k0)
    int sy, sz; // strides

    __device__ inline void setup(const T* y, int ex, int ey, int ez) {
        ax[0] = locate<T>(y[0], ex);
        ax[1] = locate<T>(y[1], ey);
        if (D == 3) ax[2] = locate<T>(y[2], ez);
        sy = ex;
        sz = ex * ey;
        base = ax[0].i0 + ax[1].i0 * sy + (D == 3 ? ax[2].i0 * sz : 0);
    }

    // Backtrace from integer node X by displacement delta (see locate_disp).
    __device__ inline void setup_disp(const int* X, const T* delta, int ex, int ey, int ez) {
        ax[0] = locate_disp<T>(X[0], delta[0], ex);
        ax[1] = locate_disp<T>(X[1], delta[1], ey);
        if (D == 3) ax[2] = locate_disp<T>(X[2], delta[2], ez);
        sy = ex;
        sz = ex * ey;
        base = ax[0].i0 + ax[1].i0 * sy + (D == 3 ? ax[2].i0 * sz : 0);
    }

    // C1 variant of the weights, used by the velocity self-advection: every
    // fraction t becomes the smoothstep s(t) = t^2 (3 - 2t) and the position
    // derivative gains the factor s'(t) = 6t(1 - t).  The weights stay convex
    // and interpolate the nodes; the gradient, which the plain multilinear
    // weights make jump across lattice lines, becomes continuous (s' vanishes
    // on both sides of every lattice line).  Call after setup/setup_disp.
    __device__ inline void c1() {
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const T t = ax[a].t;
            ax[a].in *= (T)6 * t * ((T)1 - t);
            ax[a].t = t * t * ((T)3 - (T)2 * t);
        }
    }

    __device__ inline int corner(int c) const {
        return base + (c & 1) + ((c >> 1) & 1) * sy + (D == 3 ? ((c >> 2) & 1) * sz : 0);
    }

    __device__ inline T weight(int c) const {
        T w = (c & 1) ? ax[0].t : (T)1 - ax[0].t;
        w *= ((c >> 1) & 1) ? ax[1].t : (T)1 - ax[1].t;
        if (D == 3) w *= ((c >> 2) & 1) ? ax[2].t : (T)1 - ax[2].t;
        return w;
    }

    // d weight(c) / d y_a (times the clamp derivative).
    __device__ inline T dweight(int c, int a) const {
        T w = ax[a].in * (((c >> a) & 1) ? (T)1 : (T)-1);
        for (int b = 0; b < D; ++b) {
            if (b == a) continue;
            w *= ((c >> b) & 1) ? ax[b].t : (T)1 - ax[b].t;
        }
        return w;
    }

    __device__ inline T value(const T* q) const {
        T s = 0;
#pragma unroll
        for (int c = 0; c < (1 << D); ++c) s += weight(c) * q[corner(c)];
        return s;
    }

    __device__ inline void grad(const T* q, T* g) const {
#pragma unroll
        for (int a = 0; a < D; ++a) g[a] = 0;
#pragma unroll
        for (int c = 0; c < (1 << D); ++c) {
            const T qc = q[corner(c)];
#pragma unroll
            for (int a = 0; a < D; ++a) g[a] += dweight(c, a) * qc;
        }
    }
};

// a[i] for a small array and a runtime index, by selects (no private memory).
template <typename U, int K>
__device__ inline U pick(const U (&a)[K], int i) {
    U r = a[0];
#pragma unroll
    for (int e = 1; e < K; ++e) r = (e == i) ? a[e] : r;
    return r;
}

template <typename T>
__device__ inline void atomic_add(T* p, T v) {
    atomicAdd(p, v);
}

inline int blocks_for(long n, int bs) { return (int)((n + bs - 1) / bs); }

}  // namespace stfas
