// Velocity-subproblem kernels: KKT residual (Sec. 4.2 eq:KKTAO with the
// semi-Lagrangian step), spacetime SCGS smoother (Sec. 4.3, eq:HESS) and the
// FAS transfers (Sec. 4.3).
//
// State of one level (N slots per field): v[j] = v_{j+1}, pbar[j] =
// pbar_{j+1}, u[j] = u_j, p[j] = p_{j+1}; v_0 = 0 is fixed.  Residual rows
// use the same slots: F1 ~ v, F2 ~ pbar, F3 ~ u, F4 ~ p.
//   F1_i = (K/r)[i<N](v_i - w_i) - [i<N] J_S(v_i)^T u_i/dt + u_{i-1}/dt + G pbar_i
//   F2_i = D v_i
//   F3_i = (v_{i+1} - S(v_i))/dt - u_i + G p_{i+1}      (S(v_0) = 0)
//   F4_i = D u_i
// Kernels compute out = res + sgn f (sgn = -1: residual res - f; sgn = +1:
// the FAS right-hand side f(R x) + R r).
//
// With the rotational operator of eq:NSA (2D, k_rot.hpp) the rows are those
// of eq:KKTAO as printed:
//   F1_i = (K/r)[i<N](v_i - w_i) - [i<N] u_i/dt + u_{i-1}/dt + J_Adv(v_i)^T u_{i-1} + G pbar_i
//   F3_i = (v_{i+1} - v_i)/dt + Adv[v_{i+1}] - u_i + G p_{i+1}
// all local stencils (no transpose part).
#pragma once
#include "common.hpp"
#include "k_advect.hpp"
#include "k_rot.hpp"

namespace stfas {

// Face rows F1, F3 of face f, slice j, without the J_S^T term of F1 (added
// by the velocity-advection transpose).
template <typename T, int D>
__device__ inline void kkt_face(const Grid& g, int N, T dt, T kr, T cfl, T sgn, const T* __restrict__ v,
                                const T* __restrict__ pb, const T* __restrict__ u, const T* __restrict__ p,
                                const T* __restrict__ w, const T* res1, const T* res3, T* out1, T* out3, int f,
                                int j, int vort = 0) {
    const long F = g.nface, C = g.ncell;
    int a, i, jj, k;
    face_decode(g, f, a, i, jj, k);
    const long e = j * F + f;
    if (!face_interior(g, a, i, jj, k)) {
        out1[e] = (T)0;
        out3[e] = (T)0;
        return;
    }
    const int c = cell_index(g, i, jj, k);
    const int cm = cell_index(g, i - (a == 0), jj - (a == 1), k - (a == 2));
    const T ih = (T)(1.0 / g.h);
    if (vort) {
        // F1_{j+1} = u_j/dt + G pbar + J_Adv(v_{j+1})^T u_j [+ (K/r)(v - w) - u_{j+1}/dt]
        T f1 = u[e] / dt + (pb[j * C + c] - pb[j * C + cm]) * ih;
        f1 += rot_adv_T<T, D>(g, v + j * F, u + j * F, a, i, jj, k, ih);
        if (j < N - 1) f1 += kr * (v[e] - w[(j + 1) * F + f]) - u[e + F] / dt;
        // F3_j = (v_{j+1} - v_j)/dt + Adv[v_{j+1}] - u_j + G p_{j+1}
        const T vprev = j >= 1 ? v[e - F] : (T)0;
        const T f3 = (v[e] - vprev) / dt + rot_adv<T, D>(g, v + j * F, a, i, jj, k, ih) - u[e] +
                     (p[j * C + c] - p[j * C + cm]) * ih;
        out1[e] = (res1 ? res1[e] : (T)0) + sgn * f1;
        out3[e] = (res3 ? res3[e] : (T)0) + sgn * f3;
        return;
    }
    // F1_{j+1}
    T f1 = u[e] / dt + (pb[j * C + c] - pb[j * C + cm]) * ih;
    if (j < N - 1) f1 += kr * (v[e] - w[(j + 1) * F + f]);
    // F3_j
    T s = 0;
    if (j >= 1) {
        const T* vp = v + (j - 1) * F;
        T vh[3];
        face_velocity<T, D>(g, vp, a, i, jj, k, vh);
        const int idx[3] = {i, jj, k};
        T y[3];
        for (int b = 0; b < D; ++b) y[b] = -cfl * vh[b];
        Interp<T, D> it;
        it.setup_disp(idx, y, face_ext(g, a, 0), face_ext(g, a, 1), face_ext(g, a, 2));
        it.c1();
        s = it.value(vp + g.foff[a]);
    }
    const T f3 = (v[e] - s) / dt - u[e] + (p[j * C + c] - p[j * C + cm]) * ih;
    out1[e] = (res1 ? res1[e] : (T)0) + sgn * f1;
    out3[e] = (res3 ? res3[e] : (T)0) + sgn * f3;
}

// Cell rows F2 = D v_j, F4 = D u_j of cell c, slice j.
template <typename T, int D>
__device__ inline void kkt_cell(const Grid& g, T sgn, const T* __restrict__ v, const T* __restrict__ u,
                                const T* res2, const T* res4, T* out2, T* out4, int c, int j) {
    const long F = g.nface;
    const int i = c % g.n[0], jj = (c / g.n[0]) % g.n[1], k = c / (g.n[0] * g.n[1]);
    const T* vj = v + j * F;
    const T* uj = u + j * F;
    T dv = 0, du = 0;
    for (int a = 0; a < D; ++a) {
        const int hi = face_index(g, a, i + (a == 0), jj + (a == 1), k + (a == 2));
        const int lo = face_index(g, a, i, jj, k);
        dv += vj[hi] - vj[lo];
        du += uj[hi] - uj[lo];
    }
    const T ih = (T)(1.0 / g.h);
    const long e = (long)j * g.ncell + c;
    out2[e] = (res2 ? res2[e] : (T)0) + sgn * dv * ih;
    out4[e] = (res4 ? res4[e] : (T)0) + sgn * du * ih;
}

// The split residual of one level: blocks [0, nbf N) face rows, then
// [.., + nbc N) cell rows, then the tiles of the velocity-advection transpose
// (slices 0..N-2, d axes), which add their J_S^T term into t1 (zero on entry)
// instead of F1, then blocks that clear t1z.  All parts read only the state,
// so they run side by side; a launch uses any subset of them (nbf, nbc,
// ntile, nbz zero for the parts it leaves out).  An SCGS sweep launches the
// transpose (with the clear of the next sweep's t1) once and then, per colour,
// the rows of that colour (`rows` set: the faces of its cells and the cells
// themselves, all that its pass reads); the pass reads F1 + t1.
struct KktSplit {
    int nbf, nbc, ntile, nbz;
    int direct;     // 1: the transpose part runs one thread per source (ntile = blocks per slice)
    int rows;       // 1: face and cell rows of the colour (par, cnt) only
    int par[3];     // coordinate parities of the colour's cells
    int cnt[3];     // cells of the colour along each axis
    int nfc;        // faces of the colour's cells (per slice), with rows set
    void* gq;       // tiled transpose: where the quarters for the other axes go (k_quarter_gather adds them)
    int vort;       // 1: face rows of the rotational operator (no transpose part)
};

// Face e (0 <= e < nfc) of the colour's cells: a-faces whose coordinates
// across a have the colour's parities, a-faces first, then b, then c.
__device__ inline int colour_face(const Grid& g, const KktSplit& ks, int e) {
    const int m0 = (g.n[0] + 1) * ks.cnt[1] * ks.cnt[2];
    if (e < m0) {
        const int i = e % (g.n[0] + 1), r = e / (g.n[0] + 1);
        return face_index(g, 0, i, 2 * (r % ks.cnt[1]) + ks.par[1], 2 * (r / ks.cnt[1]) + ks.par[2]);
    }
    e -= m0;
    const int m1 = ks.cnt[0] * (g.n[1] + 1) * ks.cnt[2];
    if (e < m1) {
        const int ii = e % ks.cnt[0], r = e / ks.cnt[0];
        return face_index(g, 1, 2 * ii + ks.par[0], r % (g.n[1] + 1), 2 * (r / (g.n[1] + 1)) + ks.par[2]);
    }
    e -= m1;
    const int ii = e % ks.cnt[0], r = e / ks.cnt[0];
    return face_index(g, 2, 2 * ii + ks.par[0], 2 * (r % ks.cnt[1]) + ks.par[1], r / ks.cnt[1]);
}

template <typename T, int D>
__global__ void __launch_bounds__(256) k_kkt_split(Grid g, int N, T dt, T kr, T cfl, T sgn, KktSplit ks,
                                                   const T* __restrict__ v, const T* __restrict__ pb,
                                                   const T* __restrict__ u, const T* __restrict__ p,
                                                   const T* __restrict__ w, const T* res1, const T* res2,
                                                   const T* res3, const T* res4, T* out1, T* out2, T* out3,
                                                   T* out4, T* t1, T* t1z) {
    long b = blockIdx.x;
    const long bf = (long)ks.nbf * N, bc = (long)ks.nbc * N;
    const long bt = (long)ks.ntile * (N - 1) * (ks.direct ? 1 : D);
    if (b < bf) {
        const int e = (int)(b % ks.nbf) * 256 + threadIdx.x;
        if (e >= (ks.rows ? ks.nfc : g.nface)) return;
        const int f = ks.rows ? colour_face(g, ks, e) : e;
        kkt_face<T, D>(g, N, dt, kr, cfl, sgn, v, pb, u, p, w, res1, res3, out1, out3, f, (int)(b / ks.nbf), ks.vort);
        return;
    }
    b -= bf;
    if (b < bc) {
        const int e = (int)(b % ks.nbc) * 256 + threadIdx.x;
        if (e >= (ks.rows ? ks.cnt[0] * ks.cnt[1] * ks.cnt[2] : g.ncell)) return;
        const int c = ks.rows ? cell_index(g, 2 * (e % ks.cnt[0]) + ks.par[0],
                                           2 * ((e / ks.cnt[0]) % ks.cnt[1]) + ks.par[1],
                                           2 * (e / (ks.cnt[0] * ks.cnt[1])) + ks.par[2])
                              : e;
        kkt_cell<T, D>(g, sgn, v, u, res2, res4, out2, out4, c, (int)(b / ks.nbc));
        return;
    }
    b -= bc;
    if (b < bt) {
        const int slice = (int)((b / ks.ntile) % (N - 1));
        if (ks.direct) {
            // one thread per (slice, face); y = u_{j+1} (the u slots shifted by one), scale -sgn/dt
            const int f = (int)(b % ks.ntile) * 256 + threadIdx.x;
            if (f < g.nface) {
                int a, i, j, k;
                face_decode(g, f, a, i, j, k);
                self_advect_T_source<T, D>(g, cfl, v + (long)slice * g.nface, u + (long)(slice + 1) * g.nface,
                                           -sgn / dt, t1 + (long)slice * g.nface, a, i, j, k);
            }
            return;
        }
        // tile, slice, axis; y = u_{j+1} (the u slots shifted by one), scale -sgn/dt
        const int tile = (int)(b % ks.ntile);
        const int a = (int)(b / ((long)ks.ntile * (N - 1)));
        self_advect_T_tile<T, D>(g, cfl, v, u + g.nface, -sgn / dt, t1, g.nface, tile, slice, a, (T*)ks.gq);
        return;
    }
    b -= bt;
    const long tot = (long)N * g.nface;
    for (long e = b * 256 + threadIdx.x; e < tot; e += (long)ks.nbz * 256) t1z[e] = (T)0;
}

// ---------------------------------------------------------------- SCGS
// Cells of one colour (parity bits of the coordinates) and their faces.
struct ColourSet {
    int p[3];
    int cnt[3];
    int total;
};

inline ColourSet colour_set(const Grid& g, int colour) {
    ColourSet s{};
    for (int a = 0; a < 3; ++a) {
        s.p[a] = (a < g.dim) ? ((colour >> a) & 1) : 0;
        s.cnt[a] = (a < g.dim) ? (g.n[a] - s.p[a] + 1) / 2 : 1;
    }
    s.total = s.cnt[0] * s.cnt[1] * s.cnt[2];
    return s;
}

// Local geometry of one cell: face indices, interior flags, 1/|g|, ghat.
template <int D>
struct CellFaces {
    int face[2 * D];
    bool inner[2 * D];
    int m;
};

template <int D>
__device__ inline void cell_faces(const Grid& g, int i, int j, int k, CellFaces<D>& cf) {
    const int idx[3] = {i, j, k};
    cf.m = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        cf.face[2 * a] = face_index(g, a, i, j, k);
        cf.face[2 * a + 1] = face_index(g, a, i + (a == 0), j + (a == 1), k + (a == 2));
        cf.inner[2 * a] = idx[a] >= 1;
        cf.inner[2 * a + 1] = idx[a] + 1 <= g.n[a] - 1;
        cf.m += cf.inner[2 * a] + cf.inner[2 * a + 1];
    }
}

__device__ inline void colour_cell(const ColourSet& cs, int q, int& i, int& j, int& k) {
    const int ci = q % cs.cnt[0];
    const int cj = (q / cs.cnt[0]) % cs.cnt[1];
    const int ck = q / (cs.cnt[0] * cs.cnt[1]);
    i = 2 * ci + cs.p[0];
    j = 2 * cj + cs.p[1];
    k = 2 * ck + cs.p[2];
}

// Face part of the local spacetime solve.  With ghat = g/|g| (g the
// divergence coefficients -1/h, +1/h of the cell's interior faces) and
// P = I - ghat ghat^T, the local system [T (x) I, -g; g^T, 0] (blocks in time
// order (u_0,p_1), (v_1,pbar_1), ..., (v_N,pbar_N)) splits into
//   P x_k = (T^-1 P r)_k          (one scalar tridiagonal solve per face)
//   ghat^T x_k = xi_k = s_k/|g|   (s = divergence-row residual)
// so dx_k = (T^-1 P r)_k + ghat xi_k.  T is shared by all cells: the host
// passes its Thomas factors (sub-diagonal, c', 1/pivot).
//
// Two kernels: k_scgs_project forms (P r)_k for every (cell, face, block) in
// parallel into scratch[k][cell*2d + face]; k_scgs_thomas runs the
// recurrence per (cell, face) in place on that column and applies omega dx
// (omega is the relaxation weight of the smoother).

template <typename T, int D>
__global__ void k_scgs_project(Grid g, int N, ColourSet cs, const T* __restrict__ r1, const T* __restrict__ r3,
                               T* __restrict__ scratch) {
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int ncol = cs.total * 2 * D;
    if (tid >= (long)ncol * 2 * N) return;
    const int kk = (int)(tid / ncol);
    const int col = (int)(tid % ncol);
    const int q = col / (2 * D), s = col % (2 * D);
    int i, j, k;
    colour_cell(cs, q, i, j, k);
    CellFaces<D> cf;
    cell_faces<D>(g, i, j, k, cf);
    if (!pick(cf.inner, s)) return;
    const T ginv = (T)1 / sqrt((T)cf.m);
    const long jo = (long)(kk >> 1) * g.nface;
    const T* r = (kk & 1) ? r1 + jo : r3 + jo;
    T gr = 0;
#pragma unroll
    for (int t = 0; t < 2 * D; ++t)
        if (cf.inner[t]) gr += ((t & 1) ? ginv : -ginv) * r[cf.face[t]];
    const T ghs = (s & 1) ? ginv : -ginv;
    scratch[tid] = r[pick(cf.face, s)] - ghs * gr;
}

// Recurrence of the face solve, one thread per (cell, face) column.  The
// Thomas factors are staged in LDS (dynamic, 3 * 2N values) so that the
// recurrence reads them with LDS latency; each chunk of U blocks issues its
// loads before the dependent arithmetic.
template <typename T, int D>
__global__ void k_scgs_thomas(Grid g, int N, ColourSet cs, const T* __restrict__ r2, const T* __restrict__ r4, T* v,
                              T* u, const T* __restrict__ tsub, const T* __restrict__ tcp,
                              const T* __restrict__ tinv, T omega, T* __restrict__ scratch) {
    extern __shared__ unsigned char smem_raw[];
    T* tc = reinterpret_cast<T*>(smem_raw);
    const int M = 2 * N;
    for (int e = threadIdx.x; e < M; e += blockDim.x) {
        tc[e] = tsub[e];
        tc[M + e] = tinv[e];
        tc[2 * M + e] = tcp[e];
    }
    __syncthreads();
    const T* sub = tc;
    const T* inv = tc + M;
    const T* cp = tc + 2 * M;
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int ncol = cs.total * 2 * D;
    if (col >= ncol) return;
    const int q = col / (2 * D), s = col % (2 * D);
    int i, j, k;
    colour_cell(cs, q, i, j, k);
    CellFaces<D> cf;
    cell_faces<D>(g, i, j, k, cf);
    if (!pick(cf.inner, s)) return;
    const T ginv = (T)1 / sqrt((T)cf.m);
    const T ghs = (s & 1) ? ginv : -ginv;
    const T gn_inv = (T)g.h * ginv;             // 1/|g| = h/sqrt(m)
    const long F = g.nface, C = g.ncell;
    const int c = cell_index(g, i, j, k);
    const int own = pick(cf.face, s);
    T* col_p = scratch + col;
    constexpr int U = 16;
    // forward elimination
    T dprev = 0;
    int k0 = 0;
    for (; k0 + U <= M; k0 += U) {
        T buf[U];
#pragma unroll
        for (int t = 0; t < U; ++t) buf[t] = col_p[(long)(k0 + t) * ncol];
#pragma unroll
        for (int t = 0; t < U; ++t) {
            dprev = (buf[t] - sub[k0 + t] * dprev) * inv[k0 + t];
            buf[t] = dprev;
        }
#pragma unroll
        for (int t = 0; t < U; ++t) col_p[(long)(k0 + t) * ncol] = buf[t];
    }
    for (; k0 < M; ++k0) {
        dprev = (col_p[(long)k0 * ncol] - sub[k0] * dprev) * inv[k0];
        col_p[(long)k0 * ncol] = dprev;
    }
    // back substitution and update (blocks M-1 down to 0)
    T x = 0;
    int k1 = M - 1;
    for (; k1 - (U - 1) >= 0; k1 -= U) {
        T buf[U], sk[U], fv[U];
#pragma unroll
        for (int t = 0; t < U; ++t) {
            const int kk = k1 - t;
            const long jj = kk >> 1;
            buf[t] = col_p[(long)kk * ncol];
            sk[t] = (kk & 1) ? r2[jj * C + c] : r4[jj * C + c];
            fv[t] = ((kk & 1) ? v : u)[jj * F + own];
        }
#pragma unroll
        for (int t = 0; t < U; ++t) {
            const int kk = k1 - t;
            x = buf[t] - cp[kk] * x;
            ((kk & 1) ? v : u)[(long)(kk >> 1) * F + own] = fv[t] + omega * (x + ghs * sk[t] * gn_inv);
        }
    }
    for (; k1 >= 0; --k1) {
        const long jj = k1 >> 1;
        x = col_p[(long)k1 * ncol] - cp[k1] * x;
        const T sk = (k1 & 1) ? r2[jj * C + c] : r4[jj * C + c];
        ((k1 & 1) ? v : u)[jj * F + own] += omega * (x + ghs * sk * gn_inv);
    }
}

// Whole colour in one kernel, time-parallel; the F1 rows arrive split as
// r1 + t1 (k_kkt_split).  One lane per (cell, chunk of
// L <= CH consecutive blocks, chunks starting at even blocks); the G lanes
// of a cell are adjacent.  The lane reads its cell's 2d face residuals once
// per block, forms ghat^T r and P r for every face, and runs the two Thomas
// passes of all 2d faces together (T is shared, so the running product of
// multipliers is too); chunk maps are joined across lanes by a log2(G)-step
// shuffle scan.  The same lane applies the pressure correction of its
// blocks, which needs only the divergence residual of the neighbouring
// blocks.  Every load is unconditional (blocks past the end read a clamped
// block of the same parity and are masked), so all of a lane's loads are in
// flight together.
// ROWS = false: the G lanes of a cell are adjacent in one wave (lane = chunk)
// and the chunk maps are joined with shuffles.  ROWS = true: a workgroup
// takes CPW consecutive cells of the colour and all G chunks, thread
// g * CPW + c holding chunk g of cell c, so that each load of a wave reads
// CPW neighbouring cells at one block (coalesced); the chunk maps are joined
// through LDS (sc: G x (1 + 2d) x CPW values).
template <typename T, int D, int G, int CH, bool ROWS, int CPW = 64>
__device__ inline void scgs_colour_body(const Grid& g, int N, int L, const ColourSet& cs, int q, int lane, T* sc,
                                        const T* __restrict__ r1, const T* __restrict__ t1,
                                        const T* __restrict__ r2, const T* __restrict__ r3,
                                        const T* __restrict__ r4, T* v, T* pb, T* u, T* p,
                                        const T* __restrict__ tdiag, const T* __restrict__ tsub,
                                        const T* __restrict__ tsup, const T* __restrict__ tcp,
                                        const T* __restrict__ tinv, T omega) {
    constexpr int NF = 2 * D;
    const int M = 2 * N;
    const bool active = q < cs.total;
    // lanes past the last cell work on the last cell and write nothing
    int i, j, k;
    colour_cell(cs, min(q, cs.total - 1), i, j, k);
    CellFaces<D> cf;
    cell_faces<D>(g, i, j, k, cf);
    const T ginv = (T)1 / sqrt((T)cf.m);
    const T gn_inv = (T)g.h * ginv;
    T gh[NF];
#pragma unroll
    for (int e = 0; e < NF; ++e) gh[e] = cf.inner[e] ? ((e & 1) ? ginv : -ginv) : (T)0;
    const long F = g.nface, C = g.ncell;
    const int c = cell_index(g, i, j, k);
    const int k0 = lane * L;
    const int len = active ? max(0, min(L, M - k0)) : 0;
    // ---- loads: face residuals, old unknowns, divergence residual of the
    // blocks k0-1 .. k0+CH, old pressures, temporal factors
    T rv[CH][NF], fo[CH][NF], po[CH], sk[CH + 2];
    T iv[CH], cm[CH], td[CH], ts[CH], tp[CH];
#pragma unroll
    for (int t = 0; t < CH; ++t) {
        const int kk = min(k0 + t, M - 2 + (t & 1));
        const long jf = (long)(kk >> 1) * F;
        const T* x = (t & 1) ? v : u;
#pragma unroll
        for (int e = 0; e < NF; ++e) {
            // F1 rows (v-blocks) are split into r1 and the J_S^T term t1
            rv[t][e] = (t & 1) ? r1[jf + cf.face[e]] + t1[jf + cf.face[e]] : r3[jf + cf.face[e]];
            fo[t][e] = x[jf + cf.face[e]];
        }
        po[t] = ((t & 1) ? pb : p)[(long)(kk >> 1) * C + c];
        iv[t] = tinv[kk];
        cm[t] = tcp[kk];
        td[t] = tdiag[kk];
        ts[t] = tsub[kk];
        tp[t] = tsup[kk];
    }
#pragma unroll
    for (int t = -1; t <= CH; ++t) {
        // block k0+t, clamped into range with its parity kept (odd t: v-block)
        const int kk = (t & 1) ? min(max(k0 + t, 1), M - 1) : min(k0 + t, M - 2);
        sk[t + 1] = ((t & 1) ? r2 : r4)[(long)(kk >> 1) * C + c];
    }
    // ---- projection: gr_t = ghat^T r_t, P r_t = r_t - ghat gr_t
    T gr[CH];
#pragma unroll
    for (int t = 0; t < CH; ++t) {
        T acc = 0;
#pragma unroll
        for (int e = 0; e < NF; ++e) acc += gh[e] * rv[t][e];
        gr[t] = acc;
#pragma unroll
        for (int e = 0; e < NF; ++e) rv[t][e] -= gh[e] * acc;
    }
    // ---- forward elimination, chunk-local from a zero carry
    T pv[CH], val[NF], prod = 1;
#pragma unroll
    for (int e = 0; e < NF; ++e) val[e] = 0;
#pragma unroll
    for (int t = 0; t < CH; ++t) {
        const bool on = t < len;
        const T a = -ts[t] * iv[t];
#pragma unroll
        for (int e = 0; e < NF; ++e) {
            val[e] = on ? a * val[e] + rv[t][e] * iv[t] : val[e];
            rv[t][e] = val[e];
        }
        prod = on ? a * prod : prod;
        pv[t] = prod;
    }
    if constexpr (ROWS) {
        // chunk maps to LDS, then each chunk folds the maps of the chunks before it
        const int l = threadIdx.x & (CPW - 1);
        sc[(lane * (1 + NF)) * CPW + l] = prod;
#pragma unroll
        for (int e = 0; e < NF; ++e) sc[(lane * (1 + NF) + 1 + e) * CPW + l] = val[e];
        __syncthreads();
        T cin[NF];
#pragma unroll
        for (int e = 0; e < NF; ++e) cin[e] = 0;
        for (int h = 0; h < lane; ++h) {
            const T Ah = sc[(h * (1 + NF)) * CPW + l];
#pragma unroll
            for (int e = 0; e < NF; ++e) cin[e] = Ah * cin[e] + sc[(h * (1 + NF) + 1 + e) * CPW + l];
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < NF; ++e)
#pragma unroll
            for (int t = 0; t < CH; ++t) rv[t][e] += pv[t] * cin[e];
    } else {
        T A = prod;
#pragma unroll
        for (int off = 1; off < G; off <<= 1) {
            const T Ap = __shfl_up(A, off, G);
            T Bp[NF];
#pragma unroll
            for (int e = 0; e < NF; ++e) Bp[e] = __shfl_up(val[e], off, G);
            if (lane >= off) {
#pragma unroll
                for (int e = 0; e < NF; ++e) val[e] = A * Bp[e] + val[e];
                A = A * Ap;
            }
        }
#pragma unroll
        for (int e = 0; e < NF; ++e) {
            T cin = __shfl_up(val[e], 1, G);
            cin = lane == 0 ? (T)0 : cin;
#pragma unroll
            for (int t = 0; t < CH; ++t) rv[t][e] += pv[t] * cin;
        }
    }
    // ---- back substitution, chunk-local from a zero carry
    prod = 1;
#pragma unroll
    for (int e = 0; e < NF; ++e) val[e] = 0;
#pragma unroll
    for (int t = CH - 1; t >= 0; --t) {
        const bool on = t < len;
        const T cc = -cm[t];
#pragma unroll
        for (int e = 0; e < NF; ++e) {
            val[e] = on ? cc * val[e] + rv[t][e] : val[e];
            rv[t][e] = val[e];
        }
        prod = on ? cc * prod : prod;
        pv[t] = prod;
    }
    if constexpr (ROWS) {
        // each chunk folds the maps of the chunks after it, last first
        const int l = threadIdx.x & (CPW - 1);
        sc[(lane * (1 + NF)) * CPW + l] = prod;
#pragma unroll
        for (int e = 0; e < NF; ++e) sc[(lane * (1 + NF) + 1 + e) * CPW + l] = val[e];
        __syncthreads();
        T cin[NF];
#pragma unroll
        for (int e = 0; e < NF; ++e) cin[e] = 0;
        for (int h = G - 1; h > lane; --h) {
            const T Ah = sc[(h * (1 + NF)) * CPW + l];
#pragma unroll
            for (int e = 0; e < NF; ++e) cin[e] = Ah * cin[e] + sc[(h * (1 + NF) + 1 + e) * CPW + l];
        }
#pragma unroll
        for (int e = 0; e < NF; ++e)
#pragma unroll
            for (int t = 0; t < CH; ++t) rv[t][e] += pv[t] * cin[e];
    } else {
        T A = prod;
#pragma unroll
        for (int off = 1; off < G; off <<= 1) {
            const T An = __shfl_down(A, off, G);
            T Bn[NF];
#pragma unroll
            for (int e = 0; e < NF; ++e) Bn[e] = __shfl_down(val[e], off, G);
            if (lane + off < G) {
#pragma unroll
                for (int e = 0; e < NF; ++e) val[e] = A * Bn[e] + val[e];
                A = A * An;
            }
        }
#pragma unroll
        for (int e = 0; e < NF; ++e) {
            T cin = __shfl_down(val[e], 1, G);
            cin = lane == G - 1 ? (T)0 : cin;
#pragma unroll
            for (int t = 0; t < CH; ++t) rv[t][e] += pv[t] * cin;
        }
    }
    // ---- apply the corrections of this chunk (relaxed by omega)
#pragma unroll
    for (int t = 0; t < CH; ++t) {
        if (t < len) {
            const int kk = k0 + t;
            const long jj = kk >> 1;
            T* x = (t & 1) ? v : u;
#pragma unroll
            for (int e = 0; e < NF; ++e)
                if (cf.inner[e]) x[jj * F + cf.face[e]] = fo[t][e] + omega * (rv[t][e] + gh[e] * sk[t + 1] * gn_inv);
            T acc = td[t] * sk[t + 1];
            if (kk > 0) acc += ts[t] * sk[t];
            if (kk < M - 1) acc += tp[t] * sk[t + 2];
            ((t & 1) ? pb : p)[jj * C + c] = po[t] + omega * (acc * gn_inv - gr[t]) * gn_inv;
        }
    }
}

template <typename T, int D, int G, int CH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2)))
k_scgs_colour(Grid g, int N, int L, ColourSet cs, const T* __restrict__ r1, const T* __restrict__ t1,
              const T* __restrict__ r2, const T* __restrict__ r3, const T* __restrict__ r4, T* v, T* pb, T* u, T* p,
              const T* __restrict__ tdiag, const T* __restrict__ tsub, const T* __restrict__ tsup,
              const T* __restrict__ tcp, const T* __restrict__ tinv, T omega) {
    scgs_colour_body<T, D, G, CH, false>(g, N, L, cs, (int)((blockIdx.x * blockDim.x + threadIdx.x) / G),
                                         (int)(threadIdx.x % G), nullptr, r1, t1, r2, r3, r4, v, pb, u, p, tdiag,
                                         tsub, tsup, tcp, tinv, omega);
}

template <typename T, int D, int G, int CH, int CPW>
__global__ void __launch_bounds__(CPW * G) k_scgs_colour_rows(Grid g, int N, int L, ColourSet cs,
                                                             const T* __restrict__ r1, const T* __restrict__ t1,
                                                             const T* __restrict__ r2, const T* __restrict__ r3,
                                                             const T* __restrict__ r4, T* v, T* pb, T* u, T* p,
                                                             const T* __restrict__ tdiag,
                                                             const T* __restrict__ tsub,
                                                             const T* __restrict__ tsup,
                                                             const T* __restrict__ tcp,
                                                             const T* __restrict__ tinv, T omega) {
    __shared__ T sc[G * (1 + 2 * D) * CPW];
    scgs_colour_body<T, D, G, CH, true, CPW>(g, N, L, cs, (int)(blockIdx.x * CPW + (threadIdx.x & (CPW - 1))),
                                             (int)(threadIdx.x / CPW), sc, r1, t1, r2, r3, r4, v, pb, u, p, tdiag,
                                             tsub, tsup, tcp, tinv, omega);
}

// Pressure part: dpi_k = (sum_l T_kl xi_l - ghat^T r_k) / |g|, one thread per
// (cell, block).
template <typename T, int D>
__global__ void k_scgs_cells(Grid g, int N, ColourSet cs, const T* __restrict__ r1, const T* __restrict__ r2,
                             const T* __restrict__ r3, const T* __restrict__ r4, T* pb, T* p,
                             const T* __restrict__ tdiag, const T* __restrict__ tsub, const T* __restrict__ tsup,
                             T omega) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= cs.total * 2 * N) return;
    const int q = tid % cs.total, kk = tid / cs.total;
    int i, j, k;
    colour_cell(cs, q, i, j, k);
    CellFaces<D> cf;
    cell_faces<D>(g, i, j, k, cf);
    const T ginv = (T)1 / sqrt((T)cf.m);
    const T gn_inv = (T)g.h * ginv;
    const long F = g.nface, C = g.ncell;
    const int c = cell_index(g, i, j, k);
    auto srow = [&](int b) -> T {
        const long jj = b >> 1;
        return ((b & 1) ? r2[jj * C + c] : r4[jj * C + c]) * gn_inv;
    };
    T acc = tdiag[kk] * srow(kk);
    if (kk > 0) acc += tsub[kk] * srow(kk - 1);
    if (kk < 2 * N - 1) acc += tsup[kk] * srow(kk + 1);
    const long jo = (long)(kk >> 1) * F;
    const T* r = (kk & 1) ? r1 + jo : r3 + jo;
    T gr = 0;
    for (int t = 0; t < 2 * D; ++t)
        if (cf.inner[t]) gr += ((t & 1) ? ginv : -ginv) * r[cf.face[t]];
    T* fld = (kk & 1) ? pb : p;
    fld[(long)(kk >> 1) * C + c] += omega * (acc - gr) * gn_inv;
}

// ---------------------------------------------------------------- transfers
// Interpolation weight of coarse node I for a fine sample at coarse
// position y on an axis with M coarse nodes.
template <typename T>
__device__ inline T axis_weight(T y, int M, int I) {
    const Axis<T> s = locate<T>(y, M);
    if (I == s.i0) return (T)1 - s.t;
    if (I == s.i0 + 1) return s.t;
    return (T)0;
}

// Coarse position of fine index j: cell-type axis (j + 1/2)/2 - 1/2, node-type j/2.
template <typename T>
__device__ inline T fine_pos(int j, bool node) {
    return node ? (T)j * (T)0.5 : ((T)j + (T)0.5) * (T)0.5 - (T)0.5;
}

// coarse = 2^-d P^T fine on the cell lattice (gather form), coarse cell c.
template <typename T, int D>
__device__ inline void restrict_cell_at(const Grid& gf, const Grid& gc, const T* __restrict__ fine,
                                        T* __restrict__ coarse, int c) {
    const int I[3] = {c % gc.n[0], (c / gc.n[0]) % gc.n[1], c / (gc.n[0] * gc.n[1])};
    T s = 0;
    const int lo2 = D == 3 ? 2 * I[2] - 1 : 0, hi2 = D == 3 ? 2 * I[2] + 2 : 0;
    for (int k = lo2; k <= hi2; ++k) {
        if (k < 0 || k >= gf.n[2]) continue;
        const T wk = D == 3 ? axis_weight<T>(fine_pos<T>(k, false), gc.n[2], I[2]) : (T)1;
        if (wk == (T)0) continue;
        for (int j = 2 * I[1] - 1; j <= 2 * I[1] + 2; ++j) {
            if (j < 0 || j >= gf.n[1]) continue;
            const T wj = axis_weight<T>(fine_pos<T>(j, false), gc.n[1], I[1]);
            if (wj == (T)0) continue;
            for (int i = 2 * I[0] - 1; i <= 2 * I[0] + 2; ++i) {
                if (i < 0 || i >= gf.n[0]) continue;
                const T wi = axis_weight<T>(fine_pos<T>(i, false), gc.n[0], I[0]);
                s += wi * wj * wk * fine[cell_index(gf, i, j, k)];
            }
        }
    }
    coarse[c] = s * (T)(D == 3 ? 0.125 : 0.25);
}

// Face lattices, coarse face f; coarse wall faces are set to zero.
template <typename T, int D>
__device__ inline void restrict_face_at(const Grid& gf, const Grid& gc, const T* __restrict__ fine,
                                        T* __restrict__ coarse, int f) {
    int a, I0, I1, I2;
    face_decode(gc, f, a, I0, I1, I2);
    if (!face_interior(gc, a, I0, I1, I2)) {
        coarse[f] = (T)0;
        return;
    }
    const int I[3] = {I0, I1, I2};
    // the 1D weights of each axis once (3 along a, 4 across; 0 outside the
    // fine lattice), then the tensor-product sum in k, j, i order
    int lo[3];
    T wt[3][4];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        lo[b] = b < D ? 2 * I[b] - 1 : 0;
        const int cnt = b >= D ? 1 : (b == a ? 3 : 4);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int x = lo[b] + t;
            wt[b][t] = (T)0;
            if (t >= cnt) continue;
            if (b >= D) {
                wt[b][t] = (T)1;
                continue;
            }
            if (x < 0 || x >= face_ext(gf, a, b)) continue;
            wt[b][t] = axis_weight<T>(fine_pos<T>(x, a == b), face_ext(gc, a, b), I[b]);
        }
    }
    T s = 0;
#pragma unroll
    for (int tk = 0; tk < 4; ++tk) {
        const T wk = wt[2][tk];
        if (wk == (T)0) continue;
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) {
            const T wj = wt[1][tj];
            if (wj == (T)0) continue;
#pragma unroll
            for (int ti = 0; ti < 4; ++ti) {
                const T wi = wt[0][ti];
                if (wi == (T)0) continue;
                s += wi * wj * wk * fine[face_index(gf, a, lo[0] + ti, lo[1] + tj, lo[2] + tk)];
            }
        }
    }
    coarse[f] = s * (T)(D == 3 ? 0.125 : 0.25);
}

// fine += sign * P coarse on the cell lattice, fine cell c.
template <typename T, int D>
__device__ inline void prolong_cell_at(const Grid& gf, const Grid& gc, const T* __restrict__ coarse, T sign,
                                       T* __restrict__ fine, int c) {
    const int idx[3] = {c % gf.n[0], (c / gf.n[0]) % gf.n[1], c / (gf.n[0] * gf.n[1])};
    T y[3];
    for (int b = 0; b < D; ++b) y[b] = fine_pos<T>(idx[b], false);
    Interp<T, D> it;
    it.setup(y, gc.n[0], gc.n[1], gc.n[2]);
    fine[c] += sign * it.value(coarse);
}

// fine += sign * P coarse on the face lattices (fine walls untouched), fine face f.
template <typename T, int D>
__device__ inline void prolong_face_at(const Grid& gf, const Grid& gc, const T* __restrict__ coarse, T sign,
                                       T* __restrict__ fine, int f) {
    int a, i, j, k;
    face_decode(gf, f, a, i, j, k);
    if (!face_interior(gf, a, i, j, k)) return;
    const int idx[3] = {i, j, k};
    T y[3];
    for (int b = 0; b < D; ++b) y[b] = fine_pos<T>(idx[b], b == a);
    Interp<T, D> it;
    it.setup(y, face_ext(gc, a, 0), face_ext(gc, a, 1), face_ext(gc, a, 2));
    fine[f] += sign * it.value(coarse + gc.foff[a]);
}

template <typename T, int D>
__global__ void k_restrict_cells(Grid gf, Grid gc, const T* __restrict__ fine, T* __restrict__ coarse) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= gc.ncell) return;
    restrict_cell_at<T, D>(gf, gc, fine + (long)blockIdx.y * gf.ncell, coarse + (long)blockIdx.y * gc.ncell, c);
}
template <typename T, int D>
__global__ void k_restrict_faces(Grid gf, Grid gc, const T* __restrict__ fine, T* __restrict__ coarse) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= gc.nface) return;
    restrict_face_at<T, D>(gf, gc, fine + (long)blockIdx.y * gf.nface, coarse + (long)blockIdx.y * gc.nface, f);
}
template <typename T, int D>
__global__ void k_prolong_cells(Grid gf, Grid gc, const T* __restrict__ coarse, T sign, T* __restrict__ fine) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= gf.ncell) return;
    prolong_cell_at<T, D>(gf, gc, coarse + (long)blockIdx.y * gc.ncell, sign, fine + (long)blockIdx.y * gf.ncell, c);
}
template <typename T, int D>
__global__ void k_prolong_faces(Grid gf, Grid gc, const T* __restrict__ coarse, T sign, T* __restrict__ fine) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= gf.nface) return;
    prolong_face_at<T, D>(gf, gc, coarse + (long)blockIdx.y * gc.nface, sign, fine + (long)blockIdx.y * gf.nface, f);
}

// Several transfers in one launch (blockIdx.z picks the array): the first
// nf entries are face sequences, the rest cell sequences; blockIdx.y is the
// time slot.  Restriction: dst (coarse) = R src (fine).  Prolongation:
// dst (fine) += sign P src (coarse).
template <typename T>
struct XferSet {
    const T* src[8];
    T* dst[8];
};

template <typename T, int D>
__global__ void k_restrict_set(Grid gf, Grid gc, XferSet<T> x, int nf) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int z = blockIdx.z;
    const long s = blockIdx.y;
    if (z < nf) {
        if (e < gc.nface) restrict_face_at<T, D>(gf, gc, x.src[z] + s * gf.nface, x.dst[z] + s * gc.nface, e);
    } else {
        if (e < gc.ncell) restrict_cell_at<T, D>(gf, gc, x.src[z] + s * gf.ncell, x.dst[z] + s * gc.ncell, e);
    }
}

template <typename T, int D>
__global__ void k_prolong_set(Grid gf, Grid gc, XferSet<T> x, int nf, T sign) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int z = blockIdx.z;
    const long s = blockIdx.y;
    if (z < nf) {
        if (e < gf.nface) prolong_face_at<T, D>(gf, gc, x.src[z] + s * gc.nface, sign, x.dst[z] + s * gf.nface, e);
    } else {
        if (e < gf.ncell) prolong_cell_at<T, D>(gf, gc, x.src[z] + s * gc.ncell, sign, x.dst[z] + s * gf.ncell, e);
    }
}

}  // namespace stfas
