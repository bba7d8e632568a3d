// SCGS local solve of the rotational operator (2D): the cell's spacetime
// system of Sec. 4.3 eq:HESS with the cell's block of dAdv/dv in it.
//
// Unknowns of one cell, for every slot s = 0..N-1 (v[s] = v_{s+1},
// u[s] = u_s, p[s] = p_{s+1}, pbar[s] = pbar_{s+1}): the corrections of v and
// u at the cell's four faces and of p, pbar at its centre.  Face slots: 0 low
// x-face (i, j), 1 high x-face (i+1, j), 2 low y-face (i, j), 3 high y-face
// (i, j+1); wall faces are not unknowns.  With g the divergence coefficients
// of the cell's interior faces (-1/h low, +1/h high), M the interior mask,
// B_s = I/dt + dAdv/dv at v_{s+1} (rows and columns of the cell's interior
// faces) and kappa_s = K/r [s < N-1] + the smoother's perturbation, the
// rows are (a, b, c, e: the residual of F3_s, F4_s, F1_{s+1}, F2_{s+1})
//   F3_s:  -du_s - dv_{s-1}/dt + B_s dv_s - g dp_s            = a_s   (dv_{-1} = 0)
//   F4_s:   g^T du_s                                          = b_s
//   F1:     B_s^T du_s + kappa_s dv_s - [s<N-1] du_{s+1}/dt - g dpbar_s = c_s
//   F2:     g^T dv_s                                          = e_s
// The u rows give du_s = -P q_s + g b_s/|g|^2 and dp_s = -(b_s + g^T q_s)/|g|^2
// with q_s = a_s + dv_{s-1}/dt - B_s dv_s and P = M - g g^T/|g|^2.  Put into
// the v rows, and with dv_s = Z y_s + g e_s/|g|^2 (Z an orthonormal basis of
// the interior faces' divergence-free directions, at most 3 of them), the
// corrections y form a block tridiagonal system with 3x3 blocks
//   D_s = beta_s^T beta_s + kappa_s + [s<N-1]/dt^2,   beta_s = Z^T B_s Z,
//   coupling of y_{s-1} (row) and y_s (column): -beta_s/dt,
// which is symmetric positive definite (the Schur complement of the u
// blocks, which are -I), so block elimination needs no pivoting.  The
// eliminated quantities follow from y: du, dp from the u rows, and
//   dpbar_s = (kappa_s e_s + g^T B_s^T du_s - [s<N-1] b_{s+1}/dt - g^T c_s)/|g|^2
// (g^T du_{s+1} = b_{s+1}).  Every correction is relaxed by omega.
//
// Three launches per colour: k_rot_blk_setup forms beta_s, D_s and the
// reduced right-hand side for every (cell, slot) in parallel;
// k_rot_blk_thomas runs the elimination in time, one thread per cell;
// k_rot_blk_apply forms and adds the corrections, again per (cell, slot).
// Cells of one colour share no face and no face of one is read by another's
// block (their faces share no node), so the launches need no atomics.
#pragma once
#include "common.hpp"
#include "k_kkt.hpp"
#include "k_rot.hpp"

namespace stfas {

// Scratch per (cell of the colour, slot), one record of ROT_BLK_WORDS words
// (21 used, padded to a multiple of 16 bytes so the elimination reads it
// with 16-byte loads): [0, 9) F_s = -beta_s/dt (row-major), the coupling of
// y_{s-1} and y_s, [9, 18) D_s, [18, 21) the reduced right-hand side, which
// the elimination replaces by y_s.
constexpr int ROT_BLK_WORDS = 24;

// The cell's block of dAdv/dv at v (rows: Adv at the face slots, columns: v
// at the face slots).  With the node quantities of k_rot.hpp, for an x-face
// Adv = -1/4 sum over its end nodes n of w_n Sy_n and for a y-face
// +1/4 sum of w_n Sx_n, so the derivative by v at slot s is the sum over the
// end nodes of dw_n/dv_s Sy_n + w_n dSy_n/dv_s (Sx_n for y-faces).  The end
// nodes of the cell's faces are its corners c = 0 (i, j), 1 (i+1, j),
// 2 (i, j+1), 3 (i+1, j+1); at corner c, w_n takes the slots
//   c0: +y_low -x_low   c1: -y_low -x_high   c2: +y_high +x_low   c3: -y_high +x_high
// (times 1/h, interior nodes only), Sx_n the x-slot and Sy_n the y-slot
// meeting there.
template <typename T>
__device__ inline void rot_cell_jacobian(const Grid& g, const T* v, int i, int j, T ih, T (&J)[4][4]) {
    constexpr int ci[4] = {0, 1, 0, 1}, cj[4] = {0, 0, 1, 1};
    constexpr T wc[4][4] = {{-1, 0, 1, 0}, {0, -1, -1, 0}, {1, 0, 0, 1}, {0, 1, 0, -1}};
    constexpr int xs[4] = {0, 1, 0, 1};      // x-slot meeting at corner c
    constexpr int ys[4] = {2, 2, 3, 3};      // y-slot meeting at corner c
    constexpr int ends[4][2] = {{0, 2}, {1, 3}, {0, 1}, {2, 3}};
    T w[4], sx[4], sy[4], in[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int I = i + ci[c], Jn = j + cj[c];
        rot_sums(g, v, I, Jn, false, sx[c], sy[c]);
        w[c] = rot_vorticity(g, v, I, Jn, ih);
        in[c] = (I > 0 && I < g.n[0] && Jn > 0 && Jn < g.n[1]) ? ih : (T)0;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const bool xface = t < 2;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            T acc = 0;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int c = ends[t][e];
                const T sum = xface ? sy[c] : sx[c];
                const bool hit = xface ? (ys[c] == s) : (xs[c] == s);
                acc += wc[c][s] * in[c] * sum + (hit ? w[c] : (T)0);
            }
            J[t][s] = xface ? (T)-0.25 * acc : (T)0.25 * acc;
        }
    }
}

// Geometry of one cell's local system: g, |g|^2, the interior mask and Z.
template <typename T>
struct RotCell {
    int face[4];
    int cell;
    T m[4], gv[4], gg;
    T Z[4][3];
    T act[3];      // 1 for the columns of Z in use

    __device__ void init(const Grid& g, int i, int j) {
        CellFaces<2> cf;
        cell_faces<2>(g, i, j, 0, cf);
        cell = cell_index(g, i, j, 0);
        const T ih = (T)(1.0 / g.h);
        gg = 0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            face[s] = cf.face[s];
            m[s] = cf.inner[s] ? (T)1 : (T)0;
            gv[s] = (s & 1 ? ih : -ih) * m[s];
            gg += gv[s] * gv[s];
        }
        // Gram-Schmidt on the projections of the interior unit vectors; a
        // candidate is dependent when almost nothing is left of it (for the
        // masks a cell can have, a kept vector keeps at least half of its
        // squared length, a dropped one none)
        int nk = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            act[k] = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) Z[r][k] = 0;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            T z[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) z[r] = (r == s ? m[s] : (T)0) - gv[r] * gv[s] / gg;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                T d = 0;
#pragma unroll
                for (int r = 0; r < 4; ++r) d += Z[r][k] * z[r];
#pragma unroll
                for (int r = 0; r < 4; ++r) z[r] -= d * Z[r][k];
            }
            T n2 = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) n2 += z[r] * z[r];
            if (m[s] > 0 && n2 > (T)0.1 && nk < 3) {
                const T inv = (T)1 / sqrt(n2);
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    if (k == nk) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) Z[r][k] = z[r] * inv;
                        act[k] = 1;
                    }
                ++nk;
            }
        }
    }
    // P x = M x - g (g^T x)/|g|^2
    __device__ void proj(const T (&x)[4], T (&o)[4]) const {
        T d = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) d += gv[r] * x[r];
        d /= gg;
#pragma unroll
        for (int r = 0; r < 4; ++r) o[r] = m[r] * x[r] - gv[r] * d;
    }
    __device__ T gdot(const T (&x)[4]) const {
        T d = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) d += gv[r] * x[r];
        return d;
    }
    // Z^T x and Z y
    __device__ void zt(const T (&x)[4], T (&o)[3]) const {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            o[k] = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) o[k] += Z[r][k] * x[r];
        }
    }
    __device__ void zy(const T (&y)[3], T (&o)[4]) const {
#pragma unroll
        for (int r = 0; r < 4; ++r) o[r] = Z[r][0] * y[0] + Z[r][1] * y[1] + Z[r][2] * y[2];
    }
};

// B_s = I/dt + dAdv/dv at the face slots of the cell, rows and columns of wall faces zero.
template <typename T>
__device__ inline void rot_cell_B(const Grid& g, const RotCell<T>& rc, const T* v, int i, int j, T dt,
                                  T (&B)[4][4]) {
    rot_cell_jacobian<T>(g, v, i, j, (T)(1.0 / g.h), B);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s) B[t][s] = (B[t][s] + (t == s ? (T)1 / dt : (T)0)) * rc.m[t] * rc.m[s];
}

template <typename T>
__device__ inline void mat4_vec(const T (&B)[4][4], const T (&x)[4], T (&o)[4]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) o[t] = B[t][0] * x[0] + B[t][1] * x[1] + B[t][2] * x[2] + B[t][3] * x[3];
}
template <typename T>
__device__ inline void mat4t_vec(const T (&B)[4][4], const T (&x)[4], T (&o)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) o[s] = B[0][s] * x[0] + B[1][s] * x[1] + B[2][s] * x[2] + B[3][s] * x[3];
}

// Right-hand side quantities of slot s: ahat_s = P a_s - g b_s/|g|^2 and vbar_s = g e_s/|g|^2.
template <typename T>
__device__ inline void rot_slot_rhs(const Grid& g, const RotCell<T>& rc, const T* r2, const T* r3, const T* r4,
                                    int s, T (&ahat)[4], T (&vbar)[4]) {
    T a[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = rc.m[r] > 0 ? r3[(long)s * g.nface + rc.face[r]] : (T)0;
    rc.proj(a, ahat);
    const T b = r4[(long)s * g.ncell + rc.cell] / rc.gg, e = r2[(long)s * g.ncell + rc.cell] / rc.gg;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        ahat[r] -= rc.gv[r] * b;
        vbar[r] = rc.gv[r] * e;
    }
}

template <typename P>
__device__ inline P* rot_sc(P* sc, int w, int s, int total, int q, int N) {
    (void)N;
    return sc + ((long)s * total + q) * ROT_BLK_WORDS + w;
}

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    using type = float4;
};
template <>
struct Vec16<double> {
    using type = double2;
};

// The record of (colour cell q, slot s): beta_s, D_s and the reduced right-hand side.
template <typename T>
__device__ inline void rot_setup_item(const Grid& g, int N, const ColourSet& cs, int q, int s, T dt, T kr, T lm,
                                      const T* __restrict__ v, const T* __restrict__ r1, const T* __restrict__ r2,
                                      const T* __restrict__ r3, const T* __restrict__ r4, T* rec) {
    int i, j, k;
    colour_cell(cs, q, i, j, k);
    RotCell<T> rc;
    rc.init(g, i, j);
    T B[4][4];
    rot_cell_B<T>(g, rc, v + (long)s * g.nface, i, j, dt, B);
    // beta_s = Z^T B_s Z
    T BZ[4][3], beta[3][3];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int k2 = 0; k2 < 3; ++k2) BZ[t][k2] = B[t][0] * rc.Z[0][k2] + B[t][1] * rc.Z[1][k2] +
                                                   B[t][2] * rc.Z[2][k2] + B[t][3] * rc.Z[3][k2];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) beta[a][b] = rc.Z[0][a] * BZ[0][b] + rc.Z[1][a] * BZ[1][b] +
                                                rc.Z[2][a] * BZ[2][b] + rc.Z[3][a] * BZ[3][b];
    const bool last = s == N - 1;
    const T kap = (last ? (T)0 : kr) + lm + (last ? (T)0 : (T)1 / (dt * dt));
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            T d = beta[0][a] * beta[0][b] + beta[1][a] * beta[1][b] + beta[2][a] * beta[2][b];
            if (a == b) d += rc.act[a] > 0 ? kap : (T)1;
            rec[a * 3 + b] = -beta[a][b] / dt;
            rec[9 + a * 3 + b] = d;
        }
    // w4 = c_s + B_s^T ahat_s - B_s^T P B_s vbar_s  [- ahat_{s+1}/dt + P B_{s+1} vbar_{s+1}/dt]
    T ahat[4], vbar[4], w4[4], t4[4], p4[4];
    rot_slot_rhs(g, rc, r2, r3, r4, s, ahat, vbar);
    mat4_vec(B, vbar, t4);
    rc.proj(t4, p4);
#pragma unroll
    for (int r = 0; r < 4; ++r) p4[r] = ahat[r] - p4[r];
    mat4t_vec(B, p4, w4);
#pragma unroll
    for (int r = 0; r < 4; ++r) w4[r] += rc.m[r] > 0 ? r1[(long)s * g.nface + rc.face[r]] : (T)0;
    if (!last) {
        T B1[4][4];
        rot_cell_B<T>(g, rc, v + (long)(s + 1) * g.nface, i, j, dt, B1);
        rot_slot_rhs(g, rc, r2, r3, r4, s + 1, ahat, vbar);
        mat4_vec(B1, vbar, t4);
        rc.proj(t4, p4);
#pragma unroll
        for (int r = 0; r < 4; ++r) w4[r] += (p4[r] - ahat[r]) / dt;
    }
    T rr[3];
    rc.zt(w4, rr);
#pragma unroll
    for (int a = 0; a < 3; ++a) rec[18 + a] = rr[a];
}


template <typename T>
__global__ void __launch_bounds__(256) k_rot_blk_setup(Grid g, int N, ColourSet cs, T dt, T kr, T lm, const T* __restrict__ v,
                                const T* __restrict__ r1, const T* __restrict__ r2, const T* __restrict__ r3,
                                const T* __restrict__ r4, T* __restrict__ sc) {
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (long)cs.total * N) return;
    const int q = (int)(tid % cs.total), s = (int)(tid / cs.total);
    rot_setup_item(g, N, cs, q, s, dt, kr, lm, v, r1, r2, r3, r4, rot_sc(sc, 0, s, cs.total, q, N));
}

__device__ inline float rot_rsq(float x) { return __builtin_amdgcn_rsqf(x); }   // x >= 1/dt^2 here
__device__ inline double rot_rsq(double x) { return 1.0 / sqrt(x); }

// Cholesky factor of a symmetric positive definite 3x3 matrix S = L L^T:
// the three off-diagonal entries and the reciprocals of the diagonal.
template <typename T>
struct Chol3 {
    T i0, i1, i2, l10, l20, l21;
    __device__ void factor(const T (&S)[3][3]) {
        i0 = rot_rsq(S[0][0]);
        l10 = S[1][0] * i0;
        l20 = S[2][0] * i0;
        i1 = rot_rsq(S[1][1] - l10 * l10);
        l21 = (S[2][1] - l20 * l10) * i1;
        i2 = rot_rsq(S[2][2] - l20 * l20 - l21 * l21);
    }
    __device__ void lower(const T (&f)[3], T (&o)[3]) const {     // L o = f
        o[0] = f[0] * i0;
        o[1] = (f[1] - l10 * o[0]) * i1;
        o[2] = (f[2] - l20 * o[0] - l21 * o[1]) * i2;
    }
    __device__ void upper(const T (&f)[3], T (&o)[3]) const {     // L^T o = f
        o[2] = f[2] * i2;
        o[1] = (f[1] - l21 * o[2]) * i1;
        o[0] = (f[0] - l10 * o[1] - l20 * o[2]) * i0;
    }
};

// Words of LDS per (thread, slot) in the elimination: W_s (9) and t_s (3).
constexpr int ROT_BLK_LDS = 12;

// Elimination in time, one thread per cell of the colour.  Step s factors
// the running Schur complement S = L L^T, forms G = L^-1 F and L^-1 z for the
// coupling F = -beta_s/dt, updates S <- D_s - G^T G and z <- rhs_s - G^T L^-1 z,
// and keeps W = S^-1 F, t = S^-1 z for the back substitution
// y_s = t_s - W_s y_{s+1} in LDS (blockDim.x threads x N slots x 12 words);
// the next steps' blocks are loaded RB steps ahead of their use (they do not
// depend on the recurrence), and no global store sits between those loads.
template <typename T>
__global__ void __launch_bounds__(64) k_rot_blk_thomas(int N, int total, T* __restrict__ sc) {
    extern __shared__ __align__(16) unsigned char rot_lds_raw[];
    T* lds = reinterpret_cast<T*>(rot_lds_raw);
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;          // no barrier below: every thread works alone
    const int TB = blockDim.x;
    auto lw = [&](int s, int w) -> T& { return lds[((long)s * ROT_BLK_LDS + w) * TB + threadIdx.x]; };
    constexpr int RB = sizeof(T) == 4 ? 8 : 4;
    T buf[RB][ROT_BLK_WORDS];
    using V = typename Vec16<T>::type;
    constexpr int NV = 16 / sizeof(T);
    auto load = [&](int s, T (&o)[ROT_BLK_WORDS]) {
        if (s < N) {
            const V* src = reinterpret_cast<const V*>(rot_sc(sc, 0, s, total, q, N));
#pragma unroll
            for (int k = 0; k < ROT_BLK_WORDS / NV; ++k) {
                const V x = src[k];
                __builtin_memcpy(&o[k * NV], &x, sizeof(V));
            }
        }
    };
#pragma unroll
    for (int b = 0; b < RB; ++b) load(b, buf[b]);
    T S[3][3], z[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        z[a] = buf[0][18 + a];
#pragma unroll
        for (int b = 0; b < 3; ++b) S[a][b] = buf[0][9 + a * 3 + b];
    }
    load(RB, buf[0]);
    for (int s0 = 1; s0 < N; s0 += RB) {
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const int s = s0 + u;
            if (s >= N) break;
            T(&cur)[ROT_BLK_WORDS] = buf[(1 + u) % RB];
            Chol3<T> ch;
            ch.factor(S);
            // G = L^-1 F column by column (F = -beta_s/dt), zz = L^-1 z
            T G[3][3], zz[3];
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const T f[3] = {cur[b], cur[3 + b], cur[6 + b]};
                T gcol[3];
                ch.lower(f, gcol);
#pragma unroll
                for (int a = 0; a < 3; ++a) G[a][b] = gcol[a];
            }
            ch.lower(z, zz);
            // W = L^-T G, t = L^-T zz, kept for the back substitution
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const T gcol[3] = {G[0][b], G[1][b], G[2][b]};
                T wcol[3];
                ch.upper(gcol, wcol);
#pragma unroll
                for (int a = 0; a < 3; ++a) lw(s - 1, a * 3 + b) = wcol[a];
            }
            T t[3];
            ch.upper(zz, t);
#pragma unroll
            for (int a = 0; a < 3; ++a) lw(s - 1, 9 + a) = t[a];
            // S = D_s - G^T G, z = rhs_s - G^T zz
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                z[a] = cur[18 + a] - (G[0][a] * zz[0] + G[1][a] * zz[1] + G[2][a] * zz[2]);
#pragma unroll
                for (int b = 0; b <= a; ++b) {
                    S[a][b] = cur[9 + a * 3 + b] - (G[0][a] * G[0][b] + G[1][a] * G[1][b] + G[2][a] * G[2][b]);
                    S[b][a] = S[a][b];
                }
            }
            load(s + RB, cur);
        }
    }
    T y[3];
    {
        Chol3<T> ch;
        ch.factor(S);
        T zz[3];
        ch.lower(z, zz);
        ch.upper(zz, y);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) *rot_sc(sc, 18 + a, N - 1, total, q, N) = y[a];
    for (int s = N - 2; s >= 0; --s) {
        T yn[3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            yn[a] = lw(s, 9 + a) - (lw(s, a * 3) * y[0] + lw(s, a * 3 + 1) * y[1] + lw(s, a * 3 + 2) * y[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            y[a] = yn[a];
            *rot_sc(sc, 18 + a, s, total, q, N) = y[a];
        }
    }
}

// Threads per block of the elimination: LDS holds 12 words per (thread,
// slot), within 64 KB; at least one thread (N <= 1024 fits even in FP64).
template <typename T>
inline int rot_blk_threads(int N) {
    int tb = 64;
    while (tb > 1 && (long)tb * N * ROT_BLK_LDS * sizeof(T) > 65536) tb >>= 1;
    return tb;
}

// The corrections of (colour cell q, slot s) from y_s (in rec) and y_{s-1}
// (in prev, used when s > 0), relaxed by omega and added to the state.
template <typename T>
__device__ inline void rot_apply_item(const Grid& g, int N, const ColourSet& cs, int q, int s, T dt, T kr, T lm,
                                      T omega, T* __restrict__ v, T* __restrict__ pb, T* __restrict__ u,
                                      T* __restrict__ p, const T* __restrict__ r1, const T* __restrict__ r2,
                                      const T* __restrict__ r3, const T* __restrict__ r4, const T* rec,
                                      const T* prev) {
    int i, j, k;
    colour_cell(cs, q, i, j, k);
    RotCell<T> rc;
    rc.init(g, i, j);
    T* vs = v + (long)s * g.nface;
    T B[4][4];
    rot_cell_B<T>(g, rc, vs, i, j, dt, B);       // before this thread changes v_s
    T y[3], dv[4], dvp[4] = {0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < 3; ++a) y[a] = rec[18 + a];
    rc.zy(y, dv);
    const T e = r2[(long)s * g.ncell + rc.cell];
#pragma unroll
    for (int r = 0; r < 4; ++r) dv[r] += rc.gv[r] * e / rc.gg;
    if (s > 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) y[a] = prev[18 + a];
        rc.zy(y, dvp);
        const T ep = r2[(long)(s - 1) * g.ncell + rc.cell];
#pragma unroll
        for (int r = 0; r < 4; ++r) dvp[r] += rc.gv[r] * ep / rc.gg;
    }
    // q = a_s + dv_{s-1}/dt - B_s dv_s;  du = -P q + g b/|g|^2;  dp = -(b + g^T q)/|g|^2
    T qv[4], bdv[4], du[4];
    mat4_vec(B, dv, bdv);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        qv[r] = (rc.m[r] > 0 ? r3[(long)s * g.nface + rc.face[r]] : (T)0) + dvp[r] / dt - bdv[r];
    const T b = r4[(long)s * g.ncell + rc.cell];
    rc.proj(qv, du);
#pragma unroll
    for (int r = 0; r < 4; ++r) du[r] = -du[r] + rc.gv[r] * b / rc.gg;
    const T dp = -(b + rc.gdot(qv)) / rc.gg;
    // dpbar = (kappa e + g^T B^T du - [s<N-1] b_{s+1}/dt - g^T c)/|g|^2
    const bool last = s == N - 1;
    T btdu[4], c[4];
    mat4t_vec(B, du, btdu);
#pragma unroll
    for (int r = 0; r < 4; ++r) c[r] = rc.m[r] > 0 ? r1[(long)s * g.nface + rc.face[r]] : (T)0;
    const T kap = (last ? (T)0 : kr) + lm;
    T num = kap * e + rc.gdot(btdu) - rc.gdot(c);
    if (!last) num -= r4[(long)(s + 1) * g.ncell + rc.cell] / dt;
    const T dpb = num / rc.gg;
    T* us = u + (long)s * g.nface;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (rc.m[r] > 0) {
            vs[rc.face[r]] += omega * dv[r];
            us[rc.face[r]] += omega * du[r];
        }
    p[(long)s * g.ncell + rc.cell] += omega * dp;
    pb[(long)s * g.ncell + rc.cell] += omega * dpb;
}


template <typename T>
__global__ void __launch_bounds__(256) k_rot_blk_apply(Grid g, int N, ColourSet cs, T dt, T kr, T lm, T omega, T* __restrict__ v,
                                T* __restrict__ pb, T* __restrict__ u, T* __restrict__ p, const T* __restrict__ r1,
                                const T* __restrict__ r2, const T* __restrict__ r3, const T* __restrict__ r4,
                                const T* __restrict__ sc) {
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (long)cs.total * N) return;
    const int q = (int)(tid % cs.total), s = (int)(tid / cs.total);
    rot_apply_item(g, N, cs, q, s, dt, kr, lm, omega, v, pb, u, p, r1, r2, r3, r4, rot_sc(sc, 0, s, cs.total, q, N),
                   s > 0 ? rot_sc(sc, 0, s - 1, cs.total, q, N) : (const T*)nullptr);
}

// Elimination of one cell whose records (slot s at rec + s * stride) are in
// LDS: the same steps as k_rot_blk_thomas; W_{s-1}, t_{s-1} replace D_{s-1}
// and the right-hand side of slot s - 1, y_s replaces t_s.  Each step reads
// the next step's record before it writes its own results, so the reads
// need not wait for the writes (the compiler cannot tell the two apart).
template <typename T>
__device__ inline void rot_eliminate_local(T* rec, int stride, int N) {
    T S[3][3], z[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        z[a] = rec[18 + a];
#pragma unroll
        for (int b = 0; b < 3; ++b) S[a][b] = rec[9 + a * 3 + b];
    }
    auto load = [&](int s, T (&o)[21]) {
        const T* x = rec + (long)s * stride;
#pragma unroll
        for (int w = 0; w < 21; ++w) o[w] = x[w];
    };
    // one step: S = L L^T, G = L^-1 F_s, zz = L^-1 z; S <- D_s - G^T G,
    // z <- rhs_s - G^T zz; slot s - 1 keeps W = L^-T G and t = L^-T zz
    auto step = [&](int s, const T (&cur)[21]) {
        T* prv = rec + (long)(s - 1) * stride;
        Chol3<T> ch;
        ch.factor(S);
        T G[3][3], zz[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const T f[3] = {cur[b], cur[3 + b], cur[6 + b]};
            T gcol[3];
            ch.lower(f, gcol);
#pragma unroll
            for (int a = 0; a < 3; ++a) G[a][b] = gcol[a];
        }
        ch.lower(z, zz);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            z[a] = cur[18 + a] - (G[0][a] * zz[0] + G[1][a] * zz[1] + G[2][a] * zz[2]);
#pragma unroll
            for (int b = 0; b <= a; ++b) {
                S[a][b] = cur[9 + a * 3 + b] - (G[0][a] * G[0][b] + G[1][a] * G[1][b] + G[2][a] * G[2][b]);
                S[b][a] = S[a][b];
            }
        }
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const T gcol[3] = {G[0][b], G[1][b], G[2][b]};
            T wcol[3];
            ch.upper(gcol, wcol);
#pragma unroll
            for (int a = 0; a < 3; ++a) prv[9 + a * 3 + b] = wcol[a];
        }
        T t[3];
        ch.upper(zz, t);
#pragma unroll
        for (int a = 0; a < 3; ++a) prv[18 + a] = t[a];
    };
    // two buffers in turn: the next record is read before a step writes
    T ba[21], bb[21];
    if (N > 1) load(1, ba);
    for (int s = 1; s < N; s += 2) {
        if (s + 1 < N) load(s + 1, bb);
        step(s, ba);
        if (s + 1 >= N) break;
        if (s + 2 < N) load(s + 2, ba);
        step(s + 1, bb);
    }
    T y[3];
    {
        Chol3<T> ch;
        ch.factor(S);
        T zz[3];
        ch.lower(z, zz);
        ch.upper(zz, y);
    }
    T* last = rec + (long)(N - 1) * stride;
#pragma unroll
    for (int a = 0; a < 3; ++a) last[18 + a] = y[a];
    auto loadb = [&](int s, T (&o)[12]) {
        const T* x = rec + (long)s * stride + 9;
#pragma unroll
        for (int w = 0; w < 12; ++w) o[w] = x[w];
    };
    auto back = [&](int s, const T (&r)[12]) {
        T yn[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) yn[a] = r[9 + a] - (r[a * 3] * y[0] + r[a * 3 + 1] * y[1] + r[a * 3 + 2] * y[2]);
        T* o = rec + (long)s * stride + 18;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            y[a] = yn[a];
            o[a] = y[a];
        }
    };
    T ca[12], cb[12];
    if (N > 1) loadb(N - 2, ca);
    for (int s = N - 2; s >= 0; s -= 2) {
        if (s > 0) loadb(s - 1, cb);
        back(s, ca);
        if (s == 0) break;
        if (s > 1) loadb(s - 2, ca);
        back(s - 1, cb);
    }
}

// One launch per colour for horizons whose records fit in LDS: a block takes
// TB cells of the colour; its threads form the records of every (cell, slot)
// in LDS, one thread per cell eliminates in time, and the threads add the
// corrections per (cell, slot).  Cells of one colour share nothing the
// others write, so blocks need no ordering among themselves.
template <typename T>
__global__ void __launch_bounds__(512) k_rot_blk_fused(Grid g, int N, ColourSet cs, int TB, T dt, T kr, T lm, T omega,
                                                       T* __restrict__ v, T* __restrict__ pb, T* __restrict__ u,
                                                       T* __restrict__ p, const T* __restrict__ r1,
                                                       const T* __restrict__ r2, const T* __restrict__ r3,
                                                       const T* __restrict__ r4) {
    extern __shared__ __align__(16) unsigned char rot_lds_raw[];
    T* lds = reinterpret_cast<T*>(rot_lds_raw);
    const int stride = ROT_BLK_WORDS;
    const int cstride = N * ROT_BLK_WORDS + 16 / (int)sizeof(T);     // per cell, padded off the bank stride
    const int c0 = blockIdx.x * TB;
    const int nc = min(TB, cs.total - c0);
    const int items = nc * N;
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
        const int cl = it % nc, s = it / nc;
        rot_setup_item(g, N, cs, c0 + cl, s, dt, kr, lm, v, r1, r2, r3, r4, lds + (long)cl * cstride + s * stride);
    }
    __syncthreads();
    if ((int)threadIdx.x < nc) rot_eliminate_local(lds + (long)threadIdx.x * cstride, stride, N);
    __syncthreads();
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
        const int cl = it % nc, s = it / nc;
        const T* rec = lds + (long)cl * cstride + s * stride;
        rot_apply_item(g, N, cs, c0 + cl, s, dt, kr, lm, omega, v, pb, u, p, r1, r2, r3, r4, rec,
                       s > 0 ? rec - stride : (const T*)nullptr);
    }
}

// Cells per block of the fused launch (records within 64 KB of LDS), 0 when
// one cell's records do not fit (the three-launch form then runs).
template <typename T>
inline int rot_fused_cells(int N) {
    const long per = ((long)N * ROT_BLK_WORDS + 16 / (long)sizeof(T)) * (long)sizeof(T);
    return (int)std::min<long>(8, 65536 / per);
}

}  // namespace stfas
