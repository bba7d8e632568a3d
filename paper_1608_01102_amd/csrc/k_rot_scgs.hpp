// SCGS local solve of the rotational operator: the cell's spacetime system
// of Sec. 4.3 eq:HESS with the cell's block of dAdv/dv in it (2D: 4 faces and
// the centre, the paper's 5x5 blocks; 3D: 6 faces and the centre, 7x7).
//
// Unknowns of one cell, for every slot s = 0..N-1 (v[s] = v_{s+1},
// u[s] = u_s, p[s] = p_{s+1}, pbar[s] = pbar_{s+1}): the corrections of v and
// u at the cell's 2d faces and of p, pbar at its centre.  Face slots: 2a the
// low a-face, 2a + 1 the high one; wall faces are not unknowns.  With g the
// divergence coefficients of the cell's interior faces (-1/h low, +1/h high),
// M the interior mask, B_s = I/dt + dAdv/dv at v_{s+1} (rows and columns of
// the cell's interior faces) and kappa_s = K/r [s < N-1] + the smoother's
// perturbation, the rows are (a, b, c, e: the residual of F3_s, F4_s,
// F1_{s+1}, F2_{s+1})
//   F3_s:  -du_s - dv_{s-1}/dt + B_s dv_s - g dp_s            = a_s   (dv_{-1} = 0)
//   F4_s:   g^T du_s                                          = b_s
//   F1:     B_s^T du_s + kappa_s dv_s - [s<N-1] du_{s+1}/dt - g dpbar_s = c_s
//   F2:     g^T dv_s                                          = e_s
// The u rows give du_s = -P q_s + g b_s/|g|^2 and dp_s = -(b_s + g^T q_s)/|g|^2
// with q_s = a_s + dv_{s-1}/dt - B_s dv_s and P = M - g g^T/|g|^2.  Put into
// the v rows, and with dv_s = Z y_s + g e_s/|g|^2 (Z an orthonormal basis of
// the interior faces' divergence-free directions, at most K = 2d - 1 of them),
// the corrections y form a block tridiagonal system with KxK blocks
//   D_s = beta_s^T beta_s + kappa_s + [s<N-1]/dt^2,   beta_s = Z^T B_s Z,
//   coupling of y_{s-1} (row) and y_s (column): F_s = -beta_s/dt,
// which is symmetric positive definite (the Schur complement of the u
// blocks, which are -I), so block elimination needs no pivoting.  The
// eliminated quantities follow from y: du, dp from the u rows, and
//   dpbar_s = (kappa_s e_s + g^T B_s^T du_s - [s<N-1] b_{s+1}/dt - g^T c_s)/|g|^2
// (g^T du_{s+1} = b_{s+1}).  Every correction is relaxed by omega.
//
// One launch per colour while a cell's records fit in LDS (k_rot_blk_fused:
// records per (cell, slot) formed in parallel, one thread per cell
// eliminates in time, corrections in parallel); three launches through the
// workspace otherwise.  Cells of one colour share no face and no face of one
// is read by another's block (their faces share no edge), so nothing needs
// atomics.
#pragma once
#include "common.hpp"
#include "k_kkt.hpp"
#include "k_rot.hpp"

namespace stfas {

// Sizes of the local system: NS face slots, K reduced directions, and the
// record of one (cell, slot): [0, K*K) F_s (row-major), [K*K, 2K*K) D_s,
// [2K*K, 2K*K + K) the reduced right-hand side (replaced by y_s), padded to a
// multiple of 16 bytes.
template <int D>
struct RotDims {
    static constexpr int NS = 2 * D, K = 2 * D - 1;
    static constexpr int OF = 0, OD = K * K, OR = 2 * K * K;
    static constexpr int USED = 2 * K * K + K;
    static constexpr int REC = (USED + 3) / 4 * 4;      // 24 in 2D, 56 in 3D
};

// The cell's block of dAdv/dv at v (rows: Adv at the face slots, columns: v
// at the face slots), from the edge form of k_rot.hpp: every edge of the cell
// meets one p-face (slot tp) and one q-face (slot tq) of the cell; the p-face
// gets -1/4 w S_q and the q-face +1/4 w S_p there.  The cell's q-face enters w
// with +1/h at the edge's lower p-end and -1/h at its upper one, its p-face
// with -1/h at the lower q-end and +1/h at the upper (interior edges only),
// and each enters its own sum with 1.
template <typename T, int D>
__device__ inline void rot_cell_jacobian(const Grid& g, const T* v, int i, int j, int k, T ih,
                                         T (&J)[2 * D][2 * D]) {
#pragma unroll
    for (int t = 0; t < 2 * D; ++t)
#pragma unroll
        for (int s = 0; s < 2 * D; ++s) J[t][s] = 0;
    const int cx[3] = {i, j, k};
#pragma unroll
    for (int tr = 0; tr < RotTriples<D>::n; ++tr) {
        const int p = RotTriples<D>::t[tr][1], q = RotTriples<D>::t[tr][2];
#pragma unroll
        for (int dp = 0; dp < 2; ++dp)
#pragma unroll
            for (int dq = 0; dq < 2; ++dq) {
                int e[3] = {cx[0], cx[1], cx[2]};
                e[p] += dp;
                e[q] += dq;
                T w, sp, sq;
                const bool in = rot_edge(g, v, p, q, e, ih, false, w, sp, sq);
                const T cp = in ? (dq == 0 ? -ih : ih) : (T)0, cq = in ? (dp == 0 ? ih : -ih) : (T)0;
                const int tp = 2 * p + dp, tq = 2 * q + dq;
                J[tp][tp] -= (T)0.25 * cp * sq;
                J[tp][tq] -= (T)0.25 * (cq * sq + w);
                J[tq][tp] += (T)0.25 * (cp * sp + w);
                J[tq][tq] += (T)0.25 * cq * sp;
            }
    }
}

// Geometry of one cell's local system: g, |g|^2, the interior mask and Z.
template <typename T, int D>
struct RotCell {
    static constexpr int NS = RotDims<D>::NS, K = RotDims<D>::K;
    int face[NS];
    int cell;
    T m[NS], gv[NS], gg;
    T Z[NS][K];
    T act[K];      // 1 for the columns of Z in use

    __device__ void init(const Grid& g, int i, int j, int k) {
        CellFaces<D> cf;
        cell_faces<D>(g, i, j, k, cf);
        cell = cell_index(g, i, j, k);
        const T ih = (T)(1.0 / g.h);
        gg = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
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
        for (int c = 0; c < K; ++c) {
            act[c] = 0;
#pragma unroll
            for (int r = 0; r < NS; ++r) Z[r][c] = 0;
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            T z[NS];
#pragma unroll
            for (int r = 0; r < NS; ++r) z[r] = (r == s ? m[s] : (T)0) - gv[r] * gv[s] / gg;
#pragma unroll
            for (int c = 0; c < K; ++c) {
                T d = 0;
#pragma unroll
                for (int r = 0; r < NS; ++r) d += Z[r][c] * z[r];
#pragma unroll
                for (int r = 0; r < NS; ++r) z[r] -= d * Z[r][c];
            }
            T n2 = 0;
#pragma unroll
            for (int r = 0; r < NS; ++r) n2 += z[r] * z[r];
            if (m[s] > 0 && n2 > (T)0.1 && nk < K) {
                const T inv = (T)1 / sqrt(n2);
#pragma unroll
                for (int c = 0; c < K; ++c)
                    if (c == nk) {
#pragma unroll
                        for (int r = 0; r < NS; ++r) Z[r][c] = z[r] * inv;
                        act[c] = 1;
                    }
                ++nk;
            }
        }
    }
    // P x = M x - g (g^T x)/|g|^2
    __device__ void proj(const T (&x)[NS], T (&o)[NS]) const {
        const T d = gdot(x) / gg;
#pragma unroll
        for (int r = 0; r < NS; ++r) o[r] = m[r] * x[r] - gv[r] * d;
    }
    __device__ T gdot(const T (&x)[NS]) const {
        T d = 0;
#pragma unroll
        for (int r = 0; r < NS; ++r) d += gv[r] * x[r];
        return d;
    }
    // Z^T x and Z y
    __device__ void zt(const T (&x)[NS], T (&o)[K]) const {
#pragma unroll
        for (int c = 0; c < K; ++c) {
            o[c] = 0;
#pragma unroll
            for (int r = 0; r < NS; ++r) o[c] += Z[r][c] * x[r];
        }
    }
    __device__ void zy(const T (&y)[K], T (&o)[NS]) const {
#pragma unroll
        for (int r = 0; r < NS; ++r) {
            o[r] = 0;
#pragma unroll
            for (int c = 0; c < K; ++c) o[r] += Z[r][c] * y[c];
        }
    }
};

// B_s = I/dt + dAdv/dv at the face slots of the cell, rows and columns of wall faces zero.
template <typename T, int D>
__device__ inline void rot_cell_B(const Grid& g, const RotCell<T, D>& rc, const T* v, int i, int j, int k, T dt,
                                  T (&B)[2 * D][2 * D]) {
    rot_cell_jacobian<T, D>(g, v, i, j, k, (T)(1.0 / g.h), B);
#pragma unroll
    for (int t = 0; t < 2 * D; ++t)
#pragma unroll
        for (int s = 0; s < 2 * D; ++s) B[t][s] = (B[t][s] + (t == s ? (T)1 / dt : (T)0)) * rc.m[t] * rc.m[s];
}

template <typename T, int NS>
__device__ inline void rot_mv(const T (&B)[NS][NS], const T (&x)[NS], T (&o)[NS]) {
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        o[t] = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s) o[t] += B[t][s] * x[s];
    }
}
template <typename T, int NS>
__device__ inline void rot_mtv(const T (&B)[NS][NS], const T (&x)[NS], T (&o)[NS]) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        o[s] = 0;
#pragma unroll
        for (int t = 0; t < NS; ++t) o[s] += B[t][s] * x[t];
    }
}

// Right-hand side quantities of slot s: ahat_s = P a_s - g b_s/|g|^2 and vbar_s = g e_s/|g|^2.
template <typename T, int D>
__device__ inline void rot_slot_rhs(const Grid& g, const RotCell<T, D>& rc, const T* r2, const T* r3, const T* r4,
                                    int s, T (&ahat)[2 * D], T (&vbar)[2 * D]) {
    T a[2 * D];
#pragma unroll
    for (int r = 0; r < 2 * D; ++r) a[r] = rc.m[r] > 0 ? r3[(long)s * g.nface + rc.face[r]] : (T)0;
    rc.proj(a, ahat);
    const T b = r4[(long)s * g.ncell + rc.cell] / rc.gg, e = r2[(long)s * g.ncell + rc.cell] / rc.gg;
#pragma unroll
    for (int r = 0; r < 2 * D; ++r) {
        ahat[r] -= rc.gv[r] * b;
        vbar[r] = rc.gv[r] * e;
    }
}

// The record of (colour cell q, slot s): F_s, D_s and the reduced right-hand side.
template <typename T, int D>
__device__ inline void rot_setup_item(const Grid& g, int N, const ColourSet& cs, int q, int s, T dt, T kr, T lm,
                                      const T* __restrict__ v, const T* __restrict__ r1, const T* __restrict__ r2,
                                      const T* __restrict__ r3, const T* __restrict__ r4, T* rec) {
    using RD = RotDims<D>;
    constexpr int NS = RD::NS, K = RD::K;
    int i, j, k;
    colour_cell(cs, q, i, j, k);
    RotCell<T, D> rc;
    rc.init(g, i, j, k);
    T B[NS][NS];
    rot_cell_B<T, D>(g, rc, v + (long)s * g.nface, i, j, k, dt, B);
    // beta_s = Z^T B_s Z
    T BZ[NS][K], beta[K][K];
#pragma unroll
    for (int t = 0; t < NS; ++t)
#pragma unroll
        for (int c = 0; c < K; ++c) {
            T acc = 0;
#pragma unroll
            for (int r = 0; r < NS; ++r) acc += B[t][r] * rc.Z[r][c];
            BZ[t][c] = acc;
        }
#pragma unroll
    for (int a = 0; a < K; ++a)
#pragma unroll
        for (int b = 0; b < K; ++b) {
            T acc = 0;
#pragma unroll
            for (int r = 0; r < NS; ++r) acc += rc.Z[r][a] * BZ[r][b];
            beta[a][b] = acc;
        }
    const bool last = s == N - 1;
    const T kap = (last ? (T)0 : kr) + lm + (last ? (T)0 : (T)1 / (dt * dt));
#pragma unroll
    for (int a = 0; a < K; ++a)
#pragma unroll
        for (int b = 0; b < K; ++b) {
            T d = 0;
#pragma unroll
            for (int c = 0; c < K; ++c) d += beta[c][a] * beta[c][b];
            if (a == b) d += rc.act[a] > 0 ? kap : (T)1;
            rec[RD::OF + a * K + b] = -beta[a][b] / dt;
            rec[RD::OD + a * K + b] = d;
        }
    // w = c_s + B_s^T ahat_s - B_s^T P B_s vbar_s  [- ahat_{s+1}/dt + P B_{s+1} vbar_{s+1}/dt]
    T ahat[NS], vbar[NS], w4[NS], t4[NS], p4[NS];
    rot_slot_rhs<T, D>(g, rc, r2, r3, r4, s, ahat, vbar);
    rot_mv<T, NS>(B, vbar, t4);
    rc.proj(t4, p4);
#pragma unroll
    for (int r = 0; r < NS; ++r) p4[r] = ahat[r] - p4[r];
    rot_mtv<T, NS>(B, p4, w4);
#pragma unroll
    for (int r = 0; r < NS; ++r) w4[r] += rc.m[r] > 0 ? r1[(long)s * g.nface + rc.face[r]] : (T)0;
    if (!last) {
        T B1[NS][NS];
        rot_cell_B<T, D>(g, rc, v + (long)(s + 1) * g.nface, i, j, k, dt, B1);
        rot_slot_rhs<T, D>(g, rc, r2, r3, r4, s + 1, ahat, vbar);
        rot_mv<T, NS>(B1, vbar, t4);
        rc.proj(t4, p4);
#pragma unroll
        for (int r = 0; r < NS; ++r) w4[r] += (p4[r] - ahat[r]) / dt;
    }
    T rr[K];
    rc.zt(w4, rr);
#pragma unroll
    for (int a = 0; a < K; ++a) rec[RD::OR + a] = rr[a];
}

__device__ inline float rot_rsq(float x) { return __builtin_amdgcn_rsqf(x); }   // x >= 1/dt^2 here
__device__ inline double rot_rsq(double x) { return 1.0 / sqrt(x); }

// Cholesky factor of a symmetric positive definite KxK matrix S = L L^T: the
// entries below the diagonal and the reciprocals of the diagonal.
template <typename T, int K>
struct Chol {
    T l[K][K];
    T id[K];
    __device__ void factor(const T (&S)[K][K]) {
#pragma unroll
        for (int c = 0; c < K; ++c) {
            T d = S[c][c];
#pragma unroll
            for (int x = 0; x < c; ++x) d -= l[c][x] * l[c][x];
            id[c] = rot_rsq(d);
#pragma unroll
            for (int r = c + 1; r < K; ++r) {
                T t = S[r][c];
#pragma unroll
                for (int x = 0; x < c; ++x) t -= l[r][x] * l[c][x];
                l[r][c] = t * id[c];
            }
        }
    }
    __device__ void lower(const T (&f)[K], T (&o)[K]) const {     // L o = f
#pragma unroll
        for (int r = 0; r < K; ++r) {
            T t = f[r];
#pragma unroll
            for (int x = 0; x < r; ++x) t -= l[r][x] * o[x];
            o[r] = t * id[r];
        }
    }
    __device__ void upper(const T (&f)[K], T (&o)[K]) const {     // L^T o = f
#pragma unroll
        for (int r = K - 1; r >= 0; --r) {
            T t = f[r];
#pragma unroll
            for (int x = r + 1; x < K; ++x) t -= l[x][r] * o[x];
            o[r] = t * id[r];
        }
    }
};

// One step of the elimination: S = L L^T, G = L^-1 F_s, zz = L^-1 z; then
// S <- D_s - G^T G, z <- rhs_s - G^T zz; W = L^-T G and t = L^-T zz go to
// put(word, value) at the words of D and the right-hand side (for the back
// substitution y_{s-1} = t - W y_s).
template <typename T, int K, typename Put>
__device__ inline void rot_elim_step(T (&S)[K][K], T (&z)[K], const T* cur, Put put) {
    using RD = RotDims<(K + 1) / 2>;
    Chol<T, K> ch;
    ch.factor(S);
    T G[K][K], zz[K];
#pragma unroll
    for (int b = 0; b < K; ++b) {
        T f[K], gcol[K];
#pragma unroll
        for (int a = 0; a < K; ++a) f[a] = cur[RD::OF + a * K + b];
        ch.lower(f, gcol);
#pragma unroll
        for (int a = 0; a < K; ++a) G[a][b] = gcol[a];
    }
    ch.lower(z, zz);
#pragma unroll
    for (int a = 0; a < K; ++a) {
        T acc = cur[RD::OR + a];
#pragma unroll
        for (int c = 0; c < K; ++c) acc -= G[c][a] * zz[c];
        z[a] = acc;
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            T sab = cur[RD::OD + a * K + b];
#pragma unroll
            for (int c = 0; c < K; ++c) sab -= G[c][a] * G[c][b];
            S[a][b] = sab;
            S[b][a] = sab;
        }
    }
#pragma unroll
    for (int b = 0; b < K; ++b) {
        T gcol[K], wcol[K];
#pragma unroll
        for (int a = 0; a < K; ++a) gcol[a] = G[a][b];
        ch.upper(gcol, wcol);
#pragma unroll
        for (int a = 0; a < K; ++a) put(RD::OD + a * K + b, wcol[a]);
    }
    T t[K];
    ch.upper(zz, t);
#pragma unroll
    for (int a = 0; a < K; ++a) put(RD::OR + a, t[a]);
}

template <typename T, int K>
__device__ inline void rot_elim_last(const T (&S)[K][K], const T (&z)[K], T (&y)[K]) {
    Chol<T, K> ch;
    ch.factor(S);
    T zz[K];
    ch.lower(z, zz);
    ch.upper(zz, y);
}

template <typename P>
__device__ inline P* rot_sc(P* sc, int rec, int w, int s, int total, int q) {
    return sc + ((long)s * total + q) * rec + w;
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

template <typename T, int D>
__global__ void __launch_bounds__(256) k_rot_blk_setup(Grid g, int N, ColourSet cs, T dt, T kr, T lm,
                                                       const T* __restrict__ v, const T* __restrict__ r1,
                                                       const T* __restrict__ r2, const T* __restrict__ r3,
                                                       const T* __restrict__ r4, T* __restrict__ sc) {
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (long)cs.total * N) return;
    const int q = (int)(tid % cs.total), s = (int)(tid / cs.total);
    rot_setup_item<T, D>(g, N, cs, q, s, dt, kr, lm, v, r1, r2, r3, r4,
                         rot_sc(sc, RotDims<D>::REC, 0, s, cs.total, q));
}

// Words of LDS per (thread, slot) in the elimination through the workspace: W_s and t_s.
template <int D>
constexpr int rot_blk_lds_words() {
    return RotDims<D>::K * RotDims<D>::K + RotDims<D>::K;
}

// Elimination in time through the workspace, one thread per cell of the
// colour: the records are read with 16-byte loads RB steps ahead of their use
// (they do not depend on the recurrence) and W, t stay in LDS (blockDim.x
// threads x N slots), so no global store sits between those loads.
template <typename T, int D>
__global__ void __launch_bounds__(64) k_rot_blk_thomas(int N, int total, T* __restrict__ sc) {
    using RD = RotDims<D>;
    constexpr int K = RD::K, REC = RD::REC, LW = rot_blk_lds_words<D>();
    extern __shared__ __align__(16) unsigned char rot_lds_raw[];
    T* lds = reinterpret_cast<T*>(rot_lds_raw);
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;          // no barrier below: every thread works alone
    const int TB = blockDim.x;
    auto lw = [&](int s, int w) -> T& { return lds[((long)s * LW + w) * TB + threadIdx.x]; };
    constexpr int RB = (D == 2 && sizeof(T) == 4) ? 8 : 4;
    using V = typename Vec16<T>::type;
    constexpr int NV = 16 / sizeof(T);
    T buf[RB][REC];
    auto load = [&](int s, T (&o)[REC]) {
        if (s < N) {
            const V* src = reinterpret_cast<const V*>(rot_sc(sc, REC, 0, s, total, q));
#pragma unroll
            for (int x = 0; x < REC / NV; ++x) {
                const V val = src[x];
                __builtin_memcpy(&o[x * NV], &val, sizeof(V));
            }
        }
    };
#pragma unroll
    for (int b = 0; b < RB; ++b) load(b, buf[b]);
    T S[K][K], z[K];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        z[a] = buf[0][RD::OR + a];
#pragma unroll
        for (int b = 0; b < K; ++b) S[a][b] = buf[0][RD::OD + a * K + b];
    }
    load(RB, buf[0]);
    for (int s0 = 1; s0 < N; s0 += RB) {
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const int s = s0 + u;
            if (s >= N) break;
            T(&cur)[REC] = buf[(1 + u) % RB];
            // W at LDS words [0, K*K), t at [K*K, K*K + K)
            rot_elim_step<T, K>(S, z, cur, [&](int w, T x) {
                lw(s - 1, w < RD::OR ? w - RD::OD : K * K + (w - RD::OR)) = x;
            });
            load(s + RB, cur);
        }
    }
    T y[K];
    rot_elim_last<T, K>(S, z, y);
#pragma unroll
    for (int a = 0; a < K; ++a) *rot_sc(sc, REC, RD::OR + a, N - 1, total, q) = y[a];
    for (int s = N - 2; s >= 0; --s) {
        T yn[K];
#pragma unroll
        for (int a = 0; a < K; ++a) {
            T acc = lw(s, K * K + a);
#pragma unroll
            for (int b = 0; b < K; ++b) acc -= lw(s, a * K + b) * y[b];
            yn[a] = acc;
        }
#pragma unroll
        for (int a = 0; a < K; ++a) {
            y[a] = yn[a];
            *rot_sc(sc, REC, RD::OR + a, s, total, q) = y[a];
        }
    }
}

// Threads per block of the elimination through the workspace: LDS holds W, t
// per (thread, slot), within 64 KB; at least one thread.
template <typename T, int D>
inline int rot_blk_threads(int N) {
    int tb = 64;
    while (tb > 1 && (long)tb * N * rot_blk_lds_words<D>() * (long)sizeof(T) > 65536) tb >>= 1;
    return tb;
}

// The corrections of (colour cell q, slot s) from y_s (in rec) and y_{s-1}
// (in prev, used when s > 0), relaxed by omega and added to the state.
template <typename T, int D>
__device__ inline void rot_apply_item(const Grid& g, int N, const ColourSet& cs, int q, int s, T dt, T kr, T lm,
                                      T omega, T* __restrict__ v, T* __restrict__ pb, T* __restrict__ u,
                                      T* __restrict__ p, const T* __restrict__ r1, const T* __restrict__ r2,
                                      const T* __restrict__ r3, const T* __restrict__ r4, const T* rec,
                                      const T* prev) {
    using RD = RotDims<D>;
    constexpr int NS = RD::NS, K = RD::K;
    int i, j, k;
    colour_cell(cs, q, i, j, k);
    RotCell<T, D> rc;
    rc.init(g, i, j, k);
    T* vs = v + (long)s * g.nface;
    T B[NS][NS];
    rot_cell_B<T, D>(g, rc, vs, i, j, k, dt, B);       // before this thread changes v_s
    T y[K], dv[NS], dvp[NS];
#pragma unroll
    for (int a = 0; a < K; ++a) y[a] = rec[RD::OR + a];
    rc.zy(y, dv);
    const T e = r2[(long)s * g.ncell + rc.cell];
#pragma unroll
    for (int r = 0; r < NS; ++r) {
        dv[r] += rc.gv[r] * e / rc.gg;
        dvp[r] = 0;
    }
    if (s > 0) {
#pragma unroll
        for (int a = 0; a < K; ++a) y[a] = prev[RD::OR + a];
        rc.zy(y, dvp);
        const T ep = r2[(long)(s - 1) * g.ncell + rc.cell];
#pragma unroll
        for (int r = 0; r < NS; ++r) dvp[r] += rc.gv[r] * ep / rc.gg;
    }
    // q = a_s + dv_{s-1}/dt - B_s dv_s;  du = -P q + g b/|g|^2;  dp = -(b + g^T q)/|g|^2
    T qv[NS], bdv[NS], du[NS];
    rot_mv<T, NS>(B, dv, bdv);
#pragma unroll
    for (int r = 0; r < NS; ++r)
        qv[r] = (rc.m[r] > 0 ? r3[(long)s * g.nface + rc.face[r]] : (T)0) + dvp[r] / dt - bdv[r];
    const T b = r4[(long)s * g.ncell + rc.cell];
    rc.proj(qv, du);
#pragma unroll
    for (int r = 0; r < NS; ++r) du[r] = -du[r] + rc.gv[r] * b / rc.gg;
    const T dp = -(b + rc.gdot(qv)) / rc.gg;
    // dpbar = (kappa e + g^T B^T du - [s<N-1] b_{s+1}/dt - g^T c)/|g|^2
    const bool last = s == N - 1;
    T btdu[NS], c[NS];
    rot_mtv<T, NS>(B, du, btdu);
#pragma unroll
    for (int r = 0; r < NS; ++r) c[r] = rc.m[r] > 0 ? r1[(long)s * g.nface + rc.face[r]] : (T)0;
    const T kap = (last ? (T)0 : kr) + lm;
    T num = kap * e + rc.gdot(btdu) - rc.gdot(c);
    if (!last) num -= r4[(long)(s + 1) * g.ncell + rc.cell] / dt;
    const T dpb = num / rc.gg;
    T* us = u + (long)s * g.nface;
#pragma unroll
    for (int r = 0; r < NS; ++r)
        if (rc.m[r] > 0) {
            vs[rc.face[r]] += omega * dv[r];
            us[rc.face[r]] += omega * du[r];
        }
    p[(long)s * g.ncell + rc.cell] += omega * dp;
    pb[(long)s * g.ncell + rc.cell] += omega * dpb;
}

template <typename T, int D>
__global__ void __launch_bounds__(256) k_rot_blk_apply(Grid g, int N, ColourSet cs, T dt, T kr, T lm, T omega,
                                                       T* __restrict__ v, T* __restrict__ pb, T* __restrict__ u,
                                                       T* __restrict__ p, const T* __restrict__ r1,
                                                       const T* __restrict__ r2, const T* __restrict__ r3,
                                                       const T* __restrict__ r4, const T* __restrict__ sc) {
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (long)cs.total * N) return;
    const int q = (int)(tid % cs.total), s = (int)(tid / cs.total);
    constexpr int REC = RotDims<D>::REC;
    rot_apply_item<T, D>(g, N, cs, q, s, dt, kr, lm, omega, v, pb, u, p, r1, r2, r3, r4,
                         rot_sc(sc, REC, 0, s, cs.total, q),
                         s > 0 ? rot_sc(sc, REC, 0, s - 1, cs.total, q) : (const T*)nullptr);
}

// Elimination of one cell whose records (slot s at rec + s * REC) are in LDS:
// W_{s-1}, t_{s-1} replace D_{s-1} and the right-hand side of slot s - 1, y_s
// replaces t_s.  Each step reads the next step's record before it writes its
// own results (two register buffers in turn), so the reads need not wait for
// the writes (the compiler cannot tell the two apart).
template <typename T, int D>
__device__ inline void rot_eliminate_local(T* rec, int N) {
    using RD = RotDims<D>;
    constexpr int K = RD::K, REC = RD::REC, USED = RD::USED;
    T S[K][K], z[K];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        z[a] = rec[RD::OR + a];
#pragma unroll
        for (int b = 0; b < K; ++b) S[a][b] = rec[RD::OD + a * K + b];
    }
    auto load = [&](int s, T (&o)[USED]) {
        const T* x = rec + (long)s * REC;
#pragma unroll
        for (int w = 0; w < USED; ++w) o[w] = x[w];
    };
    auto step = [&](int s, const T (&cur)[USED]) {
        T* prv = rec + (long)(s - 1) * REC;
        rot_elim_step<T, K>(S, z, cur, [&](int w, T x) { prv[w] = x; });
    };
    T ba[USED], bb[USED];
    if (N > 1) load(1, ba);
    for (int s = 1; s < N; s += 2) {
        if (s + 1 < N) load(s + 1, bb);
        step(s, ba);
        if (s + 1 >= N) break;
        if (s + 2 < N) load(s + 2, ba);
        step(s + 1, bb);
    }
    T y[K];
    rot_elim_last<T, K>(S, z, y);
    T* last = rec + (long)(N - 1) * REC;
#pragma unroll
    for (int a = 0; a < K; ++a) last[RD::OR + a] = y[a];
    constexpr int BW = K * K + K;       // W (at OD) and t (at OR) of one slot
    auto loadb = [&](int s, T (&o)[BW]) {
        const T* x = rec + (long)s * REC;
#pragma unroll
        for (int w = 0; w < K * K; ++w) o[w] = x[RD::OD + w];
#pragma unroll
        for (int w = 0; w < K; ++w) o[K * K + w] = x[RD::OR + w];
    };
    auto back = [&](int s, const T (&r)[BW]) {
        T yn[K];
#pragma unroll
        for (int a = 0; a < K; ++a) {
            T acc = r[K * K + a];
#pragma unroll
            for (int b = 0; b < K; ++b) acc -= r[a * K + b] * y[b];
            yn[a] = acc;
        }
        T* o = rec + (long)s * REC + RD::OR;
#pragma unroll
        for (int a = 0; a < K; ++a) {
            y[a] = yn[a];
            o[a] = y[a];
        }
    };
    T ca[BW], cb[BW];
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
template <typename T, int D>
__global__ void __launch_bounds__(512) k_rot_blk_fused(Grid g, int N, ColourSet cs, int TB, T dt, T kr, T lm, T omega,
                                                       T* __restrict__ v, T* __restrict__ pb, T* __restrict__ u,
                                                       T* __restrict__ p, const T* __restrict__ r1,
                                                       const T* __restrict__ r2, const T* __restrict__ r3,
                                                       const T* __restrict__ r4) {
    constexpr int REC = RotDims<D>::REC;
    extern __shared__ __align__(16) unsigned char rot_lds_raw[];
    T* lds = reinterpret_cast<T*>(rot_lds_raw);
    const int cstride = N * REC + 16 / (int)sizeof(T);     // per cell, padded off the bank stride
    const int c0 = blockIdx.x * TB;
    const int nc = min(TB, cs.total - c0);
    const int items = nc * N;
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
        const int cl = it % nc, s = it / nc;
        rot_setup_item<T, D>(g, N, cs, c0 + cl, s, dt, kr, lm, v, r1, r2, r3, r4, lds + (long)cl * cstride + s * REC);
    }
    __syncthreads();
    if ((int)threadIdx.x < nc) rot_eliminate_local<T, D>(lds + (long)threadIdx.x * cstride, N);
    __syncthreads();
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
        const int cl = it % nc, s = it / nc;
        const T* rec = lds + (long)cl * cstride + s * REC;
        rot_apply_item<T, D>(g, N, cs, c0 + cl, s, dt, kr, lm, omega, v, pb, u, p, r1, r2, r3, r4, rec,
                             s > 0 ? rec - REC : (const T*)nullptr);
    }
}

// Cells per block of the fused launch (records within 64 KB of LDS), 0 when
// one cell's records do not fit (the three-launch form then runs).
template <typename T, int D>
inline int rot_fused_cells(int N) {
    const long per = ((long)N * RotDims<D>::REC + 16 / (long)sizeof(T)) * (long)sizeof(T);
    return (int)std::min<long>(8, 65536 / per);
}

}  // namespace stfas
