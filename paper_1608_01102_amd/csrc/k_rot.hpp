// The rotational velocity operator of Sec. 3.1 eq:NSA on the MAC grid:
// Adv[v] discretises (curl v) x v (the gradient part of (v . grad) v goes
// into the kinetic pressure), with the vorticity on the grid's edges (in 2D
// the edges along z are the grid nodes).  Adv is bilinear in (w(v), v); the
// transpose of its Jacobian, J_Adv(v)^T y, is the gradient in v of
// <y, Adv[v]>, again a stencil of edge quantities.  Everything is evaluated
// per face from the edges at its ends; wall faces carry nothing.
#pragma once
#include "common.hpp"

namespace stfas {

// The operator on the edges of a 2D or 3D grid.  For each cyclic triple
// of axes (c, p, q) = (z, x, y), (x, y, z), (y, z, x) (2D: the first only, the
// z-edges being the nodes) a c-edge sits at a p-node, a q-node and a c-cell
// (lattice coordinates e[3]) and carries the circulation
//   w_c = (D_p v_q - D_q v_p)/h (zero on walls) and the sums S_p, S_q of its
// two incident p-faces and q-faces; each incident p-face gains -1/4 w_c S_q and
// each incident q-face +1/4 w_c S_p: (curl v) x v, with every pair of faces
// meeting at an edge entering both components with opposite signs (no work).
// In 2D, with (c, p, q) = (z, x, y) only: node vorticity
// w_n = (v_y right - v_y left - v_x above + v_x below)/h, Adv_x(f) = -1/4 sum
// over the end nodes n of x-face f of w_n Sy_n, Adv_y(g) = +1/4 sum over the
// end nodes of y-face g of w_n Sx_n.
template <int D>
struct RotTriples;
template <>
struct RotTriples<2> {
    static constexpr int n = 1;
    static constexpr int t[1][3] = {{2, 0, 1}};
};
template <>
struct RotTriples<3> {
    static constexpr int n = 3;
    static constexpr int t[3][3] = {{2, 0, 1}, {0, 1, 2}, {1, 2, 0}};
};

// Face value of axis a at lattice coordinates x; 0 outside the lattice (and,
// masked, on wall faces).
template <typename T>
__device__ inline T rot_face(const Grid& g, const T* f, int a, const int (&x)[3], bool masked) {
    if (x[0] < 0 || x[1] < 0 || x[2] < 0 || x[0] >= face_ext(g, a, 0) || x[1] >= face_ext(g, a, 1) ||
        x[2] >= face_ext(g, a, 2))
        return (T)0;
    if (masked && !face_interior(g, a, x[0], x[1], x[2])) return (T)0;
    return f[face_index(g, a, x[0], x[1], x[2])];
}

// w (0 off the interior edges), S_p and S_q of face field f at the c-edge e of triple (c, p, q).
template <typename T>
__device__ inline bool rot_edge(const Grid& g, const T* f, int p, int q, const int (&e)[3], T ih, bool masked, T& w,
                                T& sp, T& sq) {
    int m[3] = {e[0], e[1], e[2]};
    const T vq1 = rot_face(g, f, q, m, masked), vp1 = rot_face(g, f, p, m, masked);
    m[p] -= 1;
    const T vq0 = rot_face(g, f, q, m, masked);
    m[p] += 1;
    m[q] -= 1;
    const T vp0 = rot_face(g, f, p, m, masked);
    sp = vp0 + vp1;
    sq = vq0 + vq1;
    const bool in = e[p] > 0 && e[p] < g.n[p] && e[q] > 0 && e[q] < g.n[q];
    w = in ? ((vq1 - vq0) - (vp1 - vp0)) * ih : (T)0;
    return in;
}

// Adv[v] at interior face (a, i, j, k) (wall faces are the caller's).
template <typename T, int D>
__device__ inline T rot_adv(const Grid& g, const T* v, int a, int i, int j, int k, T ih) {
    const int fx[3] = {i, j, k};
    T acc = 0;
#pragma unroll
    for (int t = 0; t < RotTriples<D>::n; ++t) {
        const int p = RotTriples<D>::t[t][1], q = RotTriples<D>::t[t][2];
        if (a != p && a != q) continue;
#pragma unroll
        for (int e2 = 0; e2 < 2; ++e2) {
            int e[3] = {fx[0], fx[1], fx[2]};
            e[a == p ? q : p] += e2;          // the two c-edges at the face's ends across the other axis
            T w, sp, sq;
            rot_edge(g, v, p, q, e, ih, false, w, sp, sq);
            acc += a == p ? (T)-0.25 * w * sq : (T)0.25 * w * sp;
        }
    }
    return acc;
}

// J_Adv(v)^T y at interior face (a, i, j, k): the gradient in v of
// <y, Adv[v]> = sum over interior edges of w_c (S_p Y_q - S_q Y_p)/4 (y read
// with its wall faces as 0).  A p-face enters w_c at the edges of its q-ends
// with -1/h (lower) and +1/h (upper) and S_p at both; a q-face enters w_c at
// the edges of its p-ends with +1/h (lower) and -1/h (upper) and S_q at both.
template <typename T, int D>
__device__ inline T rot_adv_T(const Grid& g, const T* v, const T* y, int a, int i, int j, int k, T ih) {
    const int fx[3] = {i, j, k};
    T acc = 0;
#pragma unroll
    for (int t = 0; t < RotTriples<D>::n; ++t) {
        const int p = RotTriples<D>::t[t][1], q = RotTriples<D>::t[t][2];
        if (a != p && a != q) continue;
        T P[2], ws[2];
#pragma unroll
        for (int e2 = 0; e2 < 2; ++e2) {
            int e[3] = {fx[0], fx[1], fx[2]};
            e[a == p ? q : p] += e2;
            T w, sp, sq, wy, yp, yq;
            const bool in = rot_edge(g, v, p, q, e, ih, false, w, sp, sq);
            rot_edge(g, y, p, q, e, ih, true, wy, yp, yq);
            P[e2] = in ? (T)0.25 * (sp * yq - sq * yp) : (T)0;
            ws[e2] = a == p ? w * yq : w * yp;
        }
        acc += a == p ? (P[1] - P[0]) * ih + (T)0.25 * (ws[0] + ws[1])
                      : (P[0] - P[1]) * ih - (T)0.25 * (ws[0] + ws[1]);
    }
    return acc;
}

// One fixed-point step of the implicit update (v' - v)/dt + Adv[v'] = u - G p'
// before its projection: out = v + dt u - dt Adv[vk] on interior faces, 0 on
// walls (vk = null: without the Adv term, the first iterate).
template <typename T, int D>
__global__ void k_rot_rhs(Grid g, T dt, const T* __restrict__ v, const T* __restrict__ u, const T* __restrict__ vk,
                          T* __restrict__ out) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= g.nface) return;
    int a, i, j, k;
    face_decode(g, f, a, i, j, k);
    if (!face_interior(g, a, i, j, k)) {
        out[f] = (T)0;
        return;
    }
    T w = v[f] + dt * u[f];
    if (vk) w -= dt * rot_adv<T, D>(g, vk, a, i, j, k, (T)(1.0 / g.h));
    out[f] = w;
}

// One step of the adjoint of the fixed-point steps: out = -dt J_Adv(y)^T x
// on interior faces (y = null: out = x there), 0 on walls.
template <typename T, int D>
__global__ void k_rot_adj(Grid g, T dt, const T* __restrict__ y, const T* __restrict__ x, T* __restrict__ out) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= g.nface) return;
    int a, i, j, k;
    face_decode(g, f, a, i, j, k);
    if (!face_interior(g, a, i, j, k)) {
        out[f] = (T)0;
        return;
    }
    out[f] = y ? -dt * rot_adv_T<T, D>(g, y, x, a, i, j, k, (T)(1.0 / g.h)) : x[f];
}

}  // namespace stfas
