// The rotational velocity operator of Sec. 3.1 eq:NSA on the 2D MAC grid:
// Adv[v] discretises (curl v) x v (the gradient part of (v . grad) v goes
// into the kinetic pressure).
//
//   node vorticity (cell corners, the circulation around the node's dual
//   cell; zero on the walls):  w_n = (v_y right - v_y left - v_x above + v_x below)/h
//   node sums:  Sx_n, Sy_n = the two incident x-faces, y-faces of node n
//   Adv_x(f) = -1/4 sum over the end nodes n of x-face f of w_n Sy_n
//   Adv_y(g) = +1/4 sum over the end nodes n of y-face g of w_n Sx_n
//
// Each (x-face, y-face) pair that meets at a node enters both components
// with the same weight and opposite signs, so sum_f v_f Adv_f(v) = 0: the
// operator does no work, as (curl v) x v does not.  Adv is bilinear in
// (w(v), v); the transpose of its Jacobian, J_Adv(v)^T y, is the gradient in
// v of <y, Adv[v]> = 1/4 sum_n w_n (Sx_n Yy_n - Sy_n Yx_n), again a stencil
// of node quantities.  Everything is evaluated per face from its two end
// nodes; wall faces carry nothing.
#pragma once
#include "common.hpp"

namespace stfas {

// v_x at x-face (I, j) and v_y at y-face (i, J); 0 outside the lattice.
template <typename T>
__device__ inline T rot_vx(const Grid& g, const T* f, int I, int j) {
    return (I >= 0 && I <= g.n[0] && j >= 0 && j < g.n[1]) ? f[face_index(g, 0, I, j, 0)] : (T)0;
}
template <typename T>
__device__ inline T rot_vy(const Grid& g, const T* f, int i, int J) {
    return (i >= 0 && i < g.n[0] && J >= 0 && J <= g.n[1]) ? f[face_index(g, 1, i, J, 0)] : (T)0;
}

// Node sums of a face field at node (I, J).  masked: wall faces count as 0.
template <typename T>
__device__ inline void rot_sums(const Grid& g, const T* f, int I, int J, bool masked, T& sx, T& sy) {
    const int n0 = g.n[0], n1 = g.n[1];
    const bool wx = masked && (I == 0 || I == n0);      // both incident x-faces lie on a wall column
    sx = (T)0;
    if (!wx) {
        if (J <= n1 - 1) sx += rot_vx(g, f, I, J);
        if (J >= 1) sx += rot_vx(g, f, I, J - 1);
    }
    const bool wy = masked && (J == 0 || J == n1);
    sy = (T)0;
    if (!wy) {
        if (I <= n0 - 1) sy += rot_vy(g, f, I, J);
        if (I >= 1) sy += rot_vy(g, f, I - 1, J);
    }
}

template <typename T>
__device__ inline T rot_vorticity(const Grid& g, const T* v, int I, int J, T ih) {
    if (I <= 0 || I >= g.n[0] || J <= 0 || J >= g.n[1]) return (T)0;
    return (rot_vy(g, v, I, J) - rot_vy(g, v, I - 1, J) - rot_vx(g, v, I, J) + rot_vx(g, v, I, J - 1)) * ih;
}

// The two end nodes of interior face (a, i, j): x-face (i, j) ends at nodes
// (i, j) and (i, j + 1); y-face (i, j) at nodes (i, j) and (i + 1, j).
__device__ inline void rot_ends(int a, int i, int j, int (&n)[2][2]) {
    n[0][0] = i;
    n[0][1] = j;
    n[1][0] = a == 0 ? i : i + 1;
    n[1][1] = a == 0 ? j + 1 : j;
}

// Adv[v] at interior face (a, i, j) (a 2D face; wall faces are the caller's).
template <typename T>
__device__ inline T rot_adv(const Grid& g, const T* v, int a, int i, int j, T ih) {
    int n[2][2];
    rot_ends(a, i, j, n);
    T acc[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        T sx, sy;
        rot_sums(g, v, n[e][0], n[e][1], false, sx, sy);
        acc[e] = rot_vorticity(g, v, n[e][0], n[e][1], ih) * (a == 0 ? sy : sx);
    }
    return a == 0 ? (T)-0.25 * (acc[0] + acc[1]) : (T)0.25 * (acc[0] + acc[1]);
}

// J_Adv(v)^T y at interior face (a, i, j); y is read with its wall faces as 0.
template <typename T>
__device__ inline T rot_adv_T(const Grid& g, const T* v, const T* y, int a, int i, int j, T ih) {
    int n[2][2];
    rot_ends(a, i, j, n);
    T P[2], wy[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int I = n[e][0], J = n[e][1];
        T sx, sy, yx, yy;
        rot_sums(g, v, I, J, false, sx, sy);
        rot_sums(g, y, I, J, true, yx, yy);
        const bool interior = I > 0 && I < g.n[0] && J > 0 && J < g.n[1];
        P[e] = interior ? (T)0.25 * (sx * yy - sy * yx) : (T)0;
        wy[e] = rot_vorticity(g, v, I, J, ih) * (a == 0 ? yy : yx);
    }
    // through the vorticity: an x-face enters w at its lower end node with -1/h and at its
    // upper one with +1/h; a y-face at its left end node with +1/h and at its right one with -1/h
    const T gw = a == 0 ? (P[1] - P[0]) * ih : (P[0] - P[1]) * ih;
    return a == 0 ? gw + (T)0.25 * (wy[0] + wy[1]) : gw - (T)0.25 * (wy[0] + wy[1]);
}

// One fixed-point step of the implicit update (v' - v)/dt + Adv[v'] = u - G p'
// before its projection: out = v + dt u - dt Adv[vk] on interior faces, 0 on
// walls (vk = null: without the Adv term, the first iterate).
template <typename T>
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
    if (vk) w -= dt * rot_adv<T>(g, vk, a, i, j, (T)(1.0 / g.h));
    out[f] = w;
}

}  // namespace stfas
