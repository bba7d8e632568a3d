// Host driver of the solver: workspace layout, the multigrid projection,
// the FAS V-cycle and velocity subproblem, the density subproblem, the ADMM
// outer loop and the re-simulated outputs.  Every device step is a kernel of
// this library launched on the context's stream; the host only sequences
// them and reads back the scalars the stop tests need.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <vector>

#include "../../include/stfas.h"
#include "../../include/stfas_ops.h"
#include "common.hpp"
#include "k_advect.hpp"
#include "k_kkt.hpp"
#include "k_misc.hpp"
#include "k_poisson.hpp"
#include "k_rot_scgs.hpp"
#include "k_upwind.hpp"

namespace stfas {

constexpr int BS = 256;
constexpr int RED_BLOCKS = 512;
constexpr int MAX_COARSE_CELLS = 4096;
constexpr int MAX_PROJECT_CYCLES = 60;
constexpr long DIRECT_T_SLOTS = 131072;   // face slots up to which the residual's transpose runs untiled
constexpr int ROT_PICARD = 4;             // fixed-point steps of the rotational operator's implicit update


// Bump allocator with a planning pass: plan() sizes every buffer, carve()
// hands out the same offsets inside one allocation.
struct Arena {
    char* base = nullptr;
    size_t off = 0;
    template <typename U>
    U* take(size_t count) {
        const size_t bytes = ((count * sizeof(U)) + 255) & ~size_t(255);
        U* p = base ? reinterpret_cast<U*>(base + off) : nullptr;
        off += bytes;
        return p;
    }
};

// Resolved problem constants (defaults of stfas.h applied).
struct Params {
    int dim, n[3], N;
    double dt, r, K, beta, eps_stfas, eps_admm, poisson_rtol, omega, al_tol, lm;
    int ao_iters, max_admm, max_vcycles, metric_levels, fixed_counts, precision, density;
    int vort;   // 1: the rotational velocity operator (eq:NSA's Adv)
    int rot_exact;   // levels (from the finest) whose smoother's local matrix holds the cell's block of dAdv/dv
};

inline int default_metric_levels(const int* n, int dim) {
    int m = n[0];
    for (int a = 1; a < dim; ++a) m = std::min(m, n[a]);
    int L = 0;
    while (std::ldexp(1.0, L) <= m / 8.0) ++L;
    return L;
}

inline bool resolve(const stfas_problem* p, Params& o) {
    if (!p) return false;
    if (p->dim != 2 && p->dim != 3) return false;
    o.dim = p->dim;
    for (int a = 0; a < 3; ++a) o.n[a] = a < p->dim ? p->n[a] : 1;
    for (int a = 0; a < o.dim; ++a)
        if (o.n[a] < 4 || o.n[a] > (1 << 14)) return false;
    if (o.dim == 2 && p->n[2] > 1) return false;
    // the SCGS recurrence stages 3 * 2N temporal factors in 64 KB of LDS
    if (p->num_steps < 1 || p->num_steps > 1024) return false;
    if (!(p->r > 0) || !std::isfinite(p->r)) return false;
    if (p->precision != STFAS_FP64 && p->precision != STFAS_MIXED) return false;
    o.N = p->num_steps;
    o.dt = p->dt > 0 ? p->dt : 1.0 / o.n[0];
    o.r = p->r;
    o.K = p->K > 0 ? p->K : o.r / (o.dt * o.dt);
    o.beta = p->beta > 0 ? p->beta : 1.0;
    o.ao_iters = p->ao_iters > 0 ? p->ao_iters : 2;
    o.eps_stfas = p->eps_stfas > 0 ? p->eps_stfas : 1e-5;
    o.eps_admm = p->eps_admm;   // <= 0: max(rho0)/100, fixed at solve time
    o.max_admm = p->max_admm > 0 ? p->max_admm : 50;
    o.max_vcycles = p->max_vcycles > 0 ? p->max_vcycles : 30;
    o.metric_levels = p->metric_levels >= 0 ? p->metric_levels : default_metric_levels(o.n, o.dim);
    o.precision = p->precision;
    o.poisson_rtol = p->poisson_rtol > 0 ? p->poisson_rtol : (o.precision == STFAS_FP64 ? 1e-13 : 1e-6);
    o.fixed_counts = p->fixed_counts ? 1 : 0;
    if (p->velocity_op != STFAS_VELOCITY_SL && p->velocity_op != STFAS_VELOCITY_ROTATIONAL) return false;
    o.vort = p->velocity_op == STFAS_VELOCITY_ROTATIONAL ? 1 : 0;
    // the local block of dAdv/dv: by default on the finest level in 2D and on
    // none in 3D (where it saves no V-cycles and costs a serial elimination)
    if (p->scgs_local != 0 && !(o.vort && p->scgs_local >= 1 && p->scgs_local <= 3)) return false;
    o.rot_exact = !o.vort ? 0
                          : p->scgs_local == 0 ? (o.dim == 2 ? 1 : 0)
                                               : p->scgs_local == 1 ? 0 : (p->scgs_local == 2 ? 1 << 20 : 1);
    // the rotational operator's smoother: no relaxation, and no perturbation
    // where its finest level holds the local block (without it the
    // perturbation stays)
    o.omega = p->scgs_omega > 0 ? p->scgs_omega : (o.vort ? 1.0 : 0.7);
    if (!(o.omega <= 2.0)) return false;
    if (p->density_op != STFAS_DENSITY_SL && p->density_op != STFAS_DENSITY_UPWIND) return false;
    o.density = p->density_op;
    if (!(p->al_tol >= 0) || !std::isfinite(p->al_tol)) return false;
    o.al_tol = p->al_tol;
    if (std::isnan(p->scgs_lm) || std::isinf(p->scgs_lm)) return false;
    o.lm = (p->scgs_lm < 0 ? 0.0 : (p->scgs_lm > 0 ? p->scgs_lm : (o.rot_exact > 0 ? 0.0 : 1.0))) / (o.dt * o.dt);
    const double total = (double)o.n[0] * o.n[1] * o.n[2];
    if (total > 2.0e9 / (o.dim + 1)) return false;
    return true;
}

// STFAS levels: coarsen every axis by 2 while every n_a / 2^l >= 4.
inline std::vector<Grid> stfas_levels(const Grid& g0) {
    std::vector<Grid> v{g0};
    for (;;) {
        const Grid& g = v.back();
        bool ok = true;
        for (int a = 0; a < g.dim; ++a) ok = ok && (g.n[a] % 2 == 0) && (g.n[a] / 2 >= 4);
        if (!ok) break;
        v.push_back(coarse_grid(g));
    }
    return v;
}

// Poisson levels: coarsen while every n_a is even and n_a / 2 >= 2.
inline std::vector<Grid> poisson_levels(const Grid& g0) {
    std::vector<Grid> v{g0};
    for (;;) {
        const Grid& g = v.back();
        bool ok = true;
        for (int a = 0; a < g.dim; ++a) ok = ok && (g.n[a] % 2 == 0) && (g.n[a] / 2 >= 2);
        if (!ok) break;
        v.push_back(coarse_grid(g));
    }
    return v;
}

// Pseudo-inverse of the Neumann Laplacian of a small grid, row-major m x m:
// pinv = (L - 11^T/m)^-1 + 11^T/m (the constant is L's only null vector).
inline void coarse_pinv(const Grid& g, std::vector<double>& out) {
    const int m = g.ncell;
    std::vector<double> A((size_t)m * m, 0.0), I((size_t)m * m, 0.0);
    const double ih2 = 1.0 / (g.h * g.h);
    for (int k = 0; k < g.n[2]; ++k)
        for (int j = 0; j < g.n[1]; ++j)
            for (int i = 0; i < g.n[0]; ++i) {
                const int c = cell_index(g, i, j, k);
                const int nb[6][3] = {{i - 1, j, k}, {i + 1, j, k}, {i, j - 1, k}, {i, j + 1, k}, {i, j, k - 1}, {i, j, k + 1}};
                for (int q = 0; q < 6; ++q) {
                    const int a = nb[q][0], b = nb[q][1], cc = nb[q][2];
                    if (a < 0 || a >= g.n[0] || b < 0 || b >= g.n[1] || cc < 0 || cc >= g.n[2]) continue;
                    A[(size_t)c * m + cell_index(g, a, b, cc)] += ih2;
                    A[(size_t)c * m + c] -= ih2;
                }
            }
    for (size_t e = 0; e < A.size(); ++e) A[e] -= 1.0 / m;
    for (int d = 0; d < m; ++d) I[(size_t)d * m + d] = 1.0;
    // Gauss-Jordan with partial pivoting
    for (int col = 0; col < m; ++col) {
        int piv = col;
        for (int r = col + 1; r < m; ++r)
            if (std::fabs(A[(size_t)r * m + col]) > std::fabs(A[(size_t)piv * m + col])) piv = r;
        if (piv != col)
            for (int q = 0; q < m; ++q) {
                std::swap(A[(size_t)piv * m + q], A[(size_t)col * m + q]);
                std::swap(I[(size_t)piv * m + q], I[(size_t)col * m + q]);
            }
        const double inv = 1.0 / A[(size_t)col * m + col];
        for (int q = 0; q < m; ++q) {
            A[(size_t)col * m + q] *= inv;
            I[(size_t)col * m + q] *= inv;
        }
        for (int r = 0; r < m; ++r) {
            if (r == col) continue;
            const double f = A[(size_t)r * m + col];
            if (f == 0.0) continue;
            for (int q = 0; q < m; ++q) {
                A[(size_t)r * m + q] -= f * A[(size_t)col * m + q];
                I[(size_t)r * m + q] -= f * I[(size_t)col * m + q];
            }
        }
    }
    out.assign((size_t)m * m, 0.0);
    for (size_t e = 0; e < out.size(); ++e) out[e] = I[e] + 1.0 / m;
}

// Normalised Gaussian taps exp(-t^2 / (2 sigma^2)), t = -R..R, R = ceil(3 sigma).
inline std::vector<double> gauss_taps(double sigma) {
    const int R = (int)std::ceil(3.0 * sigma);
    std::vector<double> k(2 * R + 1);
    double s = 0;
    for (int t = -R; t <= R; ++t) s += (k[t + R] = std::exp(-(double)t * t / (2.0 * sigma * sigma)));
    for (auto& x : k) x /= s;
    return k;
}

// Thomas factors of the temporal matrix of the SCGS local system (blocks
// u_0, v_1, u_1, ..., v_N): diagonal -1 (u), K/r (v_i, i<N), 0 (v_N);
// T(u_{i-1}, v_i) = 1/dt, T(v_i, u_i) = -1/dt.
struct TFactors {
    std::vector<double> diag, sub, sup, cp, inv;
};

// The temporal matrix of the smoother's local system (collapsed form) and its
// Thomas factors.  kr = K/r; mu = the Levenberg-Marquardt perturbation of K/r
// on every v block (Sec. 5, convergence analysis).
inline TFactors temporal_factors(int N, double dt, double kr, double mu) {
    TFactors f;
    const int M = 2 * N;
    f.diag.resize(M);
    f.sub.assign(M, 0.0);
    f.sup.assign(M, 0.0);
    f.cp.assign(M, 0.0);
    f.inv.resize(M);
    for (int k = 0; k < M; ++k) {
        f.diag[k] = (k % 2 == 0) ? -1.0 : (((k + 1) / 2 < N) ? kr : 0.0) + mu;
        if (k + 1 < M) f.sup[k] = (k % 2 == 0) ? 1.0 / dt : -1.0 / dt;
        if (k > 0) f.sub[k] = f.sup[k - 1];
    }
    double cprev = 0;
    for (int k = 0; k < M; ++k) {
        const double den = f.diag[k] - f.sub[k] * cprev;
        f.inv[k] = 1.0 / den;
        f.cp[k] = f.sup[k] * f.inv[k];
        cprev = f.cp[k];
    }
    return f;
}

// Multigrid projection Q for B independent slices (Sec. 4.1).
template <typename T, int D>
struct Poisson {
    std::vector<Grid> PG;
    std::vector<T*> phi, b;
    double* pinv = nullptr;
    double* pool = nullptr;   // per-slice residual partials
    double* out = nullptr;    // 8 doubles of reduction results
    int Bmax = 1;
    hipStream_t st = nullptr;

    // single-launch projection in LDS (one workgroup per slice), when the
    // hierarchy fits: at least two levels, a coarsest level of <= 256 cells,
    // <= 16384 finest cells (16 per thread in registers) and LDS for every
    // level's phi and every coarse level's right-hand side
    PLevels plv{};
    size_t lds_bytes = 0;
    int lds_cpt = 0;
    int* cyc_dev = nullptr;

    void init(const Grid& g0, int bmax, hipStream_t s) {
        PG = poisson_levels(g0);
        Bmax = bmax;
        st = s;
        lds_cpt = 0;
        lds_checked = false;
        const int nl = (int)PG.size();
        if (nl < 2 || nl > PL_MAX || PG.back().ncell > 256 || g0.ncell > 16 * 1024) return;
        size_t off = 0;
        for (int l = 0; l < nl; ++l) {
            plv.g[l] = PG[l];
            plv.dx[l] = make_fastdiv((unsigned)PG[l].n[0]);
            plv.dy[l] = make_fastdiv((unsigned)PG[l].n[1]);
            plv.dh[l] = make_fastdiv((unsigned)((PG[l].n[0] + 1) / 2));
            plv.off_phi[l] = (int)off;
            off += PG[l].ncell;
            plv.off_b[l] = l == 0 ? -1 : (int)off;
            if (l > 0) off += PG[l].ncell;
        }
        plv.n = nl;
        plv.coarse_m = PG.back().ncell;
        lds_bytes = 256 + off * sizeof(T);
        lds_cpt = g0.ncell <= 2048 ? 2 : (g0.ncell <= 4096 ? 4 : (g0.ncell <= 8192 ? 8 : 16));
    }
    // first use on the device: keep the LDS path only if the device allows
    // that much LDS per workgroup
    bool lds_checked = false;
    void check_lds() {
        lds_checked = true;
        if (lds_cpt == 0) return;
        int dev = 0, maxlds = 0;
        HCK(hipGetDevice(&dev));
        HCK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        if (lds_bytes + sizeof(PLevels) > (size_t)maxlds) {
            lds_cpt = 0;
            return;
        }
        set_lds_attr();
    }
    void set_lds_attr() {
        switch (lds_cpt) {
            case 2: HCK(hipFuncSetAttribute((const void*)k_project_lds<T, D, 2>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes)); break;
            case 4: HCK(hipFuncSetAttribute((const void*)k_project_lds<T, D, 4>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes)); break;
            case 8: HCK(hipFuncSetAttribute((const void*)k_project_lds<T, D, 8>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes)); break;
            case 16: HCK(hipFuncSetAttribute((const void*)k_project_lds<T, D, 16>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes)); break;
            default: break;
        }
    }
    void launch_lds(const T* w, T* o, T* phi_out, int B, double rtol, int fixed) {
        const long F = PG[0].nface, C = PG[0].ncell;
        switch (lds_cpt) {
#define STFAS_PLDS(CC)                                                                                           \
    case CC:                                                                                                     \
        k_project_lds<T, D, CC><<<B, 1024, lds_bytes, st>>>(plv, pinv, w, o, phi_out, b[0], rtol, fixed,         \
                                                            MAX_PROJECT_CYCLES, cyc_dev, F, C);                  \
        break;
            STFAS_PLDS(2)
            STFAS_PLDS(4)
            STFAS_PLDS(8)
            STFAS_PLDS(16)
#undef STFAS_PLDS
            default: break;
        }
    }
    bool coarse_ok() const { return PG.back().ncell <= MAX_COARSE_CELLS; }
    void layout(Arena& A, double* shared_pinv) {
        phi.assign(PG.size(), nullptr);
        b.assign(PG.size(), nullptr);
        for (size_t l = 0; l < PG.size(); ++l) {
            phi[l] = A.take<T>((size_t)Bmax * PG[l].ncell);
            b[l] = A.take<T>((size_t)Bmax * PG[l].ncell);
        }
        pinv = shared_pinv ? shared_pinv : A.take<double>((size_t)PG.back().ncell * PG.back().ncell);
        pool = A.take<double>((size_t)Bmax * RED_BLOCKS * 2);
        out = A.take<double>(8);
        cyc_dev = A.take<int>(64);
    }
    void upload_pinv() {
        std::vector<double> pv;
        coarse_pinv(PG.back(), pv);
        HCK(hipMemcpyAsync(pinv, pv.data(), pv.size() * sizeof(double), hipMemcpyHostToDevice, st));
        HCK(hipStreamSynchronize(st));
    }

    void vcycle(int l, int B) {
        const Grid& g = PG[l];
        const long C = g.ncell;
        if (l == (int)PG.size() - 1) {
            k_coarse_solve<T><<<B, BS, C * sizeof(double), st>>>((int)C, pinv, b[l], phi[l], C);
            return;
        }
        const int half = (g.n[0] + 1) / 2 * g.n[1] * g.n[2];
        const dim3 gr(blocks_for(half, BS), B);
        for (int s = 0; s < 2; ++s) {
            k_rbgs<T, D><<<gr, BS, 0, st>>>(g, phi[l], b[l], 0, C);
            k_rbgs<T, D><<<gr, BS, 0, st>>>(g, phi[l], b[l], 1, C);
        }
        const Grid& gc = PG[l + 1];
        k_resid_restrict<T, D><<<dim3(blocks_for(gc.ncell, BS), B), BS, 0, st>>>(g, gc, phi[l], b[l], b[l + 1], C,
                                                                                gc.ncell);
        k_fill<T><<<blocks_for((long)B * gc.ncell, BS), BS, 0, st>>>((long)B * gc.ncell, phi[l + 1], (T)0);
        vcycle(l + 1, B);
        k_prolong_add<T, D><<<dim3(blocks_for(C, BS), B), BS, 0, st>>>(g, gc, phi[l + 1], phi[l], C, gc.ncell);
        for (int s = 0; s < 2; ++s) {
            k_rbgs<T, D><<<gr, BS, 0, st>>>(g, phi[l], b[l], 1, C);
            k_rbgs<T, D><<<gr, BS, 0, st>>>(g, phi[l], b[l], 0, C);
        }
    }

    // max over slices of |b - L phi| / |b| (synchronises; host mirror given).
    double ratio(int B, double* host) {
        const Grid& g = PG[0];
        const int nb = std::min(RED_BLOCKS, blocks_for(g.ncell, BS));
        k_poisson_resid_norm<T, D><<<dim3(nb, B), BS, 0, st>>>(g, phi[0], b[0], pool, g.ncell);
        k_poisson_ratio<<<1, BS, 0, st>>>(B, nb, pool, out, 0);
        HCK(hipMemcpyAsync(host, out, sizeof(double), hipMemcpyDeviceToHost, st));
        HCK(hipStreamSynchronize(st));
        return host[0];
    }

    // out = Q w for B slices (out may alias w).  fixed > 0: exactly that many
    // cycles and no host synchronisation; otherwise cycles until the
    // relative residual of every slice is <= rtol.  Returns the cycle count.
    // With the LDS kernel the cycle count is per slice and decided on the
    // device; it is read back (synchronising) only when `count` is set, else
    // -1 is returned.
    int project(const T* w, T* o, T* phi_out, int B, double rtol, int fixed, double* host, bool count = true) {
        const Grid& g = PG[0];
        const long C = g.ncell;
        if (!lds_checked) check_lds();
        if (lds_cpt > 0) {
            const bool want = count && fixed <= 0;
            if (want) k_fill<int><<<1, 64, 0, st>>>(1, cyc_dev, 0);
            launch_lds(w, o, phi_out, B, rtol, fixed);
            if (fixed > 0) return fixed;
            if (!want) return -1;
            int c = 0;
            HCK(hipMemcpyAsync(&c, cyc_dev, sizeof(int), hipMemcpyDeviceToHost, st));
            HCK(hipStreamSynchronize(st));
            return c;
        }
        k_divergence<T, D><<<dim3(blocks_for(C, BS), B), BS, 0, st>>>(g, w, b[0], g.nface, C);
        k_fill<T><<<blocks_for((long)B * C, BS), BS, 0, st>>>((long)B * C, phi[0], (T)0);
        int cycles = 0;
        double prev = 0;
        for (;;) {
            vcycle(0, B);
            ++cycles;
            if (fixed > 0) {
                if (cycles >= fixed) break;
                continue;
            }
            if (cycles >= MAX_PROJECT_CYCLES) break;
            const double r = ratio(B, host);
            if (!std::isfinite(r) || r <= rtol) break;
            if (cycles >= 2 && r > PROJECT_STALL * prev) break;    // at the rounding floor
            prev = r;
        }
        k_project_apply<T, D><<<dim3(blocks_for(g.nface, BS), B), BS, 0, st>>>(g, w, phi[0], o, g.nface, C);
        if (phi_out) {
            k_slice_sum<T><<<B, BS, 0, st>>>((int)C, phi[0], pool, C);
            k_sub_mean<T><<<dim3(blocks_for(C, BS), B), BS, 0, st>>>((int)C, phi[0], pool, C);
            HCK(hipMemcpyAsync(phi_out, phi[0], (size_t)B * C * sizeof(T), hipMemcpyDeviceToDevice, st));
        }
        return cycles;
    }
};

// Pinned host buffer for scalar readbacks, one per host thread, kept for the
// life of the process (freeing pinned memory would synchronise the device).
inline double* thread_pinned() {
    thread_local double* buf = nullptr;
    if (!buf) HCK(hipHostMalloc((void**)&buf, 64 * sizeof(double), hipHostMallocDefault));
    return buf;
}

class SolverBase {
public:
    virtual ~SolverBase() {}
    Params P;
    hipStream_t st = nullptr;
    size_t bytes = 0;
    char* mem = nullptr;
    bool owns_mem = true;
    virtual size_t plan() = 0;
    virtual bool valid() const = 0;
    virtual void carve(char* base) = 0;
    virtual void init_tables() = 0;
    virtual stfas_status solve(const void*, int, const int*, const void*, void*, stfas_stats*) = 0;
    virtual int nlevels() const = 0;
    virtual const Grid& level(int l) const = 0;
    virtual void op_advect(int, const void*, const void*, void*) = 0;
    virtual void op_advect_T(int, const void*, const void*, const void*, void*) = 0;
    virtual void op_advect_dv_T(int, const void*, const void*, const void*, const void*, double, void*) = 0;
    virtual void op_self_advect(int, int, const void*, const void*, void*) = 0;
    virtual void op_self_advect_T(int, int, const void*, const void*, double, void*) = 0;
    virtual int op_project(int, const void*, void*, void*) = 0;
    virtual void op_metric(const void*, void*) = 0;
    virtual void op_kkt(int, stfas_state, const void*, stfas_state, stfas_state) = 0;
    virtual void op_sweep(int, stfas_state, const void*, stfas_state) = 0;
    virtual void op_restrict(int, stfas_state, stfas_state) = 0;
    virtual void op_prolong(int, stfas_state, double, stfas_state) = 0;
    virtual int op_nso(stfas_state, const void*, double*) = 0;
    virtual void op_ao(const void*, int, const int*, const void*, const void*, void*, void*, double*) = 0;
    virtual int lbfgs(const void*, int, const int*, const void*, void*, int, double, double*) = 0;
    virtual bool has_upwind() const = 0;
    virtual int op_upwind(const void*, const void*, void*) = 0;
    virtual void op_upwind_adj(const void*, const void*, const void*, void*, void*) = 0;
    Tracer tr;
    void trace_enable(int kind, int cap) {
        tr.reset();
        if (kind == TR_NONE || cap <= 0) return;
        tr.ev.resize(2 * (size_t)cap);
        for (auto& e : tr.ev) HCK(hipEventCreate(&e));
        tr.id = kind;
        tr.cap = cap;
    }
    // launches, total milliseconds, the method's and the implementation's bytes of the recorded launches
    void trace_read(long* n, double* ms, double* bytes, double* impl_bytes) {
        double tot = 0;
        for (int q = 0; q < tr.used; ++q) {
            HCK(hipEventSynchronize(tr.ev[2 * q + 1]));
            float t = 0;
            HCK(hipEventElapsedTime(&t, tr.ev[2 * q], tr.ev[2 * q + 1]));
            tot += t;
        }
        *n = tr.launches;
        *ms = tot;
        *bytes = tr.bytes;
        if (impl_bytes) *impl_bytes = tr.impl_bytes;
    }
};

// Launch shape of the whole-colour SCGS kernel for 2N = M blocks and `cells`
// cells of the colour: G lanes per cell (a power of two <= 64), chunks of L
// blocks (even), unrolled to CH >= L.  The longest chunk is bounded by the
// registers a lane holds (2d face values per block).  Measured on 128x128
// x 40: the finest colour (4096 cells) runs in 18 us with 8 lanes per cell,
// 20 us with 16 and 29 us with 64; the 64x64 colour prefers 64 lanes.
// Returns false when 2N does not fit in 64 chunks (the two-kernel path).
template <typename T, int D>
inline bool colour_shape(int M, long cells, int& G, int& L, int& CH) {
    const int chmax = (sizeof(T) == 4 && D == 2) ? 16 : 8;
    G = 1;
    while (G < 64 && (M + G - 1) / G > chmax) G <<= 1;
    if ((M + G - 1) / G > chmax) return false;
    // large colours are throughput-bound: as few lanes per cell as the
    // registers allow; small ones are latency-bound: up to 64 lanes per cell
    if (cells < 4096)
        while (G < 64 && (M + 2 * G - 1) / (2 * G) >= 2) G <<= 1;
    else    // row layout: chunks short enough for its register budget (see launch_scgs_colour)
        while (G < 16 && (M + G - 1) / G > (sizeof(T) == 8 ? 4 : 8)) G <<= 1;
    L = (M + G - 1) / G;
    L += L & 1;
    while (G > 1 && (long)(G / 2) * L >= M) G >>= 1;
    CH = L <= 2 ? 2 : (L + 3) & ~3;
    return CH <= chmax;
}

template <typename T, int D>
inline void launch_scgs_colour(int G, int L, int CH, const Grid& g, int N, const ColourSet& cs, const T* r1,
                               const T* t1, const T* r2, const T* r3, const T* r4, T* v, T* pb, T* u, T* p,
                               const T* tdiag, const T* tsub, const T* tsup, const T* tcp, const T* tinv, T omega,
                               hipStream_t st) {
    constexpr int CHMAX = (sizeof(T) == 4 && D == 2) ? 16 : 8;
    // row-layout chunk lengths that fit the 256 registers of a 512-thread workgroup without spilling
    constexpr int RMAX = sizeof(T) == 8 ? 4 : (D == 3 ? 8 : 12);
    if (cs.total >= 4096 && G <= 16 && CH <= RMAX) {
        // large colours: row layout, 512 threads = G chunks x (512 / G) neighbouring cells
        constexpr int NT = 512;
#define STFAS_ROWS_CASE(GG, CC)                                                                                  \
    if constexpr (CC <= RMAX)                                                                                    \
        if (G == GG && CH == CC) {                                                                               \
            constexpr int CPW = NT / GG > 64 ? 64 : NT / GG;                                                     \
            k_scgs_colour_rows<T, D, GG, CC, CPW><<<(cs.total + CPW - 1) / CPW, CPW * GG, 0, st>>>(             \
                g, N, L, cs, r1, t1, r2, r3, r4, v, pb, u, p, tdiag, tsub, tsup, tcp, tinv, omega);              \
            return;                                                                                              \
        }
#define STFAS_ROWS_G(GG)                                                                                         \
    STFAS_ROWS_CASE(GG, 2) STFAS_ROWS_CASE(GG, 4) STFAS_ROWS_CASE(GG, 8) STFAS_ROWS_CASE(GG, 12)
        STFAS_ROWS_G(1)
        STFAS_ROWS_G(2)
        STFAS_ROWS_G(4)
        STFAS_ROWS_G(8)
        STFAS_ROWS_G(16)
#undef STFAS_ROWS_G
#undef STFAS_ROWS_CASE
    }
    const long threads = (long)cs.total * G;
    const int blocks = (int)((threads + 255) / 256);
#define STFAS_COLOUR_CASE(GG, CC)                                                                                \
    if constexpr (CC <= CHMAX)                                                                                   \
        if (G == GG && CH == CC)                                                                                 \
            k_scgs_colour<T, D, GG, CC><<<blocks, 256, 0, st>>>(g, N, L, cs, r1, t1, r2, r3, r4, v, pb, u, p,     \
                                                                tdiag, tsub, tsup, tcp, tinv, omega);
#define STFAS_COLOUR_G(GG)                                                                                       \
    STFAS_COLOUR_CASE(GG, 2) STFAS_COLOUR_CASE(GG, 4) STFAS_COLOUR_CASE(GG, 8) STFAS_COLOUR_CASE(GG, 12)          \
    STFAS_COLOUR_CASE(GG, 16)
    STFAS_COLOUR_G(1)
    STFAS_COLOUR_G(2)
    STFAS_COLOUR_G(4)
    STFAS_COLOUR_G(8)
    STFAS_COLOUR_G(16)
    STFAS_COLOUR_G(32)
    STFAS_COLOUR_G(64)
#undef STFAS_COLOUR_G
#undef STFAS_COLOUR_CASE
}

// out[b] += scale J_S(v[b])^T y[b] for `batch` slices (tiled scatter).
template <typename T, int D>
inline void launch_self_advect_T(const Grid& g, T cfl, const T* v, const T* y, T scale, T* out, int batch,
                                 hipStream_t st) {
    using TS = TileShape<D>;
    int tiles = 0;
    for (int a = 0; a < D; ++a) {
        const int ex = face_ext(g, a, 0), ey = face_ext(g, a, 1), ez = face_ext(g, a, 2);
        const int t = ((ex + TS::X - 1) / TS::X) * ((ey + TS::Y - 1) / TS::Y) * (D == 3 ? (ez + TS::Z - 1) / TS::Z : 1);
        tiles = std::max(tiles, t);
    }
    if ((long)batch * g.nface <= DIRECT_T_SLOTS) {
        k_self_advect_T_direct<T, D><<<dim3(blocks_for(g.nface, 256), batch), 256, 0, st>>>(g, cfl, v, y, scale, out,
                                                                                        g.nface);
        return;
    }
    // blocks whose tile lies beyond a smaller lattice exit after the (empty) flush
    k_self_advect_T_tiled<T, D><<<dim3(tiles, batch, D), 256, 0, st>>>(g, cfl, v, y, scale, out, g.nface);
}

template <typename T, int D>
class Solver : public SolverBase {
public:
    // ---- levels and constant tables
    std::vector<Grid> L;      // STFAS levels
    int N = 0;
    // STFAS per-level buffers
    struct Lev {
        T *v, *pb, *u, *p;       // state
        T *r1, *r2, *r3, *r4;    // residual
        T *s1, *s2, *s3, *s4;    // FAS right-hand side (unused on level 0)
        T* w;                    // targets
    };
    std::vector<Lev> lev;
    T* scgs_scratch = nullptr;   // two-kernel SCGS path only (horizons too long for the fused kernel)
    T* rot_scratch = nullptr;    // rotational operator: the local records of one colour (three-launch form)
    T *t1a = nullptr, *t1b = nullptr;   // J_S^T part of F1 for the SCGS colour passes (any level)
    T *t1_zero = nullptr, *t1_used = nullptr;   // t1a / t1b: the one that is all zero, the other
    T* tq = nullptr;                            // quarters of the 3D sweep transpose (k_quarter_gather)
    T *t_diag, *t_sub, *t_sup, *t_cp, *t_inv;
    Poisson<T, D> pois;      // projection, batched over up to N slices
    // density subproblem
    T *rho, *rho_t, *mu, *vt, *vstar, *cand, *trial;
    T *ce_e, *ce_acc, *ce_t1, *ce_t2;
    T* taps = nullptr;
    std::vector<int> tap_off, tap_R;
    // ADMM
    T *lam, *rho_last, *wt;
    // re-simulation
    T *rs_rho[2], *rs_v[2], *rs_w;
    // upwind exponential density operator (only when selected)
    UpwindExp<T, D> up;
    bool upwind() const { return P.density == STFAS_DENSITY_UPWIND; }
    int *up_kd = nullptr, *up_okd = nullptr;      // per step: k and "stopped" of the last sweep (device)
    std::vector<int> up_pred;                     // launches per step predicted from the previous sweep
    std::vector<int> k_rho, k_rho_t, lb_k;        // k per step of the trajectories in rho, rho_t, lb_rho
    // reductions
    double *red_part, *red_out;
    double* host_out = nullptr;   // pinned mirror of red_out

    explicit Solver(const Params& p, hipStream_t s) {
        P = p;
        st = s;
        N = p.N;
        const int n[3] = {p.n[0], p.n[1], p.n[2]};
        Grid g0 = make_grid(p.dim, n, 1.0 / p.n[0]);
        L = stfas_levels(g0);
        pois.init(g0, p.N, s);
    }
    ~Solver() override {
        if (lb) (void)hipFree(lb);
    }

    int nlevels() const override { return (int)L.size(); }
    const Grid& level(int l) const override { return L[l]; }

    bool valid() const override { return pois.coarse_ok(); }

    void layout(Arena& A) {
        const long F0 = L[0].nface, C0 = L[0].ncell;
        lev.assign(L.size(), Lev{});
        for (size_t l = 0; l < L.size(); ++l) {
            const long F = L[l].nface, C = L[l].ncell;
            Lev& q = lev[l];
            q.v = A.take<T>(N * F);
            q.pb = A.take<T>(N * C);
            q.u = A.take<T>(N * F);
            q.p = A.take<T>(N * C);
            q.r1 = A.take<T>(N * F);
            q.r2 = A.take<T>(N * C);
            q.r3 = A.take<T>(N * F);
            q.r4 = A.take<T>(N * C);
            if (l > 0) {
                q.s1 = A.take<T>(N * F);
                q.s2 = A.take<T>(N * C);
                q.s3 = A.take<T>(N * F);
                q.s4 = A.take<T>(N * C);
            } else {
                q.s1 = q.s2 = q.s3 = q.s4 = nullptr;
            }
            q.w = A.take<T>(N * F);
        }
        // the J_S^T part of F1 held over a sweep, and its cleared successor (any level)
        t1a = A.take<T>(N * F0);
        t1b = A.take<T>(N * F0);
        // 3D: the foot-point quarters of the sweep's transpose, two per face slot (any level)
        tq = D == 3 ? A.take<T>((size_t)2 * N * F0) : nullptr;
        // SCGS scratch of long horizons: the largest colour of level 0, 2N blocks, 2d faces per cell
        int Gs, Ls, CHs;
        if (colour_shape<T, D>(2 * N, 1, Gs, Ls, CHs)) {
            scgs_scratch = nullptr;
        } else {
            long maxcol = 0;
            for (int c = 0; c < (1 << D); ++c) maxcol = std::max<long>(maxcol, colour_set(L[0], c).total);
            scgs_scratch = A.take<T>((size_t)maxcol * 2 * D * 2 * N);
        }
        if (P.rot_exact && !rot_use_fused(colour_set(L[0], 0).total)) {
            long maxcol = 0;
            for (int c = 0; c < (1 << D); ++c) maxcol = std::max<long>(maxcol, colour_set(L[0], c).total);
            rot_scratch = A.take<T>((size_t)maxcol * N * RotDims<D>::REC);
        }
        t_diag = A.take<T>(2 * N);
        t_sub = A.take<T>(2 * N);
        t_sup = A.take<T>(2 * N);
        t_cp = A.take<T>(2 * N);
        t_inv = A.take<T>(2 * N);
        pois.layout(A, nullptr);
        rho = A.take<T>((N + 1) * C0);
        rho_t = A.take<T>((N + 1) * C0);
        mu = A.take<T>(N * C0);
        vt = A.take<T>(N * F0);
        vstar = A.take<T>(N * F0);
        cand = A.take<T>(N * F0);
        trial = A.take<T>(N * F0);
        ce_e = A.take<T>(C0);
        ce_acc = A.take<T>(C0);
        ce_t1 = A.take<T>(C0);
        ce_t2 = A.take<T>(C0);
        size_t ntaps = 0;
        for (int l = 1; l <= P.metric_levels; ++l) ntaps += gauss_taps(std::ldexp(1.0, l - 1)).size();
        taps = A.take<T>(std::max<size_t>(ntaps, 1));
        lam = A.take<T>(N * F0);
        rho_last = A.take<T>((N + 1) * C0);
        wt = A.take<T>(N * F0);
        rs_rho[0] = A.take<T>(C0);
        rs_rho[1] = A.take<T>(C0);
        rs_v[0] = A.take<T>(F0);
        rs_v[1] = A.take<T>(F0);
        rs_w = A.take<T>(F0);
        red_part = A.take<double>(RED_BLOCKS);
        red_out = A.take<double>(64);
        if (upwind()) {
            up.layout(A, C0, N);
            up.tr = &tr;
            up_kd = A.template take<int>(N);
            up_okd = A.template take<int>(N);
        }
    }

    size_t plan() override {
        Arena A;
        layout(A);
        return A.off;
    }
    void carve(char* base) override {
        Arena A;
        A.base = base;
        layout(A);
    }

    template <typename U>
    void upload(U* dst, const std::vector<double>& src) {
        std::vector<U> tmp(src.begin(), src.end());
        HCK(hipMemcpyAsync(dst, tmp.data(), tmp.size() * sizeof(U), hipMemcpyHostToDevice, st));
        HCK(hipStreamSynchronize(st));
    }

    void init_tables() override {
        host_out = thread_pinned();
        // t1_zero is all zero between SCGS sweeps: each sweep's transpose
        // launch fills the other buffer's successor (see sweep)
        fill(t1a, (long)N * L[0].nface, (T)0);
        t1_zero = t1a;
        t1_used = t1b;
        TFactors f = temporal_factors(N, P.dt, P.K / P.r, P.lm);
        upload(t_diag, f.diag);
        upload(t_sub, f.sub);
        upload(t_sup, f.sup);
        upload(t_cp, f.cp);
        upload(t_inv, f.inv);
        pois.upload_pinv();
        std::vector<double> all;
        tap_off.clear();
        tap_R.clear();
        for (int l = 1; l <= P.metric_levels; ++l) {
            auto k = gauss_taps(std::ldexp(1.0, l - 1));
            tap_off.push_back((int)all.size());
            tap_R.push_back(((int)k.size() - 1) / 2);
            all.insert(all.end(), k.begin(), k.end());
        }
        if (!all.empty()) upload(taps, all);
    }

    // ------------------------------------------------------------ helpers
    T cfl(int l) const { return (T)(P.dt / L[l].h); }
    void fill(T* x, long n, T val) {
        if (n <= 0) return;
        k_fill<T><<<blocks_for(n, BS), BS, 0, st>>>(n, x, val);
    }
    void copy(T* dst, const T* src, long n) {
        if (n <= 0) return;
        HCK(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToDevice, st));
    }
    void axpby(long n, T a, const T* x, T b, const T* y, T* out) {
        k_axpby<T><<<blocks_for(n, BS), BS, 0, st>>>(n, a, x, b, y, out);
    }
    // red_out[slot] (op)= reduce(x, y) over n elements
    void reduce(int op, long n, const T* x, const T* y, int slot, bool accumulate) {
        const int nb = (int)std::min<long>(RED_BLOCKS, std::max<long>(1, blocks_for(n, RED_BS)));
        k_reduce_part<T><<<nb, RED_BS, 0, st>>>(n, op, x, y, red_part);
        k_reduce_final<<<1, RED_BS, 0, st>>>(nb, op, red_part, red_out, slot, accumulate ? 1 : 0);
    }
    // red_out[slot] = max |x| over the four arrays
    void maxabs4(long n0, const T* x0, long n1, const T* x1, long n2, const T* x2, long n3, const T* x3, int slot) {
        const long n = std::max(std::max(n0, n1), std::max(n2, n3));
        const int nb = (int)std::min<long>(RED_BLOCKS, std::max<long>(1, blocks_for(n, RED_BS)));
        k_maxabs4_part<T><<<nb, RED_BS, 0, st>>>(n0, x0, n1, x1, n2, x2, n3, x3, red_part);
        k_reduce_final<<<1, RED_BS, 0, st>>>(nb, RED_MAXABS_DIFF, red_part, red_out, slot, 0);
    }
    // red_out[slot] = max |x| over the interior faces of `slices` level-0 face fields
    void maxabs_interior(long slices, const T* x, int slot) {
        const long n = slices * L[0].nface;
        const int nb = (int)std::min<long>(RED_BLOCKS, std::max<long>(1, blocks_for(n, RED_BS)));
        k_maxabs_interior_part<T><<<nb, RED_BS, 0, st>>>(L[0], slices, x, red_part);
        k_reduce_final<<<1, RED_BS, 0, st>>>(nb, RED_MAXABS_DIFF, red_part, red_out, slot, 0);
    }
    void zero_slots(int n) { k_fill<double><<<1, 64, 0, st>>>(n, red_out, 0.0); }
    void readback(int n) {
        HCK(hipMemcpyAsync(host_out, red_out, n * sizeof(double), hipMemcpyDeviceToHost, st));
        HCK(hipStreamSynchronize(st));
    }

    // ------------------------------------------------------------ advection
    void advect(const T* r, const T* v, T* out, int batch) {
        const Grid& g = L[0];
        k_advect<T, D><<<dim3(blocks_for(g.ncell, BS), batch), BS, 0, st>>>(g, cfl(0), r, v, out, g.ncell, g.nface);
    }
    void advect_T(const T* m, const T* v, T* out, int batch) { launch_advect_T<T, D>(L[0], cfl(0), m, v, out, batch, st); }
    void advect_dv_T(const T* m, const T* r, const T* v, const T* vtt, T scale, T* gv, int batch) {
        const Grid& g = L[0];
        k_advect_dv_T<T, D><<<dim3(blocks_for(g.nface, BS), batch), BS, 0, st>>>(g, cfl(0), m, r, v, vtt, scale,
                                                                                gv, g.ncell, g.nface);
    }
    // one fixed-point step's right-hand side of the rotational update on level 0:
    // out = v + dt u - dt Adv[vk] on interior faces (vk = null: without Adv)
    void rot_rhs(const T* v, const T* u, const T* vk, T* out) {
        const Grid& g = L[0];
        k_rot_rhs<T, D><<<blocks_for(g.nface, BS), BS, 0, st>>>(g, (T)P.dt, v, u, vk, out);
    }
    // out = -dt J_Adv(y)^T x on interior faces of level 0 (y = null: out = x there), 0 on walls
    void rot_adj(const T* y, const T* x, T* out) {
        const Grid& g = L[0];
        k_rot_adj<T, D><<<blocks_for(g.nface, BS), BS, 0, st>>>(g, (T)P.dt, y, x, out);
    }
    void self_advect(int l, const T* v, const T* u, T* out, int batch) {
        const Grid& g = L[l];
        k_self_advect<T, D><<<dim3(blocks_for(g.nface, BS), batch), BS, 0, st>>>(g, cfl(l), (T)P.dt, v, u, out,
                                                                                g.nface);
    }
    void self_advect_T(int l, const T* v, const T* y, T scale, T* out, int batch) {
        if (batch <= 0) return;
        launch_self_advect_T<T, D>(L[l], cfl(l), v, y, scale, out, batch, st);
    }

    // Density operator of eq:Conv, semi-Lagrangian or upwind exponential.
    void dens_fwd(const T* r, const T* v, T* out) {
        if (upwind())
            up.forward(L[0], P.dt, r, v, out, st);
        else
            advect(r, v, out, 1);
    }
    // grho += (dA/drho)^T m (grho may be null); gv = base + scale (dA/dv)^T m
    // on interior faces, 0 on walls (base may be null); k_known: the upwind
    // series' k for (r, v) when the forward sweep measured it
    void dens_adj(const T* m, const T* r, const T* v, T* grho, T* gv, const T* base, T scale, int k_known = -1,
                  const T* stored = nullptr) {
        if (upwind()) {
            up.adjoint(L[0], P.dt, m, r, v, grho, gv, base, scale, st, k_known, stored);
            return;
        }
        if (grho) advect_T(m, v, grho, 1);
        advect_dv_T(m, r, v, base, scale, gv, 1);
    }

    // ------------------------------------------------------------ projection
    int project(const T* w, T* out, T* phi_out, int B, int fixed = 0, bool count = false) {
        return pois.project(w, out, phi_out, B, P.poisson_rtol, fixed, host_out, count);
    }

    // ------------------------------------------------------------ metric
    // out = C e = e + sum_l G_l G_l e   (separable Gaussians, zero padding)
    void metric(const T* e, T* out) {
        const Grid& g = L[0];
        const long C = g.ncell;
        copy(out, e, C);
        for (int l = 0; l < P.metric_levels; ++l) {
            const T* src = e;
            T* bufs[2] = {ce_t1, ce_t2};
            int cur = 0;
            for (int pass = 0; pass < 2 * D; ++pass) {
                k_blur_axis<T><<<blocks_for(C, BS), BS, 0, st>>>(g, pass % D, tap_R[l], taps + tap_off[l], src,
                                                                 bufs[cur]);
                src = bufs[cur];
                cur ^= 1;
            }
            axpby(C, (T)1, out, (T)1, src, out);
        }
    }

    // ------------------------------------------------------------ KKT
    // out = res + sgn f(x) on level l.
    void kkt(int l, const T* v, const T* pb, const T* u, const T* p, const T* w, const T* s1, const T* s2,
             const T* s3, const T* s4, T* o1, T* o2, T* o3, T* o4, T sgn) {
        const Grid& g = L[l];
        const T dt = (T)P.dt;
        const double sz = sizeof(T);
        const double fslots = (double)g.nface * N, cslots = (double)g.ncell * N;
        // face and cell rows in one launch (the split residual kernel without its transpose part):
        // v, u, w in and out1, out3 out per face slot (+ res1, res3); pbar, p in and out2, out4 out
        // per cell slot (+ res2, res4)
        KktSplit ks{};
        ks.nbf = blocks_for(g.nface, 256);
        ks.nbc = blocks_for(g.ncell, 256);
        ks.vort = P.vort;
        const long blocks = (long)(ks.nbf + ks.nbc) * N;
        traced(tr, st, l == 0 ? TR_KKT_FACES : TR_NONE,
               sz * (fslots * (5 + (s1 ? 2 : 0)) + cslots * (4 + (s2 ? 2 : 0))), [&] {
                   k_kkt_split<T, D><<<(unsigned)blocks, 256, 0, st>>>(g, N, dt, (T)(P.K / P.r), cfl(l), sgn, ks, v,
                                                                      pb, u, p, w, s1, s2, s3, s4, o1, o2, o3, o4,
                                                                      nullptr, nullptr);
               });
        if (N > 1 && !P.vort) {
            // v, y read, out read-modify-write, per face
            traced(tr, st, l == 0 ? TR_SELF_ADVECT_T : TR_NONE, sz * (double)g.nface * (N - 1) * 4,
                   [&] { self_advect_T(l, v, u + g.nface, (T)(-sgn / dt), o1, N - 1); });
        }
    }
    // The two launches of a sweep's residual (r = res - f(x) on level l), both
    // with the split residual kernel:
    //  kkt_transpose: the J_S^T u / dt part of F1 from the state at the start of
    //    the sweep into t1 (zero on entry; all faces), with t1z cleared for the
    //    next sweep;
    //  kkt_rows: per colour, the face and cell rows of that colour without that
    //    part (r1 .. r4), from the current state.
    void kkt_transpose(int l, T* t1, T* t1z) {
        const Grid& g = L[l];
        Lev& q = lev[l];
        using TS = TileShape<D>;
        KktSplit ks{};
        // small levels: the transpose without tiles (no LDS window, no barriers), since there a launch is
        // a chain of dependent memory steps and its few atomics are cheap
        ks.direct = (long)N * g.nface <= DIRECT_T_SLOTS ? 1 : 0;
        ks.ntile = 0;
        if (N > 1) {
            if (ks.direct) {
                ks.ntile = blocks_for(g.nface, 256);
            } else {
                for (int a = 0; a < D; ++a) {
                    const int ex = face_ext(g, a, 0), ey = face_ext(g, a, 1), ez = face_ext(g, a, 2);
                    const int t = ((ex + TS::X - 1) / TS::X) * ((ey + TS::Y - 1) / TS::Y) *
                                  (D == 3 ? (ez + TS::Z - 1) / TS::Z : 1);
                    ks.ntile = std::max(ks.ntile, t);
                }
            }
        }
        ks.nbz = std::min(blocks_for((long)N * g.nface, 256), 2048);
        // 3D tiles: the quarters of the foot-point term for the other axes through tq and a gather
        const bool gather = D == 3 && !ks.direct && N > 1;
        ks.gq = gather ? (void*)tq : nullptr;
        const long blocks = (long)ks.ntile * std::max(N - 1, 0) * (ks.direct ? 1 : D) + ks.nbz;
        const double sz = sizeof(T);
        // the method's bytes (v, y -> J_S^T y): 3d words per spacetime cell (24 B in 2D, 36 B in 3D, FP32);
        // the launch also clears t1z
        const double method = sz * 3.0 * D * (double)g.ncell * std::max(N - 1, 0);
        const double impl = sz * ((double)g.nface * std::max(N - 1, 0) * 3 + (double)g.nface * N);
        traced(tr, st, l == 0 ? TR_SELF_ADVECT_T : TR_NONE, method, [&] {
            k_kkt_split<T, D><<<(unsigned)blocks, 256, 0, st>>>(g, N, (T)P.dt, (T)(P.K / P.r), cfl(l), (T)-1, ks,
                                                               q.v, q.pb, q.u, q.p, q.w, q.s1, q.s2, q.s3, q.s4,
                                                               q.r1, q.r2, q.r3, q.r4, t1, t1z);
            if (gather)
                k_quarter_gather<T, D><<<dim3(blocks_for(g.nface, 256), N - 1), 256, 0, st>>>(g, tq, t1, g.nface);
        }, impl + (gather ? sz * (double)g.nface * (N - 1) * (2 * 2 + 1 + 1) : 0.0));
    }
    // t1 != nullptr: the same launch also computes the J_S^T part (every
    // face, into t1, zero on entry) and clears t1z: one launch per colour
    // with the transpose refreshed for that colour.
    void kkt_rows(int l, int colour, T* t1 = nullptr, T* t1z = nullptr) {
        const Grid& g = L[l];
        Lev& q = lev[l];
        using TS = TileShape<D>;
        KktSplit ks{};
        const ColourSet cs = colour_set(g, colour);
        ks.rows = 1;
        for (int a = 0; a < 3; ++a) {
            ks.par[a] = cs.p[a];
            ks.cnt[a] = cs.cnt[a];
        }
        ks.nfc = 0;
        for (int a = 0; a < D; ++a) {
            long m = g.n[a] + 1;
            for (int b2 = 0; b2 < 3; ++b2)
                if (b2 != a) m *= cs.cnt[b2];
            ks.nfc += (int)m;
        }
        const long nfr = ks.nfc, ncr = cs.total;     // face and cell rows per slice
        ks.nbf = blocks_for(nfr, 256);
        ks.nbc = blocks_for(ncr, 256);
        ks.vort = P.vort;
        if (P.vort) t1 = t1z = nullptr;    // the rotational rows have no transpose part
        if (t1 && N > 1) {
            ks.direct = (long)N * g.nface <= DIRECT_T_SLOTS ? 1 : 0;
            if (ks.direct) {
                ks.ntile = blocks_for(g.nface, 256);
            } else {
                for (int a = 0; a < D; ++a) {
                    const int ex = face_ext(g, a, 0), ey = face_ext(g, a, 1), ez = face_ext(g, a, 2);
                    const int t = ((ex + TS::X - 1) / TS::X) * ((ey + TS::Y - 1) / TS::Y) *
                                  (D == 3 ? (ez + TS::Z - 1) / TS::Z : 1);
                    ks.ntile = std::max(ks.ntile, t);
                }
            }
        }
        if (t1z) ks.nbz = std::min(blocks_for((long)N * g.nface, 256), 2048);
        const long blocks = (long)(ks.nbf + ks.nbc) * N + (long)ks.ntile * std::max(N - 1, 0) * (ks.direct ? 1 : D) +
                            ks.nbz;
        const double sz = sizeof(T);
        const double rslots = (double)nfr * N, cslots = (double)ncr * N;
        // every sequence the launch reads or writes, once: v, u, w in and r1, r3 out per face-row slot
        // (+ s1, s3 on coarse levels; the S gather reads v around each face); pbar, p in and r2, r4
        // out per cell-row slot (+ s2, s4); with the transpose, v, u in and t1, t1z out per face slot
        const double impl = sz * (rslots * (5 + (q.s1 ? 2 : 0)) + cslots * (4 + (q.s2 ? 2 : 0)) +
                                  (t1 ? (double)g.nface * N * 4 : 0.0));
        // the method's bytes: (v, u, pbar, p, w, res -> r) once per spacetime cell whose rows the launch
        // computes, 2d + 2 + d + 2 (2d + 2) words: 20 words (80 B FP32) in 2D, 27 (108 B) in 3D
        const double method = sz * (D == 2 ? 20.0 : 27.0) * cslots;
        traced(tr, st, l == 0 ? TR_KKT_SPLIT : TR_NONE, method, [&] {
            k_kkt_split<T, D><<<(unsigned)blocks, 256, 0, st>>>(g, N, (T)P.dt, (T)(P.K / P.r), cfl(l), (T)-1, ks,
                                                               q.v, q.pb, q.u, q.p, q.w, q.s1, q.s2, q.s3, q.s4,
                                                               q.r1, q.r2, q.r3, q.r4, t1, t1z);
        }, impl);
    }
    void kkt_level(int l, bool fas_rhs) {
        Lev& q = lev[l];
        if (fas_rhs)
            kkt(l, q.v, q.pb, q.u, q.p, q.w, q.s1, q.s2, q.s3, q.s4, q.s1, q.s2, q.s3, q.s4, (T)1);
        else
            kkt(l, q.v, q.pb, q.u, q.p, q.w, q.s1, q.s2, q.s3, q.s4, q.r1, q.r2, q.r3, q.r4, (T)-1);
    }

    // Interior face slots of the cells of one colour (sum of m over cells).
    static long colour_inner_faces(const Grid& g, int colour) {
        const ColourSet cs = colour_set(g, colour);
        long tot = 0;
        for (int a = 0; a < g.dim; ++a) {
            long lo = 0, hi = 0;
            for (int c = 0; c < cs.cnt[a]; ++c) {
                const int idx = 2 * c + cs.p[a];
                lo += idx >= 1;
                hi += idx + 1 <= g.n[a] - 1;
            }
            const long other = (long)cs.total / cs.cnt[a];
            tot += (lo + hi) * other;
        }
        return tot;
    }

    // Local solves of one colour with the rotational operator: eq:HESS with the
    // cell's block of dAdv/dv, reduced to 3x3 blocks and eliminated in time;
    // one launch while a cell's records fit in LDS, else three through rot_scratch.
    void rot_local_solve(int l, int colour) {
        const Grid& g = L[l];
        Lev& q = lev[l];
        const ColourSet cs = colour_set(g, colour);
        const long n = (long)cs.total * N;
        const T dt = (T)P.dt, kr = (T)(P.K / P.r), lm = (T)P.lm;
        if (rot_use_fused(cs.total)) {
            const int tbc = rot_fused_cells<T, D>(N);
            const size_t lds = (size_t)tbc * ((size_t)N * RotDims<D>::REC + 16 / sizeof(T)) * sizeof(T);
            k_rot_blk_fused<T, D><<<blocks_for(cs.total, tbc), 512, lds, st>>>(
                g, N, cs, tbc, dt, kr, lm, (T)P.omega, q.v, q.pb, q.u, q.p, q.r1, q.r2, q.r3, q.r4);
            return;
        }
        k_rot_blk_setup<T, D><<<blocks_for(n, 256), 256, 0, st>>>(g, N, cs, dt, kr, lm, q.v, q.r1, q.r2, q.r3,
                                                                 q.r4, rot_scratch);
        const int tb = rot_blk_threads<T, D>(N);
        k_rot_blk_thomas<T, D><<<blocks_for(cs.total, tb), tb, (size_t)tb * N * rot_blk_lds_words<D>() * sizeof(T),
                                 st>>>(N, cs.total, rot_scratch);
        k_rot_blk_apply<T, D><<<blocks_for(n, 256), 256, 0, st>>>(g, N, cs, dt, kr, lm, (T)P.omega, q.v, q.pb,
                                                                 q.u, q.p, q.r1, q.r2, q.r3, q.r4, rot_scratch);
    }
    // The fused launch while a cell's records fit in LDS and its blocks (a few
    // cells each, one eliminating thread per cell) fill the chip about twice;
    // beyond, the three launches, whose elimination runs 64 cells per wave.
    bool rot_use_fused(long cells) const {
        const int tbc = rot_fused_cells<T, D>(N);
        return tbc >= 1 && blocks_for(cells, tbc) <= 512;
    }

    // One SCGS sweep on level l.  3D: the J_S^T part of F1 once from the state
    // at the sweep's start, held for every colour, then per colour its rows
    // and its local solves.  2D: per colour, its rows and the J_S^T part from
    // the current state in one launch, then its local solves.
    void sweep(int l) {
        const Grid& g = L[l];
        Lev& q = lev[l];
        T* t1 = nullptr;
        if (D == 3) {
            t1 = t1_zero;
            if (!P.vort) {                          // the rotational rows have no transpose part
                kkt_transpose(l, t1, t1_used);      // t1_used is cleared for the next sweep
                std::swap(t1_zero, t1_used);
            }
        }
        for (int colour = 0; colour < (1 << D); ++colour) {
            const ColourSet cs = colour_set(g, colour);
            const int nf = cs.total * 2 * D;
            const double inner = (double)colour_inner_faces(g, colour);
            const double sz = sizeof(T), M2 = 2.0 * N;
            int G = 1, Lc = 0, CH = 0;
            if (l < P.rot_exact) {
                kkt_rows(l, colour);                // the rows carry every term of F1
                rot_local_solve(l, colour);
                continue;
            } else if (D == 3) {
                kkt_rows(l, colour);
            } else if (P.vort) {
                t1 = t1_zero;                       // stays zero: the rows carry every term of F1
                kkt_rows(l, colour);
            } else {
                t1 = t1_zero;
                kkt_rows(l, colour, t1, t1_used);   // t1_used is cleared for the next colour
                std::swap(t1_zero, t1_used);
            }
            if (colour_shape<T, D>(2 * N, cs.total, G, Lc, CH)) {
                // one kernel reads r1 + t1, r2..r4 once and updates u/v and p/pbar;
                // per block pair: r1, t1, r3 read, u and v read + written at each interior face;
                // per block: the divergence residual read, p or pbar read + written at each cell
                traced(tr, st, l == 0 ? TR_SCGS_COLOUR : TR_NONE, sz * M2 * (inner * 3.5 + cs.total * 3), [&] {
                    launch_scgs_colour<T, D>(G, Lc, CH, g, N, cs, q.r1, t1, q.r2, q.r3, q.r4, q.v, q.pb, q.u,
                                             q.p, t_diag, t_sub, t_sup, t_cp, t_inv, (T)P.omega, st);
                });
                continue;
            }
            // long horizons: r1 += t1, then project: read r1/r3 at the colour's faces, write (P r)
            axpby((long)N * g.nface, (T)1, q.r1, (T)1, t1, q.r1);
            traced(tr, st, l == 0 ? TR_SCGS_PROJECT : TR_NONE, sz * M2 * inner * 2, [&] {
                k_scgs_project<T, D><<<blocks_for((long)nf * 2 * N, BS), BS, 0, st>>>(g, N, cs, q.r1, q.r3,
                                                                                      scgs_scratch);
            });
            // thomas: read (P r), read the cells' divergence residual, update u/v at the faces
            traced(tr, st, l == 0 ? TR_SCGS_THOMAS : TR_NONE, sz * M2 * (inner * 3 + cs.total), [&] {
                k_scgs_thomas<T, D><<<blocks_for(nf, 64), 64, 3 * 2 * N * sizeof(T), st>>>(
                    g, N, cs, q.r2, q.r4, q.v, q.u, t_sub, t_cp, t_inv, (T)P.omega, scgs_scratch);
            });
            const int nc = cs.total * 2 * N;
            traced(tr, st, l == 0 ? TR_SCGS_CELLS : TR_NONE, sz * M2 * (inner + cs.total * 3), [&] {
                k_scgs_cells<T, D><<<blocks_for(nc, BS), BS, 0, st>>>(g, N, cs, q.r1, q.r2, q.r3, q.r4, q.pb, q.p,
                                                                     t_diag, t_sub, t_sup, (T)P.omega);
            });
        }
    }

    // n transfers in one launch, the first nf on face sequences
    void restrict_set(int l, std::initializer_list<const T*> src, std::initializer_list<T*> dst, int nf, int n) {
        XferSet<T> x{};
        int z = 0;
        for (const T* p : src) x.src[z++] = p;
        z = 0;
        for (T* p : dst) x.dst[z++] = p;
        const Grid& gc = L[l + 1];
        const int m = (int)std::max<long>(gc.nface, gc.ncell);
        k_restrict_set<T, D><<<dim3(blocks_for(m, BS), N, n), BS, 0, st>>>(L[l], gc, x, nf);
    }
    void prolong_set(int l, std::initializer_list<const T*> src, std::initializer_list<T*> dst, int nf, int n, T sign) {
        XferSet<T> x{};
        int z = 0;
        for (const T* p : src) x.src[z++] = p;
        z = 0;
        for (T* p : dst) x.dst[z++] = p;
        const Grid& gf = L[l];
        const int m = (int)std::max<long>(gf.nface, gf.ncell);
        k_prolong_set<T, D><<<dim3(blocks_for(m, BS), N, n), BS, 0, st>>>(gf, L[l + 1], x, nf, sign);
    }
    void restrict_faces(int l, const T* fine, T* coarse) {
        k_restrict_faces<T, D><<<dim3(blocks_for(L[l + 1].nface, BS), N), BS, 0, st>>>(L[l], L[l + 1], fine, coarse);
    }
    void restrict_cells(int l, const T* fine, T* coarse) {
        k_restrict_cells<T, D><<<dim3(blocks_for(L[l + 1].ncell, BS), N), BS, 0, st>>>(L[l], L[l + 1], fine, coarse);
    }
    void prolong_faces(int l, const T* coarse, T sign, T* fine) {
        k_prolong_faces<T, D><<<dim3(blocks_for(L[l].nface, BS), N), BS, 0, st>>>(L[l], L[l + 1], coarse, sign, fine);
    }
    void prolong_cells(int l, const T* coarse, T sign, T* fine) {
        k_prolong_cells<T, D><<<dim3(blocks_for(L[l].ncell, BS), N), BS, 0, st>>>(L[l], L[l + 1], coarse, sign, fine);
    }

    void vcycle(int l) {
        Lev& q = lev[l];
        if (l == (int)L.size() - 1) {
            for (int s = 0; s < 10; ++s) sweep(l);
            return;
        }
        sweep(l);
        sweep(l);
        kkt_level(l, false);                                   // r = res - f(x_s)
        Lev& c = lev[l + 1];
        // x^{2h} = R x_s and the residual part of res^{2h} = R r + f(x^{2h}), one launch
        restrict_set(l, {q.v, q.u, q.r1, q.r3, q.pb, q.p, q.r2, q.r4}, {c.v, c.u, c.s1, c.s3, c.pb, c.p, c.s2, c.s4},
                     4, 8);
        prolong_set(l, {c.v, c.u, c.pb, c.p}, {q.v, q.u, q.pb, q.p}, 2, 4, (T)-1);   // x = x_s - P x^{2h}
        kkt_level(l + 1, true);
        vcycle(l + 1);
        prolong_set(l, {c.v, c.u, c.pb, c.p}, {q.v, q.u, q.pb, q.p}, 2, 4, (T)1);    // x += P x^{2h}
        sweep(l);
        sweep(l);
    }

    double residual_inf() {
        Lev& q = lev[0];
        kkt_level(0, false);
        const long F = L[0].nface, C = L[0].ncell;
        maxabs4(N * F, q.r1, N * C, q.r2, N * F, q.r3, N * C, q.r4, 0);
        readback(1);
        return host_out[0];
    }

    // Velocity subproblem on lev[0] state with lev[0].w targets.
    int nso(double* hist, double* last) {
        for (size_t l = 0; l + 1 < L.size(); ++l) restrict_faces((int)l, lev[l].w, lev[l + 1].w);
        const long F = L[0].nface;
        // |f(0)|_inf: at the zero state only F1 = -(K/r) w_i (i = 1..N-1, interior faces) is nonzero
        double f0 = 0;
        if (N > 1) {
            maxabs_interior(N - 1, lev[0].w + F, 0);
            readback(1);
            f0 = (P.K / P.r) * host_out[0];
        }
        double h = residual_inf();
        if (hist) hist[0] = h;
        int n = 0;
        while (n < P.max_vcycles) {
            if (!P.fixed_counts && h <= P.eps_stfas * f0) break;
            vcycle(0);
            ++n;
            h = residual_inf();
            if (hist) hist[n] = h;
            if (!std::isfinite(h)) break;
        }
        if (last) *last = h;
        return n;
    }

    // ------------------------------------------------------------ density subproblem
    // hset >= 0 (upwind, 2D): the series' terms of every step are kept in stored trajectory hset
    void forward_sweep(const T* rho0, const T* vs, T* r, std::vector<int>* kout = nullptr, int hset = -1) {
        const long C = L[0].ncell, F = L[0].nface;
        copy(r, rho0, C);
        if (upwind()) {
            up_sweep(r, vs, kout, hset);
            return;
        }
        for (int i = 0; i < N; ++i) dens_fwd(r + i * C, vs + i * F, r + (i + 1) * C);
    }

    // Density sweep r_{i+1} = A(r_i, v_i), i = 0..N-1, with the upwind
    // exponential (r_0 already set).  Each step's series is launched only to
    // the k of the previous sweep plus 3; one readback after the sweep shows
    // which steps had not stopped by then, and the sweep is run again from
    // the first of them with the full 48 launches for that step.  k per step
    // goes to kout.
    void up_sweep(T* r, const T* vs, std::vector<int>* kout, int hset = -1) {
        const long C = L[0].ncell, F = L[0].nface;
        if ((int)up_pred.size() != N) up_pred.assign(N, UP_KMAX);
        std::vector<int> nl(up_pred), kh(N), okh(N);
        int from = 0;
        while (from < N) {
            for (int i = from; i < N; ++i) {
                up.forward(L[0], P.dt, r + i * C, vs + i * F, r + (i + 1) * C, st, nl[i], true, up_kd + i,
                           up_okd + i, hset >= 0 ? up.hist_step(hset, i, C) : nullptr);
            }
            HCK(hipMemcpyAsync(kh.data() + from, up_kd + from, (N - from) * sizeof(int), hipMemcpyDeviceToHost, st));
            HCK(hipMemcpyAsync(okh.data() + from, up_okd + from, (N - from) * sizeof(int), hipMemcpyDeviceToHost,
                               st));
            HCK(hipStreamSynchronize(st));
            // the launches past each series' stop did no work: take back their credit
            for (int i = from; i < N; ++i)
                tr.credit(TR_UP_TERM, -(double)(nl[i] - kh[i]) * UpwindExp<T, D>::term_bytes(L[0]));
            int bad = N;
            for (int i = from; i < N; ++i)
                if (!okh[i]) {
                    bad = i;
                    break;
                }
            from = bad;
            if (from < N) nl[from] = UP_KMAX;   // the steps after it are re-run with their predictions
        }
        for (int i = 0; i < N; ++i) up_pred[i] = std::min(UP_KMAX, kh[i] + 3);
        if (kout) *kout = kh;
    }

    // Phi = 1/2 sum_key <e, C e> + K/2 |vt - vs|^2 (reduced in double).
    double ao_objective(const T* r, const T* vs, int nk, const int* ks, const T* keys) {
        const long C = L[0].ncell, F = L[0].nface;
        zero_slots(2);
        for (int q = 0; q < nk; ++q) {
            axpby(C, (T)1, r + (long)ks[q] * C, (T)-1, keys + q * C, ce_e);
            metric(ce_e, ce_acc);
            reduce(RED_DOT, C, ce_e, ce_acc, 0, true);
        }
        reduce(RED_SUMSQ_DIFF, N * F, vt, vs, 1, false);
        readback(2);
        return 0.5 * host_out[0] + 0.5 * P.K * host_out[1];
    }

    // mu_i for i = 0..N-1; with the upwind operator also the candidate
    // directions cand_i = vt_i + (dA/dv)^T mu_i / K (the semi-Lagrangian
    // form computes them afterwards in one batched launch)
    void ao_backward(const T* r, const T* vs, int nk, const int* ks, const T* keys) {
        const long C = L[0].ncell, F = L[0].nface;
        const T ik = (T)(1.0 / P.K);
        for (int i = N; i >= 1; --i) {
            T* out = mu + (i - 1) * C;
            int kq = -1;
            for (int q = 0; q < nk; ++q)
                if (ks[q] == i) kq = q;
            if (kq >= 0) {
                axpby(C, (T)1, r + (long)i * C, (T)-1, keys + kq * C, ce_e);
                metric(ce_e, ce_acc);
                axpby(C, (T)-1, ce_acc, (T)0, nullptr, out);
            } else {
                fill(out, C, (T)0);
            }
            if (i < N) {
                if (upwind())
                    dens_adj(mu + i * C, r + i * C, vs + i * F, out, cand + i * F, vt + i * F, ik, kr_of(i),
                             stored_of(i));
                else
                    advect_T(mu + i * C, vs + i * F, out, 1);
            }
        }
        if (upwind()) dens_adj(mu, r, vs, nullptr, cand, vt, ik, kr_of(0), stored_of(0));
    }
    // k of step i of the accepted AO trajectory (-1: unknown)
    int kr_of(int i) const { return (int)k_rho.size() == N ? k_rho[i] : -1; }
    // the terms of step i of the accepted AO trajectory, when its forward sweep kept them
    int up_hcur = 0;             // stored trajectory of rho (the other one takes the line search's trials)
    const T* stored_of(int i) const { return kr_of(i) >= 0 ? up.hist_step(up_hcur, i, L[0].ncell) : nullptr; }

    // Alg:Passive with blending; vt must hold v + lambda/K.  Result in vstar, rho.
    void ao(const T* rho0, int nk, const int* ks, const T* keys, double* hist) {
        const long C = L[0].ncell, F = L[0].nface;
        copy(vstar, vt, N * F);
        forward_sweep(rho0, vstar, rho, &k_rho, up_hcur);
        double phi = ao_objective(rho, vstar, nk, ks, keys);
        if (hist) hist[0] = phi;
        for (int it = 0; it < P.ao_iters; ++it) {
            ao_backward(rho, vstar, nk, ks, keys);
            if (!upwind()) advect_dv_T(mu, rho, vstar, vt, (T)(1.0 / P.K), cand, N);
            project(cand, cand, nullptr, N);
            double alpha = 1.0;
            for (int hv = 0; hv <= 10; ++hv) {
                blend(vstar, cand, (T)alpha, trial, N * F);
                forward_sweep(rho0, trial, rho_t, &k_rho_t, up_hcur ^ 1);
                const double pt = ao_objective(rho_t, trial, nk, ks, keys);
                if (pt <= phi) {
                    std::swap(vstar, trial);
                    std::swap(rho, rho_t);
                    std::swap(k_rho, k_rho_t);
                    up_hcur ^= 1;
                    phi = pt;
                    break;
                }
                alpha *= 0.5;
            }
            if (hist) hist[it + 1] = phi;
        }
    }

    void blend(const T* x, const T* y, T alpha, T* out, long n);

    // ------------------------------------------------------------ L-BFGS baseline
    // The gradient-based optimiser the paper compares against: L-BFGS on the
    // reduced objective J(u) = 1/2 sum_k <e_k, C e_k> + r/2 |u|^2 with the
    // simulation eliminated, its gradient by the adjoint of the step chain.
    // History 8, gamma = s'y / y'y (1/|g| on the first iteration), Armijo
    // backtracking (c1 = 1e-4, first step 1, up to 20 halvings); pairs with
    // y's <= 1e-12 |s||y| are not kept.  With eps_stop > 0 it stops after an
    // accepted iterate whose density trajectory differs from the previous
    // one by at most eps_stop (max over all steps and cells), the ADMM stop
    // of Alg:outter, which the paper applies to both optimisers (Sec. 5).
    // Buffers are allocated on the first
    // call and freed with the context.  Returns the iterations done, -1 when
    // the buffers cannot be allocated, -2 for a non-finite objective.
    static constexpr int LB_M = 8;
    T* lb = nullptr;
    static constexpr int LB_R = LB_M + 1;   // ring slots: the newest pair is written into a free one
    T *lb_rho, *lb_rho_prev, *lb_v, *lb_x, *lb_g, *lb_xt, *lb_gt, *lb_d, *lb_s[LB_R], *lb_y[LB_R];
    T *lb_grho, *lb_grho2, *lb_gv, *lb_gw;
    T *lb_ys[ROT_PICARD] = {}, *lb_gy = nullptr, *lb_gb = nullptr;   // rotational step adjoint
    bool lb_alloc() {
        if (lb) return true;
        const long C = L[0].ncell, F = L[0].nface;
        Arena A;
        auto plan = [&](Arena& a) {
            lb_rho = a.take<T>((N + 1) * C);
            lb_rho_prev = a.take<T>((N + 1) * C);
            lb_v = a.take<T>((N + 1) * F);
            lb_x = a.take<T>(N * F);
            lb_g = a.take<T>(N * F);
            lb_xt = a.take<T>(N * F);
            lb_gt = a.take<T>(N * F);
            lb_d = a.take<T>(N * F);
            for (int k = 0; k < LB_R; ++k) {
                lb_s[k] = a.take<T>(N * F);
                lb_y[k] = a.take<T>(N * F);
            }
            lb_grho = a.take<T>(C);
            lb_grho2 = a.take<T>(C);
            lb_gv = a.take<T>(F);
            lb_gw = a.take<T>(F);
            if (P.vort) {
                for (int m = 0; m < ROT_PICARD; ++m) lb_ys[m] = a.take<T>(F);
                lb_gy = a.take<T>(F);
                lb_gb = a.take<T>(F);
            }
        };
        plan(A);
        if (hipMalloc((void**)&lb, A.off) != hipSuccess) {
            (void)hipGetLastError();
            lb = nullptr;
            return false;
        }
        Arena B;
        B.base = (char*)lb;
        plan(B);
        return true;
    }
    double lb_dot(const T* a, const T* b) {
        reduce(RED_DOT, (long)N * L[0].nface, a, b, 0, false);
        readback(1);
        return host_out[0];
    }
    // trajectory of u from (rho0, v = 0) into lb_rho, lb_v; returns J(u)
    double lb_forward(const T* rho0, const T* u, int nk, const int* ks, const T* keys) {
        const long C = L[0].ncell, F = L[0].nface;
        fill(lb_v, F, (T)0);
        for (int i = 0; i < N; ++i) {
            if (P.vort) {
                // the implicit rotational update: ROT_PICARD fixed-point steps from Q(v + dt u)
                T* vn = lb_v + (i + 1) * F;
                rot_rhs(lb_v + i * F, u + i * F, nullptr, rs_w);
                project(rs_w, vn, nullptr, 1);
                for (int m = 0; m < ROT_PICARD; ++m) {
                    rot_rhs(lb_v + i * F, u + i * F, vn, rs_w);
                    project(rs_w, vn, nullptr, 1);
                }
                continue;
            }
            self_advect(0, lb_v + i * F, u + i * F, rs_w, 1);
            project(rs_w, lb_v + (i + 1) * F, nullptr, 1);
        }
        forward_sweep(rho0, lb_v, lb_rho, &lb_k);        // the densities follow the velocities
        zero_slots(2);
        for (int q = 0; q < nk; ++q) {
            axpby(C, (T)1, lb_rho + (long)ks[q] * C, (T)-1, keys + q * C, ce_e);
            metric(ce_e, ce_acc);
            reduce(RED_DOT, C, ce_e, ce_acc, 0, true);
        }
        reduce(RED_SUMSQ_DIFF, N * F, u, nullptr, 1, false);
        readback(2);
        return 0.5 * host_out[0] + 0.5 * P.r * host_out[1];
    }
    // gradient of J at the trajectory in lb_rho, lb_v into gout
    void lb_gradient(const T* u, int nk, const int* ks, const T* keys, T* gout) {
        const long C = L[0].ncell, F = L[0].nface;
        fill(lb_grho, C, (T)0);
        fill(lb_gv, F, (T)0);
        for (int i = N; i >= 1; --i) {
            for (int q = 0; q < nk; ++q)
                if (ks[q] == i) {
                    axpby(C, (T)1, lb_rho + (long)i * C, (T)-1, keys + q * C, ce_e);
                    metric(ce_e, ce_acc);
                    axpby(C, (T)1, lb_grho, (T)1, ce_acc, lb_grho);
                }
            const T* rho = lb_rho + (long)(i - 1) * C;
            const T* v = lb_v + (long)(i - 1) * F;
            if (P.vort) {
                // the adjoint of the fixed-point steps (as in the step's adjoint): their
                // iterates again, then g_w = Q g_y into g_b and g_y <- -dt J_Adv^T g_w
                const T* ui = u + (long)(i - 1) * F;
                rot_rhs(v, ui, nullptr, rs_w);
                project(rs_w, lb_ys[0], nullptr, 1);
                for (int m = 1; m < ROT_PICARD; ++m) {
                    rot_rhs(v, ui, lb_ys[m - 1], rs_w);
                    project(rs_w, lb_ys[m], nullptr, 1);
                }
                rot_adj(nullptr, lb_gv, lb_gy);
                fill(lb_gb, F, (T)0);
                for (int m = ROT_PICARD; m >= 0; --m) {
                    project(lb_gy, lb_gw, nullptr, 1);
                    axpby(F, (T)1, lb_gw, (T)1, lb_gb, lb_gb);
                    if (m > 0) rot_adj(lb_ys[m - 1], lb_gw, lb_gy);
                }
                axpby(F, (T)P.dt, lb_gb, (T)0, nullptr, gout + (long)(i - 1) * F);   // g_u = dt g_b
                fill(lb_grho2, C, (T)0);
                dens_adj(lb_grho, rho, v, lb_grho2, lb_gv, nullptr, (T)1,
                         (int)lb_k.size() == N ? lb_k[i - 1] : -1);             // (dA/drho)^T, (dA/dv)^T g_rho'
                axpby(F, (T)1, lb_gb, (T)1, lb_gv, lb_gv);                          // + g_b
                std::swap(lb_grho, lb_grho2);
                continue;
            }
            project(lb_gv, lb_gw, nullptr, 1);                                   // g_w = Q g_v'
            axpby(F, (T)P.dt, lb_gw, (T)0, nullptr, gout + (long)(i - 1) * F);   // g_u = dt g_w
            fill(lb_grho2, C, (T)0);
            dens_adj(lb_grho, rho, v, lb_grho2, lb_gv, nullptr, (T)1,
                     (int)lb_k.size() == N ? lb_k[i - 1] : -1);                 // (dA/drho)^T, (dA/dv)^T g_rho'
            self_advect_T(0, v, lb_gw, (T)1, lb_gv, 1);                          // + J_S^T g_w
            std::swap(lb_grho, lb_grho2);
        }
        axpby(N * F, (T)1, gout, (T)P.r, u, gout);                               // + r u
    }
    int lbfgs(const void* rho0v, int nk, const int* ks, const void* keysv, void* uv, int iters, double eps_stop,
              double* hist) override {
        const T* rho0 = (const T*)rho0v;
        const T* keys = (const T*)keysv;
        T* u = (T*)uv;
        const long n = (long)N * L[0].nface;
        if (!lb_alloc()) return -1;
        copy(lb_x, u, n);
        double f = lb_forward(rho0, lb_x, nk, ks, keys);
        lb_gradient(lb_x, nk, ks, keys, lb_g);
        if (hist) hist[0] = f;
        int ns = 0, head = 0, done = 0;    // ns stored pairs; the newest at head - 1, slot head free
        double rho_s[LB_R];
        for (int it = 0; it < iters; ++it) {
            // two-loop recursion: d = -H g
            copy(lb_d, lb_g, n);
            double al[LB_M];
            for (int k = 0; k < ns; ++k) {
                const int sl = (head - 1 - k + LB_R) % LB_R;
                al[k] = rho_s[sl] * lb_dot(lb_s[sl], lb_d);
                axpby(n, (T)1, lb_d, (T)(-al[k]), lb_y[sl], lb_d);
            }
            double gamma;
            if (ns > 0) {
                const int sl = (head - 1 + LB_R) % LB_R;
                gamma = lb_dot(lb_s[sl], lb_y[sl]) / lb_dot(lb_y[sl], lb_y[sl]);
            } else {
                gamma = 1.0 / std::max(std::sqrt(lb_dot(lb_g, lb_g)), 1e-300);
            }
            axpby(n, (T)gamma, lb_d, (T)0, nullptr, lb_d);
            for (int k = ns - 1; k >= 0; --k) {
                const int sl = (head - 1 - k + LB_R) % LB_R;
                const double b = rho_s[sl] * lb_dot(lb_y[sl], lb_d);
                axpby(n, (T)1, lb_d, (T)(al[k] - b), lb_s[sl], lb_d);
            }
            axpby(n, (T)-1, lb_d, (T)0, nullptr, lb_d);
            const double slope = lb_dot(lb_g, lb_d);
            if (!(slope < 0)) break;
            if (eps_stop > 0) copy(lb_rho_prev, lb_rho, (N + 1) * L[0].ncell);
            // Armijo backtracking
            double alpha = 1.0, ft = 0;
            bool ok = false;
            for (int h = 0; h <= 20; ++h) {
                axpby(n, (T)1, lb_x, (T)alpha, lb_d, lb_xt);
                ft = lb_forward(rho0, lb_xt, nk, ks, keys);
                if (ft <= f + 1e-4 * alpha * slope) {
                    ok = true;
                    break;
                }
                alpha *= 0.5;
            }
            if (!ok) break;
            bool stop = false;
            if (eps_stop > 0) {                      // lb_rho holds the accepted trajectory
                reduce(RED_MAXABS_DIFF, (N + 1) * L[0].ncell, lb_rho, lb_rho_prev, 0, false);
                readback(1);
                stop = host_out[0] <= eps_stop;
            }
            if (stop) {
                std::swap(lb_x, lb_xt);
                f = ft;
                ++done;
                if (hist) hist[done] = f;
                break;
            }
            lb_gradient(lb_xt, nk, ks, keys, lb_gt);
            // new pair s = xt - x, y = gt - g
            T* sn = lb_s[head];
            T* yn = lb_y[head];
            axpby(n, (T)1, lb_xt, (T)-1, lb_x, sn);
            axpby(n, (T)1, lb_gt, (T)-1, lb_g, yn);
            const double ys = lb_dot(yn, sn);
            const double nss = lb_dot(sn, sn), nyy = lb_dot(yn, yn);
            if (ys > 1e-12 * std::sqrt(nss) * std::sqrt(nyy)) {
                rho_s[head] = 1.0 / ys;
                head = (head + 1) % LB_R;
                ns = std::min(ns + 1, LB_M);
            }
            std::swap(lb_x, lb_xt);
            std::swap(lb_g, lb_gt);
            f = ft;
            ++done;
            if (hist) hist[done] = f;
        }
        copy(u, lb_x, n);
        HCK(hipStreamSynchronize(st));
        return std::isfinite(f) ? done : -2;
    }

    // ------------------------------------------------------------ ADMM
    stfas_status solve(const void* rho0v, int nk, const int* ks, const void* keysv, void* u_out,
                       stfas_stats* stats) override {
        const auto t0 = std::chrono::steady_clock::now();
        const T* rho0 = (const T*)rho0v;
        const T* keys = (const T*)keysv;
        const long C = L[0].ncell, F = L[0].nface;
        Lev& q = lev[0];
        fill(q.v, N * F, (T)0);
        fill(q.pb, N * C, (T)0);
        fill(q.u, N * F, (T)0);
        fill(q.p, N * C, (T)0);
        fill(lam, N * F, (T)0);
        for (int i = 0; i <= N; ++i) copy(rho_last + i * C, rho0, C);
        double eps_admm = P.eps_admm;
        if (eps_admm <= 0) {
            reduce(RED_MAXABS_DIFF, C, rho0, nullptr, 0, false);
            readback(1);
            eps_admm = host_out[0] / 100.0;
        }
        const T invK = (T)(1.0 / P.K);
        int it = 0, conv = 0, vcs = 0, updates = 0;
        double last_res = 0, diff = 0, phi_prev = 0;
        std::vector<double> phis((size_t)P.ao_iters + 1);
        while (it < P.max_admm) {
            ++it;
            // vt = v + lambda/K (v_0 = 0)
            k_shift_combine<T><<<blocks_for(N * F, BS), BS, 0, st>>>(F, N, (T)1, q.v, invK, lam, (T)0, nullptr, vt);
            ao(rho0, nk, ks, keys, phis.data());
            // w = v* - lambda/K
            axpby(N * F, (T)1, vstar, -invK, lam, q.w);
            vcs += nso(nullptr, &last_res);
            if (!std::isfinite(last_res)) return STFAS_E_NONFINITE;
            reduce(RED_MAXABS_DIFF, (N + 1) * C, rho_last, rho, 0, false);
            readback(1);
            diff = host_out[0];
            if (!std::isfinite(diff)) return STFAS_E_NONFINITE;
            if (!P.fixed_counts && diff < eps_admm) {
                conv = 1;
                break;
            }
            copy(rho_last, rho, (N + 1) * C);
            // augmented-Lagrangian fallback: hold the multipliers while the density subproblem's
            // objective still falls by more than al_tol (relative) per iteration
            const double phi = phis[P.ao_iters];
            const bool update =
                !(P.al_tol > 0 && it > 1) || (phi_prev - phi) / std::max(std::fabs(phi_prev), 1e-300) <= P.al_tol;
            phi_prev = phi;
            if (update) {
                const T kb = (T)(P.K * P.beta);
                k_shift_combine<T><<<blocks_for(N * F, BS), BS, 0, st>>>(F, N, kb, q.v, (T)1, lam, -kb, vstar,
                                                                        lam);
                ++updates;
            }
        }
        copy((T*)u_out, q.u, N * F);
        // re-simulate and evaluate the objective
        zero_slots(3);
        copy(rs_rho[0], rho0, C);
        fill(rs_v[0], F, (T)0);
        int cur = 0;
        for (int i = 0; i < N; ++i) {
            dens_fwd(rs_rho[cur], rs_v[cur], rs_rho[cur ^ 1]);
            if (P.vort) {
                // the implicit update by ROT_PICARD fixed-point steps from Q(v + dt u)
                const Grid& g = L[0];
                k_rot_rhs<T, D><<<blocks_for(F, BS), BS, 0, st>>>(g, (T)P.dt, rs_v[cur], q.u + i * F, nullptr, rs_w);
                project(rs_w, rs_v[cur ^ 1], nullptr, 1);
                for (int m = 0; m < ROT_PICARD; ++m) {
                    k_rot_rhs<T, D><<<blocks_for(F, BS), BS, 0, st>>>(g, (T)P.dt, rs_v[cur], q.u + i * F,
                                                                    rs_v[cur ^ 1], rs_w);
                    project(rs_w, rs_v[cur ^ 1], nullptr, 1);
                }
            } else {
                self_advect(0, rs_v[cur], q.u + i * F, rs_w, 1);
                project(rs_w, rs_v[cur ^ 1], nullptr, 1);
            }
            cur ^= 1;
            for (int kq = 0; kq < nk; ++kq)
                if (ks[kq] == i + 1) {
                    axpby(C, (T)1, rs_rho[cur], (T)-1, keys + kq * C, ce_e);
                    metric(ce_e, ce_acc);
                    reduce(RED_DOT, C, ce_e, ce_acc, 0, true);
                    reduce(RED_SUMSQ_DIFF, C, ce_e, nullptr, 1, true);
                }
        }
        reduce(RED_SUMSQ_DIFF, N * F, q.u, nullptr, 2, false);
        readback(3);
        const double reg = 0.5 * P.r * host_out[2];
        if (stats) {
            stats->admm_iters = it;
            stats->vcycles = vcs;
            stats->converged = conv;
            stats->objective = 0.5 * host_out[0] + reg;
            stats->objective_l2 = 0.5 * host_out[1] + reg;
            stats->reg_term = reg;
            stats->kkt_res_inf = last_res;
            stats->visual_diff = diff;
            stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            stats->multiplier_updates = updates;
        }
        if (!std::isfinite(0.5 * host_out[0] + reg)) return STFAS_E_NONFINITE;
        return STFAS_OK;
    }

    // ------------------------------------------------------------ ops
    void op_advect(int batch, const void* r, const void* v, void* out) override {
        advect((const T*)r, (const T*)v, (T*)out, batch);
    }
    void op_advect_T(int batch, const void* m, const void* v, const void* add, void* out) override {
        const long C = L[0].ncell;
        if (add)
            copy((T*)out, (const T*)add, batch * C);
        else
            fill((T*)out, batch * C, (T)0);
        advect_T((const T*)m, (const T*)v, (T*)out, batch);
    }
    void op_advect_dv_T(int batch, const void* m, const void* r, const void* v, const void* vtt, double scale,
                        void* gv) override {
        advect_dv_T((const T*)m, (const T*)r, (const T*)v, (const T*)vtt, (T)scale, (T*)gv, batch);
    }
    bool has_upwind() const override { return upwind(); }
    // out = A(rho, v) with the upwind exponential; returns k (synchronises)
    int op_upwind(const void* r, const void* v, void* out) override {
        up.forward(L[0], P.dt, (const T*)r, (const T*)v, (T*)out, st);
        int k = -1;
        HCK(hipMemcpyAsync(&k, up.ctl.k, sizeof(int), hipMemcpyDeviceToHost, st));
        HCK(hipStreamSynchronize(st));
        return k;
    }
    // grho = (dA/drho)^T mu, gv = (dA/dv)^T mu (0 on walls)
    void op_upwind_adj(const void* m, const void* r, const void* v, void* grho, void* gv) override {
        fill((T*)grho, L[0].ncell, (T)0);
        up.adjoint(L[0], P.dt, (const T*)m, (const T*)r, (const T*)v, (T*)grho, (T*)gv, nullptr, (T)1, st);
    }
    void op_self_advect(int l, int batch, const void* v, const void* u, void* out) override {
        self_advect(l, (const T*)v, (const T*)u, (T*)out, batch);
    }
    void op_self_advect_T(int l, int batch, const void* v, const void* y, double scale, void* out) override {
        self_advect_T(l, (const T*)v, (const T*)y, (T)scale, (T*)out, batch);
    }
    int op_project(int batch, const void* w, void* out, void* phi) override {
        return project((const T*)w, (T*)out, (T*)phi, batch, 0, true);
    }
    void op_metric(const void* e, void* out) override { metric((const T*)e, (T*)out); }
    void op_kkt(int l, stfas_state x, const void* w, stfas_state res, stfas_state out) override {
        kkt(l, (const T*)x.v, (const T*)x.pbar, (const T*)x.u, (const T*)x.p, (const T*)w, (const T*)res.v,
            (const T*)res.pbar, (const T*)res.u, (const T*)res.p, (T*)out.v, (T*)out.pbar, (T*)out.u, (T*)out.p,
            (T)-1);
    }
    // Copy caller state into level l, run, copy back.
    void load(int l, stfas_state x, const void* w, const stfas_state* res) {
        const long F = L[l].nface, C = L[l].ncell;
        Lev& q = lev[l];
        copy(q.v, (const T*)x.v, N * F);
        copy(q.pb, (const T*)x.pbar, N * C);
        copy(q.u, (const T*)x.u, N * F);
        copy(q.p, (const T*)x.p, N * C);
        copy(q.w, (const T*)w, N * F);
        if (res && l > 0) {
            copy(q.s1, (const T*)res->v, N * F);
            copy(q.s2, (const T*)res->pbar, N * C);
            copy(q.s3, (const T*)res->u, N * F);
            copy(q.s4, (const T*)res->p, N * C);
        }
    }
    void store(int l, stfas_state x) {
        const long F = L[l].nface, C = L[l].ncell;
        Lev& q = lev[l];
        copy((T*)x.v, q.v, N * F);
        copy((T*)x.pbar, q.pb, N * C);
        copy((T*)x.u, q.u, N * F);
        copy((T*)x.p, q.p, N * C);
    }
    void op_sweep(int l, stfas_state x, const void* w, stfas_state res) override {
        load(l, x, w, &res);
        sweep(l);
        store(l, x);
    }
    void op_restrict(int l, stfas_state f, stfas_state c) override {
        restrict_faces(l, (const T*)f.v, (T*)c.v);
        restrict_cells(l, (const T*)f.pbar, (T*)c.pbar);
        restrict_faces(l, (const T*)f.u, (T*)c.u);
        restrict_cells(l, (const T*)f.p, (T*)c.p);
    }
    void op_prolong(int l, stfas_state c, double sign, stfas_state f) override {
        prolong_faces(l, (const T*)c.v, (T)sign, (T*)f.v);
        prolong_cells(l, (const T*)c.pbar, (T)sign, (T*)f.pbar);
        prolong_faces(l, (const T*)c.u, (T)sign, (T*)f.u);
        prolong_cells(l, (const T*)c.p, (T)sign, (T*)f.p);
    }
    int op_nso(stfas_state x, const void* w, double* hist) override {
        load(0, x, w, nullptr);
        const int n = nso(hist, nullptr);
        store(0, x);
        return n;
    }
    void op_ao(const void* rho0, int nk, const int* ks, const void* keys, const void* vtt, void* vs, void* r,
               double* hist) override {
        const long C = L[0].ncell, F = L[0].nface;
        copy(vt, (const T*)vtt, N * F);
        ao((const T*)rho0, nk, ks, (const T*)keys, hist);
        copy((T*)vs, vstar, N * F);
        copy((T*)r, rho, (N + 1) * C);
    }
};

// out = x + alpha (y - x), the blend of the density subproblem.
template <typename T>
__global__ void k_blend(long n, const T* __restrict__ x, const T* __restrict__ y, T alpha, T* __restrict__ out) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = x[e] + alpha * (y[e] - x[e]);
}

template <typename T, int D>
void Solver<T, D>::blend(const T* x, const T* y, T alpha, T* out, long n) {
    k_blend<T><<<blocks_for(n, BS), BS, 0, st>>>(n, x, y, alpha, out);
}

}  // namespace stfas
