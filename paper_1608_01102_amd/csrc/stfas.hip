// C interface of the solver (include/stfas.h, include/stfas_ops.h).
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <tuple>

#include "solver.hpp"

using namespace stfas;

struct stfas_ctx {
    std::unique_ptr<SolverBase> s;
    int device = 0;
};

namespace {

template <typename F>
stfas_status guard(F&& f) {
    try {
        return f();
    } catch (const HipError&) {
        return STFAS_E_DEVICE;
    } catch (const std::bad_alloc&) {
        return STFAS_E_NOMEM;
    }
}

std::unique_ptr<SolverBase> make_solver(const Params& p, hipStream_t st) {
    if (p.precision == STFAS_FP64) {
        if (p.dim == 2) return std::make_unique<Solver<double, 2>>(p, st);
        return std::make_unique<Solver<double, 3>>(p, st);
    }
    if (p.dim == 2) return std::make_unique<Solver<float, 2>>(p, st);
    return std::make_unique<Solver<float, 3>>(p, st);
}

// ---------------------------------------------------------------- step engine
// Projection workspace for one slice carved from caller memory, with the
// coarsest-level pseudo-inverse cached per device and grid.
std::mutex g_pinv_mu;
std::map<std::tuple<int, int, int, int, int>, double*> g_pinv;

double* cached_pinv(const Grid& coarse, hipStream_t st) {
    int dev = 0;
    HCK(hipGetDevice(&dev));
    const auto key = std::make_tuple(dev, coarse.dim, coarse.n[0], coarse.n[1], coarse.n[2]);
    std::lock_guard<std::mutex> lk(g_pinv_mu);
    auto it = g_pinv.find(key);
    if (it != g_pinv.end()) return it->second;
    std::vector<double> pv;
    coarse_pinv(coarse, pv);
    double* d = nullptr;
    HCK(hipMalloc((void**)&d, pv.size() * sizeof(double)));
    HCK(hipMemcpy(d, pv.data(), pv.size() * sizeof(double), hipMemcpyHostToDevice));
    g_pinv[key] = d;
    return d;
}

int step_cycles(const Params& p) { return p.precision == STFAS_FP64 ? 24 : 10; }

template <typename T, int D>
struct Step {
    Grid g;
    Poisson<T, D> pois;
    T *w, *gw;
    T *ys[ROT_PICARD] = {}, *gy = nullptr, *gbase = nullptr;   // rotational adjoint: iterates, cotangents
    UpwindExp<T, D> up;
    bool upwind, vort;
    hipStream_t st;
    Step(const Params& p, hipStream_t s) : upwind(p.density == STFAS_DENSITY_UPWIND), vort(p.vort != 0), st(s) {
        const int n[3] = {p.n[0], p.n[1], p.n[2]};
        g = make_grid(p.dim, n, 1.0 / p.n[0]);
        pois.init(g, 1, s);
    }
    void layout(Arena& A, double* pinv) {
        pois.layout(A, pinv);
        w = A.take<T>(g.nface);
        gw = A.take<T>(g.nface);
        if (vort) {
            for (int m = 0; m < ROT_PICARD; ++m) ys[m] = A.take<T>(g.nface);
            gy = A.take<T>(g.nface);
            gbase = A.take<T>(g.nface);
        }
        if (upwind) up.layout(A, g.ncell);
    }
    size_t bytes() {
        Arena A;
        layout(A, (double*)1);
        return A.off;
    }

    void forward(const Params& p, const T* rho, const T* v, const T* u, T* rho_o, T* v_o, T* p_o) {
        const T cfl = (T)(p.dt / g.h);
        if (upwind)
            up.forward(g, p.dt, rho, v, rho_o, st);
        else
            k_advect<T, D><<<blocks_for(g.ncell, BS), BS, 0, st>>>(g, cfl, rho, v, rho_o, g.ncell, g.nface);
        if (p.vort) {
            // the implicit rotational update: ROT_PICARD fixed-point steps from Q(v + dt u)
            k_rot_rhs<T, D><<<blocks_for(g.nface, BS), BS, 0, st>>>(g, (T)p.dt, v, u, nullptr, w);
            pois.project(w, v_o, p_o, 1, p.poisson_rtol, step_cycles(p), nullptr);
            for (int m = 0; m < ROT_PICARD; ++m) {
                k_rot_rhs<T, D><<<blocks_for(g.nface, BS), BS, 0, st>>>(g, (T)p.dt, v, u, v_o, w);
                pois.project(w, v_o, p_o, 1, p.poisson_rtol, step_cycles(p), nullptr);
            }
        } else {
            k_self_advect<T, D><<<blocks_for(g.nface, BS), BS, 0, st>>>(g, cfl, (T)p.dt, v, u, w, g.nface);
            pois.project(w, v_o, p_o, 1, p.poisson_rtol, step_cycles(p), nullptr);
        }
        if (p_o) k_axpby<T><<<blocks_for(g.ncell, BS), BS, 0, st>>>(g.ncell, (T)(1.0 / p.dt), p_o, (T)0, nullptr, p_o);
    }

    void backward(const Params& p, const T* rho, const T* v, const T* grho_o, const T* gv_o, T* grho, T* gv,
                  T* gu, const T* u) {
        const T cfl = (T)(p.dt / g.h);
        if (vort) {
            backward_rotational(p, rho, v, u, grho_o, gv_o, grho, gv, gu);
            return;
        }
        pois.project(gv_o, gw, nullptr, 1, p.poisson_rtol, step_cycles(p), nullptr);       // g_w = Q g_v'
        k_axpby<T><<<blocks_for(g.nface, BS), BS, 0, st>>>(g.nface, (T)p.dt, gw, (T)0, nullptr, gu);
        // g_v = (dA/dv)^T g_rho' + J_S^T g_w,  g_rho = (dA/drho)^T g_rho'
        k_fill<T><<<blocks_for(g.ncell, BS), BS, 0, st>>>(g.ncell, grho, (T)0);
        if (upwind) {
            up.adjoint(g, p.dt, grho_o, rho, v, grho, gv, nullptr, (T)1, st);
        } else {
            k_advect_dv_T<T, D><<<blocks_for(g.nface, BS), BS, 0, st>>>(g, cfl, grho_o, rho, v, nullptr, (T)1, gv,
                                                                       g.ncell, g.nface);
            launch_advect_T<T, D>(g, cfl, grho_o, v, grho, 1, st);
        }
        launch_self_advect_T<T, D>(g, cfl, v, gw, (T)1, gv, 1, st);
    }

    // The adjoint of the rotational step's fixed-point steps as computed:
    // y_0 = Q(b), y_m = Q(b - dt Adv[y_{m-1}]) with b = v + dt u (walls 0),
    // v' = y_M.  Backward from g_y = g_v': g_w = Q g_y adds to g_b and
    // g_y <- -dt J_Adv(y_{m-1})^T g_w, for m = M .. 1, then g_w = Q g_y adds
    // to g_b; g_u = dt g_b, g_v = g_b + the density part.
    void backward_rotational(const Params& p, const T* rho, const T* v, const T* u, const T* grho_o,
                             const T* gv_o, T* grho, T* gv, T* gu) {
        const T cfl = (T)(p.dt / g.h), dt = (T)p.dt;
        const int nb = blocks_for(g.nface, BS);
        k_rot_rhs<T, D><<<nb, BS, 0, st>>>(g, dt, v, u, nullptr, w);
        pois.project(w, ys[0], nullptr, 1, p.poisson_rtol, step_cycles(p), nullptr);
        for (int m = 1; m < ROT_PICARD; ++m) {
            k_rot_rhs<T, D><<<nb, BS, 0, st>>>(g, dt, v, u, ys[m - 1], w);
            pois.project(w, ys[m], nullptr, 1, p.poisson_rtol, step_cycles(p), nullptr);
        }
        k_rot_adj<T, D><<<nb, BS, 0, st>>>(g, dt, nullptr, gv_o, gy);        // g_y = g_v' (walls 0)
        k_fill<T><<<nb, BS, 0, st>>>(g.nface, gbase, (T)0);
        for (int m = ROT_PICARD; m >= 0; --m) {
            pois.project(gy, gw, nullptr, 1, p.poisson_rtol, step_cycles(p), nullptr);
            k_axpby<T><<<nb, BS, 0, st>>>(g.nface, (T)1, gw, (T)1, gbase, gbase);
            if (m > 0) k_rot_adj<T, D><<<nb, BS, 0, st>>>(g, dt, ys[m - 1], gw, gy);
        }
        k_axpby<T><<<nb, BS, 0, st>>>(g.nface, dt, gbase, (T)0, nullptr, gu);
        k_fill<T><<<blocks_for(g.ncell, BS), BS, 0, st>>>(g.ncell, grho, (T)0);
        if (upwind) {
            up.adjoint(g, p.dt, grho_o, rho, v, grho, gv, nullptr, (T)1, st);
        } else {
            k_advect_dv_T<T, D><<<nb, BS, 0, st>>>(g, cfl, grho_o, rho, v, nullptr, (T)1, gv, g.ncell, g.nface);
            launch_advect_T<T, D>(g, cfl, grho_o, v, grho, 1, st);
        }
        k_axpby<T><<<nb, BS, 0, st>>>(g.nface, (T)1, gbase, (T)1, gv, gv);
    }
};

// Scratch of the allocation-free forward step: the coarsest level's
// pseudo-inverse (m x m doubles) followed by the step's own buffers.  The
// array lives once per device for the life of the process; host code only
// ever uses its device address from hipGetSymbolAddress (the array's name is
// a host-side stand-in there).
__device__ __align__(256) char scratch[STFAS_NOALLOC_SCRATCH_BYTES];

struct NoallocDevice {
    char* ptr = nullptr;      // device address of `scratch` on this device
    Grid pinv_grid{};         // coarse grid whose pseudo-inverse the scratch holds
    bool pinv_valid = false;
};
std::mutex g_noalloc_mu;
std::map<int, NoallocDevice> g_noalloc;
// host copies of the coarse pseudo-inverses, kept for the life of the process
// (an asynchronous upload reads them after the call returns)
std::map<std::tuple<int, int, int, int>, std::vector<double>> g_pinv_host;

size_t pinv_bytes(const Grid& coarse) {
    const size_t b = (size_t)coarse.ncell * coarse.ncell * sizeof(double);
    return (b + 255) & ~(size_t)255;
}

bool same_grid(const Grid& a, const Grid& b) {
    return a.dim == b.dim && a.n[0] == b.n[0] && a.n[1] == b.n[1] && a.n[2] == b.n[2];
}

// The device address of `scratch` on the current device, fetched once per
// device; with `coarse` set, also makes sure its head holds that grid's
// pseudo-inverse (uploaded on `st` when another grid's is there).
char* noalloc_scratch(const Grid& coarse, hipStream_t st) {
    int dev = 0;
    HCK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    NoallocDevice& nd = g_noalloc[dev];
    if (!nd.ptr) {
        void* ptr = nullptr;
        HCK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        nd.ptr = (char*)ptr;
    }
    if (!nd.pinv_valid || !same_grid(nd.pinv_grid, coarse)) {
        auto& pv = g_pinv_host[std::make_tuple(coarse.dim, coarse.n[0], coarse.n[1], coarse.n[2])];
        if (pv.empty()) coarse_pinv(coarse, pv);
        HCK(hipMemcpyAsync(nd.ptr, pv.data(), pv.size() * sizeof(double), hipMemcpyHostToDevice, st));
        nd.pinv_grid = coarse;
        nd.pinv_valid = true;
    }
    return nd.ptr;
}

template <typename T, int D>
stfas_status run_step(const Params& p, hipStream_t st, void* work, bool fwd, const void* a0, const void* a1,
                      const void* a2, const void* a3, void* o0, void* o1, void* o2, bool noalloc = false,
                      const void* a4 = nullptr) {
    Step<T, D> s(p, st);
    if (!s.pois.coarse_ok()) return STFAS_E_INVALID;
    Arena A;
    double* pinv = nullptr;
    if (noalloc) {
        const Grid& coarse = s.pois.PG.back();
        const size_t head = pinv_bytes(coarse);
        if (head + s.bytes() > (size_t)STFAS_NOALLOC_SCRATCH_BYTES) return STFAS_E_INVALID;
        char* base = noalloc_scratch(coarse, st);
        pinv = (double*)base;
        A.base = base + head;
    } else {
        A.base = (char*)work;
        pinv = cached_pinv(s.pois.PG.back(), st);
    }
    s.layout(A, pinv);
    if (fwd)
        s.forward(p, (const T*)a0, (const T*)a1, (const T*)a2, (T*)o0, (T*)o1, (T*)o2);
    else
        s.backward(p, (const T*)a0, (const T*)a1, (const T*)a2, (const T*)a3, (T*)o0, (T*)o1, (T*)o2, (const T*)a4);
    HCK(hipPeekAtLastError());
    return STFAS_OK;
}

stfas_status dispatch_step(const Params& p, hipStream_t st, void* work, bool fwd, const void* a0, const void* a1,
                           const void* a2, const void* a3, void* o0, void* o1, void* o2, bool noalloc = false,
                           const void* a4 = nullptr) {
    if (p.precision == STFAS_FP64) {
        if (p.dim == 2) return run_step<double, 2>(p, st, work, fwd, a0, a1, a2, a3, o0, o1, o2, noalloc, a4);
        return run_step<double, 3>(p, st, work, fwd, a0, a1, a2, a3, o0, o1, o2, noalloc, a4);
    }
    if (p.dim == 2) return run_step<float, 2>(p, st, work, fwd, a0, a1, a2, a3, o0, o1, o2, noalloc, a4);
    return run_step<float, 3>(p, st, work, fwd, a0, a1, a2, a3, o0, o1, o2, noalloc, a4);
}

size_t step_bytes(const Params& p) {
    if (p.precision == STFAS_FP64) {
        if (p.dim == 2) return Step<double, 2>(p, nullptr).bytes();
        return Step<double, 3>(p, nullptr).bytes();
    }
    if (p.dim == 2) return Step<float, 2>(p, nullptr).bytes();
    return Step<float, 3>(p, nullptr).bytes();
}

}  // namespace

extern "C" {

const char* stfas_status_string(stfas_status s) {
    switch (s) {
        case STFAS_OK: return "ok";
        case STFAS_E_INVALID: return "invalid argument";
        case STFAS_E_NOMEM: return "out of device memory";
        case STFAS_E_DEVICE: return "HIP error";
        case STFAS_E_NONFINITE: return "non-finite value";
    }
    return "unknown status";
}

const char* stfas_build_info(void) { return "stfas HIP/CDNA4 gfx950 build; fp64 and mixed fp32/fp64 paths"; }

size_t stfas_workspace_bytes(const stfas_problem* prob) {
    Params p;
    if (!resolve(prob, p)) return 0;
    auto s = make_solver(p, nullptr);
    if (!s->valid()) return 0;
    return s->plan();
}

stfas_status stfas_create(const stfas_problem* prob, void* hip_stream, stfas_ctx** out) {
    if (!out) return STFAS_E_INVALID;
    *out = nullptr;
    Params p;
    if (!resolve(prob, p)) return STFAS_E_INVALID;
    return guard([&]() -> stfas_status {
        auto c = std::make_unique<stfas_ctx>();
        c->s = make_solver(p, (hipStream_t)hip_stream);
        if (!c->s->valid()) return STFAS_E_INVALID;
        HCK(hipGetDevice(&c->device));
        const size_t bytes = c->s->plan();
        char* mem = nullptr;
        if (hipMalloc((void**)&mem, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return STFAS_E_NOMEM;
        }
        c->s->mem = mem;
        c->s->bytes = bytes;
        c->s->carve(mem);
        c->s->init_tables();
        *out = c.release();
        return STFAS_OK;
    });
}

stfas_status stfas_create_in(const stfas_problem* prob, void* hip_stream, void* workspace, size_t workspace_bytes,
                             stfas_ctx** out) {
    if (!out) return STFAS_E_INVALID;
    *out = nullptr;
    Params p;
    if (!resolve(prob, p) || !workspace || (reinterpret_cast<uintptr_t>(workspace) & 255u)) return STFAS_E_INVALID;
    return guard([&]() -> stfas_status {
        auto c = std::make_unique<stfas_ctx>();
        c->s = make_solver(p, (hipStream_t)hip_stream);
        if (!c->s->valid()) return STFAS_E_INVALID;
        const size_t bytes = c->s->plan();
        if (workspace_bytes < bytes) return STFAS_E_INVALID;
        HCK(hipGetDevice(&c->device));
        c->s->mem = (char*)workspace;
        c->s->bytes = bytes;
        c->s->owns_mem = false;
        c->s->carve((char*)workspace);
        c->s->init_tables();
        *out = c.release();
        return STFAS_OK;
    });
}

void stfas_destroy(stfas_ctx* ctx) {
    if (!ctx) return;
    if (ctx->s && ctx->s->mem) {
        (void)hipStreamSynchronize(ctx->s->st);
        if (ctx->s->owns_mem) (void)hipFree(ctx->s->mem);
    }
    delete ctx;
}

static bool valid_keys(const stfas_ctx* ctx, int32_t num_key, const int32_t* key_steps, const void* key_rho) {
    if (num_key < 0) return false;
    if (num_key > 0 && (!key_steps || !key_rho)) return false;
    for (int q = 0; q < num_key; ++q) {
        if (key_steps[q] < 1 || key_steps[q] > ctx->s->P.N) return false;
        if (q > 0 && key_steps[q] <= key_steps[q - 1]) return false;
    }
    return true;
}

stfas_status stfas_solve(stfas_ctx* ctx, const void* rho0, int32_t num_key, const int32_t* key_steps,
                         const void* key_rho, void* u_out, stfas_stats* stats) {
    if (!ctx || !rho0 || !u_out) return STFAS_E_INVALID;
    if (!valid_keys(ctx, num_key, key_steps, key_rho)) return STFAS_E_INVALID;
    return guard([&]() -> stfas_status {
        const stfas_status s = ctx->s->solve(rho0, num_key, key_steps, key_rho, u_out, stats);
        HCK(hipPeekAtLastError());
        HCK(hipStreamSynchronize(ctx->s->st));
        return s;
    });
}

stfas_status stfas_lbfgs(stfas_ctx* ctx, const void* rho0, int32_t num_key, const int32_t* key_steps,
                         const void* key_rho, void* u_inout, int32_t iters, double eps_stop, int32_t* iters_done,
                         double* J_hist) {
    if (!ctx || !rho0 || !u_inout || iters < 0 || !(eps_stop >= 0)) return STFAS_E_INVALID;
    if (!valid_keys(ctx, num_key, key_steps, key_rho)) return STFAS_E_INVALID;
    if (!ctx->s->owns_mem) return STFAS_E_INVALID;
    return guard([&]() -> stfas_status {
        const int done = ctx->s->lbfgs(rho0, num_key, key_steps, key_rho, u_inout, iters, eps_stop, J_hist);
        HCK(hipPeekAtLastError());
        HCK(hipStreamSynchronize(ctx->s->st));
        if (done == -1) return STFAS_E_NOMEM;
        if (iters_done) *iters_done = done < 0 ? 0 : done;
        return done == -2 ? STFAS_E_NONFINITE : STFAS_OK;
    });
}

size_t stfas_step_work_bytes(const stfas_problem* prob) {
    Params p;
    if (!resolve(prob, p)) return 0;
    return step_bytes(p);
}

int32_t stfas_step_vcycles(const stfas_problem* prob) {
    Params p;
    if (!resolve(prob, p)) return 0;
    return step_cycles(p);
}

stfas_status stfas_step_forward(const stfas_problem* prob, void* hip_stream, const void* rho, const void* v,
                                const void* u, void* rho_out, void* v_out, void* p_out, void* work) {
    Params p;
    if (!resolve(prob, p)) return STFAS_E_INVALID;
    if (!rho || !v || !u || !rho_out || !v_out || !work) return STFAS_E_INVALID;
    return guard([&]() {
        return dispatch_step(p, (hipStream_t)hip_stream, work, true, rho, v, u, nullptr, rho_out, v_out, p_out);
    });
}

stfas_status stfas_step_forward_noalloc(const stfas_problem* prob, void* hip_stream, const void* rho, const void* v,
                                        const void* u, void* rho_out, void* v_out, void* p_out) {
    Params p;
    if (!resolve(prob, p)) return STFAS_E_INVALID;
    if (!rho || !v || !u || !rho_out || !v_out) return STFAS_E_INVALID;
    return guard([&]() {
        return dispatch_step(p, (hipStream_t)hip_stream, nullptr, true, rho, v, u, nullptr, rho_out, v_out, p_out,
                             true);
    });
}

stfas_status stfas_step_backward(const stfas_problem* prob, void* hip_stream, const void* rho, const void* v,
                                 const void* g_rho_out, const void* g_v_out, void* g_rho, void* g_v, void* g_u,
                                 void* work) {
    Params p;
    if (!resolve(prob, p) || p.vort) return STFAS_E_INVALID;
    if (!rho || !v || !g_rho_out || !g_v_out || !g_rho || !g_v || !g_u || !work) return STFAS_E_INVALID;
    return guard([&]() {
        return dispatch_step(p, (hipStream_t)hip_stream, work, false, rho, v, g_rho_out, g_v_out, g_rho, g_v, g_u);
    });
}

stfas_status stfas_step_backward_u(const stfas_problem* prob, void* hip_stream, const void* rho, const void* v,
                                   const void* u, const void* g_rho_out, const void* g_v_out, void* g_rho, void* g_v,
                                   void* g_u, void* work) {
    Params p;
    if (!resolve(prob, p)) return STFAS_E_INVALID;
    if (!rho || !v || !u || !g_rho_out || !g_v_out || !g_rho || !g_v || !g_u || !work) return STFAS_E_INVALID;
    return guard([&]() {
        return dispatch_step(p, (hipStream_t)hip_stream, work, false, rho, v, g_rho_out, g_v_out, g_rho, g_v, g_u,
                             false, u);
    });
}

// ---------------------------------------------------------------- operator level
int32_t stfas_num_levels(const stfas_ctx* ctx) { return ctx ? ctx->s->nlevels() : 0; }

int64_t stfas_level_cells(const stfas_ctx* ctx, int32_t level) {
    if (!ctx || level < 0 || level >= ctx->s->nlevels()) return 0;
    return ctx->s->level(level).ncell;
}

int64_t stfas_level_faces(const stfas_ctx* ctx, int32_t level) {
    if (!ctx || level < 0 || level >= ctx->s->nlevels()) return 0;
    return ctx->s->level(level).nface;
}

static bool ok_batch(const stfas_ctx* ctx, int32_t batch) { return ctx && batch >= 1 && batch <= 65535; }
static bool ok_level(const stfas_ctx* ctx, int32_t l) { return ctx && l >= 0 && l < ctx->s->nlevels(); }

#define OP_BODY(stmt)                     \
    return guard([&]() -> stfas_status { \
        stmt;                             \
        HCK(hipPeekAtLastError());        \
        return STFAS_OK;                  \
    })

stfas_status stfas_op_advect(stfas_ctx* ctx, int32_t batch, const void* rho, const void* v, void* out) {
    if (!ok_batch(ctx, batch) || !rho || !v || !out) return STFAS_E_INVALID;
    OP_BODY(ctx->s->op_advect(batch, rho, v, out));
}

stfas_status stfas_op_advect_T(stfas_ctx* ctx, int32_t batch, const void* mu, const void* v, const void* add,
                               void* out) {
    if (!ok_batch(ctx, batch) || !mu || !v || !out) return STFAS_E_INVALID;
    OP_BODY(ctx->s->op_advect_T(batch, mu, v, add, out));
}

stfas_status stfas_op_advect_dv_T(stfas_ctx* ctx, int32_t batch, const void* mu, const void* rho, const void* v,
                                  const void* vt, double scale, void* gv) {
    if (!ok_batch(ctx, batch) || !mu || !rho || !v || !gv) return STFAS_E_INVALID;
    OP_BODY(ctx->s->op_advect_dv_T(batch, mu, rho, v, vt, scale, gv));
}

stfas_status stfas_op_upwind(stfas_ctx* ctx, const void* rho, const void* v, void* out, int32_t* k_out) {
    if (!ctx || !rho || !v || !out || !ctx->s->has_upwind()) return STFAS_E_INVALID;
    return guard([&]() -> stfas_status {
        const int k = ctx->s->op_upwind(rho, v, out);
        HCK(hipPeekAtLastError());
        if (k_out) *k_out = k;
        return STFAS_OK;
    });
}

stfas_status stfas_op_upwind_adj(stfas_ctx* ctx, const void* mu, const void* rho, const void* v, void* g_rho,
                                 void* g_v) {
    if (!ctx || !mu || !rho || !v || !g_rho || !g_v || !ctx->s->has_upwind()) return STFAS_E_INVALID;
    OP_BODY(ctx->s->op_upwind_adj(mu, rho, v, g_rho, g_v));
}

stfas_status stfas_op_self_advect(stfas_ctx* ctx, int32_t level, int32_t batch, const void* v, const void* u,
                                  void* out) {
    if (!ok_batch(ctx, batch) || !ok_level(ctx, level) || !v || !out) return STFAS_E_INVALID;
    OP_BODY(ctx->s->op_self_advect(level, batch, v, u, out));
}

stfas_status stfas_op_self_advect_T(stfas_ctx* ctx, int32_t level, int32_t batch, const void* v, const void* y,
                                    double scale, void* out) {
    if (!ok_batch(ctx, batch) || !ok_level(ctx, level) || !v || !y || !out) return STFAS_E_INVALID;
    OP_BODY(ctx->s->op_self_advect_T(level, batch, v, y, scale, out));
}

stfas_status stfas_op_project(stfas_ctx* ctx, int32_t batch, const void* w, void* out, void* phi, int32_t* cycles) {
    if (!ok_batch(ctx, batch) || batch > ctx->s->P.N || !w || !out) return STFAS_E_INVALID;
    return guard([&]() -> stfas_status {
        const int c = ctx->s->op_project(batch, w, out, phi);
        if (cycles) *cycles = c;
        HCK(hipPeekAtLastError());
        return STFAS_OK;
    });
}

stfas_status stfas_op_metric(stfas_ctx* ctx, const void* e, void* out) {
    if (!ctx || !e || !out) return STFAS_E_INVALID;
    OP_BODY(ctx->s->op_metric(e, out));
}

static bool ok_state(const stfas_state& x) { return x.v && x.pbar && x.u && x.p; }

stfas_status stfas_op_kkt_residual(stfas_ctx* ctx, int32_t level, stfas_state x, const void* w, stfas_state res,
                                   stfas_state out) {
    if (!ok_level(ctx, level) || !ok_state(x) || !ok_state(out) || !w) return STFAS_E_INVALID;
    OP_BODY(ctx->s->op_kkt(level, x, w, res, out));
}

stfas_status stfas_op_scgs_sweep(stfas_ctx* ctx, int32_t level, stfas_state x, const void* w, stfas_state res) {
    if (!ok_level(ctx, level) || !ok_state(x) || !w) return STFAS_E_INVALID;
    if (level > 0 && !ok_state(res)) return STFAS_E_INVALID;
    if (level == 0 && (res.v || res.pbar || res.u || res.p)) return STFAS_E_INVALID;
    OP_BODY(ctx->s->op_sweep(level, x, w, res));
}

stfas_status stfas_op_restrict(stfas_ctx* ctx, int32_t level, stfas_state fine, stfas_state coarse) {
    if (!ctx || level < 0 || level + 1 >= ctx->s->nlevels() || !ok_state(fine) || !ok_state(coarse))
        return STFAS_E_INVALID;
    OP_BODY(ctx->s->op_restrict(level, fine, coarse));
}

stfas_status stfas_op_prolong(stfas_ctx* ctx, int32_t level, stfas_state coarse, double sign, stfas_state fine) {
    if (!ctx || level < 0 || level + 1 >= ctx->s->nlevels() || !ok_state(fine) || !ok_state(coarse))
        return STFAS_E_INVALID;
    OP_BODY(ctx->s->op_prolong(level, coarse, sign, fine));
}

stfas_status stfas_op_nso(stfas_ctx* ctx, stfas_state x, const void* w, int32_t* vcycles, double* hist) {
    if (!ctx || !ok_state(x) || !w) return STFAS_E_INVALID;
    return guard([&]() -> stfas_status {
        const int n = ctx->s->op_nso(x, w, hist);
        if (vcycles) *vcycles = n;
        HCK(hipPeekAtLastError());
        HCK(hipStreamSynchronize(ctx->s->st));
        return STFAS_OK;
    });
}

stfas_status stfas_op_ao(stfas_ctx* ctx, const void* rho0, int32_t num_key, const int32_t* key_steps,
                         const void* key_rho, const void* vt, void* vstar, void* rho, double* phi_hist) {
    if (!ctx || !rho0 || !vt || !vstar || !rho) return STFAS_E_INVALID;
    if (!valid_keys(ctx, num_key, key_steps, key_rho)) return STFAS_E_INVALID;
    return guard([&]() -> stfas_status {
        ctx->s->op_ao(rho0, num_key, key_steps, key_rho, vt, vstar, rho, phi_hist);
        HCK(hipPeekAtLastError());
        HCK(hipStreamSynchronize(ctx->s->st));
        return STFAS_OK;
    });
}

stfas_status stfas_trace_enable(stfas_ctx* ctx, int32_t kernel, int32_t max_launches) {
    if (!ctx || kernel < 0 || kernel > TR_UP_TERM || max_launches < 0 || max_launches > (1 << 20))
        return STFAS_E_INVALID;
    return guard([&]() -> stfas_status {
        HCK(hipStreamSynchronize(ctx->s->st));
        ctx->s->trace_enable(kernel, max_launches);
        return STFAS_OK;
    });
}

stfas_status stfas_trace_read(stfas_ctx* ctx, int64_t* launches, double* total_ms, double* bytes,
                              double* impl_bytes) {
    if (!ctx || !launches || !total_ms || !bytes) return STFAS_E_INVALID;
    return guard([&]() -> stfas_status {
        long n = 0;
        ctx->s->trace_read(&n, total_ms, bytes, impl_bytes);
        *launches = n;
        return STFAS_OK;
    });
}

}  // extern "C"
