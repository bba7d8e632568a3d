/*
 * stfas_ops.h - operator-level entry points of the same library.
 *
 * Each call runs one stage of the solver on caller buffers, with the
 * constants (grid, dt, K/r, N, precision) of a context made by stfas_create.
 * They exist so that every stage can be checked and timed on its own; the
 * solver itself uses the same kernels.  Layouts, dtype and ownership follow
 * stfas.h.  All calls are asynchronous on the context's stream unless noted,
 * return STFAS_E_INVALID for a bad level or batch before launching anything,
 * and write only their outputs.
 *
 * Level l in 0..stfas_num_levels()-1 selects the spatial multigrid level of
 * the velocity subproblem (grid n / 2^l, cell size 2^l h, Sec. 4.3); fields
 * passed at level l have that level's sizes.
 */
#ifndef STFAS_OPS_H
#define STFAS_OPS_H

#include "stfas.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Number of STFAS levels (coarsen by 2 while every n_a / 2^l >= 4, Sec. 4.3). */
int32_t stfas_num_levels(const stfas_ctx* ctx);
/* Cell and face counts of level l (0 if l is out of range). */
int64_t stfas_level_cells(const stfas_ctx* ctx, int32_t level);
int64_t stfas_level_faces(const stfas_ctx* ctx, int32_t level);

/* Semi-Lagrangian density advection (Sec. 3.1 eq:Conv, the operator A of
 * Sec. 4.1), batched over `batch` independent slices:
 *   out[b] = A(rho[b], v[b]) with backtrace Y = X - (dt/h) vbar.  Level 0 grid. */
stfas_status stfas_op_advect(stfas_ctx* ctx, int32_t batch, const void* rho, const void* v, void* out);

/* Its transposes (the partials in eq:KKTPO):
 *   out[b]  = W(v[b])^T mu[b] + add[b]          (add may be NULL)
 *   gv[b]   = vt[b] + (dA(rho[b], v[b])/dv)^T mu[b] * scale   (vt may be NULL) */
stfas_status stfas_op_advect_T(stfas_ctx* ctx, int32_t batch, const void* mu, const void* v, const void* add,
                               void* out);
stfas_status stfas_op_advect_dv_T(stfas_ctx* ctx, int32_t batch, const void* mu, const void* rho, const void* v,
                                  const void* vt, double scale, void* gv);

/* Upwind exponential density advection (Sec. 3.1 eq:Adv; the operator of
 * STFAS_DENSITY_UPWIND), one slice on the level 0 grid, for a context whose
 * problem selects it (otherwise STFAS_E_INVALID):
 *   out = sum_{j<=k} (dt^j/j!) A(v)^j rho;  *k_out (host, may be NULL) = k.
 * Synchronises (k is read back). */
stfas_status stfas_op_upwind(stfas_ctx* ctx, const void* rho, const void* v, void* out, int32_t* k_out);

/* Its partials at the same k (the series is linear in rho for fixed k):
 *   g_rho = (dA(rho, v)/drho)^T mu,  g_v = (dA(rho, v)/dv)^T mu (0 on walls).
 * Asynchronous. */
stfas_status stfas_op_upwind_adj(stfas_ctx* ctx, const void* mu, const void* rho, const void* v, void* g_rho,
                                 void* g_v);

/* Velocity self-advection on level l: out[b] = S(v[b]) + dt u[b] (u may be NULL). */
stfas_status stfas_op_self_advect(stfas_ctx* ctx, int32_t level, int32_t batch, const void* v, const void* u,
                                  void* out);
/* out[b] += scale * J_S(v[b])^T y[b] on level l (accumulates). */
stfas_status stfas_op_self_advect_T(stfas_ctx* ctx, int32_t level, int32_t batch, const void* v, const void* y,
                                    double scale, void* out);

/* Projection Q on the level-0 grid for `batch` independent slices
 * (Sec. 4.1): out = w - G phi with L phi = D w, mean(phi) = 0; phi may be
 * NULL.  Runs multigrid cycles until the relative residual of every slice
 * is <= poisson_rtol (synchronises); the cycle count goes to *cycles
 * (may be NULL).  batch <= N. */
stfas_status stfas_op_project(stfas_ctx* ctx, int32_t batch, const void* w, void* out, void* phi,
                              int32_t* cycles);

/* Keyframe metric (Sec. 4.1): out = C e on the level-0 grid. */
stfas_status stfas_op_metric(stfas_ctx* ctx, const void* e, void* out);

/* Spacetime state of one level: N slots each of v (faces), pbar (cells),
 * u (faces), p (cells); slot j holds v_{j+1}, pbar_{j+1}, u_j, p_{j+1}
 * (Sec. 4.2; v_0 = 0 is fixed).  The residual uses the same four arrays. */
typedef struct {
    void* v;
    void* pbar;
    void* u;
    void* p;
} stfas_state;

/* KKT residual of eq:KKTAO on level l: out = res - f(x) (res.* may be NULL
 * for zero).  w: targets [N][faces] with slot i = w_i. */
stfas_status stfas_op_kkt_residual(stfas_ctx* ctx, int32_t level, stfas_state x, const void* w, stfas_state res,
                                   stfas_state out);

/* One spacetime SCGS sweep (Sec. 4.3, eq:HESS; all 2^d colours) on level l,
 * updating x in place for f(x) = res. */
stfas_status stfas_op_scgs_sweep(stfas_ctx* ctx, int32_t level, stfas_state x, const void* w, stfas_state res);

/* Transfers between levels l and l+1 (Sec. 4.3):
 *   restrict: coarse = R fine (R = 2^-d P^T), all four arrays;
 *   prolong:  fine += sign * P coarse. */
stfas_status stfas_op_restrict(stfas_ctx* ctx, int32_t level, stfas_state fine, stfas_state coarse);
stfas_status stfas_op_prolong(stfas_ctx* ctx, int32_t level, stfas_state coarse, double sign, stfas_state fine);

/* Velocity subproblem (Alg:STFAS inside the NSO loop of Alg:outter) on
 * caller state x (level 0, updated in place) with targets w.  Runs V-cycles
 * until |f|_inf <= eps_stfas |f(0)|_inf or max_vcycles (exactly
 * max_vcycles if fixed_counts).  Writes the |f|_inf history (host, up to
 * max_vcycles + 1 entries) and returns the number of V-cycles in
 * *vcycles.  Synchronises. */
stfas_status stfas_op_nso(stfas_ctx* ctx, stfas_state x, const void* w, int32_t* vcycles, double* hist);

/* Density subproblem (Alg:Passive with the blending safeguard of Sec. 5):
 * from vt [N][faces] produce vstar [N][faces] and the accepted densities
 * rho [N+1][cells]; phi_hist (host, ao_iters + 1 entries) gets the objective
 * after each iteration.  Synchronises. */
stfas_status stfas_op_ao(stfas_ctx* ctx, const void* rho0, int32_t num_key, const int32_t* key_steps,
                         const void* key_rho, const void* vt, void* vstar, void* rho, double* phi_hist);

/* Event tracing of one kernel family (for roofline measurements): after
 * stfas_trace_enable(ctx, kernel, max_launches), up to max_launches
 * launches of that family on the finest level (level 0) made by later
 * calls on this context are
 * bracketed by HIP events on the context's stream, and the algorithmic
 * bytes each launch must move (its inputs and outputs once) are summed.
 * kernel = 0 disables tracing.  Families: 1 SCGS recurrence, 2 SCGS
 * projection, 3 KKT face and cell rows (one launch), 4 velocity-advection
 * transpose, 5 Poisson red-black sweep, 6 density advection, 7 (no
 * separate launch any more; records nothing), 8 SCGS pressure
 * (1, 2 and 8 run only for horizons too long for the fused kernel), 9 SCGS
 * whole-colour kernel (faces and pressure of one colour, time-parallel),
 * 10 the residual rows of one SCGS colour (in 2D with the velocity-advection
 * transpose in the same launch; in 3D the transpose is launched once per
 * sweep and counts as family 4), 11 the working terms (j >= 1) of the upwind
 * exponential density operator's series (a launch after the series has
 * stopped returns at once and is still counted).
 * stfas_trace_read synchronises and returns the recorded launch count,
 * their summed duration in milliseconds, their algorithmic bytes (for
 * family 10: the method's bytes of the rows the launch computes, 80 B per
 * spacetime cell in 2D and 108 B in 3D in FP32, twice that in FP64) and,
 * if impl_bytes is not NULL, the bytes of every buffer the launches read or
 * write once, the implementation's scratch included. */
stfas_status stfas_trace_enable(stfas_ctx* ctx, int32_t kernel, int32_t max_launches);
stfas_status stfas_trace_read(stfas_ctx* ctx, int64_t* launches, double* total_ms, double* bytes,
                              double* impl_bytes);

#ifdef __cplusplus
}
#endif
#endif /* STFAS_OPS_H */
