/*
 * stfas.h - C interface of the MI355X spacetime-multigrid smoke-control solver.
 *
 * The solver computes the keyframe smoke-control problem of Pan & Manocha,
 * "Efficient Optimal Control of Smoke using Spacetime Multigrid"
 * (arXiv:1608.01102), Sec. 3.2 eq:opt:
 *
 *   minimise over u_0..u_{N-1}
 *     1/2 sum_t <rho_t - rho*_t, C (rho_t - rho*_t)>  +  r/2 sum_i |u_i|^2
 *   subject to the simulation step (Sec. 3.1 eq:NSA-eq:Conv, with
 *   semi-Lagrangian advection as allowed in Sec. 4.1):
 *     rho_{i+1} = A(rho_i, v_i),   v_{i+1} = Q(S(v_i) + dt u_i),   v_0 = 0,
 *
 * by the ADMM outer loop of Alg:outter: the density subproblem of Sec. 4.1
 * (Alg:Passive) and the velocity subproblem of Sec. 4.2, whose KKT system
 * (eq:KKTAO) is solved by the spacetime FAS V-cycle of Alg:STFAS with the
 * spacetime SCGS smoother of Sec. 4.3 (eq:HESS).  C is the Gaussian keyframe
 * metric of Sec. 4.1.
 *
 * Grid and layout (every pointer below uses it):
 *   dim in {2,3}, n = (n0, n1, n2) with n2 = 1 in 2D, cell size h = 1/n0.
 *   cells  [n2][n1][n0]                 (x fastest)
 *   faces  x | y | z concatenated, shapes [n2][n1][n0+1], [n2][n1+1][n0],
 *          [n2+1][n1][n0] (no z block in 2D); wall faces (index 0 or n_a
 *          along the normal) are stored and are always zero.
 *   a sequence of N fields is N consecutive fields (time major).
 *
 * Precision: STFAS_FP64 - every device buffer is double.  STFAS_MIXED -
 * every device buffer is float; the coarsest Poisson level and all
 * reductions (objective, line search, stop tests) run in double.
 *
 * Streams and ownership: all device pointers are caller-owned, contiguous
 * and on the device of the stream passed at creation.  The library keeps no
 * caller pointer after a call returns.  A context owns its workspace, which
 * is allocated in stfas_create and freed in stfas_destroy.  One context per
 * host thread; contexts on different streams may run concurrently.
 *
 * Errors: every call returns a status; nothing is thrown across the
 * interface.  Invalid arguments are rejected before any device work.
 */
#ifndef STFAS_H
#define STFAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stfas_ctx stfas_ctx;

typedef enum {
    STFAS_OK = 0,
    STFAS_E_INVALID = 1,   /* bad argument; nothing was launched */
    STFAS_E_NOMEM = 2,     /* device allocation failed */
    STFAS_E_DEVICE = 3,    /* a HIP call failed */
    STFAS_E_NONFINITE = 4  /* a reduction (objective, residual) was not finite */
} stfas_status;

typedef enum { STFAS_FP64 = 0, STFAS_MIXED = 1 } stfas_precision;

/* Density operator A(rho, v) of Sec. 3.1 eq:Conv.  Semi-Lagrangian: one
 * backtrace per cell and clamped multilinear interpolation.  Upwind
 * exponential (eq:Adv): sum_{j<=k} (dt^j/j!) A(v)^j rho with a flux-form
 * second-order upwind stencil A(v) and k the first j whose term has max norm
 * below 1e-5 (at most 48); Sec. 4.1 allows either, as long as the partials
 * in rho and v exist. */
typedef enum { STFAS_DENSITY_SL = 0, STFAS_DENSITY_UPWIND = 1 } stfas_density;

/* Velocity operator of the dynamics (Sec. 3.1 eq:NSA).  Semi-Lagrangian:
 * v_{i+1} = Q(S(v_i) + dt u_i) with the self-advection S.  Rotational: the
 * paper's implicit update (v_{i+1} - v_i)/dt + Adv[v_{i+1}] = u_i - G p_{i+1}
 * with Adv the vorticity form (curl v) x v, discretised with the vorticity
 * on the grid's edges (the nodes in 2D) and edge-paired face products so
 * that it does no work; the KKT residual is eq:KKTAO as printed
 * (du_{i-1}/dv_i = I/dt + dAdv/dv_i); the smoother's local matrix is
 * eq:HESS with the cell's block of dAdv/dv (Sec. 4.3, solved by block
 * elimination in time), by default on the finest level in 2D (scgs_local); the
 * re-simulation of the outputs (and stfas_step_forward) takes 4 fixed-point
 * steps per time step.  stfas_step_backward accepts only the semi-Lagrangian
 * operator (STFAS_E_INVALID otherwise); stfas_step_backward_u and stfas_lbfgs
 * take both (for the rotational operator the gradient is the adjoint of its
 * fixed-point steps as computed). */
typedef enum { STFAS_VELOCITY_SL = 0, STFAS_VELOCITY_ROTATIONAL = 1 } stfas_velocity;

/* Problem description (Sec. 3.2 eq:opt and the parameter table of Sec. 5).
 * A field <= 0 selects the documented default. */
typedef struct {
    int32_t dim;            /* 2 or 3 */
    int32_t n[3];           /* n0, n1, n2 (n2 = 1 in 2D); every n_a >= 4 */
    int32_t num_steps;      /* N >= 1 */
    double dt;              /* time step; default 1/n0 */
    double r;               /* control regularisation weight, > 0 (required) */
    double K;               /* ADMM penalty; default r / dt^2 */
    double beta;            /* multiplier step factor; default 1 */
    int32_t ao_iters;       /* fixed-point iterations of the density subproblem; default 2 */
    double eps_stfas;       /* relative KKT residual target |f| <= eps |f(0)|; default 1e-5 */
    double eps_admm;        /* stop when max_i |rho_i - rho_i^last|_inf < eps; default max(rho0)/100 */
    int32_t max_admm;       /* ADMM iteration cap; default 50 */
    int32_t max_vcycles;    /* V-cycles per velocity subproblem cap; default 30 */
    int32_t metric_levels;  /* Gaussian filters in C; < 0 selects largest L with 2^(L-1) <= min(n)/8 */
    double poisson_rtol;    /* projection relative residual; default 1e-13 (FP64) / 1e-6 (MIXED) */
    int32_t fixed_counts;   /* 1: ignore eps_*, run exactly max_admm and max_vcycles (parity mode) */
    int32_t precision;      /* stfas_precision */
    double scgs_omega;      /* relaxation weight of the SCGS smoother (Sec. 4.3), in (0, 2]; <= 0 selects 0.7
                             * (1 with the rotational velocity operator) */
    int32_t density_op;     /* stfas_density; 0 = semi-Lagrangian */
    double al_tol;          /* augmented-Lagrangian fallback of the ADMM loop (Sec. 5, convergence
                             * analysis): > 0 makes the multiplier update of an iteration t > 1 only
                             * when the density subproblem's objective fell by at most al_tol
                             * (relative) since iteration t - 1; 0 = plain ADMM; < 0 invalid */
    double scgs_lm;         /* Levenberg-Marquardt perturbation of K in the smoother's local matrix
                             * (Sec. 5, convergence analysis; eq:HESS): K/r on every v block becomes
                             * K/r + scgs_lm / dt^2 (the residual is unchanged, so is the solution);
                             * 0 selects 1 (off where the rotational operator's smoother holds the
                             * local block, see scgs_local); < 0 turns it off */
    int32_t velocity_op;    /* stfas_velocity; 0 = semi-Lagrangian, 1 = rotational */
    int32_t scgs_local;     /* local matrix of the SCGS smoother with the rotational operator (Sec. 4.3
                             * eq:HESS): 1 = without the cell's block of dAdv/dv on every level
                             * (du_{i-1}/dv_i = I/dt, the scalar temporal solve of the semi-Lagrangian
                             * operator); 2 = with it on every level (block elimination in time);
                             * 3 = with it on the finest level only; 0 = 3 in 2D, 1 in 3D; other
                             * values invalid; must be 0 with the semi-Lagrangian operator */
} stfas_problem;

typedef struct {
    int32_t admm_iters;     /* ADMM iterations run */
    int32_t vcycles;        /* V-cycles run in total */
    int32_t converged;      /* 1 if the ADMM stop test fired */
    double objective;       /* J with the metric C, on the re-simulated trajectory */
    double objective_l2;    /* same with C replaced by the identity */
    double reg_term;        /* r/2 sum |u_i|^2 */
    double kkt_res_inf;     /* |f|_inf of the last velocity subproblem */
    double visual_diff;     /* last max_i |rho_i - rho_i^last|_inf */
    double seconds;         /* wall time of the solve */
    int32_t multiplier_updates; /* ADMM multiplier updates made (all iterations but a converged last
                                 * one, unless al_tol > 0 held some back) */
} stfas_stats;

/* Device bytes stfas_create allocates for this problem (exact); used for
 * admission control.  Returns 0 for an invalid problem. */
size_t stfas_workspace_bytes(const stfas_problem* prob);

/* Validate the problem, allocate the workspace on the current device and bind
 * the context to hip_stream (a hipStream_t; NULL = default stream). */
stfas_status stfas_create(const stfas_problem* prob, void* hip_stream, stfas_ctx** out);

/* Same as stfas_create, but the workspace is caller memory: `workspace`
 * points to at least stfas_workspace_bytes(prob) bytes of device memory on
 * the stream's device (256-byte aligned), which the caller keeps alive until
 * stfas_destroy and frees itself.  The context then makes no device
 * allocation and its destroy frees nothing, so contexts can come and go
 * while other streams run (a device free would wait for all of them).
 * workspace_bytes too small or a misaligned pointer: STFAS_E_INVALID. */
stfas_status stfas_create_in(const stfas_problem* prob, void* hip_stream, void* workspace, size_t workspace_bytes,
                             stfas_ctx** out);

/* Solve (Alg:outter).  rho0: initial density [cells].  key_steps: host array
 * of num_key step indices in 1..N, strictly increasing.  key_rho: keyframe
 * densities [num_key][cells].  u_out: the control sequence [N][faces].
 * Stats go to the host struct.  Blocks until the outputs are complete.
 * Non-convergence is not an error (stats->converged = 0). */
stfas_status stfas_solve(stfas_ctx* ctx, const void* rho0, int32_t num_key, const int32_t* key_steps,
                         const void* key_rho, void* u_out, stfas_stats* stats);

/* Gradient-based baseline (Sec. 5, the comparison with LBFGS; Sec. 3.2 for
 * the reduced problem): L-BFGS over the controls with the simulation
 * eliminated, J(u) = 1/2 sum_k <e_k, C e_k> + r/2 |u|^2 (eq:opt), its
 * gradient by the adjoint of the step chain (one forward and one backward
 * simulation per evaluation, each projection to poisson_rtol).  History 8,
 * initial Hessian scale s'y / y'y (1 / |g| at the first iteration), Armijo
 * backtracking line search (c1 = 1e-4, first step 1, up to 20 halvings).
 * Runs at most iters iterations; stops early when the line search finds no
 * decrease, or, for eps_stop > 0, after an iterate whose density trajectory
 * differs from the previous one by at most eps_stop (max over steps and
 * cells: the ADMM stop of Alg:outter, which Sec. 5 applies to both
 * optimisers).  eps_stop < 0 or NaN: STFAS_E_INVALID.
 * Keys as for stfas_solve.  u_inout [N][faces] (device): the starting
 * controls in, the last accepted iterate out.  J_hist (host, may be NULL):
 * iters + 1 entries, J at the start and after each accepted iteration;
 * *iters_done (may be NULL): the iterations done.  The first call on a
 * context allocates the optimiser's buffers ((N+3)(cells+faces) + (N+1) cells + 23 N faces
 * elements, and 6 faces more with the rotational operator, whose backward
 * pass recomputes each step's fixed-point iterates), freed by stfas_destroy; a context made by stfas_create_in makes
 * no allocation, so there the call returns STFAS_E_INVALID.  Blocks. */
stfas_status stfas_lbfgs(stfas_ctx* ctx, const void* rho0, int32_t num_key, const int32_t* key_steps,
                         const void* key_rho, void* u_inout, int32_t iters, double eps_stop, int32_t* iters_done,
                         double* J_hist);

/* One simulation step (Sec. 3.1 eq:NSA-eq:Conv with semi-Lagrangian advection):
 *   rho_out = A(rho, v),  v_out = Q(S(v) + dt u),  p_out = phi/dt (may be NULL).
 * work: caller scratch of stfas_step_work_bytes(prob) bytes.  Asynchronous
 * on the stream; the projection runs a fixed number of multigrid cycles
 * (stfas_step_vcycles) so that the call never synchronises. */
stfas_status stfas_step_forward(const stfas_problem* prob, void* hip_stream, const void* rho, const void* v,
                                const void* u, void* rho_out, void* v_out, void* p_out, void* work);

/* Adjoint of stfas_step_forward: given the cotangents g_rho_out, g_v_out of
 * (rho_out, v_out), writes g_rho = W(v)^T g_rho_out,
 * g_v = J_S(v)^T Q g_v_out + (dA/dv)^T g_rho_out and g_u = dt Q g_v_out
 * (Q is symmetric).  Asynchronous. */
stfas_status stfas_step_backward(const stfas_problem* prob, void* hip_stream, const void* rho, const void* v,
                                 const void* g_rho_out, const void* g_v_out, void* g_rho, void* g_v, void* g_u,
                                 void* work);

/* The adjoint of stfas_step_forward for either velocity operator, given
 * also the step's control u (the rotational operator's fixed-point iterates
 * depend on it; it is read only there).  For the rotational operator it is
 * the exact adjoint of the fixed-point steps as computed (Sec. 3.1 eq:NSA
 * solved by 4 of them, forward again inside the call): with b = v + dt u,
 * y_0 = Q b and y_m = Q(b - dt Adv[y_{m-1}]), v_out = y_4,
 *   g_y <- g_v_out; for m = 4 .. 0: g_w = Q g_y, g_b += g_w,
 *   g_y <- -dt J_Adv(y_{m-1})^T g_w (m > 0);
 * g_u = dt g_b and g_v = g_b + (dA/dv)^T g_rho_out; g_rho as in
 * stfas_step_backward.  For the semi-Lagrangian operator it equals
 * stfas_step_backward.  Asynchronous; work as for stfas_step_forward. */
stfas_status stfas_step_backward_u(const stfas_problem* prob, void* hip_stream, const void* rho, const void* v,
                                   const void* u, const void* g_rho_out, const void* g_v_out, void* g_rho, void* g_v,
                                   void* g_u, void* work);

size_t stfas_step_work_bytes(const stfas_problem* prob);

/* Size of the library's static device scratch used by
 * stfas_step_forward_noalloc (one array per device, held until the process
 * ends). */
#define STFAS_NOALLOC_SCRATCH_BYTES (80u << 20)

/* stfas_step_forward without the work argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The step's scratch (the coarsest
 * Poisson level's pseudo-inverse followed by stfas_step_work_bytes(prob)
 * bytes of projection buffers) lives in a static device array of
 * STFAS_NOALLOC_SCRATCH_BYTES per device, which the call never allocates or
 * frees.  A problem whose scratch exceeds that size returns STFAS_E_INVALID
 * before any launch (SL steps fit up to 128^3 in FP32 and 96^3 in FP64).
 * The first call on a device looks the array up (hipGetSymbolAddress); a
 * call whose coarse grid differs from the previous call's uploads that
 * grid's pseudo-inverse (computed and cached on the host) to the array on
 * the stream.  Inputs, outputs, results and asynchrony are those of
 * stfas_step_forward.  Every call on one device shares the one array and it
 * keeps the last call's contents: calls that overlap on a device (other
 * streams, other host threads) race and must be serialised by the caller. */
stfas_status stfas_step_forward_noalloc(const stfas_problem* prob, void* hip_stream, const void* rho, const void* v,
                                        const void* u, void* rho_out, void* v_out, void* p_out);

/* Number of projection V-cycles the step functions run (depends on the
 * precision only; chosen so that the relative residual reaches
 * poisson_rtol on smooth data). */
int32_t stfas_step_vcycles(const stfas_problem* prob);

void stfas_destroy(stfas_ctx* ctx);
const char* stfas_status_string(stfas_status s);

/* Library version and build information (static string). */
const char* stfas_build_info(void);

#ifdef __cplusplus
}
#endif
#endif /* STFAS_H */
