"""Plain FP64 CPU oracle for the spacetime-multigrid smoke-control solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the test-suite, the package smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP path.

Every function follows a passage of Pan & Manocha, "Efficient Optimal Control
of Smoke using Spacetime Multigrid" (arXiv:1608.01102), and is written for
readability rather than speed: plain NumPy in float64, Python loops over time
steps and colours, no blocking or fusion beyond what the paper states.

Module map
  grid      staggered MAC grid, divergence / gradient (Sec. 3.1)
  interp    clamped multilinear interpolation and its derivatives
  advect    semi-Lagrangian density and velocity advection + adjoints
            (Sec. 3.1 eq:Conv, Sec. 4.1 eq:KKTPO, and the remark in Sec. 4.1
            that any advection operator with known partials may be used)
  poisson   solenoidal projection Q (Sec. 4.1, after eq:KKTPO)
  metric    keyframe metric C built from Gaussian filters (Sec. 4.1)
  step      one simulation step and its adjoint (Sec. 3.1 eq:NSA-eq:Conv)
  ao        density subproblem: fixed-point iteration (Alg:Passive) with the
            blending safeguard of Sec. 5 (convergence analysis)
  kkt       KKT residual of the velocity subproblem (Sec. 4.2 eq:KKTAO, App. A)
  scgs      spacetime SCGS smoother (Sec. 4.3, eq:HESS)
  transfer  restriction / prolongation (Sec. 4.3)
  stfas     FAS V-cycle (Alg:STFAS) and the NSO loop
  admm      ADMM outer loop (Alg:outter) and the re-simulated outputs

Parity-unpinned parts (no worked example in the paper; pinned only through
invariants, special cases and brute force on tiny grids): the full ADMM
trajectory (admm.solve).  The FAS V-cycle on nonlinear problems (stfas.vcycle
with advection switched on) is pinned by two exact properties rather than
printed values: a cycle started at an exact solution of f(x) = res returns
it unchanged, and a cycle contracts the residual near such a solution.
"""
