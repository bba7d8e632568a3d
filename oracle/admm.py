"""ADMM outer loop (Alg:outter, Sec. 4 eq:optAdmm) and the outputs.

Problem (Sec. 3.2 eq:opt): minimise over u
  1/2 sum_i c_i |rho_i - rho*_i|_C^2 + r/2 sum_{i<N} |u_i|^2
subject to the simulation step, starting from rho_0 and v_0 = 0.

Loop (one iteration):
  AO:   v* from the density subproblem with vt = v + lambda/K
  NSO:  (v, pbar, u, p) from STFAS with targets w = v* - lambda/K
  stop: max_i |rho^last_i - rho_i|_inf < eps_admm   (rho_i from AO)
  else: rho^last = rho;  lambda_i += K beta (v_i - v*_i)
Start: v, u, p, pbar, lambda = 0, rho^last_i = rho_0.

Readings: v_0 is the given initial state (zero) and is not optimised; the
defaults rescale the paper's parameter table to a unit domain (h = 1/n0,
dt = 1/n0, K = r/dt^2, beta = 1, 2 AO iterations, eps_STFAS = 1e-5
relative, eps_ADMM = max(rho_0)/100); the smoother is relaxed with
omega = 0.7 and its local matrix carries the Levenberg-Marquardt
perturbation K/r + 1/dt^2 of Sec. 5 (without it the velocity subproblem
stalls or diverges once the flow moves about a cell per step, because the
smoother's local matrix leaves out the advection derivative).

Augmented-Lagrangian fallback (Sec. 5, convergence analysis: ADMM falls
back to a standard augmented Lagrangian method by leaving out the multiplier
update until the decrease in function value drops below a threshold).
Reading: the function value is the density subproblem's objective Phi at
the end of the iteration's AO; with al_tol > 0 the multiplier update of
iteration t > 1 is made only when (Phi_{t-1} - Phi_t) / |Phi_{t-1}| <= al_tol
(the first iteration always updates); al_tol = 0 is plain ADMM.

Outputs: u from the NSO; a re-simulation from (rho_0, 0) with u; the
objective J = 1/2 sum_k <e_k, C e_k> + r/2 sum|u_i|^2, its plain-L2 variant
and the regularisation term.
"""
from dataclasses import dataclass, field

import numpy as np

from .grid import Grid
from . import ao, metric, stfas
from .step import step_forward


@dataclass
class Problem:
    n: tuple
    num_steps: int
    r: float
    dt: float = 0.0
    K: float = 0.0
    beta: float = 1.0
    ao_iters: int = 2
    eps_stfas: float = 1e-5
    eps_admm: float = 0.0
    max_admm: int = 50
    max_vcycles: int = 30
    metric_levels: int = -1
    fixed_counts: bool = False
    scgs_omega: float = 0.0           # relaxation weight of the smoother (<= 0: 0.7, 1 with "vorticity")
    density: str = "sl"               # density operator: "sl" or "upwind" (eq:Adv)
    al_tol: float = 0.0               # augmented-Lagrangian fallback threshold (0: plain ADMM)
    scgs_lm: float = 0.0              # smoother's Levenberg-Marquardt perturbation times dt^2
                                      # (< 0: off; 0: 1, off with "vorticity")
    velocity: str = "sl"              # velocity operator: "sl" or "vorticity" (eq:NSA's Adv)
    local_adv: object = "default"     # vorticity: dAdv/dv in the smoother's local matrix (eq:HESS):
                                      # "finest" (level 0 only), True (every level), False (none);
                                      # "default": "finest" in 2D, False in 3D

    def resolved(self, rho0):
        p = Problem(**self.__dict__)
        if p.dt <= 0:
            p.dt = 1.0 / p.n[0]
        if p.K <= 0:
            p.K = p.r / (p.dt * p.dt)
        if p.metric_levels < 0:
            p.metric_levels = metric.default_levels(p.n)
        # with the rotational operator the smoother solves eq:HESS with its local
        # block: no relaxation and no perturbation unless asked for (without
        # the block the perturbation stays)
        rot = p.velocity == "vorticity"
        if p.local_adv == "default":
            p.local_adv = "finest" if len(p.n) == 2 else False
        if p.scgs_omega <= 0:
            p.scgs_omega = 1.0 if rot else 0.7
        if p.scgs_lm == 0:
            p.scgs_lm = -1.0 if rot and p.local_adv is not False else 1.0
        if p.eps_admm <= 0:
            p.eps_admm = float(np.max(rho0)) / 100.0
        return p


@dataclass
class Result:
    u: np.ndarray
    v: np.ndarray
    vstar: np.ndarray
    rho_ao: np.ndarray
    rho_sim: np.ndarray
    objective: float
    objective_l2: float
    reg_term: float
    admm_iters: int
    vcycles: int
    converged: bool
    history: dict = field(default_factory=dict)


def resimulate(g: Grid, rho0, u, dt, kind="sl", velocity="sl"):
    N = u.shape[0]
    rho = np.zeros((N + 1, g.ncell))
    v = np.zeros((N + 1, g.nface))
    rho[0] = rho0
    for i in range(N):
        rho[i + 1], v[i + 1], _ = step_forward(g, rho[i], v[i], u[i], dt, kind=kind, velocity=velocity)
    return rho, v


def objectives(g, rho, keys, u, r, levels):
    reg = 0.5 * r * float(np.sum(u * u))
    jc = 0.0
    jl2 = 0.0
    for t, target in keys.items():
        e = rho[t] - target
        jc += 0.5 * float(e @ metric.apply_metric(g, e, levels))
        jl2 += 0.5 * float(e @ e)
    return jc + reg, jl2 + reg, reg


def solve(prob: Problem, rho0, keys):
    """keys: {step t (1..N): keyframe density (flat)}."""
    p = prob.resolved(rho0)
    g = Grid(p.n)
    N = p.num_steps
    kr = p.K / p.r
    H = stfas.Hierarchy(g, N, p.dt, kr, omega=p.scgs_omega, lm=max(p.scgs_lm, 0.0), velocity=p.velocity,
                          local_adv=p.local_adv)
    F = g.nface
    v_all = np.zeros((N, F))          # v_i, i = 0..N-1 as seen by AO (v_0 = 0)
    lam = np.zeros((N, F))
    x = [np.zeros((N, F)), np.zeros((N, g.ncell)), np.zeros((N, F)), np.zeros((N, g.ncell))]
    rho_last = np.tile(rho0, (N + 1, 1))
    hist = {"visual_diff": [], "ao_phi": [], "nso_res": [], "nso_f0": [], "updates": 0}
    phi_prev = None
    total_vc = 0
    converged = False
    it = 0
    vstar = np.zeros((N, F))
    rho = rho_last.copy()
    while it < p.max_admm:
        it += 1
        vt = v_all + lam / p.K
        vstar, rho, phis = ao.solve(g, rho0, keys, vt, p.K, p.dt, p.metric_levels, p.ao_iters, kind=p.density)
        hist["ao_phi"].append(phis)
        w = vstar - lam / p.K
        info = {}
        nv, rh = stfas.nso(H, x, w, p.eps_stfas, p.max_vcycles, p.fixed_counts, info)
        total_vc += nv
        hist["nso_res"].append(rh)
        hist["nso_f0"].append(info["f0"])
        # v_i for i = 1..N-1 lives in slots 0..N-2 of x[0]
        v_all = np.zeros((N, F))
        v_all[1:] = x[0][:N - 1]
        diff = float(np.max(np.abs(rho_last - rho)))
        hist["visual_diff"].append(diff)
        if not p.fixed_counts and diff < p.eps_admm:
            converged = True
            break
        rho_last = rho.copy()
        phi = phis[-1]
        update = True
        if p.al_tol > 0 and phi_prev is not None:
            update = (phi_prev - phi) / max(abs(phi_prev), 1e-300) <= p.al_tol
        phi_prev = phi
        if update:
            lam = lam + p.K * p.beta * (v_all - vstar)
            hist["updates"] += 1
    u = x[2].copy()
    rho_sim, _ = resimulate(g, rho0, u, p.dt, p.density, p.velocity)
    J, Jl2, reg = objectives(g, rho_sim, keys, u, p.r, p.metric_levels)
    return Result(u=u, v=x[0].copy(), vstar=vstar, rho_ao=rho, rho_sim=rho_sim, objective=J,
                  objective_l2=Jl2, reg_term=reg, admm_iters=it, vcycles=total_vc,
                  converged=converged, history=hist)
