"""Differentiation form: one simulation step (Sec. 3.1 eq:NSA-eq:Conv with
semi-Lagrangian advection, or the rotational velocity operator's implicit
update by fixed-point steps) as a torch.autograd.Function whose backward is
the library's adjoint kernels, and a checkpointed trajectory.

  forward:  rho' = A(rho, v),  v' = Q(S(v) + dt u)
  backward: g_rho = W(v)^T g_rho',  g_u = dt Q g_v',
            g_v = J_S(v)^T Q g_v' + (dA/dv)^T g_rho'

The adjoint of the whole trajectory is the chain of step adjoints, which is
the gradient the paper's gradient-based baseline needs (Sec. 3.2; one
gradient costs about two simulations, Sec. 5).
"""
import torch
import torch.utils.checkpoint

from . import stfas as S


class _Work:
    """Step scratch per (byte count, device), allocated once.  The key is the
    library's own byte count for the problem, so problems that need more
    scratch (a larger grid, FP64, the upwind density operator's series terms)
    never share a smaller buffer."""

    _cache = {}

    @classmethod
    def get(cls, prob, device):
        nbytes = S.stfas_step_work_bytes(prob)
        key = (nbytes, str(device))
        buf = cls._cache.get(key)
        if buf is None:
            buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
            cls._cache[key] = buf
        return buf


class SimStep(torch.autograd.Function):
    """(rho, v, u) -> (rho', v') on the device through the HIP library."""

    @staticmethod
    def forward(ctx, rho, v, u, prob):
        rho = rho.contiguous()
        v = v.contiguous()
        u = u.contiguous()
        rho_o = torch.empty_like(rho)
        v_o = torch.empty_like(v)
        S.stfas_step_forward(prob, rho, v, u, rho_o, v_o, work=_Work.get(prob, rho.device))
        ctx.save_for_backward(rho, v, u)
        ctx.prob = prob
        return rho_o, v_o

    @staticmethod
    def backward(ctx, g_rho_o, g_v_o):
        rho, v, u = ctx.saved_tensors
        prob = ctx.prob
        g_rho_o = torch.zeros_like(rho) if g_rho_o is None else g_rho_o.contiguous()
        g_v_o = torch.zeros_like(v) if g_v_o is None else g_v_o.contiguous()
        g_rho = torch.empty_like(rho)
        g_v = torch.empty_like(v)
        g_u = torch.empty_like(v)
        # the control enters the rotational step's fixed-point iterates, so its adjoint takes u
        S.stfas_step_backward_u(prob, rho, v, u, g_rho_o, g_v_o, g_rho, g_v, g_u, work=_Work.get(prob, rho.device))
        return g_rho, g_v, g_u, None


def step(rho, v, u, prob):
    return SimStep.apply(rho, v, u, prob)


def rollout(prob, rho0, v0, us, checkpoint_every=0, keep=()):
    """Run len(us) steps from (rho0, v0).  Returns (rho_N, v_N, {t: rho_t for
    t in keep}).  checkpoint_every = k > 0 stores only every k-th state for
    the backward pass and recomputes each k-step segment from its stored
    start (memory ~ N/k states instead of N)."""
    rho, v = rho0, v0
    kept = {}
    N = len(us)
    t = 0
    while t < N:
        seg = N - t if checkpoint_every <= 0 else min(checkpoint_every, N - t)

        def run(r, vv, *useg, t0=t):
            out = []
            for q, uq in enumerate(useg):
                r, vv = step(r, vv, uq, prob)
                if t0 + q + 1 in keep:
                    out.append(r)
            return (r, vv, *out)

        useg = [us[t + q] for q in range(seg)]
        if checkpoint_every > 0 and torch.is_grad_enabled():
            res = torch.utils.checkpoint.checkpoint(run, rho, v, *useg, use_reentrant=False)
        else:
            res = run(rho, v, *useg)
        rho, v = res[0], res[1]
        extra = list(res[2:])
        for q in range(seg):
            if t + q + 1 in keep:
                kept[t + q + 1] = extra.pop(0)
        t += seg
    return rho, v, kept
