"""Python binding of libstfas with the names of the C interface.

Argument marshalling only: every step of the solver runs in the HIP library.
Device buffers are torch tensors on the current CUDA(HIP) device,
contiguous, float64 for STFAS_FP64 and float32 for STFAS_MIXED; the stream
is torch's current stream unless one is passed.
"""
import ctypes

import torch

from . import _lib
from ._lib import StfasProblem, StfasState, StfasStats, check

PRECISIONS = {"fp64": _lib.STFAS_FP64, "mixed": _lib.STFAS_MIXED}
DENSITY_OPS = {"sl": 0, "upwind": 1}
VELOCITY_OPS = {"sl": 0, "rotational": 1, "vorticity": 1}
SCGS_LOCAL = {"default": 0, "collapsed": 1, "exact": 2, "finest": 3}


def make_problem(n, num_steps, r, dt=0.0, K=0.0, beta=0.0, ao_iters=0, eps_stfas=0.0, eps_admm=0.0, max_admm=0,
                 max_vcycles=0, metric_levels=-1, poisson_rtol=0.0, fixed_counts=False, precision="fp64",
                 scgs_omega=0.0, density="sl", al_tol=0.0, scgs_lm=0.0, velocity="sl", scgs_local="default"):
    """stfas_problem with the C defaults for every field left at 0 (-1 for metric_levels)."""
    p = StfasProblem()
    n = tuple(int(x) for x in n)
    p.dim = len(n)
    p.n[0], p.n[1] = n[0], n[1]
    p.n[2] = n[2] if len(n) == 3 else 1
    p.num_steps = int(num_steps)
    p.dt, p.r, p.K, p.beta = float(dt), float(r), float(K), float(beta)
    p.ao_iters = int(ao_iters)
    p.eps_stfas, p.eps_admm = float(eps_stfas), float(eps_admm)
    p.max_admm, p.max_vcycles, p.metric_levels = int(max_admm), int(max_vcycles), int(metric_levels)
    p.poisson_rtol = float(poisson_rtol)
    p.fixed_counts = 1 if fixed_counts else 0
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.scgs_omega = float(scgs_omega)
    p.density_op = DENSITY_OPS[density] if isinstance(density, str) else int(density)
    p.al_tol = float(al_tol)
    p.scgs_lm = float(scgs_lm)
    p.velocity_op = VELOCITY_OPS[velocity] if isinstance(velocity, str) else int(velocity)
    p.scgs_local = SCGS_LOCAL[scgs_local] if isinstance(scgs_local, str) else int(scgs_local)
    return p


def dtype_of(prob):
    return torch.float64 if prob.precision == _lib.STFAS_FP64 else torch.float32


def counts(prob):
    """(cells, faces) of the level-0 grid."""
    n = [prob.n[0], prob.n[1], prob.n[2] if prob.dim == 3 else 1]
    cells = n[0] * n[1] * n[2]
    faces = n[2] * n[1] * (n[0] + 1) + n[2] * (n[1] + 1) * n[0]
    if prob.dim == 3:
        faces += (n[2] + 1) * n[1] * n[0]
    return cells, faces


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t, dtype, numel=None, name="tensor", optional=False):
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {numel}")
    return ctypes.c_void_p(t.data_ptr())


def stfas_workspace_bytes(prob):
    return int(_lib.load().stfas_workspace_bytes(ctypes.byref(prob)))


def stfas_step_work_bytes(prob):
    return int(_lib.load().stfas_step_work_bytes(ctypes.byref(prob)))


def stfas_step_vcycles(prob):
    return int(_lib.load().stfas_step_vcycles(ctypes.byref(prob)))


def stfas_build_info():
    return _lib.load().stfas_build_info().decode()


class Context:
    """Owns one stfas_ctx (its workspace lives on the device until destroy)."""

    def __init__(self, prob, stream=None, workspace=None):
        lib = _lib.load()
        self.prob = prob
        self.dtype = dtype_of(prob)
        self.stream = torch.cuda.current_stream() if stream is None else stream
        self.cells, self.faces = counts(prob)
        self.N = prob.num_steps
        self.workspace = workspace          # keeps caller memory alive until destroy
        h = ctypes.c_void_p()
        if workspace is None:
            check(lib.stfas_create(ctypes.byref(prob), _stream(self.stream), ctypes.byref(h)), "stfas_create")
        else:
            if not (isinstance(workspace, torch.Tensor) and workspace.is_cuda and workspace.is_contiguous()):
                raise TypeError("workspace must be a contiguous device tensor")
            nbytes = workspace.numel() * workspace.element_size()
            check(lib.stfas_create_in(ctypes.byref(prob), _stream(self.stream), ctypes.c_void_p(workspace.data_ptr()),
                                      nbytes, ctypes.byref(h)), "stfas_create_in")
        self.handle = h

    def __del__(self):
        self.destroy()

    def destroy(self):
        if getattr(self, "handle", None) and self.handle.value and _lib is not None:
            _lib.load().stfas_destroy(self.handle)
            self.handle = ctypes.c_void_p()
        self.workspace = None

    def num_levels(self):
        return int(_lib.load().stfas_num_levels(self.handle))

    def level_counts(self, level):
        lib = _lib.load()
        return int(lib.stfas_level_cells(self.handle, level)), int(lib.stfas_level_faces(self.handle, level))

    def state(self, x, level=0, name="state", optional=False):
        """StfasState from a (v, pbar, u, p) tuple of tensors (or None)."""
        if x is None:
            if optional:
                return StfasState()
            raise ValueError(f"{name} is required")
        c, f = self.level_counts(level)
        N = self.N
        v, pb, u, p = x
        return StfasState(_ptr(v, self.dtype, N * f, name + ".v"), _ptr(pb, self.dtype, N * c, name + ".pbar"),
                          _ptr(u, self.dtype, N * f, name + ".u"), _ptr(p, self.dtype, N * c, name + ".p"))


def stfas_create(prob, stream=None):
    return Context(prob, stream)


def stfas_create_in(prob, workspace, stream=None):
    """Context on caller device memory (a contiguous tensor of at least
    stfas_workspace_bytes(prob) bytes, 256-byte aligned)."""
    return Context(prob, stream, workspace)


def stfas_destroy(ctx):
    ctx.destroy()


def stfas_solve(ctx, rho0, key_steps, key_rho, u_out):
    """Returns the stats as a dict; u_out [N][faces] is written."""
    lib = _lib.load()
    nk = len(key_steps)
    ks = (ctypes.c_int32 * max(nk, 1))(*[int(k) for k in key_steps])
    st = StfasStats()
    check(lib.stfas_solve(ctx.handle, _ptr(rho0, ctx.dtype, ctx.cells, "rho0"), nk, ks,
                          _ptr(key_rho, ctx.dtype, nk * ctx.cells, "key_rho", optional=nk == 0),
                          _ptr(u_out, ctx.dtype, ctx.N * ctx.faces, "u_out"), ctypes.byref(st)), "stfas_solve")
    return {k: getattr(st, k) for k, _ in StfasStats._fields_}


def stfas_lbfgs(ctx, rho0, key_steps, key_rho, u_inout, iters, eps_stop=0.0):
    """L-BFGS baseline on the reduced objective; u_inout [N][faces] holds the
    start and receives the result; eps_stop > 0 adds the visual-difference
    stop.  Returns (J history, iterations done)."""
    lib = _lib.load()
    nk = len(key_steps)
    ks = (ctypes.c_int32 * max(nk, 1))(*[int(k) for k in key_steps])
    hist = (ctypes.c_double * (int(iters) + 1))()
    done = ctypes.c_int32(0)
    check(lib.stfas_lbfgs(ctx.handle, _ptr(rho0, ctx.dtype, ctx.cells, "rho0"), nk, ks,
                          _ptr(key_rho, ctx.dtype, nk * ctx.cells, "key_rho", optional=nk == 0),
                          _ptr(u_inout, ctx.dtype, ctx.N * ctx.faces, "u_inout"), int(iters), float(eps_stop), ctypes.byref(done),
                          hist), "stfas_lbfgs")
    return list(hist[:done.value + 1]), done.value


def _step_work(prob, work, device):
    """The step's scratch: allocated here when not given; a given buffer must
    hold at least the library's byte count for this problem (the C calls take
    no size, so a short buffer would be overrun)."""
    need = stfas_step_work_bytes(prob)
    if work is None:
        return torch.empty(need, dtype=torch.uint8, device=device)
    have = work.numel() * work.element_size()
    if not work.is_contiguous() or have < need:
        raise ValueError(f"step work buffer holds {have} bytes (contiguous: {work.is_contiguous()}); "
                         f"this problem needs {need}")
    return work


def stfas_step_forward(prob, rho, v, u, rho_out, v_out, p_out=None, work=None, stream=None):
    dt = dtype_of(prob)
    c, f = counts(prob)
    work = _step_work(prob, work, rho.device)
    check(_lib.load().stfas_step_forward(
        ctypes.byref(prob), _stream(stream), _ptr(rho, dt, c, "rho"), _ptr(v, dt, f, "v"), _ptr(u, dt, f, "u"),
        _ptr(rho_out, dt, c, "rho_out"), _ptr(v_out, dt, f, "v_out"), _ptr(p_out, dt, c, "p_out", optional=True),
        ctypes.c_void_p(work.data_ptr())), "stfas_step_forward")


def stfas_step_forward_noalloc(prob, rho, v, u, rho_out, v_out, p_out=None, stream=None):
    """stfas_step_forward on the library's static device scratch (no work buffer, no allocation)."""
    dt = dtype_of(prob)
    c, f = counts(prob)
    check(_lib.load().stfas_step_forward_noalloc(
        ctypes.byref(prob), _stream(stream), _ptr(rho, dt, c, "rho"), _ptr(v, dt, f, "v"), _ptr(u, dt, f, "u"),
        _ptr(rho_out, dt, c, "rho_out"), _ptr(v_out, dt, f, "v_out"), _ptr(p_out, dt, c, "p_out", optional=True)),
        "stfas_step_forward_noalloc")


def stfas_step_backward(prob, rho, v, g_rho_out, g_v_out, g_rho, g_v, g_u, work=None, stream=None):
    dt = dtype_of(prob)
    c, f = counts(prob)
    work = _step_work(prob, work, rho.device)
    check(_lib.load().stfas_step_backward(
        ctypes.byref(prob), _stream(stream), _ptr(rho, dt, c, "rho"), _ptr(v, dt, f, "v"),
        _ptr(g_rho_out, dt, c, "g_rho_out"), _ptr(g_v_out, dt, f, "g_v_out"), _ptr(g_rho, dt, c, "g_rho"),
        _ptr(g_v, dt, f, "g_v"), _ptr(g_u, dt, f, "g_u"), ctypes.c_void_p(work.data_ptr())), "stfas_step_backward")


def stfas_step_backward_u(prob, rho, v, u, g_rho_out, g_v_out, g_rho, g_v, g_u, work=None, stream=None):
    dt = dtype_of(prob)
    c, f = counts(prob)
    work = _step_work(prob, work, rho.device)
    check(_lib.load().stfas_step_backward_u(
        ctypes.byref(prob), _stream(stream), _ptr(rho, dt, c, "rho"), _ptr(v, dt, f, "v"), _ptr(u, dt, f, "u"),
        _ptr(g_rho_out, dt, c, "g_rho_out"), _ptr(g_v_out, dt, f, "g_v_out"), _ptr(g_rho, dt, c, "g_rho"),
        _ptr(g_v, dt, f, "g_v"), _ptr(g_u, dt, f, "g_u"), ctypes.c_void_p(work.data_ptr())), "stfas_step_backward_u")


# ---------------------------------------------------------------- operator level
def stfas_op_advect(ctx, batch, rho, v, out):
    c, f = ctx.cells, ctx.faces
    check(_lib.load().stfas_op_advect(ctx.handle, batch, _ptr(rho, ctx.dtype, batch * c, "rho"),
                                      _ptr(v, ctx.dtype, batch * f, "v"), _ptr(out, ctx.dtype, batch * c, "out")),
          "stfas_op_advect")


def stfas_op_advect_T(ctx, batch, mu, v, add, out):
    c, f = ctx.cells, ctx.faces
    check(_lib.load().stfas_op_advect_T(ctx.handle, batch, _ptr(mu, ctx.dtype, batch * c, "mu"),
                                        _ptr(v, ctx.dtype, batch * f, "v"),
                                        _ptr(add, ctx.dtype, batch * c, "add", optional=True),
                                        _ptr(out, ctx.dtype, batch * c, "out")), "stfas_op_advect_T")


def stfas_op_advect_dv_T(ctx, batch, mu, rho, v, vt, scale, gv):
    c, f = ctx.cells, ctx.faces
    check(_lib.load().stfas_op_advect_dv_T(ctx.handle, batch, _ptr(mu, ctx.dtype, batch * c, "mu"),
                                           _ptr(rho, ctx.dtype, batch * c, "rho"), _ptr(v, ctx.dtype, batch * f, "v"),
                                           _ptr(vt, ctx.dtype, batch * f, "vt", optional=True), float(scale),
                                           _ptr(gv, ctx.dtype, batch * f, "gv")), "stfas_op_advect_dv_T")


def stfas_op_upwind(ctx, rho, v, out):
    """Upwind exponential advection of one slice; returns k."""
    c, f = ctx.cells, ctx.faces
    k = ctypes.c_int32(-1)
    check(_lib.load().stfas_op_upwind(ctx.handle, _ptr(rho, ctx.dtype, c, "rho"), _ptr(v, ctx.dtype, f, "v"),
                                      _ptr(out, ctx.dtype, c, "out"), ctypes.byref(k)), "stfas_op_upwind")
    return k.value


def stfas_op_upwind_adj(ctx, mu, rho, v, g_rho, g_v):
    c, f = ctx.cells, ctx.faces
    check(_lib.load().stfas_op_upwind_adj(ctx.handle, _ptr(mu, ctx.dtype, c, "mu"), _ptr(rho, ctx.dtype, c, "rho"),
                                          _ptr(v, ctx.dtype, f, "v"), _ptr(g_rho, ctx.dtype, c, "g_rho"),
                                          _ptr(g_v, ctx.dtype, f, "g_v")), "stfas_op_upwind_adj")


def stfas_op_self_advect(ctx, level, batch, v, u, out):
    _, f = ctx.level_counts(level)
    check(_lib.load().stfas_op_self_advect(ctx.handle, level, batch, _ptr(v, ctx.dtype, batch * f, "v"),
                                           _ptr(u, ctx.dtype, batch * f, "u", optional=True),
                                           _ptr(out, ctx.dtype, batch * f, "out")), "stfas_op_self_advect")


def stfas_op_self_advect_T(ctx, level, batch, v, y, scale, out):
    _, f = ctx.level_counts(level)
    check(_lib.load().stfas_op_self_advect_T(ctx.handle, level, batch, _ptr(v, ctx.dtype, batch * f, "v"),
                                             _ptr(y, ctx.dtype, batch * f, "y"), float(scale),
                                             _ptr(out, ctx.dtype, batch * f, "out")), "stfas_op_self_advect_T")


def stfas_op_project(ctx, batch, w, out, phi=None):
    cyc = ctypes.c_int32()
    check(_lib.load().stfas_op_project(ctx.handle, batch, _ptr(w, ctx.dtype, batch * ctx.faces, "w"),
                                       _ptr(out, ctx.dtype, batch * ctx.faces, "out"),
                                       _ptr(phi, ctx.dtype, batch * ctx.cells, "phi", optional=True),
                                       ctypes.byref(cyc)), "stfas_op_project")
    return cyc.value


def stfas_op_metric(ctx, e, out):
    check(_lib.load().stfas_op_metric(ctx.handle, _ptr(e, ctx.dtype, ctx.cells, "e"),
                                      _ptr(out, ctx.dtype, ctx.cells, "out")), "stfas_op_metric")


def stfas_op_kkt_residual(ctx, level, x, w, res, out):
    _, f = ctx.level_counts(level)
    check(_lib.load().stfas_op_kkt_residual(ctx.handle, level, ctx.state(x, level, "x"),
                                            _ptr(w, ctx.dtype, ctx.N * f, "w"),
                                            ctx.state(res, level, "res", optional=True),
                                            ctx.state(out, level, "out")), "stfas_op_kkt_residual")


def stfas_op_scgs_sweep(ctx, level, x, w, res=None):
    _, f = ctx.level_counts(level)
    check(_lib.load().stfas_op_scgs_sweep(ctx.handle, level, ctx.state(x, level, "x"),
                                          _ptr(w, ctx.dtype, ctx.N * f, "w"),
                                          ctx.state(res, level, "res", optional=True)), "stfas_op_scgs_sweep")


def stfas_op_restrict(ctx, level, fine, coarse):
    check(_lib.load().stfas_op_restrict(ctx.handle, level, ctx.state(fine, level, "fine"),
                                        ctx.state(coarse, level + 1, "coarse")), "stfas_op_restrict")


def stfas_op_prolong(ctx, level, coarse, sign, fine):
    check(_lib.load().stfas_op_prolong(ctx.handle, level, ctx.state(coarse, level + 1, "coarse"), float(sign),
                                       ctx.state(fine, level, "fine")), "stfas_op_prolong")


def stfas_op_nso(ctx, x, w):
    """Returns (V-cycles, |f|_inf history list)."""
    n = ctypes.c_int32()
    hist = (ctypes.c_double * (ctx.prob.max_vcycles + 1 if ctx.prob.max_vcycles > 0 else 31))()
    check(_lib.load().stfas_op_nso(ctx.handle, ctx.state(x, 0, "x"), _ptr(w, ctx.dtype, ctx.N * ctx.faces, "w"),
                                   ctypes.byref(n), hist), "stfas_op_nso")
    return n.value, list(hist[:n.value + 1])


def stfas_op_ao(ctx, rho0, key_steps, key_rho, vt, vstar, rho):
    """Returns the objective history (ao_iters + 1 values)."""
    nk = len(key_steps)
    ks = (ctypes.c_int32 * max(nk, 1))(*[int(k) for k in key_steps])
    iters = ctx.prob.ao_iters if ctx.prob.ao_iters > 0 else 2
    hist = (ctypes.c_double * (iters + 1))()
    c, f, N = ctx.cells, ctx.faces, ctx.N
    check(_lib.load().stfas_op_ao(ctx.handle, _ptr(rho0, ctx.dtype, c, "rho0"), nk, ks,
                                  _ptr(key_rho, ctx.dtype, nk * c, "key_rho", optional=nk == 0),
                                  _ptr(vt, ctx.dtype, N * f, "vt"), _ptr(vstar, ctx.dtype, N * f, "vstar"),
                                  _ptr(rho, ctx.dtype, (N + 1) * c, "rho"), hist), "stfas_op_ao")
    return list(hist)


TRACE_KERNELS = {"scgs_thomas": 1, "scgs_project": 2, "kkt_faces": 3, "self_advect_T": 4, "rbgs": 5, "advect": 6,
                 "kkt_cells": 7, "scgs_cells": 8, "scgs_colour": 9,
                 "kkt_split": 10, "up_term": 11}


def stfas_trace_enable(ctx, kernel, max_launches=4096):
    k = TRACE_KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    check(_lib.load().stfas_trace_enable(ctx.handle, k, int(max_launches)), "stfas_trace_enable")


def stfas_trace_read(ctx):
    """(launches, total_ms, algorithmic_bytes, implementation_bytes) of the traced kernel family."""
    n, ms, b, ib = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    check(_lib.load().stfas_trace_read(ctx.handle, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(b),
                                       ctypes.byref(ib)), "stfas_trace_read")
    return n.value, ms.value, b.value, ib.value
