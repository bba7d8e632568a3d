"""Serving form: continuous batching of control requests on one GPU.

Requests (mixed 2D/3D grids and step counts) arrive over time.  A request is
admitted into a free slot as soon as its exact device footprint (the
solver workspace from stfas_workspace_bytes plus its input and output
buffers) fits in the remaining HBM budget; each slot owns a HIP stream
(default priority) and a solver context, and runs its solve on a worker
thread (the C call releases the Python interpreter lock, so slots overlap on
the device).  When a solve finishes its memory is released and waiting
requests are admitted.  Admission is in arrival order, except that a request
that has arrived and fits may pass a waiting head that does not fit (a large
request waiting for memory); the head can be passed at most `max_bypass`
times, after which nothing passes it until it is admitted.  Latency is
measured from arrival to result.

The sequential baseline runs the same requests first-in first-out, one at a
time, on the same arrivals, in real time.
"""
import dataclasses
import threading
import time

import numpy as np
import torch

from . import stfas as S


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds from the start of the stream
    n: tuple
    num_steps: int
    r: float
    rho0: np.ndarray
    key_steps: list
    key_rho: np.ndarray            # [num_key, cells]
    options: dict = dataclasses.field(default_factory=dict)   # extra make_problem fields


@dataclasses.dataclass
class Result:
    rid: int
    u: np.ndarray
    stats: dict
    arrival: float
    admitted: float
    finished: float
    footprint: int

    @property
    def latency(self):
        return self.finished - self.arrival


def problem_of(req, precision):
    return S.make_problem(req.n, req.num_steps, req.r, precision=precision, **req.options)


def footprint(req, precision):
    """Exact device bytes a request holds while it runs."""
    prob = problem_of(req, precision)
    ws = S.stfas_workspace_bytes(prob)
    if ws == 0:
        raise ValueError(f"request {req.rid}: invalid problem")
    cells, faces = S.counts(prob)
    word = 8 if precision == "fp64" else 4
    io = word * (cells * (1 + len(req.key_steps)) + faces * req.num_steps)
    return ws + 256 + io            # + alignment slack of the workspace


def _solve_on(req, precision, stream):
    """Create a context on `stream`, upload, solve, download.  Returns (u, stats)."""
    prob = problem_of(req, precision)
    dt = S.dtype_of(prob)
    with torch.cuda.stream(stream):
        # workspace from torch's caching allocator on this stream: no device
        # allocation or free (both would wait for the other slots) per request
        ws = torch.empty(S.stfas_workspace_bytes(prob) + 256, dtype=torch.uint8, device="cuda")
        off = (-ws.data_ptr()) % 256
        ctx = S.stfas_create_in(prob, ws[off:], stream=stream)
        try:
            rho0 = torch.tensor(req.rho0, dtype=dt, device="cuda").contiguous()
            keys = torch.tensor(req.key_rho, dtype=dt, device="cuda").contiguous()
            u = torch.empty(req.num_steps * ctx.faces, dtype=dt, device="cuda")
            stats = S.stfas_solve(ctx, rho0, req.key_steps, keys, u)
            out = u.cpu().numpy().reshape(req.num_steps, -1)
        finally:
            ctx.destroy()
    return out, stats


def pick_next(pending, fps, now, free_bytes, bypassed, max_bypass):
    """Index in `pending` (sorted by arrival) of the request to admit now, or
    None.  now = None: every request has arrived.  The first arrived request
    whose footprint fits in free_bytes is taken, except that once the head
    has been passed max_bypass times only the head may be taken."""
    for pos, q in enumerate(pending):
        if now is not None and now < q.arrival:
            return None                       # later ones have not arrived either
        if fps[q.rid] <= free_bytes:
            return pos
        if pos == 0 and bypassed >= max_bypass:
            return None                       # the head waits; nothing may pass it now
    return None


class Server:
    """Continuous-batching request loop.

    budget_bytes: HBM the server may hold for admitted requests.
    max_slots:    concurrent solves (each a stream, a context and a thread).
    """

    def __init__(self, budget_bytes=None, max_slots=4, precision="mixed", max_bypass=8):
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(0.8 * free)
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.precision = precision
        self.max_bypass = int(max_bypass)
        self.streams = [torch.cuda.Stream() for _ in range(self.max_slots)]

    def run(self, requests, realtime=True):
        """Serve `requests` (sorted by arrival).  realtime=False admits every
        request as if it had arrived at time 0 (closed-loop throughput)."""
        reqs = sorted(requests, key=lambda q: q.arrival)
        for q in reqs:
            if footprint(q, self.precision) > self.budget:
                raise ValueError(f"request {q.rid} needs more than the whole budget")
        lock = threading.Condition()
        state = {"used": 0, "free_slots": list(range(self.max_slots)), "errors": []}
        results = {}
        threads = []
        t0 = time.perf_counter()

        def worker(q, slot, fp, admitted):
            try:
                u, stats = _solve_on(q, self.precision, self.streams[slot])
                fin = time.perf_counter() - t0
                results[q.rid] = Result(q.rid, u, stats, q.arrival if realtime else 0.0, admitted, fin, fp)
            except Exception as e:      # reported after the loop
                state["errors"].append((q.rid, e))
            finally:
                with lock:
                    state["used"] -= fp
                    state["free_slots"].append(slot)
                    lock.notify_all()

        pending = list(reqs)
        fps = {q.rid: footprint(q, self.precision) for q in reqs}
        bypassed = 0                      # times the current head has been passed
        while pending:
            with lock:
                while True:
                    now = time.perf_counter() - t0
                    pick = None
                    if state["free_slots"]:
                        pick = pick_next(pending, fps, now if realtime else None, self.budget - state["used"],
                                         bypassed, self.max_bypass)
                    if pick is not None:
                        break
                    future = [q.arrival - now for q in pending if realtime and q.arrival > now]
                    wait = min(future) if future else 0.5
                    lock.wait(timeout=max(1e-3, min(wait, 0.5)))
                q = pending.pop(pick)
                bypassed = bypassed + 1 if pick > 0 else 0
                slot = state["free_slots"].pop(0)
                fp = fps[q.rid]
                state["used"] += fp
                admitted = time.perf_counter() - t0
            th = threading.Thread(target=worker, args=(q, slot, fp, admitted), daemon=True)
            th.start()
            threads.append(th)
        for th in threads:
            th.join()
        if state["errors"]:
            rid, e = state["errors"][0]
            raise RuntimeError(f"request {rid} failed: {e}")
        makespan = time.perf_counter() - t0
        return [results[q.rid] for q in reqs], makespan


def run_sequential(requests, precision="mixed", realtime=True):
    """FIFO baseline: one request at a time on one stream."""
    reqs = sorted(requests, key=lambda q: q.arrival)
    stream = torch.cuda.Stream()
    out = []
    t0 = time.perf_counter()
    for q in reqs:
        if realtime:
            wait = q.arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
        adm = time.perf_counter() - t0
        u, stats = _solve_on(q, precision, stream)
        fin = time.perf_counter() - t0
        out.append(Result(q.rid, u, stats, q.arrival if realtime else 0.0, adm, fin, footprint(q, precision)))
    return out, time.perf_counter() - t0


def summary(results, makespan):
    lat = np.array([r.latency for r in results])
    return {"requests": len(results), "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
            "makespan_s": makespan, "solves_per_hour": 3600.0 * len(results) / makespan}
