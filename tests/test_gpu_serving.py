"""Serving form: results are the same alone and inside the concurrent mix,
and admission never holds more than the HBM budget."""
import pytest

import synthetic
from gpu_common import flag, rel

pytestmark = pytest.mark.gpu


def _requests(count=6, seed=5):
    from paper_1608_01102_amd import serving
    raw = synthetic.c5_requests(seed, count, rate=50.0, sizes2d=(32, 48), sizes3d=(16,), steps2d=(4, 8),
                                steps3d=(3, 5))
    return [serving.Request(q["rid"], q["arrival"], q["n"], q["num_steps"], q["r"], q["rho0"], q["key_steps"],
                            q["key_rho"], dict(dt=q["dt"], max_admm=2, max_vcycles=3, fixed_counts=True))
            for q in raw]


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_same_alone_and_in_the_mix(precision):
    from paper_1608_01102_amd import serving
    reqs = _requests()
    flag(f"serving alone {precision}")
    alone, _ = serving.run_sequential(reqs, precision=precision, realtime=False)
    flag(f"serving mix {precision}")
    srv = serving.Server(budget_bytes=8 << 30, max_slots=3, precision=precision)
    mix, _ = srv.run(reqs, realtime=False)
    tol = 1e-4 if precision == "mixed" else 1e-10
    for a, b in zip(alone, mix):
        assert a.rid == b.rid
        assert rel(b.u, a.u) <= tol, a.rid
        assert abs(b.stats["objective"] - a.stats["objective"]) <= tol * abs(a.stats["objective"])
    # the mix overlapped: some request was admitted before another finished
    ints = sorted((r.admitted, r.finished) for r in mix)
    assert any(ints[i + 1][0] < ints[i][1] for i in range(len(ints) - 1))


def test_admission_respects_budget():
    from paper_1608_01102_amd import serving
    reqs = _requests(8, seed=9)
    fps = [serving.footprint(q, "mixed") for q in reqs]
    budget = max(fps) + min(fps)
    flag("serving budget")
    srv = serving.Server(budget_bytes=budget, max_slots=4, precision="mixed")
    res, _ = srv.run(reqs, realtime=True)
    events = sorted([(r.admitted, r.footprint) for r in res] + [(r.finished, -r.footprint) for r in res],
                    key=lambda e: (e[0], e[1]))
    held = 0
    for _, d in events:
        held += d
        assert held <= budget
    assert all(r.admitted >= r.arrival - 1e-6 for r in res)
