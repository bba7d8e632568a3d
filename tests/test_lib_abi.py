"""CPU checks of the C interface: the library loads, exports every function
the headers declare, and validates problems without a device."""
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(stfas_[a-zA-Z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_function():
    from paper_1608_01102_amd import _lib
    lib = _lib.load()
    declared = _declared()
    assert len(declared) >= 20
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_lib.EXPORTED) == declared


def test_workspace_bytes_and_validation():
    from paper_1608_01102_amd import stfas as S
    ok = S.make_problem((32, 32), 10, 1e-3)
    b = S.stfas_workspace_bytes(ok)
    assert b > 0
    # more steps -> more memory, and 3D footprint within the paper's bound
    # M = 8 n^d (1+d) N values (memory analysis of Sec. 5) times the word size
    assert S.stfas_workspace_bytes(S.make_problem((32, 32), 20, 1e-3)) > b
    p3 = S.make_problem((64, 64, 64), 60, 1e-3, precision="mixed")
    b3 = S.stfas_workspace_bytes(p3)
    assert 0 < b3 < 2 * (4 * 8 * 64 ** 3 * 4 * 60)
    bad = [S.make_problem((2, 32), 10, 1e-3), S.make_problem((32, 32), 0, 1e-3), S.make_problem((32, 32), 10, 0.0),
           S.make_problem((32, 32), 10, -1.0), S.make_problem((33, 33), 4, 1.0)]
    bad[-1].dim = 4
    for p in bad:
        assert S.stfas_workspace_bytes(p) == 0
    # a grid whose coarsest Poisson level would be too large for the dense solve
    assert S.stfas_workspace_bytes(S.make_problem((97, 97), 2, 1.0)) == 0
    assert S.stfas_step_work_bytes(S.make_problem((128, 128, 128), 1, 1.0, precision="mixed")) > 0
    assert S.stfas_step_vcycles(ok) > 0


def test_density_operator_selection():
    """The density operator is part of the problem: an unknown value is
    rejected, and the upwind exponential adds its series buffers (48 terms,
    two recursion fields, per-step counts) to the workspace and the step's
    scratch, and in 2D the solver's workspace also keeps the 48 terms of every
    step of two density trajectories."""
    from paper_1608_01102_amd import stfas as S
    sl = S.make_problem((32, 32), 10, 1e-3)
    up = S.make_problem((32, 32), 10, 1e-3, density="upwind")
    bad = S.make_problem((32, 32), 10, 1e-3)
    bad.density_op = 2
    assert S.stfas_workspace_bytes(bad) == 0 and S.stfas_step_work_bytes(bad) == 0
    cells = 32 * 32
    extra = S.stfas_workspace_bytes(up) - S.stfas_workspace_bytes(sl)
    stored = 2 * 10 * 48 * cells * 8
    assert 50 * cells * 8 + stored <= extra <= 50 * cells * 8 + stored + 4096
    extra_step = S.stfas_step_work_bytes(up) - S.stfas_step_work_bytes(sl)
    assert 50 * cells * 8 <= extra_step <= 50 * cells * 8 + 4096


def test_velocity_operator_selection():
    """The rotational velocity operator: an unknown value is rejected before
    any allocation; the forward step takes it with the same scratch as the
    semi-Lagrangian one plus the adjoint's iterates."""
    from paper_1608_01102_amd import stfas as S
    ok = S.make_problem((32, 32), 10, 1e-3, velocity="rotational")
    assert S.stfas_workspace_bytes(ok) > 0
    # its smoother keeps a record of 24 words (21 used) per (cell, slot) in
    # LDS while one cell's N records fit in 64 KB (no workspace); beyond, per
    # (cell of the largest colour, slot) in the workspace (256-byte rounded)
    for prec, word in (("fp64", 8), ("mixed", 4)):
        for N in (10, 65536 // (24 * word) + 1):
            extra = (S.stfas_workspace_bytes(S.make_problem((32, 32), N, 1e-3, velocity="rotational", precision=prec)) -
                     S.stfas_workspace_bytes(S.make_problem((32, 32), N, 1e-3, precision=prec)))
            assert extra == (0 if N == 10 else (16 * 16 * N * 24 * word + 255) // 256 * 256), (prec, N)
    # the step's scratch gains the adjoint's fixed-point iterates (4) and two cotangents, one face field each
    nf = 33 * 32 + 32 * 33
    assert S.stfas_step_work_bytes(ok) == S.stfas_step_work_bytes(S.make_problem((32, 32), 10, 1e-3)) + \
        6 * ((nf * 8 + 255) // 256 * 256)
    # 3D: the local records of a 16^3 x 10 colour fit the one-launch form (no workspace); at 64^3 the
    # finest colour (32^3 cells) takes the three launches, records of 56 words per (cell, slot)
    for loc in ("finest", "collapsed", "exact"):
        p3 = S.make_problem((16, 16, 16), 10, 1e-3, velocity="rotational", scgs_local=loc)
        assert S.stfas_workspace_bytes(p3) == S.stfas_workspace_bytes(S.make_problem((16, 16, 16), 10, 1e-3))
    big = S.stfas_workspace_bytes(S.make_problem((64, 64, 64), 8, 1e-3, velocity="rotational", precision="mixed",
                                                 scgs_local="finest"))
    assert big - S.stfas_workspace_bytes(S.make_problem((64, 64, 64), 8, 1e-3, precision="mixed")) == \
        (32 ** 3 * 8 * 56 * 4 + 255) // 256 * 256
    bad = S.make_problem((32, 32), 10, 1e-3)
    bad.velocity_op = 2
    assert S.stfas_workspace_bytes(bad) == 0
    # the smoother's local matrix: the collapsed form keeps no block scratch; the
    # switch is the rotational operator's only, and 0, 1 or 2
    for loc in ("collapsed", "finest", "default"):
        col = S.make_problem((32, 32), 10, 1e-3, velocity="rotational", scgs_local=loc)
        assert S.stfas_workspace_bytes(col) == S.stfas_workspace_bytes(S.make_problem((32, 32), 10, 1e-3))
    for vel, loc in (("sl", 1), ("sl", 3), ("rotational", 4), ("rotational", -1)):
        assert S.stfas_workspace_bytes(S.make_problem((32, 32), 10, 1e-3, velocity=vel, scgs_local=loc)) == 0


def test_status_strings():
    from paper_1608_01102_amd import _lib
    lib = _lib.load()
    assert lib.stfas_status_string(1) == b"invalid argument"
    assert b"gfx950" in lib.stfas_build_info()


def test_serving_footprint_is_exact_and_monotone():
    from paper_1608_01102_amd import serving, stfas as S
    raw = synthetic_requests()
    fps = []
    for q in raw:
        req = serving.Request(q["rid"], q["arrival"], q["n"], q["num_steps"], q["r"], q["rho0"], q["key_steps"],
                              q["key_rho"], dict(dt=q["dt"]))
        fp = serving.footprint(req, "mixed")
        prob = serving.problem_of(req, "mixed")
        assert fp > S.stfas_workspace_bytes(prob) > 0
        fps.append((int(np.prod(q["n"])) * q["num_steps"], fp))
    fps.sort()
    # larger spacetime problems never need less memory
    assert all(fps[i][1] <= fps[i + 1][1] for i in range(len(fps) - 1) if fps[i][0] < fps[i + 1][0])


def synthetic_requests():
    import synthetic
    return synthetic.c5_requests(0, 12, rate=1.0)


def test_missing_library_fails_loudly():
    """Without the built HIP library every entry point raises: there is no
    CPU fallback.  Run in a fresh interpreter with the library path pointed
    at a file that does not exist."""
    import subprocess
    import sys
    code = (
        "import paper_1608_01102_amd._lib as L\n"
        "L.LIB_PATH = '/nonexistent/libstfas.so'\n"
        "from paper_1608_01102_amd import stfas as S\n"
        "try:\n"
        "    S.stfas_workspace_bytes(S.make_problem((8, 8), 2, 1e-2))\n"
        "except RuntimeError as e:\n"
        "    print('raised:', e)\n"
        "    raise SystemExit(0)\n"
        "raise SystemExit(3)\n"
    )
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "no CPU fallback" in out.stdout


def test_step_work_cache_keyed_on_byte_count(monkeypatch):
    """The differentiation form's cached step scratch is keyed on the
    library's byte count for the problem, so an upwind step (series terms in
    its scratch) after a semi-Lagrangian one of the same grid never reuses
    the smaller buffer; a given buffer shorter than that count is refused
    before any C call."""
    import torch
    from paper_1608_01102_amd import autograd as AG
    from paper_1608_01102_amd import stfas as S
    sl = S.make_problem((32, 32), 1, 1e-3)
    up = S.make_problem((32, 32), 1, 1e-3, density="upwind")
    assert S.stfas_step_work_bytes(up) > S.stfas_step_work_bytes(sl)
    made = []

    def fake_empty(n, dtype=None, device=None):
        made.append(n)
        return torch.zeros(n, dtype=dtype)
    monkeypatch.setattr(AG.torch, "empty", fake_empty)
    monkeypatch.setattr(AG._Work, "_cache", {})
    a = AG._Work.get(sl, "cpu")
    b = AG._Work.get(up, "cpu")
    assert a is not b and b.numel() == S.stfas_step_work_bytes(up)
    assert AG._Work.get(sl, "cpu") is a and made == [S.stfas_step_work_bytes(sl), S.stfas_step_work_bytes(up)]
    monkeypatch.undo()
    short = torch.zeros(S.stfas_step_work_bytes(up) - 1, dtype=torch.uint8)
    with pytest.raises(ValueError):
        S._step_work(up, short, "cpu")
    assert S._step_work(sl, short, "cpu") is short
