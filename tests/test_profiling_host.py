"""Host logic of the measurement module, on synthetic inputs (CPU only):
the counter calibration, the selection of the upwind series' working
launches, and the source hash that guards a committed counter summary."""
import csv
import os

from paper_1608_01102_amd import profiling as P

FIELDS = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]


def _write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_pmc_scales_by_the_calibration_copy(tmp_path):
    """A counter that reads half of the copy's bytes is scaled by 2; other
    kernels, other grid sizes and small copies are ignored."""
    copy_kib = P.COPY_BYTES / 1024.0
    rows = [("__amd_rocclr_copyBuffer", 131072, "FETCH_SIZE", copy_kib / 2)] * 4
    rows += [("__amd_rocclr_copyBuffer", 64, "FETCH_SIZE", 3.0)]                 # small copy
    rows += [("void stfas::k_kkt_split<float, 2>(...)", 2951168, "FETCH_SIZE", 100.0),
             ("void stfas::k_kkt_split<float, 2>(...)", 2951168, "FETCH_SIZE", 300.0),
             ("void stfas::k_kkt_split<float, 2>(...)", 1024, "FETCH_SIZE", 1e9),     # other level
             ("void stfas::k_advect<float, 2>(...)", 2951168, "FETCH_SIZE", 1e9),     # other kernel
             ("void stfas::k_kkt_split<float, 2>(...)", 2951168, "WRITE_SIZE", 1e9)]  # other counter
    _write_csv(str(tmp_path / "run" / "run_counter_collection.csv"), rows)
    out = P.pmc(str(tmp_path), "FETCH_SIZE", "kkt_split", 2951168)
    assert out["dispatches"] == 2 and out["copy_dispatches"] == 4
    assert abs(out["scale"] - 2.0) < 1e-12
    assert abs(out["bytes_per_dispatch"] - 200.0 * 1024 * 2.0) < 1e-6


def test_pmc_min_frac_drops_launches_that_return_at_once(tmp_path):
    """Dispatches reading below min_frac of the largest (series terms past the
    stop) leave the average; none is dropped without min_frac."""
    copy_kib = P.COPY_BYTES / 1024.0
    rows = [("__amd_rocclr_copyBuffer", 131072, "WRITE_SIZE", copy_kib)] * 4
    rows += [("void stfas::k_up_term<float, 2>(...)", 16384, "WRITE_SIZE", v)
             for v in (64.0, 64.0, 48.0, 0.0, 0.0, 0.06)]
    _write_csv(str(tmp_path / "run" / "run_counter_collection.csv"), rows)
    out = P.pmc(str(tmp_path), "WRITE_SIZE", "up_term", 16384, "0.25")
    assert out["dispatches"] == 3 and out["dropped_below_min_frac"] == 3
    assert abs(out["bytes_per_dispatch"] - (176.0 / 3) * 1024) < 1e-6
    out = P.pmc(str(tmp_path), "WRITE_SIZE", "up_term", 16384)
    assert out["dispatches"] == 6 and out["dropped_below_min_frac"] == 0


def test_upwind_term_row_takes_terms_one_to_k():
    """Launches of each 49-launch series in order: term 0 (the copy) and
    the terms after k are left out of the average."""
    k = 3
    rows = []
    for _ in range(2):
        durs = [1000.0] + [8000.0] * k + [500.0] * (49 - 1 - k)
        rows += [("void stfas::k_up_term<float, 3>(...)", 256, 1, 1, d) for d in durs]
    rows.insert(5, ("void stfas::k_fill<float>(...)", 64, 1, 1, 99999.0))
    C, F = 1000, 3300
    line = P.upwind_term_row(rows, k, C, F)
    cells = [c.strip() for c in line.strip("|").split("|")]
    assert cells[2] == str(2 * k)                          # launches averaged
    assert cells[3] == "8.0"                               # µs
    assert cells[4] == f"{(16 * C + 4 * F) / 1e6:.1f}"
    # an incomplete trace (not a whole number of series) gives no row
    assert P.upwind_term_row(rows[:-1], k, C, F) is None


def test_source_hash_covers_the_kernel_sources():
    h = P.kernel_source_hash()
    assert h == P.kernel_source_hash() and len(h) == 16
    int(h, 16)


def test_serving_admission_order():
    """Admission of the continuous-batching server (host logic): arrival
    order, a fitting request may pass a head that does not fit, at most
    max_bypass times in a row, and nothing that has not arrived is taken."""
    import types
    from paper_1608_01102_amd.serving import pick_next
    q = [types.SimpleNamespace(rid=i, arrival=float(i)) for i in range(4)]
    fps = {0: 10, 1: 3, 2: 3, 3: 1}
    assert pick_next(q, fps, None, 20, 0, 8) == 0          # head fits: first come first served
    assert pick_next(q, fps, None, 5, 0, 8) == 1           # head does not fit: the next fitting one passes it
    assert pick_next(q, fps, None, 5, 8, 8) is None        # passed too often: nothing passes it any more
    assert pick_next(q, fps, 1.5, 5, 0, 8) == 1            # request 1 has arrived at t = 1.5
    assert pick_next(q, fps, 0.5, 5, 0, 8) is None         # at t = 0.5 only the (too large) head has arrived
    assert pick_next(q, fps, None, 2, 0, 8) == 3           # only the smallest fits
    assert pick_next(q, fps, None, 0, 0, 8) is None
