"""The oracle's ADMM solve against its regression record (tests/golden/
oracle_tiny_solves.json, written by tests/golden/make_golden.py from the
oracle alone).  The record is not an independent pin: it makes any change to
the oracle's arithmetic visible, so that it is regenerated on purpose.
Iteration and V-cycle counts exactly; values to 1e-10 relative (summation
order may differ between BLAS builds)."""
import json

import numpy as np
import pytest

from golden import make_golden

with open(make_golden.OUT) as f:
    RECORD = json.load(f)


@pytest.mark.parametrize("name", sorted(make_golden.CASES))
def test_oracle_matches_its_record(name):
    want = RECORD["cases"][name]
    got = make_golden.run(name)
    assert got["admm_iters"] == want["admm_iters"]
    assert got["vcycles"] == want["vcycles"]
    for k in ("objective", "objective_l2", "reg_term", "u_norm"):
        assert abs(got[k] - want[k]) <= 1e-10 * max(abs(want[k]), 1e-300), k
    assert np.allclose(got["u_sample"], want["u_sample"], rtol=1e-10, atol=1e-12 * want["u_norm"])


def test_record_covers_every_case():
    assert sorted(RECORD["cases"]) == sorted(make_golden.CASES)
    assert RECORD["sample_stride"] == make_golden.SAMPLE
