"""The oracle against its stored results on one small seeded grid
(tests/golden/oracle_small_case.json, written by tests/golden/make_golden.py
from the oracle alone): a later change to the oracle's arithmetic shows up
here.  Assembly is compared to rounding; solve-derived values to what the
summation order of the dot products (thread count) can move them."""
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_golden  # noqa: E402


def _close(got, want, rtol):
    got, want = np.asarray(got, float), np.asarray(want, float)
    assert np.all(np.abs(got - want) <= rtol * np.maximum(np.abs(want), 1e-300)), (got, want)


def test_oracle_matches_stored_small_case():
    want = json.load(open(os.path.join(HERE, "golden", "oracle_small_case.json")))
    got = make_golden.compute()
    assert got["recipe"] == want["recipe"] and got["sample_cells"] == want["sample_cells"]
    # the shell's volume is (4 pi / 3)(2.5^3 - 1) = 19.5 pi whatever the grid
    assert abs(want["volume_sum"] - 19.5 * math.pi) <= 1e-13 * 19.5 * math.pi
    for k in ("dt", "volume_sum", "diag", "cp", "apply_rhs"):
        _close(got[k], want[k], 1e-13)
    for k in ("x", "x_pc2", "grad_nu", "grad_rhs", "rkl2_u1"):
        _close(got[k], want[k], 1e-9)
    assert abs(got["pcg_iterations"] - want["pcg_iterations"]) <= 1
    assert abs(got["pc2_iterations"] - want["pc2_iterations"]) <= 1
    assert got["rkl2_stages"] == want["rkl2_stages"]
