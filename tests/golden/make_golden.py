"""Writes tests/golden/oracle_small_case.json: the FP64 oracle's results on one
small seeded grid, stored so that a later change to the oracle's arithmetic
shows up as a difference.  The paper prints no worked example for this
operator (its numbers are iteration counts and timings of the MAS run), so
these fixtures are the oracle's own, not the paper's; what pins the oracle to
the mathematics are the tests in tests/test_oracle_*.py.

Calls only oracle/ (and the seeded input generator, which holds none of the
method's arithmetic):

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1811_02605_amd import workloads as W  # noqa: E402

SHAPE = (5, 6, 8)
BC = (0, 1)  # Dirichlet at r = 1, Neumann at r = 2.5
SAMPLE = [0, 7, 61, 123, 239]  # flat cell indices (phi fastest)


def compute():
    p = W.make_problem(W.small_config(*SHAPE, seed_index=3))
    ora = oracle.Operator(p.r_faces, p.t_faces, SHAPE[2], p.nu, p.dt, *BC)
    b = ora.rhs_to_b(p.rhs)
    x, it, _, rt = ora.pcg(b, tol=1e-13)
    x2, it2, _, _ = ora.pcg_pc2(b, (2, 3, 4), tol=1e-13)
    lam = ora.pcg(x, tol=1e-13)[0]
    gnu, grhs = ora.gradient(x, lam)
    s = ora.rkl2_stages()
    u1 = ora.rkl2_step(p.rhs, stages=s)
    f = lambda a: [float(v) for v in np.asarray(a).reshape(-1)[SAMPLE]]
    return {
        "recipe": f"workloads.small_config{SHAPE}, seed_index=3, walls {BC}; "
                  "PCG and PC2-PCG (blocks 2 x 3 x 4) to 1e-13 from x0 = 0; "
                  "lambda = A^-1 x; RKL2 step of dt from u0 = rhs",
        "sample_cells": SAMPLE,
        "dt": p.dt,
        "volume_sum": float(ora.V.sum()),
        "diag": f(ora.diag),
        "cp": f(ora.cp),
        "apply_rhs": f(ora.apply(p.rhs)),
        "pcg_iterations": int(it),
        "pc2_iterations": int(it2),
        "x": f(x),
        "x_pc2": f(x2),
        "grad_nu": f(gnu),
        "grad_rhs": f(grhs),
        "rkl2_stages": int(s),
        "rkl2_u1": f(u1),
    }


if __name__ == "__main__":
    out = os.path.join(HERE, "oracle_small_case.json")
    with open(out, "w") as fh:
        json.dump(compute(), fh, indent=1)
        fh.write("\n")
    print(out)
