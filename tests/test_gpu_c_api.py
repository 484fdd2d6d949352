"""The solve of tests/c_api_solve.c: C99 code calling include/mas.h directly
(hipMalloc'd storage and workspace, default options, the null stream), in
FP64 and in FP32 inside FP64 refinement.  Its solutions must equal those of
the Python binding on the same inputs bit for bit, and meet the tolerance in
the oracle's residual."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from gpu_util import DEV, to_host
from paper_1811_02605_amd import build as B
from paper_1811_02605_amd import solver as S

pytestmark = pytest.mark.gpu

NR, NT, NP = 16, 24, 48


def test_c_program_matches_binding_and_oracle(tmp_path):
    lib = ctypes.CDLL(B.C_PROGRAM)
    lib.c_api_solve_run.argtypes = [ctypes.c_char_p]
    lib.c_api_solve_run.restype = ctypes.c_int
    out = tmp_path / "c_api_solve.bin"
    assert lib.c_api_solve_run(str(out).encode()) == 0
    n = NR * NT * NP
    data = np.fromfile(out, dtype=np.float64)
    assert data.size == NR + 1 + NT + 1 + 3 * n
    rf, tf = data[:NR + 1], data[NR + 1:NR + NT + 2]
    rhs = data[NR + NT + 2:NR + NT + 2 + n].reshape(NR, NT, NP)
    x64 = data[NR + NT + 2 + n:NR + NT + 2 + 2 * n].reshape(NR, NT, NP)
    x32 = data[NR + NT + 2 + 2 * n:].reshape(NR, NT, NP)

    grid = S.Grid(rf, tf, NP)
    nu = np.full((NR, NT, NP), 1e-3)
    op = S.Operator(grid, torch.from_numpy(nu).to(DEV), 1.0, precision="fp32_refined")
    r = torch.from_numpy(rhs).to(DEV)
    y64, _ = op.solve(r, S.make_opts(), allow_notconv=False)
    y32, _ = op.solve(r, S.make_opts(precision="fp32_refined"), allow_notconv=False)
    assert np.array_equal(to_host(y64), x64)
    assert np.array_equal(to_host(y32), x32)

    ora = oracle.Operator(rf, tf, NP, nu, 1.0)
    b = ora.rhs_to_b(rhs)
    assert ora.rel_residual(b, x64) <= 1e-10
    assert ora.rel_residual(b, x32) <= 1e-10
