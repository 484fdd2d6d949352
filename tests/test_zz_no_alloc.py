"""The allocation-free solve (mas_pcg_solve_noalloc, workspace in the
library's static device array) against the solve with a caller workspace
(mas_pcg_solve), through the C ABI: two calls in a row, the second on a
smaller grid, so the second call runs on the array the first one left
behind; and the size limit."""
import ctypes

import pytest
import torch

from gpu_util import DEV, gpu_operator, problem, to_dev
from paper_1811_02605_amd import _abi as abi
from paper_1811_02605_amd import solver as S

pytestmark = pytest.mark.gpu

CASES = [
    ("fp64", "pc1"),
    ("fp32_refined", "pc1"),
    ("fp64", "pc2"),
    ("fp32_refined", "pc2"),
]


def _noalloc(op, rhs, o, x=None):
    x = torch.empty_like(rhs) if x is None else x
    info = abi.mas_pcg_info()
    st = abi.load().mas_pcg_solve_noalloc(op.handle, rhs.data_ptr(), x.data_ptr(), ctypes.byref(o),
                                          None, ctypes.byref(info))
    torch.cuda.synchronize()
    return st, x, info.as_dict()


@pytest.mark.parametrize("precision,precond", CASES)
def test_noalloc_equals_workspace_solve_on_two_calls(precision, precond):
    # c0 (32 x 32 x 64, 65,536 cells), then a smaller ragged grid
    for shape in ("c0", (5, 7, 13)):
        p = problem(shape)
        print(f"noalloc {precision}/{precond} on {p.shape}", flush=True)
        _, op = gpu_operator(p, precision)
        rhs = to_dev(p.rhs)
        o = S.make_opts(rtol=1e-10, precision=precision, precond=precond)
        x_ref, i_ref = op.solve(rhs, o, allow_notconv=False)
        st, x, info = _noalloc(op, rhs, o)
        assert st == abi.MAS_OK, abi.last_error()
        assert info["iters"] == i_ref["iters"] and info["outer_iters"] == i_ref["outer_iters"]
        # the same kernels on the same data in the same order: the same bits
        assert torch.equal(x, x_ref)
        assert info["rel_resid_true"] == i_ref["rel_resid_true"] <= 1e-10


def test_noalloc_limits():
    lib = abi.load()
    p = problem((5, 7, 13))
    _, op = gpu_operator(p)
    rhs = to_dev(p.rhs)
    o = S.make_opts(sample_timing=1)
    st, _, _ = _noalloc(op, rhs, o)
    assert st == abi.MAS_EINVAL and "sample_timing" in abi.last_error()
    # a grid whose workspace exceeds the static array is refused before any work
    p = problem((64, 128, 256))
    _, big = gpu_operator(p)
    o = S.make_opts()
    need = lib.mas_pcg_workspace_bytes(big.handle, ctypes.byref(o))
    assert need > abi.MAS_NOALLOC_WORK_BYTES
    x = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
    st, _, _ = _noalloc(big, to_dev(p.rhs), o, x)
    assert st == abi.MAS_ENOMEM and "allocation-free" in abi.last_error()
    # the solution buffer was not touched
    assert torch.count_nonzero(x) == 0
