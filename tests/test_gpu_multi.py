"""GPU parity of the solve with several right-hand sides (mas_pcg_solve_multi):
each component against the FP64 oracle (its residual of the GPU solution and
the error against its own tight solution), against the single-right-hand-side
solve of the same component, independent stopping of the components, and the
error paths."""
import sys

import numpy as np
import pytest
import torch

from gpu_util import DEV, gpu_operator, oracle_operator, problem, rel, to_dev, to_host
from paper_1811_02605_amd import _abi as abi
from paper_1811_02605_amd import solver as S
from paper_1811_02605_amd import workloads as W

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4, 8), (5, 7, 13), (3, 9, 70), (33, 17, 129), (65, 8, 64), (1, 3, 2), (6, 3, 1),
          (9, 16, 32)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rhs(p, m):
    return W.component_rhs(p.cfg, m)


# 0: the automatic r-chunk length (short chunks on these small grids); 16:
# the chunk length of grids large enough to fill the GPU
@pytest.mark.parametrize("chunk", [0, 16])
@pytest.mark.parametrize("m", [2, 3, 4])
@pytest.mark.parametrize("shape", SHAPES + ["c0"])
def test_components_match_oracle(shape, m, chunk):
    p = problem(shape, (0, 1))
    _, op = gpu_operator(p)
    ora = oracle_operator(p)
    B = _rhs(p, m)
    X, infos = op.solve_multi(to_dev(B), S.make_opts(rtol=1e-10, chunk_planes=chunk),
                              allow_notconv=False)
    X = to_host(X)
    for h in range(m):
        b = ora.rhs_to_b(B[h])
        res = ora.rel_residual(b, X[h])
        assert infos[h]["status"] == abi.MAS_OK and res <= 1e-10, (h, res, infos[h])
        xo = ora.pcg(b, tol=1e-13)[0]
        assert rel(X[h], xo) <= 1e-6


@pytest.mark.parametrize("chunk", [0, 16])
@pytest.mark.parametrize("m", [1, 3])
@pytest.mark.parametrize("shape", [(33, 17, 129), (9, 16, 32), "c0"])
def test_components_match_single_solves(shape, m, chunk):
    """The per-component iterations are those of the single solve launched
    per iteration (the same blocking of the dot products): same iteration
    counts, solutions equal to rounding."""
    p = problem(shape, (0, 0))
    _, op = gpu_operator(p)
    B = _rhs(p, m)
    # (one right-hand side would otherwise go into the persistent launch,
    # with its own chunks)
    o = S.make_opts(rtol=1e-10, chunk_planes=chunk, launch="per_iteration")
    X, infos = op.solve_multi(to_dev(B), o, allow_notconv=False)
    for h in range(m):
        x1, i1 = op.solve(to_dev(B[h]), o, allow_notconv=False)
        assert infos[h]["iters"] == i1["iters"], (h, infos[h], i1)
        assert rel(to_host(X[h]), to_host(x1)) <= 1e-13
        say(f"{shape} m={m} h={h}: {i1['iters']} iterations, bitwise equal: "
            f"{bool(torch.equal(X[h], x1))}")


def test_independent_stopping():
    """A zero component, a component already solved (warm start) and two hard
    ones of very different scale: each stops on its own test, the finished
    ones are left untouched."""
    p = problem((33, 17, 129), (0, 0))
    _, op = gpu_operator(p)
    ora = oracle_operator(p)
    B = _rhs(p, 4)
    B[0] = 0.0
    B[3] *= 1e-9
    x_sol, _ = op.solve(to_dev(B[2]), S.make_opts(rtol=1e-12), allow_notconv=False)
    X0 = np.zeros_like(B)
    X0[2] = to_host(x_sol)
    X, infos = op.solve_multi(to_dev(B), S.make_opts(rtol=1e-10), x0=to_dev(X0),
                              allow_notconv=False)
    X = to_host(X)
    assert np.all(X[0] == 0.0) and infos[0]["iters"] == 0 and infos[0]["status"] == abi.MAS_OK
    # the warm start is scaled by w and back: equal to rounding
    assert infos[2]["iters"] == 0 and rel(X[2], X0[2]) <= 1e-15
    for h in (1, 3):
        assert infos[h]["iters"] > 0
        assert ora.rel_residual(ora.rhs_to_b(B[h]), X[h]) <= 1e-10


def test_deterministic_and_timing():
    p = problem("c0", (0, 0))
    _, op = gpu_operator(p)
    B = to_dev(_rhs(p, 3))
    # timing samples need the launches per iteration; the untimed run is
    # launched the same way (the automatic choice here is the persistent
    # launch, whose chunks sum the dot products in another order)
    a, ia = op.solve_multi(B, S.make_opts(sample_timing=1))
    b, _ = op.solve_multi(B, S.make_opts(launch="per_iteration"))
    assert torch.equal(a, b)
    c, ic = op.solve_multi(B)
    d, _ = op.solve_multi(B)
    assert torch.equal(c, d) and ic[0]["launch"] == abi.MAS_LAUNCH_PERSISTENT
    assert all(i["iter_kernel_samples"] > 0 and i["iter_kernel_us"] > 0 for i in ia)


# single-precision inner PCG inside double-precision refinement, several
# right-hand sides: PC1 with either refinement strategy, PC2 (restarted)
REFINED = [("pc1", "reliable"), ("pc1", "restart"), ("pc2", "restart")]


@pytest.mark.parametrize("chunk", [0, 16])
@pytest.mark.parametrize("m", [2, 3, 4])
@pytest.mark.parametrize("precond,refine", REFINED)
@pytest.mark.parametrize("shape", [(5, 7, 13), (33, 17, 129), (1, 3, 2), (9, 16, 32), "c0"])
def test_refined_components_match_oracle(shape, precond, refine, m, chunk):
    """Each component of a refined solve of several right-hand sides meets
    1e-10 by the oracle's own residual and lies within 1e-6 of its 1e-13
    solution."""
    p = problem(shape, (0, 1))
    _, op = gpu_operator(p, "fp32_refined")
    ora = oracle_operator(p)
    B = _rhs(p, m)
    o = S.make_opts(rtol=1e-10, precision="fp32_refined", precond=precond, refine=refine,
                    chunk_planes=chunk)
    X, infos = op.solve_multi(to_dev(B), o, allow_notconv=False)
    X = to_host(X)
    for h in range(m):
        b = ora.rhs_to_b(B[h])
        res = ora.rel_residual(b, X[h])
        assert infos[h]["status"] == abi.MAS_OK and res <= 1e-10, (h, res, infos[h])
        assert infos[h]["outer_iters"] >= 1
        assert rel(X[h], ora.pcg(b, tol=1e-13)[0]) <= 1e-6


@pytest.mark.parametrize("m", [2, 3])
@pytest.mark.parametrize("precond,refine", REFINED)
@pytest.mark.parametrize("shape", [(33, 17, 129), "c0"])
def test_refined_components_equal_single_refined_solves(shape, precond, refine, m):
    """Each component of the shared refined solve takes the inner and outer
    iterations of its single refined solve launched per iteration and gives
    the same solution bit for bit (the same kernels and sums per
    component)."""
    p = problem(shape, (0, 0))
    _, op = gpu_operator(p, "fp32_refined")
    B = _rhs(p, m)
    # both launched per iteration (the same blocking of the dot products)
    o = S.make_opts(rtol=1e-10, precision="fp32_refined", precond=precond, refine=refine,
                    launch="per_iteration")
    X, infos = op.solve_multi(to_dev(B), o, allow_notconv=False)
    for h in range(m):
        x1, i1 = op.solve(to_dev(B[h]), o, allow_notconv=False)
        assert (infos[h]["iters"], infos[h]["outer_iters"]) == (i1["iters"], i1["outer_iters"]), h
        assert torch.equal(X[h], x1), h


def test_refined_independent_stopping():
    """A zero component, a warm start at the solution and a component 1e9
    smaller stop on their own in the refined solve of several right-hand
    sides."""
    p = problem((9, 16, 32), (0, 0))
    _, op = gpu_operator(p, "fp32_refined")
    ora = oracle_operator(p)
    B = _rhs(p, 4)
    B[0] = 0.0
    B[3] *= 1e-9
    o = S.make_opts(rtol=1e-10, precision="fp32_refined")
    x_sol, _ = op.solve(to_dev(B[2]), S.make_opts(rtol=1e-12, precision="fp32_refined"),
                        allow_notconv=False)
    X0 = np.zeros_like(B)
    X0[2] = to_host(x_sol)
    X, infos = op.solve_multi(to_dev(B), o, x0=to_dev(X0), allow_notconv=False)
    X = to_host(X)
    assert np.all(X[0] == 0.0) and infos[0]["iters"] == 0 and infos[0]["status"] == abi.MAS_OK
    assert infos[2]["iters"] == 0 and rel(X[2], X0[2]) <= 1e-15
    for h in (1, 3):
        assert ora.rel_residual(ora.rhs_to_b(B[h]), X[h]) <= 1e-10


def test_error_paths():
    p = problem((9, 16, 32), (0, 0))
    _, op = gpu_operator(p, "fp32_refined")
    B = to_dev(_rhs(p, 3))
    # an operator built without single-precision couplings cannot run refined
    _, op64 = gpu_operator(p)
    with pytest.raises(abi.MasError, match="single-precision coefficients"):
        op64.solve_multi(B, S.make_opts(precision="fp32_refined"))
    # refinement-step and iteration limits: ENOTCONV with the last iterates
    X, infos = op.solve_multi(B, S.make_opts(precision="fp32_refined", max_outer=1, inner_rtol=0.5))
    assert all(i["status"] == abi.MAS_ENOTCONV and i["outer_iters"] == 1 for i in infos)
    lib = abi.load()
    assert lib.mas_pcg_multi_workspace_bytes(op.handle, 5) == abi.MAS_EINVAL
    assert lib.mas_pcg_multi_workspace_bytes(op.handle, 0) == abi.MAS_EINVAL
    need = int(lib.mas_pcg_multi_workspace_bytes(op.handle, 3))
    one = int(lib.mas_pcg_multi_workspace_bytes(op.handle, 1))
    assert need > 2.9 * (one - 4096)
    x = torch.empty_like(B)
    st = lib.mas_pcg_solve_multi(op.handle, 3, B.data_ptr(), x.data_ptr(), None, x.data_ptr(),
                                 need - 256, None, None)
    assert st == abi.MAS_ENOMEM
    st = lib.mas_pcg_solve_multi(op.handle, 5, B.data_ptr(), x.data_ptr(), None, x.data_ptr(),
                                 need, None, None)
    assert st == abi.MAS_EINVAL
    # too few iterations: ENOTCONV with the last iterates, per-component status
    _, op64 = gpu_operator(p)
    X, infos = op64.solve_multi(B, S.make_opts(max_iters=3, max_restarts=0))
    assert all(i["status"] == abi.MAS_ENOTCONV for i in infos)
