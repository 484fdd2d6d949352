"""GPU parity of the block-Jacobi ILU(0) preconditioner (PC2) against the FP64
oracle's PC2-PCG (same blocks 8 x 8 x 64, natural order, periodic phi
coupling left out of the blocks) on seeded inputs: solutions, iterates,
iteration counts, ragged grids in every direction, and the error paths."""
import sys

import numpy as np
import pytest

from gpu_util import (gpu_operator, oracle_operator, problem, rel, residual_rounding_floor, to_dev,
                      to_host)
from paper_1811_02605_amd import _abi as abi
from paper_1811_02605_amd import solver as S

pytestmark = pytest.mark.gpu

BLOCKS = (8, 8, 64)
# one block, several blocks with ragged ends in every direction, 1-cell directions
SHAPES = [(4, 4, 8), (9, 17, 33), (17, 9, 70), (8, 8, 64), (3, 1, 5), (1, 3, 2), (6, 3, 1),
          (12, 10, 130), "c0"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", [(0, 0), (1, 0)])
def test_pc2_solve_matches_oracle(shape, bc):
    p = problem(shape, bc)
    _, op = gpu_operator(p)
    ora = oracle_operator(p)
    b = ora.rhs_to_b(p.rhs)
    x, info = op.solve(to_dev(p.rhs), S.make_opts(rtol=1e-10, precond="pc2"), allow_notconv=False)
    x = to_host(x)
    res = ora.rel_residual(b, x)
    xo, it_o, _, _ = ora.pcg_pc2(b, BLOCKS, tol=1e-10)
    say(f"{shape} bc={bc}: gpu {info['iters']} it, oracle {it_o} it, residual {res:.2e}")
    assert res <= 1e-10
    # both test the residual at every iteration; only the summation order of
    # the dot products differs (R17), which can move the crossing by one
    assert abs(info["iters"] - it_o) <= 1
    xt = ora.pcg_pc2(b, BLOCKS, tol=1e-13)[0]
    assert rel(x, xt) <= 1e-6


@pytest.mark.parametrize("chunk", [0, 16])
@pytest.mark.parametrize("shape", [(9, 17, 33), (17, 9, 70), "c0"])
def test_pc2_iterates_match_oracle(shape, chunk):
    p = problem(shape, (0, 0))
    _, op = gpu_operator(p)
    ora = oracle_operator(p)
    b = ora.rhs_to_b(p.rhs)
    rhs = to_dev(p.rhs)
    for k in (1, 2, 5, 10):
        o = S.make_opts(rtol=0.0, max_iters=k, max_restarts=0, precond="pc2", chunk_planes=chunk)
        x, info = op.solve(rhs, o)
        assert info["iters"] == k
        xo = ora.pcg_pc2(b, BLOCKS, tol=0.0, max_iters=k)[0]
        assert rel(to_host(x), xo) <= 1e-11 * k, k


def test_pc2_needs_fewer_iterations_than_pc1():
    p = problem("c0", (0, 0))
    _, op = gpu_operator(p)
    rhs = to_dev(p.rhs)
    _, i1 = op.solve(rhs, S.make_opts(rtol=1e-10), allow_notconv=False)
    _, i2 = op.solve(rhs, S.make_opts(rtol=1e-10, precond="pc2"), allow_notconv=False)
    say(f"c0: PC1 {i1['iters']} iterations, PC2 {i2['iters']}")
    assert i2["iters"] < i1["iters"]


def test_pc2_adjoint_and_warm_start():
    p = problem((9, 17, 33), (0, 1))
    _, op = gpu_operator(p)
    ora = oracle_operator(p)
    o = S.make_opts(rtol=1e-12, precond="pc2")
    x, _ = op.solve(to_dev(p.rhs), o, allow_notconv=False)
    gx = x.clone()
    lam, gnu, grhs, ainfo = op.adjoint(x, gx, o, allow_notconv=False)
    xh, lamh = to_host(x), to_host(lam)
    assert ora.rel_residual(to_host(gx), lamh) <= 1e-12
    gnu_o, grhs_o = ora.gradient(xh, lamh)
    assert rel(to_host(gnu), gnu_o) <= 1e-12
    x2, i2 = op.solve(to_dev(p.rhs), o, x0=x, allow_notconv=False)
    assert i2["iters"] <= 1


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", [(0, 0), (1, 0)])
def test_pc2_refined_matches_oracle(shape, bc):
    """Single-precision PC2-PCG inside double-precision refinement: the
    oracle's residual of the result meets 1e-10 and the result is the
    oracle's 1e-13 PC2 solution to its conditioning."""
    p = problem(shape, bc)
    _, op = gpu_operator(p, "fp32_refined")
    ora = oracle_operator(p)
    b = ora.rhs_to_b(p.rhs)
    x, info = op.solve(to_dev(p.rhs), S.make_opts(rtol=1e-10, precision="fp32_refined",
                                                  precond="pc2"), allow_notconv=False)
    x = to_host(x)
    res = ora.rel_residual(b, x)
    say(f"{shape} bc={bc}: refined PC2 {info['iters']} inner, {info['outer_iters']} outer, "
        f"residual {res:.2e}")
    assert res <= 1e-10
    assert abs(info["rel_resid_true"] - res) <= 1e-3 * res + 1e-13
    assert info["outer_iters"] >= 1
    xt = ora.pcg_pc2(b, BLOCKS, tol=1e-13)[0]
    assert rel(x, xt) <= 1e-6


def test_pc2_refined_fewer_iterations_and_adjoint():
    p = problem("c0", (0, 0))
    _, op = gpu_operator(p, "fp32_refined")
    ora = oracle_operator(p)
    rhs = to_dev(p.rhs)
    o1 = S.make_opts(rtol=1e-10, precision="fp32_refined")
    o2 = S.make_opts(rtol=1e-10, precision="fp32_refined", precond="pc2")
    x1, i1 = op.solve(rhs, o1, allow_notconv=False)
    x2, i2 = op.solve(rhs, o2, allow_notconv=False)
    say(f"c0 refined: PC1 {i1['iters']} inner iterations, PC2 {i2['iters']}")
    assert i2["iters"] < i1["iters"]
    gx = x2.clone()
    lam, gnu, grhs, _ = op.adjoint(x2, gx, o2, allow_notconv=False)
    lamh = to_host(lam)
    assert ora.rel_residual(to_host(gx), lamh) <= 1e-10
    gnu_o, grhs_o = ora.gradient(to_host(x2), lamh)
    assert rel(to_host(gnu), gnu_o) <= 1e-12 and rel(to_host(grhs), grhs_o) <= 1e-14


def test_pc2_refined_autograd():
    """The differentiable solve with PC2 inside refinement: gradients of
    L = 1/2 ||x||^2 against the oracle's formula at its own solutions."""
    import torch
    p = problem((6, 8, 16), (0, 0))
    grid = S.Grid.from_problem(p)
    nu = to_dev(p.nu).requires_grad_(True)
    rhs = to_dev(p.rhs).requires_grad_(True)
    x = S.solve(nu, rhs, grid, p.dt, rtol=1e-12, precision="fp32_refined", precond="pc2")
    (0.5 * (x ** 2).sum()).backward()
    ora = oracle_operator(p)
    xo = ora.solve_rhs(p.rhs, tol=1e-13)
    lo = ora.pcg(xo, tol=1e-13)[0]
    gnu_o, grhs_o = ora.gradient(xo, lo)
    assert rel(to_host(nu.grad), gnu_o) <= 1e-8
    assert rel(to_host(rhs.grad), grhs_o) <= 1e-8


@pytest.mark.parametrize("shape", [(9, 17, 33), (17, 9, 70), (12, 10, 130), (3, 1, 5), "c0"])
@pytest.mark.parametrize("m", [2, 3, 4])
def test_pc2_several_rhs_equal_single_solves(shape, m):
    """PC2 for several right-hand sides (one SpMV launch for all of them):
    each component's iterations and solution are those of its single PC2
    solve, bit for bit, and the oracle's residual of each meets 1e-10."""
    import torch
    from paper_1811_02605_amd import workloads as W
    p = problem(shape, (0, 1))
    _, op = gpu_operator(p)
    ora = oracle_operator(p)
    B = to_dev(W.component_rhs(p.cfg, m))
    o = S.make_opts(rtol=1e-10, precond="pc2")
    X, infos = op.solve_multi(B, o, allow_notconv=False)
    for h in range(m):
        x1, i1 = op.solve(B[h].contiguous(), o, allow_notconv=False)
        assert infos[h]["iters"] == i1["iters"], (h, infos[h]["iters"], i1["iters"])
        assert torch.equal(X[h], x1), h
        res = ora.rel_residual(ora.rhs_to_b(to_host(B[h])), to_host(X[h]))
        floor = residual_rounding_floor(ora, ora.rhs_to_b(to_host(B[h])), to_host(X[h]))
        assert res <= 1e-10 and abs(infos[h]["rel_resid_true"] - res) <= floor


def test_pc2_several_rhs_independent_stopping():
    """A zero component, a component already solved (warm start) and one a
    factor 1e9 smaller stop on their own."""
    import torch
    from paper_1811_02605_amd import workloads as W
    p = problem((9, 17, 33), (0, 0))
    _, op = gpu_operator(p)
    B = to_dev(W.component_rhs(p.cfg, 3))
    B[1] = 0.0
    B[2] *= 1e-9
    o = S.make_opts(rtol=1e-10, precond="pc2")
    X, infos = op.solve_multi(B, o, allow_notconv=False)
    assert infos[1]["iters"] == 0 and float(X[1].abs().max()) == 0.0
    x0, _ = op.solve(B[0].contiguous(), o, allow_notconv=False)
    x2, _ = op.solve(B[2].contiguous(), o, allow_notconv=False)
    assert torch.equal(X[0], x0) and torch.equal(X[2], x2)
    X0 = torch.stack([x0, torch.zeros_like(x0), x2]).contiguous()
    X2, infos2 = op.solve_multi(B, o, x0=X0, allow_notconv=False)
    assert all(i["iters"] <= 1 for i in infos2)


def test_pc2_error_paths():
    p = problem((9, 16, 32), (0, 0))
    _, op = gpu_operator(p, "fp32_refined")
    rhs = to_dev(p.rhs)
    o = S.make_opts(precision="fp32_refined", precond="pc2", max_iters=3, max_outer=20)
    x, info = op.solve(rhs, o)
    assert info["status"] == abi.MAS_ENOTCONV and info["iters"] == 3
    o = S.make_opts()
    o.precond = 7
    with pytest.raises(abi.MasError, match="preconditioner"):
        op.solve(rhs, o)
    _, op64 = gpu_operator(p)
    import torch
    B = torch.stack([rhs, rhs]).contiguous()
    with pytest.raises(abi.MasError, match="single-precision coefficients"):
        op64.solve_multi(B, S.make_opts(precond="pc2", precision="fp32_refined"))
    x, info = op64.solve(rhs, S.make_opts(max_iters=2, max_restarts=0, precond="pc2"))
    assert info["status"] == abi.MAS_ENOTCONV and info["iters"] == 2
