"""Grids above 2^31 bytes per FP64 array.  272 x 1030 x 1002 = 280.7M cells
(2.25 GB per array, ragged in theta and phi).  Every marching kernel
addresses a block's r planes with 32-bit offsets from the block's first
plane, so cells past the 2 GiB mark of an array must come out exactly as
below it.  Checked through what the FP64 oracle computes at any size: its
residual of the GPU solutions (FP64 PCG, FP32/FP64 refinement, and PC2 in
both), its gradient formula at the GPU's x and lambda, and its RKL2 step
(both the two-stage and the one-stage kernels) on every cell."""
import sys

import numpy as np
import pytest
import torch

from gpu_util import oracle_operator, rel, residual_rounding_floor, to_dev, to_host
from paper_1811_02605_amd import solver as S
from paper_1811_02605_amd import workloads as W

pytestmark = pytest.mark.gpu

SHAPE = (272, 1030, 1002)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def big():
    p = W.make_problem(W.small_config(*SHAPE, seed_index=7))
    assert p.cfg.n * 8 > 2 ** 31
    say(f"large grid inputs ready: {p.cfg.shape} = {p.cfg.n} cells, "
        f"{p.cfg.n * 8 / 2 ** 30:.2f} GiB per FP64 array")
    return p


@pytest.fixture(scope="module")
def big_oracle(big):
    ora = oracle_operator(big)
    say("large grid oracle assembled")
    return ora


@pytest.mark.timeout(600)
def test_large_grid_fp64_and_refined_solves(big, big_oracle):
    grid = S.Grid.from_problem(big)
    rhs = to_dev(big.rhs)
    op = S.Operator(grid, to_dev(big.nu), big.dt, precision="fp32_refined")
    x64, i64 = op.solve(rhs, S.make_opts(rtol=1e-10), allow_notconv=False)
    say(f"large FP64 solve: {i64['iters']} iterations, {i64['seconds']:.3f} s, "
        f"reported residual {i64['rel_resid_true']:.3e}")
    x64 = to_host(x64)
    xr, ir = op.solve(rhs, S.make_opts(rtol=1e-10, precision="fp32_refined"), allow_notconv=False)
    say(f"large refined solve: {ir['iters']} inner, {ir['outer_iters']} outer, {ir['seconds']:.3f} s")
    xr = to_host(xr)
    del op, rhs
    torch.cuda.empty_cache()
    b = big_oracle.rhs_to_b(big.rhs)
    r64, rr = big_oracle.rel_residual(b, x64), big_oracle.rel_residual(b, xr)
    say(f"large grid oracle residuals: fp64 {r64:.3e}, refined {rr:.3e}")
    assert r64 <= 1e-10 and rr <= 1e-10
    # the reported FP64 residual is the oracle's up to rounding
    floor = residual_rounding_floor(big_oracle, b, x64)
    assert abs(i64["rel_resid_true"] - r64) <= floor, (i64["rel_resid_true"], r64, floor)


@pytest.mark.timeout(600)
def test_large_grid_pc2_solves(big, big_oracle):
    """PC2 (block ILU(0) factor and block solves, ragged blocks in theta and
    phi) in FP64 and inside refinement: the factor and the solve address each
    r plane through its own resource, so planes past the 2 GiB mark must
    come out as below it."""
    grid = S.Grid.from_problem(big)
    op = S.Operator(grid, to_dev(big.nu), big.dt, precision="fp32_refined")
    rhs = to_dev(big.rhs)
    xs = {}
    for prec in ("fp64", "fp32_refined"):
        x, info = op.solve(rhs, S.make_opts(rtol=1e-10, precond="pc2", precision=prec),
                           allow_notconv=False)
        say(f"large PC2 solve ({prec}): {info['iters']} iterations, {info['outer_iters']} outer, "
            f"{info['seconds']:.3f} s")
        xs[prec] = to_host(x)
    del op, rhs
    torch.cuda.empty_cache()
    b = big_oracle.rhs_to_b(big.rhs)
    for prec, x in xs.items():
        r = big_oracle.rel_residual(b, x)
        say(f"large PC2 ({prec}) oracle residual {r:.3e}")
        assert r <= 1e-10, prec


@pytest.mark.timeout(600)
def test_large_grid_adjoint_and_gradient(big, big_oracle):
    grid = S.Grid.from_problem(big)
    op = S.Operator(grid, to_dev(big.nu), big.dt)
    o = S.make_opts(rtol=1e-10)
    x, _ = op.solve(to_dev(big.rhs), o, allow_notconv=False)
    gx = (0.05 * x).contiguous()
    lam, gnu, grhs, ainfo = op.adjoint(x, gx, o, allow_notconv=False)
    say(f"large adjoint: {ainfo['iters']} iterations, {ainfo['seconds']:.3f} s")
    x, lam, gnu, grhs, gx = (to_host(t) for t in (x, lam, gnu, grhs, gx))
    del op
    torch.cuda.empty_cache()
    ra = big_oracle.rel_residual(gx, lam)
    gnu_o, grhs_o = big_oracle.gradient(x, lam)
    e_nu, e_rhs = rel(gnu, gnu_o), rel(grhs, grhs_o)
    say(f"large adjoint oracle residual {ra:.3e}; gradient vs oracle formula: nu {e_nu:.2e}, "
        f"rhs {e_rhs:.2e}")
    assert ra <= 1e-10 and e_nu <= 1e-12 and e_rhs <= 1e-14
    # every plane, the ones past the 2 GiB mark included
    n_plane = SHAPE[1] * SHAPE[2]
    m_cross = (2 ** 31) // (8 * n_plane)
    for m in (0, m_cross - 1, m_cross, m_cross + 1, SHAPE[0] - 1):
        assert rel(gnu[m], gnu_o[m]) <= 1e-12, m


@pytest.mark.timeout(600)
def test_large_grid_sts_step(big):
    """One RKL2 step at dt/10 (a few stages, so that the oracle's step
    stays short, and at least three, so that the two-stage kernel runs), by
    the two-stage kernel and by one stage per kernel."""
    dt = big.dt / 10.0
    grid = S.Grid.from_problem(big)
    op = S.Operator(grid, to_dev(big.nu), dt)
    u0 = to_dev(big.rhs)
    u1, info = op.sts_step(u0)
    u1s, info_s = op.sts_step(u0, stage_pairs=False)
    s = info["stages"]
    assert s >= 3 and info["stages_per_kernel"] == 2
    same = bool(torch.equal(u1, u1s))
    u1, u1s = to_host(u1), to_host(u1s)
    del op, u0
    torch.cuda.empty_cache()
    ora = oracle_operator(big, dt=dt)
    assert s == ora.rkl2_stages() and info_s["stages"] == s
    want = ora.rkl2_step(big.rhs, stages=s)
    scale = float(np.abs(big.rhs).max())
    err = float(np.abs(u1 - want).max()) / scale
    err_s = float(np.abs(u1s - want).max()) / scale
    say(f"large RKL2 ({s} stages): max error vs oracle {err:.2e} (pairs), {err_s:.2e} (single), "
        f"bitwise equal: {same}")
    assert err <= 1e-12 and err_s <= 1e-12 and same


# 16M-cell theta-phi planes: a block's window of 16 planes plus halos would
# pass 2 GiB, so every marching kernel's chunk is capped (at 9 planes here:
# 2^31 bytes / 128 MiB per plane, less the halo allowance), and the grid,
# 20 x 4000 x 4000 = 320M cells, has 2.56 GB per FP64 array.
WIDE = (20, 4000, 4000)


@pytest.fixture(scope="module")
def wide():
    p = W.make_problem(W.small_config(*WIDE, seed_index=8))
    say(f"wide-plane inputs ready: {p.cfg.shape} = {p.cfg.n} cells")
    return p


@pytest.mark.timeout(900)
def test_wide_planes_capped_chunks(wide):
    grid = S.Grid.from_problem(wide)
    op = S.Operator(grid, to_dev(wide.nu), wide.dt)
    x, info = op.solve(to_dev(wide.rhs), S.make_opts(rtol=1e-10), allow_notconv=False)
    say(f"wide FP64 solve: {info['iters']} iterations, {info['seconds']:.3f} s")
    x = to_host(x)
    dt = wide.dt / 10.0
    del op
    op = S.Operator(grid, to_dev(wide.nu), dt)
    u0 = to_dev(wide.rhs)
    u1, sinfo = op.sts_step(u0)
    assert sinfo["stages"] >= 3 and sinfo["stages_per_kernel"] == 2
    u1s, _ = op.sts_step(u0, stage_pairs=False)
    same = bool(torch.equal(u1, u1s))
    u1 = to_host(u1)
    del op, u0, u1s
    torch.cuda.empty_cache()
    ora = oracle_operator(wide)
    r = ora.rel_residual(ora.rhs_to_b(wide.rhs), x)
    del ora, x
    ora = oracle_operator(wide, dt=dt)
    want = ora.rkl2_step(wide.rhs, stages=sinfo["stages"])
    err = float(np.abs(u1 - want).max()) / float(np.abs(wide.rhs).max())
    say(f"wide grid: oracle residual {r:.3e}; RKL2 ({sinfo['stages']} stages) max error {err:.2e}, "
        f"pairs equal single stages: {same}")
    assert r <= 1e-10 and err <= 1e-12 and same
