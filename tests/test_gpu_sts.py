"""GPU parity of the RKL2 super time-step (mas_sts_step) against the FP64 CPU
oracle on seeded inputs: small and ragged grids spanning several tiles of both
stage kernels (one stage: 64-cell phi segments, 8-row theta tiles, 16-plane r
chunks; two stages: 60-cell by 12-row tiles with a two-cell overlap ring,
32-plane r chunks; chunks marched in alternating directions), ragged tails in
every direction, odd np (one stage per kernel), every wall combination,
automatic and fixed stage counts, in-place steps.  Steps with two stages per
kernel must equal steps with one stage per kernel bit for bit."""
import sys

import numpy as np
import pytest
import torch

from gpu_util import DEV, gpu_operator, oracle_operator, problem, to_dev, to_host
from paper_1811_02605_amd import _abi as abi

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4, 8), (5, 7, 13), (3, 9, 70), (33, 17, 129), (65, 8, 64), (1, 3, 2), (6, 3, 1),
          (2, 1, 5), (9, 16, 32), (17, 9, 66), (70, 25, 130), (600, 2, 4)]
# spans of the two-stage kernel's tiles: 60 phi cells, 12 theta rows, 32 r
# planes (more beyond 256 planes: 261 gives eight 33-plane chunks)
# (600, 2, 4): 64-plane chunks of the two-stage kernel (its longest), ten of
# them, the last one 24 planes marching down
PAIR_SHAPES = [(70, 25, 130), (33, 13, 64), (3, 1, 2), (1, 12, 4), (40, 26, 122), (65, 8, 64),
               (9, 16, 32), (2, 3, 6), (261, 2, 4), (600, 2, 4)]
BCS = [(0, 0), (1, 0), (1, 1)]

# Both sides round each stage differently (the oracle forms u - (A u)/V from
# assembled coefficients, the kernel the flux sum from nu on the fly, and runs
# the recursion on Y - u0).  With enough stages the recursion is stable and
# the difference stays at a few hundred ulps of max|u0|; below the stable
# count stiff modes grow, rounding with them, so the scale is the larger of
# max|u0| and max|u1|.
ATOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _max_err(got, want, u0):
    scale = max(np.abs(u0).max(), np.abs(want).max(), 1e-300)
    return float(np.abs(got - want).max() / scale)


@pytest.mark.parametrize("shape", SHAPES + ["c0"])
@pytest.mark.parametrize("bc", BCS)
def test_step_matches_oracle(shape, bc):
    p = problem(shape, bc)
    _, op = gpu_operator(p)
    ora = oracle_operator(p)
    s = op.sts_stages()
    assert s == ora.rkl2_stages()
    u0 = np.random.default_rng(21).standard_normal(p.shape)
    u1, info = op.sts_step(to_dev(u0))
    assert info["stages"] == s
    err = _max_err(to_host(u1), ora.rkl2_step(u0, stages=s), u0)
    say(f"{shape} bc={bc}: s={s} z_max={info['z_max']:.4g} max err {err:.2e}")
    assert err <= ATOL


@pytest.mark.parametrize("stages", [2, 3, 4, 5, 8, 61])
@pytest.mark.parametrize("shape", [(33, 17, 129), (9, 16, 32), (6, 3, 1)])
def test_fixed_stage_counts(shape, stages):
    p = problem(shape, (0, 1))
    _, op = gpu_operator(p)
    ora = oracle_operator(p)
    u0 = np.random.default_rng(22).standard_normal(p.shape)
    u1, info = op.sts_step(to_dev(u0), stages=stages)
    assert info["stages"] == stages
    err = _max_err(to_host(u1), ora.rkl2_step(u0, stages=stages), u0)
    assert err <= ATOL, err


def test_z_max_matches_oracle_bound():
    for shape in ((33, 17, 129), "c0"):
        p = problem(shape, (0, 0))
        _, op = gpu_operator(p)
        ora = oracle_operator(p)
        _, info = op.sts_step(to_dev(np.zeros(p.shape)))
        zo = float(np.max(2.0 * (ora.diag - ora.V) / ora.V))
        assert abs(info["z_max"] - zo) <= 1e-13 * zo


def test_in_place_and_repeated_steps():
    p = problem((17, 9, 66), (1, 0))
    _, op = gpu_operator(p)
    ora = oracle_operator(p)
    u0 = np.random.default_rng(23).standard_normal(p.shape)
    u = to_dev(u0)
    want = u0
    for _ in range(4):
        u, _ = op.sts_step(u, out=u)
        want = ora.rkl2_step(want)
    assert _max_err(to_host(u), want, u0) <= 4 * ATOL


def test_fp32_refined_operator_steps_in_double():
    p = problem((9, 16, 32), (0, 0))
    _, op = gpu_operator(p, "fp32_refined")
    ora = oracle_operator(p)
    u0 = np.random.default_rng(24).standard_normal(p.shape)
    u1, _ = op.sts_step(to_dev(u0))
    assert _max_err(to_host(u1), ora.rkl2_step(u0), u0) <= ATOL


def test_neumann_conserves_volume_integral():
    p = problem((33, 17, 129), (1, 1))
    _, op = gpu_operator(p)
    ora = oracle_operator(p)
    u0 = np.random.default_rng(25).standard_normal(p.shape)
    u1, _ = op.sts_step(to_dev(u0))
    u1 = to_host(u1)
    assert abs(np.sum(ora.V * u1) - np.sum(ora.V * u0)) <= 1e-13 * np.sum(ora.V * np.abs(u0))
    # constants are steady states
    c = np.full(p.shape, -3.25)
    cu, _ = op.sts_step(to_dev(c))
    np.testing.assert_allclose(to_host(cu), c, rtol=1e-14, atol=0)


def test_zero_dt_and_zero_field():
    p = problem((9, 16, 32), (0, 0))
    _, op = gpu_operator(p, dt=0.0)
    assert op.sts_stages() == 2
    u0 = np.random.default_rng(26).standard_normal(p.shape)
    u1, info = op.sts_step(to_dev(u0))
    # A_cc = V_c exactly, z_c = 2 (A_cc - V_c)/V_c is zero up to the rounding of V_c
    assert 0.0 <= info["z_max"] <= 1e-15
    np.testing.assert_array_equal(to_host(u1), u0)
    _, op = gpu_operator(p)
    z, _ = op.sts_step(torch.zeros(p.shape, dtype=torch.float64, device=DEV))
    assert torch.count_nonzero(z).item() == 0


def test_deterministic():
    p = problem("c0", (0, 0))
    _, op = gpu_operator(p)
    u0 = to_dev(np.random.default_rng(27).standard_normal(p.shape))
    a, _ = op.sts_step(u0)
    b, _ = op.sts_step(u0)
    assert torch.equal(a, b)


@pytest.mark.parametrize("shape", PAIR_SHAPES + [(5, 7, 13)])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("stages", [0, 2, 3, 4, 5, 8, 13])
def test_stage_pairs_equal_single_stage_kernels(shape, bc, stages):
    p = problem(shape, bc)
    _, op = gpu_operator(p)
    u0 = to_dev(np.random.default_rng(29).standard_normal(p.shape))
    a, ia = op.sts_step(u0, stages=stages)
    b, ib = op.sts_step(u0, stages=stages, stage_pairs=False)
    s = ia["stages"]
    assert ib["stages_per_kernel"] == 1
    assert ia["stages_per_kernel"] == (2 if p.shape[2] % 2 == 0 and s >= 3 else 1)
    if not torch.equal(a, b):
        d = float((a - b).abs().max() / b.abs().max())
        pytest.fail(f"{shape} bc={bc} s={s}: pairs differ from single stages by {d:.3e} (max rel)")


def test_stage_pairs_in_place_and_repeated():
    p = problem((40, 26, 122), (1, 0))
    _, op = gpu_operator(p)
    u0 = to_dev(np.random.default_rng(30).standard_normal(p.shape))
    u, v = u0.clone(), u0.clone()
    for _ in range(3):
        u, _ = op.sts_step(u, out=u)
        v, _ = op.sts_step(v, out=v, stage_pairs=False)
    assert torch.equal(u, v)


@pytest.mark.parametrize("pairs", [True, False])
def test_timing_info_and_argument_errors(pairs):
    p = problem("c0", (0, 0))
    _, op = gpu_operator(p)
    u0 = to_dev(np.random.default_rng(28).standard_normal(p.shape))
    s = op.sts_stages()
    _, info = op.sts_step(u0, sample_timing=True, stage_pairs=pairs)
    if pairs:
        # general pairs: (4, 5), (6, 7), ... short of the last stage
        ngen = (s - 3) // 2 - (1 if (s - 3) % 2 == 0 else 0)
        assert info["stages_per_kernel"] == 2
    else:
        ngen = s - 4
        assert info["stages_per_kernel"] == 1
    # one event pair around the back-to-back run of all general kernels
    assert info["stage_kernel_samples"] == ngen
    assert 0.0 < info["stage_kernel_us"] * ngen < info["step_us"]
    with pytest.raises(abi.MasError, match="stages"):
        op.sts_step(u0, stages=1)
    lib = abi.load()
    out = torch.empty_like(u0)
    need = int(lib.mas_sts_workspace_bytes(op.handle))
    assert need >= 5 * 8 * p.cfg.n
    st = lib.mas_sts_step(op.handle, u0.data_ptr(), out.data_ptr(), None, out.data_ptr(), need - 8,
                          None, None)
    assert st == abi.MAS_ENOMEM
