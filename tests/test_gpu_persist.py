"""The persistent launch (one cooperative kernel for a whole PC1 run, a grid
barrier per iteration) against the launch per iteration at the same r
chunks: the same x bit for bit and the same iteration counts and residuals,
on small grids in both precisions, with warm starts and fixed iteration
counts of both parities; the automatic choice (its own chunks, checked
against the oracle); and the requests it must refuse."""
import numpy as np
import pytest
import torch

from gpu_util import gpu_operator, oracle_operator, problem, to_dev, to_host
from paper_1811_02605_amd import _abi as abi
from paper_1811_02605_amd import solver as S

pytestmark = pytest.mark.gpu

SHAPES = [(5, 7, 13), (33, 17, 129), (1, 3, 2), (9, 16, 32), (6, 3, 1), "c0"]


CHUNKS = [1, 2]


def _pair(op, rhs, **kw):
    out = {}
    for mode in ("per_iteration", "persistent"):
        x, info = op.solve(rhs, S.make_opts(launch=mode, **kw))
        out[mode] = (x, info)
    return out


def _same(out):
    (xa, ia), (xb, ib) = out["per_iteration"], out["persistent"]
    assert ia["launch"] == abi.MAS_LAUNCH_PER_ITERATION and ib["launch"] == abi.MAS_LAUNCH_PERSISTENT
    assert torch.equal(xa, xb)
    for k in ("status", "iters", "outer_iters", "restarts", "rel_resid_true", "rel_resid_recursive"):
        assert ia[k] == ib[k], (k, ia[k], ib[k])


@pytest.mark.parametrize("chunk", CHUNKS)
@pytest.mark.parametrize("bc", [(0, 0), (1, 0)])
@pytest.mark.parametrize("shape", SHAPES)
def test_persistent_equals_per_iteration_fp64(shape, bc, chunk):
    p = problem(shape, bc)
    _, op = gpu_operator(p)
    out = _pair(op, to_dev(p.rhs), rtol=1e-10, chunk_planes=chunk)
    _same(out)
    x, info = out["persistent"]
    ora = oracle_operator(p)
    assert info["status"] == abi.MAS_OK
    assert ora.rel_residual(ora.rhs_to_b(p.rhs), to_host(x)) <= 1e-10


@pytest.mark.parametrize("chunk", CHUNKS)
@pytest.mark.parametrize("refine", ["reliable", "restart"])
@pytest.mark.parametrize("shape", SHAPES)
def test_persistent_equals_per_iteration_refined(shape, refine, chunk):
    p = problem(shape)
    _, op = gpu_operator(p, "fp32_refined")
    _same(_pair(op, to_dev(p.rhs), rtol=1e-10, precision="fp32_refined", refine=refine,
                chunk_planes=chunk))


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
@pytest.mark.parametrize("m", [2, 3, 4])
@pytest.mark.parametrize("shape", [(5, 7, 13), (9, 16, 32), "c0"])
def test_persistent_several_rhs(shape, m, precision):
    """Several right-hand sides, one of them zero (it stops at once while the
    others run on): the same x and counts in both launch modes."""
    p = problem(shape)
    _, op = gpu_operator(p, precision)
    rng = np.random.default_rng(40 + m)
    B = to_dev(np.stack([rng.standard_normal(p.shape) for _ in range(m)]))
    B[1].zero_()  # a zero right-hand side stops at once
    outs = {}
    for mode in ("per_iteration", "persistent"):
        X, infos = op.solve_multi(B, S.make_opts(rtol=1e-10, precision=precision, launch=mode,
                                                 chunk_planes=2))
        outs[mode] = (X, infos)
    (Xa, ia), (Xb, ib) = outs["per_iteration"], outs["persistent"]
    assert torch.equal(Xa, Xb)
    for h in range(m):
        assert ia[h]["launch"] == abi.MAS_LAUNCH_PER_ITERATION
        assert ib[h]["launch"] == abi.MAS_LAUNCH_PERSISTENT
        for k in ("status", "iters", "outer_iters", "rel_resid_true"):
            assert ia[h][k] == ib[h][k], (h, k, ia[h][k], ib[h][k])
    ora = oracle_operator(p)
    Xh = to_host(Xb)
    for h in range(m):
        if h != 1:
            assert ora.rel_residual(ora.rhs_to_b(to_host(B[h])), Xh[h]) <= 1e-10


@pytest.mark.parametrize("k", [0, 1, 2, 3, 6, 7])
@pytest.mark.parametrize("shape", [(5, 7, 13), "c0"])
def test_persistent_fixed_iteration_counts(shape, k):
    # a run stopped after k iterations: the catch-up of x after an odd
    # launch, and the iterate itself, as the oracle's PCG gives it
    p = problem(shape)
    _, op = gpu_operator(p)
    out = _pair(op, to_dev(p.rhs), rtol=0.0, max_iters=k, check_every=1, chunk_planes=2)
    _same(out)
    x, info = out["persistent"]
    assert info["iters"] == k
    ora = oracle_operator(p)
    xo = ora.pcg(ora.rhs_to_b(p.rhs), tol=0.0, max_iters=k)[0]
    d = float(np.linalg.norm(to_host(x) - xo) / max(np.linalg.norm(xo), 1e-300))
    assert d <= 1e-11 * max(1, k)


def test_persistent_warm_start_and_adjoint():
    p = problem("c0")
    _, op = gpu_operator(p)
    rhs = to_dev(p.rhs)
    x0 = 0.9 * op.solve(rhs, S.make_opts(rtol=1e-6))[0]
    outs = {}
    for mode in ("per_iteration", "persistent"):
        o = S.make_opts(rtol=1e-10, launch=mode, chunk_planes=2)
        x, info = op.solve(rhs, o, x0=x0.clone())
        gx = (0.1 * x).contiguous()
        lam, gnu, grhs, ainfo = op.adjoint(x, gx, o)
        outs[mode] = (x, info["iters"], lam, gnu, ainfo["iters"], ainfo["launch"])
    a, b = outs["per_iteration"], outs["persistent"]
    assert torch.equal(a[0], b[0]) and a[1] == b[1]
    assert torch.equal(a[2], b[2]) and torch.equal(a[3], b[3]) and a[4] == b[4]
    assert b[5] == abi.MAS_LAUNCH_PERSISTENT


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
@pytest.mark.parametrize("shape", SHAPES)
def test_automatic_persistent_solve_matches_oracle(shape, precision):
    p = problem(shape)
    _, op = gpu_operator(p, precision)
    x, info = op.solve(to_dev(p.rhs), S.make_opts(rtol=1e-10, precision=precision),
                       allow_notconv=False)
    assert info["launch"] == abi.MAS_LAUNCH_PERSISTENT
    ora = oracle_operator(p)
    assert ora.rel_residual(ora.rhs_to_b(p.rhs), to_host(x)) <= 1e-10


def test_automatic_choice():
    p = problem("c0")
    _, op = gpu_operator(p)
    _, info = op.solve(to_dev(p.rhs), S.make_opts(rtol=1e-10))
    assert info["launch"] == abi.MAS_LAUNCH_PERSISTENT
    # timing samples need the launches per iteration
    _, info = op.solve(to_dev(p.rhs), S.make_opts(rtol=1e-10, sample_timing=1))
    assert info["launch"] == abi.MAS_LAUNCH_PER_ITERATION and info["iter_kernel_samples"] > 0
    # above 2^17 cells the launch per iteration
    q = problem((32, 64, 128))
    _, op2 = gpu_operator(q)
    _, info = op2.solve(to_dev(q.rhs), S.make_opts(rtol=1e-10))
    assert info["launch"] == abi.MAS_LAUNCH_PER_ITERATION


def test_persistent_requests_refused():
    p = problem("c0")
    _, op = gpu_operator(p)
    rhs = to_dev(p.rhs)
    with pytest.raises(abi.MasError, match="persistent launch needs PC1"):
        op.solve(rhs, S.make_opts(launch="persistent", precond="pc2"))
    with pytest.raises(abi.MasError, match="persistent launch needs PC1"):
        op.solve(rhs, S.make_opts(launch="persistent", sample_timing=1))
    with pytest.raises(abi.MasError, match="unknown launch mode"):
        op.solve(rhs, S.make_opts(launch=7))
    # one-plane chunks of a grid whose iteration kernel then has more blocks
    # than the GPU holds at once
    q = problem((64, 256, 512))
    _, op2 = gpu_operator(q)
    with pytest.raises(abi.MasError, match="do not fit"):
        op2.solve(to_dev(q.rhs), S.make_opts(launch="persistent", chunk_planes=1))
