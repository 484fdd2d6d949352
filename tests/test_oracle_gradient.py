"""Pins for the oracle's adjoint gradient of L = 1/2 ||x(nu, rhs) - x_t||^2:
brute-force central differences of dense solves per component, the exact
derivative from re-assembly (A is affine in nu), and the Euler identity."""
import numpy as np
import pytest

from oracle import dense
from paper_1811_02605_amd import workloads as W


def _setup(ora, shape, bc=(0, 0), seed=0):
    nr, nt, np_ = shape
    cfg = W.small_config(nr, nt, np_, seed_index=seed)
    p = W.make_problem(cfg)
    op = ora.Operator(p.r_faces, p.t_faces, np_, p.nu, p.dt, *bc)
    xt = dense.dense_solve(ora.Operator(p.r_faces, p.t_faces, np_, W.target_viscosity(p.nu),
                                        p.dt, *bc), op.rhs_to_b(p.rhs))
    return p, op, xt


def _loss(ora, p, nu, rhs, xt, bc):
    op = ora.Operator(p.r_faces, p.t_faces, p.cfg.np_, nu, p.dt, *bc)
    x = dense.dense_solve(op, op.rhs_to_b(rhs))
    return 0.5 * float(np.sum((x - xt) ** 2))


def _grad(op, rhs, xt):
    x = dense.dense_solve(op, op.rhs_to_b(rhs))
    lam = dense.dense_solve(op, x - xt)
    return x, lam, op.gradient(x, lam)


@pytest.mark.parametrize("bc", [(0, 0), (1, 0)])
def test_gradient_matches_componentwise_central_differences(ora, bc):
    p, op, xt = _setup(ora, (4, 4, 8), bc)
    x, lam, (gnu, grhs) = _grad(op, p.rhs, xt)
    rng = np.random.default_rng(7)
    comps = rng.choice(p.nu.size, size=24, replace=False)
    gscale = np.abs(gnu).max()
    for c in comps:
        h = 1e-4 * p.nu.reshape(-1)[c]
        e = np.zeros(p.nu.size)
        e[c] = h
        e = e.reshape(p.nu.shape)
        fd = (_loss(ora, p, p.nu + e, p.rhs, xt, bc) - _loss(ora, p, p.nu - e, p.rhs, xt, bc)) / (2 * h)
        assert abs(fd - gnu.reshape(-1)[c]) <= 1e-6 * gscale + 1e-6 * abs(fd), c
    for c in comps[:8]:
        e = np.zeros(p.rhs.size)
        e[c] = 1e-4
        e = e.reshape(p.rhs.shape)
        fd = (_loss(ora, p, p.nu, p.rhs + e, xt, bc) - _loss(ora, p, p.nu, p.rhs - e, xt, bc)) / 2e-4
        assert abs(fd - grhs.reshape(-1)[c]) <= 1e-7 * np.abs(grhs).max()


@pytest.mark.parametrize("shape,bc", [((4, 4, 8), (0, 0)), ((3, 5, 7), (0, 1)), ((2, 3, 2), (1, 1))])
def test_gradient_equals_exact_reassembly_derivative(ora, shape, bc):
    # A(nu) is affine in nu, so dA/dnu_c = A(nu + e_c) - A(nu) up to rounding
    p, op, xt = _setup(ora, shape, bc)
    x, lam, (gnu, _) = _grad(op, p.rhs, xt)
    A0 = dense.dense_matrix(op)
    xf, lf = x.reshape(-1), lam.reshape(-1)
    for c in range(p.nu.size):
        nu1 = p.nu.copy().reshape(-1)
        nu1[c] += 1.0
        op1 = ora.Operator(p.r_faces, p.t_faces, shape[2], nu1, p.dt, *bc)
        dA = dense.dense_matrix(op1) - A0
        want = -lf @ dA @ xf
        assert abs(gnu.reshape(-1)[c] - want) <= 1e-9 * np.abs(gnu).max(), c


@pytest.mark.parametrize("cfg", ["c0", (5, 7, 13), (6, 3, 1)])
def test_euler_identity(ora, cfg):
    # A - diag(V) is linear in nu  =>  <g_nu, nu> = -lam^T (A - diag V) x = sum V lam x - lam^T b
    if isinstance(cfg, str):
        p = W.make_problem(cfg)
    else:
        p = W.make_problem(W.small_config(*cfg))
    op = ora.Operator(p.r_faces, p.t_faces, p.cfg.np_, p.nu, p.dt)
    b = op.rhs_to_b(p.rhs)
    x = op.pcg(b, tol=1e-13)[0]
    gx = np.random.default_rng(3).standard_normal(p.shape)
    lam = op.pcg(gx, tol=1e-13)[0]
    gnu, grhs = op.gradient(x, lam)
    lhs = float(np.sum(gnu * p.nu))
    rhs = float(np.sum(op.V * lam * x) - np.sum(lam * b))
    assert abs(lhs - rhs) <= 1e-10 * (abs(rhs) + np.sum(np.abs(op.V * lam * x)))
    np.testing.assert_allclose(grhs, op.V * lam, rtol=1e-15)
