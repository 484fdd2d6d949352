"""Pins for the oracle's assembled operator A = diag(V) + dt K(nu):
symmetry, row sums, positive definiteness, special cases, a dense
re-assembly, and a manufactured solution with an analytic div(nu grad u)."""
import math

import numpy as np
import pytest

from oracle import dense
from paper_1811_02605_amd import workloads as W


def _prob(ora, nr, nt, np_, q=1.02, th="uniform", bc=(0, 0), seed=0, R=100.0):
    cfg = W.small_config(nr, nt, np_, q=q, theta=th, seed_index=seed, diff_number=R)
    p = W.make_problem(cfg)
    return p, ora.Operator(p.r_faces, p.t_faces, np_, p.nu, p.dt, *bc)


SHAPES = [(4, 4, 8), (5, 7, 13), (3, 6, 2), (6, 3, 1), (1, 4, 6)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", [(0, 0), (1, 0), (1, 1)])
def test_apply_matches_independent_dense_assembly(ora, shape, bc):
    p, op = _prob(ora, *shape, bc=bc)
    A = dense.dense_matrix(op)
    x = np.random.default_rng(1).standard_normal(A.shape[0])
    y = op.apply(x).reshape(-1)
    np.testing.assert_allclose(y, A @ x, rtol=0, atol=1e-14 * np.abs(A).max() * np.abs(x).max() * 8)
    np.testing.assert_allclose(np.diag(A), op.diag.reshape(-1), rtol=1e-14)


@pytest.mark.parametrize("shape", SHAPES + [(32, 32, 64)])
def test_symmetry(ora, shape):
    p, op = _prob(ora, *shape)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(op.shape)
    y = rng.standard_normal(op.shape)
    a, b = op.dot(y, op.apply(x)), op.dot(x, op.apply(y))
    assert abs(a - b) <= 1e-13 * max(abs(a), abs(b))


@pytest.mark.parametrize("shape", SHAPES + [(32, 32, 64)])
@pytest.mark.parametrize("bc", [(0, 0), (0, 1), (1, 1)])
def test_row_sums_equal_volume_plus_wall_conductance(ora, shape, bc):
    # A 1 = V + (Dirichlet wall conductances): every interior flux term cancels
    p, op = _prob(ora, *shape, bc=bc)
    y = op.apply(np.ones(op.shape))
    want = op.V.copy()
    want[0] += op.cr[0]
    want[-1] += op.cr[-1]
    np.testing.assert_allclose(y, want, rtol=1e-12, atol=1e-13 * op.diag.max())
    if bc[0] == 1:
        assert np.all(op.cr[0] == 0)
    else:
        assert np.all(op.cr[0] > 0)


@pytest.mark.parametrize("shape", [(4, 4, 8), (5, 7, 13), (3, 6, 2)])
def test_positive_definite(ora, shape):
    p, op = _prob(ora, *shape, bc=(1, 1))
    A = dense.dense_matrix(op)
    np.linalg.cholesky(A)  # raises if not SPD
    off = np.abs(A).sum(axis=1) - np.abs(np.diag(A))
    assert np.all(np.diag(A) > off)  # strict diagonal dominance


def test_zero_time_step_is_identity_step(ora):
    p, _ = _prob(ora, 5, 7, 13)
    op = ora.Operator(p.r_faces, p.t_faces, 13, p.nu, 0.0)
    np.testing.assert_array_equal(op.diag, op.V)
    x, it, rr, rt = op.pcg(op.rhs_to_b(p.rhs), tol=1e-10)
    assert it == 1
    np.testing.assert_allclose(x, p.rhs, rtol=1e-14)


def test_phi_independent_data_gives_phi_independent_solution(ora):
    p, _ = _prob(ora, 6, 8, 12)
    nu = np.repeat(p.nu[:, :, :1], 12, axis=2)
    rhs = np.repeat(p.rhs[:, :, :1], 12, axis=2)
    op = ora.Operator(p.r_faces, p.t_faces, 12, nu, p.dt)
    x = op.solve_rhs(rhs)
    np.testing.assert_allclose(x, np.repeat(x[:, :, :1], 12, axis=2), rtol=1e-10, atol=1e-12)


def test_phi_shift_equivariance(ora):
    p, op = _prob(ora, 5, 6, 10)
    x = op.solve_rhs(p.rhs)
    op2 = ora.Operator(p.r_faces, p.t_faces, 10, np.roll(p.nu, 3, axis=2), p.dt)
    x2 = op2.solve_rhs(np.roll(p.rhs, 3, axis=2))
    np.testing.assert_allclose(x2, np.roll(x, 3, axis=2), rtol=1e-9, atol=1e-11)


def test_theta_reflection(ora):
    p, op = _prob(ora, 5, 8, 10)
    x = op.solve_rhs(p.rhs)
    op2 = ora.Operator(p.r_faces, p.t_faces, 10, p.nu[:, ::-1], p.dt)
    x2 = op2.solve_rhs(p.rhs[:, ::-1])
    np.testing.assert_allclose(x2, x[:, ::-1], rtol=1e-9, atol=1e-11)


# ---------------------------------------------------------------- manufactured solution
#   u = p(r) Y(theta, phi), Y = sin^2(t) cos(t) cos(2 phi)  (a degree-3 spherical harmonic)
#   solves u - dt div(nu grad u) = f with f from the closed form below.


def _mms_error(ora, nr, nt, np_, beta, variable_nu, neumann):
    rf = W.radial_faces_mapped(nr, beta)
    tf = W.theta_faces(nt)
    R, T, Ph = np.meshgrid(W.centres(rf), W.centres(tf), W.phi_centres(np_), indexing="ij")
    dt = 50.0
    if neumann:
        # p = (r-1)^2 (r-2.5)^2 has p' = 0 at both walls
        pr = np.polynomial.Polynomial.fromroots([1, 1, 2.5, 2.5])
    else:
        pr = np.polynomial.Polynomial.fromroots([1, 2.5]) * -1.0  # (r-1)(2.5-r)
    p, dp, d2p = pr(R), pr.deriv(1)(R), pr.deriv(2)(R)
    Y = np.sin(T) ** 2 * np.cos(T) * np.cos(2 * Ph)
    Yt = np.sin(T) * np.cos(2 * Ph) * (2 * np.cos(T) ** 2 - np.sin(T) ** 2)
    Yp = -2 * np.sin(T) ** 2 * np.cos(T) * np.sin(2 * Ph)
    a, da = 1e-3 * (1 + R ** 2), 2e-3 * R
    if variable_nu:
        bfac = 1 + 0.3 * np.sin(T) * np.cos(Ph)      # = 1 + 0.3 x/r, smooth at the poles
        b_t = 0.3 * np.cos(T) * np.cos(Ph)
        b_p = -0.3 * np.sin(T) * np.sin(Ph)
    else:
        bfac, b_t, b_p = np.ones_like(R), 0.0 * R, 0.0 * R
    nu = a * bfac
    lap = Y * (d2p + 2 * dp / R - 12 * p / R ** 2)
    grad_dot = (da * bfac * dp * Y + a * b_t * p * Yt / R ** 2
                + a * b_p * p * Yp / (R ** 2 * np.sin(T) ** 2))
    u = p * Y
    f = u - dt * (nu * lap + grad_dot)
    bc = 1 if neumann else 0
    op = ora.Operator(rf, tf, np_, nu, dt, bc, bc)
    x = op.solve_rhs(f, tol=1e-13)
    e = x - u
    return math.sqrt((op.V * e * e).sum() / (op.V * u * u).sum())


@pytest.mark.parametrize("beta,variable_nu,neumann", [(0.0, False, False), (1.5, False, False),
                                                      (1.5, True, False), (0.0, True, True)])
def test_manufactured_solution_second_order(ora, beta, variable_nu, neumann):
    errs = [_mms_error(ora, 12 * m, 12 * m, 24 * m, beta, variable_nu, neumann) for m in (1, 2, 4)]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 5e-3
    assert min(orders) >= 1.8, (errs, orders)
