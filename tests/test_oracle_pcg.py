"""Pins for the oracle's Jacobi-preconditioned CG: dense LU, library CG,
finite termination, energy-norm monotonicity and the Chebyshev iteration
bound."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import dense
from paper_1811_02605_amd import workloads as W


def _prob(ora, nr, nt, np_, bc=(0, 0), seed=0):
    cfg = W.small_config(nr, nt, np_, seed_index=seed)
    p = W.make_problem(cfg)
    return p, ora.Operator(p.r_faces, p.t_faces, np_, p.nu, p.dt, *bc)


@pytest.mark.parametrize("shape", [(4, 4, 8), (6, 6, 12), (8, 8, 16), (3, 5, 7), (2, 3, 1)])
@pytest.mark.parametrize("bc", [(0, 0), (1, 1)])
def test_pcg_matches_dense_lu(ora, shape, bc):
    p, op = _prob(ora, *shape, bc=bc)
    b = op.rhs_to_b(p.rhs)
    xd = dense.dense_solve(op, b)
    x, it, rr, rt = op.pcg(b, tol=1e-13)
    assert rr <= 1e-13 and rt <= 5e-13
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)


def test_finite_termination(ora):
    p, op = _prob(ora, 2, 2, 4)
    n = 16
    x, it, rr, rt = op.pcg(op.rhs_to_b(p.rhs), tol=1e-14, max_iters=10 * n)
    assert it <= n + 2 and rt < 1e-13


def test_energy_norm_error_decreases(ora):
    p, op = _prob(ora, 4, 4, 8)
    b = op.rhs_to_b(p.rhs)
    xs = dense.dense_solve(op, b)
    errs = []
    for k in range(0, 40):
        xk = op.pcg(b, tol=0.0, max_iters=k)[0]
        e = xk - xs
        errs.append(op.dot(e, op.apply(e)))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-10) for i in range(len(errs) - 1))
    assert errs[-1] < 1e-20 * errs[0]


@pytest.mark.parametrize("shape", [(4, 4, 8), (8, 8, 16)])
def test_iterations_within_cg_bound(ora, shape):
    p, op = _prob(ora, *shape)
    kappa = dense.jacobi_condition_number(op)
    tol = 1e-10
    b = op.rhs_to_b(p.rhs)
    x, it, rr, rt = op.pcg(b, tol=tol)
    # ||r|| <= sqrt(kappa_A) ||e||_A-based bound: A-norm error contracts by
    # 2((sqrt k - 1)/(sqrt k + 1))^m; converting to the residual costs a factor
    # sqrt(cond(A)) which we bound generously through kappa of the scaled matrix
    # and the diagonal spread.
    A = dense.dense_matrix(op)
    dmax, dmin = np.diag(A).max(), np.diag(A).min()
    factor = math.sqrt(kappa * dmax / dmin)
    bound = math.ceil(0.5 * math.sqrt(kappa) * math.log(2 * factor / tol)) + 1
    assert it <= bound, (it, bound, kappa)


def test_matches_library_cg_at_small_config(ora):
    p = W.make_problem("c0")
    op = ora.Operator(p.r_faces, p.t_faces, 64, p.nu, p.dt)
    b = op.rhs_to_b(p.rhs).reshape(-1)
    x, it, rr, rt = op.pcg(b, tol=1e-12)
    n = b.size
    Aop = spla.LinearOperator((n, n), matvec=lambda v: op.apply(v).reshape(-1), dtype=np.float64)
    dinv = 1.0 / op.diag.reshape(-1)
    M = spla.LinearOperator((n, n), matvec=lambda v: dinv * v, dtype=np.float64)
    xs, info = spla.cg(Aop, b, rtol=1e-12, atol=0.0, M=M, maxiter=5000)
    assert info == 0
    assert np.linalg.norm(x.reshape(-1) - xs) <= 1e-9 * np.linalg.norm(xs)
    assert rt <= 1e-12 * 1.5


def test_warm_start_from_solution_takes_no_iterations(ora):
    p, op = _prob(ora, 5, 6, 7)
    b = op.rhs_to_b(p.rhs)
    xs = dense.dense_solve(op, b)
    x, it, rr, rt = op.pcg(b, tol=1e-10, x0=xs)
    assert it == 0 and rt < 1e-12


def test_recursive_and_true_residual_agree(ora):
    p = W.make_problem("c0")
    op = ora.Operator(p.r_faces, p.t_faces, 64, p.nu, p.dt)
    x, it, rr, rt, hist = op.pcg(op.rhs_to_b(p.rhs), tol=1e-10, history=True)
    assert rr <= 1e-10 and abs(rt - rr) <= 1e-3 * rr
    assert hist[0] == pytest.approx(1.0) and hist.size == it + 1
