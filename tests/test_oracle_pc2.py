"""Pins for the oracle's block-Jacobi ILU(0) preconditioner (PC2, Section 2.2)
and its PCG, against what the definitions fix independently of the oracle's
sweeps:
  * textbook ILU(0) (the IKJ elimination restricted to the matrix's nonzero
    pattern) of a block-diagonal matrix assembled here in numpy: M^-1 r by a
    dense solve equals the oracle's forward/backward sweeps;
  * one block holding a 1-D chain: ILU(0) is the exact LU, PCG converges in
    one iteration;
  * single-cell blocks: PC2 is point Jacobi, PCG iterates equal PC1's;
  * M is symmetric positive definite; PCG with it reaches the dense solution.
"""
import numpy as np
import pytest

from oracle import dense
from paper_1811_02605_amd import workloads as W


def _op(ora, shape, bc=(0, 0), seed=0):
    p = W.make_problem(W.small_config(*shape, seed_index=seed))
    return p, ora.Operator(p.r_faces, p.t_faces, shape[2], p.nu, p.dt, *bc)


def _block_matrix(op, blocks):
    """Block-diagonal part of A: couplings between cells of one block, the
    periodic phi coupling between k = np-1 and k = 0 left out."""
    nr, nt, n_p = op.shape
    bi, bj, bk = blocks
    n = nr * nt * n_p
    idx = np.arange(n).reshape(op.shape)
    A = np.diag(op.diag.reshape(-1).copy())
    i, j, k = np.meshgrid(np.arange(nr), np.arange(nt), np.arange(n_p), indexing="ij")

    def couple(mask, a, b, c):
        a, b, c = a[mask], b[mask], c[mask]
        A[a, b] -= c
        A[b, a] -= c

    # r faces between planes i-1 and i: op.cr[i]
    m = (i > 0) & ((i - 1) // bi == i // bi)
    couple(m, idx, np.roll(idx, 1, axis=0), op.cr[:nr])
    m = (j > 0) & ((j - 1) // bj == j // bj)
    couple(m, idx, np.roll(idx, 1, axis=1), op.ct[:, :nt])
    # phi face k-1/2 (op.cp[k-1]); k = 0 would be the periodic one
    m = (k > 0) & ((k - 1) // bk == k // bk)
    couple(m, idx, np.roll(idx, 1, axis=2), np.roll(op.cp, 1, axis=2))
    return A


def _ilu0(A):
    """Textbook ILU(0): Gaussian elimination keeping only A's nonzero pattern."""
    a = A.copy()
    n = a.shape[0]
    nz = A != 0.0
    for i in range(1, n):
        for k in range(i):
            if not nz[i, k]:
                continue
            a[i, k] /= a[k, k]
            for j in range(k + 1, n):
                if nz[i, j]:
                    a[i, j] -= a[i, k] * a[k, j]
    L = np.tril(a, -1) + np.eye(n)
    U = np.triu(a)
    return L, U


@pytest.mark.parametrize("shape,blocks", [
    ((4, 4, 8), (2, 2, 4)), ((4, 4, 8), (8, 8, 32)), ((3, 5, 7), (2, 3, 3)),
    ((5, 3, 6), (1, 1, 6)), ((2, 2, 3), (2, 2, 3)), ((3, 4, 2), (2, 2, 2)), ((4, 3, 1), (3, 2, 1)),
])
@pytest.mark.parametrize("bc", [(0, 0), (1, 1)])
def test_apply_equals_textbook_ilu0(ora, shape, blocks, bc):
    p, op = _op(ora, shape, bc)
    L, U = _ilu0(_block_matrix(op, blocks))
    r = np.random.default_rng(7).standard_normal(op.shape).reshape(-1)
    want = np.linalg.solve(U, np.linalg.solve(L, r))
    got = op.pc2_apply(r, blocks).reshape(-1)
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
    # the modified diagonal is U's diagonal
    np.testing.assert_allclose(op.pc2_factor(blocks).reshape(-1), np.diag(U), rtol=1e-13)


@pytest.mark.parametrize("shape,blocks", [((4, 4, 8), (2, 2, 4)), ((3, 5, 7), (2, 3, 3)),
                                          ((5, 3, 6), (1, 1, 6))])
def test_energy_of_the_forward_sweep(ora, shape, blocks):
    """A symmetric matrix's ILU(0) is M = L D L^T (L unit lower, D = diag U),
    so (r, M^-1 r) = u^T D^-1 u with u = L^-1 r: the dot product of a PC2
    iteration follows from the forward sweep alone (the GPU solve kernel
    forms it so)."""
    p, op = _op(ora, shape, (0, 1))
    L, U = _ilu0(_block_matrix(op, blocks))
    d = np.diag(U)
    np.testing.assert_allclose(U, d[:, None] * L.T, rtol=1e-12, atol=1e-15)  # U = D L^T
    r = np.random.default_rng(11).standard_normal(op.shape).reshape(-1)
    u = np.linalg.solve(L, r)
    rz = float(r @ op.pc2_apply(r, blocks).reshape(-1))
    assert abs(rz - float(np.sum(u * u / d))) <= 1e-12 * abs(rz)


def test_preconditioner_is_spd(ora):
    p, op = _op(ora, (4, 5, 6), seed=2)
    blocks = (2, 3, 4)
    n = op.V.size
    Minv = np.stack([op.pc2_apply(e, blocks).reshape(-1) for e in np.eye(n)], axis=1)
    assert np.abs(Minv - Minv.T).max() <= 1e-12 * np.abs(Minv).max()
    np.linalg.cholesky(0.5 * (Minv + Minv.T))


def test_single_block_chain_is_exact(ora):
    """nt = np = 1 and one block: A is tridiagonal, ILU(0) = LU, M = A."""
    p, op = _op(ora, (12, 1, 1))
    b = op.rhs_to_b(p.rhs)
    z = op.pc2_apply(b, (12, 1, 1))
    np.testing.assert_allclose(z, dense.dense_solve(op, b), rtol=1e-12, atol=0)
    x, it, rr, rt = op.pcg_pc2(b, (12, 1, 1), tol=1e-12)
    assert it == 1 and rt <= 1e-13


@pytest.mark.parametrize("shape", [(4, 4, 8), (3, 5, 7)])
def test_single_cell_blocks_are_jacobi(ora, shape):
    p, op = _op(ora, shape)
    np.testing.assert_array_equal(op.pc2_factor((1, 1, 1)), op.diag)
    b = op.rhs_to_b(p.rhs)
    for k in (1, 5, 12):
        x1 = op.pcg(b, tol=0.0, max_iters=k)[0]
        x2 = op.pcg_pc2(b, (1, 1, 1), tol=0.0, max_iters=k)[0]
        np.testing.assert_allclose(x2, x1, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("shape,blocks", [((6, 6, 12), (2, 3, 4)), ((8, 8, 16), (8, 8, 32)),
                                          ((5, 7, 13), (4, 4, 8))])
@pytest.mark.parametrize("bc", [(0, 0), (1, 0)])
def test_pcg_pc2_reaches_dense_solution(ora, shape, blocks, bc):
    p, op = _op(ora, shape, bc)
    b = op.rhs_to_b(p.rhs)
    xd = dense.dense_solve(op, b)
    x, it, rr, rt = op.pcg_pc2(b, blocks, tol=1e-12)
    assert rt <= 5e-12
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    # a stronger preconditioner than point Jacobi: no more iterations
    it1 = op.pcg(b, tol=1e-12)[1]
    assert it <= it1
