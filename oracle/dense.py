"""Dense-matrix helpers for tiny grids -- TEST INFRASTRUCTURE ONLY.

The dense matrix is assembled here in numpy from the oracle's face
conductances, with its own (independent) neighbour indexing, so that the
C operator apply, the C PCG and the C gradient can be checked against a
library dense solve on grids of a few hundred cells.
"""
from __future__ import annotations

import numpy as np


def dense_matrix(op) -> np.ndarray:
    """A = diag(V) + sum over faces c_f (e_a - e_b)(e_a - e_b)^T, walls as
    diagonal-only terms (Dirichlet: the wall conductance; Neumann: 0)."""
    nr, nt, n_p = op.shape
    n = nr * nt * n_p
    idx = np.arange(n).reshape(op.shape)
    A = np.diag(op.V.reshape(-1).copy())

    def couple(a, b, c):
        a, b, c = a.reshape(-1), b.reshape(-1), c.reshape(-1)
        np.add.at(A, (a, a), c)
        np.add.at(A, (b, b), c)
        np.add.at(A, (a, b), -c)
        np.add.at(A, (b, a), -c)

    # interior r faces 1..nr-1 couple planes i-1 and i
    couple(idx[:-1], idx[1:], op.cr[1:nr])
    # walls
    np.add.at(A, (idx[0].reshape(-1), idx[0].reshape(-1)), op.cr[0].reshape(-1))
    np.add.at(A, (idx[-1].reshape(-1), idx[-1].reshape(-1)), op.cr[nr].reshape(-1))
    # interior theta faces 1..nt-1
    couple(idx[:, :-1], idx[:, 1:], op.ct[:, 1:nt])
    # phi faces k+1/2 couple k and k+1 mod np (for np == 1 the face couples a cell to itself)
    couple(idx, np.roll(idx, -1, axis=2), op.cp)
    return A


def dense_solve(op, b) -> np.ndarray:
    A = dense_matrix(op)
    return np.linalg.solve(A, np.asarray(b, dtype=np.float64).reshape(-1)).reshape(op.shape)


def jacobi_condition_number(op) -> float:
    """kappa(D^-1/2 A D^-1/2) from a dense symmetric eigen-solve."""
    A = dense_matrix(op)
    d = np.sqrt(np.diag(A))
    ev = np.linalg.eigvalsh(A / d[:, None] / d[None, :])
    return float(ev[-1] / ev[0])
