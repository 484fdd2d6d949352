"""Shared helpers for the GPU parity tests (seeded inputs -> both sides)."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_1811_02605_amd import solver as S
from paper_1811_02605_amd import workloads as W

DEV = "cuda:0"


def problem(spec, bc=(0, 0), theta="uniform", q=1.02, seed=0, R=100.0):
    if isinstance(spec, str):
        p = W.make_problem(spec)
    else:
        p = W.make_problem(W.small_config(*spec, q=q, theta=theta, seed_index=seed, diff_number=R))
    p.bc_inner, p.bc_outer = bc
    return p


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def to_host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def gpu_operator(p, precision="fp64", dt=None):
    grid = S.Grid.from_problem(p)
    op = S.Operator(grid, to_dev(p.nu), p.dt if dt is None else dt, precision=precision)
    return grid, op


def oracle_operator(p, dt=None):
    return oracle.Operator(p.r_faces, p.t_faces, p.cfg.np_, p.nu, p.dt if dt is None else dt,
                           p.bc_inner, p.bc_outer)


def oracle_plus_face_arrays(ora):
    """Oracle conductances laid out like mas_op_export (coupling to the + neighbour)."""
    nr, nt, n_p = ora.shape
    cr = np.zeros(ora.shape)
    cr[:-1] = ora.cr[1:nr]
    ct = np.zeros(ora.shape)
    ct[:, :-1] = ora.ct[:, 1:nt]
    return cr, ct, ora.cp.copy(), ora.diag.copy()


def rel(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def residual_rounding_floor(ora, b, x) -> float:
    """How far two correct evaluations of ||b - A x||/||b|| may differ by
    rounding alone.  Each side forms every component of b - A x from about
    ten products and sums (and the GPU's x passes through the symmetric
    scaling once more), so the computed residual vectors differ by at most
    c eps (|b| + |A||x|) componentwise with c about 10; in norm the reported
    values differ by at most 16 eps (||b|| + || |A||x| ||)/||b||.  A has a
    positive diagonal D and non-positive off-diagonal entries, so
    |A||x| = 2 D|x| - A|x|."""
    ax = np.abs(np.asarray(x, dtype=np.float64).reshape(ora.shape))
    abs_ax = 2.0 * ora.diag * ax - ora.apply(ax)
    nb = np.linalg.norm(np.asarray(b).reshape(-1))
    return 16.0 * np.finfo(np.float64).eps * (nb + np.linalg.norm(abs_ax.reshape(-1))) / nb
