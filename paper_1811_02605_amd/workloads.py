"""Seeded synthetic workloads for the implicit viscous solve.

This module only *makes inputs*: grid faces, the viscosity field nu, the
right-hand side, the time step and the perturbations used by the gradient
checks.  It holds none of the solver's arithmetic (no operator, no
conductance, no iteration), so that the HIP path and the FP64 CPU oracle
can both consume exactly the same arrays while sharing no code.

The paper's own workload (a ~11M-cell flux-rope eruption on a strongly
non-uniform spherical grid, Section 3) is not available; the configurations
below are synthetic stand-ins with the same structure: a spherical shell
r in [1, 2.5], logically rectangular (r, theta, phi) cells, periodic phi, a
large spatially varying viscosity coefficient and an implicit time step far
beyond the explicit diffusion limit.

Array layout: every cell array is float64, C order, shape (nr, nt, np), so
phi is the fastest index, then theta, then r.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

R_INNER = 1.0
R_OUTER = 2.5

BC_DIRICHLET0 = 0
BC_NEUMANN0 = 1


@dataclasses.dataclass(frozen=True)
class Config:
    """One synthetic workload.  Sizes are cells; q is the radial cell ratio."""
    name: str
    nr: int
    nt: int
    np_: int
    q: float                  # geometric radial ratio dr_{i+1}/dr_i (1.0 = uniform)
    theta: str                # "uniform" or "clustered"
    modes: int                # Fourier modes in the smooth log-viscosity field
    alpha: float | None       # nu = 1e-3 exp(alpha g); None -> from contrast
    contrast: float | None    # max(nu)/min(nu) when alpha is None
    diff_number: float        # R = dt * max(nu) / min(dx)^2
    smooth_rhs: bool          # one 2/3-weighted Jacobi smoothing of the rhs
    precision: str            # "fp64" or "fp32_refined"
    rtol: float = 1e-10
    seed_index: int = 0       # nu seed = 100 + seed_index, rhs seed = 200 + seed_index

    @property
    def shape(self):
        return (self.nr, self.nt, self.np_)

    @property
    def n(self):
        return self.nr * self.nt * self.np_


CONFIGS = {
    # small case: 32 x 32 x 64, the oracle finishes it in well under a second
    "c0": Config("c0", 32, 32, 64, 1.02, "uniform", 8, 0.5, None, 100.0, False,
                 "fp64", seed_index=0),
    # production-like FP64 solve: 256 x 320 x 640 = 52.4M cells
    "c1": Config("c1", 256, 320, 640, 1.01, "uniform", 16, None, 100.0, 1000.0, True,
                 "fp64", seed_index=1),
    # same grid and data, FP32 inner solve inside FP64 iterative refinement
    "c2": Config("c2", 256, 320, 640, 1.01, "uniform", 16, None, 100.0, 1000.0, True,
                 "fp32_refined", seed_index=1),
    # differentiable solve: 128 x 192 x 384 = 9.4M cells
    "c3": Config("c3", 128, 192, 384, 1.01, "uniform", 8, 0.5, None, 100.0, False,
                 "fp64", seed_index=3),
    # stress case: 300 x 400 x 800 = 96M cells, polar theta clustering
    "c4": Config("c4", 300, 400, 800, 1.01, "clustered", 16, None, 1000.0, 5000.0, False,
                 "fp32_refined", seed_index=4),
}


def small_config(nr, nt, np_, q=1.02, theta="uniform", modes=8, alpha=0.5,
                 diff_number=100.0, seed_index=0, name=None):
    """A config with the c0 recipe at another (usually tiny or ragged) size."""
    return Config(name or f"g{nr}x{nt}x{np_}", nr, nt, np_, q, theta, modes, alpha,
                  None, diff_number, False, "fp64", seed_index=seed_index)


# ----------------------------------------------------------------------------- grid

def radial_faces(nr: int, q: float) -> np.ndarray:
    """nr+1 radial faces from 1 to 2.5 with dr_i = dr_0 q^i (uniform if q == 1).

    The last face is set to exactly 2.5."""
    if nr < 1:
        raise ValueError("nr must be >= 1")
    span = R_OUTER - R_INNER
    if q == 1.0:
        dr = np.full(nr, span / nr)
    else:
        dr0 = span * (q - 1.0) / (q ** nr - 1.0)
        dr = dr0 * q ** np.arange(nr, dtype=np.float64)
    f = np.empty(nr + 1)
    f[0] = R_INNER
    f[1:] = R_INNER + np.cumsum(dr)
    f[-1] = R_OUTER
    return f


def radial_faces_mapped(nr: int, beta: float) -> np.ndarray:
    """Faces r(s) = 1 + 1.5 (e^{beta s} - 1)/(e^beta - 1) at s = i/nr.

    A fixed smooth map, so refining nr keeps the stretching profile (used by
    the manufactured-solution convergence study)."""
    s = np.arange(nr + 1, dtype=np.float64) / nr
    if beta == 0.0:
        f = R_INNER + (R_OUTER - R_INNER) * s
    else:
        f = R_INNER + (R_OUTER - R_INNER) * np.expm1(beta * s) / math.expm1(beta)
    f[0], f[-1] = R_INNER, R_OUTER
    return f


def theta_faces(nt: int, kind: str = "uniform") -> np.ndarray:
    """nt+1 colatitude faces from 0 to pi.

    "clustered": cell width proportional to 0.3 + 0.7 sin(theta at the
    uniform cell centre), normalised so the widths sum to pi; this makes
    the polar cells about 3.3x narrower than the equatorial ones."""
    if nt < 1:
        raise ValueError("nt must be >= 1")
    if kind == "uniform":
        f = np.arange(nt + 1, dtype=np.float64) * (math.pi / nt)
    elif kind == "clustered":
        tc = (np.arange(nt, dtype=np.float64) + 0.5) * (math.pi / nt)
        w = 0.3 + 0.7 * np.sin(tc)
        w *= math.pi / w.sum()
        f = np.empty(nt + 1)
        f[0] = 0.0
        f[1:] = np.cumsum(w)
    else:
        raise ValueError(f"unknown theta spacing {kind!r}")
    f[0], f[-1] = 0.0, math.pi
    return f


def centres(faces: np.ndarray) -> np.ndarray:
    return 0.5 * (faces[1:] + faces[:-1])


def phi_centres(np_: int) -> np.ndarray:
    return (np.arange(np_, dtype=np.float64) + 0.5) * (2.0 * math.pi / np_)


def min_cell_width(r_faces, t_faces, np_) -> float:
    """Smallest cell edge over the grid: min(dr, r dtheta, r sin(theta) dphi)."""
    rc, tc = centres(r_faces), centres(t_faces)
    dr, dt = np.diff(r_faces), np.diff(t_faces)
    dphi = 2.0 * math.pi / np_
    return float(min(dr.min(), (rc[:, None] * dt[None, :]).min(),
                     (rc[:, None] * np.sin(tc)[None, :] * dphi).min()))


# ----------------------------------------------------------------------------- fields

def fourier_modes(rng: np.random.Generator, m: int):
    """Draw m modes (k, l, n, a, psi) in a fixed order per mode:
    k, l, n in {0..3} (redrawn while all zero), then a ~ N(0,1), then
    psi ~ U[0, 2 pi)."""
    ks, ls, ns, amps, psis = [], [], [], [], []
    for _ in range(m):
        while True:
            k, l, n = (int(v) for v in rng.integers(0, 4, size=3))
            if k or l or n:
                break
        ks.append(k), ls.append(l), ns.append(n)
        amps.append(float(rng.standard_normal()))
        psis.append(float(rng.uniform(0.0, 2.0 * math.pi)))
    return (np.array(ks), np.array(ls), np.array(ns), np.array(amps), np.array(psis))


def smooth_field(rng, r_faces, t_faces, np_, modes, chunk=16) -> np.ndarray:
    """g(r,theta,phi) = sum_m a_m cos(pi k_m (r-1)/1.5 + l_m theta + n_m phi + psi_m)
    at cell centres, standardised to population mean 0 and variance 1.

    Evaluated as the real part of a rank-m product of 1-D complex
    exponentials (one matrix product per block of r planes)."""
    ks, ls, ns, amps, psis = fourier_modes(rng, modes)
    rc, tc, pc = centres(r_faces), centres(t_faces), phi_centres(np_)
    nr, nt = rc.size, tc.size
    er = amps[:, None] * np.exp(1j * (math.pi * ks[:, None] * (rc[None, :] - R_INNER)
                                      / (R_OUTER - R_INNER) + psis[:, None]))
    et = np.exp(1j * ls[:, None] * tc[None, :])
    ep = np.exp(1j * ns[:, None] * pc[None, :])
    g = np.empty((nr, nt, np_))
    for i0 in range(0, nr, chunk):
        i1 = min(nr, i0 + chunk)
        a = (er[:, i0:i1, None] * et[:, None, :]).reshape(modes, -1)
        g[i0:i1] = (a.T @ ep).real.reshape(i1 - i0, nt, np_)
    mean = g.mean()
    g -= mean
    g /= math.sqrt(float(np.mean(g * g)))
    return g


def viscosity(cfg: Config, r_faces, t_faces) -> np.ndarray:
    rng = np.random.default_rng(100 + cfg.seed_index)
    g = smooth_field(rng, r_faces, t_faces, cfg.np_, cfg.modes)
    if cfg.alpha is not None:
        alpha = cfg.alpha
    else:
        alpha = math.log(cfg.contrast) / float(g.max() - g.min())
    g *= alpha
    np.exp(g, out=g)
    g *= 1e-3
    return g


def jacobi_smooth(u: np.ndarray, weight: float = 2.0 / 3.0) -> np.ndarray:
    """u + w (mean of index-space neighbours - u); phi periodic, missing
    r/theta neighbours left out of the mean."""
    nr, nt, _ = u.shape
    # phi neighbours k-1 and k+1 (periodic), summed in that order
    s = np.empty_like(u)
    s[:, :, 1:] = u[:, :, :-1]
    s[:, :, 0] = u[:, :, -1]
    s[:, :, :-1] += u[:, :, 1:]
    s[:, :, -1] += u[:, :, 0]
    s[1:] += u[:-1]
    s[:-1] += u[1:]
    s[:, 1:] += u[:, :-1]
    s[:, :-1] += u[:, 1:]
    ir, it = np.arange(nr), np.arange(nt)
    cr = 2.0 + (ir > 0).astype(np.float64) + (ir < nr - 1).astype(np.float64)
    ct = (it > 0).astype(np.float64) + (it < nt - 1).astype(np.float64)
    s /= (cr[:, None] + ct[None, :])[:, :, None]
    s -= u
    s *= weight
    s += u
    return s


def right_hand_side(cfg: Config) -> np.ndarray:
    rng = np.random.default_rng(200 + cfg.seed_index)
    rhs = rng.standard_normal(cfg.n).reshape(cfg.shape)
    if cfg.smooth_rhs:
        rhs = jacobi_smooth(rhs)
    return rhs


def component_rhs(cfg: Config, m: int) -> np.ndarray:
    """m right-hand sides (the components of a vector field), shape (m, nr, nt, np):
    component 0 is right_hand_side(cfg); component h >= 1 uses the same recipe
    with seed 500 + 10 seed_index + h."""
    out = np.empty((m,) + cfg.shape)
    out[0] = right_hand_side(cfg)
    for h in range(1, m):
        rng = np.random.default_rng(500 + 10 * cfg.seed_index + h)
        u = rng.standard_normal(cfg.n).reshape(cfg.shape)
        out[h] = jacobi_smooth(u) if cfg.smooth_rhs else u
    return out


def target_viscosity(nu: np.ndarray, seed: int = 303, rel: float = 0.05) -> np.ndarray:
    """nu * (1 + rel xi), xi ~ N(0,1) clipped to [-4, 4]."""
    rng = np.random.default_rng(seed)
    xi = np.clip(rng.standard_normal(nu.size), -4.0, 4.0).reshape(nu.shape)
    return nu * (1.0 + rel * xi)


def fd_direction(shape, k: int):
    """Joint finite-difference direction (d_nu, d_rhs), entries N(0,1)."""
    rng = np.random.default_rng(400 + k)
    n = int(np.prod(shape))
    d_nu = rng.standard_normal(n).reshape(shape)
    d_rhs = rng.standard_normal(n).reshape(shape)
    return d_nu, d_rhs


@dataclasses.dataclass
class Problem:
    cfg: Config
    r_faces: np.ndarray
    t_faces: np.ndarray
    nu: np.ndarray
    rhs: np.ndarray
    dt: float
    bc_inner: int = BC_DIRICHLET0
    bc_outer: int = BC_DIRICHLET0

    @property
    def shape(self):
        return self.cfg.shape


def make_problem(cfg: Config | str) -> Problem:
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    rf = radial_faces(cfg.nr, cfg.q)
    tf = theta_faces(cfg.nt, cfg.theta)
    nu = viscosity(cfg, rf, tf)
    rhs = right_hand_side(cfg)
    dx = min_cell_width(rf, tf, cfg.np_)
    dt = cfg.diff_number * dx * dx / float(nu.max())
    return Problem(cfg, rf, tf, nu, rhs, dt)
