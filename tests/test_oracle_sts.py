"""Pins for the oracle's RKL2 super time-step (second-order Runge-Kutta-Legendre
stages for the explicit viscous update, Section 2.2 of the paper).

The oracle runs the three-term stage recursion; these tests check it against
what the mathematics fixes independently of that recursion:
  * the stability polynomial's closed form a_s + b_s P_s(1 + w1 z) with P_s the
    Legendre polynomial (numpy's), applied through a dense eigendecomposition
    of dt L = I - V^-1 A (dense A assembled in numpy);
  * s = 2 reduces to Heun's method, R(z) = 1 + z + z^2/2;
  * third-order local error against scipy's matrix exponential;
  * conservation of sum(V u) and of constants with no-flux (Neumann) walls;
  * V-norm contraction at the stage count from the Gershgorin bound, that the
    bound covers the true spectrum, and that one stage fewer would not.
"""
import numpy as np
import pytest
import scipy.linalg as sla
from numpy.polynomial import legendre

from oracle import dense
from paper_1811_02605_amd import workloads as W


def _prob(ora, shape, bc=(0, 0), seed=0, dt_scale=1.0):
    cfg = W.small_config(*shape, seed_index=seed)
    p = W.make_problem(cfg)
    return p, ora.Operator(p.r_faces, p.t_faces, shape[2], p.nu, p.dt * dt_scale, *bc)


def _dense_dtL(op):
    A = dense.dense_matrix(op)
    v = op.V.reshape(-1)
    return np.eye(v.size) - A / v[:, None]


def _closed_form_R(s, z):
    w1 = 4.0 / (s * s + s - 2.0)
    bs = (s * s + s - 2.0) / (2.0 * s * (s + 1.0))
    return (1.0 - bs) + bs * legendre.legval(1.0 + w1 * z, [0.0] * s + [1.0])


def _apply_poly_of_dtL(op, u0, R):
    """R(dt L) u0 through the V-symmetric eigendecomposition of dt L."""
    A = dense.dense_matrix(op)
    v = op.V.reshape(-1)
    sv = np.sqrt(v)
    S = np.eye(v.size) - A / np.outer(sv, sv)          # V^1/2 (dt L) V^-1/2, symmetric
    lam, Q = np.linalg.eigh(0.5 * (S + S.T))
    y = Q @ (R(lam) * (Q.T @ (sv * u0.reshape(-1))))
    return (y / sv).reshape(op.shape), lam


@pytest.mark.parametrize("shape,bc", [((4, 4, 8), (0, 0)), ((3, 5, 7), (1, 1)), ((5, 4, 1), (0, 1)),
                                      ((6, 6, 12), (1, 0))])
@pytest.mark.parametrize("stages", [None, 2, 5, 33])
def test_step_matches_legendre_closed_form(ora, shape, bc, stages):
    p, op = _prob(ora, shape, bc)
    s = op.rkl2_stages() if stages is None else max(stages, 2)
    u0 = np.random.default_rng(3).standard_normal(op.shape)
    got = op.rkl2_step(u0, stages=s)
    want, lam = _apply_poly_of_dtL(op, u0, lambda z: _closed_form_R(s, z))
    scale = max(np.abs(want).max(), np.abs(u0).max())
    # the recursion and the eigen route round differently; the polynomial is
    # evaluated on |z| up to z_max, so allow a few hundred ulps of u0
    assert np.abs(got - want).max() <= 1e-12 * scale * max(1.0, float(-lam.min()))


def test_two_stages_is_heun(ora):
    """s = 2: R(z) = 1 + z + z^2/2 (the explicit trapezoid / Heun polynomial)."""
    p, op = _prob(ora, (4, 4, 8), dt_scale=1e-3)
    M = _dense_dtL(op)
    u0 = np.random.default_rng(1).standard_normal(op.shape).reshape(-1)
    want = u0 + M @ u0 + 0.5 * (M @ (M @ u0))
    got = op.rkl2_step(u0, stages=2).reshape(-1)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(u0).max()
    mu, nu, mt, gt = ora.rkl2_coefficients(2)
    # hand-derived: w1 = 1, b = 1/3 throughout
    np.testing.assert_allclose([mt[1], mu[2], nu[2], mt[2], gt[2]], [1 / 3, 1.5, -0.5, 1.5, -1.0],
                               rtol=1e-15)


@pytest.mark.parametrize("s", [2, 4, 9])
def test_third_order_local_error_vs_expm(ora, s):
    """||step(u) - exp(dt L) u|| ~ C dt^3: halving dt divides it by ~8."""
    errs = []
    for scale in (1e-3, 5e-4, 2.5e-4):
        p, op = _prob(ora, (4, 4, 8), dt_scale=scale)
        M = _dense_dtL(op)
        u0 = np.random.default_rng(2).standard_normal(op.shape).reshape(-1)
        exact = sla.expm(M) @ u0
        errs.append(np.linalg.norm(op.rkl2_step(u0, stages=s).reshape(-1) - exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 7.0 < r1 < 9.0 and 7.5 < r2 < 8.5, errs


def test_global_second_order(ora):
    """m steps of dt/m to a fixed time: error against expm falls ~4x per halving."""
    p = W.make_problem(W.small_config(4, 4, 8, seed_index=0))
    T = p.dt * 2e-3          # z_max T ~ 0.6: every mode in the asymptotic range
    exact = None
    errs = []
    u0 = np.random.default_rng(4).standard_normal((4, 4, 8))
    for m in (2, 4, 8):
        op = ora.Operator(p.r_faces, p.t_faces, 8, p.nu, T / m)
        if exact is None:
            opT = ora.Operator(p.r_faces, p.t_faces, 8, p.nu, T)
            exact = (sla.expm(_dense_dtL(opT)) @ u0.reshape(-1)).reshape(op.shape)
        u = u0.copy()
        s = op.rkl2_stages()
        for _ in range(m):
            u = op.rkl2_step(u, stages=s)
        errs.append(np.linalg.norm(u - exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.6 and 3.5 < r2 < 4.6, errs


@pytest.mark.parametrize("shape", [(4, 4, 8), (6, 5, 12), (3, 3, 1)])
def test_neumann_conserves_volume_integral_and_constants(ora, shape):
    p, op = _prob(ora, shape, bc=(1, 1))
    u0 = np.random.default_rng(5).standard_normal(op.shape)
    u = u0
    for _ in range(5):
        u = op.rkl2_step(u)
    tot0, tot = float(np.sum(op.V * u0)), float(np.sum(op.V * u))
    assert abs(tot - tot0) <= 1e-13 * float(np.sum(op.V * np.abs(u0)))
    c = np.full(op.shape, 2.75)
    np.testing.assert_allclose(op.rkl2_step(c), c, rtol=1e-14, atol=0)


def test_dirichlet_decays_constants(ora):
    """With absorbing walls a constant loses mass at the walls, never gains."""
    p, op = _prob(ora, (4, 4, 8), bc=(0, 0))
    c = np.ones(op.shape)
    u = op.rkl2_step(c)
    assert np.all(u <= 1.0 + 1e-14) and np.sum(op.V * u) < np.sum(op.V)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_stage_count_is_minimal_and_stable(ora, seed):
    p, op = _prob(ora, (6, 6, 12), seed=seed)
    s = op.rkl2_stages()
    zmax = float(np.max(2.0 * (op.diag - op.V) / op.V))
    assert (s * s + s - 2) / 2 >= zmax and (s == 2 or ((s - 1) ** 2 + (s - 1) - 2) / 2 < zmax)
    # the Gershgorin bound covers the true spectrum of dt L
    lam = np.linalg.eigvals(_dense_dtL(op)).real
    assert -lam.min() <= zmax * (1 + 1e-12) and lam.max() <= 1e-12
    # the V-norm never grows over repeated steps
    u = np.random.default_rng(seed).standard_normal(op.shape)
    nrm = [np.sqrt(np.sum(op.V * u * u))]
    for _ in range(10):
        u = op.rkl2_step(u, stages=s)
        nrm.append(np.sqrt(np.sum(op.V * u * u)))
    assert all(nrm[i + 1] <= nrm[i] * (1 + 1e-13) for i in range(10))


def test_too_few_stages_grows_stiff_mode(ora):
    """Below the bound the largest-|z| mode is amplified (the bound is needed)."""
    p, op = _prob(ora, (6, 6, 12))
    s = op.rkl2_stages()
    u0, lam = None, None
    M = _dense_dtL(op)
    w, vecs = np.linalg.eig(M)
    k = int(np.argmin(w.real))
    if -w[k].real <= 10.0:
        pytest.skip("spectrum too small to need many stages")
    u0 = vecs[:, k].real.reshape(op.shape)
    few = max(2, s // 3)
    g_few = np.linalg.norm(op.rkl2_step(u0, stages=few)) / np.linalg.norm(u0)
    g_ok = np.linalg.norm(op.rkl2_step(u0, stages=s)) / np.linalg.norm(u0)
    assert g_few > 1.0 and g_ok <= 1.0 + 1e-12


def test_zero_dt_is_identity(ora):
    p = W.make_problem(W.small_config(4, 4, 8, seed_index=0))
    op = ora.Operator(p.r_faces, p.t_faces, 8, p.nu, 0.0)
    assert op.rkl2_stages() == 2
    u0 = np.random.default_rng(6).standard_normal(op.shape)
    # dt L u = u - (V u)/V vanishes up to the rounding of one product and quotient
    np.testing.assert_allclose(op.rkl2_step(u0), u0, rtol=1e-14, atol=0)
