"""The seeded input recipe: determinism and the grid/time-step figures it fixes."""
import hashlib
import math

import numpy as np
import pytest

from paper_1811_02605_amd import workloads as W


def _h(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_problem_is_deterministic():
    a = W.make_problem("c0")
    b = W.make_problem("c0")
    for x, y in [(a.nu, b.nu), (a.rhs, b.rhs), (a.r_faces, b.r_faces), (a.t_faces, b.t_faces)]:
        assert _h(x) == _h(y)
    assert a.dt == b.dt


@pytest.mark.parametrize("nr,q", [(32, 1.02), (256, 1.01), (300, 1.01), (7, 1.0)])
def test_radial_faces(nr, q):
    f = W.radial_faces(nr, q)
    assert f[0] == 1.0 and f[-1] == 2.5 and f.size == nr + 1
    dr = np.diff(f)
    assert np.all(dr > 0)
    if q != 1.0:
        np.testing.assert_allclose(dr[1:-1] / dr[:-2], q, rtol=1e-9)


def test_c0_radial_widths():
    dr = np.diff(W.radial_faces(32, 1.02))
    assert dr[0] == pytest.approx(3.39e-2, rel=2e-3)
    assert dr[-1] == pytest.approx(6.27e-2, rel=2e-3)


def test_clustered_theta():
    f = W.theta_faces(400, "clustered")
    assert f[0] == 0.0 and f[-1] == math.pi
    w = np.diff(f)
    assert np.all(w > 0)
    assert w.min() == pytest.approx(3.189e-3, rel=1e-3)
    assert w.max() == pytest.approx(1.053e-2, rel=1e-3)


@pytest.mark.parametrize("name,dx", [("c0", 4.899e-3), ("c1", 4.822e-5), ("c3", 1.3425e-4),
                                     ("c4", 1.253e-5)])
def test_min_cell_width(name, dx):
    c = W.CONFIGS[name]
    got = W.min_cell_width(W.radial_faces(c.nr, c.q), W.theta_faces(c.nt, c.theta), c.np_)
    assert got == pytest.approx(dx, rel=1e-3)


def test_c0_time_step():
    p = W.make_problem("c0")
    assert p.dt * p.nu.max() == pytest.approx(2.400e-3, rel=1e-3)


def test_smooth_field_matches_direct_cosine_sum():
    rf = W.radial_faces(5, 1.02)
    tf = W.theta_faces(6)
    np_ = 7
    g = W.smooth_field(np.random.default_rng(5), rf, tf, np_, 4)
    ks, ls, ns, a, psi = W.fourier_modes(np.random.default_rng(5), 4)
    r, t, p = np.meshgrid(W.centres(rf), W.centres(tf), W.phi_centres(np_), indexing="ij")
    d = sum(a[m] * np.cos(math.pi * ks[m] * (r - 1) / 1.5 + ls[m] * t + ns[m] * p + psi[m])
            for m in range(4))
    d = (d - d.mean()) / d.std()
    np.testing.assert_allclose(g, d, atol=1e-12)
    assert abs(g.mean()) < 1e-14 and abs(np.mean(g * g) - 1) < 1e-12


def test_contrast_recipe():
    cfg = W.Config("t", 8, 10, 12, 1.01, "uniform", 16, None, 100.0, 1000.0, True, "fp64")
    p = W.make_problem(cfg)
    assert p.nu.max() / p.nu.min() == pytest.approx(100.0, rel=1e-10)
    assert p.dt * p.nu.max() == pytest.approx(1000.0 * W.min_cell_width(
        p.r_faces, p.t_faces, cfg.np_) ** 2, rel=1e-12)


def test_jacobi_smoothing_is_a_weighted_average():
    u = np.zeros((3, 4, 5))
    u[1, 2, 3] = 1.0
    s = W.jacobi_smooth(u)
    assert s[1, 2, 3] == pytest.approx(1 / 3)
    # six neighbours, each with six neighbours of its own except r/theta edges
    assert s[1, 2, 4] == pytest.approx(2 / 3 / 6)
    assert s[0, 2, 3] == pytest.approx(2 / 3 / 5)  # r = 0 plane: 5 neighbours
    assert s.sum() > 0


def test_target_viscosity_and_directions():
    nu = np.full((2, 3, 4), 2e-3)
    t = W.target_viscosity(nu)
    assert np.all(np.abs(t / nu - 1) <= 0.2 + 1e-15)
    a = W.fd_direction((2, 3, 4), 0)
    b = W.fd_direction((2, 3, 4), 0)
    assert _h(a[0]) == _h(b[0]) and _h(a[1]) == _h(b[1])
