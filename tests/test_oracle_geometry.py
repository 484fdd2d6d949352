"""Pins for the oracle's geometry: closed-form volumes, areas and lengths of
the spherical shell r in [1, 2.5] (independent of how cells are cut)."""
import math

import numpy as np
import pytest

from paper_1811_02605_amd import workloads as W

GRIDS = [
    (4, 4, 8, 1.02, "uniform"),
    (5, 7, 13, 1.0, "uniform"),
    (6, 9, 10, 1.05, "clustered"),
    (32, 32, 64, 1.02, "uniform"),
    (3, 1, 1, 1.1, "uniform"),
]


def _op(ora, nr, nt, np_, q, th, bc=(0, 0)):
    rf = W.radial_faces(nr, q)
    tf = W.theta_faces(nt, th)
    nu = np.full((nr, nt, np_), 1e-3)
    return ora.Operator(rf, tf, np_, nu, 0.5, *bc)


@pytest.mark.parametrize("g", GRIDS)
def test_total_volume_is_shell_volume(ora, g):
    op = _op(ora, *g)
    assert op.V.sum() == pytest.approx(4 * math.pi / 3 * (2.5 ** 3 - 1), rel=1e-13)
    assert np.all(op.V > 0)


@pytest.mark.parametrize("g", GRIDS)
def test_r_face_areas_sum_to_sphere(ora, g):
    op = _op(ora, *g)
    s = op.Ar.sum(axis=(1, 2))
    np.testing.assert_allclose(s, 4 * math.pi * op.r_faces ** 2, rtol=1e-13)


@pytest.mark.parametrize("g", GRIDS)
def test_theta_face_areas_are_cones_and_poles_vanish(ora, g):
    op = _op(ora, *g)
    s = op.At.sum(axis=(0, 2))
    want = np.sin(op.t_faces) * (2.5 ** 2 - 1) / 2 * 2 * math.pi
    want[0] = want[-1] = 0.0
    np.testing.assert_allclose(s, want, rtol=1e-13, atol=1e-15)
    assert np.all(op.At[:, 0] == 0.0) and np.all(op.At[:, -1] == 0.0)
    assert np.all(op.ct[:, 0] == 0.0) and np.all(op.ct[:, -1] == 0.0)


@pytest.mark.parametrize("g", GRIDS)
def test_phi_face_areas_are_half_annuli(ora, g):
    op = _op(ora, *g)
    s = op.Ap.sum(axis=(0, 1))
    np.testing.assert_allclose(s, math.pi * (2.5 ** 2 - 1) / 2, rtol=1e-13)


@pytest.mark.parametrize("g", GRIDS)
def test_distances(ora, g):
    op = _op(ora, *g)
    nr, nt, np_ = op.shape
    # wall-to-wall radial path: half cell + centre spacings + half cell = 1.5
    assert op.Hr[:, 0, 0].sum() == pytest.approx(1.5, rel=1e-14)
    rc = W.centres(op.r_faces)
    tc = W.centres(op.t_faces)
    if nt > 1:
        # interior theta faces span theta_c[0] .. theta_c[-1] along each ring of radius r_i
        np.testing.assert_allclose(op.Ht[:, 1:nt, 0].sum(axis=1) / rc, tc[-1] - tc[0], rtol=1e-13)
    # np phi steps go once around the circle of radius r sin(theta)
    np.testing.assert_allclose(op.Hp.sum(axis=2),
                               2 * math.pi * rc[:, None] * np.sin(tc)[None, :], rtol=1e-13)
