"""Pins of the environment-map background oracle (Sec. 3.2 "Faster
Background Model Evaluation": a spherical environment map sampled with
bilinear interpolation along each pixel's view direction)."""
import math

import numpy as np
import pytest

from oracle import envmap
from scenes import make_camera, ring_camera


def test_constant_map_samples_to_the_constant():
    cam = ring_camera(3, 8, 40, 30)
    env = np.tile(np.array([0.5, -2.0, 3.0]), (16, 32, 1))
    bg = envmap.sample(cam, env)
    np.testing.assert_allclose(bg, env[0, 0][:, None, None] * np.ones((3, 30, 40)), atol=1e-15)


def test_forward_axis_hits_the_centre_column_on_the_equator():
    """+z (the identity camera's optical axis) has phi = 0 and theta = pi/2:
    s = Wm/2, t = Hm/2, i.e. the corner shared by the four central texels."""
    cam = make_camera(2, 2, 1.0)  # pixel centres at +-0.5 around the axis
    Hm, Wm = 8, 16
    idx, wt = envmap.taps(cam, Hm, Wm, dirs=np.array([[[0.0, 0.0, 1.0]]]))
    assert sorted(idx[:, 0, 0].tolist()) == sorted([3 * Wm + 7, 3 * Wm + 8, 4 * Wm + 7,
                                                     4 * Wm + 8])
    np.testing.assert_allclose(wt[:, 0, 0], 0.25, atol=1e-12)


def test_linear_map_samples_to_the_column_coordinate():
    """A map whose texel value is its column index interpolates linearly:
    away from the wrap seam the sample equals s - 1/2 exactly."""
    cam = make_camera(24, 18, 20.0)
    Hm, Wm = 32, 64
    env = np.broadcast_to(np.arange(Wm, dtype=np.float64)[None, :, None], (Hm, Wm, 1)).copy()
    d = envmap.view_dirs(cam)
    phi = np.arctan2(d[..., 0], d[..., 2])
    s = (phi / (2 * math.pi) + 0.5) * Wm
    bg = envmap.sample(cam, env)[0]
    np.testing.assert_allclose(bg, s - 0.5, atol=1e-12)


def test_vectorised_equals_the_per_pixel_loop():
    cam = ring_camera(5, 8, 13, 9)
    env = np.random.default_rng(0).standard_normal((6, 12, 2))
    np.testing.assert_allclose(envmap.sample(cam, env), envmap.sample_loop(cam, env),
                               rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("view", [0, 3])
def test_backward_is_the_adjoint_of_the_forward(view):
    cam = ring_camera(view, 8, 31, 17)
    rng = np.random.default_rng(view)
    Hm, Wm, C = 10, 20, 3
    e = rng.standard_normal((Hm, Wm, C))
    G = rng.standard_normal((C, 17, 31))
    lhs = float((G * envmap.sample(cam, e)).sum())
    rhs = float((envmap.sample_backward(cam, G, Hm, Wm) * e).sum())
    assert lhs == pytest.approx(rhs, rel=1e-12)
