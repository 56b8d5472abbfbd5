"""Host logic of the world-space Gaussian settings and of the point ring
(no GPU): the workspace bound on projected standard deviations, the paper's
default sigma (Sec. 3.2 "Rendering Points as Small Gaussians": 5 px at the
near plane through the image centre), and PointRing's slot bookkeeping
(Sec. 3.1 "Fast and Stable View-Specific Sampling during Inference")."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2508_19140_amd import PointRing, RasterSettings, camera_struct, ewa_max_radius
from scenes import make_camera, ring_camera


@pytest.mark.parametrize("cam", [make_camera(96, 64, 40.0), ring_camera(3, 8, 200, 120),
                                 make_camera(64, 64, 20.0, z_near=0.05)])
def test_ewa_bound_covers_every_point_whose_footprint_meets_the_image(cam):
    """Random points from the near plane outwards, far beyond the image
    edges: every point the oracle keeps (its 3-sigma box meets the image)
    has sqrt(a - dil) and sqrt(c - dil) below the bound."""
    st = RasterSettings(splat="ewa")
    c = camera_struct(cam)
    sigma = st.sigma(c)
    bound = ewa_max_radius(c, sigma, st.dilation, st.cutoff)
    rng = np.random.default_rng(5)
    n = 200_000
    z = cam.z_near * np.exp(rng.uniform(0.0, 3.0, n))
    xn = rng.uniform(-3.0, 3.0, n) * (cam.width / cam.fx)
    yn = rng.uniform(-3.0, 3.0, n) * (cam.height / cam.fy)
    Xc = np.stack([xn * z, yn * z, z], 1)
    R = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    pos = ((Xc - t) @ R).astype(np.float32)  # world points with these camera coordinates
    pr = oracle.project(cam, pos, splat=oracle.SPLAT_EWA, ewa_sigma=float(np.float32(sigma)))
    vis = pr["visible"].astype(bool)
    assert vis.sum() > 1000 and (~vis).sum() > 1000
    u, v = pr["uv"][vis, 0].astype(np.float64), pr["uv"][vis, 1].astype(np.float64)
    Z = pr["xyz"][vis, 2].astype(np.float64)
    xh, yh = (u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy
    sa = sigma * cam.fx / Z * np.sqrt(1 + xh * xh)
    sc = sigma * cam.fy / Z * np.sqrt(1 + yh * yh)
    assert max(sa.max(), sc.max()) <= bound
    # and it is not loose: the largest deviation reached is within a few percent
    assert max(sa.max(), sc.max()) > 0.8 * bound


def test_default_sigma_is_five_pixels_at_the_near_plane():
    cam = camera_struct(make_camera(640, 480, 500.0, z_near=0.3))
    st = RasterSettings(splat="ewa")
    sig = st.sigma(cam)
    assert sig * cam.fx / cam.z_near == pytest.approx(5.0)
    assert RasterSettings(splat="ewa", ewa_sigma=0.01).sigma(cam) == 0.01
    o = st.opts(cam=cam)
    assert o.splat == 2 and o.ewa_sigma == pytest.approx(sig, rel=1e-6)
    # on axis at the near plane the projected deviation is exactly 5 px, and
    # off axis it grows with sqrt(1 + (x/z)^2): the bound exceeds 5 px
    assert o.max_radius > 5.0
    with pytest.raises(ValueError):
        st.opts()  # world-space splats need the camera


def test_point_ring_slots_wrap_and_checks():
    ring = PointRing(3, 10, 2, "cpu")
    clouds = []
    for k, n in enumerate((10, 4, 7, 2)):  # the fourth overwrites slot 0
        pos = torch.full((n, 3), float(k))
        s = ring.push(pos, torch.full((n,), 0.5), torch.full((n, 2), float(k)))
        clouds.append((s, n))
    assert [s for s, _ in clouds] == [0, 1, 2, 0]
    assert ring.counts == [2, 4, 7] and ring.next == 1
    assert (ring.pos[0:2] == 3.0).all() and (ring.pos[2:10] == 0.0).all()  # stale tail kept
    assert ring.slot_range(1) == slice(10, 14)
    with pytest.raises(ValueError):
        ring.push(torch.zeros(11, 3), torch.zeros(11), torch.zeros(11, 2))
    with pytest.raises(ValueError):
        ring.push(torch.zeros(3, 3), torch.zeros(3), torch.zeros(3, 5))
    with pytest.raises(ValueError):
        PointRing(17, 10, 2, "cpu")
    assert math.isclose(ring.opacity[10].item(), 0.5)
