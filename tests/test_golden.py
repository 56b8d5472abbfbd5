"""The oracle reproduces the numbers the paper prints (tests/golden/paper_numbers.txt)."""
import math
import os

import numpy as np

import oracle
from scenes import Camera

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.txt")


def golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, value, _cite = [x.strip() for x in line.split("|", 2)]
        out[name] = float(value)
    return out


def _cam(W, H):
    return Camera(width=W, height=H, fx=float(W), fy=float(W), cx=W / 2, cy=H / 2,
                  R=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32))


def mean_tiles_per_splat(T):
    """Oracle tile count averaged over a uniform grid of sub-tile positions
    for splats fully inside the image."""
    W = H = 4 * T
    cam = _cam(W, H)
    g = np.arange(T, 2 * T, 0.25) + 0.5 + 0.125
    u, v = np.meshgrid(g, g)
    u, v = u.ravel(), v.ravel()
    pos = np.stack([(u - cam.cx) * 2.0 / cam.fx, (v - cam.cy) * 2.0 / cam.fy, np.full(u.size, 2.0)], 1)
    return float(oracle.project(cam, pos.astype(np.float32), tile=T)["ntiles"].mean())


def test_tiles_per_splat():
    assert round(mean_tiles_per_splat(8), 2) == golden()["tiles_per_splat_8x8"]


def test_id_bits_and_sort_cost_model():
    gd = golden()
    tl = oracle.tile_lists(_cam(1920, 1080), np.zeros((0, 3), np.float32), tile=8)
    n_tiles = tl["ntx"] * tl["nty"]
    tile_bits = int(n_tiles - 1).bit_length()
    pixel_bits = int(1920 * 1080 - 1).bit_length()
    assert tile_bits == gd["tile_id_bits_1080p_8x8"]
    assert pixel_bits == gd["pixel_id_bits_1080p"]
    copies = round(mean_tiles_per_splat(8), 2)
    assert 4 * math.ceil((32 + pixel_bits) / 8) == gd["sort_cost_per_pixel_lists"]
    assert round(copies * math.ceil((32 + tile_bits) / 8), 2) == gd["sort_cost_tiled"]
    assert round(4 + 2 * copies, 2) == gd["sort_cost_split"]


def test_gaussian_defaults_follow_the_paper():
    """With r = 0 the footprint is the dilation Gaussian alone: a pixel at
    distance d carries exp(-d^2 / (2 * 0.16)) and nothing lies beyond
    3 * sqrt(0.16) = 1.2 px."""
    gd = golden()
    cam = Camera(width=16, height=16, fx=16.0, fy=16.0, cx=8.0, cy=8.0,
                 R=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32))
    pos = np.array([[(7.5 - 8.0) * 2 / 16, (7.5 - 8.0) * 2 / 16, 2.0]], np.float32)
    r = oracle.render(cam, pos, np.ones(1, np.float32), np.ones((1, 1), np.float32),
                      radius=np.zeros(1, np.float32), splat=1, t_min=0.0)
    img = r["out"][0]
    var = gd["gaussian_dilation_variance"]
    s2 = float(np.float32(0.0) + np.float32(var))
    assert img[7, 8] == math.exp(-0.5 * 1.0 / s2)
    reach = gd["gaussian_cutoff_sigma"] * math.sqrt(var)
    yy, xx = np.mgrid[0:16, 0:16]
    far = (xx - 7) ** 2 + (yy - 7) ** 2 > reach ** 2
    assert (img[far] == 0).all() and (img[~far] > 0).all()
