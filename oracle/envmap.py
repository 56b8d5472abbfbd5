"""Oracle of the environment-map background -- TEST INFRASTRUCTURE ONLY.

Follows the paper's Sec. 3.2 "Faster Background Model Evaluation": the
background is a spherical environment map F_bg (an equirectangular image,
[Hm][Wm][C]) sampled with bilinear interpolation along every pixel's viewing
direction; the local view directions depend only on the intrinsics.  The
sampled background enters the image behind the points, F += T_final f_bg,
which the blend oracle (``render(..., bg=<[C][H][W] image>)``) composites.

Plain float64 numpy, written from the definition (the paper prints no
mapping, so the reading below is this implementation's and is stated in the
design notes):
  d     = normalize((x + 1/2 - cx) / fx, (y + 1/2 - cy) / fy, 1)  (camera space)
  w     = R^T d                                                  (world space)
  phi   = atan2(w_x, w_z),  theta = acos(-w_y / |w|)   (OpenCV axes: -y is up)
  s     = (phi / (2 pi) + 1/2) Wm,  t = (theta / pi) Hm
  texel (i, j) has its centre at (i + 1/2, j + 1/2); bilinear weights
  between the four surrounding centres, wrapping in longitude (i mod Wm) and
  clamping rows to [0, Hm - 1].
The backward is the adjoint of that linear map: every pixel's gradient is
scattered onto the four texels with the same weights.

Pins (tests/test_oracle_envmap.py): a constant map samples to that
constant; a map linear in the column samples to the column coordinate; the
forward direction +z lands on the centre column and the equator; the
vectorised form equals a per-pixel pure-Python loop; and the backward is the
exact adjoint of the forward (<G, F e> = <F^T G, e>).
"""
from __future__ import annotations

import math

import numpy as np


def view_dirs(camera) -> np.ndarray:
    """[H, W, 3] unit camera-space directions through the pixel centres."""
    W, H = int(camera.width), int(camera.height)
    x = (np.arange(W, dtype=np.float64) + 0.5 - float(camera.cx)) / float(camera.fx)
    y = (np.arange(H, dtype=np.float64) + 0.5 - float(camera.cy)) / float(camera.fy)
    d = np.empty((H, W, 3))
    d[..., 0] = x[None, :]
    d[..., 1] = y[:, None]
    d[..., 2] = 1.0
    return d / np.linalg.norm(d, axis=-1, keepdims=True)


def taps(camera, Hm: int, Wm: int, dirs=None):
    """Texel indices [4, H, W] (row-major into [Hm*Wm]) and weights [4, H, W]."""
    d = view_dirs(camera) if dirs is None else np.asarray(dirs, np.float64)
    R = np.asarray(camera.R, np.float64).reshape(3, 3)
    w = d @ R  # row vector form of R^T d
    phi = np.arctan2(w[..., 0], w[..., 2])
    theta = np.arccos(np.clip(-w[..., 1] / np.linalg.norm(w, axis=-1), -1.0, 1.0))
    s = (phi / (2.0 * math.pi) + 0.5) * Wm - 0.5
    t = theta / math.pi * Hm - 0.5
    x0 = np.floor(s)
    y0 = np.floor(t)
    a, b = s - x0, t - y0
    x0 = x0.astype(np.int64)
    y0 = y0.astype(np.int64)
    xs = (np.mod(x0, Wm), np.mod(x0 + 1, Wm))
    ys = (np.clip(y0, 0, Hm - 1), np.clip(y0 + 1, 0, Hm - 1))
    idx = np.stack([ys[0] * Wm + xs[0], ys[0] * Wm + xs[1], ys[1] * Wm + xs[0],
                    ys[1] * Wm + xs[1]])
    wt = np.stack([(1 - a) * (1 - b), a * (1 - b), (1 - a) * b, a * b])
    return idx, wt


def sample(camera, env: np.ndarray, dirs=None) -> np.ndarray:
    """Background image [C, H, W] from env [Hm, Wm, C]."""
    Hm, Wm, C = env.shape
    idx, wt = taps(camera, Hm, Wm, dirs)
    flat = np.asarray(env, np.float64).reshape(Hm * Wm, C)
    out = np.zeros((C,) + idx.shape[1:])
    for k in range(4):
        out += wt[k][None] * flat[idx[k]].transpose(2, 0, 1)
    return out


def sample_backward(camera, grad_bg: np.ndarray, Hm: int, Wm: int, dirs=None) -> np.ndarray:
    """dL/dF_bg [Hm, Wm, C] from dL/d(background image) [C, H, W]."""
    C = grad_bg.shape[0]
    idx, wt = taps(camera, Hm, Wm, dirs)
    g = np.zeros((Hm * Wm, C))
    G = np.asarray(grad_bg, np.float64)
    for k in range(4):
        np.add.at(g, idx[k].reshape(-1), (wt[k][None] * G).reshape(C, -1).T)
    return g.reshape(Hm, Wm, C)


def sample_loop(camera, env: np.ndarray) -> np.ndarray:
    """The same sample as a per-pixel pure-Python loop (tiny images only)."""
    Hm, Wm, C = env.shape
    R = np.asarray(camera.R, np.float64).reshape(3, 3)
    out = np.zeros((C, camera.height, camera.width))
    for y in range(camera.height):
        for x in range(camera.width):
            dx = (x + 0.5 - camera.cx) / camera.fx
            dy = (y + 0.5 - camera.cy) / camera.fy
            nrm = math.sqrt(dx * dx + dy * dy + 1.0)
            d = (dx / nrm, dy / nrm, 1.0 / nrm)
            w = [sum(R[k][j] * d[k] for k in range(3)) for j in range(3)]
            phi = math.atan2(w[0], w[2])
            theta = math.acos(max(-1.0, min(1.0, -w[1] / math.sqrt(sum(v * v for v in w)))))
            s = (phi / (2 * math.pi) + 0.5) * Wm - 0.5
            t = theta / math.pi * Hm - 0.5
            i0, j0 = math.floor(s), math.floor(t)
            a, b = s - i0, t - j0
            for di, dj, wgt in ((0, 0, (1 - a) * (1 - b)), (1, 0, a * (1 - b)),
                                (0, 1, (1 - a) * b), (1, 1, a * b)):
                i = (i0 + di) % Wm
                j = min(max(j0 + dj, 0), Hm - 1)
                for c in range(C):
                    out[c, y, x] += wgt * env[j, i, c]
    return out
