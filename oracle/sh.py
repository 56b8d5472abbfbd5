"""Oracle of the view-dependent point features -- TEST INFRASTRUCTURE ONLY.

Follows the paper's Sec. 2 "Implicit Point Cloud": the appearance field
gives every point spherical-harmonics coefficients up to degree two,
f_hat in R^{C x 9} (C = 4 in the paper), which evaluated at the view
direction give the C features the rasterizer blends.

Plain float64 numpy from the definition.  Readings (the paper names only
the degree): the view direction is the unit vector from the camera centre
c = -R^T t to the point, d = (p - c) / |p - c|; the basis is the real
orthonormal spherical harmonics of degrees 0-2 in the usual graphics
ordering and sign convention (Condon-Shortley phase), in terms of the
direction's components (x, y, z):
  Y0 = k0,  Y1 = -k1 y,  Y2 = k1 z,  Y3 = -k1 x,
  Y4 = k2 x y,  Y5 = -k2 y z,  Y6 = k3 (2 z^2 - x^2 - y^2),  Y7 = -k2 x z,
  Y8 = k4 (x^2 - y^2)
with k0 = 1 / (2 sqrt(pi)), k1 = sqrt(3 / (4 pi)), k2 = sqrt(15 / (4 pi)),
k3 = sqrt(5 / (16 pi)), k4 = sqrt(15 / (16 pi)); f[c] = sum_j Y_j(d) f_hat[c][j],
no offset and no clamp (these are features, not colours).

Pins (tests/test_oracle_sh.py): orthonormality of the basis under a
spherical quadrature; the addition theorem (sum over m of Y_lm^2 =
(2l + 1) / (4 pi) for every direction); degree one proportional to the
direction's components; the feature and position gradients against torch
float64 autograd of the same formula and central differences.
"""
from __future__ import annotations

import math

import numpy as np

K0 = 0.5 / math.sqrt(math.pi)
K1 = math.sqrt(3.0 / (4.0 * math.pi))
K2 = math.sqrt(15.0 / (4.0 * math.pi))
K3 = math.sqrt(5.0 / (16.0 * math.pi))
K4 = math.sqrt(15.0 / (16.0 * math.pi))


def camera_centre(camera) -> np.ndarray:
    R = np.asarray(camera.R, np.float64).reshape(3, 3)
    t = np.asarray(camera.t, np.float64).reshape(3)
    return -R.T @ t


def basis(d: np.ndarray) -> np.ndarray:
    """[..., 9] real SH of degrees 0-2 at unit directions d [..., 3]."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    return np.stack([np.full_like(x, K0), -K1 * y, K1 * z, -K1 * x,
                     K2 * x * y, -K2 * y * z, K3 * (2 * z * z - x * x - y * y), -K2 * x * z,
                     K4 * (x * x - y * y)], axis=-1)


def basis_jacobian(d: np.ndarray) -> np.ndarray:
    """[..., 9, 3]: dY_j / d(x, y, z), the direction taken as free."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    o = np.zeros_like(x)
    rows = [
        (o, o, o),
        (o, -K1 + o, o),
        (o, o, K1 + o),
        (-K1 + o, o, o),
        (K2 * y, K2 * x, o),
        (o, -K2 * z, -K2 * y),
        (-2 * K3 * x, -2 * K3 * y, 4 * K3 * z),
        (-K2 * z, o, -K2 * x),
        (2 * K4 * x, -2 * K4 * y, o),
    ]
    return np.stack([np.stack(r, axis=-1) for r in rows], axis=-2)


def features(camera, pos: np.ndarray, sh: np.ndarray) -> np.ndarray:
    """[n, C] features from positions [n, 3] and coefficients [n, C, 9]."""
    v = np.asarray(pos, np.float64) - camera_centre(camera)
    d = v / np.linalg.norm(v, axis=-1, keepdims=True)
    return np.einsum("nj,ncj->nc", basis(d), np.asarray(sh, np.float64))


def features_backward(camera, pos: np.ndarray, sh: np.ndarray, grad_feat: np.ndarray):
    """(dL/dsh [n, C, 9], dL/dpos [n, 3]) from dL/df [n, C]."""
    v = np.asarray(pos, np.float64) - camera_centre(camera)
    r = np.linalg.norm(v, axis=-1, keepdims=True)
    d = v / r
    g = np.asarray(grad_feat, np.float64)
    shd = np.asarray(sh, np.float64)
    grad_sh = g[:, :, None] * basis(d)[:, None, :]
    # dL/dY_j = sum_c g_c sh[c][j]; dL/dd = J^T dL/dY; through d = v / |v|
    gY = np.einsum("nc,ncj->nj", g, shd)
    gd = np.einsum("nj,njk->nk", gY, basis_jacobian(d))
    gv = (gd - d * (gd * d).sum(-1, keepdims=True)) / r
    return grad_sh, gv
