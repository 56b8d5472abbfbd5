"""Pins of the spherical-harmonics feature oracle (Sec. 2 "Implicit Point
Cloud": SH coefficients up to degree two per feature channel, evaluated at
the view direction)."""
import math

import numpy as np
import pytest
import torch

from oracle import sh
from scenes import ring_camera


def _quadrature(n_theta=8, n_phi=16):
    """Gauss-Legendre in cos(theta) times uniform phi: exact for products of
    two SH of degree <= 2 (polynomials of degree <= 4 on the sphere)."""
    x, w = np.polynomial.legendre.leggauss(n_theta)
    phi = (np.arange(n_phi) + 0.5) * 2 * math.pi / n_phi
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct * ct)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wt = np.repeat(w, n_phi) * (2 * math.pi / n_phi)
    return d, wt


def test_basis_is_orthonormal_on_the_sphere():
    d, w = _quadrature()
    Y = sh.basis(d)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(9), atol=1e-12)


def test_addition_theorem_per_degree():
    """sum over m of Y_lm(d)^2 = (2l + 1) / (4 pi) for every unit d: pins
    every constant, whatever the sign convention."""
    rng = np.random.default_rng(0)
    d = rng.standard_normal((200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = sh.basis(d)
    for l, sl in ((0, slice(0, 1)), (1, slice(1, 4)), (2, slice(4, 9))):
        np.testing.assert_allclose((Y[:, sl] ** 2).sum(1), (2 * l + 1) / (4 * math.pi),
                                   rtol=1e-12)


def test_degree_one_follows_the_direction():
    """The three degree-one functions are the direction's components up to
    one common factor (sqrt(3 / 4 pi)) and the phase convention's signs."""
    rng = np.random.default_rng(1)
    d = rng.standard_normal((50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = sh.basis(d)
    np.testing.assert_allclose(np.abs(Y[:, [3, 1, 2]]), math.sqrt(3 / (4 * math.pi)) * np.abs(d),
                               rtol=1e-12)


def _torch_features(cam, pos, coef):
    c = torch.tensor(sh.camera_centre(cam))
    v = pos - c
    d = v / v.norm(dim=-1, keepdim=True)
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    Y = torch.stack([torch.full_like(x, sh.K0), -sh.K1 * y, sh.K1 * z, -sh.K1 * x,
                     sh.K2 * x * y, -sh.K2 * y * z, sh.K3 * (2 * z * z - x * x - y * y),
                     -sh.K2 * x * z, sh.K4 * (x * x - y * y)], -1)
    return (Y[:, None, :] * coef).sum(-1)


def test_backward_matches_torch_autograd():
    cam = ring_camera(3, 8, 64, 48)
    rng = np.random.default_rng(2)
    n, C = 40, 4
    pos = rng.uniform(-3, 3, (n, 3)) + np.array([0.0, 0.0, 11.0])
    coef = rng.standard_normal((n, C, 9))
    g = rng.standard_normal((n, C))
    gsh, gpos = sh.features_backward(cam, pos, coef, g)
    p = torch.tensor(pos, requires_grad=True)
    k = torch.tensor(coef, requires_grad=True)
    f = _torch_features(cam, p, k)
    np.testing.assert_allclose(f.detach().numpy(), sh.features(cam, pos, coef), rtol=1e-13)
    (f * torch.tensor(g)).sum().backward()
    np.testing.assert_allclose(gsh, k.grad.numpy(), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(gpos, p.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_position_gradient_matches_central_differences():
    cam = ring_camera(0, 8, 64, 48)
    rng = np.random.default_rng(3)
    pos = rng.uniform(-2, 2, (5, 3)) + np.array([0.0, 0.0, 11.0])
    coef = rng.standard_normal((5, 2, 9))
    g = rng.standard_normal((5, 2))
    _, gpos = sh.features_backward(cam, pos, coef, g)
    h = 1e-6
    for i in range(5):
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, a] += h
            pm[i, a] -= h
            fd = ((sh.features(cam, pp, coef) - sh.features(cam, pm, coef)) * g).sum() / (2 * h)
            assert gpos[i, a] == pytest.approx(fd, rel=1e-6, abs=1e-9)
