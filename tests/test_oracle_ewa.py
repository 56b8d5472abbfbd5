"""Pins of the oracle's world-space Gaussians (Sec. 3.2 "Rendering Points as
Small Gaussians": isotropic world-space Gaussians projected with the affine
(EWA) approximation of the perspective map, dilated by 0.16 and cut at
3 sigma): closed forms for one point, the blend and every gradient against
torch float64 autograd of Eq. (1) with the projected covariance written as
torch expressions, and central differences of positions."""
import math

import numpy as np
import pytest
import torch

import oracle
from scenes import Camera, make_camera, ring_camera, tiny_scene

E = oracle.SPLAT_EWA


def _one_point(cam, X, Y, Z, o=0.8, f=(1.0, -2.0)):
    R = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    p = (R.T @ (np.array([X, Y, Z]) - t)).astype(np.float32)[None]
    return p, np.array([o], np.float32), np.array([f], np.float64)


@pytest.mark.parametrize("X,Y", [(0.0, 0.0), (1.3, 0.0), (0.0, -0.9)])
def test_single_point_profile_closed_form(X, Y):
    """One point, t_min = 0: every pixel holds o exp(-d^T S^-1 d / 2) f with
    S = sigma^2 J J^T + 0.16 I (diagonal when X or Y is zero) and nothing
    past the 3-sigma ellipse."""
    cam = make_camera(64, 48, 40.0)
    sig, Z = 0.05, 3.0
    p, o, f = _one_point(cam, X, Y, Z)
    r = oracle.render(cam, p, o, f, splat=E, t_min=0.0, ewa_sigma=sig)
    pr = oracle.project(cam, p, splat=E, ewa_sigma=sig)
    u, v = (float(x) for x in pr["uv"][0])
    fx, fy = cam.fx, cam.fy
    xh, yh = (u - cam.cx) / fx, (v - cam.cy) / fy
    a = sig ** 2 * (fx / Z) ** 2 * (1 + xh * xh) + 0.16
    c = sig ** 2 * (fy / Z) ** 2 * (1 + yh * yh) + 0.16
    assert sig ** 2 * (fx / Z) * (fy / Z) * xh * yh == 0.0
    ys, xs = np.mgrid[0:48, 0:64]
    dx, dy = xs + 0.5 - u, ys + 0.5 - v
    q = dx * dx / a + dy * dy / c
    expect = np.where(q <= 9.0, 0.8 * np.exp(-0.5 * q), 0.0)
    inside = np.abs(q - 9.0) > 1e-4  # the cut itself is an FP32 decision
    for ch, fc in enumerate(f[0]):
        np.testing.assert_allclose(r["out"][ch][inside], (expect * fc)[inside], rtol=1e-6,
                                   atol=1e-9)
    assert (r["n_contrib"] == (q <= 9.0)).mean() > 0.999


def test_on_axis_point_matches_the_screen_space_gaussian():
    """On the optical axis the projected covariance is isotropic with
    standard deviation sigma fx / Z: the same point as a screen-space
    Gaussian of that radius gives the same image."""
    cam = make_camera(48, 48, 30.0)
    sig, Z = 0.1, 2.5
    p, o, f = _one_point(cam, 0.0, 0.0, Z)
    a = oracle.render(cam, p, o, f, splat=E, t_min=0.0, ewa_sigma=sig)
    b = oracle.render(cam, p, o, f, radius=np.array([sig * cam.fx / Z], np.float32),
                      splat=oracle.SPLAT_GAUSSIAN, t_min=0.0)
    np.testing.assert_allclose(a["out"], b["out"], rtol=1e-6, atol=1e-12)


def torch_eq1_ewa(cam, pos, opacity, feat, G, Gt, n_contrib, sig, dil=0.16, cutoff=3.0):
    """Eq. (1) with world-space Gaussian weights in torch float64.  Leaves:
    u, v, Z (as the oracle's FP32 values), o, f.  Fragment membership and
    order are the FP32 decisions, recomputed here with numpy float32."""
    f32 = np.float32
    pr = oracle.project(cam, pos, splat=E, ewa_sigma=sig)
    vis, uv32, key, rect, xyz = pr["visible"], pr["uv"], pr["key"], pr["rect"], pr["xyz"]
    n, C = feat.shape
    W, H = cam.width, cam.height
    u = torch.tensor(uv32[:, 0].astype(np.float64), requires_grad=True)
    v = torch.tensor(uv32[:, 1].astype(np.float64), requires_grad=True)
    Zt = torch.tensor(xyz[:, 2].astype(np.float64), requires_grad=True)
    o = torch.tensor(opacity.astype(np.float64), requires_grad=True)
    f = torch.tensor(feat.astype(np.float64), requires_grad=True)
    frags = {}
    fx, fy, cx, cy = f32(cam.fx), f32(cam.fy), f32(cam.cx), f32(cam.cy)
    for i in np.nonzero(vis)[0]:
        U, V, Z = uv32[i, 0], uv32[i, 1], xyz[i, 2]
        xh, yh = (U - cx) / fx, (V - cy) / fy
        jx, jy = fx / Z, fy / Z
        s2 = f32(sig) * f32(sig)
        a = s2 * ((jx * jx) * (f32(1) + xh * xh)) + f32(dil)
        b = s2 * ((jx * jy) * (xh * yh))
        c = s2 * ((jy * jy) * (f32(1) + yh * yh)) + f32(dil)
        det = a * c - b * b
        A, B, Cc = c / det, -(b / det), a / det
        for py in range(rect[i, 1], rect[i, 3] + 1):
            for px in range(rect[i, 0], rect[i, 2] + 1):
                dx = (f32(px) + f32(0.5)) - U
                dy = (f32(py) + f32(0.5)) - V
                d2 = (A * (dx * dx) + (f32(2) * B) * (dx * dy)) + Cc * (dy * dy)
                if d2 <= f32(cutoff) * f32(cutoff):
                    frags.setdefault((px, py), []).append((int(key[i]), int(i)))
    # the parameters reach the oracle as FP32 values
    sig, dil = float(np.float32(sig)), float(np.float32(dil))
    loss = torch.zeros((), dtype=torch.float64)
    for (px, py), lst in frags.items():
        lst.sort()
        lst = lst[:int(n_contrib[py, px])]
        T = torch.ones((), dtype=torch.float64)
        F = torch.zeros(C, dtype=torch.float64)
        for _, i in lst:
            xh = (u[i] - cam.cx) / cam.fx
            yh = (v[i] - cam.cy) / cam.fy
            jx, jy = cam.fx / Zt[i], cam.fy / Zt[i]
            a = sig ** 2 * jx * jx * (1 + xh * xh) + dil
            b = sig ** 2 * jx * jy * xh * yh
            c = sig ** 2 * jy * jy * (1 + yh * yh) + dil
            det = a * c - b * b
            dx = (px + 0.5) - u[i]
            dy = (py + 0.5) - v[i]
            d2 = (c * dx * dx - 2 * b * dx * dy + a * dy * dy) / det
            al = o[i] * torch.exp(-0.5 * d2)
            F = F + T * al * f[i]
            T = T * (1.0 - al)
        loss = loss + (torch.tensor(G[:, py, px].astype(np.float64)) * F).sum() \
            + float(Gt[py, px]) * T
    loss.backward()
    return dict(grad_u=u.grad.numpy(), grad_v=v.grad.numpy(), grad_z=Zt.grad.numpy(),
                grad_o=o.grad.numpy(), grad_f=f.grad.numpy())


@pytest.mark.parametrize("t_min", [0.0, 1e-4])
def test_ewa_backward_matches_torch_autograd(t_min):
    cam = ring_camera(2, 8, 24, 18)
    s = tiny_scene(40, 24, 18, channels=3, seed=41, with_grad_t=True)
    R = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    pos = ((s.pos.astype(np.float64) - t) @ R).astype(np.float32)  # in front of the camera
    sig = 0.02
    r = oracle.render(cam, pos, s.opacity, s.feat, splat=E, t_min=t_min, ewa_sigma=sig,
                      grad_out=s.grad, grad_t=s.grad_t)
    assert (r["flags"] == 0).all()
    tt = torch_eq1_ewa(cam, pos, s.opacity, s.feat, s.grad, s.grad_t, r["n_contrib"], sig)
    assert np.abs(tt["grad_z"]).max() > 1e-3  # the covariance's Z-dependence is exercised
    for k, ref in (("grad_feat", tt["grad_f"]), ("grad_opacity", tt["grad_o"])):
        np.testing.assert_allclose(r[k], ref, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(r["grad_uv"][:, 0], tt["grad_u"], rtol=1e-8, atol=1e-11)
    np.testing.assert_allclose(r["grad_uv"][:, 1], tt["grad_v"], rtol=1e-8, atol=1e-11)
    np.testing.assert_allclose(r["grad_z"], tt["grad_z"], rtol=1e-8, atol=1e-11)
    # position chain: u = fx X/Z + cx, v = fy Y/Z + cy, and Z itself
    vis = oracle.project(cam, pos, splat=E, ewa_sigma=sig)["visible"]
    p = torch.tensor(pos.astype(np.float64), requires_grad=True)
    X = p @ torch.tensor(R.T) + torch.tensor(t)
    uu = cam.fx * X[:, 0] / X[:, 2] + cam.cx
    vv = cam.fy * X[:, 1] / X[:, 2] + cam.cy
    m = torch.tensor(vis.astype(np.float64))
    ((uu * torch.tensor(r["grad_uv"][:, 0]) + vv * torch.tensor(r["grad_uv"][:, 1])
      + X[:, 2] * torch.tensor(r["grad_z"])) * m).sum().backward()
    np.testing.assert_allclose(r["grad_pos"], p.grad.numpy(), rtol=1e-9, atol=1e-12)


def test_ewa_position_gradients_match_central_differences():
    """Shifting a point along the camera axes changes u, v, Z and the
    covariance; while the fragment set stays the same the loss is smooth."""
    cam = make_camera(24, 18, 16.0)
    s = tiny_scene(30, 24, 18, channels=2, seed=42)
    sig = 0.03
    kw = dict(splat=E, t_min=0.0, ewa_sigma=sig)
    r = oracle.render(cam, s.pos, s.opacity, s.feat, grad_out=s.grad, **kw)
    pr = oracle.project(cam, s.pos, splat=E, ewa_sigma=sig)
    n0 = oracle.count_fragments(cam, s.pos, splat=E, ewa_sigma=sig)
    loss = lambda rr: float((s.grad.astype(np.float64) * rr["out"]).sum())
    checked = 0
    for i in np.nonzero(pr["visible"])[0]:
        for ax in range(3):
            h = 2.0 ** -11 * (4.0 if ax == 2 else 1.0)
            pp, pm = s.pos.copy(), s.pos.copy()
            pp[i, ax] += np.float32(h)
            pm[i, ax] -= np.float32(h)
            if any(oracle.count_fragments(cam, q, splat=E, ewa_sigma=sig) != n0 for q in (pp, pm)):
                continue
            step = float(pp[i, ax]) - float(pm[i, ax])
            fd = (loss(oracle.render(cam, pp, s.opacity, s.feat, **kw))
                  - loss(oracle.render(cam, pm, s.opacity, s.feat, **kw))) / step
            assert r["grad_pos"][i, ax] == pytest.approx(fd, rel=1e-3, abs=1e-6)
            checked += 1
        if checked >= 12:
            break
    assert checked >= 12
