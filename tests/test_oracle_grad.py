"""P10: the oracle's backward against (a) Eq. (1) written with torch float64
operations and differentiated by torch.autograd, and (b) central finite
differences of the oracle's own forward pass.  Neither shares the oracle's
hand-written backward (Appendix A, Eq. (2))."""
import numpy as np
import pytest
import torch

import oracle
from scenes import tiny_scene


def torch_eq1(cam, pos, opacity, feat, bg, G, Gt, t_min_counts=None):
    """Eq. (1) per pixel with torch float64 ops.  Fragment membership and
    order (discrete decisions) come from the projection; everything
    continuous is a torch expression of leaves u, v, o, f."""
    pr = oracle.project(cam, pos)
    vis = pr["visible"]
    uv32 = pr["uv"]
    key = pr["key"]
    n, C = feat.shape
    W, H = cam.width, cam.height
    u = torch.tensor(uv32[:, 0].astype(np.float64), requires_grad=True)
    v = torch.tensor(uv32[:, 1].astype(np.float64), requires_grad=True)
    o = torch.tensor(opacity.astype(np.float64), requires_grad=True)
    f = torch.tensor(feat.astype(np.float64), requires_grad=True)
    bgt = torch.tensor(np.zeros(C) if bg is None else np.asarray(bg, np.float64))
    x0 = np.floor(uv32[:, 0] - np.float32(0.5)).astype(np.int64)
    y0 = np.floor(uv32[:, 1] - np.float32(0.5)).astype(np.int64)
    frags = {}
    for i in np.nonzero(vis)[0]:
        for dy in (0, 1):
            for dx in (0, 1):
                px, py = x0[i] + dx, y0[i] + dy
                if 0 <= px < W and 0 <= py < H:
                    frags.setdefault((px, py), []).append((int(key[i]), int(i), dx, dy))
    loss = torch.zeros((), dtype=torch.float64)
    for (px, py), lst in frags.items():
        lst.sort()
        if t_min_counts is not None:
            lst = lst[:int(t_min_counts[py, px])]
        T = torch.ones((), dtype=torch.float64)
        F = torch.zeros(C, dtype=torch.float64)
        for _, i, dx, dy in lst:
            a = (u[i] - 0.5) - float(x0[i])
            b = (v[i] - 0.5) - float(y0[i])
            wx = a if dx else 1.0 - a
            wy = b if dy else 1.0 - b
            al = o[i] * wx * wy
            F = F + T * al * f[i]
            T = T * (1.0 - al)
        F = F + T * bgt
        loss = loss + (torch.tensor(G[:, py, px].astype(np.float64)) * F).sum() \
            + float(Gt[py, px]) * T
    # pixels without fragments contribute only G . bg and Gt, constant in the leaves
    loss.backward()
    return dict(grad_u=u.grad.numpy(), grad_v=v.grad.numpy(), grad_o=o.grad.numpy(),
                grad_f=f.grad.numpy())


@pytest.mark.parametrize("t_min", [0.0, 1e-4, 0.3])
def test_backward_matches_torch_autograd_of_eq1(t_min):
    s = tiny_scene(120, 24, 16, channels=3, seed=21, with_grad_t=True)
    bg = np.array([0.5, -0.25, 1.0])
    r = oracle.render(s.camera, s.pos, s.opacity, s.feat, bg=bg, t_min=t_min,
                      grad_out=s.grad, grad_t=s.grad_t)
    tt = torch_eq1(s.camera, s.pos, s.opacity, s.feat, bg, s.grad, s.grad_t,
                   t_min_counts=r["n_contrib"])
    np.testing.assert_allclose(r["grad_feat"], tt["grad_f"], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(r["grad_opacity"], tt["grad_o"], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(r["grad_uv"][:, 0], tt["grad_u"], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(r["grad_uv"][:, 1], tt["grad_v"], rtol=1e-10, atol=1e-12)
    # background gradient: dL/dbg = sum_p T_final(p) G(p)
    expect_bg = (r["t_final"][None] * s.grad.astype(np.float64)).sum(axis=(1, 2))
    np.testing.assert_allclose(r["grad_bg"], expect_bg, rtol=1e-12)


def test_position_chain_matches_torch_autograd():
    """a7: dL/dp = R^T (dL/dX, dL/dY, dL/dZ) for u = fx X/Z + cx, v = fy Y/Z + cy."""
    from scenes import ring_camera
    s = tiny_scene(80, 20, 14, channels=2, seed=8)
    cam = ring_camera(1, 8, 20, 14)
    # move the cloud in front of the rotated camera
    R = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    pos = ((s.pos.astype(np.float64) - t) @ R).astype(np.float32)
    r = oracle.render(cam, pos, s.opacity, s.feat, grad_out=s.grad)
    vis = oracle.project(cam, pos)["visible"]
    assert vis.sum() > 40
    p = torch.tensor(pos.astype(np.float64), requires_grad=True)
    X = p @ torch.tensor(R.T) + torch.tensor(t)
    u = cam.fx * X[:, 0] / X[:, 2] + cam.cx
    v = cam.fy * X[:, 1] / X[:, 2] + cam.cy
    gu = torch.tensor(r["grad_uv"][:, 0])
    gv = torch.tensor(r["grad_uv"][:, 1])
    ((u * gu + v * gv) * torch.tensor(vis.astype(np.float64))).sum().backward()
    np.testing.assert_allclose(r["grad_pos"], p.grad.numpy(), rtol=1e-9, atol=1e-12)


def _loss(r, G):
    return float((G.astype(np.float64) * r["out"]).sum())


def test_feature_and_opacity_gradients_match_central_differences():
    """F is affine in each feature and in each fragment's alpha = o w, and a
    point's fragments sit on distinct pixels, so with t_min = 0 the loss is
    affine in every f_i and o_i: central differences are exact."""
    s = tiny_scene(100, 20, 12, channels=2, seed=9)
    r = oracle.render(s.camera, s.pos, s.opacity, s.feat, t_min=0.0, grad_out=s.grad)
    rng = np.random.default_rng(0)
    vis = np.nonzero(oracle.project(s.camera, s.pos)["visible"])[0]
    h = 1e-6
    for i in rng.choice(vis, 8, replace=False):
        for c in range(2):
            fp = s.feat.astype(np.float64)
            fm = fp.copy()
            fp[i, c] += h
            fm[i, c] -= h
            fd = (_loss(oracle.render(s.camera, s.pos, s.opacity, fp, t_min=0.0), s.grad)
                  - _loss(oracle.render(s.camera, s.pos, s.opacity, fm, t_min=0.0), s.grad)) / (2 * h)
            assert r["grad_feat"][i, c] == pytest.approx(fd, rel=1e-6, abs=1e-9)
        hq = 2.0 ** -12  # exact shift of an FP32 opacity in [0.25, 1)
        if s.opacity[i] < 0.25:
            continue
        op, om = s.opacity.copy(), s.opacity.copy()
        op[i] += np.float32(hq)
        om[i] -= np.float32(hq)
        fd = (_loss(oracle.render(s.camera, s.pos, op, s.feat, t_min=0.0), s.grad)
              - _loss(oracle.render(s.camera, s.pos, om, s.feat, t_min=0.0), s.grad)) / (2 * hq)
        assert r["grad_opacity"][i] == pytest.approx(fd, rel=1e-9, abs=1e-12)


def test_uv_gradients_match_central_differences():
    """Away from the floor() kinks (a, b not near 0 or 1) and without depth
    changes, the loss is affine in a point's u: central differences over the
    actual FP32 shift of u are exact."""
    s = tiny_scene(100, 20, 12, channels=2, seed=10)
    r = oracle.render(s.camera, s.pos, s.opacity, s.feat, t_min=0.0, grad_out=s.grad)
    pr = oracle.project(s.camera, s.pos)
    checked = 0
    for i in np.nonzero(pr["visible"])[0]:
        u = float(pr["uv"][i, 0])
        a = (u - 0.5) - np.floor(u - 0.5)
        if not (0.05 < a < 0.95) or not (1.0 < u < s.camera.width - 1.0):
            continue
        Z = float(pr["xyz"][i, 2])
        dx = 2.0 ** -9 * Z / s.camera.fx
        pp, pm = s.pos.copy(), s.pos.copy()
        pp[i, 0] += np.float32(dx)
        pm[i, 0] -= np.float32(dx)
        up = float(oracle.project(s.camera, pp)["uv"][i, 0])
        um = float(oracle.project(s.camera, pm)["uv"][i, 0])
        fd = (_loss(oracle.render(s.camera, pp, s.opacity, s.feat, t_min=0.0), s.grad)
              - _loss(oracle.render(s.camera, pm, s.opacity, s.feat, t_min=0.0), s.grad)) / (up - um)
        assert r["grad_uv"][i, 0] == pytest.approx(fd, rel=1e-6, abs=1e-9)
        checked += 1
        if checked == 8:
            break
    assert checked == 8


def torch_eq1_gauss(cam, pos, radius, opacity, feat, bg, G, Gt, n_contrib, dilation=0.16,
                    cutoff=3.0):
    """Eq. (1) per pixel with Gaussian fragment weights, in torch float64.

    Fragment membership and order are the FP32 decisions of the screen-space
    Gaussian footprint (bounding box, then d^2 <= cutoff^2 s2), taken here
    with numpy float32 scalars; the weight exp(-d^2 / (2 s2)) is a torch
    expression of the leaves u, v, so autograd differentiates it
    independently of the oracle's hand-written dw/du, dw/dv."""
    f32 = np.float32
    pr = oracle.project(cam, pos, radius, splat=oracle.SPLAT_GAUSSIAN, dilation=dilation,
                        cutoff=cutoff)
    vis, uv32, key, rect = pr["visible"], pr["uv"], pr["key"], pr["rect"]
    n, C = feat.shape
    W, H = cam.width, cam.height
    u = torch.tensor(uv32[:, 0].astype(np.float64), requires_grad=True)
    v = torch.tensor(uv32[:, 1].astype(np.float64), requires_grad=True)
    o = torch.tensor(opacity.astype(np.float64), requires_grad=True)
    f = torch.tensor(feat.astype(np.float64), requires_grad=True)
    bgt = torch.tensor(np.zeros(C) if bg is None else np.asarray(bg, np.float64))
    frags = {}
    for i in np.nonzero(vis)[0]:
        r = f32(radius[i])
        s2 = f32(r * r) + f32(dilation)
        thr = f32(f32(cutoff) * f32(cutoff)) * s2
        for py in range(rect[i, 1], rect[i, 3] + 1):
            for px in range(rect[i, 0], rect[i, 2] + 1):
                dx = f32(f32(px) + f32(0.5)) - uv32[i, 0]
                dy = f32(f32(py) + f32(0.5)) - uv32[i, 1]
                if f32(f32(dx * dx) + f32(dy * dy)) <= thr:
                    frags.setdefault((px, py), []).append((int(key[i]), int(i), float(s2)))
    loss = torch.zeros((), dtype=torch.float64)
    for (px, py), lst in frags.items():
        lst.sort()
        lst = lst[:int(n_contrib[py, px])]
        T = torch.ones((), dtype=torch.float64)
        F = torch.zeros(C, dtype=torch.float64)
        for _, i, s2 in lst:
            d2 = ((px + 0.5) - u[i]) ** 2 + ((py + 0.5) - v[i]) ** 2
            al = o[i] * torch.exp(-0.5 * d2 / s2)
            F = F + T * al * f[i]
            T = T * (1.0 - al)
        F = F + T * bgt
        loss = loss + (torch.tensor(G[:, py, px].astype(np.float64)) * F).sum() \
            + float(Gt[py, px]) * T
    loss.backward()
    return dict(grad_u=u.grad.numpy(), grad_v=v.grad.numpy(), grad_o=o.grad.numpy(),
                grad_f=f.grad.numpy())


@pytest.mark.parametrize("t_min", [0.0, 1e-4, 0.3])
def test_gaussian_backward_matches_torch_autograd_of_eq1(t_min):
    """The oracle's Gaussian weight derivatives (dw/du = w dx / s2, dw/dv =
    w dy / s2) and the rest of Eq. (2) for Gaussian fragments, against
    autograd of the Gaussian-weighted Eq. (1) (Sec. 3.2 "Rendering Points as
    Small Gaussians": dilation 0.16, cut at 3 sigma)."""
    s = tiny_scene(40, 20, 14, channels=3, seed=31, with_grad_t=True, radius_range=(0.5, 2.0))
    bg = np.array([0.25, -0.5, 1.0])
    r = oracle.render(s.camera, s.pos, s.opacity, s.feat, radius=s.radius, bg=bg,
                      splat=oracle.SPLAT_GAUSSIAN, t_min=t_min, grad_out=s.grad,
                      grad_t=s.grad_t)
    assert (r["flags"] == 0).all()
    tt = torch_eq1_gauss(s.camera, s.pos, s.radius, s.opacity, s.feat, bg, s.grad, s.grad_t,
                         r["n_contrib"])
    assert np.abs(tt["grad_u"]).max() > 0.1  # the weights' slopes are exercised
    np.testing.assert_allclose(r["grad_feat"], tt["grad_f"], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(r["grad_opacity"], tt["grad_o"], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(r["grad_uv"][:, 0], tt["grad_u"], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(r["grad_uv"][:, 1], tt["grad_v"], rtol=1e-10, atol=1e-12)


def test_gaussian_uv_gradients_match_central_differences():
    """Moving a Gaussian without changing which pixels it covers changes the
    loss smoothly: central differences over the actual FP32 shift of u,
    with the fragment set checked unchanged at both ends."""
    s = tiny_scene(60, 20, 14, channels=2, seed=32, radius_range=(0.7, 1.5))
    kw = dict(radius=s.radius, splat=oracle.SPLAT_GAUSSIAN, t_min=0.0)
    r = oracle.render(s.camera, s.pos, s.opacity, s.feat, grad_out=s.grad, **kw)
    pr = oracle.project(s.camera, s.pos, s.radius, splat=oracle.SPLAT_GAUSSIAN)
    nfrag = oracle.count_fragments(s.camera, s.pos, s.radius, splat=oracle.SPLAT_GAUSSIAN)
    checked = 0
    for i in np.nonzero(pr["visible"])[0]:
        Z = float(pr["xyz"][i, 2])
        dx = 2.0 ** -12 * Z / s.camera.fx
        pp, pm = s.pos.copy(), s.pos.copy()
        pp[i, 0] += np.float32(dx)
        pm[i, 0] -= np.float32(dx)
        cnt = [oracle.count_fragments(s.camera, q, s.radius, splat=oracle.SPLAT_GAUSSIAN)
               for q in (pp, pm)]
        rp = oracle.project(s.camera, pp, s.radius, splat=oracle.SPLAT_GAUSSIAN)
        rm = oracle.project(s.camera, pm, s.radius, splat=oracle.SPLAT_GAUSSIAN)
        if cnt != [nfrag, nfrag] or not (rp["rect"][i] == pr["rect"][i]).all() \
                or not (rm["rect"][i] == pr["rect"][i]).all():
            continue
        up, um = float(rp["uv"][i, 0]), float(rm["uv"][i, 0])
        fd = (_loss(oracle.render(s.camera, pp, s.opacity, s.feat, **kw), s.grad)
              - _loss(oracle.render(s.camera, pm, s.opacity, s.feat, **kw), s.grad)) / (up - um)
        assert r["grad_uv"][i, 0] == pytest.approx(fd, rel=1e-4, abs=1e-7)
        checked += 1
        if checked == 8:
            break
    assert checked == 8


@pytest.mark.parametrize("splat", [oracle.SPLAT_BILINEAR, oracle.SPLAT_GAUSSIAN])
def test_pixel_mask_computes_the_same_pixels(splat):
    """The sampled-pixel forward (for scenes too large for the full fragment
    set) equals the full forward on every masked pixel and leaves the rest."""
    s = tiny_scene(300, 33, 21, channels=3, seed=33,
                   radius_range=(0.5, 2.5) if splat else None)
    rad = s.radius if splat else None
    full = oracle.render(s.camera, s.pos, s.opacity, s.feat, radius=rad, splat=splat)
    mask = np.random.default_rng(1).random((21, 33)) < 0.3
    part = oracle.render(s.camera, s.pos, s.opacity, s.feat, radius=rad, splat=splat,
                         pixel_mask=mask)
    for k in ("out", "out_abs"):
        np.testing.assert_array_equal(part[k][:, mask], full[k][:, mask])
        assert (part[k][:, ~mask] == 0).all()
    for k in ("t_final", "n_contrib", "flags"):
        np.testing.assert_array_equal(part[k][mask], full[k][mask])
    with pytest.raises(ValueError):
        oracle.render(s.camera, s.pos, s.opacity, s.feat, grad_out=s.grad, pixel_mask=mask)
