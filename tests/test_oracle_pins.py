"""Pins of the CPU oracle against closed forms and invariants (no GPU).

Every expected value here comes from the mathematics of the method, written
independently of the oracle: bilinear weights of a splat placed at a chosen
sub-pixel offset (Sec. 2 / Sec. 3.2), Eq. (1) expanded by hand for two and
three fragments, the derivative of Eq. (1) (Appendix A, Eq. (2), with the
sign of the background term that differentiation gives), tile statistics of
Sec. 3.2 "Tiled Rendering", and the Gaussian profile of Sec. 3.2 "Rendering
Points as Small Gaussians".
"""
import math

import numpy as np
import pytest

import oracle
from scenes import Camera, make_camera, tiny_scene


def cam32():
    # u = 16 * X / Z + 16, v = 16 * Y / Z + 12
    return Camera(width=32, height=24, fx=16.0, fy=16.0, cx=16.0, cy=12.0,
                  R=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32), z_near=0.2)


def place(cam, u, v, Z):
    """World point projecting exactly to (u, v) for dyadic inputs."""
    return [(u - cam.cx) * Z / cam.fx, (v - cam.cy) * Z / cam.fy, Z]


def test_projection_is_exact_for_dyadic_points():
    cam = cam32()
    pts = np.array([place(cam, 10.75, 7.5, 2.0), place(cam, 3.125, 20.25, 4.0)], np.float32)
    pr = oracle.project(cam, pts)
    np.testing.assert_array_equal(pr["uv"], np.array([[10.75, 7.5], [3.125, 20.25]], np.float32))
    assert pr["visible"].all()
    # depth key is the FP32 bit pattern of camera-space Z
    assert pr["key"][0] == np.float32(2.0).view(np.uint32)
    assert pr["key"][1] == np.float32(4.0).view(np.uint32)


def test_p1_single_bilinear_splat_closed_form():
    """P1: one splat, bg = 0, t_min = 0: F = o w f per pixel, T = 1 - o w,
    and the four weights sum to one so the image sums to o f."""
    cam = cam32()
    a, b = 0.25, 0.75  # u = x0 + 0.5 + a, v = y0 + 0.5 + b with x0 = 10, y0 = 6
    u, v = 10 + 0.5 + a, 6 + 0.5 + b
    pos = np.array([place(cam, u, v, 2.0)], np.float32)
    o = np.array([0.625], np.float32)
    f = np.array([[1.0, -2.0, 0.5]], np.float32)
    r = oracle.render(cam, pos, o, f, t_min=0.0)
    w = {(10, 6): (1 - a) * (1 - b), (11, 6): a * (1 - b), (10, 7): (1 - a) * b, (11, 7): a * b}
    expect = np.zeros((3, 24, 32))
    tf = np.ones((24, 32))
    for (x, y), wv in w.items():
        expect[:, y, x] = 0.625 * wv * f[0]
        tf[y, x] = 1 - 0.625 * wv
    np.testing.assert_allclose(r["out"], expect, rtol=0, atol=1e-15)
    np.testing.assert_allclose(r["t_final"], tf, rtol=0, atol=1e-15)
    np.testing.assert_allclose(r["out"].sum(axis=(1, 2)), 0.625 * f[0].astype(np.float64), atol=1e-14)
    nc = np.zeros((24, 32), np.uint32)
    for (x, y) in w:
        nc[y, x] = 1
    np.testing.assert_array_equal(r["n_contrib"], nc)


def test_p2_alpha_one_occludes_everything_behind():
    """P2: an o = 1 point at a pixel centre (w00 = 1) in front of others: that
    pixel shows exactly its features, T_final = 0, and the points behind get
    no feature or opacity gradient from it."""
    cam = cam32()
    x0, y0 = 9, 5
    u, v = x0 + 0.5, y0 + 0.5
    pos = np.array([place(cam, u, v, 4.0), place(cam, u, v, 2.0), place(cam, u, v, 6.0)], np.float32)
    o = np.array([0.7, 1.0, 0.4], np.float32)
    f = np.array([[1.0, 2.0], [0.25, -0.5], [3.0, 3.0]], np.float32)
    G = np.zeros((2, 24, 32), np.float32)
    G[:, y0, x0] = [1.5, -0.75]
    r = oracle.render(cam, pos, o, f, t_min=1e-4, grad_out=G)
    np.testing.assert_array_equal(r["out"][:, y0, x0], f[1].astype(np.float64))
    assert r["t_final"][y0, x0] == 0.0
    assert r["n_contrib"][y0, x0] == 1  # rank of the front point + 1
    # occluded points: no feature / opacity gradient from the occluded pixel
    np.testing.assert_array_equal(r["grad_feat"][[0, 2]], 0.0)
    np.testing.assert_array_equal(r["grad_opacity"][[0, 2]], 0.0)
    # the front point's feature gradient is its alpha times G
    np.testing.assert_allclose(r["grad_feat"][1], G[:, y0, x0].astype(np.float64), rtol=1e-15)


def test_p3_two_and_three_fragments_by_hand():
    """P3: Eq. (1) expanded by hand with a background, and its derivatives
    (the background term of d/d(alpha_1) is -(1 - a2) f_bg)."""
    cam = cam32()
    x0, y0 = 20, 11
    u, v = x0 + 0.5, y0 + 0.5  # a = b = 0: w = 1 at (x0, y0)
    o1, o2, o3 = 0.375, 0.5, 0.25
    pos = np.array([place(cam, u, v, 3.0), place(cam, u, v, 2.0), place(cam, u, v, 5.0)], np.float32)
    o = np.array([o2, o1, o3], np.float32)  # index 1 is in front, then 0, then 2
    f1, f2, f3 = np.array([1.0, -1.0]), np.array([0.5, 2.0]), np.array([-3.0, 0.25])
    feat = np.stack([f2, f1, f3]).astype(np.float32)
    bg = np.array([0.125, -0.5])
    G = np.zeros((2, 24, 32), np.float32)
    g = np.array([0.75, -1.25])
    G[:, y0, x0] = g
    Gt = np.zeros((24, 32), np.float32)
    gt = 0.5
    Gt[y0, x0] = gt
    r = oracle.render(cam, pos, o, feat, bg=bg, t_min=0.0, grad_out=G, grad_t=Gt)
    F = o1 * f1 + (1 - o1) * o2 * f2 + (1 - o1) * (1 - o2) * o3 * f3 + (1 - o1) * (1 - o2) * (1 - o3) * bg
    Tf = (1 - o1) * (1 - o2) * (1 - o3)
    np.testing.assert_allclose(r["out"][:, y0, x0], F, rtol=1e-14)
    np.testing.assert_allclose(r["t_final"][y0, x0], Tf, rtol=1e-14)
    # dF/d(alpha_k) at this pixel (w = 1 so dF/do = dF/d(alpha))
    dF1 = f1 - o2 * f2 - (1 - o2) * o3 * f3 - (1 - o2) * (1 - o3) * bg
    dF2 = (1 - o1) * (f2 - o3 * f3 - (1 - o3) * bg)
    dF3 = (1 - o1) * (1 - o2) * (f3 - bg)
    dT1, dT2, dT3 = -(1 - o2) * (1 - o3), -(1 - o1) * (1 - o3), -(1 - o1) * (1 - o2)
    exp_go = np.array([g @ dF2 + gt * dT2, g @ dF1 + gt * dT1, g @ dF3 + gt * dT3])
    np.testing.assert_allclose(r["grad_opacity"], exp_go, rtol=1e-13)
    exp_gf = np.stack([(1 - o1) * o2 * g, o1 * g, (1 - o1) * (1 - o2) * o3 * g])
    np.testing.assert_allclose(r["grad_feat"], exp_gf, rtol=1e-14)
    np.testing.assert_allclose(r["grad_bg"], Tf * g, rtol=1e-14)


def test_p4_invariants_random_scene():
    """P4: T_final in [0, 1]; f = 1 and bg = 0 gives F = 1 - T_final (the sum
    telescopes); F is linear in the features."""
    s = tiny_scene(300, 40, 32, channels=2, seed=3)
    r = oracle.render(s.camera, s.pos, s.opacity, s.feat, t_min=0.0)
    assert r["t_final"].min() >= 0.0 and r["t_final"].max() <= 1.0
    ones = np.ones((s.n, 1), np.float32)
    r1 = oracle.render(s.camera, s.pos, s.opacity, ones, t_min=0.0)
    np.testing.assert_allclose(r1["out"][0], 1.0 - r1["t_final"], atol=1e-13)
    f2 = np.random.default_rng(1).standard_normal(s.feat.shape).astype(np.float32)
    ra = oracle.render(s.camera, s.pos, s.opacity, s.feat.astype(np.float64) + 2.0 * f2, t_min=0.0)
    rb = oracle.render(s.camera, s.pos, s.opacity, f2, t_min=0.0)
    np.testing.assert_allclose(ra["out"], r["out"] + 2.0 * rb["out"], atol=1e-12)


def test_p4_transmittance_non_increasing_with_more_fragments():
    """Adding a point behind everything can only lower the transmittance."""
    s = tiny_scene(200, 32, 24, channels=1, seed=5, z_range=(2.0, 3.0))
    r0 = oracle.render(s.camera, s.pos, s.opacity, s.feat, t_min=0.0)
    extra = tiny_scene(50, 32, 24, channels=1, seed=6, z_range=(4.0, 5.0))
    pos = np.concatenate([s.pos, extra.pos])
    op = np.concatenate([s.opacity, extra.opacity])
    ft = np.concatenate([s.feat, extra.feat])
    r1 = oracle.render(s.camera, pos, op, ft, t_min=0.0)
    assert (r1["t_final"] <= r0["t_final"] + 1e-15).all()
    assert (r1["n_contrib"] >= r0["n_contrib"]).all()


def _has_key_ties(cam, pos):
    pr = oracle.project(cam, pos)
    k = pr["key"][pr["visible"]]
    return len(np.unique(k)) != len(k)


def test_p5_input_order_invariance():
    """P5: permuting the input points permutes nothing in the image (scene
    without depth-key ties) and permutes the gradients accordingly."""
    s = tiny_scene(250, 32, 24, channels=3, seed=7)
    assert not _has_key_ties(s.camera, s.pos)
    perm = np.random.default_rng(2).permutation(s.n)
    r = oracle.render(s.camera, s.pos, s.opacity, s.feat, grad_out=s.grad)
    rp = oracle.render(s.camera, s.pos[perm], s.opacity[perm], s.feat[perm], grad_out=s.grad)
    np.testing.assert_array_equal(r["n_contrib"], rp["n_contrib"])
    np.testing.assert_allclose(r["out"], rp["out"], atol=1e-13)
    np.testing.assert_allclose(r["t_final"], rp["t_final"], atol=1e-15)
    np.testing.assert_allclose(r["grad_feat"][perm], rp["grad_feat"], atol=1e-12)
    np.testing.assert_allclose(r["grad_pos"][perm], rp["grad_pos"], atol=1e-10)


@pytest.mark.parametrize("T", [8, 16, 32])
def test_p6_tiles_per_splat(T):
    """P6: a splat fully inside the image touches (1 + [x0 mod T = T-1]) x
    (1 + [y0 mod T = T-1]) tiles; over every sub-tile position the mean is
    (1 + 1/T)^2 (1.27 at T = 8, Sec. 3.2) and the single-tile share (1 - 1/T)^2."""
    W = H = 4 * T
    cam = Camera(width=W, height=H, fx=float(W), fy=float(W), cx=W / 2, cy=H / 2,
                 R=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32), z_near=0.2)
    # one point per (x0, y0) in the interior block [T, 2T) x [T, 2T), offset a = b = 0.25
    xs, ys = np.meshgrid(np.arange(T, 2 * T), np.arange(T, 2 * T))
    u = xs.ravel() + 0.75
    v = ys.ravel() + 0.75
    pos = np.stack([(u - cam.cx) * 2.0 / cam.fx, (v - cam.cy) * 2.0 / cam.fy, np.full(u.size, 2.0)], 1)
    pr = oracle.project(cam, pos.astype(np.float32), tile=T)
    x0 = xs.ravel()
    y0 = ys.ravel()
    expect = (1 + (x0 % T == T - 1)) * (1 + (y0 % T == T - 1))
    np.testing.assert_array_equal(pr["ntiles"], expect)
    assert pr["ntiles"].mean() == (1 + 1 / T) ** 2
    assert (pr["ntiles"] == 1).mean() == (1 - 1 / T) ** 2


def test_p7_tile_list_structure():
    """P7: counts sum to the copies, ranges partition the list, every list is
    ordered by (key, index), and each tile holds exactly the points whose
    footprint rect meets it."""
    s = tiny_scene(400, 50, 37, channels=1, seed=11)
    for T in (8, 16):
        tl = oracle.tile_lists(s.camera, s.pos, tile=T)
        pr = oracle.project(s.camera, s.pos, tile=T)
        assert int(tl["counts"].sum()) == int(pr["ntiles"].sum()) == len(tl["list"])
        rect = pr["rect"]
        for t in range(len(tl["counts"])):
            seg = tl["list"][tl["ranges"][t]:tl["ranges"][t + 1]]
            keys = pr["key"][seg]
            order = np.lexsort((seg, keys))
            np.testing.assert_array_equal(order, np.arange(len(seg)))
            ty, tx = divmod(t, tl["ntx"])
            vis = pr["visible"]
            meets = vis & (rect[:, 2] // T >= tx) & (rect[:, 0] // T <= tx) & \
                (rect[:, 3] // T >= ty) & (rect[:, 1] // T <= ty)
            np.testing.assert_array_equal(np.sort(seg), np.nonzero(meets)[0])


def test_p8_single_gaussian_profile():
    """P8: a Gaussian at a pixel centre gives o f there, o exp(-d^2 / (2
    sigma_eff^2)) f at distance d, zero beyond 3 sigma_eff, sigma_eff^2 = r^2 +
    0.16 (Sec. 3.2, dilation variance 0.16, cut at 3 sigma)."""
    cam = cam32()
    x0, y0 = 15, 11
    r = 1.5
    pos = np.array([place(cam, x0 + 0.5, y0 + 0.5, 2.0)], np.float32)
    o = np.array([0.8], np.float32)
    f = np.array([[2.0]], np.float32)
    res = oracle.render(cam, pos, o, f, radius=np.array([r], np.float32), splat=1, t_min=0.0)
    s2 = np.float32(np.float32(r) * np.float32(r) + np.float32(0.16))
    img = res["out"][0]
    o32 = float(np.float32(0.8))
    assert img[y0, x0] == pytest.approx(o32 * 2.0, rel=1e-15)
    for dx, dy in [(1, 0), (2, 1), (0, 3), (3, 3), (-4, 2)]:
        d2 = dx * dx + dy * dy
        if d2 <= 9.0 * float(s2):
            assert img[y0 + dy, x0 + dx] == pytest.approx(o32 * 2.0 * math.exp(-0.5 * d2 / float(s2)), rel=1e-14)
        else:
            assert img[y0 + dy, x0 + dx] == 0.0
    # nothing beyond 3 sigma_eff
    yy, xx = np.mgrid[0:24, 0:32]
    d2 = (xx - x0) ** 2 + (yy - y0) ** 2
    assert (img[d2 > 9.0 * float(s2) * (1 + 1e-6)] == 0).all()


def test_p11_zero_weight_fragments_get_position_gradients():
    """P11 (Appendix A): a point exactly on a pixel centre has zero-weight
    fragments at its right and lower neighbours; they are blended and carry
    the position gradient.  Right-derivative finite difference agrees."""
    cam = cam32()
    x0, y0 = 12, 8
    Z = 2.0
    pos = np.array([place(cam, x0 + 0.5, y0 + 0.5, Z), place(cam, x0 + 1.75, y0 + 0.5, 4.0)], np.float32)
    o = np.array([0.5, 0.75], np.float32)
    f = np.array([[1.0, -0.5], [0.25, 2.0]], np.float32)
    G = np.zeros((2, 24, 32), np.float32)
    G[:, y0, x0 + 1] = [1.0, 0.5]  # only the zero-weight neighbour carries gradient
    r = oracle.render(cam, pos, o, f, t_min=0.0, grad_out=G)
    gu = r["grad_uv"][0, 0]
    assert gu != 0.0
    h = 2.0 ** -12  # exact shift of u in FP32
    pos_h = pos.copy()
    pos_h[0, 0] += np.float32(h * Z / cam.fx)
    assert oracle.project(cam, pos_h)["uv"][0, 0] == np.float32(x0 + 0.5 + h)
    loss = lambda rr: float((G.astype(np.float64) * rr["out"]).sum())
    fd = (loss(oracle.render(cam, pos_h, o, f, t_min=0.0)) - loss(r)) / h
    # loss is bilinear in a; the right difference differs by O(h)
    assert gu == pytest.approx(fd, rel=2e-3)


def test_culled_points_and_nan():
    """Points behind the near plane, NaN positions and footprints outside the
    image are culled and get zero gradients."""
    cam = cam32()
    pos = np.array([[0.0, 0.0, 0.1], [np.nan, 0.0, 2.0], [100.0, 0.0, 2.0], [0.0, 0.0, 2.0]], np.float32)
    o = np.full(4, 0.5, np.float32)
    f = np.ones((4, 1), np.float32)
    G = np.ones((1, 24, 32), np.float32)
    pr = oracle.project(cam, pos)
    np.testing.assert_array_equal(pr["visible"], [False, False, False, True])
    np.testing.assert_array_equal(pr["ntiles"][:3], 0)
    r = oracle.render(cam, pos, o, f, grad_out=G)
    np.testing.assert_array_equal(r["grad_feat"][:3], 0.0)
    np.testing.assert_array_equal(r["grad_pos"][:3], 0.0)


def test_image_border_footprints():
    """Splats straddling the image border keep only in-image fragments."""
    cam = make_camera(16, 8, 8.0)
    pos = np.array([place(cam, -0.25, 3.75, 2.0), place(cam, 16.25, 8.25, 2.0)], np.float32)
    pr = oracle.project(cam, pos, tile=8)
    assert pr["visible"].all()
    np.testing.assert_array_equal(pr["rect"][0], [0, 3, 0, 4])
    np.testing.assert_array_equal(pr["rect"][1], [15, 7, 15, 7])
    r = oracle.render(cam, pos, np.array([1.0, 1.0], np.float32), np.ones((2, 1), np.float32), t_min=0.0)
    assert r["n_contrib"].sum() == 3
