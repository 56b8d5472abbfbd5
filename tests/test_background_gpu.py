"""GPU parity of the environment-map background (Sec. 3.2 "Faster Background
Model Evaluation"): view directions, the map sampled along them, the sampled
image composited behind the points by the blend (F += T_final f_bg), and the
backward through all of it (points and map), against the oracle."""
import math

import numpy as np
import pytest
import torch

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle  # noqa: E402
from oracle import envmap  # noqa: E402
from scenes import SceneSpec, make_scene, ring_camera  # noqa: E402

DEV = "cuda:0"


def smooth_env(Hm, Wm, C, seed):
    """A low-frequency map like a distilled sky: a few spherical waves."""
    rng = np.random.default_rng(seed)
    th = (np.arange(Hm) + 0.5) / Hm * math.pi
    ph = (np.arange(Wm) + 0.5) / Wm * 2 * math.pi - math.pi
    T, Ph = np.meshgrid(th, ph, indexing="ij")
    env = np.zeros((Hm, Wm, C))
    for c in range(C):
        a, b, d = rng.uniform(0.2, 1.0, 3)
        env[..., c] = a * np.cos(T) + b * np.sin(T) * np.cos(Ph + d) + 0.3 * c
    return env.astype(np.float32)


def test_view_dirs_and_envmap_sample():
    import paper_2508_19140_amd as inpc
    cam = ring_camera(2, 8, 320, 180)
    dirs = inpc.view_directions(cam, DEV)
    np.testing.assert_allclose(dirs.cpu().numpy(), envmap.view_dirs(cam), atol=5e-7)
    env = smooth_env(256, 512, 4, 0)
    bg = inpc.envmap_background(torch.from_numpy(env).to(DEV), cam, dirs)
    ref = envmap.sample(cam, env.astype(np.float64))
    err = np.abs(bg.cpu().numpy() - ref)
    print("  bg image max abs error", err.max(), flush=True)
    assert err.max() < 2e-5


def test_envmap_background_forward_backward():
    import paper_2508_19140_amd as inpc
    sc = make_scene(SceneSpec(n=60_000, s=4.0, z_lo=2.0, z_hi=20.0, width=240, height=160,
                              channels=4, feat_dist="normal", opacity_range=(0.05, 0.95),
                              with_grad=True, seed=4))
    cam = sc.camera
    Hm, Wm = 64, 128
    env = smooth_env(Hm, Wm, 4, 1)
    t = lambda a: torch.from_numpy(a).to(DEV)
    envt = t(env).requires_grad_(True)
    pos, op = t(sc.pos).requires_grad_(True), t(sc.opacity).requires_grad_(True)
    ft = t(sc.feat).requires_grad_(True)
    bg = inpc.envmap_background(envt, cam)
    out, tf, nc = inpc.rasterize(pos, op, ft, cam, bg=bg)
    (out * t(sc.grad)).sum().backward()
    torch.cuda.synchronize()
    bg_ref = envmap.sample(cam, env.astype(np.float64))
    rr = oracle.render(cam, sc.pos, sc.opacity, sc.feat, bg=bg_ref, grad_out=sc.grad)
    from gpu_helpers import assert_close
    assert_close("out", out.detach().cpu().numpy(), rr["out"], rr["out_abs"])
    assert_close("t_final", tf.detach().cpu().numpy(), rr["t_final"], rr["t_final"])
    np.testing.assert_array_equal(nc.cpu().numpy(), rr["n_contrib"].astype(np.int32))
    for name, g in (("grad_feat", ft.grad), ("grad_opacity", op.grad), ("grad_pos", pos.grad)):
        assert_close(name, g.cpu().numpy(), rr[name], rr[name + "_abs"])
    genv_ref = envmap.sample_backward(cam, rr["grad_bg"], Hm, Wm)
    genv_abs = envmap.sample_backward(cam, np.abs(rr["grad_bg"]), Hm, Wm)
    # The map coordinates come from FP32 atan2 / acos on the GPU and FP64 in
    # the oracle; they differ by at most DELTA texels (a few ulps of the
    # angle, times Wm / 2 pi or Hm / pi, here below 3e-5; 1e-4 with margin).
    # The sampled values are continuous in the coordinates, but a pixel
    # whose coordinate lies within DELTA of a texel centre line hands its
    # gradient to a different texel pair on the two sides, moving at most
    # DELTA |G T_final| between texels one apart.  So each texel's gradient
    # may differ by DELTA times the gradient magnitude landing on its 3x3
    # neighbourhood, on top of the usual summation bound.
    DELTA = 1e-4
    nb = np.zeros_like(genv_abs)
    for dy in (-1, 0, 1):
        rows = np.clip(np.arange(Hm) + dy, 0, Hm - 1)
        for dx in (-1, 0, 1):
            nb += genv_abs[rows][:, (np.arange(Wm) + dx) % Wm]
    err = np.abs(envt.grad.cpu().numpy().astype(np.float64) - genv_ref)
    tol = 1e-6 + 1e-5 * np.maximum(np.abs(genv_ref), genv_abs) + DELTA * nb
    print(f"  grad_env: max abs {err.max():.3e}, worst err/tol {(err / tol).max():.3f}",
          flush=True)
    assert (err <= tol).all()
