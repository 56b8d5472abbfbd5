"""GPU parity of the Gaussian splats' forward and backward passes against the
oracle: world-space Gaussians projected with the EWA approximation (Sec. 3.2
"Rendering Points as Small Gaussians": isotropic world-space Gaussians, the
affine approximation of the perspective projection, dilation 0.16, cut at
3 sigma) and screen-space Gaussians of a per-point radius.  Binning is
bit-exact; images and every gradient (features, opacities, image
positions, the depth gradient through the projected covariance, world
positions, background) within the tolerance of Eq. (1)/(2) in FP32.

Pixels whose FP64 transmittance sits on the t_min threshold (the oracle
flags them) may keep one fragment more or less in FP32: they are excluded
from the forward comparison and their upstream gradients are set to zero
on both sides, so that they contribute nothing to any gradient."""
import numpy as np
import pytest
import torch

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle  # noqa: E402
import paper_2508_19140_amd as inpc  # noqa: E402
from gpu_helpers import (  # noqa: E402
    assert_backward, assert_binning_exact, assert_close, assert_forward, mask_flagged,
    oracle_kw, run_gpu, run_oracle, settings_opts)
from scenes import multi_view_scenes, tiny_scene  # noqa: E402

DEV = "cuda:0"


def _parity(sc, st, bg=None):
    ok = mask_flagged(sc, st, bg=bg)
    assert ok.mean() > 0.99
    g = run_gpu(sc, st, bg=bg)
    proj, tl, rr = run_oracle(sc, st, bg=bg)
    assert_binning_exact(g, proj, tl)
    assert_forward(g, rr, flags_ok=ok)
    assert_backward(g, rr, sc.grad)
    return g, rr


@pytest.mark.parametrize("tile", [8, 16])
@pytest.mark.parametrize("t_min", [0.0, 1e-4])
def test_world_space_gaussians(tile, t_min):
    """Points from just past the near plane to 3 m: projected standard
    deviations from a fraction of a pixel to several pixels, footprints over
    up to 5 x 5 tiles of 8 px, a ragged last tile row and column."""
    print(f"case tile={tile} t_min={t_min}", flush=True)
    sc = tiny_scene(3000, 100, 70, channels=4, seed=31, z_range=(0.25, 3.0), with_grad_t=True)
    st = settings_opts(splat="ewa", tile=tile, t_min=t_min, ewa_sigma=0.02)
    g, rr = _parity(sc, st, bg=np.array([0.5, -1.0, 2.0, 0.25]))
    assert np.abs(g["grad_z"]).max() > 0  # the depth gradient is exercised
    split = int((g["ntiles"] > 1).sum())
    print(f"  points over several tiles: {split}, over more than four: "
          f"{int((g['ntiles'] > 4).sum())}", flush=True)
    assert split > 300  # large footprints: many points split over tiles


def test_world_space_default_sigma_and_channels():
    """The paper's default sigma (5 px at the near plane through the image
    centre) and channel counts that leave the kernels' row padding partly
    unused (3 and 9 channels); a per-pixel background image."""
    for C, seed in ((3, 32), (9, 33)):
        print(f"case C={C} seed={seed}", flush=True)
        sc = tiny_scene(2000, 64, 48, channels=C, seed=seed, z_range=(0.21, 2.0))
        st = settings_opts(splat="ewa", tile=8)
        bgi = np.random.default_rng(seed).standard_normal((C, 48, 64)).astype(np.float32)
        _parity(sc, st, bg=bgi)


@pytest.mark.parametrize("tile", [8, 16])
def test_screen_space_gaussians(tile):
    print(f"case tile={tile}", flush=True)
    sc = tiny_scene(4000, 96, 64, channels=4, seed=34, radius_range=(0.3, 4.0),
                    with_grad_t=True)
    st = settings_opts(splat="gaussian", tile=tile, max_radius=4.0)
    _parity(sc, st, bg=np.array([1.0, 0.0, -1.0, 0.5]))


def test_empty_and_culled_world_space():
    st = settings_opts(splat="ewa", tile=8, ewa_sigma=0.02)
    sc = tiny_scene(0, 16, 16, channels=2, seed=0)
    g = run_gpu(sc, st)
    assert (g["out"] == 0).all() and (g["t_final"] == 1).all() and (g["n_contrib"] == 0).all()
    sc = tiny_scene(60, 16, 16, channels=2, seed=1)
    sc.pos[:, 2] = -1.0  # behind the camera
    sc.pos[:3] = np.nan
    g = run_gpu(sc, st)
    assert (g["ntiles"] == 0).all() and (g["out"] == 0).all()
    for k in ("grad_feat", "grad_opacity", "grad_uv", "grad_z", "grad_pos"):
        assert (g[k] == 0).all(), k


def test_rasterize_autograd_world_space():
    """inpc.rasterize with world-space splats: torch autograd gradients of
    positions, opacities, features and the background against the oracle."""
    sc = tiny_scene(2500, 80, 60, channels=4, seed=35, z_range=(0.3, 3.0), with_grad_t=True)
    st = inpc.RasterSettings(splat="ewa", tile=8, ewa_sigma=0.015)
    bg = np.array([0.1, 0.2, -0.3, 0.4])
    ok = mask_flagged(sc, st, bg=bg)
    t = lambda a: torch.from_numpy(np.asarray(a, np.float32)).to(DEV)
    pos, op, ft, bgt = (t(a).requires_grad_(True) for a in (sc.pos, sc.opacity, sc.feat, bg))
    out, tf, nc = inpc.rasterize(pos, op, ft, sc.camera, bg=bgt, settings=st)
    ((out * t(sc.grad)).sum() + (tf * t(sc.grad_t)).sum()).backward()
    torch.cuda.synchronize()
    rr = oracle.render(sc.camera, sc.pos, sc.opacity, sc.feat, bg=bg, t_min=st.t_min,
                       grad_out=sc.grad, grad_t=sc.grad_t, **oracle_kw(sc, st))
    g = dict(out=out.detach().cpu().numpy(), t_final=tf.detach().cpu().numpy(),
             n_contrib=nc.cpu().numpy().view(np.uint32))
    assert_forward(g, rr, flags_ok=ok)
    assert_close("grad_pos", pos.grad.cpu().numpy(), rr["grad_pos"], rr["grad_pos_abs"])
    assert_close("grad_opacity", op.grad.cpu().numpy(), rr["grad_opacity"],
                 rr["grad_opacity_abs"])
    assert_close("grad_feat", ft.grad.cpu().numpy(), rr["grad_feat"], rr["grad_feat_abs"])
    mag = np.abs(rr["t_final"][None] * sc.grad.astype(np.float64)).sum(axis=(1, 2))
    assert_close("grad_bg", bgt.grad.cpu().numpy(), rr["grad_bg"], mag)


def test_batched_world_space(tmp_path):
    """The batched pass (one blend launch per direction over every view's
    tiles) with world-space splats: one sigma and one workspace bound for
    all views; every view's outputs and gradients against the oracle."""
    scenes = multi_view_scenes(3, seed=36, n_lo=4000, n_hi=9000, channels=4,
                               resolutions=((96, 64), (80, 48)))
    st = inpc.RasterSettings(splat="ewa", tile=8, t_min=0.0, ewa_sigma=0.03)
    t = lambda a: torch.from_numpy(a).to(DEV)
    views = [inpc.ViewInputs(pos=t(s.pos), opacity=t(s.opacity), feat=t(s.feat),
                             camera=s.camera, grad_out=t(s.grad)) for s in scenes]
    br = inpc.BatchedRasterizer(views, settings=st, autotune=False,
                                cache_path=str(tmp_path / "c.json"))
    br.step()
    torch.cuda.synchronize()
    for k, (sc, o) in enumerate(zip(scenes, br.outputs())):
        print(f"  view {k}: n={sc.pos.shape[0]} {sc.camera.width}x{sc.camera.height}",
              flush=True)
        g = {key: v.cpu().numpy() for key, v in o.items()}
        g["n_contrib"] = g["n_contrib"].view(np.uint32)
        _, _, rr = run_oracle(sc, st)
        assert_forward(g, rr)
        assert_backward(g, rr, sc.grad)
