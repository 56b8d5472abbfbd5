"""Helpers for the GPU parity tests: run the HIP path step by step through
the C ABI binding and compare against the CPU oracle."""
import numpy as np
import torch

import oracle
import paper_2508_19140_amd as inpc
from paper_2508_19140_amd import _lib as L
from paper_2508_19140_amd import raster

DEV = "cuda:0"


def settings_opts(splat="bilinear", tile=8, t_min=1e-4, max_radius=3.0, ewa_sigma=0.0):
    return inpc.RasterSettings(splat=splat, tile=tile, t_min=t_min, max_radius=max_radius,
                               ewa_sigma=ewa_sigma)


def oracle_kw(scene, settings):
    """The oracle's splat options for these rasterizer settings (the
    world-space sigma as the FP32 value the library receives)."""
    splat = {"bilinear": oracle.SPLAT_BILINEAR, "gaussian": oracle.SPLAT_GAUSSIAN,
             "ewa": oracle.SPLAT_EWA}[settings.splat]
    sigma = 0.0
    if settings.splat == "ewa":
        sigma = float(np.float32(settings.sigma(inpc.camera_struct(scene.camera))))
    return dict(splat=splat, tile=settings.tile, ewa_sigma=sigma)


def run_gpu(scene, settings, bg=None, feat_dtype=torch.float32, backward=True, feat=None,
            ring_counts=None):
    """All steps on the GPU; returns numpy copies of every intermediate
    (ring_counts: the scene's points are a ring of that many live points per
    slot, projected with inpc_project_ring)."""
    cam = inpc.camera_struct(scene.camera)
    opts = settings.opts(bg_per_pixel=bg is not None and np.ndim(bg) == 3, cam=cam)
    pos = torch.from_numpy(scene.pos).to(DEV)
    op = torch.from_numpy(scene.opacity).to(DEV)
    ft = torch.from_numpy(scene.feat if feat is None else feat).to(DEV).to(feat_dtype)
    rad = None if scene.radius is None else torch.from_numpy(scene.radius).to(DEV)
    bgt = None if bg is None else torch.as_tensor(bg, dtype=torch.float32, device=DEV)
    ws = inpc.Workspace().get(pos.shape[0], cam, opts, DEV)
    b = inpc.project_bin_sort(pos, op, cam, opts, ws, rad if settings.splat == "gaussian" else None,
                              ring_counts)
    out, tf, nc, state = inpc.blend_forward(b, ft, cam, opts, ws, bgt)
    inpc.check_capacity(ws)
    proj = b.proj.cpu().numpy()
    r = dict(uv=np.ascontiguousarray(proj[:, :2]), proj=proj, key=b.key.cpu().numpy().view(np.uint32),
             ntiles=b.ntiles.cpu().numpy().view(np.uint32),
             ranges=b.ranges.cpu().numpy().view(np.uint32), list=b.list.cpu().numpy().view(np.uint32),
             out=out.cpu().numpy(), t_final=tf.cpu().numpy(), n_contrib=nc.cpu().numpy().view(np.uint32),
             order=b.order.cpu().numpy().view(np.uint32), tile=settings.tile,
             W=cam.width, H=cam.height, opacity=scene.opacity,
             radius=(scene.radius if settings.splat == "gaussian" else
                     None if settings.splat == "ewa" else np.zeros_like(scene.opacity)),
             lpos=b.lpos.cpu().numpy().view(np.uint16) if settings.splat == "bilinear" else None)
    if backward and scene.grad is not None:
        g = torch.from_numpy(scene.grad).to(DEV)
        gt = None if scene.grad_t is None else torch.from_numpy(scene.grad_t).to(DEV)
        # outputs and scratch start as NaN: every element the backward does
        # not write shows up against the oracle
        n, C = ft.shape
        nan = lambda *s: torch.full(s, float("nan"), dtype=torch.float32, device=DEV)
        scratch = torch.full((raster.backward_scratch_bytes(n, C, cam, opts),), 0xFF,
                             dtype=torch.uint8, device=DEV)
        gr = inpc.blend_backward(b, ft, cam, opts, ws, tf, state, g, gt, bgt, scratch=scratch,
                                 outputs=(nan(n, C), nan(n), nan(n, 2)))
        gpos = inpc.project_backward(pos, b, cam, gr.uv, gr.z)
        torch.cuda.synchronize()
        r.update(grad_feat=gr.feat.cpu().numpy(), grad_opacity=gr.opacity.cpu().numpy(),
                 grad_uv=gr.uv.cpu().numpy(), grad_pos=gpos.cpu().numpy(),
                 grad_z=None if gr.z is None else gr.z.cpu().numpy(),
                 grad_bg=None if gr.bg is None else gr.bg.cpu().numpy())
    return r


def run_oracle(scene, settings, bg=None, feat=None, backward=True):
    kw = oracle_kw(scene, settings)
    f = scene.feat if feat is None else feat
    rad = scene.radius if settings.splat == "gaussian" else None
    proj = oracle.project(scene.camera, scene.pos, rad, **kw)
    tl = oracle.tile_lists(scene.camera, scene.pos, rad, **kw)
    go = scene.grad if backward else None
    rr = oracle.render(scene.camera, scene.pos, scene.opacity, f, radius=rad, bg=bg,
                       t_min=settings.t_min, grad_out=go,
                       grad_t=scene.grad_t if go is not None else None, **kw)
    return proj, tl, rr


def mask_flagged(scene, settings, bg=None):
    """Zero the upstream gradients at the pixels whose FP64 transmittance
    sits on the t_min threshold (Gaussians; the oracle flags them): there the
    GPU's FP32 termination may keep one fragment more or less, and with
    G = G_T = 0 such a pixel contributes nothing to any gradient on either
    side.  Returns the forward's keep-mask."""
    _, _, rr = run_oracle(scene, settings, bg=bg, backward=False)
    ok = rr["flags"] == 0
    if scene.grad is not None:
        scene.grad = np.where(ok[None], scene.grad, 0.0).astype(np.float32)
    if scene.grad_t is not None:
        scene.grad_t = np.where(ok, scene.grad_t, 0.0).astype(np.float32)
    return ok


def assert_binning_exact(g, proj, tl):
    vis = proj["visible"]
    np.testing.assert_array_equal(g["ntiles"] > 0, vis)
    np.testing.assert_array_equal(g["ntiles"], proj["ntiles"])
    np.testing.assert_array_equal(g["uv"][vis].view(np.uint32), proj["uv"][vis].view(np.uint32))
    if g.get("opacity") is not None:  # the projection record carries opacity and radius
        np.testing.assert_array_equal(g["proj"][:, 2], g["opacity"])
        if g.get("radius") is not None:
            np.testing.assert_array_equal(g["proj"][:, 3], g["radius"])
        else:  # world-space Gaussians: the camera-space depth, whose bits are the key
            np.testing.assert_array_equal(g["proj"][vis, 3].view(np.uint32), g["key"][vis])
    np.testing.assert_array_equal(g["key"][vis], proj["key"][vis])
    np.testing.assert_array_equal(g["ranges"].astype(np.int64), tl["ranges"])
    M = int(tl["ranges"][-1])
    np.testing.assert_array_equal(g["list"][:M], tl["list"])
    # blend order: decreasing power-of-two class of the longest copy count in
    # the tile's aligned quad (tile indices 4k .. 4k+3), then tile index
    counts = np.diff(tl["ranges"])
    nq = (len(counts) + 3) // 4
    quad = np.zeros(nq * 4, np.int64)
    quad[:len(counts)] = counts
    qmax = np.repeat(quad.reshape(nq, 4).max(axis=1), 4)[:len(counts)]
    klass = np.array([32 - int(c).bit_length() for c in qmax], np.int64)
    np.testing.assert_array_equal(g["order"][:len(counts)], np.lexsort((np.arange(len(counts)), klass)))
    if g.get("lpos") is not None:
        assert_lpos(g, proj, tl)


def assert_lpos(g, proj, tl):
    """Every list entry's tile-local 2x2 position covers exactly the in-image
    pixels of its tile that the oracle's candidate rect covers."""
    T, ntx = g["tile"], tl["ntx"]
    counts = np.diff(tl["ranges"])
    M = int(tl["ranges"][-1])
    if M == 0:
        return
    tile = np.repeat(np.arange(len(counts)), counts)
    tx0, ty0 = (tile % ntx) * T, (tile // ntx) * T
    lp = g["lpos"][:M].astype(np.int64)
    rect = proj["rect"][tl["list"]].astype(np.int64)
    for ax, (base, lo, size) in enumerate(((tx0, lp & 0xff, g["W"]), (ty0, lp >> 8, g["H"]))):
        a = base + lo - 1
        got_lo = np.maximum(np.maximum(a, base), 0)
        got_hi = np.minimum(np.minimum(a + 1, base + T - 1), size - 1)
        ref_lo = np.maximum(rect[:, ax], base)
        ref_hi = np.minimum(rect[:, ax + 2], base + T - 1)
        np.testing.assert_array_equal(got_lo, ref_lo)
        np.testing.assert_array_equal(got_hi, ref_hi)


def assert_close(name, gpu, ref, ref_abs, rel=1e-5, abs_=1e-6, mask=None):
    """Element-wise tolerance check (oracle.within_tolerance), in chunks so
    that full-size outputs (hundreds of millions of elements) stay within a
    few GB of host memory.  Prints the statistics, including how many
    elements would fail the plain test against |oracle| alone."""
    gpu, ref, ref_abs = np.asarray(gpu), np.asarray(ref), np.asarray(ref_abs)
    if mask is not None:
        gpu, ref, ref_abs = gpu[..., mask], ref[..., mask], ref_abs[..., mask]
    gpu, ref, ref_abs = gpu.reshape(-1), ref.reshape(-1), ref_abs.reshape(-1)
    st = dict(max_abs=0.0, max_rel=0.0, sq=0.0, n_bad=0, n_plain_fail=0, max_plain_excess=0.0)
    step = 1 << 23
    for k in range(0, max(gpu.size, 1), step):
        sl = slice(k, k + step)
        _, s = oracle.within_tolerance(gpu[sl].astype(np.float64), ref[sl].astype(np.float64),
                                       ref_abs[sl].astype(np.float64), rel=rel, abs_=abs_)
        for key in ("max_abs", "max_rel", "max_plain_excess"):
            st[key] = max(st[key], s[key])
        for key in ("n_bad", "n_plain_fail"):
            st[key] += s[key]
        st["sq"] += s["rms"] ** 2 * gpu[sl].size
    st["rms"] = float(np.sqrt(st.pop("sq") / max(gpu.size, 1)))
    st["n"] = int(gpu.size)
    print(f"  {name}: {st}", flush=True)
    assert st["n_bad"] == 0, f"{name}: {st}"
    return st


def assert_forward(g, rr, flags_ok=None):
    mask = None if flags_ok is None else flags_ok
    if mask is None:
        np.testing.assert_array_equal(g["n_contrib"], rr["n_contrib"])
    else:
        np.testing.assert_array_equal(g["n_contrib"][mask], rr["n_contrib"][mask])
    s1 = assert_close("out", g["out"], rr["out"], rr["out_abs"], mask=mask)
    s2 = assert_close("t_final", g["t_final"], rr["t_final"], rr["t_final"], mask=mask)
    return dict(out=s1, t_final=s2)


def assert_backward(g, rr, grad_out=None):
    st = {}
    keys = ["grad_feat", "grad_opacity", "grad_uv", "grad_pos"]
    if g.get("grad_z") is not None:
        keys.append("grad_z")
    for k in keys:
        st[k] = assert_close(k, g[k], rr[k], rr[k + "_abs"])
    if rr.get("grad_bg") is not None:
        # sum over pixels of T_final G: bounded by the sum of the magnitudes
        # (a per-pixel background: T_final G itself)
        mag = np.abs(rr["t_final"][None] * np.asarray(grad_out, np.float64))
        if np.ndim(rr["grad_bg"]) == 1:
            mag = mag.sum(axis=(1, 2))
        st["grad_bg"] = assert_close("grad_bg", g["grad_bg"], rr["grad_bg"], mag)
    return st
