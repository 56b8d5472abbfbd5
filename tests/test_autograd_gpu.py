"""The autograd entry point (rasterize + .backward) on the GPU: its gradients
against the oracle's, and against central finite differences of the GPU
forward pass itself.

The finite differences run in FP32 through the same kernels, so the step h
and the tolerance are chosen from the FP32 noise of the loss: with
|L| ~ 10 and eps = 6e-8 the rounding noise of L is ~1e-6, which with h =
1e-2 is ~1e-4 in the difference quotient.  Features enter linearly and
opacities polynomially (central differences are exact up to O(h^2)); point
positions move the bilinear weights, which are smooth only away from pixel
centres, so only points whose sub-pixel offsets stay clear of the kinks by
far more than the step are perturbed.  Every fragment is blended
(t_min = 0), so the loss has no termination jumps.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import paper_2508_19140_amd as inpc
from scenes import tiny_scene

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"


def _setup(seed=5, n=300, W=40, H=30, C=3):
    sc = tiny_scene(n, W, H, channels=C, seed=seed, with_grad_t=True)
    bg = np.array([0.3, -0.7, 1.1][:C], np.float32)
    st = inpc.RasterSettings(t_min=0.0, keep_lists=False)
    return sc, bg, st


def _loss_and_grads(sc, bg, st, pos=None, opacity=None, feat=None, grads=True):
    pos = torch.tensor(sc.pos if pos is None else pos, device=DEV, requires_grad=grads)
    op = torch.tensor(sc.opacity if opacity is None else opacity, device=DEV, requires_grad=grads)
    ft = torch.tensor(sc.feat if feat is None else feat, device=DEV, requires_grad=grads)
    bgt = torch.tensor(bg, device=DEV, requires_grad=grads)
    out, tf, _ = inpc.rasterize(pos, op, ft, sc.camera, bg=bgt, settings=st)
    G = torch.from_numpy(sc.grad).to(DEV)
    GT = torch.from_numpy(sc.grad_t).to(DEV)
    loss = (out.double() * G.double()).sum() + (tf.double() * GT.double()).sum()
    if not grads:
        return float(loss)
    loss.backward()
    return float(loss), {k: t.grad.cpu().numpy().astype(np.float64)
                         for k, t in (("pos", pos), ("opacity", op), ("feat", ft), ("bg", bgt))}


@pytest.mark.parametrize("keep_lists", [False, True])
def test_autograd_matches_oracle(keep_lists):
    """Lists recomputed in the backward or kept from the forward; either way
    the backward's zero fill runs on a side stream beside the sort (or
    before the blend) and the blend waits for it."""
    sc, bg, st = _setup()
    st = dataclasses.replace(st, keep_lists=keep_lists)
    _, g = _loss_and_grads(sc, bg, st)
    rr = oracle.render(sc.camera, sc.pos, sc.opacity, sc.feat, bg=bg, t_min=0.0,
                       grad_out=sc.grad, grad_t=sc.grad_t)
    for k, ok in (("feat", "grad_feat"), ("opacity", "grad_opacity"), ("pos", "grad_pos")):
        _, stt = oracle.within_tolerance(g[k], rr[ok], rr[ok + "_abs"])
        assert stt["n_bad"] == 0, (k, stt)
    np.testing.assert_allclose(g["bg"], rr["grad_bg"], rtol=1e-5, atol=1e-4)


def _fd(sc, bg, st, field, i, j, h):
    base = {"pos": sc.pos, "opacity": sc.opacity, "feat": sc.feat}[field]
    vals = []
    for sgn in (1.0, -1.0):
        arr = base.copy()
        if arr.ndim == 1:
            arr[i] = np.float32(arr[i] + sgn * h)
        else:
            arr[i, j] = np.float32(arr[i, j] + sgn * h)
        vals.append(_loss_and_grads(sc, bg, st, grads=False, **{field: arr}))
    return (vals[0] - vals[1]) / (2 * h)


def test_autograd_matches_finite_differences():
    sc, bg, st = _setup()
    _, g = _loss_and_grads(sc, bg, st)
    proj = oracle.project(sc.camera, sc.pos)
    rng = np.random.default_rng(0)
    checked = 0
    # features and opacities of points that are visible
    vis = np.flatnonzero(proj["visible"])
    for i in rng.choice(vis, 12, replace=False):
        c = int(rng.integers(3))
        fd = _fd(sc, bg, st, "feat", i, c, 1e-2)
        assert abs(fd - g["feat"][i, c]) <= 1e-3 + 1e-2 * abs(fd), (i, c, fd, g["feat"][i, c])
        fd = _fd(sc, bg, st, "opacity", i, None, 1e-2)
        assert abs(fd - g["opacity"][i]) <= 1e-3 + 1e-2 * abs(fd), (i, fd, g["opacity"][i])
        checked += 1
    # positions: sub-pixel offsets far from the bilinear kinks
    u, v = proj["uv"][:, 0] - 0.5, proj["uv"][:, 1] - 0.5
    fa, fb = u - np.floor(u), v - np.floor(v)
    safe = vis[(np.minimum(fa[vis], 1 - fa[vis]) > 0.2) & (np.minimum(fb[vis], 1 - fb[vis]) > 0.2)]
    for i in rng.choice(safe, 8, replace=False):
        for j in range(3):
            fd = _fd(sc, bg, st, "pos", i, j, 5e-3)
            assert abs(fd - g["pos"][i, j]) <= 2e-3 + 2e-2 * abs(fd), (i, j, fd, g["pos"][i, j])
        checked += 1
    assert checked == 20
