"""Many views in one graph launch: the autotuned, graph-captured batch gives
the same result as every view run on its own, on every replay, and matches
the oracle per view.  Forward outputs are deterministic and compared bit for
bit; gradients of points split over several tiles are summed with float
atomics in arrival order, so they are compared to rounding."""
import numpy as np
import pytest
import torch

import paper_2508_19140_amd as inpc
from gpu_helpers import assert_backward, assert_forward, run_oracle, settings_opts
from scenes import multi_view_scenes

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"
RES = [(160, 90), (128, 96), (200, 112)]


def _views(scenes):
    return [inpc.ViewInputs(pos=torch.from_numpy(s.pos).to(DEV),
                            opacity=torch.from_numpy(s.opacity).to(DEV),
                            feat=torch.from_numpy(s.feat).to(DEV), camera=s.camera,
                            grad_out=torch.from_numpy(s.grad).to(DEV)) for s in scenes]


def _snapshot(mv):
    return [{k: t.cpu().numpy().copy() for k, t in o.items()} for o in mv.outputs()]


def test_graph_batch_matches_single_views_and_oracle():
    scenes = multi_view_scenes(4, n_lo=20_000, n_hi=80_000, channels=4, resolutions=RES)
    views = _views(scenes)
    mv = inpc.MultiViewRasterizer(views, tiles=(8, 16), bin_points=(0, 1024), reps=1)
    assert len(mv.choice) == 4 and all(t in (8, 16) for t, _ in mv.choice)
    # reference: each view alone, eager, with its tuned settings
    mv.run_eager()
    torch.cuda.synchronize()
    ref = _snapshot(mv)
    for o in mv.outputs():
        for t in o.values():
            t.zero_()
    mv.capture()
    for rep in range(3):
        mv.replay()
        torch.cuda.synchronize()
        got = _snapshot(mv)
        for v, (g, r) in enumerate(zip(got, ref)):
            for k in r:
                if k.startswith("grad"):
                    # at most four shares per element, added in any order
                    tol = 1e-6 * float(np.abs(r[k]).max(initial=0.0)) + 1e-7
                    np.testing.assert_allclose(g[k], r[k], rtol=1e-5, atol=tol,
                                               err_msg=f"replay {rep} view {v} {k}")
                else:
                    np.testing.assert_array_equal(g[k], r[k], err_msg=f"replay {rep} view {v} {k}")
        # eager work between replays
        torch.ones(1 << 20, device=DEV).sum().item()
    # per-view parity with the oracle
    for v, (sc, (tile, _)) in enumerate(zip(scenes, mv.choice)):
        st = settings_opts(tile=tile)
        proj, tl, rr = run_oracle(sc, st)
        g = {k: x for k, x in got[v].items()}
        g["n_contrib"] = g["n_contrib"].view(np.uint32)
        assert_forward(g, rr)
        assert_backward(g, rr, sc.grad)
