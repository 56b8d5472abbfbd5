"""Benchmark: forward + backward rasterization of 2^23 points at 1920x1080.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--config H|C2|C3|C5] [--dtype f32|bf16|f16] [--tile 8|16]
                    [--errors] [--profile-steps S]

One step is one training pass of the whole rasterizer on one view, exactly
what rasterize(...) followed by .backward() runs:
  forward : project -> bin -> sort -> blend forward
  backward: project -> bin -> sort (lists recomputed, not stored)
            -> blend backward -> project backward
(--config C3, Gaussian splats, is forward only: the paper uses Gaussians at
inference.)  Inputs (a seeded synthetic scene shaped like the paper's
view-specific clouds) are resident in HBM before the timed region.  Every
entry point is bracketed by HIP events on the stream it runs on, inside the
timed region; the entry point with the largest share of the step is the
roofline line.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

METRIC = "points rasterized/s fwd+bwd at 1080p (8M pts); achieved HBM GB/s vs roofline"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="H", choices=["H", "C2", "C3", "C5"])
    ap.add_argument("--tile", type=int, default=8, choices=[8, 16])
    ap.add_argument("--dtype", default=None, choices=["f32", "bf16", "f16"],
                    help="feature storage type (default: bf16 for C5, f32 otherwise)")
    ap.add_argument("--keep-lists", action="store_true",
                    help="backward reuses the forward's tile lists instead of recomputing them")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--errors", action="store_true",
                    help="also compare every output with the oracle (max abs / rel / RMS), on "
                         "the stored features and on the original FP32 features")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="run only this many untimed steps (for rocprofv3) and exit")
    return ap.parse_args()


class Step:
    """Preallocated buffers and the ABI calls of one pass."""

    def __init__(self, sc, tile, keep_lists, dtype, dev):
        import torch
        import paper_2508_19140_amd as inpc
        from paper_2508_19140_amd import _lib as L
        self.torch, self.L = torch, L
        self.gauss = sc.radius is not None
        self.cam = inpc.camera_struct(sc.camera)
        self.opts = inpc.RasterSettings(splat="gaussian" if self.gauss else "bilinear", tile=tile,
                                        max_radius=float(sc.radius.max()) if self.gauss
                                        else 0.0).opts()
        self.keep_lists = keep_lists
        n, C = sc.feat.shape
        self.n, self.C = n, C
        tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[dtype]
        self.dtype_code = {"f32": L.DTYPE_F32, "bf16": L.DTYPE_BF16, "f16": L.DTYPE_F16}[dtype]
        self.bf = 4 if dtype == "f32" else 2
        self.pos = torch.from_numpy(sc.pos).to(dev)
        self.op = torch.from_numpy(sc.opacity).to(dev)
        self.feat = torch.from_numpy(sc.feat).to(dev).to(tdt).contiguous()
        self.radius = torch.from_numpy(sc.radius).to(dev) if self.gauss else None
        self.grad = None if self.gauss else torch.from_numpy(sc.grad).to(dev)
        lib = L.lib()
        cb, ob = ctypes.byref(self.cam), ctypes.byref(self.opts)
        self.cb, self.ob = cb, ob
        nt = int(lib.inpc_num_tiles(cb, ob))
        cap = int(lib.inpc_copy_capacity(n, cb, ob))
        self.nt = nt
        wsb = int(lib.inpc_workspace_bytes(n, cb, ob))
        self.ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        H, W = sc.camera.height, sc.camera.width
        self.P = H * W
        i32 = torch.int32
        mk = lambda *s, dt=torch.float32: torch.empty(*s, dtype=dt, device=dev)
        self.uv, self.key, self.ntiles = mk(n, 2), mk(n, dt=i32), mk(n, dt=i32)
        self.ranges, self.list = mk(nt + 1, dt=i32), mk(cap, dt=i32)
        self.order = mk(nt, dt=i32)
        self.lpos = mk(cap, dt=torch.int16)
        self.out, self.tf, self.nc = mk(C, H, W), mk(H, W), mk(H, W, dt=i32)
        self.state = None
        if not self.gauss:
            self.state = mk(int(lib.inpc_state_bytes(cb, ob)), dt=torch.uint8)
            self.gf, self.go, self.guv, self.gpos = mk(n, C), mk(n), mk(n, 2), mk(n, 3)
            self.scratch = mk(int(lib.inpc_backward_scratch_bytes(n, C, cb, ob)),
                              dt=torch.uint8)
        self.lib = lib
        self.stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    @staticmethod
    def p(t):
        return None if t is None else ctypes.c_void_p(t.data_ptr())

    def _chk(self, st, name):
        if st != 0:
            raise RuntimeError(f"{name}: {self.lib.inpc_last_error().decode()}")

    def project(self):
        p, lib = self.p, self.lib
        self._chk(lib.inpc_project(self.cb, self.ob, self.n, p(self.pos), p(self.radius),
                                   p(self.uv), p(self.key), p(self.ntiles), p(self.ws),
                                   self.ws.numel(), self.stream), "project")

    def bin(self):
        p, lib = self.p, self.lib
        self._chk(lib.inpc_bin(self.cb, self.ob, self.n, p(self.uv), p(self.radius), p(self.key),
                               p(self.ntiles), p(self.ranges), p(self.order), p(self.ws),
                               self.ws.numel(), self.stream), "bin")

    def sort(self):
        p, lib = self.p, self.lib
        self._chk(lib.inpc_sort(self.cb, self.ob, self.n, p(self.uv), p(self.ranges),
                                p(self.order), p(self.list), p(self.lpos), p(self.ws),
                                self.ws.numel(), self.stream), "sort")

    def blend_fwd(self):
        p, lib = self.p, self.lib
        self._chk(lib.inpc_blend_forward(self.cb, self.ob, self.n, p(self.uv), p(self.radius),
                                         p(self.op), p(self.feat), self.C, self.dtype_code, None,
                                         p(self.ranges), p(self.order), p(self.list),
                                         None if self.gauss else p(self.lpos), p(self.out),
                                         p(self.tf), p(self.nc), p(self.state), p(self.ws),
                                         self.ws.numel(), self.stream), "blend_forward")

    def blend_bwd(self):
        p, lib = self.p, self.lib
        self._chk(lib.inpc_blend_backward(self.cb, self.ob, self.n, p(self.uv), p(self.op),
                                          p(self.feat), self.C, self.dtype_code, None,
                                          p(self.ntiles), p(self.ranges), p(self.order),
                                          p(self.list), p(self.lpos), p(self.tf), p(self.state),
                                          p(self.grad), None, p(self.gf), p(self.go),
                                          p(self.guv), None, p(self.scratch),
                                          self.scratch.numel(), p(self.ws), self.ws.numel(),
                                          self.stream), "blend_backward")

    def project_bwd(self):
        p, lib = self.p, self.lib
        self._chk(lib.inpc_project_backward(self.cb, self.n, p(self.pos), p(self.ntiles),
                                            p(self.guv), p(self.gpos), self.stream),
                  "project_backward")

    def phases(self):
        fwd = [("project", self.project), ("bin", self.bin), ("sort", self.sort),
               ("blend_fwd", self.blend_fwd)]
        if self.gauss:
            return fwd
        bwd = [] if self.keep_lists else [("project", self.project), ("bin", self.bin),
                                          ("sort", self.sort)]
        bwd += [("blend_bwd", self.blend_bwd), ("project_bwd", self.project_bwd)]
        return fwd + bwd

    def run(self):
        for _, f in self.phases():
            f()


def byte_models(n, V, M, P, C, nt, bf=4, gauss=False, keep_lists=False):
    """Algorithmic bytes: the B_min / B_method models of the whole pass and
    the per-entry-point minima (each input read once, each output written once)."""
    D = M / max(V, 1)
    per_kernel = {
        # read positions (and radii), write uv + key + ntiles
        "project": 12 * n + 16 * n + (4 * n if gauss else 0),
        # read ntiles, uv and key of visible points; write one (key, index) copy per tile
        "bin": 4 * n + 12 * V + 8 * M + 8 * nt,
        # read the bucket, write the list (and the 2-byte splat positions)
        "sort": 8 * M + 4 * M + 4 * nt + (0 if gauss else 2 * M + 8 * V),
    }
    if gauss:
        # list + point data (uv, radius, opacity, features) once + image, t_final, n_contrib
        per_kernel["blend_fwd"] = 4 * M + 4 * nt + V * (16 + C * bf) + P * (4 * C + 8)
        b_min = n * (16 + 4 + C * bf) + 4 * D * V + 4 * P * (C + 2)
        return b_min, b_min + 64 * V + 24 * D * V, per_kernel
    per_kernel.update({
        # list + positions + point data once + image, t_final, n_contrib and state written
        "blend_fwd": 6 * M + 4 * nt + V * (12 + C * bf) + P * (4 * C + 20),
        # list + positions + point data + ntiles once + G, t_final, state read + gradients
        "blend_bwd": 6 * M + 4 * nt + V * (16 + C * bf) + P * (4 * C + 16) + n * (4 * C + 12),
        # positions, ntiles, grad_uv read; grad_pos written
        "project_bwd": 12 * n + 4 * n + 8 * n + 12 * n,
    })
    b_min = 2 * n * (16 + C * bf) + n * (16 + 4 * C) + 12 * D * V + 8 * P * (C + 1)
    b_sort = 64 * V + 24 * D * V
    return b_min, b_min + (1 if keep_lists else 2) * b_sort, per_kernel


def cpu_baseline(sc):
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    oracle.render(sc.camera, sc.pos, sc.opacity, sc.feat, radius=sc.radius,
                  splat=1 if sc.radius is not None else 0, grad_out=sc.grad)
    dt = time.perf_counter() - t0
    what = "fwd" if sc.radius is not None else "fwd+bwd"
    return {"value": sc.n / dt, "unit": "points/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"one full {what} frame of the same scene ({sc.n} points, "
                      f"{sc.camera.width}x{sc.camera.height}, C={sc.feat.shape[1]}), "
                      f"{dt:.1f} s wall"}


def error_table(step, sc, tile):
    """max abs / max rel / RMS of every output against the oracle, on the
    stored (possibly rounded) features and on the original FP32 features."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    step.run()
    step.torch.cuda.synchronize()
    gpu = {"out": step.out.cpu().numpy(), "t_final": step.tf.cpu().numpy()}
    if not step.gauss:
        gpu.update(grad_feat=step.gf.cpu().numpy(), grad_opacity=step.go.cpu().numpy(),
                   grad_pos=step.gpos.cpu().numpy())
    stored = step.feat.float().cpu().numpy()
    table = {}
    for label, feat in (("vs_stored_features", stored), ("vs_fp32_features", sc.feat)):
        rr = oracle.render(sc.camera, sc.pos, sc.opacity, feat, radius=sc.radius,
                           splat=1 if step.gauss else 0, tile=tile, grad_out=sc.grad)
        mask = rr["flags"] == 0
        row = {}
        for k, g in gpu.items():
            ref = rr[k]
            ref_abs = rr.get(k + "_abs", np.abs(ref))
            if k == "out":
                g, ref, ref_abs = g[:, mask], ref[:, mask], ref_abs[:, mask]
            elif k == "t_final":
                g, ref, ref_abs = g[mask], ref[mask], ref_abs[mask]
            _, st = oracle.within_tolerance(g, ref, ref_abs)
            row[k] = st
        row["flagged_pixels"] = int((~mask).sum())
        table[label] = row
    return table


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU: the rasterizer shards by view, one view per GPU, "
              "and this build measures the single-GPU path only (--gpus 1).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from scenes import CONFIGS, make_scene

    dtype = args.dtype or ("bf16" if args.config == "C5" else "f32")
    spec = CONFIGS[args.config]
    sc = make_scene(spec)
    dev = "cuda:0"
    torch.cuda.set_device(0)
    step = Step(sc, args.tile, args.keep_lists, dtype, dev)

    if args.profile_steps:
        for _ in range(args.profile_steps):
            step.run()
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps}), flush=True)
        return

    for _ in range(args.warmup):
        step.run()
    torch.cuda.synchronize()

    # Timed region: K steps, every entry point bracketed by HIP events on the
    # stream the library launches on (torch's current stream).
    names = [nm for nm, _ in step.phases()]
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    for s in range(args.steps):
        evs[s][0].record()
        for i, (_, f) in enumerate(step.phases()):
            f()
            evs[s][i + 1].record()
    torch.cuda.synchronize()
    ms = evs[0][0].elapsed_time(evs[-1][-1]) / args.steps
    phase_ms, per_launch_ms = {}, {}
    for i, nm in enumerate(names):
        t = float(np.mean([evs[s][i].elapsed_time(evs[s][i + 1]) for s in range(args.steps)]))
        phase_ms[nm] = phase_ms.get(nm, 0.0) + t
    count = {nm: names.count(nm) for nm in set(names)}
    for nm in phase_ms:
        per_launch_ms[nm] = phase_ms[nm] / count[nm]

    ntiles = step.ntiles.cpu().numpy()
    V = int((ntiles > 0).sum())
    M = int(step.ranges[-1].item())
    n, C, P = step.n, step.C, step.P
    b_min, b_method, per_kernel = byte_models(n, V, M, P, C, step.nt, step.bf, step.gauss,
                                              args.keep_lists)
    dominant = max(phase_ms, key=lambda k: phase_ms[k])
    dom_bytes = per_kernel[dominant]
    dom_gbs = dom_bytes / (per_launch_ms[dominant] * 1e-3) / 1e9
    t_s = ms * 1e-3
    pas = "fwd" if step.gauss else "fwd+bwd"
    res = {
        "metric": METRIC,
        "value": n / t_s,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic (seeded scene: 70% of points on 4 planes/spheres, 30% uniform)",
        "config": {"workload": f"{args.config}: {n} points, {sc.camera.width}x"
                               f"{sc.camera.height}, C={C} {dtype}, "
                               f"{'Gaussian' if step.gauss else 'bilinear'}, tile {args.tile}, "
                               f"{pas}" + ("" if step.gauss else
                                           (", lists kept" if args.keep_lists
                                            else ", lists recomputed in bwd")),
                   "points": n, "width": sc.camera.width, "height": sc.camera.height,
                   "channels": C, "tile": args.tile, "keep_lists": args.keep_lists},
        "visible_points_per_s": V / t_s,
        "frames_per_s": 1.0 / t_s,
        "V": V, "M": M, "D": M / max(V, 1),
        "B_min_GBps": b_min / t_s / 1e9,
        "B_method_GBps": b_method / t_s / 1e9,
        "B_min_frac": b_min / t_s / 1e9 / HBM_PEAK_GBS,
        "B_method_frac": b_method / t_s / 1e9 / HBM_PEAK_GBS,
        "phase_ms": phase_ms,
        "roofline": {"bound": "hbm", "kernel": f"inpc_{dominant}", "achieved": dom_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom_gbs / HBM_PEAK_GBS,
                     "bytes_per_launch": dom_bytes, "ms_per_launch": per_launch_ms[dominant],
                     "traffic": None},
    }
    if args.errors:
        res["errors"] = error_table(step, sc, args.tile)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(sc)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
