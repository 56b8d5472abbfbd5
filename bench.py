"""Benchmark: forward + backward rasterization of 2^23 points at 1920x1080.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--config H|C2|C3|C5|C4|R] [--splat ewa] [--dtype f32|bf16|f16]
                    [--tile 8|16] [--errors] [--profile-steps S]

One step is one training pass of the whole rasterizer on one view, exactly
what rasterize(...) followed by .backward() runs:
  forward : project -> bin -> sort -> blend forward
  backward: project -> bin -> sort (lists recomputed, not stored)
            -> blend backward -> project backward
(--config C3, screen-space Gaussian splats, is forward only: the paper uses
Gaussians at inference.  --splat ewa renders the configuration's points as
world-space Gaussians of the paper's default scale, forward + backward.
--config R renders the union of a ring buffer of four view-specific clouds,
forward only, one new cloud pushed into the ring per frame.)  Inputs (a seeded synthetic scene shaped like the paper's
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
    ap.add_argument("--config", default="H", choices=["H", "C2", "C3", "C5", "C4", "R"],
                    help="C4: 8 views of uneven size in one autotuned graph launch; R: a ring "
                         "of four clouds (2^21 points per slot, 1920x1080) rendered as one")
    ap.add_argument("--splat", default="auto", choices=["auto", "ewa"],
                    help="ewa: world-space Gaussians (EWA projection, default sigma), fwd+bwd")
    ap.add_argument("--tile", type=int, default=8, choices=[8, 16])
    ap.add_argument("--dtype", default=None, choices=["f32", "bf16", "f16"],
                    help="feature storage type (default: bf16 for C5, f32 otherwise)")
    ap.add_argument("--keep-lists", action="store_true",
                    help="backward reuses the forward's tile lists instead of recomputing them")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-zero-ahead", action="store_true",
                    help="zero the gradients inside the backward blend, on the step's stream, "
                         "instead of on a stream of their own ahead of it")
    ap.add_argument("--errors", action="store_true",
                    help="also compare every output with the oracle (max abs / rel / RMS), on "
                         "the stored features and on the original FP32 features")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="run only this many untimed steps (for rocprofv3) and exit")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="with --profile-steps: also run one plain device-to-device copy of "
                         "this many MiB (the reference for scaling HBM byte counters)")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="print a markdown table of a rocprofv3 --kernel-trace --stats run "
                         "(DIR/run_kernel_stats.csv) of --profile-steps S and exit")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="HBM traffic per launch of --entry from two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE) of --profile-steps S --copy-probe-mib M, "
                         "scaled by the copy's counters; prints a profiles/pmc_*.txt record")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="print a markdown table of any rocprofv3 --pmc run "
                         "(DIR/run_counter_collection.csv): every counter per kernel, "
                         "averaged over its calls, and exit")
    ap.add_argument("--cpu-table", action="store_true",
                    help="time the CPU oracle (fwd+bwd frames of C1, C2 and H) on one thread "
                         "and on all threads of this host, print one JSON line per row and exit")
    ap.add_argument("--entry", default="blend_bwd", help="entry point for --summarize-pmc")
    ap.add_argument("--command", default="", help="command line recorded in a summary")
    return ap.parse_args()


# Kernels launched by each C-ABI entry point (name prefixes).  Every entry
# point launches at least one of its kernels exactly once per call, so its
# number of calls in a trace is the smallest launch count among its kernels.
ENTRY_KERNELS = {
    "project": ("k_project_count", "k_colscan", "k_clear", "k_groups"),
    "bin": ("k_group_scan", "k_place", "k_scatter"),
    "sort": ("k_split", "k_sort_w", "k_sort_block", "k_sort_lx", "k_sort_x", "k_lpos"),
    "blend_fwd": ("k_blend_fwd",),
    "backward_zero": ("k_zero",),
    "blend_bwd": ("k_blend_bwd", "k_unpack_scalars", "k_bg_reduce"),
    "project_bwd": ("k_project_bwd",),
    "batch": ("k_batch_args", "k_batch_queue"),
    "background": ("k_view_dirs", "k_envmap_fwd", "k_envmap_bwd", "k_fill_zero"),
    "sh": ("k_sh_fwd", "k_sh_bwd"),
}


def _entry_calls(launches, entry):
    """Calls of `entry` from {kernel: launch count} of a trace."""
    c = [n for k, n in launches.items() if _entry_of(k) == entry and n > 0]
    return min(c) if c else 0
SOURCES = ["include/inpc_raster.h"] + [f"paper_2508_19140_amd/csrc/{f}" for f in
                                       ("api.hip", "project.hip", "sort.hip", "blend.hip",
                                        "background.hip", "batch.hip", "sh.hip", "common.h",
                                        "internal.h")]


def _kernel_short(name):
    import re
    n = re.sub(r"\(.*", "", name.replace("(anonymous namespace)::", "").replace("inpc::", ""))
    return n.replace("void ", "").strip()


def _entry_of(short):
    for e, pre in ENTRY_KERNELS.items():
        if any(short.startswith(p) for p in pre):
            return e
    return None


def summarize_trace(d, steps, command):
    import csv
    rows = list(csv.DictReader(open(os.path.join(d, "run_kernel_stats.csv"))))
    out = ["| kernel | entry point | calls | calls/step | avg us | total us/step | share |",
           "|---|---|---:|---:|---:|---:|---:|"]
    tot = sum(float(r["TotalDurationNs"]) for r in rows if _entry_of(_kernel_short(r["Name"])))
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        k = _kernel_short(r["Name"])
        e = _entry_of(k)
        if e is None:
            continue
        c = int(r["Calls"])
        t = float(r["TotalDurationNs"])
        out.append(f"| `{k}` | {e} | {c} | {c / steps:g} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{t / steps / 1e3:.1f} | {100 * t / tot:.1f}% |")
    print(f"Command: `{command}`\n\nrocprofv3 `run_kernel_stats.csv`, {steps} steps, "
          f"averages per launch.\n")
    print("\n".join(out))
    per_entry, launches = {}, {}
    for r in rows:
        k = _kernel_short(r["Name"])
        e = _entry_of(k)
        if e:
            per_entry[e] = per_entry.get(e, 0.0) + float(r["TotalDurationNs"])
            launches[k] = launches.get(k, 0) + int(r["Calls"])
    print("\n| entry point | calls/step | kernel time per call, us |\n|---|---:|---:|")
    for e, t in sorted(per_entry.items(), key=lambda x: -x[1]):
        calls = _entry_calls(launches, e)
        print(f"| inpc_{e} | {calls / steps:g} | {t / calls / 1e3:.1f} |")
    print(f"\nsum of kernel time per step: {tot / steps / 1e3:.1f} us")


def summarize_counters(d, command):
    import csv
    from collections import defaultdict
    vals = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
        k = _kernel_short(r["Kernel_Name"])
        if _entry_of(k):
            vals[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for k in vals for c in vals[k]})
    print(f"Command: `{command}`\n")
    print("rocprofv3 counters per kernel launch (mean over the launches of the run).\n")
    print("| kernel | entry point | " + " | ".join(names) + " |")
    print("|---|---|" + "---:|" * len(names))
    for k in sorted(vals):
        row = [f"{sum(vals[k][c]) / len(vals[k][c]):.4g}" if vals[k].get(c) else "-"
               for c in names]
        print(f"| `{k}` | {_entry_of(k)} | " + " | ".join(row) + " |")


def summarize_pmc(fetch_dir, write_dir, entry, steps, command):
    import csv
    import hashlib

    def read(d, counter):
        acc = {}
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            if r["Counter_Name"] != counter:
                continue
            k = _kernel_short(r["Kernel_Name"])
            acc.setdefault(k, []).append(float(r["Counter_Value"]) * 1024.0)  # KiB -> bytes
        return acc

    fetch, write = read(fetch_dir, "FETCH_SIZE"), read(write_dir, "WRITE_SIZE")
    copy = [k for k in fetch if "copyBuffer" in k]
    if not copy:
        raise SystemExit("no copy-probe kernel in the counter run (use --copy-probe-mib)")
    # the probe copies the same number of bytes it reads: its WRITE_SIZE run
    # is taken as exact (1 byte per byte) and FETCH_SIZE scaled to match
    cw = sum(write[copy[0]]) / len(write[copy[0]])
    cf = sum(fetch[copy[0]]) / len(fetch[copy[0]])
    fetch_scale, write_scale = cw / cf, 1.0
    lines = []
    per_launch_f = per_launch_w = 0.0
    calls = _entry_calls({k: len(v) for k, v in fetch.items()}, entry)
    for k in sorted(set(fetch) | set(write)):
        if _entry_of(k) != entry:
            continue
        f = sum(fetch.get(k, [])) * fetch_scale / calls
        w = sum(write.get(k, [])) * write_scale / calls
        per_launch_f += f
        per_launch_w += w
        lines.append(f"kernel {k} fetch_bytes_per_entry_call {f:.0f} write_bytes_per_entry_call "
                     f"{w:.0f}")
    print(f"# HBM traffic of inpc_{entry} per call, from rocprofv3 FETCH_SIZE and WRITE_SIZE")
    print(f"# command: {command}")
    print(f"# copy probe: FETCH_SIZE scaled by {fetch_scale:.4f} (copy reads = copy writes), "
          f"WRITE_SIZE by {write_scale:.4f}")
    for ln in lines:
        print(ln)
    print(f"fetch_bytes_per_launch {per_launch_f:.0f}")
    print(f"write_bytes_per_launch {per_launch_w:.0f}")
    print(f"traffic_bytes_per_launch {per_launch_f + per_launch_w:.0f}")
    for src in SOURCES:
        h = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
        print(f"sha256 {src} {h}")


def make_step(sc, tile, keep_lists, dtype, dev, splat="auto", ring_counts=None,
              zero_ahead=False):
    """The preallocated pipeline of one view (every buffer allocated here).
    Screen-space Gaussians (a scene with radii) and rings run forward only."""
    import torch
    import paper_2508_19140_amd as inpc
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[dtype]
    kind = "ewa" if splat == "ewa" else ("gaussian" if sc.radius is not None else "bilinear")
    backward = kind != "gaussian" and ring_counts is None
    v = inpc.ViewInputs(pos=torch.from_numpy(sc.pos).to(dev),
                        opacity=torch.from_numpy(sc.opacity).to(dev),
                        feat=torch.from_numpy(sc.feat).to(dev).to(tdt).contiguous(),
                        camera=sc.camera,
                        grad_out=torch.from_numpy(sc.grad).to(dev) if backward else None,
                        radius=torch.from_numpy(sc.radius).to(dev) if kind == "gaussian" else None,
                        ring_counts=ring_counts)
    st = inpc.RasterSettings(splat=kind, tile=tile, keep_lists=keep_lists,
                             max_radius=float(sc.radius.max()) if kind == "gaussian" else 0.0)
    step = inpc.ViewPipeline(v, st, zero_ahead=zero_ahead)
    step.kind = kind
    step.bf = 4 if dtype == "f32" else 2
    step.P = sc.camera.width * sc.camera.height
    return step


def measured_traffic(entry, config):
    """HBM bytes per launch of an entry point from a committed counter
    summary (profiles/pmc_<entry>_<config>.txt: FETCH_SIZE + WRITE_SIZE summed
    over the entry point's kernels, scaled by a plain copy's counters), or
    None when there is none or a kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"pmc_{entry}_{config}.txt")
    if not os.path.exists(path):
        return None
    traffic, ok = None, True
    for line in open(path):
        f = line.split()
        if len(f) == 3 and f[0] == "sha256":
            src = os.path.join(ROOT, f[1])
            if not os.path.exists(src) or \
                    hashlib.sha256(open(src, "rb").read()).hexdigest() != f[2]:
                ok = False
        elif len(f) == 2 and f[0] == "traffic_bytes_per_launch":
            traffic = float(f[1])
    return traffic if ok else None


def byte_models(n, V, M, P, C, nt, bf=4, gauss=False, keep_lists=False, kind=None,
                backward=None):
    """Algorithmic bytes: the B_min / B_method models of the whole pass and
    the per-entry-point minima (each input read once, each output written once).
    kind: "bilinear", "gaussian" (screen-space, forward) or "ewa" (world-space,
    forward + backward: no splat positions, and the depth gradient)."""
    kind = kind or ("gaussian" if gauss else "bilinear")
    backward = (kind != "gaussian") if backward is None else backward
    gauss = kind != "bilinear"
    D = M / max(V, 1)
    if kind == "ewa" and backward:
        per_kernel = {
            "project": 12 * n + 4 * n + 16 * n + 8 * n,
            "bin": 4 * n + 20 * V + 8 * M + 8 * nt,
            "sort": 8 * M + 4 * M + 4 * nt,
            # list + point data once + image, t_final, n_contrib, state written
            "blend_fwd": 4 * M + 4 * nt + V * (16 + C * bf) + P * (4 * C + 20),
            # list + point data once + G, t_final, state read + ntiles and the gradients
            # (features, opacity, image position, depth)
            "blend_bwd": 4 * M + 4 * nt + V * (16 + C * bf) + P * (4 * C + 16) + n * (4 * C + 20),
            # positions, ntiles, grad_uv, grad_z read; grad_pos written
            "project_bwd": 12 * n + 4 * n + 8 * n + 4 * n + 12 * n,
        }
        b_min = 2 * n * (16 + C * bf) + n * (20 + 4 * C) + 8 * D * V + 8 * P * (C + 1)
        b_sort = 64 * V + 24 * D * V
        return b_min, b_min + (1 if keep_lists else 2) * b_sort, per_kernel
    per_kernel = {
        # read positions, opacity (and radii); write the projection record, key, ntiles
        "project": 12 * n + 4 * n + 16 * n + 8 * n + (4 * n if gauss else 0),
        # read ntiles, and record and key of visible points; write one copy per tile
        "bin": 4 * n + 20 * V + 8 * M + 8 * nt,
        # read the bucket, write the list (and the 2-byte splat positions)
        "sort": 8 * M + 4 * M + 4 * nt + (0 if gauss else 2 * M),
    }
    if gauss:
        # list + point data (record, features) once + image, t_final, n_contrib
        per_kernel["blend_fwd"] = 4 * M + 4 * nt + V * (16 + C * bf) + P * (4 * C + 8)
        b_min = n * (16 + 4 + C * bf) + 4 * D * V + 4 * P * (C + 2)
        return b_min, b_min + 64 * V + 24 * D * V, per_kernel
    per_kernel.update({
        # list + splat positions + point data once + image, t_final, n_contrib, state written
        "blend_fwd": 6 * M + 4 * nt + V * (16 + C * bf) + P * (4 * C + 20),
        # list + positions + point data once + G, t_final, state read + ntiles and gradients
        "blend_bwd": 6 * M + 4 * nt + V * (16 + C * bf) + P * (4 * C + 16) + n * (4 * C + 16),
        # positions, ntiles, grad_uv read; grad_pos written
        "project_bwd": 12 * n + 4 * n + 8 * n + 12 * n,
    })
    b_min = 2 * n * (16 + C * bf) + n * (16 + 4 * C) + 12 * D * V + 8 * P * (C + 1)
    b_sort = 64 * V + 24 * D * V
    return b_min, b_min + (1 if keep_lists else 2) * b_sort, per_kernel


def oracle_args(step, sc):
    """The oracle's splat options and inputs for a bench pipeline."""
    import numpy as np
    kw = {"splat": {"bilinear": 0, "gaussian": 1, "ewa": 2}[step.kind]}
    if step.kind == "ewa":
        kw["ewa_sigma"] = float(np.float32(step.settings.sigma(step.cam)))
    rad = sc.radius if step.kind == "gaussian" else None
    return kw, rad


def cpu_baseline(sc, step, live=None):
    """The oracle on the same frame (live: the ring's live point indices)."""
    import oracle
    oracle.build(force=False)
    kw, rad = oracle_args(step, sc)
    pos, op, ft = sc.pos, sc.opacity, sc.feat
    if live is not None:
        pos, op, ft = pos[live], op[live], ft[live]
    grad = sc.grad if step.backward_enabled else None
    t0 = time.perf_counter()
    oracle.render(sc.camera, pos, op, ft, radius=rad, grad_out=grad, **kw)
    dt = time.perf_counter() - t0
    what = "fwd+bwd" if grad is not None else "fwd"
    n = pos.shape[0]
    return {"value": n / dt, "unit": "points/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"one full {what} frame of the same scene ({n} points, "
                      f"{sc.camera.width}x{sc.camera.height}, C={sc.feat.shape[1]}), "
                      f"{dt:.1f} s wall"}


def cpu_table():
    """The oracle's wall time for one forward + backward frame, single-threaded
    and on every host thread: median of 3 for C1 and C2, one run for H."""
    import statistics
    import oracle
    from scenes import CONFIGS, make_scene
    oracle.build(force=False)
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    all_threads = oracle.num_threads()
    print(json.dumps({"cpu_model": model, "nproc": os.cpu_count(),
                      "oracle_threads_all": all_threads}), flush=True)
    for cfg, reps in (("C1", 3), ("C2", 3), ("H", 1)):
        sc = make_scene(CONFIGS[cfg])
        for thr in (all_threads, 1):
            oracle.set_num_threads(thr)
            times = []
            for _ in range(reps):
                t0 = time.perf_counter()
                oracle.render(sc.camera, sc.pos, sc.opacity, sc.feat, grad_out=sc.grad)
                times.append(time.perf_counter() - t0)
            med = statistics.median(times)
            print(json.dumps({"config": cfg, "points": sc.n, "threads": thr, "runs": reps,
                              "median_s": med, "points_per_s": sc.n / med}), flush=True)
    oracle.set_num_threads(all_threads)


def error_table(step, sc, tile):
    """max abs / max rel / RMS of every output against the oracle, on the
    stored (possibly rounded) features and on the original FP32 features."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    import torch
    step.step(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    gpu = {"out": step.out.cpu().numpy(), "t_final": step.tf.cpu().numpy()}
    if step.backward_enabled:
        gpu.update(grad_feat=step.gf.cpu().numpy(), grad_opacity=step.go.cpu().numpy(),
                   grad_pos=step.gpos.cpu().numpy())
        if step.gz is not None:
            gpu["grad_z"] = step.gz.cpu().numpy()
    stored = step.v.feat.float().cpu().numpy()
    kw, rad = oracle_args(step, sc)
    grad = sc.grad if step.backward_enabled else None
    table = {}
    for label, feat in (("vs_stored_features", stored), ("vs_fp32_features", sc.feat)):
        rr = oracle.render(sc.camera, sc.pos, sc.opacity, feat, radius=rad, tile=tile,
                           grad_out=grad, **kw)
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


def run_multiview(args):
    """8 views (n_v ~ U{0.5M..6M}, mixed resolutions) as one graph launch per
    step, against the same views run one after another with default settings
    and no graph (the plain single-view form)."""
    import numpy as np
    import torch
    import paper_2508_19140_amd as inpc
    from scenes import multi_view_scenes

    dev = "cuda:0"
    torch.cuda.set_device(0)
    scenes = multi_view_scenes(8)
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[args.dtype or "f32"]
    views = [inpc.ViewInputs(pos=torch.from_numpy(s.pos).to(dev),
                             opacity=torch.from_numpy(s.opacity).to(dev),
                             feat=torch.from_numpy(s.feat).to(dev).to(tdt).contiguous(),
                             camera=s.camera, grad_out=torch.from_numpy(s.grad).to(dev))
             for s in scenes]
    n_total = sum(s.pos.shape[0] for s in scenes)
    plain = inpc.MultiViewRasterizer(views, autotune=False)
    if args.profile_steps:
        # for rocprofv3: the plain per-view steps, then the batched steps, both
        # with 8x8 tiles and default binning, eager
        batched = inpc.BatchedRasterizer(views, autotune=False,
                                         settings=inpc.RasterSettings(tile=args.tile))
        for _ in range(args.profile_steps):
            plain.run_eager()
        torch.cuda.synchronize()
        for _ in range(args.profile_steps):
            batched.step()
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps, "config": "C4"}), flush=True)
        return

    def timed(fn, k):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    for _ in range(args.warmup):
        plain.run_eager()
    ms_plain = timed(plain.run_eager, args.steps)
    del plain
    torch.cuda.empty_cache()
    # the multi-stream graph of per-view calls (views overlap, each tuned alone)
    streams = inpc.MultiViewRasterizer(views)
    streams.capture()
    for _ in range(args.warmup):
        streams.replay()
    ms_streams = timed(streams.replay, args.steps)
    stream_choice = streams.choice
    del streams
    torch.cuda.empty_cache()
    # the batched entry point: one persistent blend launch over every (view,
    # tile) item per direction, tuned for the whole batch, in one graph
    tuned = inpc.BatchedRasterizer(views)
    tuned.capture()
    for _ in range(args.warmup):
        tuned.replay()
    ms_batched = timed(tuned.replay, args.steps)
    # the value is the faster of the two one-graph forms (both autotuned)
    ms = min(ms_batched, ms_streams)
    form = ("inpc_rasterize_batched per direction" if ms_batched <= ms_streams
            else "per-view ABI calls on a stream each")
    t_s = ms * 1e-3
    res = {
        "metric": "points rasterized/s fwd+bwd, 8 views of uneven size in one graph launch",
        "value": n_total / t_s, "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.dtype or "f32",
        "data": "synthetic (8 views of one seeded scene, own point sample per view)",
        "config": {"workload": f"C4: 8 views, {n_total} points in total, fwd+bwd, lists "
                               f"recomputed, one graph launch per step ({form})",
                   "batched_tile": tuned.choice[0], "batched_bin_points": tuned.choice[1],
                   "views": [{"points": int(s.pos.shape[0]), "width": s.camera.width,
                              "height": s.camera.height} for s in scenes]},
        "plain_single_view_ms": ms_plain,
        "speedup_vs_plain_single_view": ms_plain / ms,
        "batched_graph_ms": ms_batched,
        "batched_speedup_vs_plain": ms_plain / ms_batched,
        "multistream_graph_ms": ms_streams,
        "multistream_speedup_vs_plain": ms_plain / ms_streams,
        "multistream_graph_choice": [list(c) for c in stream_choice],
        "autotune_ms": {f"{t}/{bp}": round(v, 4) for (t, bp), v in tuned.tuning.items()},
    }
    print(json.dumps(res), flush=True)


def main():
    args = parse()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.profile_steps or 1, args.command)
        return
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, args.entry, args.profile_steps or 1, args.command)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.command)
        return
    if args.cpu_table:
        cpu_table()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU: the rasterizer shards by view, one view per GPU, "
              "and this benchmark measures the single-GPU path only (--gpus 1).", file=sys.stderr)
        sys.exit(2)
    if args.config == "C4":
        run_multiview(args)
        return
    import numpy as np
    import torch
    from scenes import CONFIGS, make_scene

    dtype = args.dtype or ("bf16" if args.config == "C5" else "f32")
    dev = "cuda:0"
    torch.cuda.set_device(0)
    ring = None
    if args.config == "R":
        sc, ring = ring_scene()
        step = make_step(sc, args.tile, args.keep_lists, dtype, dev, ring_counts=ring["counts"])
        ring_push = make_ring_push(step, ring, dev)
    else:
        sc = make_scene(CONFIGS[args.config])
        step = make_step(sc, args.tile, args.keep_lists, dtype, dev, splat=args.splat,
                         zero_ahead=not args.no_zero_ahead)
    h = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def phases():
        ph = step.phases()
        return ([("push", lambda _h: ring_push())] + ph) if ring is not None else ph

    if args.profile_steps:
        for _ in range(args.profile_steps):
            for _, f in phases():
                f(h)
        if args.copy_probe_mib:
            src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps,
                          "copy_probe_bytes": args.copy_probe_mib << 20}), flush=True)
        return

    for _ in range(args.warmup):
        for _, f in phases():
            f(h)
    torch.cuda.synchronize()

    # Timed region: K steps, every entry point bracketed by HIP events on the
    # stream the library launches on (torch's current stream).
    names = [nm for nm, _ in phases()]
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    for s in range(args.steps):
        evs[s][0].record()
        for i, (_, f) in enumerate(phases()):
            f(h)
            evs[s][i + 1].record()
    torch.cuda.synchronize()
    ms = evs[0][0].elapsed_time(evs[-1][-1]) / args.steps
    ms_median = float(np.median([evs[s][0].elapsed_time(evs[s][-1])
                                 for s in range(args.steps)]))
    phase_ms, per_launch_ms = {}, {}
    for i, nm in enumerate(names):
        t = float(np.mean([evs[s][i].elapsed_time(evs[s][i + 1]) for s in range(args.steps)]))
        phase_ms[nm] = phase_ms.get(nm, 0.0) + t
    count = {nm: names.count(nm) for nm in set(names)}
    for nm in phase_ms:
        per_launch_ms[nm] = phase_ms[nm] / count[nm]

    copy_gbs = copy_bandwidth(dev)
    ntiles = step.ntiles.cpu().numpy()
    V = int((ntiles > 0).sum())
    M = int(step.ranges[-1].item())
    n, C, P = step.n, step.C, step.P
    backward = step.backward_enabled
    b_min, b_method, per_kernel = byte_models(n, V, M, P, C, step.nt, step.bf, step.gauss,
                                              args.keep_lists, kind=step.kind,
                                              backward=backward)
    if ring is not None:
        # one new cloud into the ring: positions, opacities, features read and written
        per_kernel["push"] = 2 * ring["pushed"] * (16 + C * step.bf)
    dominant = max(phase_ms, key=lambda k: phase_ms[k])
    dom_bytes = per_kernel[dominant]
    dom_gbs = dom_bytes / (per_launch_ms[dominant] * 1e-3) / 1e9
    t_s = ms * 1e-3
    pas = "fwd+bwd" if backward else "fwd"
    kind_name = {"bilinear": "bilinear", "gaussian": "screen-space Gaussian",
                 "ewa": "world-space Gaussian (EWA)"}[step.kind]
    workload = (f"{args.config}: {n} points, {sc.camera.width}x{sc.camera.height}, C={C} "
                f"{dtype}, {kind_name}, tile {args.tile}, {pas}" +
                ("" if not backward else (", lists kept" if args.keep_lists
                                          else ", lists recomputed in bwd")))
    if ring is not None:
        workload = (f"R: ring of {len(ring['counts'])} clouds ({V} visible of {n} slots' "
                    f"points, live {sum(ring['counts'])}), {sc.camera.width}x"
                    f"{sc.camera.height}, C={C} {dtype}, bilinear, tile {args.tile}, fwd; one "
                    f"{ring['pushed']}-point cloud pushed per frame")
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
        "config": {"workload": workload,
                   "points": n, "width": sc.camera.width, "height": sc.camera.height,
                   "channels": C, "tile": args.tile, "keep_lists": args.keep_lists},
        "visible_points_per_s": V / t_s,
        "frames_per_s": 1.0 / t_s,
        "V": V, "M": M, "D": M / max(V, 1),
        "B_min_GBps": b_min / t_s / 1e9,
        "B_method_GBps": b_method / t_s / 1e9,
        "B_min_frac": b_min / t_s / 1e9 / HBM_PEAK_GBS,
        "B_method_frac": b_method / t_s / 1e9 / HBM_PEAK_GBS,
        "copy_bw_GBps": copy_gbs,
        "B_min_frac_of_copy": b_min / t_s / 1e9 / copy_gbs,
        "B_method_frac_of_copy": b_method / t_s / 1e9 / copy_gbs,
        "ms_per_step_median": ms_median,
        "phase_ms": phase_ms,
        "roofline": {"bound": "hbm", "kernel": f"inpc_{dominant}",
                     # name prefixes of the kernels that entry point launches; their
                     # rocprofv3 per-kernel times are in profiles/kernels_<workload>.md
                     "kernels": list(ENTRY_KERNELS.get(dominant, ())),
                     "achieved": dom_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom_gbs / HBM_PEAK_GBS,
                     "frac_of_copy": dom_gbs / copy_gbs,
                     "bytes_per_launch": dom_bytes, "ms_per_launch": per_launch_ms[dominant],
                     # the stored summaries count the backward blend without its zero
                     # fill, which --no-zero-ahead runs inside it
                     "traffic": None if (dominant == "blend_bwd" and args.no_zero_ahead)
                     else measured_traffic(
                         dominant, args.config + ("_ewa" if step.kind == "ewa" else ""))},
    }
    if args.errors and ring is None:
        res["errors"] = error_table(step, sc, args.tile)
    if not args.no_cpu_baseline:
        live = None
        if ring is not None:
            live = np.concatenate([np.arange(k * ring["per_slot"], k * ring["per_slot"] + c)
                                   for k, c in enumerate(ring["counts"])])
        res["cpu_baseline"] = cpu_baseline(sc, step, live)
    print(json.dumps(res), flush=True)


def ring_scene(slots=4, per_slot=1 << 21):
    """Four view-specific clouds of the H scene's generator (2^21 points per
    slot, 1920x1080, C=16) in a ring: slot s holds cloud s; slots 1 and 3 hold
    a little fewer points (the rest of their slots is stale data that the
    projection culls); a fifth cloud of 2^21 points is pushed into the oldest
    slot every frame, in turn with the cloud it replaced, so that the live
    counts stay fixed."""
    import dataclasses
    import numpy as np
    from scenes import CONFIGS, Scene, make_scene
    spec = dataclasses.replace(CONFIGS["H"], n=slots * per_slot)
    full = make_scene(spec)
    counts = [per_slot, per_slot - 100_000, per_slot, per_slot - 50_000]
    extra = make_scene(dataclasses.replace(CONFIGS["H"], n=per_slot, seed=spec.seed + 7))
    sc = Scene(pos=full.pos, opacity=full.opacity, feat=full.feat, camera=full.camera,
               grad=None, spec=spec)
    return sc, {"counts": counts, "per_slot": per_slot, "extra": extra, "pushed": per_slot,
                "np": np}


def make_ring_push(step, ring, dev):
    """The frame's ring update: the new cloud is copied into a slot (the
    sampler's output buffer to the ring; stream-ordered device copies; slot 0
    every frame, which slot does not change the work), alternating between
    the extra cloud and the one it displaced, so the live counts stay fixed."""
    import torch
    ex = ring["extra"]
    per = ring["per_slot"]
    v = step.v
    src = [(torch.from_numpy(ex.pos).to(dev), torch.from_numpy(ex.opacity).to(dev),
            torch.from_numpy(ex.feat).to(dev).to(v.feat.dtype)),
           (v.pos[:per].clone(), v.opacity[:per].clone(), v.feat[:per].clone())]
    state = {"k": 0}

    def push():
        p, o, f = src[state["k"] & 1]
        v.pos[:per].copy_(p)
        v.opacity[:per].copy_(o)
        v.feat[:per].copy_(f)
        state["k"] += 1
    return push


def copy_bandwidth(dev, mib=512, reps=20):
    """Bytes read plus written per second by a plain device-to-device copy of
    `mib` MiB (torch's copy kernel), the practical HBM rate of this device."""
    import torch
    src = torch.ones(mib << 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return 2.0 * (mib << 20) / sec / 1e9


if __name__ == "__main__":
    main()
