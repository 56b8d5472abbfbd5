"""O(pixels x points) brute-force rasterizer in pure Python -- TEST INFRASTRUCTURE ONLY.

For tiny scenes (a few hundred points, a few hundred pixels).  For every
pixel it tests every point for coverage, collects the fragments, sorts them
by (depth key, point index) and alpha-blends them front to back (Eq. (1) of
Appendix A), then composites the background (Sec. 2, "Rendering Feature
Maps").  Decisions are taken with numpy float32 scalars (one rounding per
operation), blending in Python floats (FP64).  It is written independently
of ``inpc_oracle.c`` so that the two pin each other.
"""
from __future__ import annotations

import math
import struct

import numpy as np

f32 = np.float32


def _bits(z) -> int:
    return struct.unpack("<I", struct.pack("<f", float(z)))[0]


def point_decision(camera, p, radius=None, splat=0, dilation=0.16, cutoff=3.0):
    """Projection of one point; None when culled."""
    R = np.asarray(camera.R, np.float32).reshape(3, 3)
    t = np.asarray(camera.t, np.float32).reshape(3)
    x, y, z = f32(p[0]), f32(p[1]), f32(p[2])
    cam = []
    for r in range(3):
        acc = f32(R[r, 0]) * x
        acc = f32(acc + f32(R[r, 1]) * y)
        acc = f32(acc + f32(R[r, 2]) * z)
        acc = f32(acc + f32(t[r]))
        cam.append(acc)
    X, Y, Z = cam
    if not (Z > f32(camera.z_near)):
        return None
    u = f32(f32(f32(camera.fx) * f32(X / Z)) + f32(camera.cx))
    v = f32(f32(f32(camera.fy) * f32(Y / Z)) + f32(camera.cy))
    W, H = camera.width, camera.height
    d = dict(u=u, v=v, key=_bits(Z), X=X, Y=Y, Z=Z)
    if splat == 0:
        if not (u >= f32(-0.5) and u < f32(W) + f32(0.5) and v >= f32(-0.5) and v < f32(H) + f32(0.5)):
            return None
        xs, ys = f32(u - f32(0.5)), f32(v - f32(0.5))
        fx0, fy0 = np.floor(xs), np.floor(ys)
        d.update(x0=int(fx0), y0=int(fy0), a=f32(xs - fx0), b=f32(ys - fy0))
        px = [q for q in (d["x0"], d["x0"] + 1) if 0 <= q < W]
        py = [q for q in (d["y0"], d["y0"] + 1) if 0 <= q < H]
        d.update(px0=min(px), px1=max(px), py0=min(py), py1=max(py))
    else:
        s2 = f32(f32(f32(radius) * f32(radius)) + f32(dilation))
        Rc = f32(f32(cutoff) * np.sqrt(s2))
        xs, ys = f32(u - f32(0.5)), f32(v - f32(0.5))
        lx, hx = np.ceil(f32(xs - Rc)), np.floor(f32(xs + Rc))
        ly, hy = np.ceil(f32(ys - Rc)), np.floor(f32(ys + Rc))
        lx, ly = max(lx, f32(0)), max(ly, f32(0))
        hx, hy = min(hx, f32(W - 1)), min(hy, f32(H - 1))
        if not (lx <= hx and ly <= hy):
            return None
        d.update(px0=int(lx), px1=int(hx), py0=int(ly), py1=int(hy), s2=s2,
                 thr=f32(f32(f32(cutoff) * f32(cutoff)) * s2))
    return d


def fragment_at(d, px, py, splat=0):
    """(w32, w64) if the point has a fragment at pixel (px, py), else None."""
    if px < d["px0"] or px > d["px1"] or py < d["py0"] or py > d["py1"]:
        return None
    if splat == 0:
        dx, dy = px - d["x0"], py - d["y0"]
        if dx not in (0, 1) or dy not in (0, 1):
            return None
        a, b = d["a"], d["b"]
        wx32 = a if dx else f32(f32(1) - a)
        wy32 = b if dy else f32(f32(1) - b)
        wx = float(a) if dx else 1.0 - float(a)
        wy = float(b) if dy else 1.0 - float(b)
        return f32(wx32 * wy32), wx * wy
    ddx = f32(f32(f32(px) + f32(0.5)) - d["u"])
    ddy = f32(f32(f32(py) + f32(0.5)) - d["v"])
    d2 = f32(f32(ddx * ddx) + f32(ddy * ddy))
    if not (d2 <= d["thr"]):
        return None
    ex = (px + 0.5) - float(d["u"])
    ey = (py + 0.5) - float(d["v"])
    w = math.exp(-0.5 * (ex * ex + ey * ey) / float(d["s2"]))
    return f32(w), w


def render(camera, pos, opacity, feat, radius=None, bg=None, splat=0, t_min=1e-4,
           dilation=0.16, cutoff=3.0):
    """Returns out [C,H,W], t_final [H,W], n_contrib [H,W] and the per-pixel
    ordered fragment lists (point indices) for comparison."""
    n = len(pos)
    feat = np.asarray(feat, np.float64)
    C = feat.shape[1]
    W, H = camera.width, camera.height
    dec = [point_decision(camera, pos[i], None if radius is None else radius[i], splat,
                          dilation, cutoff) for i in range(n)]
    out = np.zeros((C, H, W))
    tf = np.zeros((H, W))
    nc = np.zeros((H, W), np.uint32)
    lists = {}
    for py in range(H):
        for px in range(W):
            frags = []
            for i in range(n):
                if dec[i] is None:
                    continue
                fw = fragment_at(dec[i], px, py, splat)
                if fw is not None:
                    frags.append((dec[i]["key"], i, fw[0], fw[1]))
            frags.sort(key=lambda e: (e[0], e[1]))
            lists[(px, py)] = [e[1] for e in frags]
            T, T32, cnt = 1.0, f32(1), 0
            F = [0.0] * C
            for key, i, w32, w in frags:
                o32 = f32(opacity[i])
                if splat == 0:
                    if T32 < f32(t_min):
                        break
                elif T < float(f32(t_min)):
                    break
                a = float(o32) * w
                for c in range(C):
                    F[c] += T * a * feat[i, c]
                T *= 1.0 - a
                T32 = f32(T32 * f32(f32(1) - f32(o32 * w32)))
                cnt += 1
            for c in range(C):
                out[c, py, px] = F[c] + T * (0.0 if bg is None else float(bg[c]))
            tf[py, px] = T
            nc[py, px] = cnt
    return dict(out=out, t_final=tf, n_contrib=nc, lists=lists)


def tile_lists(camera, pos, radius=None, splat=0, tile=8, dilation=0.16, cutoff=3.0):
    """For every tile, test every point's footprint rect; order by (key, idx)."""
    W, H = camera.width, camera.height
    ntx, nty = (W + tile - 1) // tile, (H + tile - 1) // tile
    dec = [point_decision(camera, pos[i], None if radius is None else radius[i], splat,
                          dilation, cutoff) for i in range(len(pos))]
    counts, lst = [], []
    for ty in range(nty):
        for tx in range(ntx):
            x0, x1 = tx * tile, min(W, (tx + 1) * tile) - 1
            y0, y1 = ty * tile, min(H, (ty + 1) * tile) - 1
            ent = []
            for i, d in enumerate(dec):
                if d is None:
                    continue
                if d["px1"] < x0 or d["px0"] > x1 or d["py1"] < y0 or d["py0"] > y1:
                    continue
                ent.append((d["key"], i))
            ent.sort()
            counts.append(len(ent))
            lst.extend(i for _, i in ent)
    return dict(counts=np.array(counts, np.uint32), list=np.array(lst, np.uint32))
