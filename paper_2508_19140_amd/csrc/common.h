// Device-side definitions shared by the rasterizer kernels.
//
// Decision arithmetic (projection, footprints, tile membership) is written
// with explicitly rounded FP32 intrinsics so that the compiler can neither
// fuse nor reorder it; the whole library is also built with
// -ffp-contract=off.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "inpc_raster.h"

namespace inpc {

constexpr int kWave = 64;

// Sort size classes (segment copy counts).
constexpr uint32_t kSortCapW = 256;
constexpr uint32_t kSortCapM = 2048;
constexpr uint32_t kSortCapL = 16384;   // largest segment the MSD split takes
constexpr uint32_t kSortCapLB = 8192;   // largest segment LSD-sorted by one block (L class)

// Largest tile count whose per-workgroup histogram fits in LDS (144 KiB).
constexpr int kLdsBins = 36864;
constexpr int kOrderClasses = 34;  // blend-order classes 0..32 and "no tile"

// Points per workgroup of the counting / scatter passes (tile counts up to
// kLdsBins): at least 8192 and at most 256 workgroups, in whole rounds of
// the 1024-thread block.
// `want` = 0 picks 8192.
inline int64_t bin_chunk(int64_t n, int64_t want) {
  const int64_t per = (n + 255) / 256;
  const int64_t w = want > 0 ? want : 8192;
  const int64_t c = per > w ? per : w;
  return (c + 1023) / 1024 * 1024;
}
inline int64_t bin_rows(int64_t n, int64_t want) {
  return n > 0 ? (n + bin_chunk(n, want) - 1) / bin_chunk(n, want) : 0;
}

// Camera in kernel-argument form (by value).
struct Cam {
  int W, H;
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
  float z_near;
};

struct Opts {
  int splat;
  int T;     // tile edge
  int ntx, nty;
  float t_min, dilation, cutoff;
  float ewa_sigma;  // world-space Gaussians: standard deviation in world units
};

// Workspace flag slots.
enum : int {
  kFlagOverflow = 0,
  kFlagCountW = 1,   // segments sorted by one wavefront (n <= 256)
  kFlagCountM = 2,   // segments sorted by a 256-thread block (n <= 2048)
  kFlagCountL = 3,   // segments LSD-sorted by a 1024-thread block (n <= kSortCapLB)
  kFlagCountX = 4,   // larger segments, sorted through global memory
  kFlagCountB0 = 5,  // tiles to split (2048 < n <= 16384)
  kFlagCountB1 = 6,  // sub-segments to split a second time
  kFlagCountG = 7,   // sub-segments of more than 16384 copies to split through global memory again
  kFlagCountX2 = 8,  // segments left for the global-memory LSD sort
  kFlagSplitNext0 = 9,   // work counters of the two split rounds (segments taken so far)
  kFlagSplitNext1 = 10,
  kFlagSlots = 16
};

// Pointers into the caller's workspace.  Segment lists hold (start, count)
// pairs of bucket ranges.
struct Ws {
  uint32_t* flags;       // [kFlagSlots]
  uint32_t* tile_count;  // [nt]   copies per tile (filled by project)
  // per group of 64 tiles: copies, tiles per sort class, tiles per blend-order
  // class (then their exclusive prefix over the groups), and the totals
  uint64_t* gsum;        // [groups]
  uint32_t* gcls;        // [groups][4]
  uint32_t* gord;        // [groups][kOrderClasses]
  uint64_t* coltot;      // [1 + 4 + kOrderClasses] column totals over the groups
  int64_t groups;
  uint32_t* blk;         // [rows][nt] per-workgroup tile counts, then their exclusive
                         //        prefix over workgroups (nt <= kLdsBins)
  uint32_t* cursor;      // [nt]   scatter cursors
  uint2* seg_w;          // segment lists per sort class
  uint2* seg_m;
  uint2* seg_l;
  uint2* seg_x;          // tiles of more than 16384 copies (split through global memory)
  uint2* seg_g;          // their sub-segments still above 16384 (second global split)
  uint2* seg_x2;         // what is left for the global-memory LSD sort
  uint2* seg_b0;
  uint2* seg_b1;
  uint2* bucket;         // [cap]  (depth key, point index) copies, bucketed by tile
  uint2* xbucket;        // [cap]  ping-pong scratch for segments beyond the LDS capacity
  uint32_t cap;          // copy capacity
  int64_t chunk, rows;   // points per workgroup of the counting / scatter passes, workgroups
  // Bilinear splats with few enough points: the index word of a bucket entry
  // is (point index << lbits) | (y code << pb) | x code, where the codes are
  // the tile-local corner of the copy's 2x2 splat plus one.  The index stays
  // in the high bits, so ordering by the packed word orders by index.
  int lbits;             // 0: plain point index
  int pb;                // bits per axis code
};

// Where a sorted copy goes: its point index into list[q] and, for packed
// entries, its tile-local splat corner into lpos[q] (x code | y code << 8).
struct ListOut {
  uint32_t* list;
  uint16_t* lpos;
  int lbits, pb;
  __device__ __forceinline__ void put(uint32_t q, uint32_t v) const {
    if (lbits) {
      const uint32_t m = (1u << pb) - 1u;
      list[q] = v >> lbits;
      lpos[q] = (uint16_t)((v & m) | (((v >> pb) & m) << 8));
    } else {
      list[q] = v;
    }
  }
};

__device__ __forceinline__ float fmul(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ float fadd(float a, float b) { return __fadd_rn(a, b); }
__device__ __forceinline__ float fsub(float a, float b) { return __fsub_rn(a, b); }
__device__ __forceinline__ float fdiv(float a, float b) { return __fdiv_rn(a, b); }
// Correctly rounded square root.  (HIP's __fsqrt_rn is the native
// v_sqrt_f32, which is off by an ulp for some inputs; sqrtf is lowered to
// the native root plus an FMA correction step, correctly rounded like the
// divide, under HIP's default correctly-rounded divide/sqrt mode.)
__device__ __forceinline__ float fsqrt(float a) { return sqrtf(a); }

// Camera-space position and image coordinates of one point.
struct Proj {
  float X, Y, Z, u, v;
  bool in_front;
};

__device__ __forceinline__ Proj project_point(const Cam& c, float x, float y, float z) {
  Proj p;
  p.X = fadd(fadd(fadd(fmul(c.R[0], x), fmul(c.R[1], y)), fmul(c.R[2], z)), c.t[0]);
  p.Y = fadd(fadd(fadd(fmul(c.R[3], x), fmul(c.R[4], y)), fmul(c.R[5], z)), c.t[1]);
  p.Z = fadd(fadd(fadd(fmul(c.R[6], x), fmul(c.R[7], y)), fmul(c.R[8], z)), c.t[2]);
  p.in_front = p.Z > c.z_near;  // false for NaN
  p.u = fadd(fmul(c.fx, fdiv(p.X, p.Z)), c.cx);
  p.v = fadd(fmul(c.fy, fdiv(p.Y, p.Z)), c.cy);
  return p;
}

// Pixel rectangle (inclusive, clipped to the image) that can hold a point's
// fragments, plus the quantities the blend needs.
struct Footprint {
  bool visible;
  int px0, py0, px1, py1;
  // bilinear
  int x0, y0;
  float a, b;
  // Gaussian
  float s2, thr;
  // world-space Gaussian: inverse of the projected covariance (conic)
  float ca, cb, cc;
};

// Bilinear 2x2 splat: the four pixels whose centres surround (u, v).
__device__ __forceinline__ Footprint bilinear_footprint(float u, float v, int W, int H) {
  Footprint f;
  const float Wf = (float)W, Hf = (float)H;
  f.visible = (u >= -0.5f) && (u < fadd(Wf, 0.5f)) && (v >= -0.5f) && (v < fadd(Hf, 0.5f));
  f.s2 = 0.f;
  f.thr = 0.f;
  f.ca = f.cb = f.cc = 0.f;
  if (!f.visible) {
    f.px0 = f.py0 = 0; f.px1 = f.py1 = -1; f.x0 = f.y0 = 0; f.a = f.b = 0.f;
    return f;
  }
  const float xs = fsub(u, 0.5f), ys = fsub(v, 0.5f);
  const float fx0 = floorf(xs), fy0 = floorf(ys);
  f.x0 = (int)fx0;
  f.y0 = (int)fy0;
  f.a = fsub(xs, fx0);
  f.b = fsub(ys, fy0);
  f.px0 = f.x0 < 0 ? 0 : f.x0;
  f.py0 = f.y0 < 0 ? 0 : f.y0;
  f.px1 = f.x0 + 1 > W - 1 ? W - 1 : f.x0 + 1;
  f.py1 = f.y0 + 1 > H - 1 ? H - 1 : f.y0 + 1;
  return f;
}

// Isotropic screen-space Gaussian with variance r^2 + dilation, truncated at
// `cutoff` standard deviations.
__device__ __forceinline__ Footprint gaussian_footprint(float u, float v, float r, int W, int H,
                                                        float dilation, float cutoff) {
  Footprint f;
  f.x0 = f.y0 = 0;
  f.a = f.b = 0.f;
  f.ca = f.cb = f.cc = 0.f;
  const float s2 = fadd(fmul(r, r), dilation);
  const float Rc = fmul(cutoff, fsqrt(s2));
  const float xs = fsub(u, 0.5f), ys = fsub(v, 0.5f);
  float lx = ceilf(fsub(xs, Rc)), hx = floorf(fadd(xs, Rc));
  float ly = ceilf(fsub(ys, Rc)), hy = floorf(fadd(ys, Rc));
  lx = lx < 0.f ? 0.f : lx;
  ly = ly < 0.f ? 0.f : ly;
  hx = hx > (float)(W - 1) ? (float)(W - 1) : hx;
  hy = hy > (float)(H - 1) ? (float)(H - 1) : hy;
  f.visible = (lx <= hx) && (ly <= hy);
  if (!f.visible) {
    f.px0 = f.py0 = 0; f.px1 = f.py1 = -1; f.s2 = f.thr = 0.f;
    return f;
  }
  f.px0 = (int)lx; f.px1 = (int)hx;
  f.py0 = (int)ly; f.py1 = (int)hy;
  f.s2 = s2;
  f.thr = fmul(fmul(cutoff, cutoff), s2);
  return f;
}

// World-space isotropic Gaussian of standard deviation sigma, projected with
// the affine (EWA) approximation of the perspective map: covariance
// sigma^2 J J^T plus the dilation, J the projection's Jacobian at the point.
// With xh = (u - cx) / fx, yh = (v - cy) / fy (= X/Z, Y/Z), jx = fx / Z,
// jy = fy / Z:  a = sigma^2 jx^2 (1 + xh^2) + dil, b = sigma^2 jx jy xh yh,
// c = sigma^2 jy^2 (1 + yh^2) + dil.  Computed from the FP32 u, v, Z (the
// projection record) with one rounding per operation, so the blend passes
// recompute exactly the projection's decisions.  Cut where the Mahalanobis
// distance exceeds `cutoff`; candidates are the ellipse's bounding box,
// |dx| <= cutoff sqrt(a), |dy| <= cutoff sqrt(c).
struct EwaCov {
  float xh, yh, jx, jy, s2w;  // X/Z, Y/Z, fx/Z, fy/Z, sigma^2
  float a, b, c;              // projected covariance [[a, b], [b, c]], dilation included
};
__device__ __forceinline__ EwaCov ewa_cov(float u, float v, float Z, const Cam& c, float dilation,
                                          float sigma) {
  EwaCov k;
  k.xh = fdiv(fsub(u, c.cx), c.fx);
  k.yh = fdiv(fsub(v, c.cy), c.fy);
  k.jx = fdiv(c.fx, Z);
  k.jy = fdiv(c.fy, Z);
  k.s2w = fmul(sigma, sigma);
  k.a = fadd(fmul(k.s2w, fmul(fmul(k.jx, k.jx), fadd(1.f, fmul(k.xh, k.xh)))), dilation);
  k.b = fmul(k.s2w, fmul(fmul(k.jx, k.jy), fmul(k.xh, k.yh)));
  k.c = fadd(fmul(k.s2w, fmul(fmul(k.jy, k.jy), fadd(1.f, fmul(k.yh, k.yh)))), dilation);
  return k;
}

__device__ __forceinline__ Footprint ewa_footprint(float u, float v, float Z, const Cam& c,
                                                   float dilation, float cutoff, float sigma) {
  Footprint f;
  f.x0 = f.y0 = 0;
  f.a = f.b = 0.f;
  f.s2 = 0.f;
  const EwaCov k = ewa_cov(u, v, Z, c, dilation, sigma);
  const float a = k.a, b = k.b, cc = k.c;
  const float det = fsub(fmul(a, cc), fmul(b, b));
  f.ca = fdiv(cc, det);
  f.cb = -fdiv(b, det);
  f.cc = fdiv(a, det);
  const float Rx = fmul(cutoff, fsqrt(a)), Ry = fmul(cutoff, fsqrt(cc));
  const float xs = fsub(u, 0.5f), ys = fsub(v, 0.5f);
  float lx = ceilf(fsub(xs, Rx)), hx = floorf(fadd(xs, Rx));
  float ly = ceilf(fsub(ys, Ry)), hy = floorf(fadd(ys, Ry));
  lx = lx < 0.f ? 0.f : lx;
  ly = ly < 0.f ? 0.f : ly;
  hx = hx > (float)(c.W - 1) ? (float)(c.W - 1) : hx;
  hy = hy > (float)(c.H - 1) ? (float)(c.H - 1) : hy;
  f.visible = (lx <= hx) && (ly <= hy);
  if (!f.visible) {
    f.px0 = f.py0 = 0; f.px1 = f.py1 = -1; f.thr = 0.f;
    return f;
  }
  f.px0 = (int)lx; f.px1 = (int)hx;
  f.py0 = (int)ly; f.py1 = (int)hy;
  f.thr = fmul(cutoff, cutoff);
  return f;
}

// Footprint of a point from its projection record: w is the screen-space
// radius (Gaussian) or the camera-space depth Z (world-space Gaussian).
__device__ __forceinline__ Footprint footprint(const Opts& o, const Cam& c, float u, float v,
                                               float w) {
  if (o.splat == INPC_SPLAT_BILINEAR) return bilinear_footprint(u, v, c.W, c.H);
  if (o.splat == INPC_SPLAT_EWA) return ewa_footprint(u, v, w, c, o.dilation, o.cutoff,
                                                      o.ewa_sigma);
  return gaussian_footprint(u, v, w, c.W, c.H, o.dilation, o.cutoff);
}

// Squared distance of pixel centre offset (dx, dy) = (px + 1/2 - u, py + 1/2 - v)
// in the Gaussian's metric, FP32 with one rounding per operation: Euclidean
// (screen-space Gaussian; compared with cutoff^2 s2) or Mahalanobis through
// the conic (world-space; compared with cutoff^2).
__device__ __forceinline__ float gauss_d2(bool ewa, float dx, float dy, float ca, float cb,
                                          float cc) {
  if (!ewa) return fadd(fmul(dx, dx), fmul(dy, dy));
  return fadd(fadd(fmul(ca, fmul(dx, dx)), fmul(fmul(2.f, cb), fmul(dx, dy))),
              fmul(cc, fmul(dy, dy)));
}

// Position in a tile order handled by workgroup b of an nb-workgroup launch.
// Workgroups go to the 8 XCDs round-robin (workgroup b to XCD b mod 8) and
// every XCD has an L2 of its own; this mapping gives each XCD runs of four
// consecutive order positions (within every 32 consecutive workgroups, so the
// start of the order still starts first), a bijection on [0, nb).
__device__ __forceinline__ uint32_t xcd_pos(uint32_t b, uint32_t nb) {
  if (b >= (nb & ~31u)) return b;
  const uint32_t r = b & 31u;
  return (b & ~31u) | ((r & 7u) << 2) | (r >> 3);
}

// Wave-wide helpers (wave64).
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t mbcnt64(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

}  // namespace inpc
