// Host-side launchers shared between the kernel files and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace inpc {

struct BlendArgs {
  Cam cam;
  Opts opts;
  int64_t n;
  const float* proj;  // [n][4] (u, v, opacity, radius | depth Z | 0)
  const void* feat;
  int C;
  int dtype;
  const float* bg;     // [C], or [C][H][W] when bg_image
  int bg_image;
  const uint32_t* ranges;
  const uint32_t* order;  // [nt] tile processing order, or NULL for tile-index order
  const uint32_t* list;
  const uint16_t* lpos;  // per list entry: tile-local 2x2 splat corner, +1 per axis (bilinear)
  // forward outputs
  float* out;
  float* t_final;
  uint32_t* n_contrib;
  uint32_t* st_last;    // [P] one past the tile-list position of the last blended fragment
  uint32_t* st_anchor;  // [P] one past the position of the last blended fragment with T > 0
  float* st_tanchor;    // [P] transmittance in front of that fragment
  uint32_t* st_tile;    // [nt] largest st_last over the tile's pixels
  // backward
  const uint32_t* ntiles;
  const float* grad_out;
  const float* grad_t;
  float* grad_feat;
  float* grad_opacity;
  float* grad_uv;
  float* grad_z;      // [n] dL/dZ at fixed (u, v) (world-space Gaussians), or NULL
  float* grad_bg;     // [C], or [C][H][W] when bg_image (written per pixel)
  float* bg_partial;  // [num_tiles][C] per-tile background gradients (constant background)
  float4* gsc;        // [n] (dL/do, dL/du, dL/dv, dL/dZ) per point, unpacked into
                      // grad_opacity, grad_uv and grad_z at the end (one 16-byte row per
                      // point for the atomics)
  const uint32_t* flags;
  int prezeroed;  // host side only: grad_feat and gsc are already zero (no fill before the tiles)
};

// A batch's work queue for the batched blend kernels: per-view arguments
// (device) and the (view, position in the view's tile order) slots, one
// workgroup per slot.  Views contribute whole quads of four slots; slots past
// a view's last tile hold kNoItem.
constexpr uint32_t kNoItem = 0xffffffffu;
struct BatchQueue {
  const BlendArgs* args;
  const uint2* items;
  uint32_t total;  // slots
};

// Blend arguments of one view of a batch (host and device: the batched
// entry point builds them on the host for the per-view steps, and a kernel
// builds the same from the device-resident view table for the persistent
// blend kernels).
__host__ __device__ inline BlendArgs make_view_args(const inpc_view_t& w, const Opts& shared,
                                                    int C, int dtype, int bg_image) {
  BlendArgs a = {};
  a.cam.W = w.cam.width;
  a.cam.H = w.cam.height;
  a.cam.fx = w.cam.fx;
  a.cam.fy = w.cam.fy;
  a.cam.cx = w.cam.cx;
  a.cam.cy = w.cam.cy;
  for (int k = 0; k < 9; ++k) a.cam.R[k] = w.cam.R[k];
  for (int k = 0; k < 3; ++k) a.cam.t[k] = w.cam.t[k];
  a.cam.z_near = w.cam.z_near;
  a.opts = shared;
  a.opts.ntx = (w.cam.width + shared.T - 1) / shared.T;
  a.opts.nty = (w.cam.height + shared.T - 1) / shared.T;
  a.n = w.n;
  a.proj = w.proj;
  a.feat = w.feat;
  a.C = C;
  a.dtype = dtype;
  a.bg = w.bg;
  a.bg_image = bg_image;
  a.ranges = w.tile_ranges;
  a.order = w.tile_order;
  a.list = w.list;
  a.lpos = w.lpos;
  a.out = w.out;
  a.t_final = w.t_final;
  a.n_contrib = w.n_contrib;
  const int64_t P = (int64_t)w.cam.width * w.cam.height;
  if (w.state) {
    a.st_last = static_cast<uint32_t*>(w.state);
    a.st_anchor = a.st_last + P;
    a.st_tanchor = reinterpret_cast<float*>(a.st_anchor + P);
    a.st_tile = a.st_last + 3 * P;
  }
  a.ntiles = w.ntiles;
  a.grad_out = w.grad_out;
  a.grad_t = w.grad_t;
  a.grad_feat = w.grad_feat;
  a.grad_opacity = w.grad_opacity;
  a.grad_uv = w.grad_uv;
  a.grad_z = w.grad_z;
  a.grad_bg = w.grad_bg;
  a.gsc = static_cast<float4*>(w.scratch);
  // the scratch holds a 16-byte row per point (rounded up to 256 bytes),
  // then the per-tile background shares
  a.bg_partial = (w.grad_bg && !bg_image && w.scratch)
                     ? reinterpret_cast<float*>(static_cast<char*>(w.scratch) +
                                                ((size_t)w.n * 16 + 255) / 256 * 256)
                     : nullptr;
  a.flags = static_cast<const uint32_t*>(w.ws);  // the workspace starts with its flags
  return a;
}

// Quad counts (ceil(tiles / 4)) of the views of a batch as an exclusive
// prefix, and the tile counts (kernel argument of the queue builder).
constexpr int kMaxBatchViews = 64;
struct BatchTiles {
  int nv;
  int64_t start[kMaxBatchViews + 1];
  int64_t tiles[kMaxBatchViews];
};

// A ring buffer of point clouds in one allocation: `slots` slots of `cap`
// points; point j of slot s is index s * cap + j, and only the first
// count[s] points of slot s are live (the others are culled).  slots = 0: every
// point is live.
constexpr int kMaxRingSlots = 16;
struct Ring {
  int slots;
  uint32_t cap;
  uint32_t count[kMaxRingSlots];
};
__host__ __device__ inline bool ring_live(const Ring& r, int64_t i) {
  if (r.slots == 0) return true;
  const uint32_t s = (uint32_t)i / r.cap;
  return (uint32_t)i - s * r.cap < r.count[s];
}

// Channel capacity of the kernel instantiation used for C channels.
inline int channel_capacity(int C) { return C <= 4 ? 4 : (C <= 8 ? 8 : (C <= 16 ? 16 : 32)); }

hipError_t launch_clear(uint32_t* p, size_t n, hipStream_t s);
hipError_t launch_project(const Cam& cam, const Opts& o, int64_t n, const float* pos,
                          const float* opacity, const float* radius, float* proj, uint32_t* key,
                          uint32_t* ntiles, const Ws& ws, const Ring& ring, hipStream_t s);
hipError_t launch_bin(const Cam& cam, const Opts& o, int64_t n, const float* proj,
                      const uint32_t* key, const uint32_t* ntiles, uint32_t* ranges,
                      uint32_t* order, const Ws& ws, hipStream_t s);
hipError_t launch_sort(const Ws& ws, uint32_t* list, uint16_t* lpos, int64_t nt, hipStream_t s);
hipError_t launch_lpos(const Cam& cam, const Opts& o, const uint32_t* ranges,
                       const uint32_t* order, const float* proj, const uint32_t* list,
                       uint16_t* lpos, const uint32_t* flags, hipStream_t s);
hipError_t launch_blend_forward(const BlendArgs& a, hipStream_t s);
hipError_t launch_blend_backward(const BlendArgs& a, hipStream_t s);
hipError_t launch_view_dirs(const Cam& c, float* dirs, hipStream_t s);
hipError_t launch_envmap_forward(const Cam& c, const float* dirs, const float* env, int Hm, int Wm,
                                 int C, float* bg, hipStream_t s);
hipError_t launch_envmap_backward(const Cam& c, const float* dirs, const float* grad_bg, int Hm,
                                  int Wm, int C, float* grad_env, hipStream_t s);
hipError_t launch_blend_backward_pre(const BlendArgs& a, hipStream_t s);
// The fill the backward blend starts with: grad_feat [n][C] and the scalar
// rows [n][4] at the start of its scratch, to zero.
hipError_t launch_backward_zero(float* grad_feat, int64_t n, int C, void* scratch, hipStream_t s);
hipError_t launch_blend_backward_post(const BlendArgs& a, hipStream_t s);
hipError_t launch_blend_batched(bool forward, const BlendArgs& shape, const BatchQueue& q,
                                hipStream_t s);
hipError_t launch_batch_prepare(const inpc_view_t* views_dev, int nv, const Opts& shared, int C,
                                int dtype, int bg_image, const BatchTiles& bt, BlendArgs* args,
                                uint2* items, hipStream_t s);
hipError_t launch_sh_forward(const Cam& c, int64_t n, int C, const float* pos, const float* sh,
                             float* feat, hipStream_t s);
hipError_t launch_sh_backward(const Cam& c, int64_t n, int C, const float* pos, const float* sh,
                              const float* grad_feat, float* grad_sh, float* grad_pos,
                              hipStream_t s);
hipError_t launch_project_backward(const Cam& cam, int64_t n, const float* pos,
                                   const uint32_t* ntiles, const float* grad_uv,
                                   const float* grad_z, float* grad_pos, hipStream_t s);

}  // namespace inpc
