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
  const float* proj;  // [n][4] (u, v, opacity, radius)
  const void* feat;
  int C;
  int dtype;
  const float* bg;
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
  float* grad_bg;
  float* bg_partial;  // [num_tiles][C] per-tile background gradients
  float4* gsc;        // [n] (dL/do, dL/du, dL/dv, -) per point, unpacked into grad_opacity
                      // and grad_uv at the end (one 16-byte row per point for the atomics)
  const uint32_t* flags;
};

// Channel capacity of the kernel instantiation used for C channels.
inline int channel_capacity(int C) { return C <= 4 ? 4 : (C <= 8 ? 8 : (C <= 16 ? 16 : 32)); }

hipError_t launch_clear(uint32_t* p, size_t n, hipStream_t s);
hipError_t launch_project(const Cam& cam, const Opts& o, int64_t n, const float* pos,
                          const float* opacity, const float* radius, float* proj, uint32_t* key,
                          uint32_t* ntiles, const Ws& ws, hipStream_t s);
hipError_t launch_bin(const Cam& cam, const Opts& o, int64_t n, const float* proj,
                      const uint32_t* key, const uint32_t* ntiles, uint32_t* ranges,
                      uint32_t* order, const Ws& ws, hipStream_t s);
hipError_t launch_sort(const Ws& ws, uint32_t* list, uint16_t* lpos, int64_t nt, hipStream_t s);
hipError_t launch_lpos(const Cam& cam, const Opts& o, const uint32_t* ranges,
                       const uint32_t* order, const float* proj, const uint32_t* list,
                       uint16_t* lpos, const uint32_t* flags, hipStream_t s);
hipError_t launch_blend_forward(const BlendArgs& a, hipStream_t s);
hipError_t launch_blend_backward(const BlendArgs& a, hipStream_t s);
hipError_t launch_project_backward(const Cam& cam, int64_t n, const float* pos,
                                   const uint32_t* ntiles, const float* grad_uv, float* grad_pos,
                                   hipStream_t s);

}  // namespace inpc
