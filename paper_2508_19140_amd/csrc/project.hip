// Projection, tile counting, binning and the projection's backward pass.
//
// Step 1 (Sec. 2 and Sec. 3.2 of the paper): every point is moved into
// camera space, projected, culled against the near plane and the image, and
// given its 32-bit depth key and the set of tiles its footprint meets.  The
// per-tile copy counts are accumulated here with atomics (only counts: no
// order depends on them).
// Step 2 (Sec. 3.2, "Tiled Rendering"): one exclusive scan over the tile
// counts places every tile's bucket; every visible point then drops one
// (depth key, index) copy into the bucket of each tile it touches.  The
// order inside a bucket is irrelevant because the sort that follows orders
// every bucket by the unique pair (depth key, point index).
#include "common.h"
#include "internal.h"

namespace inpc {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int tile_shift(int T) { return T == 8 ? 3 : (T == 16 ? 4 : 5); }

__global__ void k_clear(uint32_t* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_project(Cam cam, Opts o, int64_t n,
                                                    const float* __restrict__ pos,
                                                    const float* __restrict__ radius,
                                                    float2* __restrict__ uv,
                                                    uint32_t* __restrict__ key,
                                                    uint32_t* __restrict__ ntiles,
                                                    uint32_t* __restrict__ tile_count) {
  const int sh = tile_shift(o.T);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    const Proj p = project_point(cam, x, y, z);
    bool vis = p.in_front;
    Footprint f;
    if (vis) {
      f = footprint(o, cam, p.u, p.v, radius ? radius[i] : 0.f);
      vis = f.visible;
    }
    uv[i] = make_float2(p.u, p.v);
    key[i] = __float_as_uint(p.Z);
    uint32_t nt = 0;
    if (vis) {
      const int tx0 = f.px0 >> sh, tx1 = f.px1 >> sh, ty0 = f.py0 >> sh, ty1 = f.py1 >> sh;
      nt = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
      for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) atomicAdd(&tile_count[ty * o.ntx + tx], 1u);
    }
    ntiles[i] = nt;
  }
}

// Block-wide inclusive scan of 64-bit values (1024 threads).
__device__ uint64_t block_scan_u64(uint64_t v, uint64_t* s) {
  const int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint64_t add = t >= o ? s[t - o] : 0ull;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  const uint64_t r = s[t];
  __syncthreads();
  return r;
}

__device__ __forceinline__ int sort_class(uint32_t c) {
  return c == 0 ? -1 : (c <= kSortCapW ? 0 : (c <= kSortCapM ? 1 : (c <= kSortCapL ? 2 : 3)));
}

// Single 1024-thread block: ranges = exclusive scan of the tile counts,
// scatter cursors, and the tile lists of the four sort classes (in tile
// order).  Flags an overflow when the copies exceed the capacity.
__global__ __launch_bounds__(1024) void k_scan(int64_t nt, const uint32_t* __restrict__ count,
                                               uint32_t* __restrict__ ranges,
                                               uint32_t* __restrict__ cursor, Ws ws) {
  __shared__ uint64_t s[1024];
  const int t = threadIdx.x;
  const int64_t seg = (nt + 1023) / 1024;
  const int64_t b = min<int64_t>(nt, t * seg), e = min<int64_t>(nt, b + seg);
  uint64_t tot = 0, cwm = 0, clx = 0;  // packed class counts: (W | M << 32), (L | X << 32)
  for (int64_t i = b; i < e; ++i) {
    const uint32_t c = count[i];
    tot += c;
    const int k = sort_class(c);
    if (k == 0) cwm += 1ull;
    if (k == 1) cwm += 1ull << 32;
    if (k == 2) clx += 1ull;
    if (k == 3) clx += 1ull << 32;
  }
  const uint64_t incl = block_scan_u64(tot, s);
  const uint64_t iwm = block_scan_u64(cwm, s);
  const uint64_t ilx = block_scan_u64(clx, s);
  uint64_t off = incl - tot;
  uint32_t ow = (uint32_t)(iwm - cwm), om = (uint32_t)((iwm - cwm) >> 32);
  uint32_t ol = (uint32_t)(ilx - clx), ox = (uint32_t)((ilx - clx) >> 32);
  for (int64_t i = b; i < e; ++i) {
    const uint32_t c = count[i];
    ranges[i] = (uint32_t)off;
    cursor[i] = (uint32_t)off;
    off += c;
    const int k = sort_class(c);
    if (k == 0) ws.list_w[ow++] = (uint32_t)i;
    if (k == 1) ws.list_m[om++] = (uint32_t)i;
    if (k == 2) ws.list_l[ol++] = (uint32_t)i;
    if (k == 3) ws.list_x[ox++] = (uint32_t)i;
  }
  if (t == 1023) {
    ranges[nt] = (uint32_t)incl;
    ws.flags[kFlagCountW] = (uint32_t)iwm;
    ws.flags[kFlagCountM] = (uint32_t)(iwm >> 32);
    ws.flags[kFlagCountL] = (uint32_t)ilx;
    ws.flags[kFlagCountX] = (uint32_t)(ilx >> 32);
    if (incl > (uint64_t)ws.cap) ws.flags[kFlagOverflow] = 1u;
  }
}

__global__ __launch_bounds__(kBlock) void k_scatter(Cam cam, Opts o, int64_t n,
                                                    const float2* __restrict__ uv,
                                                    const float* __restrict__ radius,
                                                    const uint32_t* __restrict__ key,
                                                    const uint32_t* __restrict__ ntiles,
                                                    uint32_t* __restrict__ cursor,
                                                    uint32_t* __restrict__ bkey,
                                                    uint32_t* __restrict__ bidx, uint32_t cap,
                                                    const uint32_t* __restrict__ flags) {
  if (flags[kFlagOverflow]) return;
  const int sh = tile_shift(o.T);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (ntiles[i] == 0) continue;
    const float2 p = uv[i];
    const Footprint f = footprint(o, cam, p.x, p.y, radius ? radius[i] : 0.f);
    const uint32_t k = key[i];
    const int tx0 = f.px0 >> sh, tx1 = f.px1 >> sh, ty0 = f.py0 >> sh, ty1 = f.py1 >> sh;
    for (int ty = ty0; ty <= ty1; ++ty)
      for (int tx = tx0; tx <= tx1; ++tx) {
        const uint32_t slot = atomicAdd(&cursor[ty * o.ntx + tx], 1u);
        if (slot < cap) {  // always true when the counts of step 1 hold
          bkey[slot] = k;
          bidx[slot] = (uint32_t)i;
        }
      }
  }
}

// Gradients of points that no single tile owns (culled points and points
// split over several tiles) start at zero; single-tile points are written
// with plain stores by the blend backward.
__global__ __launch_bounds__(kBlock) void k_grad_init(int64_t n, int C,
                                                      const uint32_t* __restrict__ ntiles,
                                                      float* __restrict__ grad_feat,
                                                      float* __restrict__ grad_opacity,
                                                      float2* __restrict__ grad_uv,
                                                      float* __restrict__ grad_bg) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid == 0 && grad_bg)
    for (int c = 0; c < C; ++c) grad_bg[c] = 0.f;
  for (int64_t i = gid; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (ntiles[i] == 1) continue;
    for (int c = 0; c < C; ++c) grad_feat[i * C + c] = 0.f;
    grad_opacity[i] = 0.f;
    grad_uv[i] = make_float2(0.f, 0.f);
  }
}

// u = fx X/Z + cx, v = fy Y/Z + cy, (X, Y, Z) = R p + t.
__global__ __launch_bounds__(kBlock) void k_project_bwd(Cam cam, int64_t n,
                                                        const float* __restrict__ pos,
                                                        const uint32_t* __restrict__ ntiles,
                                                        const float2* __restrict__ grad_uv,
                                                        float* __restrict__ grad_pos) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    float g0 = 0.f, g1 = 0.f, g2 = 0.f;
    if (ntiles[i] != 0) {
      const Proj p = project_point(cam, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]);
      const float2 g = grad_uv[i];
      const float iz = 1.0f / p.Z;
      const float gx = g.x * cam.fx * iz;
      const float gy = g.y * cam.fy * iz;
      const float gz = -(gx * p.X + gy * p.Y) * iz;
      g0 = cam.R[0] * gx + cam.R[3] * gy + cam.R[6] * gz;
      g1 = cam.R[1] * gx + cam.R[4] * gy + cam.R[7] * gz;
      g2 = cam.R[2] * gx + cam.R[5] * gy + cam.R[8] * gz;
    }
    grad_pos[3 * i] = g0;
    grad_pos[3 * i + 1] = g1;
    grad_pos[3 * i + 2] = g2;
  }
}

int grid_for(int64_t n, int block) {
  const int64_t g = (n + block - 1) / block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 1 << 20));
}

}  // namespace

hipError_t launch_clear(uint32_t* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_clear, dim3((unsigned)std::min<size_t>((n + 255) / 256, 4096)), dim3(256), 0, s,
                     p, n);
  return hipGetLastError();
}

hipError_t launch_project(const Cam& cam, const Opts& o, int64_t n, const float* pos,
                          const float* radius, float* uv, uint32_t* key, uint32_t* ntiles,
                          const Ws& ws, hipStream_t s) {
  const int64_t nt = (int64_t)o.ntx * o.nty;
  hipError_t e = launch_clear(ws.tile_count, (size_t)nt, s);
  if (e != hipSuccess) return e;
  e = launch_clear(ws.flags, kFlagSlots, s);
  if (e != hipSuccess) return e;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_project, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, cam, o, n, pos,
                     radius, reinterpret_cast<float2*>(uv), key, ntiles, ws.tile_count);
  return hipGetLastError();
}

hipError_t launch_bin(const Cam& cam, const Opts& o, int64_t n, const float* uv,
                      const float* radius, const uint32_t* key, const uint32_t* ntiles,
                      uint32_t* ranges, const Ws& ws, hipStream_t s) {
  const int64_t nt = (int64_t)o.ntx * o.nty;
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, nt, ws.tile_count, ranges, ws.cursor, ws);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n == 0) return e;
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, cam, o, n,
                     reinterpret_cast<const float2*>(uv), radius, key, ntiles, ws.cursor, ws.bkey,
                     ws.bidx, ws.cap, ws.flags);
  return hipGetLastError();
}

hipError_t launch_grad_init(int64_t n, int C, const uint32_t* ntiles, float* grad_feat,
                            float* grad_opacity, float* grad_uv, float* grad_bg, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_init, dim3(grid_for(std::max<int64_t>(n, 1), kBlock)), dim3(kBlock), 0, s,
                     n, C, ntiles, grad_feat, grad_opacity, reinterpret_cast<float2*>(grad_uv),
                     grad_bg);
  return hipGetLastError();
}

hipError_t launch_project_backward(const Cam& cam, int64_t n, const float* pos,
                                   const uint32_t* ntiles, const float* grad_uv, float* grad_pos,
                                   hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_project_bwd, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, cam, n, pos,
                     ntiles, reinterpret_cast<const float2*>(grad_uv), grad_pos);
  return hipGetLastError();
}

}  // namespace inpc
