// Projection, tile counting, binning and the projection's backward pass.
//
// Step 1 (Sec. 2 and Sec. 3.2 of the paper): every point is moved into
// camera space, projected, culled against the near plane and the image, and
// given its 32-bit depth key and the set of tiles its footprint meets.
// Step 2 (Sec. 3.2, "Tiled Rendering"): one exclusive scan over the per-tile
// copy counts places every tile's bucket; every visible point then drops one
// (depth key, index) copy into the bucket of each tile it touches.  The
// order inside a bucket is irrelevant because the sort that follows orders
// every bucket by the unique pair (depth key, point index).
//
// Counting and slot reservation are privatised per workgroup: a workgroup
// histograms the tiles of a large chunk of points in LDS and then issues one
// global atomic per non-empty tile, instead of one per copy.  The points are
// in random order, so hot tiles (thousands of copies) would otherwise
// serialise on a single global counter.
#include "common.h"
#include "internal.h"

namespace inpc {
namespace {

constexpr int kBlock = 256;
constexpr int kBinBlock = 1024;  // threads of the privatised counting / scatter blocks

__device__ __forceinline__ int tile_shift(int T) { return T == 8 ? 3 : (T == 16 ? 4 : 5); }

__global__ void k_clear(uint32_t* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Project one point; returns its tile rectangle (empty when culled).
struct TileRect {
  int tx0, ty0, tx1, ty1;
  __device__ __forceinline__ uint32_t count() const {
    return tx1 < tx0 ? 0u : (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
  }
};

__device__ __forceinline__ TileRect tile_rect(const Footprint& f, int sh) {
  TileRect r;
  if (!f.visible) {
    r.tx0 = r.ty0 = 0;
    r.tx1 = r.ty1 = -1;
    return r;
  }
  r.tx0 = f.px0 >> sh; r.tx1 = f.px1 >> sh;
  r.ty0 = f.py0 >> sh; r.ty1 = f.py1 >> sh;
  return r;
}

__device__ __forceinline__ TileRect project_one(const Cam& cam, const Opts& o, int sh,
                                                const float* __restrict__ pos,
                                                const float* __restrict__ radius, int64_t i,
                                                float2* __restrict__ uv,
                                                uint32_t* __restrict__ key,
                                                uint32_t* __restrict__ ntiles) {
  const float x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
  const Proj p = project_point(cam, x, y, z);
  Footprint f;
  f.visible = false;
  if (p.in_front) f = footprint(o, cam, p.u, p.v, radius ? radius[i] : 0.f);
  uv[i] = make_float2(p.u, p.v);
  key[i] = __float_as_uint(p.Z);
  const TileRect r = tile_rect(f, sh);
  ntiles[i] = r.count();
  return r;
}

// Points [b * chunk, (b + 1) * chunk) of block b.
struct Chunk {
  int64_t begin, end;
};
__device__ __forceinline__ Chunk chunk_of(int64_t n, int64_t chunk) {
  Chunk c;
  c.begin = (int64_t)blockIdx.x * chunk;
  c.end = c.begin + chunk < n ? c.begin + chunk : n;
  return c;
}

// Step 1 with per-workgroup tile histograms in LDS (nt <= kLdsBins).
__global__ __launch_bounds__(kBinBlock) void k_project_count(Cam cam, Opts o, int64_t n,
                                                             int64_t chunk,
                                                             const float* __restrict__ pos,
                                                             const float* __restrict__ radius,
                                                             float2* __restrict__ uv,
                                                             uint32_t* __restrict__ key,
                                                             uint32_t* __restrict__ ntiles,
                                                             uint32_t* __restrict__ tile_count) {
  __shared__ uint32_t bins[kLdsBins];
  const int nt = o.ntx * o.nty;
  for (int t = threadIdx.x; t < nt; t += kBinBlock) bins[t] = 0u;
  __syncthreads();
  const int sh = tile_shift(o.T);
  const Chunk c = chunk_of(n, chunk);
  for (int64_t i = c.begin + threadIdx.x; i < c.end; i += kBinBlock) {
    const TileRect r = project_one(cam, o, sh, pos, radius, i, uv, key, ntiles);
    for (int ty = r.ty0; ty <= r.ty1; ++ty)
      for (int tx = r.tx0; tx <= r.tx1; ++tx) atomicAdd(&bins[ty * o.ntx + tx], 1u);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nt; t += kBinBlock) {
    const uint32_t v = bins[t];
    if (v) atomicAdd(&tile_count[t], v);
  }
}

// Step 1 for very large tile counts: one global atomic per copy.
__global__ __launch_bounds__(kBlock) void k_project_count_global(
    Cam cam, Opts o, int64_t n, const float* __restrict__ pos, const float* __restrict__ radius,
    float2* __restrict__ uv, uint32_t* __restrict__ key, uint32_t* __restrict__ ntiles,
    uint32_t* __restrict__ tile_count) {
  const int sh = tile_shift(o.T);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const TileRect r = project_one(cam, o, sh, pos, radius, i, uv, key, ntiles);
    for (int ty = r.ty0; ty <= r.ty1; ++ty)
      for (int tx = r.tx0; tx <= r.tx1; ++tx) atomicAdd(&tile_count[ty * o.ntx + tx], 1u);
  }
}

__device__ __forceinline__ int sort_class(uint32_t c) {
  return c == 0 ? -1 : (c <= kSortCapW ? 0 : (c <= kSortCapM ? 1 : (c <= kSortCapL ? 2 : 3)));
}

// Inclusive scan of one 64-bit value per thread over a 1024-thread block;
// also returns the block total.
__device__ uint64_t block_incl_scan_u64(uint64_t v, uint64_t* s_wave, uint64_t& total) {
  const uint32_t lane = __lane_id(), w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t t = __shfl_up(v, o, 64);
    if (lane >= (uint32_t)o) v += t;
  }
  if (lane == 63) s_wave[w] = v;
  __syncthreads();
  uint64_t pre = 0;
  total = 0;
  for (uint32_t k = 0; k < 16; ++k) {
    const uint64_t x = s_wave[k];
    if (k < w) pre += x;
    total += x;
  }
  __syncthreads();
  return v + pre;
}

// Single 1024-thread block: ranges = exclusive scan of the tile counts,
// scatter cursors, and the initial sort segments (one per non-empty tile, in
// tile order, per size class), in chunks of 8192 tiles (8 consecutive tiles
// per thread).  Flags an overflow when the copies exceed the capacity.
__global__ __launch_bounds__(1024) void k_scan(int64_t nt, const uint32_t* __restrict__ count,
                                               uint32_t* __restrict__ ranges,
                                               uint32_t* __restrict__ cursor,
                                               uint32_t* __restrict__ order, Ws ws) {
  __shared__ uint64_t s_wave[16];
  constexpr int PER = 8;
  uint64_t base = 0;                       // copies before this chunk
  uint32_t cb[4] = {0u, 0u, 0u, 0u};       // class list sizes before this chunk
  uint2* lists[4] = {ws.seg_w, ws.seg_m, ws.seg_b0, ws.seg_x};
  for (int64_t c0 = 0; c0 < nt; c0 += 1024 * PER) {
    const int64_t b = c0 + (int64_t)threadIdx.x * PER;
    uint32_t v[PER];
    uint64_t tot = 0, cls = 0;  // class counts packed 16 bits each (<= 8192 per chunk)
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      v[k] = b + k < nt ? count[b + k] : 0u;
      tot += v[k];
      const int c = sort_class(v[k]);
      if (c >= 0) cls += 1ull << (16 * c);
    }
    uint64_t tot_all, cls_all;
    uint64_t off = block_incl_scan_u64(tot, s_wave, tot_all) - tot + base;
    uint64_t coff = block_incl_scan_u64(cls, s_wave, cls_all) - cls;
    uint32_t pos[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) pos[c] = cb[c] + (uint32_t)((coff >> (16 * c)) & 0xffffu);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      if (b + k >= nt) break;
      ranges[b + k] = (uint32_t)off;
      cursor[b + k] = (uint32_t)off;
      const int c = sort_class(v[k]);
      if (c >= 0) lists[c][pos[c]++] = make_uint2((uint32_t)off, v[k]);
      off += v[k];
    }
    base += tot_all;
#pragma unroll
    for (int c = 0; c < 4; ++c) cb[c] += (uint32_t)((cls_all >> (16 * c)) & 0xffffu);
  }
  if (threadIdx.x == 0) {
    ranges[nt] = (uint32_t)base;
    ws.flags[kFlagCountW] = cb[0];
    ws.flags[kFlagCountM] = cb[1];
    ws.flags[kFlagCountB0] = cb[2];
    ws.flags[kFlagCountX] = cb[3];
    if (base > (uint64_t)ws.cap) ws.flags[kFlagOverflow] = 1u;
  }
  if (!order) return;
  // Blend order: tiles by decreasing copy count in power-of-two classes (so
  // the longest lists start first and do not form a tail), ascending tile
  // index inside a class.  A stable counting sort over 33 classes; lanes of
  // a wavefront with the same class are matched with ballots so that one
  // lane per class and wavefront touches the shared counters.
  __shared__ uint32_t s_h[34];
  __shared__ uint32_t s_wc[16][34];
  const uint32_t lane = __lane_id(), w = threadIdx.x >> 6;
  const uint64_t lt = (1ull << lane) - 1ull;
  auto klass = [&](int64_t t) -> uint32_t {  // 0 = longest ... 32 = empty, 33 = no tile
    if (t >= nt) return 33u;
    const uint32_t c = count[t];
    return c ? (uint32_t)__clz(c) : 32u;
  };
  auto match6 = [&](uint32_t k) {
    uint64_t m = ~0ull;
#pragma unroll
    for (int bit = 0; bit < 6; ++bit) {
      const uint64_t bb = __ballot((k >> bit) & 1u);
      m &= ((k >> bit) & 1u) ? bb : ~bb;
    }
    return m;
  };
  if (threadIdx.x < 34) s_h[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t t0 = 0; t0 < nt; t0 += 1024) {
    const uint32_t k = klass(t0 + threadIdx.x);
    const uint64_t m = match6(k);
    if ((m & lt) == 0ull && k < 33u) atomicAdd(&s_h[k], (uint32_t)__popcll(m));
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int b = 0; b < 34; ++b) {
      const uint32_t h = s_h[b];
      s_h[b] = acc;
      acc += h;
    }
  }
  for (int64_t t0 = 0; t0 < nt; t0 += 1024) {
    for (int i = threadIdx.x; i < 16 * 34; i += 1024) (&s_wc[0][0])[i] = 0u;
    __syncthreads();
    const int64_t t = t0 + threadIdx.x;
    const uint32_t k = klass(t);
    const uint64_t m = match6(k);
    if ((m & lt) == 0ull) s_wc[w][k] = (uint32_t)__popcll(m);
    __syncthreads();
    if (k < 33u) {
      uint32_t pos = s_h[k] + (uint32_t)__popcll(m & lt);
      for (uint32_t v = 0; v < w; ++v) pos += s_wc[v][k];
      order[pos] = (uint32_t)t;
    }
    __syncthreads();
    if (threadIdx.x < 33) {
      uint32_t add = 0;
      for (int v = 0; v < 16; ++v) add += s_wc[v][threadIdx.x];
      s_h[threadIdx.x] += add;
    }
    __syncthreads();
  }
}

// Index word of a bucket entry (see Ws::lbits).
__device__ __forceinline__ uint32_t entry_word(const Footprint& f, int64_t i, int tx, int ty,
                                               int T, int lbits, int pb) {
  if (!lbits) return (uint32_t)i;
  const uint32_t cx = (uint32_t)(f.x0 - tx * T + 1), cy = (uint32_t)(f.y0 - ty * T + 1);
  return ((uint32_t)i << lbits) | (cy << pb) | cx;
}

// Step 2 with per-workgroup slot reservation: histogram the chunk's tiles in
// LDS, reserve one contiguous run per non-empty tile with a single global
// atomic, then hand out slots inside the run with LDS atomics.
__global__ __launch_bounds__(kBinBlock) void k_scatter(Cam cam, Opts o, int64_t n, int64_t chunk,
                                                       const float2* __restrict__ uv,
                                                       const float* __restrict__ radius,
                                                       const uint32_t* __restrict__ key,
                                                       const uint32_t* __restrict__ ntiles,
                                                       uint32_t* __restrict__ cursor,
                                                       uint2* __restrict__ bucket, uint32_t cap,
                                                       int lbits, int pb,
                                                       const uint32_t* __restrict__ flags) {
  __shared__ uint32_t bins[kLdsBins];
  if (flags[kFlagOverflow]) return;
  const int nt = o.ntx * o.nty;
  for (int t = threadIdx.x; t < nt; t += kBinBlock) bins[t] = 0u;
  __syncthreads();
  const int sh = tile_shift(o.T);
  const Chunk c = chunk_of(n, chunk);
  for (int64_t i = c.begin + threadIdx.x; i < c.end; i += kBinBlock) {
    if (ntiles[i] == 0) continue;
    const float2 p = uv[i];
    const TileRect r = tile_rect(footprint(o, cam, p.x, p.y, radius ? radius[i] : 0.f), sh);
    for (int ty = r.ty0; ty <= r.ty1; ++ty)
      for (int tx = r.tx0; tx <= r.tx1; ++tx) atomicAdd(&bins[ty * o.ntx + tx], 1u);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nt; t += kBinBlock) {
    const uint32_t v = bins[t];
    if (v) bins[t] = atomicAdd(&cursor[t], v);
  }
  __syncthreads();
  for (int64_t i = c.begin + threadIdx.x; i < c.end; i += kBinBlock) {
    if (ntiles[i] == 0) continue;
    const float2 p = uv[i];
    const Footprint f = footprint(o, cam, p.x, p.y, radius ? radius[i] : 0.f);
    const TileRect r = tile_rect(f, sh);
    const uint32_t k = key[i];
    for (int ty = r.ty0; ty <= r.ty1; ++ty)
      for (int tx = r.tx0; tx <= r.tx1; ++tx) {
        const uint32_t slot = atomicAdd(&bins[ty * o.ntx + tx], 1u);
        // always in range when the counts of step 1 hold
        if (slot < cap) bucket[slot] = make_uint2(k, entry_word(f, i, tx, ty, o.T, lbits, pb));
      }
  }
}

// Step 2 for very large tile counts: one global atomic per copy.
__global__ __launch_bounds__(kBlock) void k_scatter_global(
    Cam cam, Opts o, int64_t n, const float2* __restrict__ uv, const float* __restrict__ radius,
    const uint32_t* __restrict__ key, const uint32_t* __restrict__ ntiles,
    uint32_t* __restrict__ cursor, uint2* __restrict__ bucket, uint32_t cap, int lbits, int pb,
    const uint32_t* __restrict__ flags) {
  if (flags[kFlagOverflow]) return;
  const int sh = tile_shift(o.T);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (ntiles[i] == 0) continue;
    const float2 p = uv[i];
    const Footprint f = footprint(o, cam, p.x, p.y, radius ? radius[i] : 0.f);
    const TileRect r = tile_rect(f, sh);
    const uint32_t k = key[i];
    for (int ty = r.ty0; ty <= r.ty1; ++ty)
      for (int tx = r.tx0; tx <= r.tx1; ++tx) {
        const uint32_t slot = atomicAdd(&cursor[ty * o.ntx + tx], 1u);
        if (slot < cap) bucket[slot] = make_uint2(k, entry_word(f, i, tx, ty, o.T, lbits, pb));
      }
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

// Points per privatised block: one wave of blocks over the whole GPU for
// large clouds, at least 8192 points per block so the per-block flush of the
// tile histogram stays small next to the copies it replaces.
int64_t bin_chunk(int64_t n) {
  const int64_t per = (n + 255) / 256;
  const int64_t c = std::max<int64_t>(8192, per);
  return (c + kBinBlock - 1) / kBinBlock * kBinBlock;
}

}  // namespace

hipError_t launch_clear(uint32_t* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_clear, dim3((unsigned)std::min<size_t>((n + 255) / 256, 4096)), dim3(256),
                     0, s, p, n);
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
  if (nt <= kLdsBins) {
    const int64_t chunk = bin_chunk(n);
    hipLaunchKernelGGL(k_project_count, dim3((unsigned)((n + chunk - 1) / chunk)), dim3(kBinBlock),
                       0, s, cam, o, n, chunk, pos, radius, reinterpret_cast<float2*>(uv), key,
                       ntiles, ws.tile_count);
  } else {
    hipLaunchKernelGGL(k_project_count_global, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, cam,
                       o, n, pos, radius, reinterpret_cast<float2*>(uv), key, ntiles,
                       ws.tile_count);
  }
  return hipGetLastError();
}

hipError_t launch_bin(const Cam& cam, const Opts& o, int64_t n, const float* uv,
                      const float* radius, const uint32_t* key, const uint32_t* ntiles,
                      uint32_t* ranges, uint32_t* order, const Ws& ws, hipStream_t s) {
  const int64_t nt = (int64_t)o.ntx * o.nty;
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, nt, ws.tile_count, ranges, ws.cursor,
                     order, ws);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n == 0) return e;
  if (nt <= kLdsBins) {
    const int64_t chunk = bin_chunk(n);
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)((n + chunk - 1) / chunk)), dim3(kBinBlock), 0, s,
                       cam, o, n, chunk, reinterpret_cast<const float2*>(uv), radius, key, ntiles,
                       ws.cursor, ws.bucket, ws.cap, ws.lbits, ws.pb, ws.flags);
  } else {
    hipLaunchKernelGGL(k_scatter_global, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, cam, o, n,
                       reinterpret_cast<const float2*>(uv), radius, key, ntiles, ws.cursor,
                       ws.bucket, ws.cap, ws.lbits, ws.pb, ws.flags);
  }
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
