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
constexpr int kUnroll = 4;       // points per thread and round in those blocks

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

__device__ __forceinline__ TileRect project_one(const Cam& cam, const Opts& o, int sh, float x,
                                                float y, float z, float rad, int64_t i, float op,
                                                bool live, float4* __restrict__ proj,
                                                uint32_t* __restrict__ key,
                                                uint32_t* __restrict__ ntiles) {
  const Proj p = project_point(cam, x, y, z);
  // the record's last slot: the radius, or for world-space Gaussians the
  // depth their projected covariance is recomputed from
  const float w = o.splat == INPC_SPLAT_EWA ? p.Z : rad;
  Footprint f;
  f.visible = false;
  if (p.in_front && live) f = footprint(o, cam, p.u, p.v, w);
  proj[i] = make_float4(p.u, p.v, op, w);
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
__global__ __launch_bounds__(kBinBlock) void k_project_count(Cam cam, Opts o, Ring ring,
                                                             int64_t n, int64_t chunk,
                                                             const float* __restrict__ pos,
                                                             const float* __restrict__ opacity,
                                                             const float* __restrict__ radius,
                                                             float4* __restrict__ proj,
                                                             uint32_t* __restrict__ key,
                                                             uint32_t* __restrict__ ntiles,
                                                             uint32_t* __restrict__ blk,
                                                             uint32_t* __restrict__ flags) {
  __shared__ uint32_t bins[kLdsBins];
  const int nt = o.ntx * o.nty;
  // the per-build counters of the workspace start at zero (no other block of
  // this kernel reads them); the overflow flag is sticky: only
  // inpc_check_sync, which reports it, clears it
  if (blockIdx.x == 0 && threadIdx.x < kFlagSlots && threadIdx.x != kFlagOverflow)
    flags[threadIdx.x] = 0u;
  for (int t = threadIdx.x; t < nt; t += kBinBlock) bins[t] = 0u;
  __syncthreads();
  const int sh = tile_shift(o.T);
  const Chunk c = chunk_of(n, chunk);
  // kUnroll points per thread and round: their loads are all in flight
  // before the first is used
  for (int64_t i0 = c.begin + threadIdx.x; i0 < c.end; i0 += kUnroll * kBinBlock) {
    float x[kUnroll], y[kUnroll], z[kUnroll], rad[kUnroll], op[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const int64_t i = i0 + (int64_t)k * kBinBlock;
      const int64_t j = i < c.end ? i : c.begin;
      x[k] = pos[3 * j]; y[k] = pos[3 * j + 1]; z[k] = pos[3 * j + 2];
      rad[k] = radius ? radius[j] : 0.f;
      op[k] = opacity[j];
    }
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const int64_t i = i0 + (int64_t)k * kBinBlock;
      if (i >= c.end) break;
      const TileRect r =
          project_one(cam, o, sh, x[k], y[k], z[k], rad[k], i, op[k], ring_live(ring, i), proj,
                      key, ntiles);
      for (int ty = r.ty0; ty <= r.ty1; ++ty)
        for (int tx = r.tx0; tx <= r.tx1; ++tx) atomicAdd(&bins[ty * o.ntx + tx], 1u);
    }
  }
  __syncthreads();
  uint32_t* row = blk + (size_t)blockIdx.x * nt;
  for (int t = threadIdx.x; t < nt; t += kBinBlock) row[t] = bins[t];
}

__device__ __forceinline__ int sort_class(uint32_t c) {
  return c == 0 ? -1 : (c <= kSortCapW ? 0 : (c <= kSortCapM ? 1 : (c <= kSortCapL ? 2 : 3)));
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v, uint32_t lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t t = __shfl_up(v, o, 64);
    if (lane >= (uint32_t)o) v += t;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Lanes of the wavefront whose 6-bit value equals this lane's.
__device__ __forceinline__ uint64_t match6(uint32_t k) {
  uint64_t m = ~0ull;
#pragma unroll
  for (int bit = 0; bit < 6; ++bit) {
    const uint64_t bb = __ballot((k >> bit) & 1u);
    m &= ((k >> bit) & 1u) ? bb : ~bb;
  }
  return m;
}

// Blend-order class of a tile: 0 = longest lists ... 31 = one copy, 32 =
// empty; 33 marks a lane without a tile.  A tile takes the class of the
// longest list among the four tiles of its aligned quad (tile indices 4k ..
// 4k + 3, side by side in a row), so that the four are consecutive in the
// blend order: they then run on one XCD together (see xcd_pos) and share
// the L2 lines of the image rows they read and write.  Every lane of the
// wavefront takes part (lane = tile index mod 64).
__device__ __forceinline__ uint32_t order_class(bool valid, uint32_t c) {
  uint32_t q = valid ? c : 0u;
  q = max(q, (uint32_t)__shfl_xor((int)q, 1, 64));
  q = max(q, (uint32_t)__shfl_xor((int)q, 2, 64));
  return valid ? (q ? (uint32_t)__clz(q) : 32u) : 33u;
}

// Tiles are handled in groups of 64 (one wavefront, lane = tile).  Per
// group the count pass leaves its copies, its tiles per sort class and its
// tiles per blend-order class; one small block scans these columns over the
// groups, and one wavefront per group then writes the ranges, the sort
// segments and the blend order of its tiles.  No step walks all tiles in
// sequence.
//
// Blend order: tiles by decreasing power-of-two class of their copy count (so
// that the longest lists start first and do not form a tail), ascending tile
// index inside a class.  Lanes with the same class are matched with ballots.
__device__ __forceinline__ void group_table(int64_t g, bool valid, uint32_t c, const Ws& ws,
                                            uint32_t* __restrict__ s_hist) {
  const uint32_t lane = __lane_id();
  const uint64_t sum = wave_sum_u64(valid ? c : 0u);
  const int sc = valid ? sort_class(c) : -1;
  uint32_t cls[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) cls[q] = (uint32_t)__popcll(__ballot(sc == q));
  const uint32_t k = order_class(valid, c);
  const uint64_t m = match6(k);
  if (lane < kOrderClasses) s_hist[lane] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if ((m & ((1ull << lane) - 1ull)) == 0ull) s_hist[k] = (uint32_t)__popcll(m);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (lane < kOrderClasses) ws.gord[(size_t)g * kOrderClasses + lane] = s_hist[lane];
  if (lane == 0) {
    ws.gsum[g] = sum;
#pragma unroll
    for (int q = 0; q < 4; ++q) ws.gcls[(size_t)g * 4 + q] = cls[q];
  }
}

// Per tile: exclusive prefix of the workgroup counts over the workgroups (in
// place) and the tile's total.  64 tiles per block (one tile group, see
// group_table), the rows split over 16 sets of threads.
__global__ __launch_bounds__(1024) void k_colscan(int64_t nt, int rows, uint32_t* __restrict__ blk,
                                                  uint32_t* __restrict__ tile_count, Ws ws) {
  __shared__ uint32_t s_sum[16][64];
  __shared__ uint32_t s_hist[kOrderClasses];
  const int tl = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t t = (int64_t)blockIdx.x * 64 + tl;
  const int per = (rows + 15) / 16;
  const int r0 = g * per, r1 = min(rows, r0 + per);
  uint32_t v[16];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int r = r0 + k;
    v[k] = (t < nt && r < r1) ? blk[(size_t)r * nt + t] : 0u;
    sum += v[k];
  }
  s_sum[g][tl] = sum;
  __syncthreads();
  uint32_t run = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const uint32_t x = s_sum[k][tl];
    run += k < g ? x : 0u;
    tot += x;
  }
  if (t < nt) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int r = r0 + k;
      if (r < r1) blk[(size_t)r * nt + t] = run;
      run += v[k];
    }
    if (g == 0) tile_count[t] = tot;
  }
  if (g == 0) group_table(blockIdx.x, t < nt, t < nt ? tot : 0u, ws, s_hist);
}

// Step 1 for very large tile counts: one global atomic per copy.
__global__ __launch_bounds__(kBlock) void k_project_count_global(
    Cam cam, Opts o, Ring ring, int64_t n, const float* __restrict__ pos,
    const float* __restrict__ opacity,
    const float* __restrict__ radius, float4* __restrict__ proj, uint32_t* __restrict__ key,
    uint32_t* __restrict__ ntiles,
    uint32_t* __restrict__ tile_count) {
  const int sh = tile_shift(o.T);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const TileRect r = project_one(cam, o, sh, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2],
                                   radius ? radius[i] : 0.f, i, opacity[i], ring_live(ring, i),
                                   proj, key, ntiles);
    for (int ty = r.ty0; ty <= r.ty1; ++ty)
      for (int tx = r.tx0; tx <= r.tx1; ++tx) atomicAdd(&tile_count[ty * o.ntx + tx], 1u);
  }
}


// Group tables straight from the tile counts (the global counting path, or
// no points at all).
__global__ __launch_bounds__(64) void k_groups(int64_t nt, const uint32_t* __restrict__ tile_count,
                                               Ws ws) {
  __shared__ uint32_t s_hist[kOrderClasses];
  const int64_t t = (int64_t)blockIdx.x * 64 + __lane_id();
  const bool valid = t < nt;
  group_table(blockIdx.x, valid, valid ? tile_count[t] : 0u, ws, s_hist);
}

// Exclusive scan of every group column over the groups (in place), one
// wavefront per column; the column totals (copies, sort segments per class,
// tiles per blend-order class) go to ws.coltot.  Each lane holds up to 16
// rounds of the column in registers so that their loads overlap.
__global__ __launch_bounds__(64) void k_group_scan(int64_t groups, Ws ws) {
  constexpr int kRounds = 16;
  const uint32_t lane = __lane_id();
  const int col = blockIdx.x;
  auto at = [&](int64_t g) -> size_t {
    return col < 5 ? (size_t)g * 4 + (col - 1) : (size_t)g * kOrderClasses + (col - 5);
  };
  uint32_t* colp = col == 0 ? nullptr : (col < 5 ? ws.gcls : ws.gord);
  uint64_t carry = 0;
  for (int64_t g0 = 0; g0 < groups; g0 += 64 * kRounds) {
    uint64_t v[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const int64_t g = g0 + r * 64 + lane;
      v[r] = g < groups ? (col == 0 ? ws.gsum[g] : (uint64_t)colp[at(g)]) : 0ull;
    }
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const int64_t g = g0 + r * 64 + lane;
      const uint64_t incl = wave_incl_scan_u64(v[r], lane);
      if (g < groups) {
        const uint64_t ex = carry + incl - v[r];
        if (col == 0)
          ws.gsum[g] = ex;
        else
          colp[at(g)] = (uint32_t)ex;
      }
      carry += __shfl(incl, 63, 64);
    }
  }
  if (lane == 0) ws.coltot[col] = carry;
}

// One wavefront per group of 64 tiles: tile ranges (and scatter cursors for
// the global scatter), the initial sort segments (one per non-empty tile,
// per size class) and the tiles' places in the blend order.
__global__ __launch_bounds__(64) void k_place(int64_t nt, const uint32_t* __restrict__ count,
                                              uint32_t* __restrict__ ranges,
                                              uint32_t* __restrict__ cursor,
                                              uint32_t* __restrict__ order, Ws ws) {
  const uint32_t lane = __lane_id();
  const uint64_t lt = (1ull << lane) - 1ull;
  const int64_t g = blockIdx.x;
  const int64_t t = g * 64 + lane;
  const bool valid = t < nt;
  const uint32_t c = valid ? count[t] : 0u;
  const uint64_t incl = wave_incl_scan_u64(c, lane);
  const uint32_t off = (uint32_t)(ws.gsum[g] + incl - c);
  if (valid) {
    ranges[t] = off;
    if (cursor) cursor[t] = off;
  }
  const int sc = valid ? sort_class(c) : -1;
  uint2* lists[4] = {ws.seg_w, ws.seg_m, ws.seg_b0, ws.seg_x};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint64_t mq = __ballot(sc == q);
    if (sc == q)
      lists[q][ws.gcls[(size_t)g * 4 + q] + (uint32_t)__popcll(mq & lt)] = make_uint2(off, c);
  }
  if (g == 0 && lane == 0) {
    const uint64_t total = ws.coltot[0];
    ranges[nt] = (uint32_t)total;
    ws.flags[kFlagCountW] = (uint32_t)ws.coltot[1];
    ws.flags[kFlagCountM] = (uint32_t)ws.coltot[2];
    ws.flags[kFlagCountB0] = (uint32_t)ws.coltot[3];
    ws.flags[kFlagCountX] = (uint32_t)ws.coltot[4];
    // the sort's own counters start at zero for every bin
    ws.flags[kFlagCountB1] = 0u;
    ws.flags[kFlagCountG] = 0u;
    ws.flags[kFlagCountL] = 0u;
    ws.flags[kFlagCountX2] = 0u;
    ws.flags[kFlagSplitNext0] = 0u;
    ws.flags[kFlagSplitNext1] = 0u;
    if (total > (uint64_t)ws.cap) ws.flags[kFlagOverflow] = 1u;
  }
  if (order) {
    // first order position of each class: exclusive scan of the class totals
    const uint32_t tk = lane < 33u ? (uint32_t)ws.coltot[5 + lane] : 0u;
    const uint32_t kbase = (uint32_t)wave_incl_scan_u64(tk, lane) - tk;
    const uint32_t k = order_class(valid, c);
    const uint64_t m = match6(k);
    const uint32_t cb = (uint32_t)__shfl((int)kbase, (int)(k < 33u ? k : 0u), 64);
    if (k < 33u)
      order[cb + ws.gord[(size_t)g * kOrderClasses + k] + (uint32_t)__popcll(m & lt)] =
          (uint32_t)t;
  }
}

// Index word of a bucket entry (see Ws::lbits).
__device__ __forceinline__ uint32_t entry_word(const Footprint& f, int64_t i, int tx, int ty,
                                               int T, int lbits, int pb) {
  if (!lbits) return (uint32_t)i;
  const uint32_t cx = (uint32_t)(f.x0 - tx * T + 1), cy = (uint32_t)(f.y0 - ty * T + 1);
  return ((uint32_t)i << lbits) | (cy << pb) | cx;
}

// Step 2 with per-workgroup slot ranges: workgroup b owns, in every tile's
// bucket, the run that starts at the tile's range start plus the counts of
// workgroups 0..b-1 (from the count pass); slots inside the run come from
// LDS atomics.  No global atomics.
__global__ __launch_bounds__(kBinBlock) void k_scatter(Cam cam, Opts o, int64_t n, int64_t chunk,
                                                       const float4* __restrict__ proj,
                                                       const uint32_t* __restrict__ key,
                                                       const uint32_t* __restrict__ ntiles,
                                                       const uint32_t* __restrict__ ranges,
                                                       const uint32_t* __restrict__ blk,
                                                       uint2* __restrict__ bucket, uint32_t cap,
                                                       int lbits, int pb,
                                                       const uint32_t* __restrict__ flags) {
  __shared__ uint32_t bins[kLdsBins];
  if (flags[kFlagOverflow]) return;
  const int nt = o.ntx * o.nty;
  const uint32_t* row = blk + (size_t)blockIdx.x * nt;
  for (int t = threadIdx.x; t < nt; t += kBinBlock) bins[t] = ranges[t] + row[t];
  __syncthreads();
  const int sh = tile_shift(o.T);
  const Chunk c = chunk_of(n, chunk);
  for (int64_t i0 = c.begin + threadIdx.x; i0 < c.end; i0 += kUnroll * kBinBlock) {
    uint32_t nts[kUnroll], ks[kUnroll];
    float4 ps[kUnroll];
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {  // all loads first, culled points included
      const int64_t i = i0 + (int64_t)q * kBinBlock;
      const int64_t j = i < c.end ? i : c.begin;
      nts[q] = ntiles[j];
      ps[q] = proj[j];
      ks[q] = key[j];
    }
    if (o.splat == INPC_SPLAT_BILINEAR) {
      // At most 2 x 2 tiles per point: every slot of the round is reserved
      // (independent LDS atomics, all in flight together) before the first
      // copy is stored.
      uint32_t slot[kUnroll][4], word[kUnroll][4];
      bool put[kUnroll][4];
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
        const int64_t i = i0 + (int64_t)q * kBinBlock;
        const bool live = i < c.end && nts[q] != 0;
        const Footprint f = bilinear_footprint(ps[q].x, ps[q].y, cam.W, cam.H);
        const TileRect r = tile_rect(f, sh);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int tx = r.tx0 + (k & 1), ty = r.ty0 + (k >> 1);
          put[q][k] = live && tx <= r.tx1 && ty <= r.ty1;
          slot[q][k] = put[q][k] ? atomicAdd(&bins[ty * o.ntx + tx], 1u) : 0u;
          word[q][k] = entry_word(f, i, tx, ty, o.T, lbits, pb);
        }
      }
#pragma unroll
      for (int q = 0; q < kUnroll; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k)
          // always in range when the counts of step 1 hold
          if (put[q][k] && slot[q][k] < cap) bucket[slot[q][k]] = make_uint2(ks[q], word[q][k]);
      continue;
    }
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      const int64_t i = i0 + (int64_t)q * kBinBlock;
      if (i >= c.end) break;
      if (nts[q] == 0) continue;
      const Footprint f = footprint(o, cam, ps[q].x, ps[q].y, ps[q].w);
      const TileRect r = tile_rect(f, sh);
      for (int ty = r.ty0; ty <= r.ty1; ++ty)
        for (int tx = r.tx0; tx <= r.tx1; ++tx) {
          const uint32_t slot = atomicAdd(&bins[ty * o.ntx + tx], 1u);
          // always in range when the counts of step 1 hold
          if (slot < cap)
            bucket[slot] = make_uint2(ks[q], entry_word(f, i, tx, ty, o.T, lbits, pb));
        }
    }
  }
}

// Step 2 for very large tile counts: one global atomic per copy.
__global__ __launch_bounds__(kBlock) void k_scatter_global(
    Cam cam, Opts o, int64_t n, const float4* __restrict__ proj,
    const uint32_t* __restrict__ key, const uint32_t* __restrict__ ntiles,
    uint32_t* __restrict__ cursor, uint2* __restrict__ bucket, uint32_t cap, int lbits, int pb,
    const uint32_t* __restrict__ flags) {
  if (flags[kFlagOverflow]) return;
  const int sh = tile_shift(o.T);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (ntiles[i] == 0) continue;
    const float4 p = proj[i];
    const Footprint f = footprint(o, cam, p.x, p.y, p.w);
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
                                                        const float* __restrict__ grad_z,
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
      const float gz = (grad_z ? grad_z[i] : 0.f) - (gx * p.X + gy * p.Y) * iz;
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

}  // namespace

hipError_t launch_clear(uint32_t* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_clear, dim3((unsigned)std::min<size_t>((n + 255) / 256, 4096)), dim3(256),
                     0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_project(const Cam& cam, const Opts& o, int64_t n, const float* pos,
                          const float* opacity, const float* radius, float* proj, uint32_t* key,
                          uint32_t* ntiles, const Ws& ws, const Ring& ring, hipStream_t s) {
  const int64_t nt = (int64_t)o.ntx * o.nty;
  hipError_t e = hipSuccess;
  if (n == 0 || nt > kLdsBins) {  // else k_project_count clears the counters
    static_assert(kFlagOverflow == 0, "the sticky overflow flag is slot 0");
    e = launch_clear(ws.flags + 1, kFlagSlots - 1, s);
    if (e != hipSuccess) return e;
    e = launch_clear(ws.tile_count, (size_t)nt, s);
    if (e != hipSuccess) return e;
  }
  if (n == 0) {
    hipLaunchKernelGGL(k_groups, dim3((unsigned)ws.groups), dim3(64), 0, s, nt, ws.tile_count, ws);
    return hipGetLastError();
  }
  if (nt <= kLdsBins) {
    const int64_t chunk = ws.chunk, rows = ws.rows;
    hipLaunchKernelGGL(k_project_count, dim3((unsigned)rows), dim3(kBinBlock), 0, s, cam, o, ring,
                       n, chunk, pos, opacity, radius, reinterpret_cast<float4*>(proj), key, ntiles,
                       ws.blk, ws.flags);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colscan, dim3((unsigned)ws.groups), dim3(1024), 0, s, nt, (int)rows,
                       ws.blk, ws.tile_count, ws);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_project_count_global, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, cam, o,
                     ring, n, pos, opacity, radius, reinterpret_cast<float4*>(proj), key, ntiles,
                     ws.tile_count);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_groups, dim3((unsigned)ws.groups), dim3(64), 0, s, nt, ws.tile_count, ws);
  return hipGetLastError();
}

hipError_t launch_bin(const Cam& cam, const Opts& o, int64_t n, const float* proj,
                      const uint32_t* key, const uint32_t* ntiles,
                      uint32_t* ranges, uint32_t* order, const Ws& ws, hipStream_t s) {
  const int64_t nt = (int64_t)o.ntx * o.nty;
  hipLaunchKernelGGL(k_group_scan, dim3(1 + 4 + kOrderClasses), dim3(64), 0, s, ws.groups, ws);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_place, dim3((unsigned)ws.groups), dim3(64), 0, s, nt, ws.tile_count, ranges,
                     nt <= kLdsBins ? nullptr : ws.cursor, order, ws);
  e = hipGetLastError();
  if (e != hipSuccess || n == 0) return e;
  if (nt <= kLdsBins) {
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)ws.rows), dim3(kBinBlock), 0, s, cam, o, n,
                       ws.chunk, reinterpret_cast<const float4*>(proj), key, ntiles,
                       ranges, ws.blk, ws.bucket, ws.cap, ws.lbits, ws.pb, ws.flags);
  } else {
    hipLaunchKernelGGL(k_scatter_global, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, cam, o, n,
                       reinterpret_cast<const float4*>(proj), key, ntiles, ws.cursor,
                       ws.bucket, ws.cap, ws.lbits, ws.pb, ws.flags);
  }
  return hipGetLastError();
}

hipError_t launch_project_backward(const Cam& cam, int64_t n, const float* pos,
                                   const uint32_t* ntiles, const float* grad_uv,
                                   const float* grad_z, float* grad_pos, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_project_bwd, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, cam, n, pos,
                     ntiles, reinterpret_cast<const float2*>(grad_uv), grad_z, grad_pos);
  return hipGetLastError();
}

}  // namespace inpc
