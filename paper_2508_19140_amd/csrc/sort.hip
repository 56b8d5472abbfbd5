// Per-tile depth sort.
//
// Sec. 3.2 of the paper splits sorting into a stable depth sort of the
// points followed by a stable sort of the per-tile copies by tile id, which
// leaves every tile's copies ordered by (depth key, point index).  Here the
// copies are first bucketed by tile (inpc_bin) and every bucket is then
// sorted on its own, which yields the same order with far less memory
// traffic: the bucket of a tile is loaded once, sorted in LDS and written
// once.
//
// Each bucket is sorted by an LSD radix sort on the depth key minus the
// bucket's smallest key (8-bit digits, only as many passes as the key range
// needs).  Ranks inside a wavefront come from 8 ballots per element (the
// lanes sharing a digit), so no element order is ever decided by an atomic.
// Equal depth keys are then put in point-index order; a bucket with a long
// run of equal keys is re-sorted on the full (key, index) pair instead.
//
// Size classes (chosen per tile by inpc_bin):
//   W: n <= 256    one wavefront per tile, 4 elements per lane
//   M: n <= 2048   256 threads, 8 elements per lane
//   L: n <= 16384  1024 threads, 16 elements per lane
//   X: larger      1024 threads, rounds of 16384 through global memory
#include "common.h"
#include "internal.h"

namespace inpc {
namespace {

constexpr int kRunMax = 64;  // longest run of equal keys fixed in place

template <bool WAVE_ONLY>
__device__ __forceinline__ void bsync() {
  if constexpr (WAVE_ONLY) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  } else {
    __syncthreads();
  }
}

// Lanes of the wave whose 8-bit digit equals this lane's.
__device__ __forceinline__ uint64_t match8(uint32_t d) {
  uint64_t m = ~0ull;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bal = __ballot(bit);
    m &= bit ? bal : ~bal;
  }
  return m;
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
  return v;
}
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
  return v;
}
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= (uint32_t)__shfl_xor((int)v, o, 64);
  return v;
}

// Inclusive scan over the 64 lanes.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const uint32_t lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = (uint32_t)__shfl_up((int)v, o, 64);
    if (lane >= (uint32_t)o) v += t;
  }
  return v;
}

__device__ __forceinline__ uint32_t nbits(uint32_t range) { return range ? 32u - __clz(range) : 0u; }

struct Digits {
  int nidx;        // passes over (idx - imin) digits, run first
  int nkey;        // passes over (key - kmin) digits
  uint32_t imin, kmin;
  __device__ __forceinline__ uint32_t get(uint32_t key, uint32_t idx, int p) const {
    return p < nidx ? ((idx - imin) >> (8 * p)) & 255u : ((key - kmin) >> (8 * (p - nidx))) & 255u;
  }
  __device__ __forceinline__ int passes() const { return nidx + nkey; }
};

// Shared-memory layout of one sorter (one tile at a time).
struct SortSmem {
  uint32_t* key;   // [CAP]
  uint32_t* idx;   // [CAP]
  uint32_t* hist;  // [NW * 256]
  uint32_t* off;   // [256] digit offsets / running bases
  uint32_t* red;   // [32] reduction scratch
};

// Rank every element among the NW*ITEMS*64 striped elements by digit,
// stably.  Element (w, j, lane) has position w*ITEMS*64 + j*64 + lane.
// With `running`, digit bases come from sm.off (and are advanced by this
// round's totals); otherwise they are the exclusive scan of the totals.
template <int NW, int ITEMS, bool WAVE_ONLY>
__device__ __forceinline__ void block_rank(const uint32_t (&d)[ITEMS], const bool (&valid)[ITEMS],
                                           uint32_t (&rank)[ITEMS], const SortSmem& sm,
                                           bool running) {
  const uint32_t lane = __lane_id();
  const uint32_t w = WAVE_ONLY ? 0u : (threadIdx.x >> 6);
  uint32_t* hist = sm.hist + w * 256;
  for (uint32_t k = lane; k < 256; k += 64) hist[k] = 0;
  bsync<true>();
  uint32_t local[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const uint64_t m = match8(d[j]) & __ballot(valid[j]);
    const uint32_t pre = valid[j] ? hist[d[j]] : 0u;
    local[j] = pre + mbcnt64(m);
    const bool leader = valid[j] && (mbcnt64(m) == 0);
    if (leader) hist[d[j]] = pre + (uint32_t)__popcll(m);
    bsync<true>();
  }
  bsync<WAVE_ONLY>();
  // per digit: exclusive prefix over waves, totals
  const int nth = WAVE_ONLY ? 64 : NW * 64;
  const int tid = WAVE_ONLY ? (int)lane : (int)threadIdx.x;
  for (int dd = tid; dd < 256; dd += nth) {
    uint32_t acc = 0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) {
      const uint32_t c = sm.hist[ww * 256 + dd];
      sm.hist[ww * 256 + dd] = acc;
      acc += c;
    }
    if (running) {
      const uint32_t base = sm.off[dd];
      sm.off[dd] = base + acc;  // next round starts after this one
      // shift this round's per-wave prefixes by the running base
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) sm.hist[ww * 256 + dd] += base;
    } else {
      sm.off[dd] = acc;  // totals, scanned below
    }
  }
  bsync<WAVE_ONLY>();
  if (!running) {
    if (WAVE_ONLY || w == 0) {
      uint32_t t4[4];
      uint32_t s = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        t4[q] = sm.off[lane * 4 + q];
        s += t4[q];
      }
      const uint32_t incl = wave_incl_scan(s);
      uint32_t e = incl - s;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        sm.off[lane * 4 + q] = e;
        e += t4[q];
      }
    }
    bsync<WAVE_ONLY>();
  }
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if (valid[j]) {
      rank[j] = local[j] + hist[d[j]] + (running ? 0u : sm.off[d[j]]);
    }
  }
  bsync<WAVE_ONLY>();
}

// Sort n <= NW*ITEMS*64 (key, idx) pairs of one tile entirely in LDS and
// write the point indices in (key, idx) order to out[0..n).
template <int NW, int ITEMS, bool WAVE_ONLY>
__device__ void sort_tile_lds(const uint32_t* __restrict__ gkey, const uint32_t* __restrict__ gidx,
                              uint32_t n, uint32_t* __restrict__ out, const SortSmem& sm) {
  constexpr int PER_WAVE = ITEMS * 64;
  const uint32_t lane = __lane_id();
  const uint32_t w = WAVE_ONLY ? 0u : (threadIdx.x >> 6);
  const uint32_t base_e = w * PER_WAVE;
  const int nth = WAVE_ONLY ? 64 : NW * 64;
  const int tid = WAVE_ONLY ? (int)lane : (int)threadIdx.x;

  uint32_t key[ITEMS], idx[ITEMS], rank[ITEMS], dg[ITEMS];
  bool valid[ITEMS];
  uint32_t kmin = 0xffffffffu, kmax = 0u, imin = 0xffffffffu, imax = 0u;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const uint32_t e = base_e + j * 64 + lane;
    valid[j] = e < n;
    key[j] = valid[j] ? gkey[e] : 0u;
    idx[j] = valid[j] ? gidx[e] : 0u;
    if (valid[j]) {
      kmin = min(kmin, key[j]); kmax = max(kmax, key[j]);
      imin = min(imin, idx[j]); imax = max(imax, idx[j]);
    }
  }
  kmin = wave_min(kmin); kmax = wave_max(kmax);
  imin = wave_min(imin); imax = wave_max(imax);
  if (!WAVE_ONLY) {
    if (lane == 0) {
      sm.red[w * 4 + 0] = kmin; sm.red[w * 4 + 1] = kmax;
      sm.red[w * 4 + 2] = imin; sm.red[w * 4 + 3] = imax;
    }
    __syncthreads();
    kmin = 0xffffffffu; kmax = 0; imin = 0xffffffffu; imax = 0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) {
      kmin = min(kmin, sm.red[ww * 4 + 0]); kmax = max(kmax, sm.red[ww * 4 + 1]);
      imin = min(imin, sm.red[ww * 4 + 2]); imax = max(imax, sm.red[ww * 4 + 3]);
    }
    __syncthreads();
  }
  Digits dp;
  dp.kmin = kmin;
  dp.imin = imin;
  dp.nkey = (int)((nbits(kmax - kmin) + 7) / 8);
  dp.nidx = 0;

  for (int attempt = 0; attempt < 2; ++attempt) {
    if (attempt == 1) {
      // long runs of equal keys: sort the full (key, index) pair, starting
      // again from the unsorted bucket
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const uint32_t e = base_e + j * 64 + lane;
        key[j] = valid[j] ? gkey[e] : 0u;
        idx[j] = valid[j] ? gidx[e] : 0u;
      }
      dp.nidx = (int)((nbits(imax - imin) + 7) / 8);
    }
    const int np = dp.passes();
    for (int p = 0; p < np; ++p) {
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) dg[j] = dp.get(key[j], idx[j], p);
      block_rank<NW, ITEMS, WAVE_ONLY>(dg, valid, rank, sm, false);
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        if (valid[j]) {
          sm.key[rank[j]] = key[j];
          sm.idx[rank[j]] = idx[j];
        }
      }
      bsync<WAVE_ONLY>();
      if (p + 1 < np) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
          const uint32_t e = base_e + j * 64 + lane;
          if (valid[j]) {
            key[j] = sm.key[e];
            idx[j] = sm.idx[e];
          }
        }
        bsync<WAVE_ONLY>();
      }
    }
    if (np == 0) {
      // a single key value: the order is the index order
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const uint32_t e = base_e + j * 64 + lane;
        if (valid[j]) {
          sm.key[e] = key[j];
          sm.idx[e] = idx[j];
        }
      }
      bsync<WAVE_ONLY>();
    }
    if (dp.nidx > 0) break;  // full-pair sort: no ties left to fix
    // Runs of equal keys: order them by point index.
    uint32_t long_run = 0;
    for (uint32_t e = tid; e < n; e += nth) {
      const uint32_t k = sm.key[e];
      const bool starts = (e == 0 || sm.key[e - 1] != k) && (e + 1 < n && sm.key[e + 1] == k);
      if (!starts) continue;
      uint32_t end = e + 1;
      while (end < n && sm.key[end] == k && end - e <= (uint32_t)kRunMax) ++end;
      if (end - e > (uint32_t)kRunMax) {
        long_run = 1;
        continue;
      }
      for (uint32_t a = e + 1; a < end; ++a) {  // insertion sort by index
        const uint32_t v = sm.idx[a];
        uint32_t b = a;
        while (b > e && sm.idx[b - 1] > v) {
          sm.idx[b] = sm.idx[b - 1];
          --b;
        }
        sm.idx[b] = v;
      }
    }
    long_run = wave_or(long_run);
    if (!WAVE_ONLY) {
      if (lane == 0) sm.red[w] = long_run;
      __syncthreads();
      long_run = 0;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) long_run |= sm.red[ww];
      __syncthreads();
    } else {
      bsync<true>();
    }
    if (!long_run) break;
    bsync<WAVE_ONLY>();
  }
  for (uint32_t e = tid; e < n; e += nth) out[e] = sm.idx[e];
  bsync<WAVE_ONLY>();
}

// Class W: one wavefront per tile, four tiles per 256-thread block.
constexpr int kW_ITEMS = 4;
constexpr int kW_CAP = kW_ITEMS * 64;

__global__ __launch_bounds__(256) void k_sort_w(const uint32_t* __restrict__ ranges,
                                                const uint32_t* __restrict__ tiles,
                                                const uint32_t* __restrict__ flags,
                                                const uint32_t* __restrict__ bkey,
                                                const uint32_t* __restrict__ bidx,
                                                uint32_t* __restrict__ list) {
  __shared__ uint32_t s_key[4][kW_CAP];
  __shared__ uint32_t s_idx[4][kW_CAP];
  __shared__ uint32_t s_hist[4][256];
  __shared__ uint32_t s_off[4][256];
  __shared__ uint32_t s_red[4][32];
  if (flags[kFlagOverflow]) return;
  const uint32_t w = threadIdx.x >> 6;
  SortSmem sm{s_key[w], s_idx[w], s_hist[w], s_off[w], s_red[w]};
  const uint32_t count = flags[kFlagCountW];
  for (uint32_t i = blockIdx.x * 4 + w; i < count; i += gridDim.x * 4) {
    const uint32_t t = tiles[i];
    const uint32_t s = ranges[t], n = ranges[t + 1] - s;
    sort_tile_lds<1, kW_ITEMS, true>(bkey + s, bidx + s, n, list + s, sm);
  }
}

// Classes M and L: one block per tile.
template <int NW, int ITEMS, int FLAG>
__global__ __launch_bounds__(NW * 64) void k_sort_block(const uint32_t* __restrict__ ranges,
                                                        const uint32_t* __restrict__ tiles,
                                                        const uint32_t* __restrict__ flags,
                                                        const uint32_t* __restrict__ bkey,
                                                        const uint32_t* __restrict__ bidx,
                                                        uint32_t* __restrict__ list) {
  constexpr int CAP = NW * ITEMS * 64;
  __shared__ uint32_t s_key[CAP];
  __shared__ uint32_t s_idx[CAP];
  __shared__ uint32_t s_hist[NW * 256];
  __shared__ uint32_t s_off[256];
  __shared__ uint32_t s_red[64];
  if (flags[kFlagOverflow]) return;
  SortSmem sm{s_key, s_idx, s_hist, s_off, s_red};
  const uint32_t count = flags[FLAG];
  for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
    const uint32_t t = tiles[i];
    const uint32_t s = ranges[t], n = ranges[t + 1] - s;
    sort_tile_lds<NW, ITEMS, false>(bkey + s, bidx + s, n, list + s, sm);
  }
}

// Class X: tiles larger than the LDS capacity.  LSD passes over the full
// (key, index) pair through global memory, in rounds of NW*ITEMS*64
// elements; each pass first histograms the whole tile so that every round
// knows where each digit's run starts.
template <int NW, int ITEMS>
__global__ __launch_bounds__(NW * 64) void k_sort_x(const uint32_t* __restrict__ ranges,
                                                    const uint32_t* __restrict__ tiles,
                                                    const uint32_t* __restrict__ flags,
                                                    uint32_t* __restrict__ bkey,
                                                    uint32_t* __restrict__ bidx,
                                                    uint32_t* __restrict__ xkey,
                                                    uint32_t* __restrict__ xidx,
                                                    uint32_t* __restrict__ list) {
  constexpr int ROUND = NW * ITEMS * 64;
  __shared__ uint32_t s_hist[NW * 256];
  __shared__ uint32_t s_off[256];
  __shared__ uint32_t s_red[64];
  __shared__ uint32_t s_glob[256];
  if (flags[kFlagOverflow]) return;
  SortSmem sm{nullptr, nullptr, s_hist, s_off, s_red};
  const uint32_t lane = __lane_id();
  const uint32_t w = threadIdx.x >> 6;
  const uint32_t count = flags[kFlagCountX];
  for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
    const uint32_t t = tiles[i];
    const uint32_t s = ranges[t], n = ranges[t + 1] - s;
    // key and index ranges
    uint32_t kmin = 0xffffffffu, kmax = 0, imin = 0xffffffffu, imax = 0;
    for (uint32_t e = threadIdx.x; e < n; e += NW * 64) {
      const uint32_t k = bkey[s + e], x = bidx[s + e];
      kmin = min(kmin, k); kmax = max(kmax, k);
      imin = min(imin, x); imax = max(imax, x);
    }
    kmin = wave_min(kmin); kmax = wave_max(kmax);
    imin = wave_min(imin); imax = wave_max(imax);
    if (lane == 0) {
      s_red[w * 4 + 0] = kmin; s_red[w * 4 + 1] = kmax;
      s_red[w * 4 + 2] = imin; s_red[w * 4 + 3] = imax;
    }
    __syncthreads();
    kmin = 0xffffffffu; kmax = 0; imin = 0xffffffffu; imax = 0;
    for (int ww = 0; ww < NW; ++ww) {
      kmin = min(kmin, s_red[ww * 4 + 0]); kmax = max(kmax, s_red[ww * 4 + 1]);
      imin = min(imin, s_red[ww * 4 + 2]); imax = max(imax, s_red[ww * 4 + 3]);
    }
    __syncthreads();
    Digits dp;
    dp.kmin = kmin;
    dp.imin = imin;
    dp.nkey = (int)((nbits(kmax - kmin) + 7) / 8);
    dp.nidx = (int)((nbits(imax - imin) + 7) / 8);
    const int np = dp.passes();
    uint32_t *sk = bkey + s, *si = bidx + s, *dk = xkey + s, *di = xidx + s;
    for (int p = 0; p < np; ++p) {
      // histogram of this pass's digit over the whole tile
      for (int k = threadIdx.x; k < 256; k += NW * 64) s_glob[k] = 0;
      __syncthreads();
      for (uint32_t e = threadIdx.x; e < n; e += NW * 64) atomicAdd(&s_glob[dp.get(sk[e], si[e], p)], 1u);
      __syncthreads();
      if (w == 0) {
        uint32_t t4[4], sum = 0;
        for (int q = 0; q < 4; ++q) { t4[q] = s_glob[lane * 4 + q]; sum += t4[q]; }
        uint32_t ex = wave_incl_scan(sum) - sum;
        for (int q = 0; q < 4; ++q) { s_off[lane * 4 + q] = ex; ex += t4[q]; }
      }
      __syncthreads();
      const bool last = p + 1 == np;
      uint32_t* out_idx = last ? list + s : di;
      for (uint32_t r0 = 0; r0 < n; r0 += ROUND) {
        uint32_t key[ITEMS], idx[ITEMS], dg[ITEMS], rank[ITEMS];
        bool valid[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
          const uint32_t e = r0 + w * ITEMS * 64 + j * 64 + lane;
          valid[j] = e < n;
          key[j] = valid[j] ? sk[e] : 0u;
          idx[j] = valid[j] ? si[e] : 0u;
          dg[j] = dp.get(key[j], idx[j], p);
        }
        block_rank<NW, ITEMS, false>(dg, valid, rank, sm, true);
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
          if (valid[j]) {
            if (!last) dk[rank[j]] = key[j];
            out_idx[rank[j]] = idx[j];
          }
        }
      }
      __syncthreads();
      if (!last) {
        uint32_t* tk = sk; sk = dk; dk = tk;
        uint32_t* ti = si; si = di; di = ti;
      }
      __threadfence_block();
      __syncthreads();
    }
    if (np == 0) {
      for (uint32_t e = threadIdx.x; e < n; e += NW * 64) list[s + e] = bidx[s + e];
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_sort(const uint32_t* ranges, const Ws& ws, uint32_t* list, int64_t nt,
                       hipStream_t stream) {
  const int grid_w = (int)std::min<int64_t>((nt + 3) / 4, 4096);
  hipLaunchKernelGGL(k_sort_w, dim3(std::max(grid_w, 1)), dim3(256), 0, stream, ranges, ws.list_w,
                     ws.flags, ws.bkey, ws.bidx, list);
  const int grid_m = (int)std::min<int64_t>(nt, 2048);
  hipLaunchKernelGGL((k_sort_block<4, 8, kFlagCountM>), dim3(std::max(grid_m, 1)), dim3(256), 0, stream,
                     ranges, ws.list_m, ws.flags, ws.bkey, ws.bidx, list);
  const int grid_l = (int)std::min<int64_t>(nt, 512);
  hipLaunchKernelGGL((k_sort_block<16, 16, kFlagCountL>), dim3(std::max(grid_l, 1)), dim3(1024), 0,
                     stream, ranges, ws.list_l, ws.flags, ws.bkey, ws.bidx, list);
  const int grid_x = (int)std::min<int64_t>(nt, 256);
  hipLaunchKernelGGL((k_sort_x<16, 16>), dim3(std::max(grid_x, 1)), dim3(1024), 0, stream, ranges,
                     ws.list_x, ws.flags, ws.bkey, ws.bidx, ws.xkey, ws.xidx, list);
  return hipGetLastError();
}

}  // namespace inpc
