// Per-tile depth sort.
//
// Sec. 3.2 of the paper splits sorting into a stable depth sort of the
// points followed by a stable sort of the per-tile copies by tile id, which
// leaves every tile's copies ordered by (depth key, point index).  Here the
// copies are first bucketed by tile (inpc_bin) and every bucket is then
// sorted on its own, which yields the same order with far less memory
// traffic: a bucket is loaded once, sorted in LDS and written once.
//
// Work items are segments [start, start + n) of the bucket array; every
// non-empty tile starts as one segment.  By size:
//   n <= 64     rank sort by one wavefront (each lane counts the smaller
//               (key, index) pairs)
//   n <= 256    bucket-rank sort by one wavefront, 4 elements per lane
//   n <= 2048   bucket-rank sort by a 256-thread block, 8 elements per lane
//               (both fall back to an LSD radix sort when a bucket is too
//               full, see bucket_sort_segment)
//   n <= 16384  MSD split: one 1024-thread block loads the segment into LDS,
//               buckets it by the top 8 bits of the (key, index) pair
//               relative to the segment's range, writes it back in place and
//               queues the sub-segments (which are then sorted on their own;
//               concatenated in digit order they give the sorted segment).
//               Small digit buckets are queued as groups of neighbouring
//               buckets rather than one by one.  Two split rounds; what is
//               still larger is sorted by a 1024-thread block (up to 8192
//               copies) or LSD-sorted through global memory.
//   larger      the same MSD split through global memory (the segment is
//               scattered into the other buffer of the pair bucket/xbucket,
//               where its sub-segments stay), two rounds, before the LDS
//               splits; whatever is still larger than 16384 copies after
//               them is LSD-sorted through global memory by a 1024-thread
//               block.  (Large Gaussian footprints give tiles of tens of
//               thousands of copies.)
//
// The LSD sorts rank elements inside a wavefront with one ballot per digit
// bit (the lanes sharing a digit), so no order is decided by an atomic.  They
// run on the depth key minus the segment's smallest key; equal keys are then
// put in index order, and a segment with a long run of equal keys is re-sorted
// on the full (key, index) pair.  Element placement by LDS atomics happens
// only in the bucketing passes (the splits and the bucket-rank sorts), whose
// buckets are then fully ordered on their own.
#include "common.h"
#include "internal.h"

namespace inpc {
namespace {

constexpr int kRunMax = 64;  // longest run of equal keys fixed in place

// A segment descriptor is (first list position, count).  Bit 31 of the count
// marks a segment whose pairs sit in the ping-pong buffer (xbucket) rather
// than in the bucket array, at the same positions: a split through global
// memory leaves its sub-segments where it scattered them.  Counts stay below
// 2^31 (a tile holds at most one copy of each point).
constexpr uint32_t kInX = 0x80000000u;
__device__ __forceinline__ uint32_t seg_count(uint2 sg) { return sg.y & ~kInX; }
template <typename P>
__device__ __forceinline__ P* seg_pairs(P* bucket, P* xbucket, uint2 sg) {
  return ((sg.y & kInX) ? xbucket : bucket) + sg.x;
}

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

// Lanes of the wave whose digit (the low `width` <= 8 bits of d, the rest
// zero) equals this lane's.  `width` is the same for every lane.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, int width) {
  uint64_t m = ~0ull;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    if (b < width) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      m &= bit ? bal : ~bal;
    }
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

// LSD digits of one segment: first the passes over (idx - imin), then over
// (key - kmin).  A field of B bits takes ceil(B / 8) passes of equal width
// (at most 8 bits), so a 25-bit key range costs 25 ballots, not 32.
struct Digits {
  int nidx, nkey;  // passes over the index and the key fields
  int widx, wkey;  // bits per pass of each field
  uint32_t imin, kmin;
  __device__ __forceinline__ void set_key(uint32_t range) {
    const uint32_t b = nbits(range);
    nkey = (int)((b + 7) / 8);
    wkey = nkey ? (int)((b + nkey - 1) / nkey) : 0;
  }
  __device__ __forceinline__ void set_idx(uint32_t range) {
    const uint32_t b = nbits(range);
    nidx = (int)((b + 7) / 8);
    widx = nidx ? (int)((b + nidx - 1) / nidx) : 0;
  }
  __device__ __forceinline__ int width(int p) const { return p < nidx ? widx : wkey; }
  __device__ __forceinline__ uint32_t get(uint32_t key, uint32_t idx, int p) const {
    if (p < nidx) return ((idx - imin) >> (widx * p)) & ((1u << widx) - 1u);
    return ((key - kmin) >> (wkey * (p - nidx))) & ((1u << wkey) - 1u);
  }
  __device__ __forceinline__ int passes() const { return nidx + nkey; }
};

// Shared-memory layout of one sorter (one segment at a time).
struct SortSmem {
  uint32_t* key;   // [CAP]
  uint32_t* idx;   // [CAP]
  uint32_t* hist;  // [NW * 256]
  uint32_t* off;   // [256] digit offsets / running bases
  uint32_t* red;   // [64] reduction scratch
};

// Rank every element among the NW*ni*64 striped elements by its digit of
// `width` bits, stably.  Element (w, j, lane) has position w*ni*64 + j*64 +
// lane; items j >= ni (ni <= ITEMS, the same for the whole block) hold no
// element and are skipped.  With `running`, digit bases come from sm.off
// (and are advanced by this round's totals); otherwise they are the
// exclusive scan of the totals.
template <int NW, int ITEMS, bool WAVE_ONLY>
__device__ __forceinline__ void block_rank(const uint32_t (&d)[ITEMS], const bool (&valid)[ITEMS],
                                           uint32_t (&rank)[ITEMS], const SortSmem& sm,
                                           bool running, int ni, int width) {
  const uint32_t lane = __lane_id();
  const uint32_t w = WAVE_ONLY ? 0u : (threadIdx.x >> 6);
  uint32_t* hist = sm.hist + w * 256;
  for (uint32_t k = lane; k < 256; k += 64) hist[k] = 0;
  bsync<true>();
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if (j >= ni) break;
    const uint64_t m = match_digit(d[j], width) & __ballot(valid[j]);
    const uint32_t pre = valid[j] ? hist[d[j]] : 0u;
    rank[j] = pre + mbcnt64(m);
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
    if (valid[j]) rank[j] += hist[d[j]] + (running ? 0u : sm.off[d[j]]);
  }
  bsync<WAVE_ONLY>();
}

// Bucket-rank sort of n <= NW*ITEMS*64 (key, idx) pairs of one segment in
// LDS: one pass splits the segment into 2^HB buckets by the top HB bits of
// the pair's offset from the segment's smallest pair, (key - kmin) followed
// by (idx - imin); then every element's place is its bucket's start plus the
// number of pairs in its bucket smaller than its own (pairs are unique, so
// this is a permutation).  No barrier separates the rank counts, and a
// segment costs one histogram, one scan and one scatter instead of a radix
// pass per digit.  Returns false (having written nothing) when a bucket holds
// more than MAXB pairs, where counting would cost more than the radix sort.
// sm.idx must follow sm.key directly (the pairs are stored as one array).
template <int NW, int ITEMS, int HB, bool WAVE_ONLY, int MAXB>
__device__ bool bucket_sort_segment(const uint2* __restrict__ seg, uint32_t n,
                                    const ListOut& out, uint32_t base, const SortSmem& sm) {
  constexpr int NB = 1 << HB;             // buckets
  constexpr int NT = WAVE_ONLY ? 64 : NW * 64;
  constexpr int BPT = NB / NT;            // buckets per thread in the scan
  static_assert(BPT >= 1 && NB % NT == 0, "bucket count must be a multiple of the threads");
  const uint32_t lane = __lane_id();
  const uint32_t w = WAVE_ONLY ? 0u : (threadIdx.x >> 6);
  const int tid = WAVE_ONLY ? (int)lane : (int)threadIdx.x;
  const int ni = (int)((n + NW * 64 - 1) / (NW * 64));
  const uint32_t base_e = w * (uint32_t)ni * 64u;
  uint32_t* hist = sm.hist;  // [NB]
  for (int b = tid; b < NB; b += NT) hist[b] = 0u;

  uint32_t key[ITEMS], idx[ITEMS], dg[ITEMS], slot[ITEMS];
  bool valid[ITEMS];
  uint32_t kmin = 0xffffffffu, kmax = 0u, imin = 0xffffffffu, imax = 0u;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const uint32_t e = base_e + j * 64 + lane;
    valid[j] = j < ni && e < n;
    const uint2 v = valid[j] ? seg[e] : make_uint2(0u, 0u);
    key[j] = v.x;
    idx[j] = v.y;
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
  }
  // digit: top HB bits of ((key - kmin) << ib) | (idx - imin)
  const uint32_t ib = nbits(imax - imin);
  const uint32_t total = nbits(kmax - kmin) + ib;
  const uint32_t sh = total > (uint32_t)HB ? total - (uint32_t)HB : 0u;
  bsync<WAVE_ONLY>();  // hist cleared, sm.red read
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if (!valid[j]) continue;
    const uint64_t c = ((uint64_t)(key[j] - kmin) << ib) | (uint64_t)(idx[j] - imin);
    dg[j] = (uint32_t)(c >> sh);
    slot[j] = atomicAdd(&hist[dg[j]], 1u);
  }
  bsync<WAVE_ONLY>();
  // exclusive scan of the bucket counts (BPT consecutive buckets per thread),
  // and the largest bucket
  uint32_t cnt[BPT];
  uint32_t sum = 0, mx = 0;
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    cnt[q] = hist[tid * BPT + q];
    sum += cnt[q];
    mx = max(mx, cnt[q]);
  }
  const uint32_t incl = wave_incl_scan(sum);
  mx = wave_max(mx);
  uint32_t wbase = 0u;
  if (!WAVE_ONLY) {
    if (lane == 63) sm.red[w] = incl;
    if (lane == 0) sm.red[NW + w] = mx;
    __syncthreads();
    mx = 0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) {
      if (ww < (int)w) wbase += sm.red[ww];
      mx = max(mx, sm.red[NW + ww]);
    }
  }
  if (mx > (uint32_t)MAXB) {
    bsync<WAVE_ONLY>();  // everybody has read hist and sm.red
    return false;
  }
  uint32_t ex = wbase + incl - sum;
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    hist[tid * BPT + q] = ex;  // bucket start
    ex += cnt[q];
  }
  bsync<WAVE_ONLY>();
  // scatter into the buckets (order inside a bucket is arbitrary); the
  // pairs go to the key and index arrays taken as one array of pairs
  uint2* kv = reinterpret_cast<uint2*>(sm.key);
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if (!valid[j]) continue;
    kv[hist[dg[j]] + slot[j]] = make_uint2(key[j], idx[j]);
  }
  bsync<WAVE_ONLY>();
  // rank inside the bucket, by position in the bucketed array: neighbouring
  // lanes mostly share a bucket, so their reads of it are broadcasts
  for (uint32_t p = tid; p < n; p += NT) {
    const uint2 v = kv[p];
    const uint64_t c = ((uint64_t)(v.x - kmin) << ib) | (uint64_t)(v.y - imin);
    const uint32_t d = (uint32_t)(c >> sh);
    const uint32_t b0 = hist[d];
    const uint32_t b1 = d + 1 < (uint32_t)NB ? hist[d + 1] : n;
    const uint64_t me = ((uint64_t)v.x << 32) | v.y;
    uint32_t r = 0;
    for (uint32_t q = b0; q < b1; ++q) {
      const uint2 o = kv[q];
      r += (((uint64_t)o.x << 32) | o.y) < me;
    }
    out.put(base + b0 + r, v.y);
  }
  bsync<WAVE_ONLY>();  // the LDS is reused by the next segment
  return true;
}

// Sort n <= NW*ITEMS*64 (key, idx) pairs of one segment entirely in LDS and
// write the point indices in (key, idx) order to out[0..n).  Each wave holds
// ni = ceil(n / (64 NW)) items per lane, so the ranking work follows the
// segment's size rather than the block's capacity.
template <int NW, int ITEMS, bool WAVE_ONLY>
__device__ void sort_segment_lds(const uint2* __restrict__ seg, uint32_t n, const ListOut& out,
                                 uint32_t base, const SortSmem& sm) {
  const uint32_t lane = __lane_id();
  const uint32_t w = WAVE_ONLY ? 0u : (threadIdx.x >> 6);
  const int ni = (int)((n + NW * 64 - 1) / (NW * 64));  // <= ITEMS as n <= NW*ITEMS*64
  const uint32_t base_e = w * (uint32_t)ni * 64u;
  const int nth = WAVE_ONLY ? 64 : NW * 64;
  const int tid = WAVE_ONLY ? (int)lane : (int)threadIdx.x;

  uint32_t key[ITEMS], idx[ITEMS], rank[ITEMS], dg[ITEMS];
  bool valid[ITEMS];
  uint32_t kmin = 0xffffffffu, kmax = 0u, imin = 0xffffffffu, imax = 0u;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const uint32_t e = base_e + j * 64 + lane;
    valid[j] = j < ni && e < n;
    const uint2 v = valid[j] ? seg[e] : make_uint2(0u, 0u);
    key[j] = v.x;
    idx[j] = v.y;
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
  dp.set_key(kmax - kmin);
  dp.nidx = dp.widx = 0;

  for (int attempt = 0; attempt < 2; ++attempt) {
    if (attempt == 1) {
      // long runs of equal keys: sort the full (key, index) pair, starting
      // again from the unsorted segment
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const uint32_t e = base_e + j * 64 + lane;
        const uint2 v = valid[j] ? seg[e] : make_uint2(0u, 0u);
        key[j] = v.x;
        idx[j] = v.y;
      }
      dp.set_idx(imax - imin);
    }
    const int np = dp.passes();
    for (int p = 0; p < np; ++p) {
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) dg[j] = dp.get(key[j], idx[j], p);
      block_rank<NW, ITEMS, WAVE_ONLY>(dg, valid, rank, sm, false, ni, dp.width(p));
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
      // a single key value: keep the loaded order, fixed below
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
  for (uint32_t e = tid; e < n; e += nth) out.put(base + e, sm.idx[e]);
  bsync<WAVE_ONLY>();
}

// n <= 64: every lane counts the (key, index) pairs smaller than its own.
// Lanes without an element publish an all-ones pair, which no element
// (key bit 31 is clear) counts as smaller, so the count runs over whole
// groups of eight with 16-byte LDS reads.
// The lane's pair of a segment of n <= 64 (all ones past the end).
__device__ __forceinline__ uint2 small_pair(const uint2* __restrict__ bucket,
                                            const uint2* __restrict__ xbucket, uint2 sg) {
  const uint32_t lane = __lane_id(), n = seg_count(sg);
  return n <= 64u && lane < n ? seg_pairs(bucket, xbucket, sg)[lane]
                              : make_uint2(0xffffffffu, 0xffffffffu);
}

// `v`: the lane's pair (small_pair).
__device__ void rank_sort_wave(uint2 v, uint32_t n, const ListOut& out, uint32_t base,
                               uint2* __restrict__ s) {
  const uint32_t lane = __lane_id();
  const bool valid = lane < n;
  s[lane] = v;
  bsync<true>();
  const uint64_t me = ((uint64_t)v.x << 32) | v.y;
  const uint4* s4 = reinterpret_cast<const uint4*>(s);
  const uint32_t groups = (n + 7u) >> 3;
  uint32_t r = 0;
  for (uint32_t g = 0; g < groups; ++g) {
    uint4 q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = s4[4 * g + k];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      r += (((uint64_t)q[k].x << 32) | q[k].y) < me;
      r += (((uint64_t)q[k].z << 32) | q[k].w) < me;
    }
  }
  if (valid) out.put(base + r, v.y);
  bsync<true>();
}

// Segments of at most 256 copies: one wavefront each, four per block (the W
// role of k_sort_wm below).
constexpr int kW_ITEMS = 4;
constexpr int kW_CAP = kW_ITEMS * 64;


// The W class (one wavefront per segment, four per block) and the M class
// (one 256-thread block per segment) in one launch: workgroups [0, gm) take
// M segments and are dispatched first (the larger sorts start first), the
// rest take W segments, so that neither class leaves a tail of idle compute
// units behind it.  Both roles carve their LDS from one arena.
constexpr int kM_NW = 4, kM_ITEMS = 8, kM_CAP = kM_NW * kM_ITEMS * 64;
// Bucket bits of the bucket-rank sorts (the bucket counts fit the radix
// histograms: 256 per wavefront) and the largest bucket worth counting in.
constexpr int kW_HB = 8, kM_HB = 10, kL_HB = 12;
constexpr int kBucketMax = 256;
constexpr int kM_WORDS = 2 * kM_CAP + kM_NW * 256 + 256 + 64;
constexpr int kW_WORDS = 2 * kW_CAP + 256 + 256 + 64;  // per wavefront
static_assert(kW_WORDS % 4 == 0, "wavefront arenas must stay 16-byte aligned");

__global__ __launch_bounds__(256, 5) void k_sort_wm(int gm, const uint2* __restrict__ seg_w,
                                                 const uint2* __restrict__ seg_m,
                                                 const uint32_t* __restrict__ flags,
                                                 const uint2* __restrict__ bucket,
                                                 const uint2* __restrict__ xbucket, ListOut out) {
  __shared__ __align__(16) uint32_t s_lds[kM_WORDS > 4 * kW_WORDS ? kM_WORDS : 4 * kW_WORDS];
  if (flags[kFlagOverflow]) return;
  if ((int)blockIdx.x < gm) {
    uint32_t* b = s_lds;
    const SortSmem sm{b, b + kM_CAP, b + 2 * kM_CAP, b + 2 * kM_CAP + kM_NW * 256,
                      b + 2 * kM_CAP + kM_NW * 256 + 256};
    const uint32_t count = flags[kFlagCountM];
    for (uint32_t i = blockIdx.x; i < count; i += (uint32_t)gm) {
      const uint2 sg = seg_m[i];
      const uint2* src = seg_pairs(bucket, xbucket, sg);
      const uint32_t n = seg_count(sg);
      if (!bucket_sort_segment<kM_NW, kM_ITEMS, kM_HB, false, kBucketMax>(src, n, out, sg.x, sm))
        sort_segment_lds<kM_NW, kM_ITEMS, false>(src, n, out, sg.x, sm);
    }
  } else {
    const uint32_t w = threadIdx.x >> 6;
    uint32_t* b = s_lds + w * kW_WORDS;  // 16-byte aligned: kW_WORDS is a multiple of 4
    const SortSmem sm{b, b + kW_CAP, b + 2 * kW_CAP, b + 2 * kW_CAP + 256, b + 2 * kW_CAP + 512};
    const uint32_t count = flags[kFlagCountW];
    const uint32_t stride = (gridDim.x - (uint32_t)gm) * 4u;
    const uint2 none = make_uint2(0u, 0u);
    // Most segments are small (the MSD split leaves thousands of sub-segments
    // of a few dozen copies), and each is a chain of two dependent loads
    // (descriptor, then pairs): the wavefront keeps the descriptor of the
    // segment after next and the pairs of the next one in flight while it
    // sorts the current one.
    uint32_t i = (blockIdx.x - (uint32_t)gm) * 4u + w;
    uint2 sg = i < count ? seg_w[i] : none;
    uint2 sg1 = i + stride < count ? seg_w[i + stride] : none;
    uint2 v = small_pair(bucket, xbucket, sg);
    for (; i < count; i += stride) {
      const uint2 sg2 = i + 2u * stride < count ? seg_w[i + 2u * stride] : none;
      const uint2 v1 = small_pair(bucket, xbucket, sg1);
      const uint2 cur = sg;
      const uint2 vc = v;
      sg = sg1;
      sg1 = sg2;
      v = v1;
      const uint32_t n = seg_count(cur);
      const uint2* src = seg_pairs(bucket, xbucket, cur);
      if (n <= 64)
        rank_sort_wave(vc, n, out, cur.x, reinterpret_cast<uint2*>(b));
      else if (!bucket_sort_segment<1, kW_ITEMS, kW_HB, true, kBucketMax>(src, n, out, cur.x, sm))
        sort_segment_lds<1, kW_ITEMS, true>(src, n, out, cur.x, sm);
    }
  }
}

// Where the sub-segments of a split go, by split round.
enum SplitRound : int { kLdsRound0 = 0, kLdsRound1 = 1, kGlobalRound0 = 2, kGlobalRound1 = 3 };

// Append one segment per thread (threads with an empty segment pass n = 0)
// to the class lists: one global atomic per (block, class).  Classes: 0 W
// (<= 256), 1 M (<= 2048); after a first-round split, the second round (the
// LDS split up to 16384 copies, the global split beyond); after a
// second-round split, the LSD sort of one 1024-thread block (<= 8192) or
// through global memory.
__device__ void push_segments(uint2 sg, int round, const Ws& ws, uint32_t* s_cnt,
                              uint32_t* s_base) {
  int c = 4;  // none
  const uint32_t n = seg_count(sg);
  if (n > 0) {
    if (n <= kSortCapW) c = 0;
    else if (n <= kSortCapM) c = 1;
    else if (round == kLdsRound0) c = 2;
    else if (round == kGlobalRound0) c = n <= kSortCapL ? 2 : 3;
    else c = n <= kSortCapLB ? 2 : 3;  // second rounds
  }
  uint2* lists[4];
  int slots[4];
  lists[0] = ws.seg_w; slots[0] = kFlagCountW;
  lists[1] = ws.seg_m; slots[1] = kFlagCountM;
  if (round == kLdsRound0 || round == kGlobalRound0) {
    // the second split round takes what is still above 2048 (the LDS split
    // up to 16384, the global split beyond)
    lists[2] = ws.seg_b1; slots[2] = kFlagCountB1;
    lists[3] = ws.seg_g; slots[3] = kFlagCountG;  // only from global splits
  } else {
    lists[2] = ws.seg_l; slots[2] = kFlagCountL;
    lists[3] = ws.seg_x2; slots[3] = kFlagCountX2;
  }
  if (threadIdx.x < 4) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  uint32_t my = 0;
  if (c < 4) my = atomicAdd(&s_cnt[c], 1u);
  __syncthreads();
  if (threadIdx.x < 4 && s_cnt[threadIdx.x])
    s_base[threadIdx.x] = atomicAdd(&ws.flags[slots[threadIdx.x]], s_cnt[threadIdx.x]);
  __syncthreads();
  if (c < 4) lists[c][s_base[c] + my] = sg;
  __syncthreads();
}

// Digit of a split: the top 8 bits of ((key - kmin) << ib) | (idx - imin),
// from the segment's key and index ranges (min/max of its pairs reduced over
// the block).
struct SplitDigit {
  uint32_t k0, i0, ib, sh;
  __device__ __forceinline__ uint32_t operator()(uint2 v) const {
    const uint64_t c = ((uint64_t)(v.x - k0) << ib) | (uint64_t)(v.y - i0);
    return (uint32_t)(c >> sh);
  }
};

__device__ __forceinline__ SplitDigit split_digit(uint32_t kmin, uint32_t kmax, uint32_t imin,
                                                  uint32_t imax, uint32_t* s_red) {
  const uint32_t lane = __lane_id(), w = threadIdx.x >> 6;
  kmin = wave_min(kmin); kmax = wave_max(kmax);
  imin = wave_min(imin); imax = wave_max(imax);
  if (lane == 0) {
    s_red[w * 4 + 0] = kmin; s_red[w * 4 + 1] = kmax;
    s_red[w * 4 + 2] = imin; s_red[w * 4 + 3] = imax;
  }
  __syncthreads();
  kmin = 0xffffffffu; kmax = 0; imin = 0xffffffffu; imax = 0;
  for (int ww = 0; ww < 16; ++ww) {
    kmin = min(kmin, s_red[ww * 4 + 0]); kmax = max(kmax, s_red[ww * 4 + 1]);
    imin = min(imin, s_red[ww * 4 + 2]); imax = max(imax, s_red[ww * 4 + 3]);
  }
  SplitDigit d;
  d.ib = nbits(imax - imin);
  const uint32_t total = nbits(kmax - kmin) + d.ib;
  d.sh = total > 8 ? total - 8 : 0;
  d.k0 = kmin;
  d.i0 = imin;
  return d;
}

// The sub-segments of a split: groups of consecutive digit buckets.  A
// bucket of more than kGroupCopies copies stands alone (the next round splits
// it if it still holds more than 2048); the other buckets are grouped by the
// window floor(start / kGroupCopies) their start falls in, so that a group
// holds fewer than 2 kGroupCopies copies.  Depth keys of a tile spread over
// 256 buckets leave hundreds of buckets of a few dozen copies; as groups they
// become a few sub-segments of block-class size, which sort at a fraction of
// the per-copy cost of as many tiny segments.
constexpr uint32_t kGroupCopies = 128;

// Exclusive scan of the 256 digit counts into s_off (first wavefront), the
// group starts into s_grp (s_grp[256]: the number of groups), and the
// sub-segment of group threadIdx.x (threads below the group count; `in_x`
// the buffer flag of where the split leaves it), taken before the offsets
// are consumed.
__device__ __forceinline__ uint2 split_offsets(uint2 sg, uint32_t in_x, const uint32_t* s_cnt,
                                               uint32_t* s_off, uint32_t* s_grp) {
  const uint32_t lane = __lane_id(), w = threadIdx.x >> 6;
  if (w == 0) {
    uint32_t t4[4], o4[4], s = 0;
    for (int q = 0; q < 4; ++q) { t4[q] = s_cnt[lane * 4 + q]; s += t4[q]; }
    uint32_t ex = wave_incl_scan(s) - s;
    for (int q = 0; q < 4; ++q) { o4[q] = ex; s_off[lane * 4 + q] = ex; ex += t4[q]; }
    // the bucket before this lane's first: the previous lane's last
    const uint32_t pc = __shfl_up(t4[3], 1, 64), po = __shfl_up(o4[3], 1, 64);
    bool f[4];
    uint32_t nst = 0;
    for (int q = 0; q < 4; ++q) {
      const uint32_t c0 = q ? t4[q - 1] : pc, p0 = q ? o4[q - 1] : po;
      f[q] = (lane == 0 && q == 0) || t4[q] > kGroupCopies || c0 > kGroupCopies ||
             o4[q] / kGroupCopies != p0 / kGroupCopies;
      nst += f[q] ? 1u : 0u;
    }
    const uint32_t incl = wave_incl_scan(nst);
    uint32_t g = incl - nst;
    for (int q = 0; q < 4; ++q)
      if (f[q]) s_grp[g++] = o4[q];
    if (lane == 63) s_grp[256] = incl;
  }
  __syncthreads();
  const uint32_t ng = s_grp[256];
  uint2 sub = make_uint2(0u, 0u);
  if (threadIdx.x < ng) {
    const uint32_t a = s_grp[threadIdx.x];
    const uint32_t b = threadIdx.x + 1 < ng ? s_grp[threadIdx.x + 1] : seg_count(sg);
    sub = make_uint2(sg.x + a, (b - a) | in_x);
  }
  __syncthreads();
  return sub;
}

// f(e, pair e) for every pair of a segment, e ascending per thread, strided
// over the 1024 threads of a split workgroup: the loads of U rounds are all
// in flight before the first pair is used (one at a time, each of the up to
// 35 rounds of a large segment would wait out a full memory latency).
template <int U, typename F>
__device__ __forceinline__ void for_each_pair(const uint2* __restrict__ g, uint32_t n, F&& f) {
  for (uint32_t e0 = threadIdx.x; e0 < n; e0 += U * 1024u) {
    uint2 v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint32_t e = e0 + (uint32_t)k * 1024u;
      v[k] = e < n ? g[e] : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint32_t e = e0 + (uint32_t)k * 1024u;
      if (e < n) f(e, v[k]);
    }
  }
}
constexpr int kSplitUnroll = 8;

// MSD split of one segment of 2048 < n <= 16384 copies in LDS (in place).
__device__ void split_lds(uint2 sg, int round, const Ws& ws, uint2* s_e, uint32_t* s_cnt,
                          uint32_t* s_off, uint32_t* s_grp, uint32_t* s_red, uint32_t* s_pc,
                          uint32_t* s_pb) {
  const uint32_t n = seg_count(sg);
  uint2* g = seg_pairs(ws.bucket, ws.xbucket, sg);  // split in place
  uint32_t kmin = 0xffffffffu, kmax = 0, imin = 0xffffffffu, imax = 0;
  for_each_pair<kSplitUnroll>(g, n, [&](uint32_t e, uint2 v) {
    s_e[e] = v;
    kmin = min(kmin, v.x); kmax = max(kmax, v.x);
    imin = min(imin, v.y); imax = max(imax, v.y);
  });
  if (threadIdx.x < 256) s_cnt[threadIdx.x] = 0;
  const SplitDigit digit = split_digit(kmin, kmax, imin, imax, s_red);
  for (uint32_t e = threadIdx.x; e < n; e += 1024) atomicAdd(&s_cnt[digit(s_e[e])], 1u);
  __syncthreads();
  const uint2 sub = split_offsets(sg, sg.y & kInX, s_cnt, s_off, s_grp);
  for (uint32_t e = threadIdx.x; e < n; e += 1024) {
    const uint2 v = s_e[e];
    g[atomicAdd(&s_off[digit(v)], 1u)] = v;
  }
  push_segments(sub, round == 0 ? kLdsRound0 : kLdsRound1, ws, s_pc, s_pb);
}

// MSD split of one segment of more than 16384 copies, through global memory:
// the same digit, the segment scattered by digit into the other buffer of
// the pair (bucket, xbucket), where its sub-segments stay.
__device__ void split_global(uint2 sg, int round, const Ws& ws, uint32_t* s_cnt, uint32_t* s_off,
                             uint32_t* s_grp, uint32_t* s_red, uint32_t* s_pc, uint32_t* s_pb) {
  const uint32_t n = seg_count(sg);
  const uint2* g = seg_pairs(ws.bucket, ws.xbucket, sg);
  const uint32_t to_x = (sg.y & kInX) ^ kInX;
  uint2* x = (to_x ? ws.xbucket : ws.bucket) + sg.x;
  uint32_t kmin = 0xffffffffu, kmax = 0, imin = 0xffffffffu, imax = 0;
  for_each_pair<kSplitUnroll>(g, n, [&](uint32_t, uint2 v) {
    kmin = min(kmin, v.x); kmax = max(kmax, v.x);
    imin = min(imin, v.y); imax = max(imax, v.y);
  });
  if (threadIdx.x < 256) s_cnt[threadIdx.x] = 0;
  const SplitDigit digit = split_digit(kmin, kmax, imin, imax, s_red);
  for_each_pair<kSplitUnroll>(g, n, [&](uint32_t, uint2 v) { atomicAdd(&s_cnt[digit(v)], 1u); });
  __syncthreads();
  const uint2 sub = split_offsets(sg, to_x, s_cnt, s_off, s_grp);
  for_each_pair<kSplitUnroll>(g, n,
                              [&](uint32_t, uint2 v) { x[atomicAdd(&s_off[digit(v)], 1u)] = v; });
  push_segments(sub, round == 0 ? kGlobalRound0 : kGlobalRound1, ws, s_pc, s_pb);
}

// One split round over a work counter: the segments of more than 16384
// copies first (each takes a workgroup far longer), then the LDS-sized ones
// (2048 < n <= 16384), each workgroup taking the next segment when done, so
// that the long global splits start at once and the rest fill in around them.
__global__ __launch_bounds__(1024) void k_split(int round, Ws ws) {
  __shared__ uint2 s_e[kSortCapL];
  __shared__ uint32_t s_cnt[256], s_off[256], s_grp[257];
  __shared__ uint32_t s_red[64];
  __shared__ uint32_t s_pc[4], s_pb[4];
  __shared__ uint32_t s_item;
  if (ws.flags[kFlagOverflow]) return;
  const uint2* big = round == 0 ? ws.seg_x : ws.seg_g;
  const uint2* mid = round == 0 ? ws.seg_b0 : ws.seg_b1;
  const uint32_t nbig = ws.flags[round == 0 ? kFlagCountX : kFlagCountG];
  const uint32_t nmid = ws.flags[round == 0 ? kFlagCountB0 : kFlagCountB1];
  uint32_t* next = &ws.flags[round == 0 ? kFlagSplitNext0 : kFlagSplitNext1];
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(next, 1u);
    __syncthreads();
    const uint32_t it = s_item;
    __syncthreads();  // every thread has read s_item before it is taken again
    if (it < nbig)
      split_global(big[it], round, ws, s_cnt, s_off, s_grp, s_red, s_pc, s_pb);
    else if (it - nbig < nmid)
      split_lds(mid[it - nbig], round, ws, s_e, s_cnt, s_off, s_grp, s_red, s_pc, s_pb);
    else
      break;
  }
}

// Segments larger than the LDS capacity.  LSD passes over the full
// (key, index) pair through global memory, in rounds of NW*ITEMS*64
// elements; each pass first histograms the whole segment so that every round
// knows where each digit's run starts.
template <int NW, int ITEMS>
__device__ void sort_x_blocks(const Ws& ws, const ListOut& out, uint32_t* s_hist,
                              uint32_t* s_off, uint32_t* s_red, uint32_t* s_glob, uint32_t b,
                              uint32_t nb) {
  constexpr int ROUND = NW * ITEMS * 64;
  SortSmem sm{nullptr, nullptr, s_hist, s_off, s_red};
  const uint32_t lane = __lane_id();
  const uint32_t w = threadIdx.x >> 6;
  const uint32_t count = ws.flags[kFlagCountX2];
  for (uint32_t i = b; i < count; i += nb) {
    const uint2 sg = ws.seg_x2[i];
    const uint32_t s = sg.x, n = seg_count(sg);
    uint2* const src0 = seg_pairs(ws.bucket, ws.xbucket, sg);
    uint32_t kmin = 0xffffffffu, kmax = 0, imin = 0xffffffffu, imax = 0;
    for (uint32_t e = threadIdx.x; e < n; e += NW * 64) {
      const uint2 v = src0[e];
      kmin = min(kmin, v.x); kmax = max(kmax, v.x);
      imin = min(imin, v.y); imax = max(imax, v.y);
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
    dp.set_key(kmax - kmin);
    dp.set_idx(imax - imin);
    const int np = dp.passes();
    uint2* src = src0;
    uint2* dst = ((sg.y & kInX) ? ws.bucket : ws.xbucket) + s;
    for (int p = 0; p < np; ++p) {
      for (int k = threadIdx.x; k < 256; k += NW * 64) s_glob[k] = 0;
      __syncthreads();
      for (uint32_t e = threadIdx.x; e < n; e += NW * 64) {
        const uint2 v = src[e];
        atomicAdd(&s_glob[dp.get(v.x, v.y, p)], 1u);
      }
      __syncthreads();
      if (w == 0) {
        uint32_t t4[4], sum = 0;
        for (int q = 0; q < 4; ++q) { t4[q] = s_glob[lane * 4 + q]; sum += t4[q]; }
        uint32_t ex = wave_incl_scan(sum) - sum;
        for (int q = 0; q < 4; ++q) { s_off[lane * 4 + q] = ex; ex += t4[q]; }
      }
      __syncthreads();
      const bool last = p + 1 == np;
      for (uint32_t r0 = 0; r0 < n; r0 += ROUND) {
        uint2 v[ITEMS];
        uint32_t dg[ITEMS], rank[ITEMS];
        bool valid[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
          const uint32_t e = r0 + w * ITEMS * 64 + j * 64 + lane;
          valid[j] = e < n;
          v[j] = valid[j] ? src[e] : make_uint2(0u, 0u);
          dg[j] = dp.get(v[j].x, v[j].y, p);
        }
        block_rank<NW, ITEMS, false>(dg, valid, rank, sm, true, ITEMS, dp.width(p));
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
          if (valid[j]) {
            if (last)
              out.put(s + rank[j], v[j].y);
            else
              dst[rank[j]] = v[j];
          }
        }
      }
      __syncthreads();
      uint2* t = src;
      src = dst;
      dst = t;
    }
    if (np == 0) {
      for (uint32_t e = threadIdx.x; e < n; e += NW * 64) out.put(s + e, src0[e].y);
    }
    __syncthreads();
  }
}

// The L class (one 1024-thread block per segment of at most 8192 copies,
// LSD in LDS) on workgroups [0, gl) and the global-memory LSD sort of what
// is larger on the rest, in one launch.
constexpr int kL_NW = 16, kL_ITEMS = kSortCapLB / 1024, kL_CAP = kL_NW * kL_ITEMS * 64;

__global__ __launch_bounds__(1024) void k_sort_lx(int gl, Ws ws, ListOut out) {
  __shared__ __align__(16) uint32_t s_kv[2 * kL_CAP];  // keys, then indices
  uint32_t* s_key = s_kv;
  uint32_t* s_idx = s_kv + kL_CAP;
  __shared__ uint32_t s_hist[kL_NW * 256];
  __shared__ uint32_t s_off[256];
  __shared__ uint32_t s_red[64];
  if (ws.flags[kFlagOverflow]) return;
  if ((int)blockIdx.x >= gl) {
    sort_x_blocks<kL_NW, 16>(ws, out, s_hist, s_off, s_red, s_key, blockIdx.x - (uint32_t)gl,
                             gridDim.x - (uint32_t)gl);
    return;
  }
  const SortSmem sm{s_key, s_idx, s_hist, s_off, s_red};
  const uint32_t count = ws.flags[kFlagCountL];
  for (uint32_t i = blockIdx.x; i < count; i += (uint32_t)gl) {
    const uint2 sg = ws.seg_l[i];
    const uint2* src = seg_pairs(ws.bucket, ws.xbucket, sg);
    const uint32_t n = seg_count(sg);
    if (!bucket_sort_segment<kL_NW, kL_ITEMS, kL_HB, false, kBucketMax>(src, n, out, sg.x, sm))
      sort_segment_lds<kL_NW, kL_ITEMS, false>(src, n, out, sg.x, sm);
  }
}

}  // namespace

hipError_t launch_sort(const Ws& ws, uint32_t* list, uint16_t* lpos, int64_t nt,
                       hipStream_t stream) {
  const ListOut out{list, lpos, ws.lbits, ws.pb};
  // Every launch costs a few microseconds even without work, so the rarely
  // busy roles (global splits of huge tiles, the L and X sorts) share
  // launches with the busy ones and get small grids.
  const int64_t big_max = std::max<int64_t>(1, (int64_t)ws.cap / (int64_t)(kSortCapM + 1));
  const int grid_split = (int)std::min<int64_t>(big_max, 1024);
  const int grid_rare = (int)std::min<int64_t>(big_max, 256);
  // the split rounds: one workgroup per CU (128 KB of LDS each) over a work
  // counter
  hipLaunchKernelGGL(k_split, dim3(std::min(grid_split, 256)), dim3(1024), 0, stream, 0, ws);
  hipLaunchKernelGGL(k_split, dim3(std::min(grid_rare, 256)), dim3(1024), 0, stream, 1, ws);
  const int grid_w = (int)std::min<int64_t>((nt + 3) / 4 + (int64_t)ws.cap / 256, 8192);
  const int grid_m = (int)std::min<int64_t>(nt + (int64_t)ws.cap / 2048, 4096);
  hipLaunchKernelGGL(k_sort_wm, dim3(std::max(grid_m, 1) + std::max(grid_w, 1)), dim3(256), 0,
                     stream, std::max(grid_m, 1), ws.seg_w, ws.seg_m, ws.flags, ws.bucket,
                     ws.xbucket, out);
  hipLaunchKernelGGL(k_sort_lx, dim3(grid_rare + 64), dim3(1024), 0, stream, grid_rare, ws, out);
  return hipGetLastError();
}

}  // namespace inpc
