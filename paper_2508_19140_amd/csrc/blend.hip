// Per-tile alpha blending, forward and backward.
//
// One workgroup per tile, one thread per pixel (an 8x8 tile is exactly one
// 64-wide wavefront).  The tile's depth-ordered list is consumed in chunks
// of copies.  For bilinear splats every copy's tile-local 2x2 position comes
// from a small per-copy array written after the sort (lpos), so coverage
// is known without touching the point data: each copy sets its bit in the
// 64-bit "which copies cover me" mask of the (at most four) pixels it
// covers, and a pixel then visits only its own fragments, in list order, by
// walking the set bits.  Only copies that cover a pixel still blending have
// their point data (position, opacity, features) fetched, and that fetch
// for the next chunk is in flight while the current chunk is blended
// (double-buffered LDS).  Long lists whose pixels have mostly terminated
// therefore cost little more than reading their indices.  Gaussians cover
// most of a tile, so there every pixel tests every staged copy.  Tiles are
// processed in the order inpc_bin produced (longest lists first).
//
// Forward (Eq. (1) of the paper, Appendix A, then the background): per pixel
// T = 1; for each fragment in order: stop if T < t_min; alpha = o w;
// F += T alpha f; T *= 1 - alpha.  F += T f_bg at the end.  The transmittance
// sequence is computed with one rounding per operation so that the
// termination decision is reproducible.  The forward records, per pixel, how
// far down the list it blended, and per tile the largest such position.
//
// Backward (Eq. (2), with the background sign that differentiation gives
// and without skipping zero-alpha fragments): per pixel the blended
// fragments are replayed back to front, over the part of the list the
// forward pass reached.  T_k is recovered from the next fragment's T by
// T_k = T_{k+1} / (1 - alpha_k), starting from the transmittance the forward
// pass recorded in front of the last blended fragment with T > 0 (so an
// alpha = 1 fragment never divides by zero).  The per-fragment terms land in
// per-(copy, corner) LDS slots; one thread per copy then sums its corners
// (the features enter only through G . f at each covered pixel, which the
// copy's thread forms from registers).  The gradients start at zero; a
// point that lies in this tile only gets its gradient written directly, a
// point split over several tiles (about a quarter of them with 8x8 tiles)
// gets this tile's share added with float atomics, one whole point row per
// group of lanes (the wavefront-level staging keeps the atomic count at one
// per 64 / C point rows instead of one per element).
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "common.h"
#include "internal.h"

namespace inpc {
namespace {

template <int T>
struct TileGeom {
  static constexpr int NTH = T * T;
  static constexpr int NW = NTH / 64;
  static constexpr int CHUNK = NTH < 256 ? NTH : 256;
  static constexpr int MW = CHUNK / 64;
  static constexpr int SH = T == 8 ? 3 : (T == 16 ? 4 : 5);
};

constexpr int fpad(int CP) { return CP + 4; }  // LDS row stride of staged features

// Barrier between the phases of a tile.  A single-wavefront tile only needs
// its LDS accesses kept in program order (LDS executes a wavefront's
// instructions in order); the global prefetches stay in flight.
template <int NW>
__device__ __forceinline__ void tile_sync() {
  if constexpr (NW == 1) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <int NW>
__device__ __forceinline__ bool tile_any(bool p) {
  if constexpr (NW == 1)
    return __ballot(p) != 0ull;
  else
    return __syncthreads_count(p) != 0;
}

__device__ __forceinline__ unsigned long long wave_or64(unsigned long long v) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo |= (uint32_t)__shfl_xor((int)lo, o, 64);
    hi |= (uint32_t)__shfl_xor((int)hi, o, 64);
  }
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t pack_xy(int x0, int y0) {
  return (uint32_t)(x0 + 1) | ((uint32_t)(y0 + 1) << 16);
}
__device__ __forceinline__ int unpack_x(uint32_t p) { return (int)(p & 0xffffu) - 1; }
__device__ __forceinline__ int unpack_y(uint32_t p) { return (int)(p >> 16) - 1; }

// Tile handled by this workgroup of a one-view launch: the order inpc_bin
// produced (longest lists first), spread over the XCDs in runs of four.
__device__ __forceinline__ uint32_t block_tile(const BlendArgs& a) {
  return a.order ? a.order[xcd_pos(blockIdx.x, gridDim.x)] : blockIdx.x;
}

// Background features behind pixel p, channel c: a constant [C] vector or a
// per-pixel image [C][H][W] (for example an environment map sampled along
// every pixel's view direction).
__device__ __forceinline__ float bg_value(const BlendArgs& a, int c, int64_t P, int64_t p) {
  return a.bg_image ? a.bg[c * P + p] : a.bg[c];
}

template <typename FT>
__device__ __forceinline__ float half_bits_to_f32(uint32_t b);
template <>
__device__ __forceinline__ float half_bits_to_f32<__half>(uint32_t b) {
  return __half2float(__ushort_as_half((unsigned short)(b & 0xffffu)));
}
template <>
__device__ __forceinline__ float half_bits_to_f32<__hip_bfloat16>(uint32_t b) {
  return __uint_as_float((b & 0xffffu) << 16);  // bf16 -> f32 is exact
}

// One feature row held in registers as raw loaded words (converted to FP32
// only when staged, so a prefetch does not wait for its data).  FULL: the
// row is exactly CP wide (vector loads); otherwise C < CP elements are read
// one by one and the rest is zero.  Loads are unconditional (the caller
// passes a valid point index), which keeps the prefetch free of branches.
template <int CP, typename FT, bool FULL>
struct RowRegs {
  static constexpr int WORDS = CP * (int)sizeof(FT) / 4;
  static constexpr int VEC = WORDS % 4 == 0 ? 4 : 2;  // 16- or 8-byte loads
  uint32_t w[WORDS];

  __device__ __forceinline__ void load(const FT* __restrict__ feat, uint32_t idx, int C) {
    const FT* row = feat + (size_t)idx * C;
    if constexpr (FULL) {
      if constexpr (VEC == 4) {
        const uint4* r = reinterpret_cast<const uint4*>(row);
#pragma unroll
        for (int q = 0; q < WORDS / 4; ++q) {
          const uint4 v = r[q];
          w[4 * q] = v.x; w[4 * q + 1] = v.y; w[4 * q + 2] = v.z; w[4 * q + 3] = v.w;
        }
      } else {
        const uint2* r = reinterpret_cast<const uint2*>(row);
#pragma unroll
        for (int q = 0; q < WORDS / 2; ++q) {
          const uint2 v = r[q];
          w[2 * q] = v.x; w[2 * q + 1] = v.y;
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < WORDS; ++k) w[k] = 0u;
      if constexpr (sizeof(FT) == 4) {
        const uint32_t* r = reinterpret_cast<const uint32_t*>(row);
#pragma unroll
        for (int c = 0; c < CP; ++c) {
          const uint32_t v = r[c < C ? c : C - 1];
          w[c] = c < C ? v : 0u;
        }
      } else {
        const uint16_t* r = reinterpret_cast<const uint16_t*>(row);
#pragma unroll
        for (int c = 0; c < CP; ++c) {
          const uint32_t v = r[c < C ? c : C - 1];
          w[c >> 1] |= (c < C ? v : 0u) << (16 * (c & 1));
        }
      }
    }
  }

  __device__ __forceinline__ void to_f32(float (&v)[CP]) const {
    if constexpr (sizeof(FT) == 4) {
#pragma unroll
      for (int c = 0; c < CP; ++c) v[c] = __uint_as_float(w[c]);
    } else {
#pragma unroll
      for (int c = 0; c < CP; ++c) v[c] = half_bits_to_f32<FT>(w[c >> 1] >> (16 * (c & 1)));
    }
  }

  __device__ __forceinline__ void store_f32(float* __restrict__ dst) const {
    float4* d4 = reinterpret_cast<float4*>(dst);
    if constexpr (sizeof(FT) == 4) {
#pragma unroll
      for (int q = 0; q < CP / 4; ++q)
        d4[q] = make_float4(__uint_as_float(w[4 * q]), __uint_as_float(w[4 * q + 1]),
                            __uint_as_float(w[4 * q + 2]), __uint_as_float(w[4 * q + 3]));
    } else {
#pragma unroll
      for (int q = 0; q < CP / 4; ++q)
        d4[q] = make_float4(half_bits_to_f32<FT>(w[2 * q]), half_bits_to_f32<FT>(w[2 * q] >> 16),
                            half_bits_to_f32<FT>(w[2 * q + 1]),
                            half_bits_to_f32<FT>(w[2 * q + 1] >> 16));
    }
  }
};

// Store CP floats of which the first C are meaningful.
template <int CP>
__device__ __forceinline__ void store_row(float* __restrict__ dst, const float (&v)[CP], int C) {
  if (C == CP) {
    float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
    for (int q = 0; q < CP / 4; ++q)
      d4[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
  } else {
#pragma unroll
    for (int c = 0; c < CP; ++c)
      if (c < C) dst[c] = v[c];
  }
}

// Register prefetch of one copy's point data.  The loads are not
// predicated: a copy that is not needed fetches point 0 instead (all such
// lanes hit the same line), which keeps the prefetch free of branches.
template <int CP, typename FT, bool FULL>
struct Prefetch {
  bool valid;
  uint32_t idx;
  float4 p;  // u, v, opacity, radius
  RowRegs<CP, FT, FULL> f;

  __device__ __forceinline__ void fetch(const BlendArgs& a, bool v, uint32_t i) {
    valid = v;
    idx = v ? i : 0u;
    p = reinterpret_cast<const float4*>(a.proj)[idx];
    f.load(reinterpret_cast<const FT*>(a.feat), idx, a.C);
  }
};

// Point data of one copy per lane gathered straight into LDS (gfx950
// global_load_lds_dwordx4: one 16-byte quad per lane and instruction, lane l
// of an instruction writes slot l of the instruction's 1 KB block).  The
// projection record of lane l's copy goes to prj[l].  The feature rows are
// fetched row-major: flat quad f = 64 k + l of instruction k is quad f mod Q
// of row f / Q, so Q neighbouring lanes read one row's contiguous bytes
// (one cache line per Q lanes instead of one per lane), and the rows land in
// LDS as fq[row * Q + quad].  Nothing passes through registers, so a fetch
// issued for the next chunk stays in flight until the chunk is staged.  For
// rows that are whole quads (C == CP and CP * sizeof(FT) a multiple of 16
// bytes).  Called by the whole wavefront; lanes with v false fetch nothing.
typedef __attribute__((address_space(3))) void lds_void_t;

template <int CP, typename FT>
struct DmaRow {
  static constexpr int Q = CP * (int)sizeof(FT) / 16;  // quads per feature row
  static constexpr bool OK = CP * (int)sizeof(FT) % 16 == 0;

  __device__ __forceinline__ static void fetch(const BlendArgs& a, bool v, uint32_t idx,
                                               float4* prj, uint4* fq) {
    const uint32_t lane = __lane_id();
    if (v) {
      const float4* pp = reinterpret_cast<const float4*>(a.proj) + idx;
      __builtin_amdgcn_global_load_lds((const void*)pp, (lds_void_t*)prj, 16, 0, 0);
    }
    const uint4* feat = reinterpret_cast<const uint4*>(a.feat);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const uint32_t f = (uint32_t)k * 64u + lane;
      const int row = (int)(f / (uint32_t)Q);
      const uint32_t ridx = (uint32_t)__shfl((int)idx, row, 64);
      const bool rv = __shfl((int)v, row, 64) != 0;
      if (rv)
        __builtin_amdgcn_global_load_lds((const void*)(feat + (size_t)ridx * Q + f % (uint32_t)Q),
                                         (lds_void_t*)(fq + k * 64), 16, 0, 0);
    }
  }

  // Feature row of this lane's copy as FP32.
  __device__ __forceinline__ static void row(const uint4* fq, uint32_t lane, float (&v)[CP]) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const uint4 w = fq[lane * Q + q];
      if constexpr (sizeof(FT) == 4) {
        v[4 * q] = __uint_as_float(w.x); v[4 * q + 1] = __uint_as_float(w.y);
        v[4 * q + 2] = __uint_as_float(w.z); v[4 * q + 3] = __uint_as_float(w.w);
      } else {
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          v[8 * q + 2 * k] = half_bits_to_f32<FT>(ws[k]);
          v[8 * q + 2 * k + 1] = half_bits_to_f32<FT>(ws[k] >> 16);
        }
      }
    }
  }
};

// The point data of the copy a lane stages next: gathered into LDS when the
// rows are whole quads (DmaRow), else into registers (Prefetch).
template <int CP, typename FT, bool FULL>
struct PointFetch {
  static constexpr bool DMA = FULL && DmaRow<CP, FT>::OK;
  static constexpr int QS = DMA ? DmaRow<CP, FT>::Q : 1;  // LDS quads per row slot
  bool valid;
  uint32_t idx;
  Prefetch<CP, FT, FULL> reg;

  __device__ __forceinline__ void fetch(const BlendArgs& a, bool v, uint32_t i, float4* prj,
                                        uint4* fq) {
    if constexpr (DMA) {
      valid = v;
      idx = v ? i : 0u;
      DmaRow<CP, FT>::fetch(a, v, idx, prj, fq);
    } else {
      reg.fetch(a, v, i);
      valid = reg.valid;
      idx = reg.idx;
    }
  }
  // Before the staged copy is read: the compiler does not order LDS reads
  // after the gather's LDS writes, so wait for every outstanding memory
  // operation of this wavefront (each lane reads only its own slots).
  __device__ __forceinline__ void wait() const {
    if constexpr (DMA) __builtin_amdgcn_s_waitcnt(0);
  }
  __device__ __forceinline__ float4 proj(const float4* prj, uint32_t lane) const {
    if constexpr (DMA) return prj[lane];
    else return reg.p;
  }
  __device__ __forceinline__ void row(const uint4* fq, uint32_t lane, float (&v)[CP]) const {
    if constexpr (DMA) DmaRow<CP, FT>::row(fq, lane, v);
    else reg.f.to_f32(v);
  }
};

// List entry (point index and tile-local 2x2 position) of a chunk slot.
struct Entry {
  bool valid;
  uint32_t idx, lp;
  __device__ __forceinline__ void load(const BlendArgs& a, bool stager, uint32_t q, uint32_t end) {
    valid = stager && q < end;
    const uint32_t qq = q < end ? q : end - 1;  // end > start
    idx = a.list[qq];
    lp = a.lpos[qq];
  }
};

// Whether a copy's point meets this tile only, from its tile-local corner
// code c = x0 - T tx + 1 (and likewise in y): both columns x0, x0 + 1 fall in
// this tile (1 <= c <= T - 1), or the other one lies outside the image (c = 0
// in the first tile column, c = T in the last).  Equals ntiles == 1 of the
// projection, whose tile rectangle is that of the clipped 2x2 footprint.
template <int T>
__device__ __forceinline__ bool single_tile(uint32_t lp, int tx, int ty, int W, int H) {
  const int cx = (int)(lp & 0xffu), cy = (int)(lp >> 8);
  const bool sx = (cx >= 1 && cx <= T - 1) || (cx == 0 && tx == 0) || (cx == T && (tx + 1) * T >= W);
  const bool sy = (cy >= 1 && cy <= T - 1) || (cy == 0 && ty == 0) || (cy == T && (ty + 1) * T >= H);
  return sx && sy;
}

// Clear the coverage masks of this thread's pixel, then set the bits of
// this thread's copy (tile-local splat corner (x0, y0) = lp - 1).
template <int T>
__device__ __forceinline__ void build_coverage(unsigned long long* __restrict__ mask,
                                               const Entry& e) {
  using G = TileGeom<T>;
  const int tid = threadIdx.x;
#pragma unroll
  for (int w = 0; w < G::MW; ++w) mask[tid * G::MW + w] = 0ull;
  tile_sync<G::NW>();
  if (e.valid) {
    const int x0 = (int)(e.lp & 0xffu) - 1, y0 = (int)(e.lp >> 8) - 1;
    const unsigned long long bit = 1ull << (tid & 63);
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const int qx = x0 + dx, qy = y0 + dy;
        if (qx >= 0 && qx < T && qy >= 0 && qy < T)
          atomicOr(&mask[(qy * T + qx) * G::MW + (tid >> 6)], bit);
      }
  }
  tile_sync<G::NW>();
}

// Copies of the chunk covering at least one pixel with `active` set: is this
// thread's copy among them?
template <int T>
__device__ __forceinline__ bool copy_needed(const unsigned long long* __restrict__ mask,
                                            bool active, unsigned long long* __restrict__ s_need) {
  using G = TileGeom<T>;
  const int tid = threadIdx.x;
  unsigned long long nd[G::MW];
#pragma unroll
  for (int w = 0; w < G::MW; ++w) nd[w] = wave_or64(active ? mask[tid * G::MW + w] : 0ull);
  if constexpr (G::NW == 1) {
    return (nd[0] >> (tid & 63)) & 1ull;
  } else {
    if ((tid & 63) == 0)
#pragma unroll
      for (int w = 0; w < G::MW; ++w) atomicOr(&s_need[w], nd[w]);
    __syncthreads();
    const bool r = tid < G::CHUNK && ((s_need[tid >> 6] >> (tid & 63)) & 1ull);
    return r;
  }
}

// ---------------------------------------------------------------------------
// Forward, bilinear splats
// ---------------------------------------------------------------------------
template <int T, int CP, typename FT, bool FULL>
__device__ __forceinline__ void blend_fwd_bilinear_tile(const BlendArgs& a, uint32_t tile) {
  using G = TileGeom<T>;
  constexpr int NW = G::NW, CH = G::CHUNK, MW = G::MW;
  __shared__ float4 s_geo[CH];
  __shared__ __align__(16) float s_feat[CH * fpad(CP)];
  __shared__ unsigned long long s_mask[2][G::NTH * MW];
  __shared__ unsigned long long s_need[MW];
  __shared__ uint32_t s_ml[NW];

  const int tid = threadIdx.x;
  const int tx = (int)(tile % (uint32_t)a.opts.ntx), ty = (int)(tile / (uint32_t)a.opts.ntx);
  const int lx = tid % T, ly = tid / T;
  const int px = tx * T + lx, py = ty * T + ly;
  const bool inside = px < a.cam.W && py < a.cam.H;
  const uint32_t start = a.ranges[tile], end = a.ranges[tile + 1];
  const float t_min = a.opts.t_min;
  const bool stager = tid < CH;

  float F[CP];
#pragma unroll
  for (int c = 0; c < CP; ++c) F[c] = 0.f;
  float Tr = 1.f, t_anchor = 1.f;
  uint32_t cnt = 0, last = 0, anchor = 0;
  bool done = !inside;

  Entry e;  // list entries of the chunk whose coverage is built next
  e.valid = false;
  e.idx = e.lp = 0;
  Prefetch<CP, FT, FULL> pf;  // point data of the chunk staged next
  pf.valid = false;
  if (end > start) {
    e.load(a, stager, start + tid, end);
    if constexpr (NW > 1) {
      if (tid < MW) s_need[tid] = 0ull;
    }
    build_coverage<T>(s_mask[0], e);
    const bool nd = copy_needed<T>(s_mask[0], !done, s_need);  // every lane takes part
    pf.fetch(a, e.valid && nd, e.idx);
    e.load(a, stager, start + CH + tid, end);
  }

  int b = 0;
  for (uint32_t base = start; base < end; base += CH, b ^= 1) {
    if (!tile_any<NW>(!done)) break;
    // stage the fetched copies of this chunk
    if (pf.valid) {
      const Footprint f = bilinear_footprint(pf.p.x, pf.p.y, a.cam.W, a.cam.H);
      s_geo[tid] = make_float4(f.a, f.b, pf.p.z, __uint_as_float(pack_xy(f.x0, f.y0)));
      pf.f.store_f32(&s_feat[tid * fpad(CP)]);
    }
    // coverage of the next chunk; fetch the copies it needs while this one blends
    if constexpr (NW > 1) {
      if (tid < MW) s_need[tid] = 0ull;
    }
    build_coverage<T>(s_mask[b ^ 1], e);
    const bool nd = copy_needed<T>(s_mask[b ^ 1], !done, s_need);
    pf.fetch(a, e.valid && nd, e.idx);
    e.load(a, stager, base + 2 * CH + tid, end);
    if (!done) {
      for (int w = 0; w < MW && !done; ++w) {
        unsigned long long m = s_mask[b][tid * MW + w];
        while (m) {
          const int j = __ffsll(m) - 1;
          m &= m - 1;
          const int kk = w * 64 + j;
          const float4 g = s_geo[kk];
          const uint32_t pk = __float_as_uint(g.w);
          const int dx = px - unpack_x(pk), dy = py - unpack_y(pk);
          const float wx = dx ? g.x : fsub(1.f, g.x);
          const float wy = dy ? g.y : fsub(1.f, g.y);
          const float al = fmul(g.z, fmul(wx, wy));
          if (Tr < t_min) {
            done = true;
            break;
          }
          const float wt = Tr * al;
          const float4* fr = reinterpret_cast<const float4*>(&s_feat[kk * fpad(CP)]);
#pragma unroll
          for (int q = 0; q < CP / 4; ++q) {
            const float4 f4 = fr[q];
            F[4 * q] = fmaf(wt, f4.x, F[4 * q]);
            F[4 * q + 1] = fmaf(wt, f4.y, F[4 * q + 1]);
            F[4 * q + 2] = fmaf(wt, f4.z, F[4 * q + 2]);
            F[4 * q + 3] = fmaf(wt, f4.w, F[4 * q + 3]);
          }
          const uint32_t q1 = base - start + (uint32_t)kk + 1u;
          if (Tr > 0.f) {
            anchor = q1;
            t_anchor = Tr;
          }
          Tr = fmul(Tr, fsub(1.f, al));
          ++cnt;
          last = q1;
        }
      }
    }
    tile_sync<NW>();
  }
  if (a.st_tile) {
    uint32_t ml = last;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ml = max(ml, (uint32_t)__shfl_xor((int)ml, o, 64));
    if constexpr (NW == 1) {
      if (tid == 0) a.st_tile[tile] = ml;
    } else {
      if ((tid & 63) == 0) s_ml[tid >> 6] = ml;
      __syncthreads();
      if (tid == 0) {
        for (int w = 0; w < NW; ++w) ml = max(ml, s_ml[w]);
        a.st_tile[tile] = ml;
      }
    }
  }
  if (!inside) return;
  const int64_t P = (int64_t)a.cam.W * a.cam.H;
  const int64_t p = (int64_t)py * a.cam.W + px;
#pragma unroll
  for (int c = 0; c < CP; ++c)
    if (c < a.C) a.out[c * P + p] = a.bg ? fmaf(Tr, bg_value(a, c, P, p), F[c]) : F[c];
  a.t_final[p] = Tr;
  a.n_contrib[p] = cnt;
  if (a.st_last) {
    a.st_last[p] = last;
    a.st_anchor[p] = anchor;
    a.st_tanchor[p] = t_anchor;
  }
}

// ---------------------------------------------------------------------------
// Forward, bilinear splats, 8x8 tiles: sparse compaction of long lists
// ---------------------------------------------------------------------------
//
// In the longest lists most pixels terminate early while a few (pixels the
// tile's surface barely covers) stay open to the last copy, so the chunk
// loop above walks thousands of copies for a handful of fragments, paying a
// memory round trip per 64 copies.  Here the list is read in super-chunks
// of 512 positions (index and 2x2 position only, prefetched one super-chunk
// ahead); from each copy's position alone the wavefront knows which copies
// cover a pixel still blending, compacts those in list order into virtual
// chunks of 64, and fetches and blends only them.  A super-chunk whose
// pixels are all open is eight full virtual chunks (the point data of the
// next is fetched while the current one blends); in the sparse tail a
// super-chunk is one short virtual chunk.

constexpr int kSubs = 8;  // chunks of 64 list positions per super-chunk

// Pixels (bit ly * 8 + lx) of an 8x8 tile covered by the 2x2 splat whose
// tile-local corner code is lp (x0 + 1 | (y0 + 1) << 8, x0, y0 in [-1, 7]).
__device__ __forceinline__ uint64_t splat_pixels8(uint32_t lp) {
  const int x0 = (int)(lp & 0xffu) - 1, y0 = (int)(lp >> 8) - 1;
  const uint64_t r = (uint64_t)(((3u << (x0 + 1)) >> 1) & 0xffu);
  uint64_t m = 0;
  if (y0 >= 0) m |= r << (8 * y0);
  if (y0 <= 6) m |= r << (8 * (y0 + 1));
  return m;
}

// List entries (point index, 2x2 position) of a super-chunk: position
// base + j * 64 + lane for j < kSubs.
struct SuperEntries {
  uint32_t idx[kSubs], lp[kSubs];
  __device__ __forceinline__ void load(const BlendArgs& a, uint32_t base, uint32_t end) {
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int j = 0; j < kSubs; ++j) {
      const uint32_t q = base + (uint32_t)j * 64u + lane;
      const uint32_t qq = q < end ? q : end - 1;  // end > base
      idx[j] = a.list[qq];
      lp[j] = a.lpos[qq];
    }
  }
};

// Copies of a super-chunk that cover a pixel in `act`, compacted in list
// order: ballot per chunk and the running count before it.
struct Compaction {
  uint64_t need[kSubs];
  uint32_t before[kSubs];
  uint32_t total;
  __device__ __forceinline__ void build(const SuperEntries& e, uint32_t base, uint32_t end,
                                        const uint64_t (&act)[kSubs]) {
    const uint32_t lane = __lane_id();
    total = 0;
#pragma unroll
    for (int j = 0; j < kSubs; ++j) {
      const bool valid = base + (uint32_t)j * 64u + lane < end;
      need[j] = __ballot(valid && (splat_pixels8(e.lp[j]) & act[j]) != 0ull);
      before[j] = total;
      total += (uint32_t)__popcll(need[j]);
    }
  }
  // Writes the selected copies with compacted rank in [vb, vb + 64) to
  // sel[rank - vb] as (point index, lp | offset in the super-chunk << 16).
  __device__ __forceinline__ void publish(const SuperEntries& e, uint32_t vb,
                                          uint2* __restrict__ sel) const {
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int j = 0; j < kSubs; ++j) {
      if ((need[j] >> lane) & 1ull) {
        const uint32_t r = before[j] + mbcnt64(need[j]) - vb;
        if (r < 64u) sel[r] = make_uint2(e.idx[j], e.lp[j] | (((uint32_t)j * 64u + lane) << 16));
      }
    }
  }
};

template <int CP, typename FT, bool FULL>
__device__ __forceinline__ void blend_fwd_bilinear8_tile(const BlendArgs& a, uint32_t tile) {
  constexpr int T = 8;
  constexpr uint32_t SC = kSubs * 64;
  __shared__ float4 s_geo[64];
  __shared__ __align__(16) float s_feat[64 * fpad(CP)];
  __shared__ unsigned long long s_mask[64];
  __shared__ uint2 s_sel[64];
  __shared__ uint32_t s_q1[64];  // one past the copy's position in the tile list

  const uint32_t lane = threadIdx.x;
  const int tx = (int)(tile % (uint32_t)a.opts.ntx), ty = (int)(tile / (uint32_t)a.opts.ntx);
  const int px = tx * T + (int)(lane % T), py = ty * T + (int)(lane / T);
  const bool inside = px < a.cam.W && py < a.cam.H;
  const uint32_t start = a.ranges[tile], end = a.ranges[tile + 1];
  const float t_min = a.opts.t_min;

  float F[CP];
#pragma unroll
  for (int c = 0; c < CP; ++c) F[c] = 0.f;
  float Tr = 1.f, t_anchor = 1.f;
  uint32_t cnt = 0, last = 0, anchor = 0;
  bool done = !inside;

  SuperEntries nxt;
  if (end > start) nxt.load(a, start, end);
  for (uint32_t base = start; base < end; base += SC) {
    const uint64_t open = __ballot(!done);
    if (open == 0ull) break;
    const SuperEntries cur = nxt;
    if (base + SC < end) nxt.load(a, base + SC, end);
    uint64_t act[kSubs];
#pragma unroll
    for (int j = 0; j < kSubs; ++j) act[j] = open;
    Compaction cp;
    cp.build(cur, base, end, act);
    const uint32_t nvc = (cp.total + 63u) / 64u;
    Prefetch<CP, FT, FULL> pf;
    uint32_t plp = 0, pq1 = 0;
    if (nvc > 0) {
      cp.publish(cur, 0, s_sel);
      tile_sync<1>();
      const bool has = lane < cp.total;
      const uint2 sl = has ? s_sel[lane] : make_uint2(0u, 0u);
      pf.fetch(a, has, sl.x);
      plp = sl.y & 0xffffu;
      pq1 = base - start + (sl.y >> 16) + 1u;
      tile_sync<1>();
    }
    for (uint32_t v = 0; v < nvc; ++v) {
      if (__ballot(!done) == 0ull) break;
      // stage virtual chunk v and its coverage
      s_mask[lane] = 0ull;
      tile_sync<1>();
      if (pf.valid) {
        const Footprint f = bilinear_footprint(pf.p.x, pf.p.y, a.cam.W, a.cam.H);
        s_geo[lane] = make_float4(f.a, f.b, pf.p.z, __uint_as_float(pack_xy(f.x0, f.y0)));
        pf.f.store_f32(&s_feat[lane * fpad(CP)]);
        s_q1[lane] = pq1;
        uint64_t pm = splat_pixels8(plp);
        const unsigned long long bit = 1ull << lane;
        while (pm) {
          const int b = __ffsll((unsigned long long)pm) - 1;
          pm &= pm - 1ull;
          atomicOr(&s_mask[b], bit);
        }
      }
      tile_sync<1>();
      // fetch virtual chunk v + 1 while v blends
      if (v + 1 < nvc) {
        cp.publish(cur, (v + 1) * 64u, s_sel);
        tile_sync<1>();
        const bool has = (v + 1) * 64u + lane < cp.total;
        const uint2 sl = has ? s_sel[lane] : make_uint2(0u, 0u);
        pf.fetch(a, has, sl.x);
        plp = sl.y & 0xffffu;
        pq1 = base - start + (sl.y >> 16) + 1u;
      }
      if (!done) {
        unsigned long long m = s_mask[lane];
        while (m) {
          const int kk = __ffsll(m) - 1;
          m &= m - 1;
          const float4 g = s_geo[kk];
          const uint32_t pk = __float_as_uint(g.w);
          const int dx = px - unpack_x(pk), dy = py - unpack_y(pk);
          const float wx = dx ? g.x : fsub(1.f, g.x);
          const float wy = dy ? g.y : fsub(1.f, g.y);
          const float al = fmul(g.z, fmul(wx, wy));
          if (Tr < t_min) {
            done = true;
            break;
          }
          const float wt = Tr * al;
          const float4* fr = reinterpret_cast<const float4*>(&s_feat[kk * fpad(CP)]);
#pragma unroll
          for (int q = 0; q < CP / 4; ++q) {
            const float4 f4 = fr[q];
            F[4 * q] = fmaf(wt, f4.x, F[4 * q]);
            F[4 * q + 1] = fmaf(wt, f4.y, F[4 * q + 1]);
            F[4 * q + 2] = fmaf(wt, f4.z, F[4 * q + 2]);
            F[4 * q + 3] = fmaf(wt, f4.w, F[4 * q + 3]);
          }
          const uint32_t q1 = s_q1[kk];
          if (Tr > 0.f) {
            anchor = q1;
            t_anchor = Tr;
          }
          Tr = fmul(Tr, fsub(1.f, al));
          ++cnt;
          last = q1;
        }
      }
      tile_sync<1>();
    }
  }
  if (a.st_tile) {
    uint32_t ml = last;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ml = max(ml, (uint32_t)__shfl_xor((int)ml, o, 64));
    if (lane == 0) a.st_tile[tile] = ml;
  }
  if (!inside) return;
  const int64_t P = (int64_t)a.cam.W * a.cam.H;
  const int64_t p = (int64_t)py * a.cam.W + px;
#pragma unroll
  for (int c = 0; c < CP; ++c)
    if (c < a.C) a.out[c * P + p] = a.bg ? fmaf(Tr, bg_value(a, c, P, p), F[c]) : F[c];
  a.t_final[p] = Tr;
  a.n_contrib[p] = cnt;
  if (a.st_last) {
    a.st_last[p] = last;
    a.st_anchor[p] = anchor;
    a.st_tanchor[p] = t_anchor;
  }
}

// ---------------------------------------------------------------------------
// Forward, screen-space Gaussians (inference)
// ---------------------------------------------------------------------------
// A staged Gaussian copy: s_g0 = (u, v, opacity, s2) and s_g1 = (cut
// threshold, packed (px0, py0), packed (px1, py1), -) for a screen-space
// Gaussian; s_g0 = (u, v, opacity, conic A) and s_g1 = (conic B, packed
// corners, conic C) for a world-space one (cut at cutoff^2, the same for
// every copy).
__device__ __forceinline__ void stage_gauss(const BlendArgs& a, bool ewa, float4 p,
                                            float4* __restrict__ g0, float4* __restrict__ g1) {
  const Footprint f = footprint(a.opts, a.cam, p.x, p.y, p.w);
  *g0 = make_float4(p.x, p.y, p.z, ewa ? f.ca : f.s2);
  *g1 = make_float4(ewa ? f.cb : f.thr, __uint_as_float(pack_xy(f.px0, f.py0)),
                    __uint_as_float(pack_xy(f.px1, f.py1)), f.cc);
}

// The pixels of this tile inside a staged Gaussian's candidate rectangle
// (packed corners lo, hi), as NW 64-bit words: word w holds tile-local
// pixels 64 w .. 64 w + 63 (those of wavefront w), bit = pixel index mod 64.
template <int T, int NW>
__device__ __forceinline__ void rect_pixel_mask(uint32_t lo, uint32_t hi, int tx, int ty,
                                                unsigned long long* __restrict__ out) {
  constexpr int RPW = 64 / T;  // pixel rows per word
  const int x0 = max(unpack_x(lo) - tx * T, 0), x1 = min(unpack_x(hi) - tx * T, T - 1);
  const int y0 = max(unpack_y(lo) - ty * T, 0), y1 = min(unpack_y(hi) - ty * T, T - 1);
  const unsigned long long row = x0 <= x1 ? (2ull << x1) - (1ull << x0) : 0ull;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    unsigned long long m = 0ull;
    for (int y = max(y0, w * RPW); y <= min(y1, w * RPW + RPW - 1); ++y)
      m |= row << ((y - w * RPW) * T);
    out[w] = m;
  }
}

// This lane's candidates among staged copies [j0, j0 + n), n <= 64: bit j
// set iff copy j0 + j's rectangle holds the lane's pixel (word `wv` of every
// copy's pixel mask, bit `lb`).  The reads are independent, so their LDS
// latencies overlap.
template <int NW>
__device__ __forceinline__ unsigned long long candidates(const unsigned long long* __restrict__ pm,
                                                         int j0, int n, int wv, uint32_t lb) {
  unsigned long long m = 0ull;
#pragma unroll 8
  for (int j = 0; j < 64; ++j)
    if (j < n) m |= ((pm[(j0 + j) * NW + wv] >> lb) & 1ull) << j;
  return m;
}

// Whether pixel-centre offset (dx, dy) lies inside a staged Gaussian's cut,
// with the squared distance in its metric (FP32, one rounding per
// operation, as in the projection).
__device__ __forceinline__ bool gauss_inside(bool ewa, float thr_ewa, float4 g0, float4 g1,
                                             float dx, float dy, float& d2) {
  d2 = ewa ? gauss_d2(true, dx, dy, g0.w, g1.x, g1.w) : gauss_d2(false, dx, dy, 0.f, 0.f, 0.f);
  return d2 <= (ewa ? thr_ewa : g1.x);
}

// Gaussian value w at squared distance d2 (the forward and the backward
// evaluate the same expression, so the replay sees the forward's alphas).
__device__ __forceinline__ float gauss_value(bool ewa, float d2, float s2) {
  return expf(ewa ? -0.5f * d2 : -0.5f * d2 / s2);
}

// Largest `last` over the tile's pixels into st_tile[tile].
template <int NW>
__device__ __forceinline__ void write_tile_last(const BlendArgs& a, uint32_t tile, uint32_t last,
                                                uint32_t* s_ml) {
  const int tid = threadIdx.x;
  uint32_t ml = last;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) ml = max(ml, (uint32_t)__shfl_xor((int)ml, o, 64));
  if constexpr (NW == 1) {
    if (tid == 0) a.st_tile[tile] = ml;
  } else {
    if ((tid & 63) == 0) s_ml[tid >> 6] = ml;
    __syncthreads();
    if (tid == 0) {
      for (int w = 0; w < NW; ++w) ml = max(ml, s_ml[w]);
      a.st_tile[tile] = ml;
    }
  }
}

template <int T, int CP, typename FT, bool FULL>
__device__ __forceinline__ void blend_fwd_gauss_tile(const BlendArgs& a, uint32_t tile) {
  using G = TileGeom<T>;
  constexpr int NW = G::NW;
  __shared__ float4 s_g0[G::CHUNK];
  __shared__ float4 s_g1[G::CHUNK];
  __shared__ __align__(16) float s_feat[G::CHUNK * fpad(CP)];
  __shared__ unsigned long long s_pm[G::CHUNK * NW];  // pixel masks of the staged copies
  __shared__ uint32_t s_ml[NW];

  const int tid = threadIdx.x;
  const int tx = (int)(tile % (uint32_t)a.opts.ntx), ty = (int)(tile / (uint32_t)a.opts.ntx);
  const int px = tx * T + tid % T, py = ty * T + tid / T;
  const bool inside = px < a.cam.W && py < a.cam.H;
  const uint32_t start = a.ranges[tile], end = a.ranges[tile + 1];
  const float t_min = a.opts.t_min;
  const bool ewa = a.opts.splat == INPC_SPLAT_EWA;
  const float thr_ewa = fmul(a.opts.cutoff, a.opts.cutoff);
  const float pxc = fadd((float)px, 0.5f), pyc = fadd((float)py, 0.5f);
  const bool stager = tid < G::CHUNK;

  float F[CP];
#pragma unroll
  for (int c = 0; c < CP; ++c) F[c] = 0.f;
  float Tr = 1.f, t_anchor = 1.f;
  uint32_t cnt = 0, last = 0, anchor = 0;
  bool done = !inside;

  Prefetch<CP, FT, FULL> pf;
  pf.valid = false;
  bool nv = false;
  uint32_t nidx = 0u;
  auto list_at = [&](uint32_t q) { return a.list[q < end ? q : end - 1]; };
  if (end > start) {
    pf.fetch(a, stager && start + tid < end, list_at(start + tid));
    nv = stager && start + G::CHUNK + tid < end;
    nidx = list_at(start + G::CHUNK + tid);
  }

  for (uint32_t base = start; base < end; base += G::CHUNK) {
    if (!tile_any<NW>(!done)) break;
    const uint32_t nh = min((uint32_t)G::CHUNK, end - base);
    if (pf.valid) {
      stage_gauss(a, ewa, pf.p, &s_g0[tid], &s_g1[tid]);
      rect_pixel_mask<T, NW>(__float_as_uint(s_g1[tid].y), __float_as_uint(s_g1[tid].z), tx, ty,
                             &s_pm[tid * NW]);
      pf.f.store_f32(s_feat + tid * fpad(CP));
    }
    pf.fetch(a, nv, nidx);
    nv = stager && base + 2 * G::CHUNK + tid < end;
    nidx = list_at(base + 2 * G::CHUNK + tid);
    tile_sync<NW>();
    for (int w0 = 0; w0 < G::MW && !done; ++w0) {
      unsigned long long m = candidates<NW>(s_pm, 64 * w0, (int)nh - 64 * w0, tid >> 6,
                                            (uint32_t)tid & 63u);
      while (m) {
        const int j = __ffsll(m) - 1;
        m &= m - 1ull;
        const uint32_t kk = 64u * (uint32_t)w0 + (uint32_t)j;
        const float4 g1 = s_g1[kk];
        const float4 g0 = s_g0[kk];
        float d2;
        if (!gauss_inside(ewa, thr_ewa, g0, g1, fsub(pxc, g0.x), fsub(pyc, g0.y), d2)) continue;
        if (Tr < t_min) {
          done = true;
          break;
        }
        const float al = g0.z * gauss_value(ewa, d2, g0.w);
        const float wt = Tr * al;
        const float4* fr = reinterpret_cast<const float4*>(s_feat + kk * fpad(CP));
#pragma unroll
        for (int q = 0; q < CP / 4; ++q) {
          const float4 f4 = fr[q];
          F[4 * q] = fmaf(wt, f4.x, F[4 * q]);
          F[4 * q + 1] = fmaf(wt, f4.y, F[4 * q + 1]);
          F[4 * q + 2] = fmaf(wt, f4.z, F[4 * q + 2]);
          F[4 * q + 3] = fmaf(wt, f4.w, F[4 * q + 3]);
        }
        const uint32_t q1 = base - start + kk + 1u;
        if (Tr > 0.f) {
          anchor = q1;
          t_anchor = Tr;
        }
        Tr = fmul(Tr, fsub(1.f, al));
        ++cnt;
        last = q1;
      }
    }
    tile_sync<NW>();
  }
  if (a.st_tile) write_tile_last<NW>(a, tile, last, s_ml);
  if (!inside) return;
  const int64_t P = (int64_t)a.cam.W * a.cam.H;
  const int64_t p = (int64_t)py * a.cam.W + px;
#pragma unroll
  for (int c = 0; c < CP; ++c)
    if (c < a.C) a.out[c * P + p] = a.bg ? fmaf(Tr, bg_value(a, c, P, p), F[c]) : F[c];
  a.t_final[p] = Tr;
  a.n_contrib[p] = cnt;
  if (a.st_last) {
    a.st_last[p] = last;
    a.st_anchor[p] = anchor;
    a.st_tanchor[p] = t_anchor;
  }
}

// ---------------------------------------------------------------------------
// Backward, bilinear splats
// ---------------------------------------------------------------------------

// Adds this tile's gradient share of every copy of the wavefront with
// `mine` set (points that lie in more than one tile) to the point's
// gradient with float atomics.  The shares are first staged as rows of
// CP + 4 floats (features, opacity, u, v, point index) in `tr`, 512 floats
// owned by this wavefront; then each group of CP lanes adds one row, so
// that one atomic instruction covers 64 / CP whole feature rows.
template <int CP>
__device__ __forceinline__ void add_split_shares(bool mine, uint32_t idx, const float (&g)[CP],
                                                 float go, float gu, float gv,
                                                 float* __restrict__ tr, const BlendArgs& a) {
  constexpr uint32_t RS = CP + 4;
  constexpr uint32_t ROWS = 512 / RS;
  constexpr uint32_t PER = 64 / CP;
  const uint64_t m = __ballot(mine);
  if (m == 0ull) return;
  const uint32_t lane = __lane_id();
  const uint32_t total = (uint32_t)__popcll(m);
  const uint32_t r = mbcnt64(m);
  const uint32_t C = (uint32_t)a.C;
  for (uint32_t b0 = 0; b0 < total; b0 += ROWS) {
    const uint32_t nb = min(total - b0, ROWS);
    if (mine && r >= b0 && r < b0 + nb) {
      float4* d = reinterpret_cast<float4*>(tr + (r - b0) * RS);
#pragma unroll
      for (int q = 0; q < CP / 4; ++q)
        d[q] = make_float4(g[4 * q], g[4 * q + 1], g[4 * q + 2], g[4 * q + 3]);
      d[CP / 4] = make_float4(go, gu, gv, __uint_as_float(idx));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // every LDS read of the batch is issued before its first atomic
    constexpr uint32_t IT = (ROWS + PER - 1) / PER;  // feature rows per lane
    constexpr uint32_t IS = (4 * ROWS + 63) / 64;    // scalar slots per lane
    const uint32_t c = lane % CP;
    uint32_t fp[IT], sp[IS];
    float fv[IT], sv[IS];
#pragma unroll
    for (uint32_t it = 0; it < IT; ++it) {
      const uint32_t row = lane / CP + it * PER;
      const bool ok = c < (uint32_t)C && row < nb;
      fp[it] = ok ? __float_as_uint(tr[row * RS + CP + 3]) : 0u;
      fv[it] = ok ? tr[row * RS + c] : 0.f;
    }
    // opacity and position: one 16-byte scalar row per point, 4 lanes each
#pragma unroll
    for (uint32_t is = 0; is < IS; ++is) {
      const uint32_t k = lane + 64u * is, row = k >> 2, comp = k & 3u;
      const bool ok = row < nb && comp < 3u;
      sp[is] = ok ? __float_as_uint(tr[row * RS + CP + 3]) : 0u;
      sv[is] = ok ? tr[row * RS + CP + comp] : 0.f;
    }
#pragma unroll
    for (uint32_t it = 0; it < IT; ++it)
      if (c < (uint32_t)C && lane / CP + it * PER < nb)
        atomicAdd(a.grad_feat + (size_t)fp[it] * C + c, fv[it]);
#pragma unroll
    for (uint32_t is = 0; is < IS; ++is) {
      const uint32_t k = lane + 64u * is;
      if ((k >> 2) < nb && (k & 3u) < 3u)
        atomicAdd(reinterpret_cast<float*>(a.gsc + sp[is]) + (k & 3u), sv[is]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}
// The 8x8 backward's gradient writes for one virtual chunk: every copy with
// `has` set is staged in `tr` as a row of CP + 4 floats (features, opacity,
// u, v, point index with bit 31 set for a single-tile point).  A single-tile
// point's row is stored whole, Q = CP / 4 neighbouring lanes writing the
// 16-byte quads of one row, so one store instruction covers 64 / Q rows; a
// split point's share is added with float atomics, CP lanes per row.
template <int CP>
__device__ __forceinline__ void write_chunk_rows(bool has, bool single, uint32_t idx,
                                                 const float (&g)[CP], float go, float gu,
                                                 float gv, float* __restrict__ tr,
                                                 const BlendArgs& a) {
  constexpr uint32_t RS = CP + 4;
  constexpr uint32_t ROWS = 512 / RS;
  constexpr uint32_t PER = 64 / CP;
  constexpr uint32_t Q = CP / 4;
  constexpr uint32_t IT = (ROWS + PER - 1) / PER;  // feature slots per lane (atomics)
  constexpr uint32_t IS = (4 * ROWS + 63) / 64;    // scalar slots per lane
  constexpr uint32_t IQ = (ROWS * Q + 63) / 64;    // quad slots per lane (stores)
  const uint64_t m = __ballot(has);
  if (m == 0ull) return;
  const uint32_t lane = __lane_id();
  const uint32_t total = (uint32_t)__popcll(m);
  const uint32_t r = mbcnt64(m);
  const uint32_t C = (uint32_t)a.C;
  const uint32_t kSingle = 0x80000000u;
  for (uint32_t b0 = 0; b0 < total; b0 += ROWS) {
    const uint32_t nb = min(total - b0, ROWS);
    if (has && r >= b0 && r < b0 + nb) {
      float4* d = reinterpret_cast<float4*>(tr + (r - b0) * RS);
#pragma unroll
      for (int q = 0; q < CP / 4; ++q)
        d[q] = make_float4(g[4 * q], g[4 * q + 1], g[4 * q + 2], g[4 * q + 3]);
      d[CP / 4] = make_float4(go, gu, gv, __uint_as_float(idx | (single ? kSingle : 0u)));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // single-tile rows: whole-row stores
    if (C == CP) {
#pragma unroll
      for (uint32_t iq = 0; iq < IQ; ++iq) {
        const uint32_t slot = lane + 64u * iq, row = slot / Q, qd = slot % Q;
        if (row < nb) {
          const uint32_t w = __float_as_uint(tr[row * RS + CP + 3]);
          if (w & kSingle) {
            const float4 v = *reinterpret_cast<const float4*>(tr + row * RS + 4 * qd);
            reinterpret_cast<float4*>(a.grad_feat + (size_t)(w & ~kSingle) * C)[qd] = v;
          }
        }
      }
    } else {
      for (uint32_t slot = lane; slot < nb * CP; slot += 64u) {
        const uint32_t row = slot / CP, c = slot % CP;
        const uint32_t w = __float_as_uint(tr[row * RS + CP + 3]);
        if ((w & kSingle) && c < C) a.grad_feat[(size_t)(w & ~kSingle) * C + c] = tr[row * RS + c];
      }
    }
    for (uint32_t row = lane; row < nb; row += 64u) {
      const uint32_t w = __float_as_uint(tr[row * RS + CP + 3]);
      if (w & kSingle)
        a.gsc[w & ~kSingle] =
            make_float4(tr[row * RS + CP], tr[row * RS + CP + 1], tr[row * RS + CP + 2], 0.f);
    }
    // split rows: every LDS read of the batch is issued before its first atomic
    const uint32_t c = lane % CP;
    uint32_t fp[IT], sp[IS];
    float fv[IT], sv[IS];
#pragma unroll
    for (uint32_t it = 0; it < IT; ++it) {
      const uint32_t row = lane / CP + it * PER;
      const bool ok = c < C && row < nb;
      fp[it] = ok ? __float_as_uint(tr[row * RS + CP + 3]) : kSingle;
      fv[it] = ok ? tr[row * RS + c] : 0.f;
    }
#pragma unroll
    for (uint32_t is = 0; is < IS; ++is) {
      const uint32_t k = lane + 64u * is, row = k >> 2, comp = k & 3u;
      const bool ok = row < nb && comp < 3u;
      sp[is] = ok ? __float_as_uint(tr[row * RS + CP + 3]) : kSingle;
      sv[is] = ok ? tr[row * RS + CP + comp] : 0.f;
    }
#pragma unroll
    for (uint32_t it = 0; it < IT; ++it)
      if (!(fp[it] & kSingle)) atomicAdd(a.grad_feat + (size_t)fp[it] * C + c, fv[it]);
#pragma unroll
    for (uint32_t is = 0; is < IS; ++is) {
      const uint32_t k = lane + 64u * is;
      if (!(sp[is] & kSingle))
        atomicAdd(reinterpret_cast<float*>(a.gsc + sp[is]) + (k & 3u), sv[is]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

template <int T, int CP, typename FT, bool FULL>
__device__ __forceinline__ void blend_bwd_bilinear_tile(const BlendArgs& a, uint32_t tile) {
  using G = TileGeom<T>;
  constexpr int NW = G::NW, CH = G::CHUNK, MW = G::MW;
  __shared__ float4 s_geo[CH];
  __shared__ unsigned long long s_mask[2][G::NTH * MW];
  __shared__ unsigned long long s_need[MW];
  __shared__ float s_gf[CH * 4];                          // per (copy, corner): G . f
  __shared__ __align__(16) float2 s_acc[CH * 4];  // per (copy, corner): (T alpha, dL/dalpha)
  __shared__ __align__(16) float s_G[G::NTH * fpad(CP)];  // dL/dF of every pixel of the tile
  __shared__ float s_red[NW][CP];

  const int tid = threadIdx.x;
  const int tx = (int)(tile % (uint32_t)a.opts.ntx), ty = (int)(tile / (uint32_t)a.opts.ntx);
  const int lx = tid % T, ly = tid / T;
  const int px = tx * T + lx, py = ty * T + ly;
  const bool inside = px < a.cam.W && py < a.cam.H;
  const uint32_t start = a.ranges[tile], end = a.ranges[tile + 1];
  const int64_t P = (int64_t)a.cam.W * a.cam.H;
  const int64_t p = (int64_t)py * a.cam.W + px;
  const int C = a.C;
  const bool stager = tid < CH;

  float Gv[CP];
  float gB = 0.f, GT = 0.f, Tf = 0.f, t_anchor = 0.f;
  uint32_t last = 0, anchor = 0;
#pragma unroll
  for (int c = 0; c < CP; ++c) Gv[c] = (inside && c < C) ? a.grad_out[c * P + p] : 0.f;
  if (inside) {
    GT = a.grad_t ? a.grad_t[p] : 0.f;
    last = a.st_last[p];
    anchor = a.st_anchor[p];
    t_anchor = a.st_tanchor[p];
    Tf = a.t_final[p];
    if (a.bg)
      for (int c = 0; c < C; ++c) gB = fmaf(Gv[c], bg_value(a, c, P, p), gB);
    if (a.bg_image && a.grad_bg)  // dL/df_bg(pixel) = T_final G
      for (int c = 0; c < C; ++c) a.grad_bg[c * P + p] = Tf * Gv[c];
  }
  {
    float4* d4 = reinterpret_cast<float4*>(s_G + tid * fpad(CP));
#pragma unroll
    for (int q = 0; q < CP / 4; ++q)
      d4[q] = make_float4(Gv[4 * q], Gv[4 * q + 1], Gv[4 * q + 2], Gv[4 * q + 3]);
  }
  tile_sync<NW>();  // s_G is read by the copies' threads below

  // background: this tile's share of sum_p T_final G
  if (a.bg_partial) {
#pragma unroll
    for (int c = 0; c < CP; ++c) {
      float v = Tf * Gv[c];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if ((tid & 63) == 0) s_red[tid >> 6][c] = v;
    }
    __syncthreads();
    if (tid < C) {
      float v = 0.f;
#pragma unroll
      for (int w = 0; w < NW; ++w) v += s_red[w][tid];
      a.bg_partial[(size_t)tile * C + tid] = v;
    }
  }

  // the forward pass blended nothing beyond list position st_tile[tile]
  const uint32_t maxlast = min(a.st_tile[tile], end - start);
  const int nchunks = (int)((maxlast + CH - 1) / CH);

  Entry e;  // list entries of the chunk whose coverage is built next
  e.valid = false;
  e.idx = e.lp = 0;
  Prefetch<CP, FT, FULL> pf;  // point data of the chunk staged next
  pf.valid = false;
  bool psingle = false;        // whether that point lies in this tile only
  if (nchunks > 0) {
    const int c0 = nchunks - 1;
    e.load(a, stager, start + (uint32_t)c0 * CH + tid, end);
    if constexpr (NW > 1) {
      if (tid < MW) s_need[tid] = 0ull;
    }
    build_coverage<T>(s_mask[c0 & 1], e);
    const bool nd = copy_needed<T>(s_mask[c0 & 1], last > (uint32_t)c0 * CH, s_need);
    pf.fetch(a, e.valid && nd, e.idx);
    psingle = single_tile<T>(e.lp, tx, ty, a.cam.W, a.cam.H);
    if (nchunks >= 2) e.load(a, stager, start + (uint32_t)(c0 - 1) * CH + tid, end);
  }

  float Pi = 1.f, Tcur = 0.f;
  for (int ci = nchunks - 1; ci >= 0; --ci) {
    const int b = ci & 1;
    const uint32_t rb = (uint32_t)ci * CH;  // relative base of the chunk
    // stage this chunk's fetched copies
    const bool cur = pf.valid;
    const uint32_t cur_idx = pf.idx;
    const bool cur_single = psingle;
    float ca = 0.f, cb = 0.f, co = 0.f;
    int X0 = 0, Y0 = 0;
    if (cur) {
      // The replay needs G . f at each covered pixel; the copy's thread forms
      // these four dot products from its features in registers, so the
      // features themselves never pass through LDS.
      const Footprint f = bilinear_footprint(pf.p.x, pf.p.y, a.cam.W, a.cam.H);
      ca = f.a; cb = f.b; co = pf.p.z; X0 = f.x0; Y0 = f.y0;
      s_geo[tid] = make_float4(f.a, f.b, pf.p.z, __uint_as_float(pack_xy(f.x0, f.y0)));
      float fv[CP];
      pf.f.to_f32(fv);
      const int x0 = X0 - tx * T, y0 = Y0 - ty * T;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int qx = x0 + (k & 1), qy = y0 + (k >> 1);
        float d = 0.f;
        if (qx >= 0 && qx < T && qy >= 0 && qy < T) {
          const float4* gp = reinterpret_cast<const float4*>(s_G + (qy * T + qx) * fpad(CP));
#pragma unroll
          for (int q = 0; q < CP / 4; ++q) {
            const float4 g4 = gp[q];
            d = fmaf(g4.x, fv[4 * q], d);
            d = fmaf(g4.y, fv[4 * q + 1], d);
            d = fmaf(g4.z, fv[4 * q + 2], d);
            d = fmaf(g4.w, fv[4 * q + 3], d);
          }
        }
        s_gf[tid * 4 + k] = d;
        s_acc[tid * 4 + k] = make_float2(0.f, 0.f);
      }
    }
    tile_sync<NW>();
    // coverage of the previous chunk; fetch what it needs while this one is replayed
    if (ci >= 1) {
      if constexpr (NW > 1) {
        if (tid < MW) s_need[tid] = 0ull;
      }
      build_coverage<T>(s_mask[b ^ 1], e);
      const bool nd = copy_needed<T>(s_mask[b ^ 1], last > rb - CH, s_need);
      pf.fetch(a, e.valid && nd, e.idx);
      psingle = single_tile<T>(e.lp, tx, ty, a.cam.W, a.cam.H);
      if (ci >= 2) e.load(a, stager, start + rb - 2 * CH + tid, end);
    }
    if (last > rb) {
      for (int w = MW - 1; w >= 0; --w) {
        unsigned long long m = s_mask[b][tid * MW + w];
        const uint32_t wb = rb + (uint32_t)w * 64;  // relative position of bit 0
        if (last <= wb) continue;
        const uint32_t lim = last - wb;             // positions < last are blended
        if (lim < 64) m &= (1ull << lim) - 1ull;
        while (m) {
          const int j = 63 - __clzll(m);
          m &= ~(1ull << j);
          const int kk = w * 64 + j;
          const uint32_t q1 = wb + (uint32_t)j + 1u;  // one past the relative position
          const float4 g = s_geo[kk];
          const uint32_t pk = __float_as_uint(g.w);
          const int dx = px - unpack_x(pk), dy = py - unpack_y(pk);
          const float wx = dx ? g.x : fsub(1.f, g.x);
          const float wy = dy ? g.y : fsub(1.f, g.y);
          const float al = fmul(g.z, fmul(wx, wy));
          const float om = fsub(1.f, al);
          float Tk;
          if (q1 > anchor)
            Tk = 0.f;
          else if (q1 == anchor)
            Tk = t_anchor;
          else
            Tk = __fdividef(Tcur, om);
          const float gf = s_gf[kk * 4 + dy * 2 + dx];
          const float da = Tk * (gf - gB) - GT * Tk * Pi;
          s_acc[kk * 4 + dy * 2 + dx] = make_float2(Tk * al, da);
          gB = fmaf(al, gf, om * gB);
          Pi = Pi * om;
          Tcur = Tk;
        }
      }
    }
    tile_sync<NW>();
    float gfeat[CP];
#pragma unroll
    for (int c = 0; c < CP; ++c) gfeat[c] = 0.f;
    float go = 0.f, gu = 0.f, gv = 0.f;
    if (cur) {
      const int x0 = X0 - tx * T, y0 = Y0 - ty * T;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int dx = k & 1, dy = k >> 1;
        const int qx = x0 + dx, qy = y0 + dy;
        if (qx < 0 || qx >= T || qy < 0 || qy >= T) continue;
        const float2 acc = s_acc[tid * 4 + k];
        const float4* gp = reinterpret_cast<const float4*>(s_G + (qy * T + qx) * fpad(CP));
#pragma unroll
        for (int q = 0; q < CP / 4; ++q) {
          const float4 g4 = gp[q];
          gfeat[4 * q] = fmaf(acc.x, g4.x, gfeat[4 * q]);
          gfeat[4 * q + 1] = fmaf(acc.x, g4.y, gfeat[4 * q + 1]);
          gfeat[4 * q + 2] = fmaf(acc.x, g4.z, gfeat[4 * q + 2]);
          gfeat[4 * q + 3] = fmaf(acc.x, g4.w, gfeat[4 * q + 3]);
        }
        const float wx = dx ? ca : 1.f - ca;
        const float wy = dy ? cb : 1.f - cb;
        go = fmaf(wx * wy, acc.y, go);
        gu = fmaf((dx ? 1.f : -1.f) * wy, acc.y, gu);
        gv = fmaf((dy ? 1.f : -1.f) * wx, acc.y, gv);
      }
      gu *= co;
      gv *= co;
      if (cur_single) {  // the only tile of this point: its whole gradient
        store_row<CP>(a.grad_feat + (size_t)cur_idx * C, gfeat, C);
        a.gsc[cur_idx] = make_float4(go, gu, gv, 0.f);
      }
    }
    // A point split over several tiles receives this tile's share by float
    // atomics, staged in this wavefront's quarter of s_acc (whose reads by
    // the corner sums above are done) so that each atomic instruction covers
    // whole point rows.
    add_split_shares<CP>(cur && !cur_single, cur_idx, gfeat, go, gu, gv,
                         reinterpret_cast<float*>(s_acc) + (tid >> 6) * 512, a);
    tile_sync<NW>();
  }
}

// Backward for 8x8 tiles with the sparse compaction of the forward: the
// part of the list the forward reached is read in super-chunks from the back;
// the copies covering a pixel whose blended range reaches them are compacted
// in list order and replayed in reverse, one virtual chunk of 64 at a time
// (the previous virtual chunk's point data is fetched during the replay).
template <int CP, typename FT, bool FULL>
__device__ __forceinline__ void blend_bwd_bilinear8_tile(const BlendArgs& a, uint32_t tile) {
  constexpr int T = 8;
  constexpr uint32_t SC = kSubs * 64;
  __shared__ float4 s_geo[64];
  __shared__ unsigned long long s_mask[64];
  __shared__ uint32_t s_q1[64];
  // per (copy, corner): (G . f, kNoAcc) from the staging until the corner's
  // pixel replays the copy, then (T alpha, dL/dalpha); kNoAcc (a NaN payload
  // that arithmetic never produces) marks a corner the pixel did not blend
  __shared__ __align__(16) float2 s_acc[64 * 4];
  constexpr uint32_t kNoAcc = 0x7fc0dea1u;
  __shared__ __align__(16) float s_G[64 * fpad(CP)];
  using PF = PointFetch<CP, FT, FULL>;
  __shared__ float4 s_prj[64];             // gathered projection records
  __shared__ uint4 s_fq[PF::QS * 64];      // gathered feature rows, row-major
  // the selection of the next virtual chunk shares the projection records'
  // space: it is published after the records were staged and read before
  // the gather that overwrites them (one wavefront, in program order)
  uint2* const s_sel = reinterpret_cast<uint2*>(s_prj);

  const uint32_t lane = threadIdx.x;
  const int tx = (int)(tile % (uint32_t)a.opts.ntx), ty = (int)(tile / (uint32_t)a.opts.ntx);
  const int px = tx * T + (int)(lane % T), py = ty * T + (int)(lane / T);
  const bool inside = px < a.cam.W && py < a.cam.H;
  const uint32_t start = a.ranges[tile], end = a.ranges[tile + 1];
  const int64_t P = (int64_t)a.cam.W * a.cam.H;
  const int64_t p = (int64_t)py * a.cam.W + px;
  const int C = a.C;

  // the forward pass blended nothing beyond list position st_tile[tile];
  // the entries of the last super-chunk it reached are loaded together with
  // this tile's upstream gradient and blend state
  const uint32_t maxlast = min(a.st_tile[tile], end - start);
  const uint32_t lend = start + maxlast;
  const int nsc = (int)((maxlast + SC - 1) / SC);
  SuperEntries nxt;
  if (nsc > 0) nxt.load(a, start + (uint32_t)(nsc - 1) * SC, lend);

  float gB = 0.f, GT = 0.f, Tf = 0.f, t_anchor = 0.f;
  uint32_t last = 0, anchor = 0;
  {
    float Gv[CP];
#pragma unroll
    for (int c = 0; c < CP; ++c) Gv[c] = (inside && c < C) ? a.grad_out[c * P + p] : 0.f;
    if (inside) {
      GT = a.grad_t ? a.grad_t[p] : 0.f;
      last = a.st_last[p];
      anchor = a.st_anchor[p];
      t_anchor = a.st_tanchor[p];
      Tf = a.t_final[p];
      if (a.bg)
        for (int c = 0; c < C; ++c) gB = fmaf(Gv[c], bg_value(a, c, P, p), gB);
      if (a.bg_image && a.grad_bg)  // dL/df_bg(pixel) = T_final G
        for (int c = 0; c < C; ++c) a.grad_bg[c * P + p] = Tf * Gv[c];
    }
    float4* d4 = reinterpret_cast<float4*>(s_G + lane * fpad(CP));
#pragma unroll
    for (int q = 0; q < CP / 4; ++q)
      d4[q] = make_float4(Gv[4 * q], Gv[4 * q + 1], Gv[4 * q + 2], Gv[4 * q + 3]);
    // background: this tile's share of sum_p T_final G
    if (a.bg_partial) {
#pragma unroll
      for (int c = 0; c < CP; ++c) {
        float v = Tf * Gv[c];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0 && c < C) a.bg_partial[(size_t)tile * C + c] = v;
      }
    }
  }
  tile_sync<1>();  // s_G is read by the copies' lanes below

  float Pi = 1.f, Tcur = 0.f;
  // the entries of the next super-chunk (towards the front) are loaded
  // while this one is compacted and replayed
  for (int k = nsc - 1; k >= 0; --k) {
    const uint32_t base = start + (uint32_t)k * SC;
    const SuperEntries cur = nxt;
    if (k >= 1) nxt.load(a, base - SC, lend);
    // a pixel takes part in chunk j if its blended range reaches the chunk
    uint64_t act[kSubs];
#pragma unroll
    for (int j = 0; j < kSubs; ++j) act[j] = __ballot(last > base - start + (uint32_t)j * 64u);
    Compaction cp;
    cp.build(cur, base, lend, act);
    const int nvc = (int)((cp.total + 63u) / 64u);
    PF pf;
    uint32_t plp = 0, pq1 = 0;
    if (nvc > 0) {
      const uint32_t vb = (uint32_t)(nvc - 1) * 64u;
      cp.publish(cur, vb, s_sel);
      tile_sync<1>();
      const bool has = vb + lane < cp.total;
      const uint2 sl = has ? s_sel[lane] : make_uint2(0u, 0u);
      pf.fetch(a, has, sl.x, s_prj, s_fq);
      plp = sl.y & 0xffffu;
      pq1 = base - start + (sl.y >> 16) + 1u;
      tile_sync<1>();
    }
    for (int v = nvc - 1; v >= 0; --v) {
      // stage virtual chunk v: geometry, G . f at the covered pixels, coverage
      const bool cur_has = pf.valid;
      const uint32_t cur_idx = pf.idx;
      const uint32_t cur_lp = plp;
      float ca = 0.f, cb = 0.f, co = 0.f;
      int X0 = 0, Y0 = 0;
      pf.wait();
      s_mask[lane] = 0ull;
      tile_sync<1>();
      if (cur_has) {
        const float4 pp = pf.proj(s_prj, lane);
        const Footprint f = bilinear_footprint(pp.x, pp.y, a.cam.W, a.cam.H);
        ca = f.a; cb = f.b; co = pp.z; X0 = f.x0; Y0 = f.y0;
        s_geo[lane] = make_float4(f.a, f.b, pp.z, __uint_as_float(pack_xy(f.x0, f.y0)));
        s_q1[lane] = pq1;
        float fv[CP];
        pf.row(s_fq, lane, fv);
        const int x0 = X0 - tx * T, y0 = Y0 - ty * T;
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) {
          const int qx = x0 + (c4 & 1), qy = y0 + (c4 >> 1);
          float d = 0.f;
          if (qx >= 0 && qx < T && qy >= 0 && qy < T) {
            const float4* gp = reinterpret_cast<const float4*>(s_G + (qy * T + qx) * fpad(CP));
#pragma unroll
            for (int q = 0; q < CP / 4; ++q) {
              const float4 g4 = gp[q];
              d = fmaf(g4.x, fv[4 * q], d);
              d = fmaf(g4.y, fv[4 * q + 1], d);
              d = fmaf(g4.z, fv[4 * q + 2], d);
              d = fmaf(g4.w, fv[4 * q + 3], d);
            }
          }
          s_acc[lane * 4 + c4] = make_float2(d, __uint_as_float(kNoAcc));
        }
        uint64_t pm = splat_pixels8(cur_lp);
        const unsigned long long bit = 1ull << lane;
        while (pm) {
          const int b = __ffsll((unsigned long long)pm) - 1;
          pm &= pm - 1ull;
          atomicOr(&s_mask[b], bit);
        }
      }
      tile_sync<1>();
      // fetch virtual chunk v - 1 while v is replayed
      if (v >= 1) {
        const uint32_t vb = (uint32_t)(v - 1) * 64u;
        cp.publish(cur, vb, s_sel);
        tile_sync<1>();
        const uint2 sl = s_sel[lane];  // virtual chunks below the last are full
        pf.fetch(a, true, sl.x, s_prj, s_fq);
        plp = sl.y & 0xffffu;
        pq1 = base - start + (sl.y >> 16) + 1u;
      }
      // reverse replay of this pixel's fragments in the chunk
      unsigned long long m = s_mask[lane];
      while (m) {
        const int kk = 63 - __clzll(m);
        m &= ~(1ull << kk);
        const uint32_t q1 = s_q1[kk];
        if (q1 > last) continue;  // behind this pixel's last blended fragment
        const float4 g = s_geo[kk];
        const uint32_t pk = __float_as_uint(g.w);
        const int dx = px - unpack_x(pk), dy = py - unpack_y(pk);
        const float wx = dx ? g.x : fsub(1.f, g.x);
        const float wy = dy ? g.y : fsub(1.f, g.y);
        const float al = fmul(g.z, fmul(wx, wy));
        const float om = fsub(1.f, al);
        float Tk;
        if (q1 > anchor)
          Tk = 0.f;
        else if (q1 == anchor)
          Tk = t_anchor;
        else
          Tk = __fdividef(Tcur, om);
        const float gf = s_acc[kk * 4 + dy * 2 + dx].x;
        const float da = Tk * (gf - gB) - GT * Tk * Pi;
        s_acc[kk * 4 + dy * 2 + dx] = make_float2(Tk * al, da);
        gB = fmaf(al, gf, om * gB);
        Pi = Pi * om;
        Tcur = Tk;
      }
      tile_sync<1>();
      float gfeat[CP];
#pragma unroll
      for (int c = 0; c < CP; ++c) gfeat[c] = 0.f;
      float go = 0.f, gu = 0.f, gv = 0.f;
      bool single = false;
      if (cur_has) {
        const int x0 = X0 - tx * T, y0 = Y0 - ty * T;
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) {
          const int dx = c4 & 1, dy = c4 >> 1;
          const int qx = x0 + dx, qy = y0 + dy;
          if (qx < 0 || qx >= T || qy < 0 || qy >= T) continue;
          float2 acc = s_acc[lane * 4 + c4];
          if (__float_as_uint(acc.y) == kNoAcc) acc = make_float2(0.f, 0.f);
          const float4* gp = reinterpret_cast<const float4*>(s_G + (qy * T + qx) * fpad(CP));
#pragma unroll
          for (int q = 0; q < CP / 4; ++q) {
            const float4 g4 = gp[q];
            gfeat[4 * q] = fmaf(acc.x, g4.x, gfeat[4 * q]);
            gfeat[4 * q + 1] = fmaf(acc.x, g4.y, gfeat[4 * q + 1]);
            gfeat[4 * q + 2] = fmaf(acc.x, g4.z, gfeat[4 * q + 2]);
            gfeat[4 * q + 3] = fmaf(acc.x, g4.w, gfeat[4 * q + 3]);
          }
          const float wx = dx ? ca : 1.f - ca;
          const float wy = dy ? cb : 1.f - cb;
          go = fmaf(wx * wy, acc.y, go);
          gu = fmaf((dx ? 1.f : -1.f) * wy, acc.y, gu);
          gv = fmaf((dy ? 1.f : -1.f) * wx, acc.y, gv);
        }
        gu *= co;
        gv *= co;
        // the only tile of a single-tile point writes its whole gradient
        single = single_tile<T>(cur_lp, tx, ty, a.cam.W, a.cam.H);
      }
      write_chunk_rows<CP>(cur_has, single, cur_idx, gfeat, go, gu, gv,
                           reinterpret_cast<float*>(s_acc), a);
      tile_sync<1>();
    }
  }
}

// ---------------------------------------------------------------------------
// Kernels: one workgroup per tile of one view, or one workgroup per
// (view, tile) slot of a batch's queue
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Backward, Gaussian splats
// ---------------------------------------------------------------------------
//
// Every pixel replays its blended fragments back to front as above.  A
// Gaussian copy covers many pixels of the tile, so its gradient is a sum over
// them, formed in two phases per chunk of copies.  In the replay the pixels
// step through the chunk's copies together (back to front); for every copy
// whose footprint rectangle holds the pixel, the pixel's lane writes two
// numbers into a (copy, pixel) table in LDS: T_k alpha_k and
// e = w dL/dalpha_k (zero where the pixel has no blended fragment of the
// copy).  Then each copy's own thread walks its rectangle (clipped to the
// tile) and sums, in parallel over the chunk's copies:
//   dL/df += (T alpha) G (G of the pixel, from LDS), dL/do += e,
//   screen-space (s2 = r^2 + dilation): dL/du += o e dx / s2,
//   dL/dv += o e dy / s2;  world-space (conic [[A, B], [B, C]] = S^-1):
//   dL/du += o e (A dx + B dy), dL/dv += o e (B dx + C dy) through the offset
//   d = (px + 1/2 - u, py + 1/2 - v), and dL/dA += -o e dx^2 / 2,
//   dL/dB += -o e dx dy, dL/dC += -o e dy^2 / 2,
// then chains (A, B, C) -> covariance (a, b, c) -> (u, v, Z) (the covariance
// a function of u, v through X/Z, Y/Z and of Z through fx/Z, fy/Z) and writes
// the point's gradient (a point inside this tile only) or adds this tile's
// share with float atomics.

// This tile's gradient share of every Gaussian copy of the wavefront with
// `mine` set, added to the point's gradient with float atomics: staged as
// rows of CP + 8 floats (features, dL/do, dL/du, dL/dv, dL/dZ, point index)
// in `tr` (512 floats owned by this wavefront), then each group of CP lanes
// adds one row, so that one atomic instruction covers 64 / CP point rows.
// The scalar row gets its first `nsc` components added (3, or 4 with dL/dZ).
template <int CP>
__device__ __forceinline__ void add_gauss_shares(bool mine, uint32_t idx, const float (&g)[CP],
                                                 float4 sc, uint32_t nsc,
                                                 float* __restrict__ tr, const BlendArgs& a) {
  constexpr uint32_t RS = CP + 8;
  constexpr uint32_t ROWS = 512 / RS;
  constexpr uint32_t PER = 64 / CP;
  const uint64_t m = __ballot(mine);
  if (m == 0ull) return;
  const uint32_t lane = __lane_id();
  const uint32_t total = (uint32_t)__popcll(m);
  const uint32_t r = mbcnt64(m);
  const uint32_t C = (uint32_t)a.C;
  for (uint32_t b0 = 0; b0 < total; b0 += ROWS) {
    const uint32_t nb = min(total - b0, ROWS);
    if (mine && r >= b0 && r < b0 + nb) {
      float4* d = reinterpret_cast<float4*>(tr + (r - b0) * RS);
#pragma unroll
      for (int q = 0; q < CP / 4; ++q)
        d[q] = make_float4(g[4 * q], g[4 * q + 1], g[4 * q + 2], g[4 * q + 3]);
      d[CP / 4] = sc;
      d[CP / 4 + 1] = make_float4(__uint_as_float(idx), 0.f, 0.f, 0.f);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // every LDS read of the batch is issued before its first atomic
    constexpr uint32_t IT = (ROWS + PER - 1) / PER;  // feature rows per lane
    constexpr uint32_t IS = (4 * ROWS + 63) / 64;    // scalar slots per lane
    const uint32_t c = lane % CP;
    uint32_t fp[IT], sp[IS];
    float fv[IT], sv[IS];
#pragma unroll
    for (uint32_t it = 0; it < IT; ++it) {
      const uint32_t row = lane / CP + it * PER;
      const bool ok = c < C && row < nb;
      fp[it] = ok ? __float_as_uint(tr[row * RS + CP + 4]) : 0u;
      fv[it] = ok ? tr[row * RS + c] : 0.f;
    }
#pragma unroll
    for (uint32_t is = 0; is < IS; ++is) {
      const uint32_t k = lane + 64u * is, row = k >> 2, comp = k & 3u;
      const bool ok = row < nb && comp < nsc;
      sp[is] = ok ? __float_as_uint(tr[row * RS + CP + 4]) : 0u;
      sv[is] = ok ? tr[row * RS + CP + comp] : 0.f;
    }
#pragma unroll
    for (uint32_t it = 0; it < IT; ++it)
      if (c < C && lane / CP + it * PER < nb)
        atomicAdd(a.grad_feat + (size_t)fp[it] * C + c, fv[it]);
#pragma unroll
    for (uint32_t is = 0; is < IS; ++is) {
      const uint32_t k = lane + 64u * is;
      if ((k >> 2) < nb && (k & 3u) < nsc)
        atomicAdd(reinterpret_cast<float*>(a.gsc + sp[is]) + (k & 3u), sv[is]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

template <int T, int CP, typename FT, bool FULL>
__device__ __forceinline__ void blend_bwd_gauss_tile(const BlendArgs& a, uint32_t tile) {
  using G = TileGeom<T>;
  constexpr int NW = G::NW, NTH = G::NTH;
  // copies per chunk: the (copy, pixel) tables stay at 2 x 8 KB
  constexpr int CH = 2048 / NTH;
  constexpr int TS = NTH + 1;  // table row stride (a copy's row; odd: no bank conflicts)
  __shared__ float4 s_g0[CH];
  __shared__ float4 s_g1[CH];
  __shared__ __align__(16) float s_feat[CH * fpad(CP)];
  __shared__ __align__(16) float s_G[NTH * fpad(CP)];  // dL/dF of every pixel of the tile
  __shared__ __align__(16) float s_ta[CH * TS];        // T alpha per (copy, pixel)
  __shared__ __align__(16) float s_e[CH * TS];         // w dL/dalpha per (copy, pixel)
  __shared__ unsigned long long s_pm[CH * NW];          // pixel masks of the staged copies
  __shared__ float s_red[NW][CP];

  const int tid = threadIdx.x;
  const int tx = (int)(tile % (uint32_t)a.opts.ntx), ty = (int)(tile / (uint32_t)a.opts.ntx);
  const int px = tx * T + tid % T, py = ty * T + tid / T;
  const bool inside = px < a.cam.W && py < a.cam.H;
  const uint32_t start = a.ranges[tile], end = a.ranges[tile + 1];
  const int64_t P = (int64_t)a.cam.W * a.cam.H;
  const int64_t p = (int64_t)py * a.cam.W + px;
  const int C = a.C;
  const bool ewa = a.opts.splat == INPC_SPLAT_EWA;
  const float thr_ewa = fmul(a.opts.cutoff, a.opts.cutoff);
  const float pxc = fadd((float)px, 0.5f), pyc = fadd((float)py, 0.5f);
  const bool stager = tid < CH;

  float Gv[CP];
  float gB = 0.f, GT = 0.f, Tf = 0.f, t_anchor = 0.f;
  uint32_t last = 0, anchor = 0;
#pragma unroll
  for (int c = 0; c < CP; ++c) Gv[c] = (inside && c < C) ? a.grad_out[c * P + p] : 0.f;
  if (inside) {
    GT = a.grad_t ? a.grad_t[p] : 0.f;
    last = a.st_last[p];
    anchor = a.st_anchor[p];
    t_anchor = a.st_tanchor[p];
    Tf = a.t_final[p];
    if (a.bg)
      for (int c = 0; c < C; ++c) gB = fmaf(Gv[c], bg_value(a, c, P, p), gB);
    if (a.bg_image && a.grad_bg)  // dL/df_bg(pixel) = T_final G
      for (int c = 0; c < C; ++c) a.grad_bg[c * P + p] = Tf * Gv[c];
  }
  {
    float4* d4 = reinterpret_cast<float4*>(s_G + tid * fpad(CP));
#pragma unroll
    for (int q = 0; q < CP / 4; ++q)
      d4[q] = make_float4(Gv[4 * q], Gv[4 * q + 1], Gv[4 * q + 2], Gv[4 * q + 3]);
  }
  if (a.bg_partial) {  // background: this tile's share of sum_p T_final G
#pragma unroll
    for (int c = 0; c < CP; ++c) {
      float v = Tf * Gv[c];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if ((tid & 63) == 0) s_red[tid >> 6][c] = v;
    }
    __syncthreads();
    if (tid < C) {
      float v = 0.f;
#pragma unroll
      for (int w = 0; w < NW; ++w) v += s_red[w][tid];
      a.bg_partial[(size_t)tile * C + tid] = v;
    }
  }

  // the forward pass blended nothing beyond list position st_tile[tile]
  const uint32_t maxlast = min(a.st_tile[tile], end - start);
  const int nchunks = (int)((maxlast + CH - 1) / CH);
  auto list_at = [&](uint32_t q) { return a.list[q < end ? q : end - 1]; };

  Prefetch<CP, FT, FULL> pf;
  pf.valid = false;
  if (nchunks > 0) {
    const uint32_t rb0 = (uint32_t)(nchunks - 1) * CH;
    pf.fetch(a, stager && rb0 + tid < maxlast, list_at(start + rb0 + tid));
  }

  float Pi = 1.f, Tcur = 0.f;
  for (int ci = nchunks - 1; ci >= 0; --ci) {
    const uint32_t rb = (uint32_t)ci * CH;
    const int nh = (int)min((uint32_t)CH, maxlast - rb);
    const bool cur = pf.valid;
    const uint32_t cur_idx = pf.idx;
    const float cur_z = pf.p.w;
    if (cur) {
      stage_gauss(a, ewa, pf.p, &s_g0[tid], &s_g1[tid]);
      rect_pixel_mask<T, NW>(__float_as_uint(s_g1[tid].y), __float_as_uint(s_g1[tid].z), tx, ty,
                             &s_pm[tid * NW]);
      pf.f.store_f32(s_feat + tid * fpad(CP));
    }
    if (ci >= 1) pf.fetch(a, stager, list_at(start + rb - CH + tid));
    tile_sync<NW>();  // staged copies (and, the first time, s_G) visible
    // replay: the (copy, pixel) table entries of every copy whose rectangle
    // holds this pixel, back to front
    unsigned long long m = candidates<NW>(s_pm, 0, nh, tid >> 6, (uint32_t)tid & 63u);
    while (m) {
      const int kk = 63 - __clzll(m);
      m &= ~(1ull << kk);
      const float4 g1 = s_g1[kk];
      const uint32_t q1 = rb + (uint32_t)kk + 1u;  // one past the relative position
      float ta = 0.f, e = 0.f;
      if (q1 <= last) {
        const float4 g0 = s_g0[kk];
        float d2;
        if (gauss_inside(ewa, thr_ewa, g0, g1, fsub(pxc, g0.x), fsub(pyc, g0.y), d2)) {
          const float w = gauss_value(ewa, d2, g0.w);
          const float al = g0.z * w;
          const float om = fsub(1.f, al);
          float Tk;
          if (q1 > anchor)
            Tk = 0.f;
          else if (q1 == anchor)
            Tk = t_anchor;
          else
            Tk = __fdividef(Tcur, om);
          const float4* fr = reinterpret_cast<const float4*>(s_feat + kk * fpad(CP));
          float gf = 0.f;
#pragma unroll
          for (int q = 0; q < CP / 4; ++q) {
            const float4 f4 = fr[q];
            gf = fmaf(Gv[4 * q], f4.x, gf);
            gf = fmaf(Gv[4 * q + 1], f4.y, gf);
            gf = fmaf(Gv[4 * q + 2], f4.z, gf);
            gf = fmaf(Gv[4 * q + 3], f4.w, gf);
          }
          const float da = Tk * (gf - gB) - GT * Tk * Pi;
          ta = Tk * al;
          e = da * w;
          gB = fmaf(al, gf, om * gB);
          Pi = Pi * om;
          Tcur = Tk;
        }
      }
      s_ta[kk * TS + tid] = ta;
      s_e[kk * TS + tid] = e;
    }
    tile_sync<NW>();
    // the copy's thread: its rectangle's table entries summed, chained, written
    float gfeat[CP];
#pragma unroll
    for (int c = 0; c < CP; ++c) gfeat[c] = 0.f;
    float4 sc = make_float4(0.f, 0.f, 0.f, 0.f);
    bool touched = false, single = false;
    if (cur) {
      const float4 g0 = s_g0[tid], g1 = s_g1[tid];
      const uint32_t lo = __float_as_uint(g1.y), hi = __float_as_uint(g1.z);
      const int x0 = max(unpack_x(lo) - tx * T, 0), x1 = min(unpack_x(hi) - tx * T, T - 1);
      const int y0 = max(unpack_y(lo) - ty * T, 0), y1 = min(unpack_y(hi) - ty * T, T - 1);
      single = (unpack_x(lo) >> G::SH) == (unpack_x(hi) >> G::SH) &&
               (unpack_y(lo) >> G::SH) == (unpack_y(hi) >> G::SH);
      float se = 0.f, su = 0.f, sv = 0.f, sxx = 0.f, sxy = 0.f, syy = 0.f;
      const float* rta = s_ta + tid * TS;
      const float* re = s_e + tid * TS;
      for (int y = y0; y <= y1; ++y) {
        const float dy = fsub(fadd((float)(ty * T + y), 0.5f), g0.y);
        for (int x = x0; x <= x1; ++x) {
          const int q = y * T + x;
          const float ta = rta[q], e = re[q];
          if (ta == 0.f && e == 0.f) continue;
          touched = true;
          const float4* gp = reinterpret_cast<const float4*>(s_G + q * fpad(CP));
#pragma unroll
          for (int k = 0; k < CP / 4; ++k) {
            const float4 g4 = gp[k];
            gfeat[4 * k] = fmaf(ta, g4.x, gfeat[4 * k]);
            gfeat[4 * k + 1] = fmaf(ta, g4.y, gfeat[4 * k + 1]);
            gfeat[4 * k + 2] = fmaf(ta, g4.z, gfeat[4 * k + 2]);
            gfeat[4 * k + 3] = fmaf(ta, g4.w, gfeat[4 * k + 3]);
          }
          const float dx = fsub(fadd((float)(tx * T + x), 0.5f), g0.x);
          se += e;
          if (ewa) {
            su = fmaf(e, g0.w * dx + g1.x * dy, su);
            sv = fmaf(e, g1.x * dx + g1.w * dy, sv);
            sxx = fmaf(e, dx * dx, sxx);
            sxy = fmaf(e, dx * dy, sxy);
            syy = fmaf(e, dy * dy, syy);
          } else {
            su = fmaf(e, dx, su);
            sv = fmaf(e, dy, sv);
          }
        }
      }
      const float o = g0.z;
      float gu, gv, gz = 0.f;
      if (!ewa) {
        gu = o * su / g0.w;
        gv = o * sv / g0.w;
      } else {
        const EwaCov k = ewa_cov(g0.x, g0.y, cur_z, a.cam, a.opts.dilation, a.opts.ewa_sigma);
        const float gA = -0.5f * o * sxx, gBc = -o * sxy, gC = -0.5f * o * syy;
        const float inv = 1.f / (k.a * k.c - k.b * k.b);
        const float ga = (-k.c * k.c * gA + k.b * k.c * gBc - k.b * k.b * gC) * inv * inv;
        const float gb = (2.f * k.b * k.c * gA - (k.a * k.c + k.b * k.b) * gBc +
                          2.f * k.a * k.b * gC) * inv * inv;
        const float gc = (-k.b * k.b * gA + k.a * k.b * gBc - k.a * k.a * gC) * inv * inv;
        const float kxx = k.s2w * k.jx * k.jx, kxy = k.s2w * k.jx * k.jy,
                    kyy = k.s2w * k.jy * k.jy;
        gu = o * su + (ga * kxx * 2.f * k.xh + gb * kxy * k.yh) / a.cam.fx;
        gv = o * sv + (gb * kxy * k.xh + gc * kyy * 2.f * k.yh) / a.cam.fy;
        gz = -2.f / cur_z *
             (ga * kxx * (1.f + k.xh * k.xh) + gb * kxy * (k.xh * k.yh) +
              gc * kyy * (1.f + k.yh * k.yh));
      }
      sc = make_float4(se, gu, gv, gz);
      if (touched && single) {  // the only tile of this point: its whole gradient
        store_row<CP>(a.grad_feat + (size_t)cur_idx * C, gfeat, C);
        a.gsc[cur_idx] = sc;
      }
    }
    // split points: this tile's share by float atomics, staged in the first
    // wavefront's part of the tables (only it holds copies; its reads above
    // are done)
    if (tid < 64)
      add_gauss_shares<CP>(cur && touched && !single, cur_idx, gfeat, sc, ewa ? 4u : 3u, s_ta,
                           a);
    tile_sync<NW>();
  }
}

template <int T, int CP, typename FT, bool FULL>
__global__ __launch_bounds__(T* T) void k_blend_fwd_bilinear(BlendArgs a) {
  if (a.flags[kFlagOverflow]) return;
  blend_fwd_bilinear_tile<T, CP, FT, FULL>(a, block_tile(a));
}
template <int T, int CP, typename FT, bool FULL>
__global__ __launch_bounds__(T* T) void k_blend_fwd_bilinear_batched(const BlendArgs* __restrict__ args,
                                                              const uint2* __restrict__ items) {
  const uint2 vk = items[xcd_pos(blockIdx.x, gridDim.x)];
  const uint32_t v = __builtin_amdgcn_readfirstlane(vk.x);
  if (v == kNoItem) return;  // padding of a view's last quad
  const BlendArgs& a = args[v];  // read-only for the whole kernel: scalar loads
  if (a.flags[kFlagOverflow]) return;
  blend_fwd_bilinear_tile<T, CP, FT, FULL>(a, a.order[__builtin_amdgcn_readfirstlane(vk.y)]);
}

template <int CP, typename FT, bool FULL>
__global__ __launch_bounds__(64) void k_blend_fwd_bilinear8(BlendArgs a) {
  if (a.flags[kFlagOverflow]) return;
  blend_fwd_bilinear8_tile<CP, FT, FULL>(a, block_tile(a));
}
template <int CP, typename FT, bool FULL>
__global__ __launch_bounds__(64) void k_blend_fwd_bilinear8_batched(const BlendArgs* __restrict__ args,
                                                              const uint2* __restrict__ items) {
  const uint2 vk = items[xcd_pos(blockIdx.x, gridDim.x)];
  const uint32_t v = __builtin_amdgcn_readfirstlane(vk.x);
  if (v == kNoItem) return;  // padding of a view's last quad
  const BlendArgs& a = args[v];  // read-only for the whole kernel: scalar loads
  if (a.flags[kFlagOverflow]) return;
  blend_fwd_bilinear8_tile<CP, FT, FULL>(a, a.order[__builtin_amdgcn_readfirstlane(vk.y)]);
}

template <int T, int CP, typename FT, bool FULL>
__global__ __launch_bounds__(T* T) void k_blend_fwd_gauss(BlendArgs a) {
  if (a.flags[kFlagOverflow]) return;
  blend_fwd_gauss_tile<T, CP, FT, FULL>(a, block_tile(a));
}
template <int T, int CP, typename FT, bool FULL>
__global__ __launch_bounds__(T* T) void k_blend_fwd_gauss_batched(const BlendArgs* __restrict__ args,
                                                              const uint2* __restrict__ items) {
  const uint2 vk = items[xcd_pos(blockIdx.x, gridDim.x)];
  const uint32_t v = __builtin_amdgcn_readfirstlane(vk.x);
  if (v == kNoItem) return;  // padding of a view's last quad
  const BlendArgs& a = args[v];  // read-only for the whole kernel: scalar loads
  if (a.flags[kFlagOverflow]) return;
  blend_fwd_gauss_tile<T, CP, FT, FULL>(a, a.order[__builtin_amdgcn_readfirstlane(vk.y)]);
}

template <int T, int CP, typename FT, bool FULL>
__global__ __launch_bounds__(T* T) void k_blend_bwd_bilinear(BlendArgs a) {
  if (a.flags[kFlagOverflow]) return;
  blend_bwd_bilinear_tile<T, CP, FT, FULL>(a, block_tile(a));
}
template <int T, int CP, typename FT, bool FULL>
__global__ __launch_bounds__(T* T) void k_blend_bwd_bilinear_batched(const BlendArgs* __restrict__ args,
                                                              const uint2* __restrict__ items) {
  const uint2 vk = items[xcd_pos(blockIdx.x, gridDim.x)];
  const uint32_t v = __builtin_amdgcn_readfirstlane(vk.x);
  if (v == kNoItem) return;  // padding of a view's last quad
  const BlendArgs& a = args[v];  // read-only for the whole kernel: scalar loads
  if (a.flags[kFlagOverflow]) return;
  blend_bwd_bilinear_tile<T, CP, FT, FULL>(a, a.order[__builtin_amdgcn_readfirstlane(vk.y)]);
}

template <int T, int CP, typename FT, bool FULL>
__global__ __launch_bounds__(T* T) void k_blend_bwd_gauss(BlendArgs a) {
  if (a.flags[kFlagOverflow]) return;
  blend_bwd_gauss_tile<T, CP, FT, FULL>(a, block_tile(a));
}
template <int T, int CP, typename FT, bool FULL>
__global__ __launch_bounds__(T* T) void k_blend_bwd_gauss_batched(const BlendArgs* __restrict__ args,
                                                              const uint2* __restrict__ items) {
  const uint2 vk = items[xcd_pos(blockIdx.x, gridDim.x)];
  const uint32_t v = __builtin_amdgcn_readfirstlane(vk.x);
  if (v == kNoItem) return;  // padding of a view's last quad
  const BlendArgs& a = args[v];  // read-only for the whole kernel: scalar loads
  if (a.flags[kFlagOverflow]) return;
  blend_bwd_gauss_tile<T, CP, FT, FULL>(a, a.order[__builtin_amdgcn_readfirstlane(vk.y)]);
}

template <int CP, typename FT, bool FULL>
__global__ __launch_bounds__(64) void k_blend_bwd_bilinear8(BlendArgs a) {
  if (a.flags[kFlagOverflow]) return;
  blend_bwd_bilinear8_tile<CP, FT, FULL>(a, block_tile(a));
}
template <int CP, typename FT, bool FULL>
__global__ __launch_bounds__(64) void k_blend_bwd_bilinear8_batched(const BlendArgs* __restrict__ args,
                                                              const uint2* __restrict__ items) {
  const uint2 vk = items[xcd_pos(blockIdx.x, gridDim.x)];
  const uint32_t v = __builtin_amdgcn_readfirstlane(vk.x);
  if (v == kNoItem) return;  // padding of a view's last quad
  const BlendArgs& a = args[v];  // read-only for the whole kernel: scalar loads
  if (a.flags[kFlagOverflow]) return;
  blend_bwd_bilinear8_tile<CP, FT, FULL>(a, a.order[__builtin_amdgcn_readfirstlane(vk.y)]);
}

// Zero n floats at p (4-byte aligned): 16-byte non-temporal stores for the
// aligned body (a streaming fill that nothing reads back soon).
__device__ __forceinline__ void zero_range(float* __restrict__ p, size_t n, size_t tid,
                                           size_t stride) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const size_t mis = (size_t)(reinterpret_cast<uintptr_t>(p) & 15u);
  const size_t head = min(n, ((16u - mis) & 15u) / 4u);
  const size_t nv = (n - head) / 4u;
  if (tid < head) p[tid] = 0.f;
  u32x4* v = reinterpret_cast<u32x4*>(p + head);
  const u32x4 z = {0u, 0u, 0u, 0u};
  for (size_t i = tid; i < nv; i += stride) __builtin_nontemporal_store(z, v + i);
  const size_t tail0 = head + nv * 4u;
  if (tid < n - tail0) p[tail0 + tid] = 0.f;
}

// Zero two float ranges in one launch.
__global__ __launch_bounds__(256) void k_zero(float* __restrict__ p0, size_t n0,
                                              float* __restrict__ p1, size_t n1) {
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  zero_range(p0, n0, tid, stride);
  if (p1) zero_range(p1, n1, tid, stride);
}

// grad_opacity, grad_uv and grad_z (if wanted) from the per-point scalar rows.
__global__ __launch_bounds__(256) void k_unpack_scalars(const float4* __restrict__ gsc, int64_t n,
                                                        float* __restrict__ go,
                                                        float2* __restrict__ guv,
                                                        float* __restrict__ gz) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float4 v = gsc[i];
    go[i] = v.x;
    guv[i] = make_float2(v.y, v.z);
    if (gz) gz[i] = v.w;
  }
}

hipError_t launch_zero(float* p0, size_t n0, float* p1, size_t n1, hipStream_t s) {
  if (n0 + n1 == 0) return hipSuccess;
  const size_t g = std::min<size_t>((std::max(n0, n1) / 4 + 255) / 256 + 1, 2048);
  hipLaunchKernelGGL(k_zero, dim3((unsigned)g), dim3(256), 0, s, p0, n0, p1, n1);
  return hipGetLastError();
}

// grad_bg[c] = sum over tiles of the per-tile shares (one block per channel).
__global__ __launch_bounds__(256) void k_bg_reduce(const float* __restrict__ part, int64_t nt, int C,
                                                   float* __restrict__ grad_bg) {
  __shared__ float s[256];
  const int c = blockIdx.x;
  float v = 0.f;
  for (int64_t t = threadIdx.x; t < nt; t += 256) v += part[t * C + c];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad_bg[c] = s[0];
}

template <int T, int CP, typename FT>
hipError_t fwd_launch(const BlendArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)((int64_t)a.opts.ntx * a.opts.nty)), block(T * T);
  const bool full = a.C == CP;
  if (a.opts.splat == INPC_SPLAT_BILINEAR && T == 8) {
    if (full)
      hipLaunchKernelGGL((k_blend_fwd_bilinear8<CP, FT, true>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((k_blend_fwd_bilinear8<CP, FT, false>), grid, block, 0, s, a);
  } else if (a.opts.splat == INPC_SPLAT_BILINEAR) {
    if (full)
      hipLaunchKernelGGL((k_blend_fwd_bilinear<T, CP, FT, true>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((k_blend_fwd_bilinear<T, CP, FT, false>), grid, block, 0, s, a);
  } else {
    if (full)
      hipLaunchKernelGGL((k_blend_fwd_gauss<T, CP, FT, true>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((k_blend_fwd_gauss<T, CP, FT, false>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

// Every gradient starts at zero: points no blended fragment reached keep
// it, single-tile points are overwritten, split points are added to.
hipError_t bwd_pre(const BlendArgs& a, hipStream_t s) {
  if (a.prezeroed) return hipSuccess;
  return launch_zero(a.grad_feat, (size_t)a.n * a.C, reinterpret_cast<float*>(a.gsc),
                     (size_t)a.n * 4, s);
}

// After the tiles: the scalar rows into grad_opacity and grad_uv, and the
// constant background's gradient from the per-tile shares.
hipError_t bwd_post(const BlendArgs& a, hipStream_t s) {
  const int64_t nt = (int64_t)a.opts.ntx * a.opts.nty;
  if (a.n > 0) {
    const int64_t g = std::min<int64_t>((a.n + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(k_unpack_scalars, dim3((unsigned)g), dim3(256), 0, s, a.gsc, a.n,
                       a.grad_opacity, reinterpret_cast<float2*>(a.grad_uv), a.grad_z);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (a.grad_bg && !a.bg_image)
    hipLaunchKernelGGL(k_bg_reduce, dim3((unsigned)a.C), dim3(256), 0, s, a.bg_partial, nt, a.C,
                       a.grad_bg);
  return hipGetLastError();
}

template <int T, int CP, typename FT>
hipError_t bwd_launch(const BlendArgs& a, hipStream_t s) {
  const int64_t nt = (int64_t)a.opts.ntx * a.opts.nty;
  hipError_t e = bwd_pre(a, s);
  if (e != hipSuccess) return e;
  if (a.opts.splat != INPC_SPLAT_BILINEAR && a.C == CP)
    hipLaunchKernelGGL((k_blend_bwd_gauss<T, CP, FT, true>), dim3((unsigned)nt), dim3(T * T), 0, s,
                       a);
  else if (a.opts.splat != INPC_SPLAT_BILINEAR)
    hipLaunchKernelGGL((k_blend_bwd_gauss<T, CP, FT, false>), dim3((unsigned)nt), dim3(T * T), 0,
                       s, a);
  else if (T == 8 && a.C == CP)
    hipLaunchKernelGGL((k_blend_bwd_bilinear8<CP, FT, true>), dim3((unsigned)nt), dim3(64), 0, s,
                       a);
  else if (T == 8)
    hipLaunchKernelGGL((k_blend_bwd_bilinear8<CP, FT, false>), dim3((unsigned)nt), dim3(64), 0, s,
                       a);
  else if (a.C == CP)
    hipLaunchKernelGGL((k_blend_bwd_bilinear<T, CP, FT, true>), dim3((unsigned)nt), dim3(T * T), 0,
                       s, a);
  else
    hipLaunchKernelGGL((k_blend_bwd_bilinear<T, CP, FT, false>), dim3((unsigned)nt), dim3(T * T),
                       0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return bwd_post(a, s);
}

// One launch over every (view, tile) slot of a batch's queue: workgroup b
// takes slot xcd_pos(b), so each quad of neighbouring tiles runs on one XCD
// (its L2) and the hardware dispatches the slots in queue order, longest
// tiles first.
template <typename K>
hipError_t launch_queue(K kernel, int threads, const BatchQueue& q, hipStream_t s) {
  hipLaunchKernelGGL(kernel, dim3(q.total), dim3(threads), 0, s, q.args, q.items);
  return hipGetLastError();
}

template <int T, int CP, typename FT>
hipError_t fwd_launch_q(const BlendArgs& a, const BatchQueue& q, hipStream_t s) {
  const bool full = a.C == CP;
  if (a.opts.splat == INPC_SPLAT_BILINEAR && T == 8)
    return full ? launch_queue(k_blend_fwd_bilinear8_batched<CP, FT, true>, 64, q, s)
                : launch_queue(k_blend_fwd_bilinear8_batched<CP, FT, false>, 64, q, s);
  if (a.opts.splat == INPC_SPLAT_BILINEAR)
    return full ? launch_queue(k_blend_fwd_bilinear_batched<T, CP, FT, true>, T * T, q, s)
                : launch_queue(k_blend_fwd_bilinear_batched<T, CP, FT, false>, T * T, q, s);
  return full ? launch_queue(k_blend_fwd_gauss_batched<T, CP, FT, true>, T * T, q, s)
              : launch_queue(k_blend_fwd_gauss_batched<T, CP, FT, false>, T * T, q, s);
}

template <int T, int CP, typename FT>
hipError_t bwd_launch_q(const BlendArgs& a, const BatchQueue& q, hipStream_t s) {
  const bool full = a.C == CP;
  if (a.opts.splat != INPC_SPLAT_BILINEAR)
    return full ? launch_queue(k_blend_bwd_gauss_batched<T, CP, FT, true>, T * T, q, s)
                : launch_queue(k_blend_bwd_gauss_batched<T, CP, FT, false>, T * T, q, s);
  if (T == 8)
    return full ? launch_queue(k_blend_bwd_bilinear8_batched<CP, FT, true>, 64, q, s)
                : launch_queue(k_blend_bwd_bilinear8_batched<CP, FT, false>, 64, q, s);
  return full ? launch_queue(k_blend_bwd_bilinear_batched<T, CP, FT, true>, T * T, q, s)
              : launch_queue(k_blend_bwd_bilinear_batched<T, CP, FT, false>, T * T, q, s);
}

template <int T, typename FT, bool FWD>
hipError_t dispatch_cp_q(const BlendArgs& a, const BatchQueue& q, hipStream_t s) {
  if (a.C <= 4) return FWD ? fwd_launch_q<T, 4, FT>(a, q, s) : bwd_launch_q<T, 4, FT>(a, q, s);
  if (a.C <= 8) return FWD ? fwd_launch_q<T, 8, FT>(a, q, s) : bwd_launch_q<T, 8, FT>(a, q, s);
  if (a.C <= 16) return FWD ? fwd_launch_q<T, 16, FT>(a, q, s) : bwd_launch_q<T, 16, FT>(a, q, s);
  return FWD ? fwd_launch_q<T, 32, FT>(a, q, s) : bwd_launch_q<T, 32, FT>(a, q, s);
}

template <typename FT, bool FWD>
hipError_t dispatch_t_q(const BlendArgs& a, const BatchQueue& q, hipStream_t s) {
  switch (a.opts.T) {
    case 8: return dispatch_cp_q<8, FT, FWD>(a, q, s);
    case 16: return dispatch_cp_q<16, FT, FWD>(a, q, s);
    default: return hipErrorInvalidValue;
  }
}

template <bool FWD>
hipError_t dispatch_q(const BlendArgs& a, const BatchQueue& q, hipStream_t s) {
  switch (a.dtype) {
    case INPC_F32: return dispatch_t_q<float, FWD>(a, q, s);
    case INPC_F16: return dispatch_t_q<__half, FWD>(a, q, s);
    case INPC_BF16: return dispatch_t_q<__hip_bfloat16, FWD>(a, q, s);
    default: return hipErrorInvalidValue;
  }
}

template <int T, typename FT, bool FWD>
hipError_t dispatch_cp(const BlendArgs& a, hipStream_t s) {
  if (a.C <= 4) return FWD ? fwd_launch<T, 4, FT>(a, s) : bwd_launch<T, 4, FT>(a, s);
  if (a.C <= 8) return FWD ? fwd_launch<T, 8, FT>(a, s) : bwd_launch<T, 8, FT>(a, s);
  if (a.C <= 16) return FWD ? fwd_launch<T, 16, FT>(a, s) : bwd_launch<T, 16, FT>(a, s);
  return FWD ? fwd_launch<T, 32, FT>(a, s) : bwd_launch<T, 32, FT>(a, s);
}

template <typename FT, bool FWD>
hipError_t dispatch_t(const BlendArgs& a, hipStream_t s) {
  switch (a.opts.T) {
    case 8: return dispatch_cp<8, FT, FWD>(a, s);
    case 16: return dispatch_cp<16, FT, FWD>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <bool FWD>
hipError_t dispatch(const BlendArgs& a, hipStream_t s) {
  switch (a.dtype) {
    case INPC_F32: return dispatch_t<float, FWD>(a, s);
    case INPC_F16: return dispatch_t<__half, FWD>(a, s);
    case INPC_BF16: return dispatch_t<__hip_bfloat16, FWD>(a, s);
    default: return hipErrorInvalidValue;
  }
}

// Tile-local position of every copy's 2x2 splat, (x0 - tile x + 1) |
// (y0 - tile y + 1) << 8, for workspaces whose bucket entries could not
// carry it.  One wavefront per tile (longest first), four copies per lane
// and round so that the position gathers of a long list overlap.
__global__ __launch_bounds__(256) void k_lpos(Cam cam, Opts o, const uint32_t* __restrict__ ranges,
                                              const uint32_t* __restrict__ order,
                                              const float4* __restrict__ proj,
                                              const uint32_t* __restrict__ list,
                                              uint16_t* __restrict__ lpos,
                                              const uint32_t* __restrict__ flags) {
  if (flags[kFlagOverflow]) return;
  const int64_t nt = (int64_t)o.ntx * o.nty;
  const uint32_t lane = threadIdx.x & 63u;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < nt;
       i += (int64_t)gridDim.x * 4) {
    const uint32_t t = order ? order[i] : (uint32_t)i;
    const uint32_t s = ranges[t], e = ranges[t + 1];
    if (s == e) continue;
    const int tx0 = (int)(t % (uint32_t)o.ntx) * o.T, ty0 = (int)(t / (uint32_t)o.ntx) * o.T;
    for (uint32_t q0 = s + lane; q0 < e; q0 += 4 * 64) {
      uint32_t idx[4];
      float4 p[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t q = q0 + k * 64;
        idx[k] = list[q < e ? q : e - 1];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) p[k] = proj[idx[k]];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t q = q0 + k * 64;
        if (q < e) {
          const Footprint f = bilinear_footprint(p[k].x, p[k].y, cam.W, cam.H);
          lpos[q] = (uint16_t)((uint32_t)(f.x0 - tx0 + 1) | ((uint32_t)(f.y0 - ty0 + 1) << 8));
        }
      }
    }
  }
}

}  // namespace

hipError_t launch_lpos(const Cam& cam, const Opts& o, const uint32_t* ranges,
                       const uint32_t* order, const float* proj, const uint32_t* list,
                       uint16_t* lpos, const uint32_t* flags, hipStream_t s) {
  const int64_t nt = (int64_t)o.ntx * o.nty;
  if (nt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lpos, dim3((unsigned)std::min<int64_t>((nt + 3) / 4, 16384)), dim3(256), 0, s,
                     cam, o,
                     ranges, order, reinterpret_cast<const float4*>(proj), list, lpos, flags);
  return hipGetLastError();
}

hipError_t launch_blend_forward(const BlendArgs& a, hipStream_t s) {
  if (a.opts.ntx == 0 || a.opts.nty == 0) return hipSuccess;
  return dispatch<true>(a, s);
}

hipError_t launch_blend_backward(const BlendArgs& a, hipStream_t s) {
  if (a.opts.ntx == 0 || a.opts.nty == 0) return hipSuccess;
  return dispatch<false>(a, s);
}

hipError_t launch_blend_backward_pre(const BlendArgs& a, hipStream_t s) { return bwd_pre(a, s); }
hipError_t launch_backward_zero(float* grad_feat, int64_t n, int C, void* scratch, hipStream_t s) {
  return launch_zero(grad_feat, (size_t)n * C, static_cast<float*>(scratch), (size_t)n * 4, s);
}
hipError_t launch_blend_backward_post(const BlendArgs& a, hipStream_t s) { return bwd_post(a, s); }

hipError_t launch_blend_batched(bool forward, const BlendArgs& shape, const BatchQueue& q,
                                hipStream_t s) {
  if (q.total == 0) return hipSuccess;
  return forward ? dispatch_q<true>(shape, q, s) : dispatch_q<false>(shape, q, s);
}

}  // namespace inpc
