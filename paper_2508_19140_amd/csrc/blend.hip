// Per-tile alpha blending, forward and backward.
//
// One workgroup per tile, one thread per pixel (an 8x8 tile is exactly one
// 64-wide wavefront).  The tile's depth-ordered list is consumed in chunks:
// the chunk's points are staged in LDS, and for bilinear splats each point
// sets its bit in the 64-bit "which points cover me" mask of the (at most
// four) pixels it covers, so a pixel then visits only its own fragments, in
// list order, by walking the set bits.  Gaussians cover most of a tile, so
// there every pixel tests every staged point.  While a chunk is blended, the
// point data of the next chunk is already being fetched into registers, so
// long lists do not pay one memory latency per chunk.  Tiles are processed
// in the order inpc_bin produced (longest lists first).
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
// per-(point, corner) LDS slots; one thread per point then sums its
// corners.  A point that lies in this tile only gets its gradient written
// directly; a point split over several tiles writes this tile's share into
// its own slot of a partial buffer.  Every write also marks the (point,
// slot) as visited; a gather pass then sums the shares of split points and
// writes zeros for points no blended fragment reached.  No floating-point
// atomics are used, so the backward pass is deterministic.
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

__device__ __forceinline__ uint32_t pack_xy(int x0, int y0) {
  return (uint32_t)(x0 + 1) | ((uint32_t)(y0 + 1) << 16);
}
__device__ __forceinline__ int unpack_x(uint32_t p) { return (int)(p & 0xffffu) - 1; }
__device__ __forceinline__ int unpack_y(uint32_t p) { return (int)(p >> 16) - 1; }

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

  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int k = 0; k < WORDS; ++k) w[k] = 0u;
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

// Register prefetch of one list entry's point data.  `i` must be a valid
// point index even when `v` is false (the loads are not predicated).
template <int CP, typename FT, bool FULL>
struct Prefetch {
  bool valid;
  uint32_t idx;
  float2 uv;
  float o;
  RowRegs<CP, FT, FULL> f;

  __device__ __forceinline__ void fetch(const BlendArgs& a, bool v, uint32_t i) {
    valid = v;
    idx = i;
    uv = reinterpret_cast<const float2*>(a.uv)[i];
    o = a.opacity[i];
    f.load(reinterpret_cast<const FT*>(a.feat), i, a.C);
  }
};

// List entry at position q, clamped to the tile's last entry (end > start,
// q >= start), so that prefetches never need a branch.
__device__ __forceinline__ uint32_t list_at(const uint32_t* __restrict__ list, uint32_t q,
                                            uint32_t end) {
  return list[q < end ? q : end - 1];
}

// ---------------------------------------------------------------------------
// Forward, bilinear splats
// ---------------------------------------------------------------------------
template <int T, int CP, typename FT, bool FULL>
__global__ __launch_bounds__(T* T) void k_blend_fwd_bilinear(BlendArgs a) {
  using G = TileGeom<T>;
  constexpr int NW = G::NW;
  __shared__ float4 s_geo[G::CHUNK];
  __shared__ __align__(16) float s_feat[G::CHUNK * fpad(CP)];
  __shared__ unsigned long long s_mask[G::NTH * G::MW];
  __shared__ uint32_t s_ml[NW];
  if (a.flags[kFlagOverflow]) return;

  const int tid = threadIdx.x;
  const uint32_t tile = a.order ? a.order[blockIdx.x] : blockIdx.x;
  const int tx = (int)(tile % (uint32_t)a.opts.ntx), ty = (int)(tile / (uint32_t)a.opts.ntx);
  const int lx = tid % T, ly = tid / T;
  const int px = tx * T + lx, py = ty * T + ly;
  const bool inside = px < a.cam.W && py < a.cam.H;
  const uint32_t start = a.ranges[tile], end = a.ranges[tile + 1];
  const float t_min = a.opts.t_min;
  const bool stager = tid < G::CHUNK;

  float F[CP];
#pragma unroll
  for (int c = 0; c < CP; ++c) F[c] = 0.f;
  float Tr = 1.f, t_anchor = 1.f;
  uint32_t cnt = 0, last = 0, anchor = 0;
  bool done = !inside;

  // chunk 0's data and chunk 1's list entry are fetched before the loop
  Prefetch<CP, FT, FULL> pf;
  pf.valid = false;
  bool nv = false;
  uint32_t nidx = 0u;
  if (end > start) {
    pf.fetch(a, stager && start + tid < end, list_at(a.list, start + tid, end));
    nv = stager && start + G::CHUNK + tid < end;
    nidx = list_at(a.list, start + G::CHUNK + tid, end);
  }

  for (uint32_t base = start; base < end; base += G::CHUNK) {
    if (!tile_any<NW>(!done)) break;
    // stage the prefetched copy of this chunk
    int x0 = 0, y0 = 0;
    const bool cur = pf.valid;
    if (cur) {
      const Footprint f = bilinear_footprint(pf.uv.x, pf.uv.y, a.cam.W, a.cam.H);
      x0 = f.x0 - tx * T;
      y0 = f.y0 - ty * T;
      s_geo[tid] = make_float4(f.a, f.b, pf.o, __uint_as_float(pack_xy(f.x0, f.y0)));
      pf.f.store_f32(s_feat + tid * fpad(CP));
    }
#pragma unroll
    for (int w = 0; w < G::MW; ++w) s_mask[tid * G::MW + w] = 0ull;
    tile_sync<NW>();
    if (cur) {
      const unsigned long long bit = 1ull << (tid & 63);
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          const int qx = x0 + dx, qy = y0 + dy;
          if (qx >= 0 && qx < T && qy >= 0 && qy < T)
            atomicOr(&s_mask[(qy * T + qx) * G::MW + (tid >> 6)], bit);
        }
    }
    // fetch the next chunk while this one is blended
    pf.fetch(a, nv, nidx);
    nv = stager && base + 2 * G::CHUNK + tid < end;
    nidx = list_at(a.list, base + 2 * G::CHUNK + tid, end);
    tile_sync<NW>();
    if (!done) {
      for (int w = 0; w < G::MW && !done; ++w) {
        unsigned long long m = s_mask[tid * G::MW + w];
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
          const float4* fr = reinterpret_cast<const float4*>(s_feat + kk * fpad(CP));
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
    if (c < a.C) a.out[c * P + p] = a.bg ? fmaf(Tr, a.bg[c], F[c]) : F[c];
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
template <int T, int CP, typename FT, bool FULL>
__global__ __launch_bounds__(T* T) void k_blend_fwd_gauss(BlendArgs a) {
  using G = TileGeom<T>;
  constexpr int NW = G::NW;
  __shared__ float4 s_g0[G::CHUNK];  // u, v, o, s2
  __shared__ float4 s_g1[G::CHUNK];  // thr, packed (px0, py0), packed (px1, py1), -
  __shared__ __align__(16) float s_feat[G::CHUNK * fpad(CP)];
  if (a.flags[kFlagOverflow]) return;

  const int tid = threadIdx.x;
  const uint32_t tile = a.order ? a.order[blockIdx.x] : blockIdx.x;
  const int tx = (int)(tile % (uint32_t)a.opts.ntx), ty = (int)(tile / (uint32_t)a.opts.ntx);
  const int px = tx * T + tid % T, py = ty * T + tid / T;
  const bool inside = px < a.cam.W && py < a.cam.H;
  const uint32_t start = a.ranges[tile], end = a.ranges[tile + 1];
  const float t_min = a.opts.t_min;
  const float pxc = fadd((float)px, 0.5f), pyc = fadd((float)py, 0.5f);
  const bool stager = tid < G::CHUNK;

  float F[CP];
#pragma unroll
  for (int c = 0; c < CP; ++c) F[c] = 0.f;
  float Tr = 1.f;
  uint32_t cnt = 0;
  bool done = !inside;

  Prefetch<CP, FT, FULL> pf;
  pf.valid = false;
  float prad = 0.f;
  bool nv = false;
  uint32_t nidx = 0u;
  if (end > start) {
    pf.fetch(a, stager && start + tid < end, list_at(a.list, start + tid, end));
    prad = a.radius[pf.idx];
    nv = stager && start + G::CHUNK + tid < end;
    nidx = list_at(a.list, start + G::CHUNK + tid, end);
  }

  for (uint32_t base = start; base < end; base += G::CHUNK) {
    if (!tile_any<NW>(!done)) break;
    const uint32_t nh = min((uint32_t)G::CHUNK, end - base);
    if (pf.valid) {
      const Footprint f = gaussian_footprint(pf.uv.x, pf.uv.y, prad, a.cam.W, a.cam.H,
                                             a.opts.dilation, a.opts.cutoff);
      s_g0[tid] = make_float4(pf.uv.x, pf.uv.y, pf.o, f.s2);
      s_g1[tid] = make_float4(f.thr, __uint_as_float(pack_xy(f.px0, f.py0)),
                              __uint_as_float(pack_xy(f.px1, f.py1)), 0.f);
      pf.f.store_f32(s_feat + tid * fpad(CP));
    }
    pf.fetch(a, nv, nidx);
    prad = a.radius[nidx];
    nv = stager && base + 2 * G::CHUNK + tid < end;
    nidx = list_at(a.list, base + 2 * G::CHUNK + tid, end);
    tile_sync<NW>();
    if (!done) {
      for (uint32_t kk = 0; kk < nh; ++kk) {
        const float4 g1 = s_g1[kk];
        const uint32_t lo = __float_as_uint(g1.y), hi = __float_as_uint(g1.z);
        if (px < unpack_x(lo) || px > unpack_x(hi) || py < unpack_y(lo) || py > unpack_y(hi))
          continue;
        const float4 g0 = s_g0[kk];
        const float dx = fsub(pxc, g0.x), dy = fsub(pyc, g0.y);
        const float d2 = fadd(fmul(dx, dx), fmul(dy, dy));
        if (!(d2 <= g1.x)) continue;
        if (Tr < t_min) {
          done = true;
          break;
        }
        const float al = g0.z * expf(-0.5f * d2 / g0.w);
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
        Tr = fmul(Tr, fsub(1.f, al));
        ++cnt;
      }
    }
    tile_sync<NW>();
  }
  if (!inside) return;
  const int64_t P = (int64_t)a.cam.W * a.cam.H;
  const int64_t p = (int64_t)py * a.cam.W + px;
#pragma unroll
  for (int c = 0; c < CP; ++c)
    if (c < a.C) a.out[c * P + p] = a.bg ? fmaf(Tr, a.bg[c], F[c]) : F[c];
  a.t_final[p] = Tr;
  a.n_contrib[p] = cnt;
}

// ---------------------------------------------------------------------------
// Backward, bilinear splats
// ---------------------------------------------------------------------------
template <int T, int CP, typename FT, bool FULL>
__global__ __launch_bounds__(T* T) void k_blend_bwd_bilinear(BlendArgs a) {
  using G = TileGeom<T>;
  constexpr int NW = G::NW;
  __shared__ float4 s_geo[G::CHUNK];
  __shared__ __align__(16) float s_feat[G::CHUNK * fpad(CP)];
  __shared__ unsigned long long s_mask[G::NTH * G::MW];
  __shared__ float2 s_acc[G::CHUNK * 4];                  // per (point, corner): (T alpha, dL/dalpha)
  __shared__ __align__(16) float s_G[G::NTH * fpad(CP)];  // dL/dF of every pixel of the tile
  __shared__ float s_red[NW][CP];
  if (a.flags[kFlagOverflow]) return;

  const int tid = threadIdx.x;
  const uint32_t tile = a.order ? a.order[blockIdx.x] : blockIdx.x;
  const int tx = (int)(tile % (uint32_t)a.opts.ntx), ty = (int)(tile / (uint32_t)a.opts.ntx);
  const int lx = tid % T, ly = tid / T;
  const int px = tx * T + lx, py = ty * T + ly;
  const bool inside = px < a.cam.W && py < a.cam.H;
  const uint32_t start = a.ranges[tile], end = a.ranges[tile + 1];
  const int64_t P = (int64_t)a.cam.W * a.cam.H;
  const int64_t p = (int64_t)py * a.cam.W + px;
  const int C = a.C;
  const bool stager = tid < G::CHUNK;

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
      for (int c = 0; c < C; ++c) gB = fmaf(Gv[c], a.bg[c], gB);
  }
  {
    float4* d4 = reinterpret_cast<float4*>(s_G + tid * fpad(CP));
#pragma unroll
    for (int q = 0; q < CP / 4; ++q) d4[q] = make_float4(Gv[4 * q], Gv[4 * q + 1], Gv[4 * q + 2], Gv[4 * q + 3]);
  }

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
  const uint32_t maxlast = a.st_tile[tile];
  const int nchunks = (int)((maxlast + G::CHUNK - 1) / G::CHUNK);

  Prefetch<CP, FT, FULL> pf;
  pf.valid = false;
  uint32_t pnt = 0;
  if (nchunks > 0) {
    const uint32_t q = start + (uint32_t)(nchunks - 1) * G::CHUNK + tid;
    pf.fetch(a, stager && q < end, list_at(a.list, q, end));
    pnt = a.ntiles[pf.idx];
  }
  bool nv = stager && nchunks >= 2;
  uint32_t nidx = 0u;
  if (nchunks >= 2) nidx = list_at(a.list, start + (uint32_t)(nchunks - 2) * G::CHUNK + tid, end);
  tile_sync<NW>();

  float Pi = 1.f, Tcur = 0.f;
  for (int ci = nchunks - 1; ci >= 0; --ci) {
    const uint32_t rb = (uint32_t)ci * G::CHUNK;  // relative base of the chunk
    // stage this chunk's copy from the prefetch registers
    const bool cur = pf.valid;
    const uint32_t cur_idx = pf.idx, cur_nt = pnt;
    float ca = 0.f, cb = 0.f, co = 0.f;
    int X0 = 0, Y0 = 0;
    if (cur) {
      const Footprint f = bilinear_footprint(pf.uv.x, pf.uv.y, a.cam.W, a.cam.H);
      ca = f.a; cb = f.b; co = pf.o; X0 = f.x0; Y0 = f.y0;
      s_geo[tid] = make_float4(f.a, f.b, pf.o, __uint_as_float(pack_xy(f.x0, f.y0)));
      pf.f.store_f32(s_feat + tid * fpad(CP));
#pragma unroll
      for (int k = 0; k < 4; ++k) s_acc[tid * 4 + k] = make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int w = 0; w < G::MW; ++w) s_mask[tid * G::MW + w] = 0ull;
    tile_sync<NW>();
    if (cur) {
      const int x0 = X0 - tx * T, y0 = Y0 - ty * T;
      const unsigned long long bit = 1ull << (tid & 63);
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          const int qx = x0 + dx, qy = y0 + dy;
          if (qx >= 0 && qx < T && qy >= 0 && qy < T)
            atomicOr(&s_mask[(qy * T + qx) * G::MW + (tid >> 6)], bit);
        }
    }
    // fetch the previous chunk while this one is processed (point 0 stands
    // in when there is none; its data is fetched and ignored)
    pf.fetch(a, nv, nidx);
    pnt = a.ntiles[nidx];
    nv = stager && ci >= 2;
    if (ci >= 2) nidx = list_at(a.list, start + (uint32_t)(ci - 2) * G::CHUNK + tid, end);
    tile_sync<NW>();
    if (last > rb) {
      for (int w = G::MW - 1; w >= 0; --w) {
        unsigned long long m = s_mask[tid * G::MW + w];
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
          s_acc[kk * 4 + dy * 2 + dx] = make_float2(Tk * al, da);
          gB = fmaf(al, gf, om * gB);
          Pi = Pi * om;
          Tcur = Tk;
        }
      }
    }
    tile_sync<NW>();
    if (cur && cur_nt > 0) {
      float gfeat[CP];
#pragma unroll
      for (int c = 0; c < CP; ++c) gfeat[c] = 0.f;
      float go = 0.f, gu = 0.f, gv = 0.f;
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
      uint8_t* vis = reinterpret_cast<uint8_t*>(a.visited);
      if (cur_nt == 1) {
        store_row<CP>(a.grad_feat + (size_t)cur_idx * C, gfeat, C);
        a.grad_opacity[cur_idx] = go;
        reinterpret_cast<float2*>(a.grad_uv)[cur_idx] = make_float2(gu, gv);
        vis[(size_t)cur_idx * 4] = 1;
      } else {
        // this tile's slot among the (at most 2 x 2) tiles of the point
        const int tx0 = max(X0, 0) >> G::SH, ty0 = max(Y0, 0) >> G::SH;
        const int slot = (tx - tx0) + 2 * (ty - ty0);
        float* dst = a.partial + ((size_t)cur_idx * 4 + slot) * a.pstride;
        float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
        for (int q = 0; q < CP / 4; ++q)
          d4[q] = make_float4(gfeat[4 * q], gfeat[4 * q + 1], gfeat[4 * q + 2], gfeat[4 * q + 3]);
        dst[C] = go;
        dst[C + 1] = gu;
        dst[C + 2] = gv;
        vis[(size_t)cur_idx * 4 + slot] = 1;
      }
    }
    tile_sync<NW>();
  }
}

// Gradients the tiles did not write directly: sums of the per-tile shares
// of points split over several tiles, zeros for culled points and for
// points no blended fragment reached.
template <int CP>
__global__ __launch_bounds__(256) void k_grad_gather(BlendArgs a) {
  const int C = a.C;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t nt = a.ntiles[i];
    const uint32_t v = a.visited[i];
    if (nt == 1 && v != 0) continue;  // written by its tile
    float gfeat[CP];
#pragma unroll
    for (int c = 0; c < CP; ++c) gfeat[c] = 0.f;
    float go = 0.f, gu = 0.f, gv = 0.f;
    if (nt > 1) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (!((v >> (8 * k)) & 0xffu)) continue;
        const float* src = a.partial + ((size_t)i * 4 + k) * a.pstride;
        const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
        for (int q = 0; q < CP / 4; ++q) {
          const float4 x = s4[q];
          gfeat[4 * q] += x.x;
          gfeat[4 * q + 1] += x.y;
          gfeat[4 * q + 2] += x.z;
          gfeat[4 * q + 3] += x.w;
        }
        go += src[C];
        gu += src[C + 1];
        gv += src[C + 2];
      }
    }
    store_row<CP>(a.grad_feat + (size_t)i * C, gfeat, C);
    a.grad_opacity[i] = go;
    reinterpret_cast<float2*>(a.grad_uv)[i] = make_float2(gu, gv);
  }
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
  if (a.opts.splat == INPC_SPLAT_BILINEAR) {
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

template <int T, int CP, typename FT>
hipError_t bwd_launch(const BlendArgs& a, hipStream_t s) {
  const int64_t nt = (int64_t)a.opts.ntx * a.opts.nty;
  hipError_t e = launch_clear(a.visited, (size_t)a.n, s);
  if (e != hipSuccess) return e;
  if (a.C == CP)
    hipLaunchKernelGGL((k_blend_bwd_bilinear<T, CP, FT, true>), dim3((unsigned)nt), dim3(T * T), 0,
                       s, a);
  else
    hipLaunchKernelGGL((k_blend_bwd_bilinear<T, CP, FT, false>), dim3((unsigned)nt), dim3(T * T),
                       0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.n > 0) {
    const int64_t g = std::min<int64_t>((a.n + 255) / 256, 1 << 16);
    hipLaunchKernelGGL((k_grad_gather<CP>), dim3((unsigned)g), dim3(256), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (a.grad_bg)
    hipLaunchKernelGGL(k_bg_reduce, dim3((unsigned)a.C), dim3(256), 0, s, a.bg_partial, nt, a.C,
                       a.grad_bg);
  return hipGetLastError();
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

}  // namespace

hipError_t launch_blend_forward(const BlendArgs& a, hipStream_t s) {
  if (a.opts.ntx == 0 || a.opts.nty == 0) return hipSuccess;
  return dispatch<true>(a, s);
}

hipError_t launch_blend_backward(const BlendArgs& a, hipStream_t s) {
  if (a.opts.ntx == 0 || a.opts.nty == 0) return hipSuccess;
  return dispatch<false>(a, s);
}

}  // namespace inpc
