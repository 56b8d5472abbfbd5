// C ABI of the rasterizer: argument checks, workspace layout, launches.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "common.h"
#include "inpc_raster.h"
#include "internal.h"

namespace inpc {
namespace {

thread_local char g_err[512] = "";

inpc_status_t fail(inpc_status_t st, const char* fmt, const char* what) {
  snprintf(g_err, sizeof(g_err), fmt, what);
  return st;
}

inpc_status_t hip_fail(hipError_t e, const char* where) {
  snprintf(g_err, sizeof(g_err), "%s: %s", where, hipGetErrorString(e));
  return INPC_ERR_HIP;
}

bool valid_cam(const inpc_camera_t* c) {
  return c && c->width > 0 && c->height > 0 && c->width < 32767 && c->height < 32767 &&
         isfinite(c->fx) && isfinite(c->fy) && isfinite(c->cx) && isfinite(c->cy);
}

bool valid_opts(const inpc_opts_t* o) {
  return o && (o->tile == 8 || o->tile == 16 || o->tile == 32) && o->bin_points >= 0 &&
         o->bin_points % 1024 == 0 &&
         (o->splat == INPC_SPLAT_BILINEAR || o->splat == INPC_SPLAT_GAUSSIAN ||
          o->splat == INPC_SPLAT_EWA) &&
         o->t_min >= 0.f && o->t_min <= 1.f && (o->bg_per_pixel == 0 || o->bg_per_pixel == 1) &&
         (o->splat == INPC_SPLAT_BILINEAR ||
          (o->dilation >= 0.f && isfinite(o->dilation) && o->cutoff > 0.f &&
           isfinite(o->cutoff) && o->max_radius >= 0.f && isfinite(o->max_radius))) &&
         (o->splat != INPC_SPLAT_EWA || (o->ewa_sigma > 0.f && isfinite(o->ewa_sigma)));
}

int64_t num_tiles(const inpc_camera_t* c, const inpc_opts_t* o) {
  const int64_t ntx = (c->width + o->tile - 1) / o->tile;
  const int64_t nty = (c->height + o->tile - 1) / o->tile;
  return ntx * nty;
}

// Most tiles a single point can touch.
int64_t max_tiles_per_point(const inpc_camera_t* c, const inpc_opts_t* o) {
  if (o->splat == INPC_SPLAT_BILINEAR) return 4;
  const double R = (double)o->cutoff * sqrt((double)o->max_radius * o->max_radius + o->dilation);
  const int64_t span = (int64_t)floor(2.0 * R + 1e-3) + 1;  // pixels per axis
  const int64_t per_axis = (span + o->tile - 1) / o->tile + 1;
  const int64_t ntx = (c->width + o->tile - 1) / o->tile, nty = (c->height + o->tile - 1) / o->tile;
  return std::min(per_axis, ntx) * std::min(per_axis, nty);
}

int64_t copy_capacity(int64_t n, const inpc_camera_t* c, const inpc_opts_t* o) {
  return n * max_tiles_per_point(c, o);
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t flags, tile_count, gsum, gcls, gord, coltot, blk, cursor, seg_w, seg_m, seg_l, seg_x,
      seg_g, seg_x2, seg_b0, seg_b1, bucket, xbucket, total;
};

// Segment-list capacities.  Every non-empty tile starts one segment; an MSD
// split of a segment with more than kSortCapM copies makes at most 256
// sub-segments, and at most cap / (kSortCapM + 1) segments are ever split
// per round (two rounds).
Layout layout(int64_t n, const inpc_camera_t* c, const inpc_opts_t* o) {
  const size_t nt = (size_t)num_tiles(c, o);
  const size_t cap = (size_t)std::max<int64_t>(copy_capacity(n, c, o), 1);
  const size_t big = cap / (kSortCapM + 1) + 1;
  const size_t small_segs = nt + 4 * 256 * big;  // two LDS and two global split rounds
  const size_t big_segs = nt + big;
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  L.flags = take(kFlagSlots * 4);
  L.tile_count = take(nt * 4);
  const size_t groups = (nt + 63) / 64;
  L.gsum = take(groups * 8);
  L.gcls = take(groups * 4 * 4);
  L.gord = take(groups * kOrderClasses * 4);
  L.coltot = take((1 + 4 + kOrderClasses) * 8);
  L.blk = take(nt <= (size_t)kLdsBins ? (size_t)bin_rows(n, o->bin_points) * nt * 4 : 0);
  L.cursor = take(nt * 4);
  L.seg_w = take(small_segs * 8);
  L.seg_m = take(small_segs * 8);
  L.seg_l = take(big_segs * 8);
  L.seg_x = take(big_segs * 8);
  L.seg_g = take(big_segs * 8);
  L.seg_x2 = take(big_segs * 8);
  L.seg_b0 = take(big_segs * 8);
  L.seg_b1 = take(big_segs * 8);
  L.bucket = take(cap * 8);
  L.xbucket = take(cap * 8);
  L.total = off;
  return L;
}

Ws make_ws(void* ws, int64_t n, const inpc_camera_t* c, const inpc_opts_t* o) {
  const Layout L = layout(n, c, o);
  char* b = static_cast<char*>(ws);
  Ws w;
  w.flags = reinterpret_cast<uint32_t*>(b + L.flags);
  w.tile_count = reinterpret_cast<uint32_t*>(b + L.tile_count);
  w.gsum = reinterpret_cast<uint64_t*>(b + L.gsum);
  w.gcls = reinterpret_cast<uint32_t*>(b + L.gcls);
  w.gord = reinterpret_cast<uint32_t*>(b + L.gord);
  w.coltot = reinterpret_cast<uint64_t*>(b + L.coltot);
  w.groups = (num_tiles(c, o) + 63) / 64;
  w.blk = reinterpret_cast<uint32_t*>(b + L.blk);
  w.cursor = reinterpret_cast<uint32_t*>(b + L.cursor);
  w.seg_w = reinterpret_cast<uint2*>(b + L.seg_w);
  w.seg_m = reinterpret_cast<uint2*>(b + L.seg_m);
  w.seg_l = reinterpret_cast<uint2*>(b + L.seg_l);
  w.seg_x = reinterpret_cast<uint2*>(b + L.seg_x);
  w.seg_g = reinterpret_cast<uint2*>(b + L.seg_g);
  w.seg_x2 = reinterpret_cast<uint2*>(b + L.seg_x2);
  w.seg_b0 = reinterpret_cast<uint2*>(b + L.seg_b0);
  w.seg_b1 = reinterpret_cast<uint2*>(b + L.seg_b1);
  w.bucket = reinterpret_cast<uint2*>(b + L.bucket);
  w.xbucket = reinterpret_cast<uint2*>(b + L.xbucket);
  w.cap = (uint32_t)std::min<int64_t>(copy_capacity(n, c, o), 0xffffffffLL);
  w.chunk = bin_chunk(n, o->bin_points);
  w.rows = bin_rows(n, o->bin_points);
  // Pack the tile-local splat corner (codes 0..T per axis) below the point
  // index when both fit one 32-bit word; otherwise inpc_sort computes it in
  // a separate pass.
  w.lbits = w.pb = 0;
  if (o->splat == INPC_SPLAT_BILINEAR) {
    const int pb = o->tile == 8 ? 4 : (o->tile == 16 ? 5 : 6);
    int ibits = 1;
    while (ibits < 32 && ((int64_t)1 << ibits) < n) ++ibits;
    if (ibits + 2 * pb <= 32) {
      w.pb = pb;
      w.lbits = 2 * pb;
    }
  }
  return w;
}

// Backward scratch: a 16-byte (dL/do, dL/du, dL/dv) row per point, then the
// per-tile shares of the background gradient.
size_t scratch_scalar_bytes(int64_t n) { return align_up((size_t)n * 16); }
size_t scratch_bytes(int64_t n, int C, const inpc_camera_t* c, const inpc_opts_t* o) {
  return scratch_scalar_bytes(n) + align_up((size_t)num_tiles(c, o) * C * 4);
}

// Per-pixel forward state (last position, anchor position, anchor
// transmittance) and the per-tile largest last position.
size_t state_bytes(const inpc_camera_t* c, const inpc_opts_t* o) {
  return (size_t)c->width * c->height * 12 + (size_t)num_tiles(c, o) * 4;
}

Cam to_cam(const inpc_camera_t* c) {
  Cam k;
  k.W = c->width;
  k.H = c->height;
  k.fx = c->fx; k.fy = c->fy; k.cx = c->cx; k.cy = c->cy;
  memcpy(k.R, c->R, sizeof(k.R));
  memcpy(k.t, c->t, sizeof(k.t));
  k.z_near = c->z_near;
  return k;
}

Opts to_opts(const inpc_camera_t* c, const inpc_opts_t* o) {
  Opts k;
  k.splat = o->splat;
  k.T = o->tile;
  k.ntx = (c->width + o->tile - 1) / o->tile;
  k.nty = (c->height + o->tile - 1) / o->tile;
  k.t_min = o->t_min;
  k.dilation = o->dilation;
  k.cutoff = o->cutoff;
  k.ewa_sigma = o->splat == INPC_SPLAT_EWA ? o->ewa_sigma : 0.f;
  return k;
}

// Common checks for entry points that take the workspace.
inpc_status_t check_common(const inpc_camera_t* cam, const inpc_opts_t* opts, int64_t n,
                           const void* ws, size_t ws_bytes) {
  if (!valid_cam(cam)) return fail(INPC_ERR_INVALID, "invalid camera%s", "");
  if (!valid_opts(opts)) return fail(INPC_ERR_INVALID, "invalid options%s", "");
  if (n < 0 || n > (int64_t)0x7fffffff) return fail(INPC_ERR_INVALID, "n out of range%s", "");
  if (num_tiles(cam, opts) >= (int64_t)0xffffffffLL)
    return fail(INPC_ERR_INVALID, "tile count does not fit 32 bits%s", "");
  if (copy_capacity(n, cam, opts) > (int64_t)0xffffffffLL)
    return fail(INPC_ERR_INVALID, "copy capacity does not fit 32 bits%s", "");
  if (!ws) return fail(INPC_ERR_INVALID, "null %s", "workspace");
  if (reinterpret_cast<uintptr_t>(ws) % 16)
    return fail(INPC_ERR_INVALID, "%s not 16-byte aligned", "workspace");
  if (ws_bytes < layout(n, cam, opts).total)
    return fail(INPC_ERR_INVALID, "workspace smaller than inpc_workspace_bytes()%s", "");
  return INPC_OK;
}

#define REQUIRE(ptr, name) \
  if (!(ptr)) return fail(INPC_ERR_INVALID, "null %s", name)

// Arrays the kernels read or write as 16-byte (or 8-byte) vectors.
#define REQUIRE_ALIGNED(ptr, name, bytes)                              \
  do {                                                                 \
    REQUIRE(ptr, name);                                                \
    if (reinterpret_cast<uintptr_t>(ptr) % (bytes))                    \
      return fail(INPC_ERR_INVALID, "%s not " #bytes "-byte aligned", name); \
  } while (0)

// Projection records are read as 16-byte vectors.
#define REQUIRE_PROJ(ptr)                                  \
  do {                                                     \
    REQUIRE(ptr, "proj");                                  \
    if (reinterpret_cast<uintptr_t>(ptr) % 16)             \
      return fail(INPC_ERR_INVALID, "%s not 16-byte aligned", "proj"); \
  } while (0)

static inpc_status_t blend_checks(const inpc_camera_t* cam, const inpc_opts_t* opts, int64_t n,
                                  int32_t C, int32_t dtype, const void* ws, size_t ws_bytes) {
  inpc_status_t st = check_common(cam, opts, n, ws, ws_bytes);
  if (st != INPC_OK) return st;
  if (C < 1 || C > 64) return fail(INPC_ERR_INVALID, "channels must be in [1, 64]%s", "");
  if (dtype != INPC_F32 && dtype != INPC_F16 && dtype != INPC_BF16)
    return fail(INPC_ERR_INVALID, "unknown feature dtype%s", "");
  if (C > 32) return fail(INPC_ERR_UNSUPPORTED, "more than 32 channels%s", "");
  if (opts->tile == 32) return fail(INPC_ERR_UNSUPPORTED, "blending with 32x32 tiles%s", "");
  return INPC_OK;
}

// Scratch of inpc_blend_backward_noalloc: a file-scope device array, one
// copy per GPU, held until the process ends.  In host code `scratch` only
// names the symbol; its device address comes from hipGetSymbolAddress,
// once per device with that device current, and is kept per device.
constexpr size_t kStaticScratchBytes = INPC_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

inpc_status_t static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "inpc_blend_backward_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(INPC_ERR_INVALID, "device index out of range%s", "");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                      "inpc_blend_backward_noalloc: hipGetSymbolAddress");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return INPC_OK;
}

static inpc_status_t blend_backward_impl(const char* who, const inpc_camera_t* cam,
                                         const inpc_opts_t* opts, int64_t n,
                                  const float* proj, const void* feat, int32_t C, int32_t dtype,
                                  const float* bg,
                                  const uint32_t* ntiles, const uint32_t* tile_ranges,
                                  const uint32_t* tile_order, const uint32_t* list,
                                  const uint16_t* lpos, const float* t_final, const void* state,
                                  const float* grad_out, const float* grad_t, float* grad_feat,
                                  float* grad_opacity, float* grad_uv, float* grad_z,
                                  float* grad_bg, void* scratch, size_t scratch_size, void* ws,
                                  size_t ws_bytes, void* stream, bool prezeroed) {
  inpc_status_t st = blend_checks(cam, opts, n, C, dtype, ws, ws_bytes);
  if (st != INPC_OK) return st;
  REQUIRE(scratch, "scratch");
  if (scratch_size < scratch_bytes(n, C, cam, opts))
    return fail(INPC_ERR_INVALID, "scratch smaller than inpc_backward_scratch_bytes()%s", "");
  REQUIRE(tile_ranges, "tile_ranges");
  REQUIRE(list, "list");
  if (opts->splat == INPC_SPLAT_BILINEAR) REQUIRE(lpos, "lpos");
  REQUIRE(t_final, "t_final");
  REQUIRE(state, "state");
  REQUIRE(grad_out, "grad_out");
  if (reinterpret_cast<uintptr_t>(scratch) % 16)
    return fail(INPC_ERR_INVALID, "%s not 16-byte aligned", "scratch");
  if (n > 0) {
    REQUIRE_PROJ(proj);
    REQUIRE_ALIGNED(feat, "feat", 16);
    REQUIRE(ntiles, "ntiles");
    REQUIRE_ALIGNED(grad_feat, "grad_feat", 16);
    REQUIRE(grad_opacity, "grad_opacity");
    REQUIRE_ALIGNED(grad_uv, "grad_uv", 8);
    if (opts->splat == INPC_SPLAT_EWA) REQUIRE(grad_z, "grad_z");
  }
  const Ws w = make_ws(ws, n, cam, opts);
  BlendArgs a;
  memset(&a, 0, sizeof(a));
  a.cam = to_cam(cam);
  a.opts = to_opts(cam, opts);
  a.n = n;
  a.proj = proj;
  a.feat = feat;
  a.C = C;
  a.dtype = dtype;
  a.bg = bg;
  a.bg_image = opts->bg_per_pixel;
  a.ranges = tile_ranges;
  a.order = tile_order;
  a.list = list;
  a.lpos = lpos;
  a.t_final = const_cast<float*>(t_final);
  const size_t P = (size_t)cam->width * cam->height;
  a.st_last = static_cast<uint32_t*>(const_cast<void*>(state));
  a.st_anchor = a.st_last + P;
  a.st_tanchor = reinterpret_cast<float*>(a.st_anchor + P);
  a.st_tile = a.st_last + 3 * P;
  a.ntiles = ntiles;
  a.grad_out = grad_out;
  a.grad_t = grad_t;
  a.grad_feat = grad_feat;
  a.grad_opacity = grad_opacity;
  a.grad_uv = grad_uv;
  a.grad_z = grad_z;
  a.grad_bg = grad_bg;
  a.gsc = static_cast<float4*>(scratch);
  a.bg_partial = grad_bg && !opts->bg_per_pixel
                     ? reinterpret_cast<float*>(static_cast<char*>(scratch) +
                                                scratch_scalar_bytes(n))
                     : nullptr;
  a.flags = w.flags;
  a.prezeroed = prezeroed;
  hipError_t e = launch_blend_backward(a, (hipStream_t)stream);
  return e == hipSuccess ? INPC_OK : hip_fail(e, who);
}

}  // namespace
}  // namespace inpc

using namespace inpc;

extern "C" {

size_t inpc_workspace_bytes(int64_t n, const inpc_camera_t* cam, const inpc_opts_t* opts) {
  if (n < 0 || !valid_cam(cam) || !valid_opts(opts)) return 0;
  return layout(n, cam, opts).total;
}

size_t inpc_backward_scratch_bytes(int64_t n, int32_t C, const inpc_camera_t* cam,
                                   const inpc_opts_t* opts) {
  if (n < 0 || C < 1 || C > 64 || !valid_cam(cam) || !valid_opts(opts)) return 0;
  return scratch_bytes(n, C, cam, opts);
}

size_t inpc_state_bytes(const inpc_camera_t* cam, const inpc_opts_t* opts) {
  if (!valid_cam(cam) || !valid_opts(opts)) return 0;
  return state_bytes(cam, opts);
}

int64_t inpc_num_tiles(const inpc_camera_t* cam, const inpc_opts_t* opts) {
  if (!valid_cam(cam) || !valid_opts(opts)) return 0;
  return num_tiles(cam, opts);
}

int64_t inpc_copy_capacity(int64_t n, const inpc_camera_t* cam, const inpc_opts_t* opts) {
  if (n < 0 || !valid_cam(cam) || !valid_opts(opts)) return 0;
  return copy_capacity(n, cam, opts);
}

namespace inpc {
namespace {

// The ring description of inpc_project_ring, checked.
inpc_status_t make_ring(int32_t n_slots, int64_t slot_cap, const int64_t* counts, Ring* r) {
  if (n_slots < 1 || n_slots > kMaxRingSlots)
    return fail(INPC_ERR_INVALID, "n_slots must be in [1, 16]%s", "");
  if (slot_cap < 1 || slot_cap * n_slots > (int64_t)0x7fffffff)
    return fail(INPC_ERR_INVALID, "slot_cap out of range%s", "");
  REQUIRE(counts, "counts");
  memset(r, 0, sizeof(*r));
  r->slots = n_slots;
  r->cap = (uint32_t)slot_cap;
  for (int s = 0; s < n_slots; ++s) {
    if (counts[s] < 0 || counts[s] > slot_cap)
      return fail(INPC_ERR_INVALID, "ring slot count outside [0, slot_cap]%s", "");
    r->count[s] = (uint32_t)counts[s];
  }
  return INPC_OK;
}

inpc_status_t project_impl(const char* who, const inpc_camera_t* cam, const inpc_opts_t* opts,
                           int64_t n, const float* pos, const float* opacity, const float* radius,
                           float* proj, uint32_t* depth_key, uint32_t* ntiles, void* ws,
                           size_t ws_bytes, const Ring& ring, void* stream) {
  inpc_status_t st = check_common(cam, opts, n, ws, ws_bytes);
  if (st != INPC_OK) return st;
  if (n > 0) {
    REQUIRE(pos, "pos");
    REQUIRE(opacity, "opacity");
    REQUIRE_PROJ(proj);
    REQUIRE(depth_key, "depth_key");
    REQUIRE(ntiles, "ntiles");
    if (opts->splat == INPC_SPLAT_GAUSSIAN) REQUIRE(radius, "radius");
  }
  const Ws w = make_ws(ws, n, cam, opts);
  hipError_t e = launch_project(to_cam(cam), to_opts(cam, opts), n, pos, opacity,
                                opts->splat == INPC_SPLAT_GAUSSIAN ? radius : nullptr, proj,
                                depth_key, ntiles, w, ring, (hipStream_t)stream);
  return e == hipSuccess ? INPC_OK : hip_fail(e, who);
}

}  // namespace
}  // namespace inpc

inpc_status_t inpc_project(const inpc_camera_t* cam, const inpc_opts_t* opts, int64_t n,
                           const float* pos, const float* opacity, const float* radius,
                           float* proj, uint32_t* depth_key, uint32_t* ntiles, void* ws,
                           size_t ws_bytes, void* stream) {
  Ring none;
  memset(&none, 0, sizeof(none));
  return project_impl("inpc_project", cam, opts, n, pos, opacity, radius, proj, depth_key,
                      ntiles, ws, ws_bytes, none, stream);
}

inpc_status_t inpc_project_ring(const inpc_camera_t* cam, const inpc_opts_t* opts,
                                int32_t n_slots, int64_t slot_cap, const int64_t* counts,
                                const float* pos, const float* opacity, const float* radius,
                                float* proj, uint32_t* depth_key, uint32_t* ntiles, void* ws,
                                size_t ws_bytes, void* stream) {
  Ring r;
  inpc_status_t st = make_ring(n_slots, slot_cap, counts, &r);
  if (st != INPC_OK) return st;
  return project_impl("inpc_project_ring", cam, opts, (int64_t)n_slots * slot_cap, pos, opacity,
                      radius, proj, depth_key, ntiles, ws, ws_bytes, r, stream);
}

inpc_status_t inpc_bin(const inpc_camera_t* cam, const inpc_opts_t* opts, int64_t n,
                       const float* proj, const uint32_t* depth_key, const uint32_t* ntiles,
                       uint32_t* tile_ranges, uint32_t* tile_order, void* ws, size_t ws_bytes,
                       void* stream) {
  inpc_status_t st = check_common(cam, opts, n, ws, ws_bytes);
  if (st != INPC_OK) return st;
  REQUIRE(tile_ranges, "tile_ranges");
  if (n > 0) {
    REQUIRE_PROJ(proj);
    REQUIRE(depth_key, "depth_key");
    REQUIRE(ntiles, "ntiles");
  }
  const Ws w = make_ws(ws, n, cam, opts);
  hipError_t e = launch_bin(to_cam(cam), to_opts(cam, opts), n, proj, depth_key, ntiles,
                            tile_ranges, tile_order, w, (hipStream_t)stream);
  return e == hipSuccess ? INPC_OK : hip_fail(e, "inpc_bin");
}

inpc_status_t inpc_sort(const inpc_camera_t* cam, const inpc_opts_t* opts, int64_t n,
                        const float* proj, const uint32_t* tile_ranges,
                        const uint32_t* tile_order, uint32_t* list, uint16_t* lpos, void* ws,
                        size_t ws_bytes, void* stream) {
  inpc_status_t st = check_common(cam, opts, n, ws, ws_bytes);
  if (st != INPC_OK) return st;
  REQUIRE(tile_ranges, "tile_ranges");
  REQUIRE(list, "list");
  const bool bilinear = opts->splat == INPC_SPLAT_BILINEAR;
  if (bilinear) {
    REQUIRE(lpos, "lpos");
    if (n > 0) REQUIRE_PROJ(proj);
  }
  const Ws w = make_ws(ws, n, cam, opts);
  hipError_t e = launch_sort(w, list, lpos, num_tiles(cam, opts), (hipStream_t)stream);
  if (e == hipSuccess && bilinear && n > 0 && w.lbits == 0)
    e = launch_lpos(to_cam(cam), to_opts(cam, opts), tile_ranges, tile_order, proj, list, lpos,
                    w.flags, (hipStream_t)stream);
  return e == hipSuccess ? INPC_OK : hip_fail(e, "inpc_sort");
}


inpc_status_t inpc_blend_forward(const inpc_camera_t* cam, const inpc_opts_t* opts, int64_t n,
                                 const float* proj, const void* feat, int32_t C, int32_t dtype,
                                 const float* bg,
                                 const uint32_t* tile_ranges, const uint32_t* tile_order,
                                 const uint32_t* list, const uint16_t* lpos, float* out,
                                 float* t_final, uint32_t* n_contrib, void* state, void* ws,
                                 size_t ws_bytes, void* stream) {
  inpc_status_t st = blend_checks(cam, opts, n, C, dtype, ws, ws_bytes);
  if (st != INPC_OK) return st;
  REQUIRE(tile_ranges, "tile_ranges");
  REQUIRE(list, "list");
  REQUIRE(out, "out");
  REQUIRE(t_final, "t_final");
  REQUIRE(n_contrib, "n_contrib");
  if (opts->splat == INPC_SPLAT_BILINEAR) REQUIRE(lpos, "lpos");
  if (n > 0) {
    REQUIRE_PROJ(proj);
    REQUIRE_ALIGNED(feat, "feat", 16);
  }
  const Ws w = make_ws(ws, n, cam, opts);
  BlendArgs a;
  memset(&a, 0, sizeof(a));
  a.cam = to_cam(cam);
  a.opts = to_opts(cam, opts);
  a.n = n;
  a.proj = proj;
  a.feat = feat;
  a.C = C;
  a.dtype = dtype;
  a.bg = bg;
  a.bg_image = opts->bg_per_pixel;
  a.ranges = tile_ranges;
  a.order = tile_order;
  a.list = list;
  a.lpos = lpos;
  a.out = out;
  a.t_final = t_final;
  a.n_contrib = n_contrib;
  if (state) {
    const size_t P = (size_t)cam->width * cam->height;
    a.st_last = static_cast<uint32_t*>(state);
    a.st_anchor = a.st_last + P;
    a.st_tanchor = reinterpret_cast<float*>(a.st_anchor + P);
    a.st_tile = a.st_last + 3 * P;
  }
  a.flags = w.flags;
  hipError_t e = launch_blend_forward(a, (hipStream_t)stream);
  return e == hipSuccess ? INPC_OK : hip_fail(e, "inpc_blend_forward");
}

inpc_status_t inpc_blend_backward(const inpc_camera_t* cam, const inpc_opts_t* opts, int64_t n,
                                  const float* proj, const void* feat, int32_t C, int32_t dtype,
                                  const float* bg,
                                  const uint32_t* ntiles, const uint32_t* tile_ranges,
                                  const uint32_t* tile_order, const uint32_t* list,
                                  const uint16_t* lpos, const float* t_final, const void* state,
                                  const float* grad_out, const float* grad_t, float* grad_feat,
                                  float* grad_opacity, float* grad_uv, float* grad_z,
                                  float* grad_bg, void* scratch, size_t scratch_size, void* ws,
                                  size_t ws_bytes, void* stream) {
  return blend_backward_impl("inpc_blend_backward", cam, opts, n, proj, feat, C, dtype, bg,
                             ntiles, tile_ranges, tile_order, list, lpos, t_final, state,
                             grad_out, grad_t, grad_feat, grad_opacity, grad_uv, grad_z, grad_bg,
                             scratch, scratch_size, ws, ws_bytes, stream, false);
}

inpc_status_t inpc_backward_zero(int64_t n, int32_t C, float* grad_feat, void* scratch,
                                 size_t scratch_size, void* stream) {
  if (n < 0 || n > (int64_t)0x7fffffff) return fail(INPC_ERR_INVALID, "n out of range%s", "");
  if (C < 1 || C > 32) return fail(INPC_ERR_INVALID, "channels must be in [1, 32]%s", "");
  if (n == 0) return INPC_OK;
  REQUIRE_ALIGNED(grad_feat, "grad_feat", 16);
  REQUIRE_ALIGNED(scratch, "scratch", 16);
  if (scratch_size < scratch_scalar_bytes(n))
    return fail(INPC_ERR_INVALID, "scratch smaller than 16 bytes per point%s", "");
  hipError_t e = launch_backward_zero(grad_feat, n, C, scratch, (hipStream_t)stream);
  return e == hipSuccess ? INPC_OK : hip_fail(e, "inpc_backward_zero");
}

inpc_status_t inpc_blend_backward_prezeroed(
    const inpc_camera_t* cam, const inpc_opts_t* opts, int64_t n, const float* proj,
    const void* feat, int32_t C, int32_t dtype, const float* bg, const uint32_t* ntiles,
    const uint32_t* tile_ranges, const uint32_t* tile_order, const uint32_t* list,
    const uint16_t* lpos, const float* t_final, const void* state, const float* grad_out,
    const float* grad_t, float* grad_feat, float* grad_opacity, float* grad_uv, float* grad_z,
    float* grad_bg, void* scratch, size_t scratch_size, void* ws, size_t ws_bytes, void* stream) {
  return blend_backward_impl("inpc_blend_backward_prezeroed", cam, opts, n, proj, feat, C, dtype,
                             bg, ntiles, tile_ranges, tile_order, list, lpos, t_final, state,
                             grad_out, grad_t, grad_feat, grad_opacity, grad_uv, grad_z, grad_bg,
                             scratch, scratch_size, ws, ws_bytes, stream, true);
}

inpc_status_t inpc_blend_backward_noalloc(
    const inpc_camera_t* cam, const inpc_opts_t* opts, int64_t n, const float* proj,
    const void* feat, int32_t C, int32_t dtype, const float* bg, const uint32_t* ntiles,
    const uint32_t* tile_ranges, const uint32_t* tile_order, const uint32_t* list,
    const uint16_t* lpos, const float* t_final, const void* state, const float* grad_out,
    const float* grad_t, float* grad_feat, float* grad_opacity, float* grad_uv, float* grad_z,
    float* grad_bg, void* ws, size_t ws_bytes, void* stream) {
  if (!valid_cam(cam)) return fail(INPC_ERR_INVALID, "invalid camera%s", "");
  if (!valid_opts(opts)) return fail(INPC_ERR_INVALID, "invalid options%s", "");
  if (n < 0 || n > (int64_t)0x7fffffff) return fail(INPC_ERR_INVALID, "n out of range%s", "");
  if (C < 1 || C > 64) return fail(INPC_ERR_INVALID, "channels must be in [1, 64]%s", "");
  const size_t need = scratch_bytes(n, C, cam, opts);
  if (need > kStaticScratchBytes) {
    snprintf(g_err, sizeof(g_err),
             "inpc_blend_backward_noalloc: needs %zu bytes of scratch (16 per point + 4 C per "
             "tile), more than the static %zu",
             need, kStaticScratchBytes);
    return INPC_ERR_INVALID;
  }
  inpc_status_t st = blend_checks(cam, opts, n, C, dtype, ws, ws_bytes);
  if (st != INPC_OK) return st;
  void* scr = nullptr;
  st = static_scratch(&scr);
  if (st != INPC_OK) return st;
  return blend_backward_impl("inpc_blend_backward_noalloc", cam, opts, n, proj, feat, C, dtype,
                             bg, ntiles, tile_ranges, tile_order, list, lpos, t_final, state,
                             grad_out, grad_t, grad_feat, grad_opacity, grad_uv, grad_z, grad_bg,
                             scr, kStaticScratchBytes, ws, ws_bytes, stream, false);
}

inpc_status_t inpc_project_backward(const inpc_camera_t* cam, int64_t n, const float* pos,
                                    const uint32_t* ntiles, const float* grad_uv,
                                    const float* grad_z, float* grad_pos, void* stream) {
  if (!valid_cam(cam)) return fail(INPC_ERR_INVALID, "invalid camera%s", "");
  if (n < 0 || n > (int64_t)0x7fffffff) return fail(INPC_ERR_INVALID, "n out of range%s", "");
  if (n > 0) {
    REQUIRE(pos, "pos");
    REQUIRE(ntiles, "ntiles");
    REQUIRE(grad_uv, "grad_uv");
    REQUIRE(grad_pos, "grad_pos");
  }
  hipError_t e = launch_project_backward(to_cam(cam), n, pos, ntiles, grad_uv, grad_z, grad_pos,
                                         (hipStream_t)stream);
  return e == hipSuccess ? INPC_OK : hip_fail(e, "inpc_project_backward");
}

inpc_status_t inpc_view_dirs(const inpc_camera_t* cam, float* dirs, void* stream) {
  if (!valid_cam(cam)) return fail(INPC_ERR_INVALID, "invalid camera%s", "");
  REQUIRE(dirs, "dirs");
  hipError_t e = launch_view_dirs(to_cam(cam), dirs, (hipStream_t)stream);
  return e == hipSuccess ? INPC_OK : hip_fail(e, "inpc_view_dirs");
}

static inpc_status_t envmap_checks(const inpc_camera_t* cam, const float* dirs, int32_t Hm,
                                   int32_t Wm, int32_t C) {
  if (!valid_cam(cam)) return fail(INPC_ERR_INVALID, "invalid camera%s", "");
  REQUIRE(dirs, "dirs");
  if (Hm < 1 || Wm < 1 || (int64_t)Hm * Wm > (int64_t)1 << 30)
    return fail(INPC_ERR_INVALID, "environment map size out of range%s", "");
  if (C < 1 || C > 64) return fail(INPC_ERR_INVALID, "channels must be in [1, 64]%s", "");
  return INPC_OK;
}

inpc_status_t inpc_envmap_forward(const inpc_camera_t* cam, const float* dirs, const float* env,
                                  int32_t Hm, int32_t Wm, int32_t C, float* bg, void* stream) {
  inpc_status_t st = envmap_checks(cam, dirs, Hm, Wm, C);
  if (st != INPC_OK) return st;
  REQUIRE(env, "env");
  REQUIRE(bg, "bg");
  hipError_t e = launch_envmap_forward(to_cam(cam), dirs, env, Hm, Wm, C, bg, (hipStream_t)stream);
  return e == hipSuccess ? INPC_OK : hip_fail(e, "inpc_envmap_forward");
}

inpc_status_t inpc_envmap_backward(const inpc_camera_t* cam, const float* dirs,
                                   const float* grad_bg, int32_t Hm, int32_t Wm, int32_t C,
                                   float* grad_env, void* stream) {
  inpc_status_t st = envmap_checks(cam, dirs, Hm, Wm, C);
  if (st != INPC_OK) return st;
  REQUIRE(grad_bg, "grad_bg");
  REQUIRE(grad_env, "grad_env");
  hipError_t e = launch_envmap_backward(to_cam(cam), dirs, grad_bg, Hm, Wm, C, grad_env,
                                        (hipStream_t)stream);
  return e == hipSuccess ? INPC_OK : hip_fail(e, "inpc_envmap_backward");
}

// Side streams of the batched entry point, per device, created on first use
// and kept until the process ends (default priority, non-blocking), with the
// events that fork them from and join them back to the caller's stream.
constexpr int kSideStreams = 8;
struct SideStreams {
  std::mutex mu;  // one batched call issues its work at a time
  hipStream_t st[kSideStreams];
  hipEvent_t fork, join[kSideStreams];
};
std::mutex g_side_mu;
SideStreams* g_side[kMaxDevices];

static inpc_status_t side_streams(SideStreams** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "inpc_rasterize_batched: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(INPC_ERR_INVALID, "device index out of range%s", "");
  std::lock_guard<std::mutex> lock(g_side_mu);
  if (!g_side[dev]) {
    SideStreams* p = new SideStreams();
    for (int k = 0; k < kSideStreams && e == hipSuccess; ++k)
      e = hipStreamCreateWithFlags(&p->st[k], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
    for (int k = 0; k < kSideStreams && e == hipSuccess; ++k)
      e = hipEventCreateWithFlags(&p->join[k], hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "inpc_rasterize_batched: side streams");
    g_side[dev] = p;
  }
  *out = g_side[dev];
  return INPC_OK;
}

// The first ns side streams wait for everything issued to s so far.
static inpc_status_t fork_sides(SideStreams* p, hipStream_t s, int ns) {
  hipError_t e = hipEventRecord(p->fork, s);
  for (int k = 0; k < ns && e == hipSuccess; ++k) e = hipStreamWaitEvent(p->st[k], p->fork, 0);
  return e == hipSuccess ? INPC_OK : hip_fail(e, "inpc_rasterize_batched: fork");
}

// s waits for everything issued to the first ns side streams.
static inpc_status_t join_sides(SideStreams* p, hipStream_t s, int ns) {
  hipError_t e = hipSuccess;
  for (int k = 0; k < ns && e == hipSuccess; ++k) {
    e = hipEventRecord(p->join[k], p->st[k]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, p->join[k], 0);
  }
  return e == hipSuccess ? INPC_OK : hip_fail(e, "inpc_rasterize_batched: join");
}

// Batch workspace: per-view blend arguments, then the queue slots (whole
// quads of four per view).
struct BatchLayout {
  size_t args, items, total;
};
static BatchLayout batch_layout(int nv, int64_t slots) {
  BatchLayout L;
  L.args = 0;
  L.items = align_up((size_t)nv * sizeof(BlendArgs));
  L.total = L.items + align_up((size_t)slots * sizeof(uint2));
  return L;
}

// Queue slots of a batch: 4 ceil(tiles / 4) per view; -1 if a camera is invalid.
static int64_t batch_items(const inpc_view_t* views, int nv, const inpc_opts_t* opts) {
  int64_t total = 0;
  for (int v = 0; v < nv; ++v) {
    if (!valid_cam(&views[v].cam)) return -1;
    total += 4 * ((num_tiles(&views[v].cam, opts) + 3) / 4);
  }
  return total;
}

size_t inpc_batch_workspace_bytes(const inpc_view_t* views_host, int32_t n_views,
                                  const inpc_opts_t* opts) {
  if (!views_host || n_views < 1 || n_views > kMaxBatchViews || !valid_opts(opts)) return 0;
  const int64_t items = batch_items(views_host, n_views, opts);
  if (items < 0 || items > (int64_t)0xffffffffLL) return 0;
  return batch_layout(n_views, items).total;
}

inpc_status_t inpc_rasterize_batched(const inpc_view_t* views_host, const inpc_view_t* views_dev,
                                     int32_t n_views, const inpc_opts_t* opts, int32_t C,
                                     int32_t dtype, int32_t pass, void* batch_ws,
                                     size_t batch_ws_bytes, void* stream) {
  REQUIRE(views_host, "views_host");
  REQUIRE(views_dev, "views_dev");
  REQUIRE_ALIGNED(batch_ws, "batch_ws", 16);
  if (n_views < 1 || n_views > kMaxBatchViews)
    return fail(INPC_ERR_INVALID, "n_views must be in [1, 64]%s", "");
  if (!valid_opts(opts)) return fail(INPC_ERR_INVALID, "invalid options%s", "");
  if (pass != INPC_PASS_FORWARD && pass != INPC_PASS_BACKWARD)
    return fail(INPC_ERR_INVALID, "unknown pass%s", "");
  const bool fwd = pass == INPC_PASS_FORWARD;
  const int64_t items = batch_items(views_host, n_views, opts);
  if (items < 0) return fail(INPC_ERR_INVALID, "invalid camera%s", "");
  if (items > (int64_t)0xffffffffLL) return fail(INPC_ERR_INVALID, "too many tiles%s", "");
  const BatchLayout BL = batch_layout(n_views, items);
  if (batch_ws_bytes < BL.total)
    return fail(INPC_ERR_INVALID, "batch_ws smaller than inpc_batch_workspace_bytes()%s", "");
  const hipStream_t s = (hipStream_t)stream;
  BatchTiles bt;
  bt.nv = n_views;
  bt.start[0] = 0;
  // every view's checks (those of the single-view calls) before any launch
  for (int v = 0; v < n_views; ++v) {
    const inpc_view_t& w = views_host[v];
    bt.tiles[v] = num_tiles(&w.cam, opts);
    bt.start[v + 1] = bt.start[v] + (bt.tiles[v] + 3) / 4;
    inpc_status_t st = blend_checks(&w.cam, opts, w.n, C, dtype, w.ws, w.ws_bytes);
    if (st != INPC_OK) return st;
    const bool bil = opts->splat == INPC_SPLAT_BILINEAR;
    REQUIRE(w.tile_ranges, "tile_ranges");
    REQUIRE(w.tile_order, "tile_order");
    REQUIRE(w.list, "list");
    if (bil) REQUIRE(w.lpos, "lpos");
    if (w.n > 0) {
      REQUIRE(w.pos, "pos");
      REQUIRE(w.opacity, "opacity");
      REQUIRE_PROJ(w.proj);
      REQUIRE(w.depth_key, "depth_key");
      REQUIRE(w.ntiles, "ntiles");
      REQUIRE_ALIGNED(w.feat, "feat", 16);
      if (opts->splat == INPC_SPLAT_GAUSSIAN) REQUIRE(w.radius, "radius");
    }
    if (w.ring_slots != 0) {
      Ring r;
      if (w.ring_slots < 0 || w.n % w.ring_slots != 0)
        return fail(INPC_ERR_INVALID, "a ring view's n must be ring_slots * slot_cap%s", "");
      st = make_ring(w.ring_slots, w.n / w.ring_slots, w.ring_counts, &r);
      if (st != INPC_OK) return st;
    }
    if (fwd) {
      REQUIRE(w.out, "out");
      REQUIRE(w.t_final, "t_final");
      REQUIRE(w.n_contrib, "n_contrib");
    } else {
      REQUIRE(w.state, "state");
      REQUIRE(w.t_final, "t_final");
      REQUIRE(w.grad_out, "grad_out");
      REQUIRE_ALIGNED(w.scratch, "scratch", 16);
      if (w.scratch_bytes < scratch_bytes(w.n, C, &w.cam, opts))
        return fail(INPC_ERR_INVALID, "scratch smaller than inpc_backward_scratch_bytes()%s", "");
      if (w.n > 0) {
        REQUIRE_ALIGNED(w.grad_feat, "grad_feat", 16);
        REQUIRE(w.grad_opacity, "grad_opacity");
        REQUIRE_ALIGNED(w.grad_uv, "grad_uv", 8);
        REQUIRE(w.grad_pos, "grad_pos");
        if (opts->splat == INPC_SPLAT_EWA) REQUIRE(w.grad_z, "grad_z");
      }
    }
  }
  // The views' own steps (lists, the backward's zero fill and its finishing
  // passes) are independent and mostly latency-bound on their own, so they
  // run side by side on the library's side streams, forked from and joined
  // back to `stream` with events (capturable into a graph).
  SideStreams* side = nullptr;
  inpc_status_t st = side_streams(&side);
  if (st != INPC_OK) return st;
  std::lock_guard<std::mutex> lock(side->mu);
  const int ns = std::min(n_views, kSideStreams);
  st = fork_sides(side, s, ns);
  if (st != INPC_OK) return st;
  for (int v = 0; v < n_views; ++v) {
    const inpc_view_t& w = views_host[v];
    void* vs = side->st[v % kSideStreams];
    if (w.ring_slots > 0)
      st = inpc_project_ring(&w.cam, opts, w.ring_slots, w.n / w.ring_slots, w.ring_counts,
                             w.pos, w.opacity, w.radius, w.proj, w.depth_key, w.ntiles, w.ws,
                             w.ws_bytes, vs);
    else
      st = inpc_project(&w.cam, opts, w.n, w.pos, w.opacity, w.radius, w.proj, w.depth_key,
                        w.ntiles, w.ws, w.ws_bytes, vs);
    if (st == INPC_OK)
      st = inpc_bin(&w.cam, opts, w.n, w.proj, w.depth_key, w.ntiles, w.tile_ranges,
                    w.tile_order, w.ws, w.ws_bytes, vs);
    if (st == INPC_OK)
      st = inpc_sort(&w.cam, opts, w.n, w.proj, w.tile_ranges, w.tile_order, w.list, w.lpos,
                     w.ws, w.ws_bytes, vs);
    if (st != INPC_OK) return st;
    if (!fwd) {
      const BlendArgs a = make_view_args(w, to_opts(&w.cam, opts), C, dtype, opts->bg_per_pixel);
      hipError_t e = launch_blend_backward_pre(a, (hipStream_t)vs);
      if (e != hipSuccess) return hip_fail(e, "inpc_rasterize_batched");
    }
  }
  st = join_sides(side, s, ns);
  if (st != INPC_OK) return st;
  char* b = static_cast<char*>(batch_ws);
  BlendArgs* args = reinterpret_cast<BlendArgs*>(b + BL.args);
  uint2* item = reinterpret_cast<uint2*>(b + BL.items);
  const Opts shared = to_opts(&views_host[0].cam, opts);
  hipError_t e = launch_batch_prepare(views_dev, n_views, shared, C, dtype, opts->bg_per_pixel,
                                      bt, args, item, s);
  if (e != hipSuccess) return hip_fail(e, "inpc_rasterize_batched");
  // one blend launch over every (view, tile) slot
  const BlendArgs shape = make_view_args(views_host[0], shared, C, dtype, opts->bg_per_pixel);
  BatchQueue q;
  q.args = args;
  q.items = item;
  q.total = (uint32_t)items;
  e = launch_blend_batched(fwd, shape, q, s);
  if (e != hipSuccess) return hip_fail(e, "inpc_rasterize_batched");
  if (fwd) return INPC_OK;
  st = fork_sides(side, s, ns);
  if (st != INPC_OK) return st;
  for (int v = 0; v < n_views; ++v) {
    const inpc_view_t& w = views_host[v];
    void* vs = side->st[v % kSideStreams];
    const BlendArgs a = make_view_args(w, to_opts(&w.cam, opts), C, dtype, opts->bg_per_pixel);
    e = launch_blend_backward_post(a, (hipStream_t)vs);
    if (e != hipSuccess) return hip_fail(e, "inpc_rasterize_batched");
    st = inpc_project_backward(&w.cam, w.n, w.pos, w.ntiles, w.grad_uv, w.grad_z, w.grad_pos,
                               vs);
    if (st != INPC_OK) return st;
  }
  return join_sides(side, s, ns);
}

inpc_status_t inpc_sh_features(const inpc_camera_t* cam, int64_t n, const float* pos,
                               const float* sh, int32_t C, float* feat, void* stream) {
  if (!valid_cam(cam)) return fail(INPC_ERR_INVALID, "invalid camera%s", "");
  if (n < 0 || n > (int64_t)0x7fffffff) return fail(INPC_ERR_INVALID, "n out of range%s", "");
  if (C < 1 || C > 64) return fail(INPC_ERR_INVALID, "channels must be in [1, 64]%s", "");
  if (n > 0) {
    REQUIRE(pos, "pos");
    REQUIRE(sh, "sh");
    REQUIRE(feat, "feat");
  }
  hipError_t e = launch_sh_forward(to_cam(cam), n, C, pos, sh, feat, (hipStream_t)stream);
  return e == hipSuccess ? INPC_OK : hip_fail(e, "inpc_sh_features");
}

inpc_status_t inpc_sh_features_backward(const inpc_camera_t* cam, int64_t n, const float* pos,
                                        const float* sh, int32_t C, const float* grad_feat,
                                        float* grad_sh, float* grad_pos, void* stream) {
  if (!valid_cam(cam)) return fail(INPC_ERR_INVALID, "invalid camera%s", "");
  if (n < 0 || n > (int64_t)0x7fffffff) return fail(INPC_ERR_INVALID, "n out of range%s", "");
  if (C < 1 || C > 64) return fail(INPC_ERR_INVALID, "channels must be in [1, 64]%s", "");
  if (n > 0) {
    REQUIRE(pos, "pos");
    REQUIRE(sh, "sh");
    REQUIRE(grad_feat, "grad_feat");
    REQUIRE(grad_sh, "grad_sh");
  }
  hipError_t e = launch_sh_backward(to_cam(cam), n, C, pos, sh, grad_feat, grad_sh, grad_pos,
                                    (hipStream_t)stream);
  return e == hipSuccess ? INPC_OK : hip_fail(e, "inpc_sh_features_backward");
}

inpc_status_t inpc_check_sync(void* ws, size_t ws_bytes, void* stream) {
  REQUIRE(ws, "workspace");
  if (ws_bytes < kFlagSlots * 4) return fail(INPC_ERR_INVALID, "workspace too small%s", "");
  uint32_t flag = 0;
  hipError_t e = hipMemcpyAsync(&flag, ws, sizeof(flag), hipMemcpyDeviceToHost, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "inpc_check_sync");
  if (flag) {
    // reported once: the flag is cleared so that the next build runs again
    e = hipMemsetAsync(ws, 0, sizeof(uint32_t), (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "inpc_check_sync");
    snprintf(g_err, sizeof(g_err), "tile copies exceeded the workspace capacity");
    return INPC_ERR_CAPACITY;
  }
  return INPC_OK;
}

const char* inpc_status_string(inpc_status_t s) {
  switch (s) {
    case INPC_OK: return "ok";
    case INPC_ERR_INVALID: return "invalid argument";
    case INPC_ERR_CAPACITY: return "workspace capacity exceeded";
    case INPC_ERR_HIP: return "HIP runtime error";
    case INPC_ERR_UNSUPPORTED: return "unsupported combination";
    default: return "unknown status";
  }
}

const char* inpc_last_error(void) { return g_err; }

}  // extern "C"
