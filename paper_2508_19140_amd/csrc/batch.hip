// Many views in one pass (the paper renders several point clouds and views
// per training step and frame, Sec. 3.1; the views of a batch differ in
// point count and resolution).  The device-resident view table
// (inpc_view_t) is turned into per-view blend arguments by one kernel, and
// the (view, tile) items of every view are laid out in one work queue that
// a single blend launch takes in order, one workgroup per slot: item (v, k)
// is view v's k-th tile in its own longest-first order, and the views are
// interleaved quad by quad in proportion to their tile counts (quad (v, k)
// sits at fraction (k + 1/2) / nq_v of the queue), so the long tiles of every
// view start early and no view's tail is left to run alone.
#include "common.h"
#include "internal.h"

namespace inpc {
namespace {

// Per-view blend arguments from the device-resident view table.
__global__ __launch_bounds__(64) void k_batch_args(const inpc_view_t* __restrict__ views, int nv,
                                                   Opts shared, int C, int dtype, int bg_image,
                                                   BlendArgs* __restrict__ out) {
  const int v = blockIdx.x * 64 + threadIdx.x;
  if (v >= nv) return;
  out[v] = make_view_args(views[v], shared, C, dtype, bg_image);
}

// The work queue, in whole quads: view v's tile order is cut into quads of
// four consecutive positions (the order keeps the four side-by-side tiles
// of an aligned quad together), and quad (v, k) goes to quad position sum
// over views u of the number of u's quads ordered before it, where (u, j)
// comes before (v, k) iff (2 j + 1) nq_v < (2 k + 1) nq_u, or the two are
// equal and u < v.  The count is closed form per view, so the positions are
// a bijection computed without a sort.  Slots past a view's last tile hold
// kNoItem.
__global__ __launch_bounds__(256) void k_batch_queue(BatchTiles bt, uint2* __restrict__ items) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= bt.start[bt.nv]) return;
  int v = 0;
  while (bt.start[v + 1] <= g) ++v;
  const int64_t k = g - bt.start[v];
  const int64_t nqv = bt.start[v + 1] - bt.start[v];
  int64_t pos = k;  // own view
  for (int u = 0; u < bt.nv; ++u) {
    if (u == v) continue;
    const int64_t nqu = bt.start[u + 1] - bt.start[u];
    const int64_t num = (2 * k + 1) * nqu - nqv;  // (2 j + 1) nqv < (2 k + 1) nqu  <=>  2 j nqv < num
    int64_t c;
    if (u < v)
      c = num >= 0 ? num / (2 * nqv) + 1 : 0;             // 2 j nqv <= num
    else
      c = num > 0 ? (num + 2 * nqv - 1) / (2 * nqv) : 0;  // 2 j nqv < num
    pos += c < nqu ? c : nqu;
  }
  for (int j = 0; j < 4; ++j) {
    const int64_t t = 4 * k + j;
    items[4 * pos + j] = t < bt.tiles[v] ? make_uint2((uint32_t)v, (uint32_t)t)
                                         : make_uint2(kNoItem, kNoItem);
  }
}

}  // namespace

hipError_t launch_batch_prepare(const inpc_view_t* views_dev, int nv, const Opts& shared, int C,
                                int dtype, int bg_image, const BatchTiles& bt, BlendArgs* args,
                                uint2* items, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_args, dim3((unsigned)((nv + 63) / 64)), dim3(64), 0, s, views_dev,
                     nv, shared, C, dtype, bg_image, args);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t quads = bt.start[bt.nv];
  hipLaunchKernelGGL(k_batch_queue, dim3((unsigned)std::max<int64_t>(1, (quads + 255) / 256)),
                     dim3(256), 0, s, bt, items);
  return hipGetLastError();
}

}  // namespace inpc
