// Many views in one pass (the paper renders several point clouds and views
// per training step and frame, Sec. 3.1; the views of a batch differ in
// point count and resolution).  The device-resident view table
// (inpc_view_t) is turned into per-view blend arguments by one kernel, and
// the (view, tile) items of every view are laid out in one work queue that
// the persistent blend kernels drain: item (v, k) is view v's k-th tile in
// its own longest-first order, and the views are interleaved in proportion
// to their tile counts (item (v, k) sits at fraction (k + 1/2) / nt_v of the
// queue), so the long tiles of every view start early and no view's tail is
// left to run alone.
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

// The work queue: item (v, k) goes to position sum over views u of the
// number of u's items ordered before it, where (u, j) comes before (v, k)
// iff (2 j + 1) nt_v < (2 k + 1) nt_u, or the two are equal and u < v.  The
// count is closed form per view, so the positions are a bijection computed
// without a sort.  Also resets the 8 per-XCD queue counters.
__global__ __launch_bounds__(256) void k_batch_queue(BatchTiles bt, uint2* __restrict__ items,
                                                     uint32_t* __restrict__ counter) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g < 8) counter[g] = 0u;
  if (g >= (int64_t)bt.start[bt.nv]) return;
  int v = 0;
  while ((int64_t)bt.start[v + 1] <= g) ++v;
  const int64_t k = g - bt.start[v];
  const int64_t ntv = bt.start[v + 1] - bt.start[v];
  int64_t pos = k;  // own view
  for (int u = 0; u < bt.nv; ++u) {
    if (u == v) continue;
    const int64_t ntu = bt.start[u + 1] - bt.start[u];
    const int64_t num = (2 * k + 1) * ntu - ntv;  // (2 j + 1) ntv < (2 k + 1) ntu  <=>  2 j ntv < num
    int64_t c;
    if (u < v)
      c = num >= 0 ? num / (2 * ntv) + 1 : 0;        // 2 j ntv <= num
    else
      c = num > 0 ? (num + 2 * ntv - 1) / (2 * ntv) : 0;  // 2 j ntv < num
    pos += c < ntu ? c : ntu;
  }
  items[pos] = make_uint2((uint32_t)v, (uint32_t)k);
}

}  // namespace

hipError_t launch_batch_prepare(const inpc_view_t* views_dev, int nv, const Opts& shared, int C,
                                int dtype, int bg_image, const BatchTiles& bt, BlendArgs* args,
                                uint2* items, uint32_t* counter, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_args, dim3((unsigned)((nv + 63) / 64)), dim3(64), 0, s, views_dev,
                     nv, shared, C, dtype, bg_image, args);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = bt.start[bt.nv];
  hipLaunchKernelGGL(k_batch_queue, dim3((unsigned)std::max<int64_t>(1, (total + 255) / 256)),
                     dim3(256), 0, s, bt, items, counter);
  return hipGetLastError();
}

}  // namespace inpc
