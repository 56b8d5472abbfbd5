// Background from a spherical environment map (paper, Sec. 3.2 "Faster
// Background Model Evaluation"): the background MLP is distilled into an
// equirectangular map F_bg [Hm][Wm][C] that is sampled with bilinear
// interpolation along every pixel's viewing direction, and the local
// (camera-space) directions, which depend only on the intrinsics, are
// computed once and cached by the caller.  The sampled image is the
// per-pixel background the blend composites behind the points
// (F += T_final f_bg(pixel)); its gradient dL/df_bg(pixel) = T_final G comes
// from the blend backward and is scattered back onto the map here.
//
// Mapping (the paper does not print one): world direction w = R^T d (the
// camera maps world to camera space as X = R p + t, OpenCV axes, +y down);
// longitude phi = atan2(w_x, w_z), polar angle theta = acos(-w_y) (0 looks
// straight up); map column coordinate s = (phi / (2 pi) + 1/2) Wm, row
// coordinate t = (theta / pi) Hm, texel (i, j) centred at (i + 1/2, j + 1/2);
// bilinear weights between the four surrounding texel centres, wrapping
// around in longitude and clamping at the poles.
#include "common.h"
#include "internal.h"

namespace inpc {
namespace {

constexpr int kBgBlock = 256;

__global__ __launch_bounds__(kBgBlock) void k_view_dirs(Cam c, float* __restrict__ dirs) {
  const int64_t P = (int64_t)c.W * c.H;
  for (int64_t p = (int64_t)blockIdx.x * kBgBlock + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * kBgBlock) {
    const int x = (int)(p % c.W), y = (int)(p / c.W);
    const float dx = ((float)x + 0.5f - c.cx) / c.fx;
    const float dy = ((float)y + 0.5f - c.cy) / c.fy;
    const float inv = 1.f / sqrtf(dx * dx + dy * dy + 1.f);
    dirs[3 * p] = dx * inv;
    dirs[3 * p + 1] = dy * inv;
    dirs[3 * p + 2] = inv;
  }
}

// Texel footprint of one pixel's direction: the four texels and weights.
struct Tap {
  int64_t t00, t10, t01, t11;  // texel indices (row-major [Hm][Wm])
  float w00, w10, w01, w11;
};

__device__ __forceinline__ Tap env_tap(const Cam& c, const float* __restrict__ dirs, int64_t p,
                                       int Hm, int Wm) {
  const float lx = dirs[3 * p], ly = dirs[3 * p + 1], lz = dirs[3 * p + 2];
  // w = R^T d
  const float wx = c.R[0] * lx + c.R[3] * ly + c.R[6] * lz;
  const float wy = c.R[1] * lx + c.R[4] * ly + c.R[7] * lz;
  const float wz = c.R[2] * lx + c.R[5] * ly + c.R[8] * lz;
  const float kInv2Pi = 0.15915494309189535f, kInvPi = 0.3183098861837907f;
  const float phi = atan2f(wx, wz);
  const float n = sqrtf(wx * wx + wy * wy + wz * wz);
  const float ct = fminf(fmaxf(-wy / n, -1.f), 1.f);
  const float theta = acosf(ct);
  const float s = (phi * kInv2Pi + 0.5f) * (float)Wm - 0.5f;
  const float t = theta * kInvPi * (float)Hm - 0.5f;
  const float fs = floorf(s), ft = floorf(t);
  const float a = s - fs, b = t - ft;
  int x0 = (int)fs, y0 = (int)ft;
  int x1 = x0 + 1, y1 = y0 + 1;
  x0 = ((x0 % Wm) + Wm) % Wm;
  x1 = ((x1 % Wm) + Wm) % Wm;
  y0 = min(max(y0, 0), Hm - 1);
  y1 = min(max(y1, 0), Hm - 1);
  Tap k;
  k.t00 = (int64_t)y0 * Wm + x0;
  k.t10 = (int64_t)y0 * Wm + x1;
  k.t01 = (int64_t)y1 * Wm + x0;
  k.t11 = (int64_t)y1 * Wm + x1;
  k.w00 = (1.f - a) * (1.f - b);
  k.w10 = a * (1.f - b);
  k.w01 = (1.f - a) * b;
  k.w11 = a * b;
  return k;
}

__global__ __launch_bounds__(kBgBlock) void k_envmap_fwd(Cam c, const float* __restrict__ dirs,
                                                         const float* __restrict__ env, int Hm,
                                                         int Wm, int C, float* __restrict__ bg) {
  const int64_t P = (int64_t)c.W * c.H;
  for (int64_t p = (int64_t)blockIdx.x * kBgBlock + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * kBgBlock) {
    const Tap k = env_tap(c, dirs, p, Hm, Wm);
    const float* e00 = env + k.t00 * C;
    const float* e10 = env + k.t10 * C;
    const float* e01 = env + k.t01 * C;
    const float* e11 = env + k.t11 * C;
    for (int ch = 0; ch < C; ++ch)
      bg[ch * P + p] = k.w00 * e00[ch] + k.w10 * e10[ch] + k.w01 * e01[ch] + k.w11 * e11[ch];
  }
}

__global__ __launch_bounds__(kBgBlock) void k_envmap_bwd(Cam c, const float* __restrict__ dirs,
                                                         const float* __restrict__ grad_bg,
                                                         int Hm, int Wm, int C,
                                                         float* __restrict__ grad_env) {
  const int64_t P = (int64_t)c.W * c.H;
  for (int64_t p = (int64_t)blockIdx.x * kBgBlock + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * kBgBlock) {
    const Tap k = env_tap(c, dirs, p, Hm, Wm);
    for (int ch = 0; ch < C; ++ch) {
      const float g = grad_bg[ch * P + p];
      if (g == 0.f) continue;
      atomicAdd(grad_env + k.t00 * C + ch, k.w00 * g);
      atomicAdd(grad_env + k.t10 * C + ch, k.w10 * g);
      atomicAdd(grad_env + k.t01 * C + ch, k.w01 * g);
      atomicAdd(grad_env + k.t11 * C + ch, k.w11 * g);
    }
  }
}

__global__ __launch_bounds__(kBgBlock) void k_fill_zero(float* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBgBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBgBlock)
    p[i] = 0.f;
}

unsigned grid_of(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kBgBlock - 1) / kBgBlock, 8192));
}

}  // namespace

hipError_t launch_view_dirs(const Cam& c, float* dirs, hipStream_t s) {
  const int64_t P = (int64_t)c.W * c.H;
  hipLaunchKernelGGL(k_view_dirs, dim3(grid_of(P)), dim3(kBgBlock), 0, s, c, dirs);
  return hipGetLastError();
}

hipError_t launch_envmap_forward(const Cam& c, const float* dirs, const float* env, int Hm, int Wm,
                                 int C, float* bg, hipStream_t s) {
  const int64_t P = (int64_t)c.W * c.H;
  hipLaunchKernelGGL(k_envmap_fwd, dim3(grid_of(P)), dim3(kBgBlock), 0, s, c, dirs, env, Hm, Wm,
                     C, bg);
  return hipGetLastError();
}

hipError_t launch_envmap_backward(const Cam& c, const float* dirs, const float* grad_bg, int Hm,
                                  int Wm, int C, float* grad_env, hipStream_t s) {
  const int64_t P = (int64_t)c.W * c.H, ne = (int64_t)Hm * Wm * C;
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_of(ne)), dim3(kBgBlock), 0, s, grad_env, ne);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_envmap_bwd, dim3(grid_of(P)), dim3(kBgBlock), 0, s, c, dirs, grad_bg, Hm,
                     Wm, C, grad_env);
  return hipGetLastError();
}

}  // namespace inpc
