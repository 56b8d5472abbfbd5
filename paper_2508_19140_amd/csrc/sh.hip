// View-dependent point features from spherical harmonics (paper, Sec. 2
// "Implicit Point Cloud": the appearance field gives every point SH
// coefficients up to degree two per feature channel, f_hat in R^{C x 9},
// evaluated at the view direction to give the C features the rasterizer
// blends).  The view direction is the unit vector from the camera centre
// c = -R^T t to the point; the basis is the real orthonormal SH of degrees
// 0-2 (graphics ordering, Condon-Shortley phase): with d = (x, y, z),
//   Y0 = k0, Y1 = -k1 y, Y2 = k1 z, Y3 = -k1 x, Y4 = k2 x y, Y5 = -k2 y z,
//   Y6 = k3 (2 z^2 - x^2 - y^2), Y7 = -k2 x z, Y8 = k4 (x^2 - y^2),
// f[c] = sum_j Y_j f_hat[c][j] (features, so no offset and no clamp).
// One elementwise pass per point, memory-bound on the 36 B per channel of
// coefficients; the backward gives dL/df_hat = Y dL/df and the position
// gradient through the direction (d = v / |v|: dL/dv = (I - d d^T) dL/dd / |v|).
#include "common.h"
#include "internal.h"

namespace inpc {
namespace {

constexpr int kShBlock = 256;
constexpr float kK0 = 0.28209479177387814f;  // 1 / (2 sqrt(pi))
constexpr float kK1 = 0.4886025119029199f;   // sqrt(3 / (4 pi))
constexpr float kK2 = 1.0925484305920792f;   // sqrt(15 / (4 pi))
constexpr float kK3 = 0.31539156525252005f;  // sqrt(5 / (16 pi))
constexpr float kK4 = 0.5462742152960396f;   // sqrt(15 / (16 pi))

struct Dir {
  float x, y, z, inv_r;
};

__device__ __forceinline__ Dir view_dir(const float* __restrict__ pos, int64_t i, float cx,
                                        float cy, float cz) {
  const float vx = pos[3 * i] - cx, vy = pos[3 * i + 1] - cy, vz = pos[3 * i + 2] - cz;
  const float inv = 1.f / sqrtf(vx * vx + vy * vy + vz * vz);
  return Dir{vx * inv, vy * inv, vz * inv, inv};
}

__device__ __forceinline__ void basis(const Dir& d, float (&Y)[9]) {
  const float x = d.x, y = d.y, z = d.z;
  Y[0] = kK0;
  Y[1] = -kK1 * y;
  Y[2] = kK1 * z;
  Y[3] = -kK1 * x;
  Y[4] = kK2 * x * y;
  Y[5] = -kK2 * y * z;
  Y[6] = kK3 * (2.f * z * z - x * x - y * y);
  Y[7] = -kK2 * x * z;
  Y[8] = kK4 * (x * x - y * y);
}

// One thread per (point, channel): nine coefficients in, one feature out.
__global__ __launch_bounds__(kShBlock) void k_sh_fwd(int64_t n, int C, float cx, float cy,
                                                     float cz, const float* __restrict__ pos,
                                                     const float* __restrict__ sh,
                                                     float* __restrict__ feat) {
  const int64_t total = n * C;
  for (int64_t k = (int64_t)blockIdx.x * kShBlock + threadIdx.x; k < total;
       k += (int64_t)gridDim.x * kShBlock) {
    const int64_t i = k / C;
    const Dir d = view_dir(pos, i, cx, cy, cz);
    float Y[9];
    basis(d, Y);
    const float* s = sh + k * 9;
    float f = 0.f;
#pragma unroll
    for (int j = 0; j < 9; ++j) f = fmaf(Y[j], s[j], f);
    feat[k] = f;
  }
}

// One thread per point: dL/df_hat for every channel and the position
// gradient through the view direction.
__global__ __launch_bounds__(kShBlock) void k_sh_bwd(int64_t n, int C, float cx, float cy,
                                                     float cz, const float* __restrict__ pos,
                                                     const float* __restrict__ sh,
                                                     const float* __restrict__ grad_feat,
                                                     float* __restrict__ grad_sh,
                                                     float* __restrict__ grad_pos) {
  for (int64_t i = (int64_t)blockIdx.x * kShBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kShBlock) {
    const Dir d = view_dir(pos, i, cx, cy, cz);
    float Y[9];
    basis(d, Y);
    float gY[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) gY[j] = 0.f;
    for (int c = 0; c < C; ++c) {
      const float g = grad_feat[i * C + c];
      const float* s = sh + (i * C + c) * 9;
      float* gs = grad_sh + (i * C + c) * 9;
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        gs[j] = g * Y[j];
        gY[j] = fmaf(g, s[j], gY[j]);
      }
    }
    if (!grad_pos) continue;
    const float x = d.x, y = d.y, z = d.z;
    // dL/dd = sum_j gY_j dY_j/dd
    const float gx = -kK1 * gY[3] + kK2 * y * gY[4] - 2.f * kK3 * x * gY[6] - kK2 * z * gY[7] +
                     2.f * kK4 * x * gY[8];
    const float gy = -kK1 * gY[1] + kK2 * x * gY[4] - kK2 * z * gY[5] - 2.f * kK3 * y * gY[6] -
                     2.f * kK4 * y * gY[8];
    const float gz = kK1 * gY[2] - kK2 * y * gY[5] + 4.f * kK3 * z * gY[6] - kK2 * x * gY[7];
    const float dot = gx * x + gy * y + gz * z;
    grad_pos[3 * i] = (gx - dot * x) * d.inv_r;
    grad_pos[3 * i + 1] = (gy - dot * y) * d.inv_r;
    grad_pos[3 * i + 2] = (gz - dot * z) * d.inv_r;
  }
}

unsigned sh_grid(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kShBlock - 1) / kShBlock, 16384));
}

// Camera centre -R^T t.
void centre(const Cam& c, float* o) {
  for (int k = 0; k < 3; ++k) o[k] = -(c.R[k] * c.t[0] + c.R[3 + k] * c.t[1] + c.R[6 + k] * c.t[2]);
}

}  // namespace

hipError_t launch_sh_forward(const Cam& c, int64_t n, int C, const float* pos, const float* sh,
                             float* feat, hipStream_t s) {
  if (n == 0) return hipSuccess;
  float o[3];
  centre(c, o);
  hipLaunchKernelGGL(k_sh_fwd, dim3(sh_grid(n * C)), dim3(kShBlock), 0, s, n, C, o[0], o[1], o[2],
                     pos, sh, feat);
  return hipGetLastError();
}

hipError_t launch_sh_backward(const Cam& c, int64_t n, int C, const float* pos, const float* sh,
                              const float* grad_feat, float* grad_sh, float* grad_pos,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  float o[3];
  centre(c, o);
  hipLaunchKernelGGL(k_sh_bwd, dim3(sh_grid(n)), dim3(kShBlock), 0, s, n, C, o[0], o[1], o[2],
                     pos, sh, grad_feat, grad_sh, grad_pos);
  return hipGetLastError();
}

}  // namespace inpc
