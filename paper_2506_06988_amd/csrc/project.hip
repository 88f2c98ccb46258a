// Forward projection of every (camera, Gaussian) pair (Sec. 3.1): one thread
// per pair, FP64 arithmetic, FP32 record out. Reads the parameters as
// structure of arrays; each output array is indexed by item = cam * n + g.
#include <algorithm>
#include <cstring>

#include "kernels.hpp"
#include "project_math.hpp"

namespace hr {
namespace {

__global__ __launch_bounds__(256) void k_project(
    SetDev S, const CamDev* __restrict__ cams, const float* __restrict__ means,
    const float* __restrict__ log_scales, const float* __restrict__ quats,
    const float* __restrict__ logits, const float* __restrict__ sh, uint32_t* __restrict__ vis, uint32_t* __restrict__ dkey, GRec* __restrict__ rec,
    uint2* __restrict__ rect, int32_t* __restrict__ rank_of, int32_t* __restrict__ radii) {
  const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t M = (int64_t)S.n * S.n_cams;
  if (item >= M) return;
  const int cam = (int)(item / S.n);
  const int g = (int)(item - (int64_t)cam * S.n);
  Proj P;
  project_gaussian(S, cams[cam], means, log_scales, quats, logits, sh, g, P, true);
  rank_of[item] = -1;
  if (radii) radii[item] = P.vis ? P.r : 0;
  if (!P.vis) {
    vis[item] = 0;
    return;
  }
  vis[item] = 1;
  dkey[item] = __float_as_uint(P.zf);
  GRec R;
  R.u = (float)P.u;
  R.v = (float)P.v;
  R.ca = (float)P.con[0];
  R.cb = (float)P.con[1];
  R.cc = (float)P.con[2];
  R.op = (float)P.opr;
  R.depth = P.zf;
  R.pad = 0.f;
  R.r = (float)P.rgb[0];
  R.g = (float)P.rgb[1];
  R.b = (float)P.rgb[2];
  R.gid = (uint32_t)g;
  rec[item] = R;
  rect[item] = make_uint2((uint32_t)P.x0 | ((uint32_t)P.x1 << 16), (uint32_t)P.y0 | ((uint32_t)P.y1 << 16));
}

// Mip-Splatting 3D filter, pass 1 (one launch per group of up to
// CAMS_PER_UPLOAD views): the running highest sampling rate fx / z of every
// Gaussian over the views that see it, kept in nu[] (0 = unseen so far).
__global__ __launch_bounds__(256) void k_f3_rate(CamUpload U, const float* __restrict__ means,
                                                 int n, float near, float* __restrict__ nu) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const double mu[3] = {means[3 * g], means[3 * g + 1], means[3 * g + 2]};
  double best = nu[g];
  for (int c = 0; c < U.count; ++c) {
    const CamDev& C = U.c[c];
    double pc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
      pc[i] = C.R[3 * i] * mu[0] + C.R[3 * i + 1] * mu[1] + C.R[3 * i + 2] * mu[2] + C.t[i];
    if (!(pc[2] > (double)near)) continue;
    const double u = C.fx * pc[0] / pc[2] + C.cx, v = C.fy * pc[1] / pc[2] + C.cy;
    if (u < -0.15 * C.W || u > 1.15 * C.W || v < -0.15 * C.H || v > 1.15 * C.H) continue;
    best = fmax(best, C.fx / pc[2]);
  }
  nu[g] = (float)best;
}

// Pass 2, one workgroup: variance scale / nu^2; unseen Gaussians take the
// largest variance of the seen ones.
__global__ __launch_bounds__(1024) void k_f3_final(int n, double scale, float* __restrict__ f3) {
  __shared__ double red[16];
  double vmax = 0.0;
  for (int g = threadIdx.x; g < n; g += blockDim.x) {
    const double nu = f3[g];
    if (nu > 0.0) vmax = fmax(vmax, scale / (nu * nu));
  }
  for (int o = 32; o > 0; o >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = vmax;
  __syncthreads();
  vmax = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) vmax = fmax(vmax, red[w]);
  for (int g = threadIdx.x; g < n; g += blockDim.x) {
    const double nu = f3[g];
    f3[g] = (float)(nu > 0.0 ? scale / (nu * nu) : vmax);
  }
}

}  // namespace

void launch_mip_filter3d(const float* means, int n, const CamDev* cams, int n_cams, float near,
                         double scale, float* f3, hipStream_t st) {
  if (n <= 0) return;
  launch_fill_u32(reinterpret_cast<uint32_t*>(f3), 0u, n, st);
  for (int c0 = 0; c0 < n_cams; c0 += CAMS_PER_UPLOAD) {
    CamUpload U;
    std::memset(&U, 0, sizeof(U));
    U.first = c0;
    U.count = std::min(CAMS_PER_UPLOAD, n_cams - c0);
    for (int k = 0; k < U.count; ++k) U.c[k] = cams[c0 + k];
    hipLaunchKernelGGL(k_f3_rate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, U, means, n,
                       near, f3);
  }
  hipLaunchKernelGGL(k_f3_final, dim3(1), dim3(1024), 0, st, n, scale, f3);
}

void launch_project(const SetDev& S, const CamDev* cams, const hr_gaussians& g, const Work& w,
                    int32_t* radii, hipStream_t st) {
  const int64_t M = (int64_t)S.n * S.n_cams;
  if (M == 0) return;
  hipLaunchKernelGGL(k_project, dim3((unsigned)((M + 127) / 128)), dim3(128), 0, st, S, cams,
                     g.means, g.log_scales, g.quats, g.opacity_logits, g.sh, w.vis,
                     w.dkey, w.rec, w.rect, w.rank_of, radii);
}

}  // namespace hr
