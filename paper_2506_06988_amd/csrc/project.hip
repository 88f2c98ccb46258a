// Forward projection of every (camera, Gaussian) pair (Sec. 3.1): one thread
// per pair, FP64 arithmetic, FP32 record out. Reads the parameters as
// structure of arrays; each output array is indexed by item = cam * n + g.
#include "kernels.hpp"
#include "project_math.hpp"

namespace hr {
namespace {

__global__ __launch_bounds__(256) void k_project(
    SetDev S, const CamDev* __restrict__ cams, const float* __restrict__ means,
    const float* __restrict__ log_scales, const float* __restrict__ quats,
    const float* __restrict__ logits, const float* __restrict__ sh, uint32_t* __restrict__ tiles,
    uint32_t* __restrict__ vis, uint32_t* __restrict__ dkey, GRec* __restrict__ rec,
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
    tiles[item] = 0;
    vis[item] = 0;
    return;
  }
  tiles[item] = (uint32_t)((P.x1 - P.x0) * (P.y1 - P.y0));
  vis[item] = 1;
  dkey[item] = __float_as_uint(P.zf);
  GRec R;
  R.u = (float)P.u;
  R.v = (float)P.v;
  R.ca = (float)P.con[0];
  R.cb = (float)P.con[1];
  R.cc = (float)P.con[2];
  R.op = (float)P.op;
  R.depth = P.zf;
  R.pad = 0.f;
  R.r = (float)P.rgb[0];
  R.g = (float)P.rgb[1];
  R.b = (float)P.rgb[2];
  R.gid = (uint32_t)g;
  rec[item] = R;
  rect[item] = make_uint2((uint32_t)P.x0 | ((uint32_t)P.x1 << 16), (uint32_t)P.y0 | ((uint32_t)P.y1 << 16));
}

}  // namespace

void launch_project(const SetDev& S, const CamDev* cams, const hr_gaussians& g, const Work& w,
                    int32_t* radii, hipStream_t st) {
  const int64_t M = (int64_t)S.n * S.n_cams;
  if (M == 0) return;
  hipLaunchKernelGGL(k_project, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, S, cams,
                     g.means, g.log_scales, g.quats, g.opacity_logits, g.sh, w.tiles, w.vis,
                     w.dkey, w.rec, w.rect, w.rank_of, radii);
}

}  // namespace hr
