// Backward of the projection (chain rule from the per-rank record gradients
// to the Gaussian parameters, summed over cameras in registers), backward of
// the bilinear texture fetch, and the loss of Sec. 3.4.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "kernels.hpp"
#include "mesh_math.hpp"
#include "project_math.hpp"

namespace hr {
namespace {

// The projection backward runs in two passes so that the FP64 recomputation
// of the projection is spread over every visible (camera, Gaussian) item
// instead of looping over the cameras inside one thread per Gaussian:
//  1. k_project_bwd_geom, one thread per visible item (depth rank): recomputes
//     the projection in FP64 (every decision is the forward's) and applies the
//     chain rule in FP32 from the record gradients of mean2D, conic and
//     opacity to the Gaussian's mean, log-scales, quaternion and opacity
//     logit: 11 values, stored by rank in 48-byte slots of memory the forward
//     no longer needs;
//  2. k_project_bwd_gauss, one thread per Gaussian: sums those slots over the
//     cameras (in FP64); the colour part - the view direction and the SH
//     colour's clamp decision recomputed in FP64, the gradients to the SH
//     coefficients and, through the view direction, to the mean - runs one
//     visible item per thread of the workgroup, into the owner's LDS sums.
struct GeomGrad {
  float4 a;  // mean x y z, opacity logit
  float4 b;  // log-scales x y z, unused
  float4 c;  // quaternion w x y z
};
static_assert(sizeof(GeomGrad) <= sizeof(GRec), "geometry gradients reuse the record slots");

__global__ __launch_bounds__(256) void k_project_bwd_geom(
    SetDev S, const CamDev* __restrict__ cams, const float* __restrict__ means,
    const float* __restrict__ log_scales, const float* __restrict__ quats,
    const float* __restrict__ logits, const float* __restrict__ sh,
    const uint32_t* __restrict__ counters, const uint32_t* __restrict__ item_s,
    const float* __restrict__ gacc, GeomGrad* __restrict__ out) {
  const uint32_t nvis = counters[0];
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < nvis;
       r += gridDim.x * blockDim.x) {
    const float* ga = gacc + (size_t)r * 9;
    float G9[6];
    bool nz = false;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      G9[q] = ga[q];
      nz = nz || G9[q] != 0.f;
    }
    if (!nz) continue;  // the Gaussian pass skips this slot too
    const uint32_t it = item_s[r];
    const int c = (int)(it / (uint32_t)S.n);
    const int g = (int)(it - (uint32_t)c * (uint32_t)S.n);
    const CamDev& cam = cams[c];
    Proj P;
    project_gaussian(S, cam, means, log_scales, quats, logits, sh, g, P, false);
    GeomGrad o;
    o.a = o.b = o.c = make_float4(0.f, 0.f, 0.f, 0.f);
    if (!P.vis) {  // not reached: a ranked item was visible in the forward
      out[r] = o;
      continue;
    }
    // the chain rule in FP32 (the projection and its decisions stay FP64)
    const float op = (float)P.op, c3 = (float)P.c3, c2 = (float)P.c2, f3 = (float)P.f3;
    const float G5 = G9[5];
    // opacity: the record holds op c3 c2 (Mip-Splatting factors, 1 otherwise)
    float glg = G5 * c3 * c2 * op * (1.f - op);
    float gls[3] = {0.f, 0.f, 0.f};
    // d c3 / d log s_i = c3 f3 / (s_i^2 + f3)
    float sc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) sc[i] = (float)P.s[i];
    if (f3 > 0.f)
#pragma unroll
      for (int i = 0; i < 3; ++i) gls[i] += G5 * op * c2 * c3 * f3 / (sc[i] * sc[i] + f3);
    // c2 = sqrt(D0 / D1), D1 = det Sigma', D0 = det(Sigma' - lp I):
    // d c2 = c2 / 2 (dD0 / D0 - dD1 / D1) on the entries (a, b, c) of Sigma'
    float gma = 0.f, gmb = 0.f, gmc = 0.f;
    if (S.mip2d && !P.c2lo) {
      const float a = (float)P.cov[0], b = (float)P.cov[1], cc = (float)P.cov[2], lp = S.low_pass;
      const float D1 = a * cc - b * b, D0 = (a - lp) * (cc - lp) - b * b;
      const float gc2 = G5 * op * c3 * 0.5f * c2;
      gma = gc2 * ((cc - lp) / D0 - cc / D1);
      gmb = gc2 * (2.f * b / D1 - 2.f * b / D0);
      gmc = gc2 * ((a - lp) / D0 - a / D1);
    }
    // conic -> Sigma': H = -Q G Q with G the symmetric gradient of the conic
    const float q00 = (float)P.con[0], q01 = (float)P.con[1], q11 = (float)P.con[2];
    const float G00 = G9[2], G01 = 0.5f * G9[3], G11 = G9[4];
    const float a00 = q00 * G00 + q01 * G01, a01 = q00 * G01 + q01 * G11;
    const float a10 = q01 * G00 + q11 * G01, a11 = q01 * G01 + q11 * G11;
    // plus the 2D filter's factor; b sits in both off-diagonal entries
    const float H00 = -(a00 * q00 + a01 * q01) + gma;
    const float H01 = -(a00 * q01 + a01 * q11) + 0.5f * gmb;
    const float H11 = -(a10 * q01 + a11 * q11) + gmc;
    // Sigma' = J Sc J^T + lp:  gSc = J^T H J,  gJ = 2 H J Sc
    const float j00 = (float)P.J[0], j02 = (float)P.J[1], j11 = (float)P.J[2], j12 = (float)P.J[3];
    // HJ (2x3): row a = H[a][0] J[0][:] + H[a][1] J[1][:], J rows (j00,0,j02), (0,j11,j12)
    const float hj00 = H00 * j00, hj01 = H01 * j11, hj02 = H00 * j02 + H01 * j12;
    const float hj10 = H01 * j00, hj11 = H11 * j11, hj12 = H01 * j02 + H11 * j12;
    // gSc[k][l] = J[0][k] HJ[0][l] + J[1][k] HJ[1][l]
    float gSc[9];
    const float J0[3] = {j00, 0.f, j02}, J1[3] = {0.f, j11, j12};
    const float HJ0[3] = {hj00, hj01, hj02}, HJ1[3] = {hj10, hj11, hj12};
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) gSc[3 * k + l] = J0[k] * HJ0[l] + J1[k] * HJ1[l];
    const float Sc[9] = {(float)P.Sc[0], (float)P.Sc[1], (float)P.Sc[2],
                         (float)P.Sc[1], (float)P.Sc[3], (float)P.Sc[4],
                         (float)P.Sc[2], (float)P.Sc[4], (float)P.Sc[5]};
    auto gJ = [&](const float* HJr, int col) {
      return 2.f * (HJr[0] * Sc[col] + HJr[1] * Sc[3 + col] + HJr[2] * Sc[6 + col]);
    };
    const float gj00 = gJ(HJ0, 0), gj02 = gJ(HJ0, 2), gj11 = gJ(HJ1, 1), gj12 = gJ(HJ1, 2);
    const float x = (float)P.pc[0], y = (float)P.pc[1];
    const float fx = (float)cam.fx, fy = (float)cam.fy, iz = (float)(1.0 / P.pc[2]), iz2 = iz * iz;
    float gpc[3] = {0.f, 0.f, 0.f};
    gpc[2] += gj00 * (-fx * iz2) + gj11 * (-fy * iz2);
    if (P.clx) {
      gpc[2] += gj02 * (fx * (float)P.xc * iz2);
    } else {
      gpc[0] += gj02 * (-fx * iz2);
      gpc[2] += gj02 * (2.f * fx * x * iz2 * iz);
    }
    if (P.cly) {
      gpc[2] += gj12 * (fy * (float)P.yc * iz2);
    } else {
      gpc[1] += gj12 * (-fy * iz2);
      gpc[2] += gj12 * (2.f * fy * y * iz2 * iz);
    }
    // mean2D
    const float G0 = G9[0], G1 = G9[1];
    gpc[0] += G0 * fx * iz;
    gpc[1] += G1 * fy * iz;
    gpc[2] += -(G0 * fx * x + G1 * fy * y) * iz2;
    float cR[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) cR[q] = (float)cam.R[q];
    float gmu[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) gmu[a] = cR[a] * gpc[0] + cR[3 + a] * gpc[1] + cR[6 + a] * gpc[2];
    // Sigma_cam = N N^T, N = W Rq S:  gN = 2 gSc N (gSc symmetric)
    float N[9], Rq[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      N[q] = (float)P.N[q];
      Rq[q] = (float)P.Rq[q];
    }
    float gN[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        gN[3 * i + j] = (gSc[3 * i] + gSc[i]) * N[j] + (gSc[3 * i + 1] + gSc[3 + i]) * N[3 + j] +
                        (gSc[3 * i + 2] + gSc[6 + i]) * N[6 + j];
    // N[i][j] = (W Rq)[i][j] s_j
    float gWR[9];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      float gs = 0.f;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const float wr = cR[3 * i] * Rq[j] + cR[3 * i + 1] * Rq[3 + j] + cR[3 * i + 2] * Rq[6 + j];
        gs += gN[3 * i + j] * wr;
        gWR[3 * i + j] = gN[3 * i + j] * sc[j];
      }
      gls[j] += gs * sc[j];
    }
    // gRq = W^T gWR
    float gR[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        gR[3 * i + j] = cR[i] * gWR[j] + cR[3 + i] * gWR[3 + j] + cR[6 + i] * gWR[6 + j];
    const float w = (float)P.qn[0], qa = (float)P.qn[1], qb = (float)P.qn[2], qc = (float)P.qn[3];
    float gqn[4];
    gqn[0] = 2.f * (-qc * gR[1] + qb * gR[2] + qc * gR[3] - qa * gR[5] - qb * gR[6] + qa * gR[7]);
    gqn[1] = 2.f * (qb * gR[1] + qc * gR[2] + qb * gR[3] - 2.f * qa * gR[4] - w * gR[5] +
                    qc * gR[6] + w * gR[7] - 2.f * qa * gR[8]);
    gqn[2] = 2.f * (-2.f * qb * gR[0] + qa * gR[1] + w * gR[2] + qa * gR[3] + qc * gR[5] -
                    w * gR[6] + qc * gR[7] - 2.f * qb * gR[8]);
    gqn[3] = 2.f * (-2.f * qc * gR[0] - w * gR[1] + qa * gR[2] + w * gR[3] - 2.f * qc * gR[4] +
                    qb * gR[5] + qa * gR[6] + qb * gR[7]);
    const float dq = gqn[0] * w + gqn[1] * qa + gqn[2] * qb + gqn[3] * qc;
    const float qn4[4] = {w, qa, qb, qc};
    const float iqn = (float)(1.0 / P.qnorm);
    float gq[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) gq[a] = (gqn[a] - qn4[a] * dq) * iqn;
    o.a = make_float4(gmu[0], gmu[1], gmu[2], glg);
    o.b = make_float4(gls[0], gls[1], gls[2], 0.f);
    o.c = make_float4(gq[0], gq[1], gq[2], gq[3]);
    out[r] = o;
  }
}

// One thread per Gaussian: the camera sum of the geometry slots, the
// densification statistics and one write per gradient array; the colour part
// of every visible item spread over the workgroup's threads.
__global__ __launch_bounds__(128) void k_project_bwd_gauss(
    SetDev S, const CamDev* __restrict__ cams, const float* __restrict__ means,
    const float* __restrict__ sh, const int32_t* __restrict__ rank_of,
    const float* __restrict__ gacc, const GeomGrad* __restrict__ geo,
    float* __restrict__ g_means, float* __restrict__ g_ls, float* __restrict__ g_q,
    float* __restrict__ g_logit, float* __restrict__ g_sh, float* __restrict__ m2d_norm,
    int32_t* __restrict__ m2d_count) {
  // the 3K SH-coefficient gradients of each thread's Gaussian live in its own
  // column of LDS, the colour part of its mean gradient in gmc
  __shared__ float shacc[48 * 128];
  __shared__ float gmc[3 * 128];
  // the (Gaussian, camera) items of a group of 8 cameras with a colour
  // gradient: owner thread | camera offset << 8, rank
  __shared__ uint2 q[8 * 128];
  __shared__ uint32_t nq;
  const int tid = threadIdx.x;
  const int g = blockIdx.x * blockDim.x + tid;
  const bool own = g < S.n;
  float stat_norm = 0.f;
  int stat_cnt = 0;
  const int K = (S.sh_degree + 1) * (S.sh_degree + 1);
  double gls[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, glg = 0, gmu[3] = {0, 0, 0};
  for (int k = 0; k < 3 * K; ++k) shacc[k * 128 + tid] = 0.f;
  gmc[3 * tid] = gmc[3 * tid + 1] = gmc[3 * tid + 2] = 0.f;
  bool any = false;
  for (int c0 = 0; c0 < S.n_cams; c0 += 8) {
    if (tid == 0) nq = 0;
    __syncthreads();
    if (own) {
      // the ranks of up to 8 cameras, loaded together
      int rk[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        rk[j] = c0 + j < S.n_cams ? rank_of[(int64_t)(c0 + j) * S.n + g] : -1;
      for (int j = 0; j < 8; ++j) {
        const int r = rk[j];
        if (r < 0) continue;
        const float* ga = gacc + (size_t)r * 9;
        float G9[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) G9[k] = ga[k];
        stat_norm += sqrtf(G9[0] * G9[0] + G9[1] * G9[1]);
        ++stat_cnt;
        const bool gnz = G9[0] != 0.f || G9[1] != 0.f || G9[2] != 0.f || G9[3] != 0.f ||
                         G9[4] != 0.f || G9[5] != 0.f;
        const bool cnz = G9[6] != 0.f || G9[7] != 0.f || G9[8] != 0.f;
        if (!gnz && !cnz) continue;
        any = true;
        if (gnz) {
          const GeomGrad o = geo[r];
          gmu[0] += o.a.x; gmu[1] += o.a.y; gmu[2] += o.a.z; glg += o.a.w;
          gls[0] += o.b.x; gls[1] += o.b.y; gls[2] += o.b.z;
          gq[0] += o.c.x; gq[1] += o.c.y; gq[2] += o.c.z; gq[3] += o.c.w;
        }
        if (cnz) q[atomicAdd(&nq, 1u)] = make_uint2((uint32_t)tid | ((uint32_t)j << 8), (uint32_t)r);
      }
    }
    __syncthreads();
    // the colour part, one item per thread (the items of a Gaussian seen by
    // few cameras would otherwise leave most lanes of its wave idle): the
    // view direction and the clamp of the forward in FP64, the gradients to
    // the SH coefficients and, through the view direction, to the mean, added
    // to the owner's LDS accumulators
    const uint32_t n_q = nq;
    for (uint32_t e = (uint32_t)tid; e < n_q; e += 128) {
      const uint2 it = q[e];
      const int o = (int)(it.x & 255u), cam_i = c0 + (int)(it.x >> 8);
      const int go = blockIdx.x * blockDim.x + o;
      const float* ga = gacc + (size_t)it.y * 9;
      const float gcol[3] = {ga[6], ga[7], ga[8]};
      const float* shg = sh + (size_t)go * K * 3;
      const CamDev& cam = cams[cam_i];
      const double d0 = (double)means[3 * go] - cam.C[0], d1 = (double)means[3 * go + 1] - cam.C[1],
                   d2 = (double)means[3 * go + 2] - cam.C[2];
      const double dnorm = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      const double dir64[3] = {d0 / dnorm, d1 / dnorm, d2 / dnorm};
      double col[3];
      sh_colour64(shg, S.sh_degree, dir64, col);
      const float dir[3] = {(float)dir64[0], (float)dir64[1], (float)dir64[2]};
      float Y[16];
      sh_eval(dir, S.sh_degree, Y);
      float wdir[16];
      for (int k = 0; k < K; ++k) wdir[k] = 0.f;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        if (col[ch] < 0.0) continue;  // clamped at 0 in the forward: no gradient
        const float gc = gcol[ch];
        for (int k = 0; k < K; ++k) {
          atomicAdd(&shacc[(3 * k + ch) * 128 + o], Y[k] * gc);
          wdir[k] += shg[3 * k + ch] * gc;
        }
      }
      float gdir[3] = {0.f, 0.f, 0.f};
      sh_grad_acc(dir, S.sh_degree, wdir, gdir);
      const float dd = gdir[0] * dir[0] + gdir[1] * dir[1] + gdir[2] * dir[2];
      const float idn = 1.f / (float)dnorm;
#pragma unroll
      for (int a = 0; a < 3; ++a) atomicAdd(&gmc[3 * o + a], (gdir[a] - dir[a] * dd) * idn);
    }
    __syncthreads();
  }
  if (!own) return;
  if (m2d_norm && stat_cnt) m2d_norm[g] += stat_norm;
  if (m2d_count && stat_cnt) m2d_count[g] += stat_cnt;
  if (!any) return;
  if (g_means)
    for (int a = 0; a < 3; ++a) g_means[3 * g + a] += (float)(gmu[a] + (double)gmc[3 * tid + a]);
  if (g_ls)
    for (int a = 0; a < 3; ++a) g_ls[3 * g + a] += (float)gls[a];
  if (g_q)
    for (int a = 0; a < 4; ++a) g_q[4 * g + a] += (float)gq[a];
  if (g_logit) g_logit[g] += (float)glg;
  if (g_sh)
    for (int k = 0; k < 3 * K; ++k) g_sh[(size_t)g * K * 3 + k] += shacc[k * 128 + tid];
}


__device__ __forceinline__ int find_cam_by_tile(const CamDev* cams, int n_cams, int tile) {
  int lo = 0, hi = n_cams - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cams[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

constexpr int TEX_LDS = 4096;  // texels of one tile's footprint accumulated in LDS

// dL/dI_m = T dL/dI_h + (direct term), scattered through the bilinear weights
// the forward used (its per-pixel footprints, so nothing of the mesh is
// recomputed). One workgroup per tile: the texels the tile's pixels read from
// its most common texture (the lowest texture id present) usually form a
// small box; when the box fits in LDS the pixels accumulate there and the box
// is added to the gradient with one global atomic per non-zero texel channel.
// Pixels on other textures, and tiles whose box is too large, add directly.
__global__ __launch_bounds__(256) void k_tex_bwd(SetDev S, const CamDev* __restrict__ cams,
                                                 const uint4* __restrict__ taps,
                                                 const float* __restrict__ T_ws,
                                                 const float* __restrict__ grad_image,
                                                 const float* __restrict__ grad_mesh,
                                                 float* __restrict__ grad_tex) {
  __shared__ float acc[3 * TEX_LDS];
  __shared__ int box[5];  // tex, x0, y0, x1, y1
  const int t = blockIdx.x;
  const int c = find_cam_by_tile(cams, S.n_cams, t);
  const CamDev& C = cams[c];
  const int lt = t - C.tile_off;
  const int ty = lt / C.TX, tx = lt - (lt / C.TX) * C.TX;
  const int i = tx * TILE + (threadIdx.x & 15), j = ty * TILE + (threadIdx.x >> 4);
  if (threadIdx.x == 0) {
    box[0] = 0x7fffffff;
    box[1] = box[2] = 0x7fffffff;
    box[3] = box[4] = -1;
  }
  bool live = false;
  float gm[3] = {0.f, 0.f, 0.f};
  int tex = 0, xa = 0, ya = 0, xb = 0, yb = 0;
  float wx = 0.f, wy = 0.f;
  if (i < C.W && j < C.H) {
    const int64_t p = C.pix_off + (int64_t)j * C.W + i;
    const uint4 tq = taps[p];
    if (tq.x != ~0u) {
      const int64_t hw = (int64_t)C.W * C.H;
      const int64_t pl = 3 * C.pix_off + (p - C.pix_off);
      const float Tf = T_ws[p];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch)
        gm[ch] = (grad_image ? Tf * grad_image[pl + ch * hw] : 0.f) +
                 (grad_mesh ? grad_mesh[pl + ch * hw] : 0.f);
      live = gm[0] != 0.f || gm[1] != 0.f || gm[2] != 0.f;
      xa = (int)(tq.x & 0xffffu);
      ya = (int)(tq.x >> 16);
      tex = (int)(tq.y & 0x3fffffffu);
      xb = xa + (int)((tq.y >> 30) & 1u);
      yb = ya + (int)(tq.y >> 31);
      wx = __uint_as_float(tq.z);
      wy = __uint_as_float(tq.w);
    }
  }
  __syncthreads();
  if (live) atomicMin(&box[0], tex);
  __syncthreads();
  const int rtex = box[0];
  const bool mine = live && tex == rtex;
  if (mine) {
    atomicMin(&box[1], xa);
    atomicMin(&box[2], ya);
    atomicMax(&box[3], xb);
    atomicMax(&box[4], yb);
  }
  __syncthreads();
  const int bx0 = box[1], by0 = box[2];
  const int bw = box[3] - bx0 + 1, bh = box[4] - by0 + 1;
  const bool use_lds = rtex != 0x7fffffff && bw > 0 && bh > 0 && bw * bh <= TEX_LDS;
  const float w4[4] = {(1.f - wx) * (1.f - wy), wx * (1.f - wy), (1.f - wx) * wy, wx * wy};
  if (use_lds) {
    for (int k = threadIdx.x; k < 3 * bw * bh; k += 256) acc[k] = 0.f;
    __syncthreads();
    if (mine) {
      const int l00 = (ya - by0) * bw + (xa - bx0), l11 = (yb - by0) * bw + (xb - bx0);
      const int l10 = (ya - by0) * bw + (xb - bx0), l01 = (yb - by0) * bw + (xa - bx0);
      const int ls[4] = {l00, l10, l01, l11};
      // the four pixels of a 2x2 quad often read the same four texels: each
      // starts at a different tap, so one atomic instruction hits four texels
      const int rot = (threadIdx.x & 1) | ((threadIdx.x >> 3) & 2);
#pragma unroll
      for (int q0 = 0; q0 < 4; ++q0) {
        const int q = (q0 + rot) & 3;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) atomicAdd(&acc[3 * ls[q] + ch], w4[q] * gm[ch]);
      }
    }
  }
  if (live && !(use_lds && mine)) {
    const int64_t row = (int64_t)S.tex_w;
    const int64_t b0 = ((int64_t)tex * S.tex_h + ya) * row;
    const int64_t b1 = ((int64_t)tex * S.tex_h + yb) * row;
    const int64_t os[4] = {(b0 + xa) * 3, (b0 + xb) * 3, (b1 + xa) * 3, (b1 + xb) * 3};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) atomicAdd(grad_tex + os[q] + ch, w4[q] * gm[ch]);
  }
  if (use_lds) {
    __syncthreads();
    const int64_t plane = (int64_t)S.tex_h * S.tex_w;
    const int64_t base = (int64_t)rtex * plane;
    // consecutive threads take consecutive floats of the box's rows (the
    // three channels interleaved as in the texture), so one atomic
    // instruction covers whole cache lines; e advances by 256 = q rows + r
    const int row3 = 3 * bw, n3 = row3 * bh;
    const int q = 256 / row3, r = 256 - q * row3;
    int yy = (int)threadIdx.x / row3, rem = (int)threadIdx.x - yy * row3;
    const int64_t pitch = (int64_t)S.tex_w * 3;
    float* const dst0 = grad_tex + (base + (int64_t)by0 * S.tex_w + bx0) * 3;
    for (int e = threadIdx.x; e < n3; e += 256) {
      const float v = acc[e];
      if (v != 0.f) atomicAdd(dst0 + yy * pitch + rem, v);
      yy += q;
      rem += r;
      if (rem >= row3) {
        rem -= row3;
        ++yy;
      }
    }
  }
}

// ------------------------------------------------------------------ loss --
constexpr int LB = 256;

// Pixel p of the packed images belongs to image i with off[i] <= p < off[i+1];
// that image's planes are [3, hw_i] starting at float 3 off[i], so channel ch
// of p sits at 2 off[i] + ch hw_i + p. Each thread takes LPP pixels LB apart
// (coalesced); each workgroup writes one partial sum of its LB * LPP pixels.
constexpr int LPP = 4;
constexpr int LPB = LB * LPP;  // pixels per loss workgroup
__global__ __launch_bounds__(LB) void k_loss(const int64_t* __restrict__ off, int n_img,
                                             const float* __restrict__ image,
                                             const float* __restrict__ T,
                                             const float* __restrict__ mesh,
                                             const int32_t* __restrict__ tri,
                                             const float* __restrict__ target, int64_t n_pix,
                                             float lambda_t, float k, int detach,
                                             float* __restrict__ g_image, float* __restrict__ g_T,
                                             float* __restrict__ g_mesh,
                                             double* __restrict__ partial) {
  __shared__ double red[LB / 64];
  __shared__ int s_img;
  const float inv = 1.0f / (3.0f * (float)n_pix);
  // the image of the workgroup's first pixel; later pixels step forward
  if (threadIdx.x == 0) {
    const int64_t p0 = (int64_t)blockIdx.x * LPB;
    int lo = 0, hi = n_img - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (off[mid] <= p0) lo = mid; else hi = mid - 1;
    }
    s_img = lo;
  }
  __syncthreads();
  int img = s_img;
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < LPP; ++j) {
    const int64_t p = (int64_t)blockIdx.x * LPB + j * LB + threadIdx.x;
    if (p >= n_pix) break;
    while (off[img + 1] <= p) ++img;
    const int64_t o = off[img], hw = off[img + 1] - o;
    const bool has = tri[p] >= 0;
    const float t = T[p];
    const float mt = 1.f / (1.f + __expf(-k * (t - 0.5f)));
    float sq = 0.f;
    for (int ch = 0; ch < 3; ++ch) {
      const int64_t q = 2 * o + ch * hw + p;
      const float d = image[q] - target[q];
      acc += fabs((double)d);
      g_image[q] = (d > 0.f ? inv : (d < 0.f ? -inv : 0.f));
      if (has) {
        const float dm = mesh[q] - target[q];
        sq += dm * dm;
        g_mesh[q] = lambda_t * mt * 2.f * dm * inv;
      } else {
        g_mesh[q] = 0.f;
      }
    }
    acc += (double)lambda_t * (double)mt * (double)sq;
    g_T[p] = (detach || !has) ? 0.f : lambda_t * sq * mt * (1.f - mt) * k * inv;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (__lane_id() == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < LB / 64; ++w) s += red[w];
    partial[blockIdx.x] = s;
  }
}

// one workgroup of 1024 threads sums the partials (fixed order: deterministic)
constexpr int LF = 1024;
__global__ __launch_bounds__(LF) void k_loss_final(const double* __restrict__ partial, int64_t nb,
                                                   int64_t n_pix, float* __restrict__ out) {
  __shared__ double red[LF / 64];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t b = threadIdx.x;
  for (; b + 3 * LF < nb; b += 4 * LF) {
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] += partial[b + q * LF];
  }
  for (; b < nb; b += LF) acc[0] += partial[b];
  double a = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  if (__lane_id() == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < LF / 64; ++w) s += red[w];
    *out = (float)(s / (3.0 * (double)n_pix));
  }
}

// image offset table by kernel argument (graph-capturable)
constexpr int OFFS_PER_UPLOAD = 480;
struct OffUpload {
  int64_t v[OFFS_PER_UPLOAD];
  int32_t first, count;
};
static_assert(sizeof(OffUpload) + 8 <= 4096, "offset upload must fit in kernel arguments");

__global__ void k_upload_offs(OffUpload u, int64_t* __restrict__ dst) {
  for (int i = threadIdx.x; i < u.count; i += blockDim.x) dst[u.first + i] = u.v[i];
}


struct AdamArgs {
  hr_adam_group g[HR_ADAM_MAX_GROUPS];
  int64_t start[HR_ADAM_MAX_GROUPS + 1];
  int32_t n_groups;
  float b1, b2, omb1, omb2, eps, c1, c2;  // omb = 1 - b; c1 = 1 - b1^step, c2 = 1 - b2^step
};

__global__ __launch_bounds__(256) void k_adam(AdamArgs A) {
  const int64_t total = A.start[A.n_groups];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    int k = 0;
    while (i >= A.start[k + 1]) ++k;
    const int64_t j = i - A.start[k];
    const hr_adam_group& G = A.g[k];
    const float lr = (G.row > 0 && (int)((uint64_t)j % (uint32_t)G.row) < G.head) ? G.lr_head : G.lr;
    const float gr = G.grad[j];
    const float m = A.b1 * G.m[j] + A.omb1 * gr;
    const float v = A.b2 * G.v[j] + A.omb2 * gr * gr;
    G.m[j] = m;
    G.v[j] = v;
    G.param[j] -= lr * (m / A.c1) / (sqrtf(v / A.c2) + A.eps);
  }
}

}  // namespace

void launch_adam(const hr_adam_group* groups, int n_groups, double b1, double b2, double eps,
                 int step, hipStream_t st) {
  AdamArgs A;
  A.n_groups = n_groups;
  A.b1 = (float)b1;
  A.b2 = (float)b2;
  A.omb1 = (float)(1.0 - b1);
  A.omb2 = (float)(1.0 - b2);
  A.eps = (float)eps;
  A.c1 = (float)(1.0 - std::pow(b1, step));
  A.c2 = (float)(1.0 - std::pow(b2, step));
  int64_t acc = 0;
  for (int k = 0; k < n_groups; ++k) {
    A.g[k] = groups[k];
    A.start[k] = acc;
    acc += groups[k].n;
  }
  A.start[n_groups] = acc;
  if (acc == 0) return;
  int64_t grid = (acc + 255) / 256;
  if (grid > 8192) grid = 8192;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)grid), dim3(256), 0, st, A);
}

void launch_project_backward(const SetDev& S, const CamDev* cams, const hr_gaussians& g,
                             const Work& w, hr_grads* grads, hipStream_t st) {
  if (S.n == 0) return;
  // the record slots (by item in the forward) hold the geometry gradients by rank
  GeomGrad* geo = reinterpret_cast<GeomGrad*>(w.rec);
  const int64_t M = (int64_t)S.n * S.n_cams;
  const unsigned gg = (unsigned)std::min<int64_t>((M + 255) / 256, 16384);
  hipLaunchKernelGGL(k_project_bwd_geom, dim3(gg), dim3(256), 0, st, S, cams, g.means,
                     g.log_scales, g.quats, g.opacity_logits, g.sh, w.counters, w.item_s, w.gacc,
                     geo);
  hipLaunchKernelGGL(k_project_bwd_gauss, dim3((S.n + 127) / 128), dim3(128), 0, st, S, cams,
                     g.means, g.sh, w.rank_of, w.gacc, (const GeomGrad*)geo, grads->means,
                     grads->log_scales, grads->quats, grads->opacity_logits, grads->sh,
                     grads->mean2d_norm, grads->mean2d_count);
}

void launch_texture_backward(const SetDev& S, const hr_mesh& m, const Work& w,
                             const float* grad_image, const float* grad_mesh_rgb, float* grad_tex,
                             hipStream_t st) {
  (void)m;
  if (S.n_faces == 0 || !grad_tex || S.n_pix == 0) return;
  hipLaunchKernelGGL(k_tex_bwd, dim3((unsigned)S.n_tiles), dim3(256), 0, st, S, w.cams,
                     (const uint4*)w.taps, w.final_T, grad_image, grad_mesh_rgb, grad_tex);
}

size_t loss_scratch_bytes(int64_t n_pix, int32_t n_img) {
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  return al(8 * ((size_t)n_img + 1)) + ((size_t)(n_pix + LPB - 1) / LPB + 1) * sizeof(double);
}

void launch_loss(const float* image, const float* T, const float* mesh_rgb, const int32_t* tri,
                 const float* target, const int64_t* img_pix, int32_t n_img, float lambda_t,
                 float k, bool detach, float* loss, float* g_image, float* g_T, float* g_mesh,
                 void* scratch, hipStream_t st) {
  // scratch: image pixel offsets [n_img + 1] | per-workgroup partial sums
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  int64_t* off = (int64_t*)scratch;
  double* partial = (double*)((char*)scratch + al(8 * ((size_t)n_img + 1)));
  int64_t n_pix = 0;
  OffUpload u;
  u.first = 0;
  u.count = 0;
  for (int i = 0; i <= n_img; ++i) {
    u.v[u.count++] = n_pix;
    if (i < n_img) n_pix += img_pix[i];
    if (u.count == OFFS_PER_UPLOAD || i == n_img) {
      hipLaunchKernelGGL(k_upload_offs, dim3(1), dim3(256), 0, st, u, off);
      u.first += u.count;
      u.count = 0;
    }
  }
  const int64_t nb = (n_pix + LPB - 1) / LPB;
  if (nb > 0)
    hipLaunchKernelGGL(k_loss, dim3((unsigned)nb), dim3(LB), 0, st, (const int64_t*)off, n_img,
                       image, T, mesh_rgb, tri, target, n_pix, lambda_t, k, detach ? 1 : 0,
                       g_image, g_T, g_mesh, partial);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(LF), 0, st, partial, nb, n_pix, loss);
}

// Library-owned scratch of hr_hybrid_loss_noalloc: one copy per GPU, held
// until the process ends. Host code never passes `loss_static_scratch` itself
// to a kernel (in host code it names a host-side stand-in); it passes the
// device address hipGetSymbolAddress returns for the current device.
constexpr size_t LOSS_STATIC_BYTES = 2304 + ((size_t)(HR_LOSS_NOALLOC_MAX_PIXELS / LPB) + 1) * 8;
static_assert((size_t)8 * (HR_LOSS_NOALLOC_MAX_IMAGES + 1) <= 2304, "image table part");
__device__ __align__(256) unsigned char loss_static_scratch[LOSS_STATIC_BYTES];

hr_status loss_static_scratch_ptr(void** out) {
  static std::mutex mu;
  static void* per_dev[64] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return HR_ERR_HIP;
  std::lock_guard<std::mutex> lock(mu);
  if (!per_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(loss_static_scratch)) != hipSuccess || !p)
      return HR_ERR_HIP;
    per_dev[dev] = p;
  }
  *out = per_dev[dev];
  return HR_OK;
}

size_t loss_static_scratch_bytes() { return LOSS_STATIC_BYTES; }

}  // namespace hr
