// Photometric loss of Eq. 3 (L1 and D-SSIM) with the transmittance-aware term
// of Sec. 3.4, forward and gradient, over several images packed like the
// renderer's outputs.
//
// SSIM per channel: 11x11 Gaussian window (sigma 1.5, separable), zero
// padding. With N1 = 2 mu_x mu_y + C1, N2 = 2 s_xy + C2, D1 = mu_x^2 + mu_y^2
// + C1, D2 = s_xx + s_yy + C2 and S = N1 N2 / (D1 D2), the gradient is
//   dS_mean/dx_q = (G * A)(q) + 2 x_q (G * B)(q) + y_q (G * C)(q)
// with A = dS/dmu_x - 2 mu_x dS/ds_xx - mu_y dS/ds_xy, B = dS/ds_xx,
// C = dS/ds_xy, so the forward stores A, B, C and the backward blurs them.
// One 256-thread workgroup per 16x16 tile; a 26x26 patch sits in LDS.
#include <cmath>
#include <vector>

#include "kernels.hpp"

namespace hr {

namespace {

constexpr int R = 5;             // window radius
constexpr int PW = TILE + 2 * R; // patch width

struct ImgInfo {
  int32_t W, H, TX, pad;
  int64_t pix_off, tile_off;
};

constexpr int IMGS_PER_UPLOAD = 96;
struct ImgUpload {
  ImgInfo im[IMGS_PER_UPLOAD];
  int32_t first, count;
};
static_assert(sizeof(ImgUpload) + 8 <= 4096, "image table must fit in kernel arguments");

__global__ void k_upload_imgs(ImgUpload u, ImgInfo* dst) {
  if ((int)threadIdx.x < u.count) dst[u.first + threadIdx.x] = u.im[threadIdx.x];
}

struct Win {
  float w[2 * R + 1];
};

__device__ __forceinline__ int find_img(const ImgInfo* im, int n, int64_t tile) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (im[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// loads a zero-padded PW x PW patch of plane `src` around tile (tx, ty)
__device__ __forceinline__ void load_patch(const float* __restrict__ src, const ImgInfo& I, int tx,
                                           int ty, float (*dst)[PW]) {
  for (int k = threadIdx.x; k < PW * PW; k += 256) {
    const int r = k / PW, c = k - r * PW;
    const int x = tx * TILE + c - R, y = ty * TILE + r - R;
    dst[r][c] = (x >= 0 && y >= 0 && x < I.W && y < I.H) ? src[(int64_t)y * I.W + x] : 0.f;
  }
}

__global__ __launch_bounds__(256) void k_ssim_fwd(const ImgInfo* __restrict__ imgs, int n_imgs,
                                                  int64_t n_pix, Win win,
                                                  const float* __restrict__ image,
                                                  const float* __restrict__ target,
                                                  const float* __restrict__ T,
                                                  const float* __restrict__ mesh,
                                                  const int32_t* __restrict__ tri, float lambda_t,
                                                  float k, int mask_mode, int detach, float c1,
                                                  float c2, float* __restrict__ g_T,
                                                  float* __restrict__ g_mesh,
                                                  float* __restrict__ abc,
                                                  double* __restrict__ partial) {
  __shared__ float px[PW][PW], py[PW][PW];
  __shared__ float hs[5][PW][TILE];
  __shared__ double red[3][4];
  const int t = blockIdx.x;
  const int ii = find_img(imgs, n_imgs, t);
  const ImgInfo& I = imgs[ii];
  const int lt = (int)(t - I.tile_off);
  const int ty = lt / I.TX, tx = lt - (lt / I.TX) * I.TX;
  const int lx = threadIdx.x & 15, ly = threadIdx.x >> 4;
  const int x = tx * TILE + lx, y = ty * TILE + ly;
  const bool inside = x < I.W && y < I.H;
  const int64_t hw = (int64_t)I.W * I.H;
  const int64_t p = I.pix_off + (int64_t)y * I.W + x;
  const int64_t pl = 3 * I.pix_off + (int64_t)y * I.W + x;
  const float inv = 1.0f / (3.0f * (float)n_pix);
  double s_l1 = 0.0, s_ssim = 0.0, s_lt = 0.0;
  for (int ch = 0; ch < 3; ++ch) {
    load_patch(image + 3 * I.pix_off + ch * hw, I, tx, ty, px);
    load_patch(target + 3 * I.pix_off + ch * hw, I, tx, ty, py);
    __syncthreads();
    // horizontal pass over PW rows x TILE columns, 5 moments
    for (int k2 = threadIdx.x; k2 < PW * TILE; k2 += 256) {
      const int r = k2 / TILE, c = k2 - r * TILE;
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f;
#pragma unroll
      for (int q = 0; q <= 2 * R; ++q) {
        const float u = px[r][c + q], v = py[r][c + q], wq = win.w[q];
        a0 += wq * u;
        a1 += wq * v;
        a2 += wq * u * u;
        a3 += wq * v * v;
        a4 += wq * u * v;
      }
      hs[0][r][c] = a0; hs[1][r][c] = a1; hs[2][r][c] = a2; hs[3][r][c] = a3; hs[4][r][c] = a4;
    }
    __syncthreads();
    float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q <= 2 * R; ++q)
#pragma unroll
      for (int j = 0; j < 5; ++j) m[j] += win.w[q] * hs[j][ly + q][lx];
    if (inside) {
      const float mx = m[0], my = m[1];
      const float sxx = m[2] - mx * mx, syy = m[3] - my * my, sxy = m[4] - mx * my;
      const float N1 = 2.f * mx * my + c1, N2 = 2.f * sxy + c2;
      const float D1 = mx * mx + my * my + c1, D2 = sxx + syy + c2;
      const float S = (N1 * N2) / (D1 * D2);
      const float dmx = (2.f * my * N2) / (D1 * D2) - 2.f * mx * S / D1;
      const float dsxx = -S / D2;
      const float dsxy = 2.f * N1 / (D1 * D2);
      abc[pl + ch * hw] = dmx - 2.f * mx * dsxx - my * dsxy;
      abc[3 * n_pix + pl + ch * hw] = dsxx;
      abc[6 * n_pix + pl + ch * hw] = dsxy;
      s_ssim += (double)S;
      s_l1 += fabs((double)(px[ly + R][lx + R] - py[ly + R][lx + R]));
    }
    __syncthreads();
  }
  if (inside) {
    const bool has = tri[p] >= 0;
    float sq = 0.f;
    if (has && mask_mode != 0) {
      for (int ch = 0; ch < 3; ++ch) {
        const float d = mesh[pl + ch * hw] - target[pl + ch * hw];
        sq += d * d;
      }
    }
    const float tt = T[p];
    float mt = 1.f, dmt = 0.f;
    if (mask_mode == 2) {
      mt = tt;
      dmt = 1.f;
    } else if (mask_mode == 3) {
      mt = 1.f / (1.f + __expf(-k * (tt - 0.5f)));
      dmt = k * mt * (1.f - mt);
    }
    s_lt = (double)mt * (double)sq;
    g_T[p] = (mask_mode == 0 || detach || !has) ? 0.f : lambda_t * sq * dmt * inv;
    for (int ch = 0; ch < 3; ++ch)
      g_mesh[pl + ch * hw] = (mask_mode == 0 || !has)
                                 ? 0.f
                                 : lambda_t * mt * 2.f * (mesh[pl + ch * hw] - target[pl + ch * hw]) * inv;
  }
  // workgroup sums
  double v[3] = {s_l1, s_ssim, s_lt};
#pragma unroll
  for (int j = 0; j < 3; ++j)
    for (int o = 32; o > 0; o >>= 1) v[j] += __shfl_xor(v[j], o, 64);
  if (__lane_id() == 0)
    for (int j = 0; j < 3; ++j) red[j][threadIdx.x >> 6] = v[j];
  __syncthreads();
  if (threadIdx.x < 3) {
    double sacc = 0.0;
    for (int w4 = 0; w4 < 4; ++w4) sacc += red[threadIdx.x][w4];
    partial[3 * (int64_t)blockIdx.x + threadIdx.x] = sacc;
  }
}

__global__ __launch_bounds__(256) void k_ssim_bwd(const ImgInfo* __restrict__ imgs, int n_imgs,
                                                  int64_t n_pix, Win win,
                                                  const float* __restrict__ image,
                                                  const float* __restrict__ target,
                                                  const float* __restrict__ abc, float lambda_c,
                                                  float* __restrict__ g_image) {
  __shared__ float pa[3][PW][PW];
  __shared__ float hs[3][PW][TILE];
  const int t = blockIdx.x;
  const int ii = find_img(imgs, n_imgs, t);
  const ImgInfo& I = imgs[ii];
  const int lt = (int)(t - I.tile_off);
  const int ty = lt / I.TX, tx = lt - (lt / I.TX) * I.TX;
  const int lx = threadIdx.x & 15, ly = threadIdx.x >> 4;
  const int x = tx * TILE + lx, y = ty * TILE + ly;
  const bool inside = x < I.W && y < I.H;
  const int64_t hw = (int64_t)I.W * I.H;
  const int64_t pl = 3 * I.pix_off + (int64_t)y * I.W + x;
  const float inv = 1.0f / (3.0f * (float)n_pix);
  for (int ch = 0; ch < 3; ++ch) {
    for (int j = 0; j < 3; ++j)
      load_patch(abc + j * 3 * n_pix + 3 * I.pix_off + ch * hw, I, tx, ty, pa[j]);
    __syncthreads();
    for (int k2 = threadIdx.x; k2 < PW * TILE; k2 += 256) {
      const int r = k2 / TILE, c = k2 - r * TILE;
      float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
      for (int q = 0; q <= 2 * R; ++q) {
        const float wq = win.w[q];
        a0 += wq * pa[0][r][c + q];
        a1 += wq * pa[1][r][c + q];
        a2 += wq * pa[2][r][c + q];
      }
      hs[0][r][c] = a0; hs[1][r][c] = a1; hs[2][r][c] = a2;
    }
    __syncthreads();
    float bA = 0.f, bB = 0.f, bC = 0.f;
#pragma unroll
    for (int q = 0; q <= 2 * R; ++q) {
      bA += win.w[q] * hs[0][ly + q][lx];
      bB += win.w[q] * hs[1][ly + q][lx];
      bC += win.w[q] * hs[2][ly + q][lx];
    }
    if (inside) {
      const float xv = image[pl + ch * hw], yv = target[pl + ch * hw];
      const float d = xv - yv;
      const float sgn = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
      g_image[pl + ch * hw] =
          (1.f - lambda_c) * sgn * inv - lambda_c * inv * (bA + 2.f * xv * bB + yv * bC);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_full_loss_final(const double* __restrict__ partial,
                                                         int64_t nb, int64_t n_pix,
                                                         float lambda_c, float lambda_t,
                                                         int mask_mode, float* __restrict__ out) {
  __shared__ double red[3][4];
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t b = threadIdx.x; b < nb; b += 256)
    for (int j = 0; j < 3; ++j) v[j] += partial[3 * b + j];
  for (int j = 0; j < 3; ++j)
    for (int o = 32; o > 0; o >>= 1) v[j] += __shfl_xor(v[j], o, 64);
  if (__lane_id() == 0)
    for (int j = 0; j < 3; ++j) red[j][threadIdx.x >> 6] = v[j];
  __syncthreads();
  if (threadIdx.x == 0) {
    double s[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < 3; ++j)
      for (int w4 = 0; w4 < 4; ++w4) s[j] += red[j][w4];
    const double n = 3.0 * (double)n_pix;
    double L = (1.0 - lambda_c) * s[0] / n + lambda_c * (1.0 - s[1] / n);
    if (mask_mode != 0) L += lambda_t * s[2] / n;
    *out = (float)L;
  }
}

}  // namespace

size_t full_loss_scratch_bytes(int64_t n_pix, int64_t n_tiles, int32_t n_imgs) {
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  return al(sizeof(ImgInfo) * (size_t)n_imgs) + al(9 * 4 * (size_t)n_pix) + al(24 * (size_t)n_tiles);
}

void launch_full_loss(const float* image, const float* T, const float* mesh, const int32_t* tri,
                      const float* target, const int32_t* sizes, int32_t n_imgs, float lambda_c,
                      float lambda_t, float k, int mask_mode, bool detach, float* loss,
                      float* g_image, float* g_T, float* g_mesh, void* scratch, hipStream_t st) {
  // scratch: image table | A B C maps | partial sums
  char* s = (char*)scratch;
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  ImgInfo* imgs = (ImgInfo*)s;
  int64_t P = 0, tiles = 0;
  std::vector<ImgInfo> info(n_imgs);
  for (int i = 0; i < n_imgs; ++i) {
    ImgInfo& I = info[i];
    I.W = sizes[2 * i];
    I.H = sizes[2 * i + 1];
    I.TX = (I.W + TILE - 1) / TILE;
    I.pad = 0;
    I.pix_off = P;
    I.tile_off = tiles;
    P += (int64_t)I.W * I.H;
    tiles += (int64_t)I.TX * ((I.H + TILE - 1) / TILE);
  }
  size_t off = al(sizeof(ImgInfo) * (size_t)n_imgs);
  float* abc = (float*)(s + off);
  off += al(9 * 4 * (size_t)P);
  double* partial = (double*)(s + off);
  for (int i0 = 0; i0 < n_imgs; i0 += IMGS_PER_UPLOAD) {
    ImgUpload u;
    u.first = i0;
    u.count = n_imgs - i0 < IMGS_PER_UPLOAD ? n_imgs - i0 : IMGS_PER_UPLOAD;
    for (int j = 0; j < u.count; ++j) u.im[j] = info[i0 + j];
    hipLaunchKernelGGL(k_upload_imgs, dim3(1), dim3(IMGS_PER_UPLOAD), 0, st, u, imgs);
  }
  Win win;
  double g[2 * R + 1], sum = 0.0;
  for (int q = 0; q <= 2 * R; ++q) {
    const double d = q - R;
    g[q] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    sum += g[q];
  }
  for (int q = 0; q <= 2 * R; ++q) win.w[q] = (float)(g[q] / sum);
  const float c1 = 0.01f * 0.01f, c2 = 0.03f * 0.03f;
  if (tiles > 0) {
    hipLaunchKernelGGL(k_ssim_fwd, dim3((unsigned)tiles), dim3(256), 0, st, imgs, n_imgs, P, win,
                       image, target, T, mesh, tri, lambda_t, k, mask_mode, detach ? 1 : 0, c1, c2,
                       g_T, g_mesh, abc, partial);
    hipLaunchKernelGGL(k_ssim_bwd, dim3((unsigned)tiles), dim3(256), 0, st, imgs, n_imgs, P, win,
                       image, target, abc, lambda_c, g_image);
  }
  hipLaunchKernelGGL(k_full_loss_final, dim3(1), dim3(256), 0, st, partial, tiles, P, lambda_c,
                     lambda_t, mask_mode, loss);
}

}  // namespace hr
