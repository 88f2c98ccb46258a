// Per-tile front-to-back blending with the mesh depth stop (Sec. 3.1 Eq. 2,
// Sec. 3.4 "Joint optimization", paragraph "Joint rasterization") and its reverse-order backward.
//
// One 256-thread workgroup (4 waves of 64) per 16x16 tile, one pixel per
// thread. The tile's depth-ordered list is streamed through LDS in batches of
// BG records; every pixel walks the batch from LDS (broadcast reads). A pixel
// stops at the first Gaussian whose depth reaches D_m, or before T would drop
// under t_min; the workgroup leaves as soon as every pixel has stopped.
#include "kernels.hpp"
#include "mesh_math.hpp"
#include "window.hpp"

namespace hr {
namespace {

__device__ __forceinline__ int find_cam_by_tile(const CamDev* cams, int n_cams, int tile) {
  int lo = 0, hi = n_cams - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cams[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// LDS form of a record: conic pre-scaled by log2(e) and the opacity folded
// into the exponent, so that the unclamped alpha = opacity * G is exp2(p2);
// alpha < alpha_min is then p2 < log2(alpha_min), one threshold for all
struct Staged {
  float4 a;  // u, v, A2 = -ca/2 log2e, B2 = -cb log2e
  float4 b;  // C2 = -cc/2 log2e, log2(opacity), depth, opacity
  float4 c;  // r, g, b, unused
};

__device__ __forceinline__ Staged stage(const GRec& R) {
  Staged s;
  s.a = make_float4(R.u, R.v, -0.5f * LOG2E * R.ca, -LOG2E * R.cb);
  s.b = make_float4(-0.5f * LOG2E * R.cc, __log2f(R.op), R.depth, R.op);
  s.c = make_float4(R.r, R.g, R.b, 0.f);
  return s;
}

// log2 of the unclamped alpha of the Gaussian at pixel centre (px, py); the
// operation order is fixed so the backward reproduces the forward bit for bit
__device__ __forceinline__ float gauss_p2(const float4& a, const float4& b, float px, float py,
                                          float& dx, float& dy) {
  dx = a.x - px;
  dy = a.y - py;
  // A2 dx^2 + B2 dx dy + C2 dy^2 + log2(op) as dx (A2 dx + B2 dy) + (C2 dy dy + log2(op))
  const float t = __builtin_fmaf(a.w, dy, a.z * dx);
  return __builtin_fmaf(dx, t, __builtin_fmaf(b.x * dy, dy, b.y));
}

struct TileCtx {
  int cam, i, j;
  bool inside;
  int64_t p;  // packed pixel
};

__device__ __forceinline__ TileCtx tile_ctx(const CamDev* cams, int n_cams, int t) {
  TileCtx c;
  c.cam = find_cam_by_tile(cams, n_cams, t);
  const CamDev& C = cams[c.cam];
  const int lt = t - C.tile_off;
  const int ty = lt / C.TX;
  const int tx = lt - ty * C.TX;
  c.i = tx * TILE + (threadIdx.x & 15);
  c.j = ty * TILE + (threadIdx.x >> 4);
  c.inside = c.i < C.W && c.j < C.H;
  c.p = C.pix_off + (int64_t)c.j * C.W + c.i;
  return c;
}

// Front-to-back blend of one staged batch for this thread's pixel.
struct PixState {
  float T, cr, cg, cb;
  int nc, nbl, npro;
  bool done;
};

// number of staged entries in front of depth Dm (depths ascend in a batch)
__device__ __forceinline__ int front_count(const Staged* sh, int n, float Dm) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (sh[mid].b.z < Dm) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ void blend_batch(const Staged* sh, int n, int64_t pos0, float px,
                                            float py, float Dm, float lthr, float amax,
                                            float tmin, PixState& ps) {
  // a Gaussian at or behind the mesh ends the pixel (Sec. 3.4)
  const int nv = front_count(sh, n, Dm);
  int stop = nv < n ? nv : -1;  // entry that ends the pixel, if any
  // single-exit loop: a T stop moves k past the end
  const Staged* e = sh;
  for (int k = 0; k < nv; ++k, ++e) {
    const float4 a = e->a, b = e->b;
    float dx, dy;
    const float p2 = gauss_p2(a, b, px, py, dx, dy);
    if (p2 >= lthr) {  // else alpha < alpha_min: skipped
      const float alpha = fminf(amax, __builtin_amdgcn_exp2f(p2));
      const float Tn = ps.T * (1.f - alpha);
      if (Tn < tmin) {
        stop = k;
        k = nv;
      } else {
        const float4 c = e->c;
        const float wgt = alpha * ps.T;
        ps.cr = __builtin_fmaf(c.x, wgt, ps.cr);
        ps.cg = __builtin_fmaf(c.y, wgt, ps.cg);
        ps.cb = __builtin_fmaf(c.z, wgt, ps.cb);
        ps.T = Tn;
        ps.nc = (int)pos0 + k + 1;
        ++ps.nbl;
      }
    }
  }
  if (stop >= 0) {
    ps.done = true;
    ps.npro = (int)pos0 + stop + 1;
  }
}

// DEPTH 1: extract ranks, barrier, load and stage, barrier, blend.
// DEPTH 2: the next batch's records are loaded into registers before the
// current batch is blended and written to the other LDS buffer after it,
// leaving one barrier per batch.
struct FwdArgs {
  SetDev S;
  const CamDev* cams;
  const uint32_t* vis_off;
  const uint32_t* mat;
  const uint32_t* tile_start;
  const uint32_t* tile_total;
  const uint32_t* tile_order;
  const uint32_t* lists;
  const GRec* rec_s;
  const unsigned long long* zbuf;
  const float* mesh_rgb;
  float* image;
  float* T_ws;
  int32_t* nc_ws;
  float* T_out;
  int32_t* nc_out;
  int32_t* nb_out;
  int32_t* np_out;
  unsigned long long* tile_np;  // [2 * n_tiles] examined, blended pairs of each tile
  // shading of the mesh pixels (SHADE kernels): triangles, textures, outputs
  const TriRec* tris;
  const float* tex;
  MeshOut mo;
};

template <int BG, int DEPTH>
struct FwdShared {
  Staged sh[DEPTH][BG];
  uint32_t rk[DEPTH][BG];
  uint32_t bitmap[WIN_WORDS];
  uint32_t red4[4];
  unsigned long long red[2];
};

// blend and composite one tile t (all 256 threads of the group); SHADE: the
// mesh colour of each pixel is computed here (mesh_shade) rather than read
template <int BG, int DEPTH, bool SHADE>
__device__ __forceinline__ void blend_tile(const FwdArgs& A, FwdShared<BG, DEPTH>& L, int t) {
  const SetDev& S = A.S;
  const CamDev* __restrict__ cams = A.cams;
  const uint32_t* __restrict__ lists = A.lists;
  const GRec* __restrict__ rec_s = A.rec_s;
  const float* mesh_rgb = A.mesh_rgb;  // written by mesh_shade in SHADE mode: no restrict
  auto& sh = L.sh;
  auto& rk = L.rk;
  auto& bitmap = L.bitmap;
  auto& red4 = L.red4;
  auto& red = L.red;
  const TileCtx tc = tile_ctx(cams, S.n_cams, t);
  const CamDev& C = cams[tc.cam];
  const WinCtx W = win_ctx(C, tc.cam, t, A.vis_off, A.mat, A.tile_start, A.tile_total, S.key_cap);
  const float px = (float)tc.i + 0.5f, py = (float)tc.j + 0.5f;
  unsigned long long key = ~0ull;
  if (tc.inside) key = A.zbuf[tc.p];
  const float Dm = key == ~0ull ? __int_as_float(0x7f800000) : __uint_as_float((uint32_t)(key >> 32));
  // the pixel's mesh shading first: its loads overlap the tile's list work,
  // and the composite reads the colour back (this thread's own store)
  if (SHADE && tc.inside) {
    float rgb[3];
    mesh_shade(S, C, tc.i, tc.j, tc.p, key, A.tris, A.tex, A.mo, rgb);
  }
  const float lthr = __log2f(S.alpha_min), amax = S.alpha_max, tmin = S.t_min;
  const uint32_t rmax = (uint32_t)((int64_t)S.n * S.n_cams - 1);
  PixState ps;
  ps.T = 1.f;
  ps.cr = ps.cg = ps.cb = 0.f;
  ps.nc = ps.nbl = 0;
  ps.npro = (int)W.lim;
  ps.done = !tc.inside;
  if (threadIdx.x == 0) red[0] = red[1] = 0;
  bool all_done = false;
  for (int w = 0; w < W.nwin && !all_done; ++w) {
    int64_t a, b;
    win_range(W, w, a, b);
    if (a >= b) continue;
    if (__syncthreads_and(ps.done)) break;
    const uint32_t wbase = W.rbase + (uint32_t)w * WIN;
    bitmap[threadIdx.x] = 0;
    __syncthreads();
    win_mark(lists, W, a, b, wbase, bitmap);
    __syncthreads();
    const uint32_t word = bitmap[threadIdx.x];
    uint32_t total;
    const uint32_t pre = group_excl_scan((uint32_t)__popc(word), red4, total);
    const int nbat = (int)((total + BG - 1) / BG);
    if (DEPTH == 1) {
      for (int bi = 0; bi < nbat; ++bi) {
        const uint32_t q = (uint32_t)bi * BG;
        const int n = (int)min((uint32_t)BG, total - q);
        if (bi > 0 && __syncthreads_and(ps.done)) {
          all_done = true;
          break;
        }
        win_extract(word, pre, q, (uint32_t)n, wbase, rk[0]);
        __syncthreads();
        if (threadIdx.x < n) sh[0][threadIdx.x] = stage(rec_s[min(rk[0][threadIdx.x], rmax)]);
        __syncthreads();
        if (!ps.done) blend_batch(sh[0], n, a + q, px, py, Dm, lthr, amax, tmin, ps);
      }
    } else {
      win_extract(word, pre, 0, (uint32_t)min((uint32_t)BG, total), wbase, rk[0]);
      __syncthreads();
      if (threadIdx.x < min((uint32_t)BG, total)) sh[0][threadIdx.x] = stage(rec_s[min(rk[0][threadIdx.x], rmax)]);
      for (int bi = 0; bi < nbat; ++bi) {
        const int cur = bi & 1;
        const uint32_t q = (uint32_t)bi * BG;
        const int n = (int)min((uint32_t)BG, total - q);
        const bool more = bi + 1 < nbat;
        const int nn = more ? (int)min((uint32_t)BG, total - q - BG) : 0;
        if (more) win_extract(word, pre, q + BG, (uint32_t)nn, wbase, rk[cur ^ 1]);
        if (__syncthreads_and(ps.done)) {
          all_done = true;
          break;
        }
        GRec nxt;
        if (threadIdx.x < nn) nxt = rec_s[min(rk[cur ^ 1][threadIdx.x], rmax)];
        if (!ps.done) blend_batch(sh[cur], n, a + q, px, py, Dm, lthr, amax, tmin, ps);
        if (threadIdx.x < nn) sh[cur ^ 1][threadIdx.x] = stage(nxt);
      }
    }
  }
  if (tc.inside) {
    const int64_t hw = (int64_t)C.W * C.H;
    const int64_t pl = 3 * C.pix_off + (tc.p - C.pix_off);
    float br, bgc, bb;
    if (key != ~0ull) {
      br = mesh_rgb[pl];
      bgc = mesh_rgb[pl + hw];
      bb = mesh_rgb[pl + 2 * hw];
    } else {
      br = S.bg[0];
      bgc = S.bg[1];
      bb = S.bg[2];
    }
    A.image[pl] = __builtin_fmaf(ps.T, br, ps.cr);
    A.image[pl + hw] = __builtin_fmaf(ps.T, bgc, ps.cg);
    A.image[pl + 2 * hw] = __builtin_fmaf(ps.T, bb, ps.cb);
    A.T_ws[tc.p] = ps.T;
    A.nc_ws[tc.p] = ps.nc;
    if (A.T_out) A.T_out[tc.p] = ps.T;
    if (A.nc_out) A.nc_out[tc.p] = ps.nc;
    if (A.nb_out) A.nb_out[tc.p] = ps.nbl;
    if (A.np_out) A.np_out[tc.p] = ps.npro;
  } else {
    ps.npro = 0;
  }
  unsigned long long sp = (unsigned long long)ps.npro, sb = (unsigned long long)ps.nbl;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sp += __shfl_xor(sp, o, 64);
    sb += __shfl_xor(sb, o, 64);
  }
  __syncthreads();
  if (__lane_id() == 0) {
    atomicAdd(&red[0], sp);
    atomicAdd(&red[1], sb);
  }
  __syncthreads();
  // per-tile sums (one plain store each); the stats export adds the tiles up,
  // which keeps thousands of same-address atomics out of the blend
  if (threadIdx.x == 0) {
    A.tile_np[2 * t] = red[0];
    A.tile_np[2 * t + 1] = red[1];
  }
  __syncthreads();  // LDS is reused by the next tile of a persistent group
}

// one workgroup per tile, in the longest-list-first order
template <int BG, int DEPTH, bool SHADE>
__global__ __launch_bounds__(256) void k_blend_fwd(FwdArgs A) {
  __shared__ FwdShared<BG, DEPTH> L;
  blend_tile<BG, DEPTH, SHADE>(A, L, (int)A.tile_order[blockIdx.x]);
}

// persistent workgroups pull tiles from an atomic queue over the same order
template <int BG, int DEPTH, bool SHADE>
__global__ __launch_bounds__(256) void k_blend_fwd_persistent(FwdArgs A, uint32_t* queue) {
  __shared__ FwdShared<BG, DEPTH> L;
  __shared__ uint32_t next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(queue, 1u);
    __syncthreads();
    const uint32_t q = next;
    __syncthreads();
    if (q >= (uint32_t)A.S.n_tiles) break;
    blend_tile<BG, DEPTH, SHADE>(A, L, (int)A.tile_order[q]);
  }
}

// ------------------------------------------------------------- backward --
// Reverse sweep over list positions [0, max n_contrib) of the tile, window by
// window from the last, batch by batch from the back. Each pixel recovers the
// transmittance in front of a Gaussian by dividing by (1 - alpha), starting
// from its stored final T. Per Gaussian and tile, the 9 record gradients (u,
// v, conic a b c, opacity, r g b) are summed over each wave and added once
// per wave.
template <int BG>
__global__ __launch_bounds__(256) void k_blend_bwd(
    SetDev S, const CamDev* __restrict__ cams, const uint32_t* __restrict__ vis_off,
    const uint32_t* __restrict__ mat, const uint32_t* __restrict__ tile_start,
    const uint32_t* __restrict__ tile_total, const uint32_t* __restrict__ tile_order,
    const uint32_t* __restrict__ lists, const GRec* __restrict__ rec_s,
    const unsigned long long* __restrict__ zbuf, const float* __restrict__ mesh_rgb,
    const float* __restrict__ T_ws,
    const int32_t* __restrict__ nc_ws, const float* __restrict__ grad_image,
    const float* __restrict__ grad_T, float* __restrict__ gacc) {
  __shared__ Staged sh[BG];
  __shared__ float4 raw[BG];  // ca, cb, cc, unused
  __shared__ uint32_t rk[BG];
  __shared__ uint32_t bitmap[WIN_WORDS];
  __shared__ uint32_t red4[4];
  __shared__ int maxnc;
  const int t = (int)tile_order[blockIdx.x];
  const TileCtx tc = tile_ctx(cams, S.n_cams, t);
  const CamDev& C = cams[tc.cam];
  const WinCtx W = win_ctx(C, tc.cam, t, vis_off, mat, tile_start, tile_total, S.key_cap);
  const float px = (float)tc.i + 0.5f, py = (float)tc.j + 0.5f;
  const float lthr = __log2f(S.alpha_min), amax = S.alpha_max;
  const uint32_t rmax = (uint32_t)((int64_t)S.n * S.n_cams - 1);
  float gr = 0.f, gg = 0.f, gb = 0.f, gT = 0.f, Tf = 1.f;
  int nc = 0;
  if (threadIdx.x == 0) maxnc = 0;
  if (tc.inside) {
    const int64_t hw = (int64_t)C.W * C.H;
    const int64_t pl = 3 * C.pix_off + (tc.p - C.pix_off);
    gr = grad_image[pl];
    gg = grad_image[pl + hw];
    gb = grad_image[pl + 2 * hw];
    Tf = T_ws[tc.p];
    nc = nc_ws[tc.p];
    float br, bgc, bb;
    if (zbuf[tc.p] != ~0ull) {
      br = mesh_rgb[pl];
      bgc = mesh_rgb[pl + hw];
      bb = mesh_rgb[pl + 2 * hw];
    } else {
      br = S.bg[0];
      bgc = S.bg[1];
      bb = S.bg[2];
    }
    // I_h = C + T (I_m or bg): T receives the background's colour gradient
    gT = (grad_T ? grad_T[tc.p] : 0.f) + gr * br + gg * bgc + gb * bb;
  }
  __syncthreads();
  if (nc > 0) atomicMax(&maxnc, nc);
  __syncthreads();
  const int64_t last = maxnc;
  if (last == 0) return;
  float T = Tf, Sr = 0.f, Sg = 0.f, Sb = 0.f;
  const int lane = __lane_id();
  for (int w = W.nwin - 1; w >= 0; --w) {
    int64_t a, b;
    win_range(W, w, a, b);
    if (a >= b || a >= last) continue;
    const uint32_t wbase = W.rbase + (uint32_t)w * WIN;
    __syncthreads();
    bitmap[threadIdx.x] = 0;
    __syncthreads();
    win_mark(lists, W, a, b, wbase, bitmap);
    __syncthreads();
    const uint32_t word = bitmap[threadIdx.x];
    uint32_t total;
    const uint32_t pre = group_excl_scan((uint32_t)__popc(word), red4, total);
    const int64_t nproc = (last < a + (int64_t)total ? last : a + (int64_t)total) - a;
    for (int64_t hi = nproc; hi > 0; hi -= BG) {
      const int64_t lo = hi - BG > 0 ? hi - BG : 0;
      const int n = (int)(hi - lo);
      __syncthreads();
      win_extract(word, pre, (uint32_t)lo, (uint32_t)n, wbase, rk);
      __syncthreads();
      if (threadIdx.x < n) {
        const uint32_t r = min(rk[threadIdx.x], rmax);
        const GRec R = rec_s[r];
        sh[threadIdx.x] = stage(R);
        raw[threadIdx.x] = make_float4(R.ca, R.cb, R.cc, 0.f);
        rk[threadIdx.x] = r;
      }
      __syncthreads();
      for (int k = n - 1; k >= 0; --k) {
        const int64_t idx = a + lo + k + 1;  // 1-based list position
        float g[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) g[q] = 0.f;
        bool contrib = idx <= nc;
        const float4 sa = sh[k].a, sb = sh[k].b;
        if (contrib) {
          float dx, dy;
          const float p2 = gauss_p2(sa, sb, px, py, dx, dy);
          contrib = p2 >= lthr;  // the forward's skip decision
          const float ag = __builtin_amdgcn_exp2f(p2);  // opacity * G
          const float alpha = fminf(amax, ag);
          if (contrib) {
            const float4 c = sh[k].c;
            // transmittance in front of this Gaussian (v_rcp: 1 ulp, against
            // the ~10 instructions of a correctly rounded division)
            const float inv = __builtin_amdgcn_rcpf(1.f - alpha);
            T = T * inv;
            const float wgt = alpha * T;
            g[6] = wgt * gr;
            g[7] = wgt * gg;
            g[8] = wgt * gb;
            const float galpha = T * ((c.x - Sr) * gr + (c.y - Sg) * gg + (c.z - Sb) * gb) -
                                 gT * Tf * inv;
            Sr = alpha * c.x + (1.f - alpha) * Sr;
            Sg = alpha * c.y + (1.f - alpha) * Sg;
            Sb = alpha * c.z + (1.f - alpha) * Sb;
            if (ag < amax) {
              g[5] = galpha * ag * __builtin_amdgcn_rcpf(sb.w);  // d alpha / d opacity = G
              // power = -1/2 (ca dx^2 + cc dy^2) - cb dx dy with dx = u - px
              const float gp = galpha * ag;
              const float4 rw = raw[k];
              g[0] = -gp * (rw.x * dx + rw.y * dy);
              g[1] = -gp * (rw.z * dy + rw.y * dx);
              g[2] = -0.5f * gp * dx * dx;
              g[3] = -gp * dx * dy;
              g[4] = -0.5f * gp * dy * dy;
            }
          }
        }
        if (__ballot(contrib)) {
#pragma unroll
          for (int q = 0; q < 9; ++q) g[q] = wave_sum_to_last(g[q]);
          if (lane == 63) {
            float* dst = gacc + (size_t)rk[k] * 9;
#pragma unroll
            for (int q = 0; q < 9; ++q) atomicAdd(dst + q, g[q]);
          }
        }
      }
    }
  }
}


// ------------------------------------------------- one wave per tile --
// A 64-lane workgroup per 16x16 tile; lane l owns the column l % 16 and the
// four rows 4 (l / 16) .. 4 (l / 16) + 3. Each staged record read from LDS
// then serves four pixels, the window bitmap is owned four words per lane,
// and one wave-wide reduction per Gaussian in the backward covers 256
// pixels. The per-pixel arithmetic is that of the 256-thread kernels, in the
// same order, so images are bit-identical.
constexpr int WPIX = 4;

// bitmap words 4 l .. 4 l + 3 of this lane: counts and exclusive prefix
struct WinWords {
  uint32_t w[WPIX];
  uint32_t pre, total;
};

__device__ __forceinline__ WinWords wave_words(const uint32_t* bitmap) {
  WinWords ww;
  const int l = threadIdx.x;
  uint32_t cnt = 0;
#pragma unroll
  for (int q = 0; q < WPIX; ++q) {
    ww.w[q] = bitmap[WPIX * l + q];
    cnt += __popc(ww.w[q]);
  }
  uint32_t inc = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(inc, o, 64);
    if (l >= o) inc += u;
  }
  ww.total = __shfl(inc, 63, 64);
  ww.pre = inc - cnt;
  return ww;
}

// ranks of the window-ordered entries [q, q + n) into rk
__device__ __forceinline__ void wave_extract(const WinWords& ww, uint32_t q, uint32_t n,
                                             uint32_t wbase, uint32_t* rk) {
  uint32_t idx = ww.pre;
#pragma unroll
  for (int h = 0; h < WPIX; ++h) {
    uint32_t wv = ww.w[h];
    const uint32_t cnt = __popc(wv);
    if (idx + cnt > q && idx < q + n) {
      const uint32_t bit0 = wbase + 32u * (WPIX * threadIdx.x + h);
      uint32_t k = idx;
      while (wv) {
        const uint32_t b = __ffs(wv) - 1;
        wv &= wv - 1;
        if (k >= q && k < q + n) rk[k - q] = bit0 + b;
        ++k;
      }
    }
    idx += cnt;
  }
}

template <int BG, bool SHADE>
__global__ __launch_bounds__(64) void k_blend_fwd_w(FwdArgs A) {
  __shared__ Staged sh[BG];
  __shared__ uint32_t rk[BG];
  __shared__ uint32_t bitmap[WIN_WORDS];
  const SetDev& S = A.S;
  const int t = (int)A.tile_order[blockIdx.x];
  const int cam = find_cam_by_tile(A.cams, S.n_cams, t);
  const CamDev& C = A.cams[cam];
  const int lt = t - C.tile_off;
  const int ty = lt / C.TX, tx = lt - (lt / C.TX) * C.TX;
  const int lane = threadIdx.x;
  const int i = tx * TILE + (lane & 15);
  const int j0 = ty * TILE + WPIX * (lane >> 4);
  const WinCtx W = win_ctx(C, cam, t, A.vis_off, A.mat, A.tile_start, A.tile_total, S.key_cap);
  const float px = (float)i + 0.5f;
  const float lthr = __log2f(S.alpha_min), amax = S.alpha_max, tmin = S.t_min;
  const uint32_t rmax = (uint32_t)((int64_t)S.n * S.n_cams - 1);
  float T[WPIX], cr[WPIX], cg[WPIX], cb[WPIX], Dm[WPIX], py[WPIX];
  int nc[WPIX], nbl[WPIX], npro[WPIX];
  bool done[WPIX];
  unsigned long long key[WPIX];
#pragma unroll
  for (int r = 0; r < WPIX; ++r) {
    const int j = j0 + r;
    const bool inside = i < C.W && j < C.H;
    key[r] = inside ? A.zbuf[C.pix_off + (int64_t)j * C.W + i] : ~0ull;
    if (SHADE && inside) {  // the mesh shading first, as in blend_tile
      float rgb[3];
      mesh_shade(S, C, i, j, C.pix_off + (int64_t)j * C.W + i, key[r], A.tris, A.tex, A.mo, rgb);
    }
    Dm[r] = key[r] == ~0ull ? __int_as_float(0x7f800000) : __uint_as_float((uint32_t)(key[r] >> 32));
    py[r] = (float)j + 0.5f;
    T[r] = 1.f;
    cr[r] = cg[r] = cb[r] = 0.f;
    nc[r] = nbl[r] = 0;
    npro[r] = (int)W.lim;
    done[r] = !inside;
  }
  auto lane_done = [&]() { return done[0] && done[1] && done[2] && done[3]; };
  bool all_done = false;
  for (int w = 0; w < W.nwin && !all_done; ++w) {
    int64_t a, b;
    win_range(W, w, a, b);
    if (a >= b) continue;
    if (__all(lane_done())) break;
    const uint32_t wbase = W.rbase + (uint32_t)w * WIN;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < WPIX; ++q) bitmap[WPIX * lane + q] = 0;
    __syncthreads();
    win_mark(A.lists, W, a, b, wbase, bitmap);
    __syncthreads();
    const WinWords ww = wave_words(bitmap);
    const int nbat = (int)((ww.total + BG - 1) / BG);
    for (int bi = 0; bi < nbat; ++bi) {
      const uint32_t q = (uint32_t)bi * BG;
      const int n = (int)min((uint32_t)BG, ww.total - q);
      if (bi > 0 && __all(lane_done())) {
        all_done = true;
        break;
      }
      __syncthreads();
      wave_extract(ww, q, (uint32_t)n, wbase, rk);
      __syncthreads();
      for (int s2 = lane; s2 < n; s2 += 64) sh[s2] = stage(A.rec_s[min(rk[s2], rmax)]);
      __syncthreads();
      const int pos0 = (int)(a + q) + 1;
      const Staged* e = sh;
      for (int k = 0; k < n; ++k, ++e) {
        if (lane_done()) continue;
        const float4 ea = e->a, eb = e->b, c = e->c;
        const float dx = ea.x - px;
        const float adx = ea.z * dx;  // the factored form of gauss_p2, A2 dx shared
        const int pos = pos0 + k;
        // the four pixels without branches: every step is computed and the
        // selects keep what a pixel that is done, skips or stops must keep
        // (a zero weight leaves the non-negative colour sums unchanged)
#pragma unroll
        for (int r = 0; r < WPIX; ++r) {
          const bool front = eb.z < Dm[r];  // at or behind the mesh the pixel ends (Sec. 3.4)
          const float dy = ea.y - py[r];
          const float p2 = __builtin_fmaf(dx, __builtin_fmaf(ea.w, dy, adx),
                                          __builtin_fmaf(eb.x * dy, dy, eb.y));
          const float alpha = fminf(amax, __builtin_amdgcn_exp2f(p2));
          const float Tn = T[r] * (1.f - alpha);
          const bool hit = !done[r] && front && p2 >= lthr;
          const bool tstop = hit && Tn < tmin;
          const bool blend = hit && !(Tn < tmin);
          const bool ends = (!done[r] && !front) || tstop;
          const float wgt = blend ? alpha * T[r] : 0.f;
          cr[r] = __builtin_fmaf(c.x, wgt, cr[r]);
          cg[r] = __builtin_fmaf(c.y, wgt, cg[r]);
          cb[r] = __builtin_fmaf(c.z, wgt, cb[r]);
          T[r] = blend ? Tn : T[r];
          nc[r] = blend ? pos : nc[r];
          nbl[r] += blend ? 1 : 0;
          npro[r] = ends ? pos : npro[r];
          done[r] = done[r] || ends;
        }
      }
    }
  }
  unsigned long long sp = 0, sb = 0;
  const int64_t hw = (int64_t)C.W * C.H;
#pragma unroll
  for (int r = 0; r < WPIX; ++r) {
    const int j = j0 + r;
    if (!(i < C.W && j < C.H)) continue;
    const int64_t p = C.pix_off + (int64_t)j * C.W + i;
    const int64_t pl = 3 * C.pix_off + (p - C.pix_off);
    float br, bgc, bb;
    if (key[r] != ~0ull) {
      br = A.mesh_rgb[pl];
      bgc = A.mesh_rgb[pl + hw];
      bb = A.mesh_rgb[pl + 2 * hw];
    } else {
      br = S.bg[0];
      bgc = S.bg[1];
      bb = S.bg[2];
    }
    A.image[pl] = __builtin_fmaf(T[r], br, cr[r]);
    A.image[pl + hw] = __builtin_fmaf(T[r], bgc, cg[r]);
    A.image[pl + 2 * hw] = __builtin_fmaf(T[r], bb, cb[r]);
    A.T_ws[p] = T[r];
    A.nc_ws[p] = nc[r];
    if (A.T_out) A.T_out[p] = T[r];
    if (A.nc_out) A.nc_out[p] = nc[r];
    if (A.nb_out) A.nb_out[p] = nbl[r];
    if (A.np_out) A.np_out[p] = npro[r];
    sp += (unsigned long long)npro[r];
    sb += (unsigned long long)nbl[r];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sp += __shfl_xor(sp, o, 64);
    sb += __shfl_xor(sb, o, 64);
  }
  if (lane == 0) {
    A.tile_np[2 * t] = sp;
    A.tile_np[2 * t + 1] = sb;
  }
}

constexpr int RB = 2;  // Gaussians whose gradients the one-wave backward sums together

template <int BG>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_blend_bwd_w(
    SetDev S, const CamDev* __restrict__ cams, const uint32_t* __restrict__ vis_off,
    const uint32_t* __restrict__ mat, const uint32_t* __restrict__ tile_start,
    const uint32_t* __restrict__ tile_total, const uint32_t* __restrict__ tile_order,
    const uint32_t* __restrict__ lists, const GRec* __restrict__ rec_s,
    const unsigned long long* __restrict__ zbuf, const float* __restrict__ mesh_rgb,
    const float* __restrict__ T_ws, const int32_t* __restrict__ nc_ws,
    const float* __restrict__ grad_image, const float* __restrict__ grad_T,
    float* __restrict__ gacc) {
  __shared__ Staged sh[BG];
  __shared__ uint32_t rk[BG];
  __shared__ uint32_t bitmap[WIN_WORDS];
  // the 9 record gradients of up to RBL Gaussians, one row of 64 lane partials
  // each (padded: the summing lanes read across the banks)
  // at batch 32 the staged records leave room for 3 Gaussians' rows in the
  // LDS that keeps 4 waves per SIMD
  constexpr int RBL = BG <= 32 ? 3 : RB;
  __shared__ float part[RBL][9][65];
  __shared__ uint32_t prk[RBL];
  const int t = (int)tile_order[blockIdx.x];
  const int cam = find_cam_by_tile(cams, S.n_cams, t);
  const CamDev& C = cams[cam];
  const int lt = t - C.tile_off;
  const int ty = lt / C.TX, tx = lt - (lt / C.TX) * C.TX;
  const int lane = threadIdx.x;
  const int i = tx * TILE + (lane & 15);
  const int j0 = ty * TILE + WPIX * (lane >> 4);
  const WinCtx W = win_ctx(C, cam, t, vis_off, mat, tile_start, tile_total, S.key_cap);
  const float px = (float)i + 0.5f;
  const float lthr = __log2f(S.alpha_min), amax = S.alpha_max;
  const uint32_t rmax = (uint32_t)((int64_t)S.n * S.n_cams - 1);
  const int64_t hw = (int64_t)C.W * C.H;
  // U: the colour of the Gaussians behind, dotted with the pixel's colour
  // gradient (the one scalar of it the alpha gradient needs)
  float gr[WPIX], gg[WPIX], gb[WPIX], gT[WPIX], Tf[WPIX], T[WPIX], U[WPIX], py[WPIX], gTf[WPIX];
  int nc[WPIX];
  int lmax = 0;
#pragma unroll
  for (int r = 0; r < WPIX; ++r) {
    const int j = j0 + r;
    py[r] = (float)j + 0.5f;
    gr[r] = gg[r] = gb[r] = gT[r] = 0.f;
    Tf[r] = 1.f;
    nc[r] = 0;
    if (i < C.W && j < C.H) {
      const int64_t p = C.pix_off + (int64_t)j * C.W + i;
      const int64_t pl = 3 * C.pix_off + (p - C.pix_off);
      gr[r] = grad_image[pl];
      gg[r] = grad_image[pl + hw];
      gb[r] = grad_image[pl + 2 * hw];
      Tf[r] = T_ws[p];
      nc[r] = nc_ws[p];
      float br, bgc, bb;
      if (zbuf[p] != ~0ull) {
        br = mesh_rgb[pl];
        bgc = mesh_rgb[pl + hw];
        bb = mesh_rgb[pl + 2 * hw];
      } else {
        br = S.bg[0];
        bgc = S.bg[1];
        bb = S.bg[2];
      }
      // I_h = C + T (I_m or bg): T receives the background's colour gradient
      gT[r] = (grad_T ? grad_T[p] : 0.f) + gr[r] * br + gg[r] * bgc + gb[r] * bb;
    }
    T[r] = Tf[r];
    gTf[r] = gT[r] * Tf[r];
    U[r] = 0.f;
    lmax = max(lmax, nc[r]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) lmax = max(lmax, __shfl_xor(lmax, o, 64));
  const int64_t last = lmax;
  if (last == 0) return;
  // RBL Gaussians' partials are summed together: row r = 9 gs + q of part
  // holds gradient q of Gaussian gs over the 64 lanes; lanes r and r + 32
  // sum its entries [0, 32) and [32, 64), lane r adds the two and the result
  // to the Gaussian's accumulators (one atomic instruction for all rows)
  static_assert(9 * RBL <= 32, "two lanes per row");
  int nb = 0;
  auto flush = [&]() {
    __syncthreads();
    const int r = lane & 31;
    float v = 0.f;
    if (r < 9 * nb) {
      const float* row = &part[0][0][0] + r * 65 + (lane & 32);
#pragma unroll 4
      for (int k = 0; k < 32; k += 2) v += row[k] + row[k + 1];
    }
    v += __shfl_down(v, 32, 64);
    if (lane < 9 * nb) {
      const int gs = lane / 9, q = lane - 9 * gs;
      atomicAdd(gacc + (size_t)prk[gs] * 9 + q, v);
    }
    __syncthreads();
  };
  for (int w = W.nwin - 1; w >= 0; --w) {
    int64_t a, b;
    win_range(W, w, a, b);
    if (a >= b || a >= last) continue;
    const uint32_t wbase = W.rbase + (uint32_t)w * WIN;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < WPIX; ++q) bitmap[WPIX * lane + q] = 0;
    __syncthreads();
    win_mark(lists, W, a, b, wbase, bitmap);
    __syncthreads();
    const WinWords ww = wave_words(bitmap);
    const int64_t nproc = (last < a + (int64_t)ww.total ? last : a + (int64_t)ww.total) - a;
    for (int64_t hi = nproc; hi > 0; hi -= BG) {
      const int64_t lo = hi - BG > 0 ? hi - BG : 0;
      const int n = (int)(hi - lo);
      __syncthreads();
      wave_extract(ww, (uint32_t)lo, (uint32_t)n, wbase, rk);
      __syncthreads();
      for (int s2 = lane; s2 < n; s2 += 64) {
        const uint32_t r = min(rk[s2], rmax);
        sh[s2] = stage(rec_s[r]);
        rk[s2] = r;
      }
      __syncthreads();
      for (int k = n - 1; k >= 0; --k) {
        const int idx = (int)(a + lo + k + 1);  // 1-based list position
        const float4 ea = sh[k].a, eb = sh[k].b;
        const float dx = ea.x - px;
        const float dxx = dx * dx;
        const float adx = ea.z * dx;  // the factored form of gauss_p2, A2 dx shared
        const float iop = __builtin_amdgcn_rcpf(eb.w);
        // per lane, over its four pixels: colour gradients, and the sums
        // s0 = sum gp, s1 = sum gp dy, s2 = sum gp dy^2 (gp = dL/dpower),
        // from which the mean, conic and opacity gradients follow since dx
        // is common to the lane's pixels
        float gc0 = 0.f, gc1 = 0.f, gc2 = 0.f, s0 = 0.f, s1 = 0.f, s2 = 0.f;
        bool any = false;
        const float4 c = sh[k].c;
#pragma unroll
        for (int r = 0; r < WPIX; ++r) {
          // every pixel slot runs the same instructions; one that does not
          // blend this Gaussian (past its last contributor, or skipped by the
          // forward's alpha test) takes alpha = 0, which leaves T and S as
          // they are and adds nothing
          const float dy = ea.y - py[r];
          const float p2 = __builtin_fmaf(dx, __builtin_fmaf(ea.w, dy, adx),
                                          __builtin_fmaf(eb.x * dy, dy, eb.y));
          const bool act = idx <= nc[r] && p2 >= lthr;  // the forward's decisions
          any = any || act;
          const float ag = act ? __builtin_amdgcn_exp2f(p2) : 0.f;  // opacity * G
          const float alpha = fminf(amax, ag);
          // transmittance in front of this Gaussian (v_rcp, 1 ulp)
          const float inv = __builtin_amdgcn_rcpf(1.f - alpha);
          T[r] = T[r] * inv;
          const float wgt = alpha * T[r];
          gc0 = __builtin_fmaf(wgt, gr[r], gc0);
          gc1 = __builtin_fmaf(wgt, gg[r], gc1);
          gc2 = __builtin_fmaf(wgt, gb[r], gc2);
          // (c - S) . g with S the colour behind, S <- S + alpha (c - S)
          const float du =
              __builtin_fmaf(c.x, gr[r], __builtin_fmaf(c.y, gg[r], c.z * gb[r])) - U[r];
          const float galpha = __builtin_fmaf(T[r], du, -gTf[r] * inv);
          U[r] = __builtin_fmaf(alpha, du, U[r]);
          // d alpha / d power = alpha' (0 where clamped at alpha_max)
          const float gp = ag < amax ? galpha * ag : 0.f;
          const float gpdy = gp * dy;
          s0 += gp;
          s1 += gpdy;
          s2 = __builtin_fmaf(gpdy, dy, s2);
        }
        if (__any(any)) {
          // power = -1/2 (ca dx^2 + cc dy^2) - cb dx dy, dx = u - px; the
          // staged exponent holds A2 = -ca log2e / 2, B2 = -cb log2e,
          // C2 = -cc log2e / 2; d alpha / d opacity = G = gp / (alpha' opacity)
          float g[9];
          g[0] = LN2F * (2.f * ea.z * dx * s0 + ea.w * s1);
          g[1] = LN2F * (2.f * eb.x * s1 + ea.w * dx * s0);
          g[2] = -0.5f * dxx * s0;
          g[3] = -dx * s1;
          g[4] = -0.5f * s2;
          g[5] = s0 * iop;
          g[6] = gc0;
          g[7] = gc1;
          g[8] = gc2;
#pragma unroll
          for (int q = 0; q < 9; ++q) part[nb][q][lane] = g[q];
          if (lane == 0) prk[nb] = rk[k];
          if (++nb == RBL) {
            flush();
            nb = 0;
          }
        }
      }
    }
  }
  if (nb) flush();
}

}  // namespace

template <int BG, int D, bool SH>
void launch_fwd(const FwdArgs& A, bool persistent, uint32_t* queue, hipStream_t st) {
  if (!persistent) {
    hipLaunchKernelGGL((k_blend_fwd<BG, D, SH>), dim3(A.S.n_tiles), dim3(256), 0, st, A);
    return;
  }
  static int grid = 0;
  if (grid == 0) {
    int dev = 0, cus = 0, per = 0;
    // a failed query leaves the fallback of one group per CU of a 256-CU chip
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_blend_fwd_persistent<BG, D, SH>, 256,
                                                     0) != hipSuccess)
      per = 0;
    grid = (cus > 0 ? cus : 256) * (per > 0 ? per : 1);
  }
  launch_fill_u32(queue, 0u, 1, st);
  hipLaunchKernelGGL((k_blend_fwd_persistent<BG, D, SH>), dim3(grid), dim3(256), 0, st, A, queue);
}

template <bool SH>
void launch_variant(const FwdArgs& A, int batch, int variant, uint32_t* queue, hipStream_t st) {
  const bool d2 = (variant & 1) != 0, pers = (variant & 2) != 0;
  if (variant & 4) {
    if (batch >= 128)
      hipLaunchKernelGGL((k_blend_fwd_w<128, SH>), dim3(A.S.n_tiles), dim3(64), 0, st, A);
    else
      hipLaunchKernelGGL((k_blend_fwd_w<64, SH>), dim3(A.S.n_tiles), dim3(64), 0, st, A);
    return;
  }
  switch (batch) {
    case 32:
      d2 ? launch_fwd<32, 2, SH>(A, pers, queue, st) : launch_fwd<32, 1, SH>(A, pers, queue, st);
      break;
    case 64:
      d2 ? launch_fwd<64, 2, SH>(A, pers, queue, st) : launch_fwd<64, 1, SH>(A, pers, queue, st);
      break;
    case 128:
      d2 ? launch_fwd<128, 2, SH>(A, pers, queue, st) : launch_fwd<128, 1, SH>(A, pers, queue, st);
      break;
    default:
      d2 ? launch_fwd<256, 2, SH>(A, pers, queue, st) : launch_fwd<256, 1, SH>(A, pers, queue, st);
      break;
  }
}

// variant bit 0: two-deep staging; bit 1: persistent workgroups on a tile
// queue; bit 2: one wave per tile. With tex_shade set the blend also shades
// the mesh pixels (their z-buffer is complete); otherwise it reads the mesh
// colour an earlier shading left in the workspace.
void launch_blend_forward(const SetDev& S, const Work& w, hr_outputs* out, int batch, int variant,
                          hipStream_t st, bool shade, const float* tex) {
  if (S.n_tiles == 0) return;
  FwdArgs A{S, w.cams, w.vis_off, w.mat, w.tile_start, w.tile_total, w.tile_order, w.lists,
            w.rec_s, (const unsigned long long*)w.zbuf, w.mesh_rgb, out->image, w.final_T,
            w.n_contrib, out->final_T, out->n_contrib, out->n_blended, out->n_processed,
            (unsigned long long*)w.tile_np, w.tris, tex,
            MeshOut{w.mesh_rgb, w.taps, out->mesh_rgb, out->mesh_depth, out->tri_id}};
  uint32_t* queue = w.counters + 14;
  if (shade)
    launch_variant<true>(A, batch, variant, queue, st);
  else
    launch_variant<false>(A, batch, variant, queue, st);
}

#define HR_BWD(BG)                                                                              \
  hipLaunchKernelGGL((k_blend_bwd<BG>), dim3(S.n_tiles), dim3(256), 0, st, S, w.cams,           \
                     w.vis_off, w.mat, w.tile_start, w.tile_total, w.tile_order, w.lists,       \
                     w.rec_s, (const unsigned long long*)w.zbuf, w.mesh_rgb, w.final_T,         \
                     w.n_contrib,                                                               \
                     grad_image, grad_T, w.gacc)

#define HR_BWD_W(BG)                                                                            \
  hipLaunchKernelGGL((k_blend_bwd_w<BG>), dim3(S.n_tiles), dim3(64), 0, st, S, w.cams,          \
                     w.vis_off, w.mat, w.tile_start, w.tile_total, w.tile_order, w.lists,       \
                     w.rec_s, (const unsigned long long*)w.zbuf, w.mesh_rgb, w.final_T,         \
                     w.n_contrib, grad_image, grad_T, w.gacc)

void launch_blend_backward(const SetDev& S, const Work& w, const float* grad_image,
                           const float* grad_T, int batch, int variant, hipStream_t st) {
  if (S.n_tiles == 0) return;
  if (variant & 8) {
    if (batch >= 128) HR_BWD_W(128);
    else if (batch >= 64) HR_BWD_W(64);
    else HR_BWD_W(32);
    return;
  }
  switch (batch) {
    case 32: HR_BWD(32); break;
    case 64: HR_BWD(64); break;
    case 128: HR_BWD(128); break;
    default: HR_BWD(256); break;
  }
}

}  // namespace hr
