// Rank windows of a tile's list (device helpers shared by the blend kernels
// and the key export).
//
// After binning, the list of a tile is a sequence of chunk sub-segments in
// chunk order; chunk c holds the Gaussians of depth ranks [c*CHUNK,
// (c+1)*CHUNK) of its camera, in no particular order inside the sub-segment.
// A window is WIN_ROWS consecutive chunks, i.e. WIN consecutive ranks, so the
// entries of window w are contiguous in the list, and their depth order is
// recovered exactly by setting one bit per rank in a WIN-bit LDS bitmap and
// reading the set bits in increasing order (each rank appears at most once).
// A kernel only orders the windows it actually reaches.
#pragma once

#include "common.hpp"

namespace hr {

constexpr int WIN_ROWS = 4;               // chunks per window
constexpr int WIN = WIN_ROWS * CHUNK;     // ranks per window
constexpr int WIN_WORDS = WIN / 32;       // bitmap words, one per thread of a 256-wide group
static_assert(WIN_WORDS == 256, "one bitmap word per thread");

struct WinCtx {
  int64_t s;            // list start of the tile
  int64_t lim;          // entries available to the tile (capacity clamp)
  uint32_t rbase;       // first depth rank of the tile's camera
  int rows;             // chunk rows used by the camera
  int nwin;             // windows of the camera
  int ntl;              // tiles of the camera (matrix row stride)
  const uint32_t* col;  // column of this tile in the camera's chunk matrix
};

__device__ __forceinline__ WinCtx win_ctx(const CamDev& cam, int cam_idx, int tile,
                                          const uint32_t* vis_off, const uint32_t* mat,
                                          const uint32_t* tile_start, const uint32_t* tile_total,
                                          int64_t key_cap) {
  WinCtx W;
  W.s = tile_start[tile];
  const int64_t e = W.s + tile_total[tile];
  W.lim = (e < key_cap ? e : key_cap) - W.s;
  if (W.lim < 0) W.lim = 0;
  W.rbase = vis_off[cam_idx];
  const int64_t nvc = (int64_t)vis_off[cam_idx + 1] - W.rbase;
  W.rows = (int)((nvc + CHUNK - 1) / CHUNK);
  W.nwin = (W.rows + WIN_ROWS - 1) / WIN_ROWS;
  W.ntl = cam.TX * cam.TY;
  W.col = mat + cam.mat_off + (tile - cam.tile_off);
  return W;
}

// List positions [a, b), relative to the tile start, of window w. After the
// scatter, the matrix entry of (row, tile) holds the end of that row's
// sub-segment.
__device__ __forceinline__ void win_range(const WinCtx& W, int w, int64_t& a, int64_t& b) {
  const int r0 = w * WIN_ROWS;
  const int r1 = r0 + WIN_ROWS < W.rows ? r0 + WIN_ROWS : W.rows;
  a = r0 == 0 ? 0 : (int64_t)W.col[(int64_t)(r0 - 1) * W.ntl];
  b = (int64_t)W.col[(int64_t)(r1 - 1) * W.ntl];
  if (b > W.lim) b = W.lim;
  if (a > b) a = b;
}

// set the bit of every rank in list entries [a, b) (relative to the window's first rank)
__device__ __forceinline__ void win_mark(const uint32_t* __restrict__ lists, const WinCtx& W,
                                         int64_t a, int64_t b, uint32_t wbase, uint32_t* bitmap) {
  for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) {
    const uint32_t rel = lists[W.s + i] - wbase;
    if (rel < (uint32_t)WIN) atomicOr(&bitmap[rel >> 5], 1u << (rel & 31u));
  }
}

// exclusive scan of one value per thread over a 256-thread group
__device__ __forceinline__ uint32_t group_excl_scan(uint32_t v, uint32_t* lds4, uint32_t& total) {
  const int w = threadIdx.x >> 6, l = __lane_id();
  uint32_t inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(inc, o, 64);
    if (l >= o) inc += u;
  }
  if (l == 63) lds4[w] = inc;
  __syncthreads();
  uint32_t base = 0;
  total = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t s = lds4[k];
    if (k < w) base += s;
    total += s;
  }
  __syncthreads();
  return base + inc - v;
}

// Ranks of the window-ordered entries [q, q + n): the thread owning bitmap
// word `word` (whose first entry has order index `pre`) writes its part.
__device__ __forceinline__ void win_extract(uint32_t word, uint32_t pre, uint32_t q, uint32_t n,
                                            uint32_t wbase, uint32_t* rk) {
  const uint32_t cnt = __popc(word);
  if (pre >= q + n || pre + cnt <= q) return;
  uint32_t idx = pre;
  uint32_t wv = word;
  const uint32_t bit0 = wbase + 32u * threadIdx.x;
  while (wv) {
    const uint32_t b = __ffs(wv) - 1;
    wv &= wv - 1;
    if (idx >= q) rk[idx - q] = bit0 + b;
    ++idx;
    if (idx >= q + n) break;
  }
}

}  // namespace hr
