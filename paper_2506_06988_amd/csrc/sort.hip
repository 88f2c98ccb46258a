// Depth ordering and tile binning (the "tile-wise sorting" of Sec. 1).
//
// Instead of radix-sorting one 64-bit (tile | depth) key per (tile, Gaussian)
// pair, the pairs are produced already grouped by tile and in depth order:
//  1. the visible (camera, Gaussian) items are radix-sorted once by
//     (camera, fp32 depth bits); stability keeps equal depths in index order,
//     so an item's position (its rank) orders it by (depth, index);
//  2. ranks are cut into chunks of CHUNK; a workgroup per chunk histograms
//     its pairs per tile in LDS; a column scan turns the chunk x tile counts
//     into each (chunk, tile) output offset and per-tile ranges;
//  3. a second pass scatters each pair's rank into its tile's segment; within
//     one (chunk, tile) sub-segment the order is that of LDS atomics;
//  4. a workgroup per tile sorts its segment by rank in LDS, in windows of
//     whole chunk groups (each window holds at most SORT_WIN ranks).
// The result equals sorting all (tile, depth bits, index) triples, and the
// key traffic is two writes and two reads of a 4-byte rank per pair.
#include "kernels.hpp"

namespace hr {
namespace {

constexpr int RS_B = 256;             // radix-sort threads per block
constexpr int RS_ROUNDS = 8;          // striped rounds per block
constexpr int RS_KPB = RS_B * RS_ROUNDS;

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = __lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// lanes of this wave holding the same 8-bit digit (among `valid` lanes)
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bal = __ballot(valid && bit);
    m &= bit ? bal : ~bal;
  }
  return valid ? m : 0ull;
}

__global__ void k_vis_offsets(const uint32_t* __restrict__ vis_scan, const uint32_t* __restrict__ vis,
                              int n, int n_cams, uint32_t* __restrict__ vis_off,
                              uint32_t* __restrict__ counters) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > n_cams) return;
  const int64_t M = (int64_t)n * n_cams;
  uint32_t v;
  if (c < n_cams) {
    v = n > 0 ? vis_scan[(int64_t)c * n] : 0u;
  } else {
    v = M > 0 ? vis_scan[M - 1] + vis[M - 1] : 0u;
    counters[0] = v;
  }
  vis_off[c] = v;
}

__global__ __launch_bounds__(256) void k_compact(const uint32_t* __restrict__ vis,
                                                 const uint32_t* __restrict__ vis_scan,
                                                 const uint32_t* __restrict__ dkey, int64_t M,
                                                 uint32_t* __restrict__ skey,
                                                 uint32_t* __restrict__ sval) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M || !vis[i]) return;
  const uint32_t p = vis_scan[i];
  skey[p] = dkey[i];
  sval[p] = (uint32_t)i;
}

__device__ __forceinline__ uint32_t rs_digit(uint32_t key, uint32_t val, int pass, int n) {
  if (pass < 4) return (key >> (8 * pass)) & 255u;
  const uint32_t cam = val / (uint32_t)n;
  return (cam >> (8 * (pass - 4))) & 255u;
}

__global__ __launch_bounds__(RS_B) void k_rs_hist(const uint32_t* __restrict__ key,
                                                  const uint32_t* __restrict__ val,
                                                  const uint32_t* __restrict__ counters, int pass,
                                                  int n, int64_t nb, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t nv = counters[0];
  const int64_t base = (int64_t)blockIdx.x * RS_KPB;
  for (int k = 0; k < RS_ROUNDS; ++k) {
    const int64_t i = base + k * RS_B + threadIdx.x;
    if (i < nv) atomicAdd(&h[rs_digit(key[i], val[i], pass, n)], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// stable scatter: keys keep their input order within a digit
__global__ __launch_bounds__(RS_B) void k_rs_scatter(const uint32_t* __restrict__ key,
                                                     const uint32_t* __restrict__ val,
                                                     uint32_t* __restrict__ key_out,
                                                     uint32_t* __restrict__ val_out,
                                                     const uint32_t* __restrict__ counters,
                                                     int pass, int n, int64_t nb,
                                                     const uint32_t* __restrict__ hist) {
  __shared__ uint32_t off[256];
  __shared__ uint32_t wcnt[RS_B / 64][256];
  const int tid = threadIdx.x, w = tid >> 6;
  off[tid] = hist[(int64_t)tid * nb + blockIdx.x];
  for (int k = 0; k < RS_B / 64; ++k) wcnt[k][tid] = 0;
  __syncthreads();
  const uint32_t nv = counters[0];
  const int64_t base = (int64_t)blockIdx.x * RS_KPB;
  if (base >= nv) return;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = base + r * RS_B + tid;
    const bool valid = i < nv;
    uint32_t kk = 0, vv = 0, d = 0;
    if (valid) {
      kk = key[i];
      vv = val[i];
      d = rs_digit(kk, vv, pass, n);
    }
    const uint64_t m = match_digit(d, valid);
    const uint32_t below = (uint32_t)__popcll(m & lanemask_lt());
    if (valid && below == 0) wcnt[w][d] = (uint32_t)__popcll(m);
    __syncthreads();
    if (valid) {
      uint32_t pos = off[d] + below;
      for (int k = 0; k < w; ++k) pos += wcnt[k][d];
      key_out[pos] = kk;
      val_out[pos] = vv;
    }
    __syncthreads();
    uint32_t s = 0;
    for (int k = 0; k < RS_B / 64; ++k) {
      s += wcnt[k][tid];
      wcnt[k][tid] = 0;
    }
    off[tid] += s;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_gather(const uint32_t* __restrict__ sval,
                                                const uint32_t* __restrict__ counters, int64_t M,
                                                const GRec* __restrict__ rec,
                                                const uint2* __restrict__ rect,
                                                const uint32_t* __restrict__ tiles,
                                                GRec* __restrict__ rec_s, uint2* __restrict__ rect_s,
                                                uint32_t* __restrict__ tiles_s,
                                                uint32_t* __restrict__ item_s,
                                                int32_t* __restrict__ rank_of) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > M) return;
  const uint32_t nv = counters[0];
  if (r >= nv) {
    tiles_s[r] = 0;
    return;
  }
  const uint32_t it = sval[r];
  rec_s[r] = rec[it];
  rect_s[r] = rect[it];
  tiles_s[r] = tiles[it];
  item_s[r] = it;
  rank_of[it] = (int32_t)r;
}

__device__ __forceinline__ int find_cam_by_row(const CamDev* cams, int n_cams, int64_t row) {
  int lo = 0, hi = n_cams - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cams[mid].row_off <= row) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int find_cam_by_tile(const CamDev* cams, int n_cams, int tile) {
  int lo = 0, hi = n_cams - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cams[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// pair j of a chunk -> (rank offset k in the chunk, tile of the camera)
__device__ __forceinline__ void pair_tile(const uint32_t* poff, int nr, uint32_t j, const uint2* rect_s,
                                          int64_t r0, int TX, int& k, int& tl) {
  int lo = 0, hi = nr - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (poff[mid] <= j) lo = mid; else hi = mid - 1;
  }
  k = lo;
  const uint2 rc = rect_s[r0 + lo];
  const uint32_t x0 = rc.x & 0xffffu, x1 = rc.x >> 16, y0 = rc.y & 0xffffu;
  const uint32_t wdt = x1 - x0;
  const uint32_t loc = j - poff[lo];
  const uint32_t ty = y0 + loc / wdt;
  const uint32_t tx = x0 + loc - (loc / wdt) * wdt;
  tl = (int)(ty * (uint32_t)TX + tx);
}

struct ChunkInfo {
  int cam;
  int64_t c, r0, r1;
};

__device__ __forceinline__ ChunkInfo chunk_info(const CamDev* cams, int n_cams,
                                                const uint32_t* vis_off, int64_t row) {
  ChunkInfo ci;
  ci.cam = find_cam_by_row(cams, n_cams, row);
  ci.c = row - cams[ci.cam].row_off;
  ci.r0 = (int64_t)vis_off[ci.cam] + ci.c * CHUNK;
  const int64_t e = (int64_t)vis_off[ci.cam + 1];
  ci.r1 = ci.r0 + CHUNK < e ? ci.r0 + CHUNK : e;
  return ci;
}

__global__ __launch_bounds__(256) void k_chunk_count(const CamDev* __restrict__ cams, int n_cams,
                                                     const uint32_t* __restrict__ vis_off,
                                                     const uint64_t* __restrict__ pair_off,
                                                     const uint2* __restrict__ rect_s,
                                                     uint32_t* __restrict__ mat) {
  __shared__ uint32_t hist[MAX_TILES_PER_CAM];
  __shared__ uint32_t poff[CHUNK + 1];
  const ChunkInfo ci = chunk_info(cams, n_cams, vis_off, blockIdx.x);
  if (ci.r0 >= ci.r1) return;
  const CamDev& cam = cams[ci.cam];
  const int ntl = cam.TX * cam.TY;
  const int nr = (int)(ci.r1 - ci.r0);
  for (int t = threadIdx.x; t < ntl; t += 256) hist[t] = 0;
  const uint64_t p0 = pair_off[ci.r0];
  for (int k = threadIdx.x; k <= nr; k += 256) poff[k] = (uint32_t)(pair_off[ci.r0 + k] - p0);
  __syncthreads();
  const uint32_t np = poff[nr];
  for (uint32_t j = threadIdx.x; j < np; j += 256) {
    int k, tl;
    pair_tile(poff, nr, j, rect_s, ci.r0, cam.TX, k, tl);
    atomicAdd(&hist[tl], 1u);
  }
  __syncthreads();
  uint32_t* row = mat + cam.mat_off + ci.c * (int64_t)ntl;
  for (int t = threadIdx.x; t < ntl; t += 256) row[t] = hist[t];
}

// per global tile: exclusive prefix over its camera's used chunk rows, and the tile total
__global__ __launch_bounds__(256) void k_colscan(const CamDev* __restrict__ cams, int n_cams,
                                                 int n_tiles, const uint32_t* __restrict__ vis_off,
                                                 uint32_t* __restrict__ mat,
                                                 uint32_t* __restrict__ tile_total) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const int c = find_cam_by_tile(cams, n_cams, t);
  const CamDev& cam = cams[c];
  const int ntl = cam.TX * cam.TY;
  const int tl = t - cam.tile_off;
  const int64_t nvc = (int64_t)vis_off[c + 1] - vis_off[c];
  const int64_t rows = (nvc + CHUNK - 1) / CHUNK;
  uint32_t acc = 0;
  uint32_t* col = mat + cam.mat_off + tl;
  for (int64_t r = 0; r < rows; ++r) {
    const uint32_t v = col[r * ntl];
    col[r * ntl] = acc;
    acc += v;
  }
  tile_total[t] = acc;
}

__global__ __launch_bounds__(256) void k_ranges(int n_tiles, const uint32_t* __restrict__ tile_start,
                                                const uint32_t* __restrict__ tile_total,
                                                uint32_t* __restrict__ ranges) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  ranges[2 * t] = tile_start[t];
  ranges[2 * t + 1] = tile_start[t] + tile_total[t];
}

__global__ __launch_bounds__(256) void k_chunk_scatter(const CamDev* __restrict__ cams, int n_cams,
                                                       const uint32_t* __restrict__ vis_off,
                                                       const uint64_t* __restrict__ pair_off,
                                                       const uint2* __restrict__ rect_s,
                                                       const uint32_t* __restrict__ mat,
                                                       const uint32_t* __restrict__ tile_start,
                                                       int64_t key_cap,
                                                       uint32_t* __restrict__ lists) {
  __shared__ uint32_t cur[MAX_TILES_PER_CAM];
  __shared__ uint32_t poff[CHUNK + 1];
  const ChunkInfo ci = chunk_info(cams, n_cams, vis_off, blockIdx.x);
  if (ci.r0 >= ci.r1) return;
  const CamDev& cam = cams[ci.cam];
  const int ntl = cam.TX * cam.TY;
  const int nr = (int)(ci.r1 - ci.r0);
  const uint32_t* row = mat + cam.mat_off + ci.c * (int64_t)ntl;
  for (int t = threadIdx.x; t < ntl; t += 256) cur[t] = tile_start[cam.tile_off + t] + row[t];
  const uint64_t p0 = pair_off[ci.r0];
  for (int k = threadIdx.x; k <= nr; k += 256) poff[k] = (uint32_t)(pair_off[ci.r0 + k] - p0);
  __syncthreads();
  const uint32_t np = poff[nr];
  for (uint32_t j = threadIdx.x; j < np; j += 256) {
    int k, tl;
    pair_tile(poff, nr, j, rect_s, ci.r0, cam.TX, k, tl);
    const uint32_t pos = atomicAdd(&cur[tl], 1u);
    if ((int64_t)pos < key_cap) lists[pos] = (uint32_t)(ci.r0 + k);
  }
}

// LDS radix sort of n <= SORT_WIN keys in a[], 8-bit digits over `bits` bits
__device__ void lds_sort(uint32_t* a, uint32_t* b, int n, int bits, uint32_t* cnt,
                         uint32_t (*wcnt)[256]) {
  const int tid = threadIdx.x, w = tid >> 6;
  for (int sh = 0; sh < bits; sh += 8) {
    cnt[tid] = 0;
    for (int k = 0; k < 4; ++k) wcnt[k][tid] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += 256) atomicAdd(&cnt[(a[i] >> sh) & 255u], 1u);
    __syncthreads();
    // exclusive scan of the 256 digit counts (one per thread)
    {
      const uint32_t v = cnt[tid];
      uint32_t inc = v;
      const int l = __lane_id();
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(inc, o, 64);
        if (l >= o) inc += u;
      }
      __syncthreads();
      if (l == 63) wcnt[0][w] = inc;  // borrow row 0 for the wave totals
      __syncthreads();
      uint32_t basev = 0;
      for (int k = 0; k < w; ++k) basev += wcnt[0][k];
      __syncthreads();
      cnt[tid] = basev + inc - v;
      wcnt[0][tid] = 0;
      __syncthreads();
    }
    for (int r0 = 0; r0 < n; r0 += 256) {
      const int i = r0 + tid;
      const bool valid = i < n;
      const uint32_t kk = valid ? a[i] : 0u;
      const uint32_t d = (kk >> sh) & 255u;
      const uint64_t m = match_digit(d, valid);
      const uint32_t below = (uint32_t)__popcll(m & lanemask_lt());
      if (valid && below == 0) wcnt[w][d] = (uint32_t)__popcll(m);
      __syncthreads();
      if (valid) {
        uint32_t pos = cnt[d] + below;
        for (int k = 0; k < w; ++k) pos += wcnt[k][d];
        b[pos] = kk;
      }
      __syncthreads();
      uint32_t s = 0;
      for (int k = 0; k < 4; ++k) {
        s += wcnt[k][tid];
        wcnt[k][tid] = 0;
      }
      cnt[tid] += s;
      __syncthreads();
    }
    for (int i = tid; i < n; i += 256) a[i] = b[i];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_tile_sort(const CamDev* __restrict__ cams, int n_cams,
                                                   int n_tiles, const uint32_t* __restrict__ vis_off,
                                                   const uint32_t* __restrict__ mat,
                                                   const uint32_t* __restrict__ tile_start,
                                                   const uint32_t* __restrict__ tile_total,
                                                   int64_t key_cap, uint32_t* __restrict__ lists) {
  __shared__ uint32_t A[SORT_WIN];
  __shared__ uint32_t B[SORT_WIN];
  __shared__ uint32_t cnt[256];
  __shared__ uint32_t wcnt[4][256];
  const int t = blockIdx.x;
  const int c = find_cam_by_tile(cams, n_cams, t);
  const CamDev& cam = cams[c];
  const int64_t s = tile_start[t];
  int64_t e = s + tile_total[t];
  if (e > key_cap) e = key_cap;
  if (e - s <= 1) return;
  const uint32_t base = vis_off[c];
  const uint32_t nvc = vis_off[c + 1] - base;
  int bits = 8;
  while (bits < 32 && (nvc >> bits) != 0) bits += 8;
  const int ntl = cam.TX * cam.TY;
  const int tl = t - cam.tile_off;
  const int64_t rows = ((int64_t)nvc + CHUNK - 1) / CHUNK;
  constexpr int G = SORT_WIN / CHUNK;  // chunk rows per window
  int64_t ws = s;
  for (int64_t r = 0; ws < e; r += G) {
    int64_t we;
    if (e - ws <= SORT_WIN) {
      we = e;
    } else {
      const int64_t rn = r + G;
      we = rn < rows ? s + (int64_t)mat[cam.mat_off + rn * ntl + tl] : e;
      if (we > e) we = e;
    }
    const int n = (int)(we - ws);
    if (n > 1) {
      for (int i = threadIdx.x; i < n; i += 256) A[i] = lists[ws + i] - base;
      __syncthreads();
      lds_sort(A, B, n, bits, cnt, wcnt);
      for (int i = threadIdx.x; i < n; i += 256) lists[ws + i] = A[i] + base;
      __syncthreads();
    }
    ws = we;
  }
}

__global__ __launch_bounds__(256) void k_pair_total(const uint64_t* __restrict__ total,
                                                    int64_t key_cap, uint32_t* __restrict__ counters) {
  const uint64_t K = *total;
  counters[2] = (uint32_t)K;
  counters[3] = (uint32_t)(K >> 32);
  counters[1] = K > (uint64_t)key_cap ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_export_keys(const CamDev* __restrict__ cams, int n_cams,
                                                     int n_tiles,
                                                     const uint32_t* __restrict__ tile_start,
                                                     const uint32_t* __restrict__ tile_total,
                                                     const uint32_t* __restrict__ lists,
                                                     const GRec* __restrict__ rec_s,
                                                     int64_t key_cap, uint64_t* __restrict__ keys,
                                                     uint32_t* __restrict__ values) {
  const int t = blockIdx.x;
  if (t >= n_tiles) return;
  const int64_t s = tile_start[t];
  int64_t e = s + tile_total[t];
  if (e > key_cap) e = key_cap;
  for (int64_t i = s + threadIdx.x; i < e; i += blockDim.x) {
    const GRec& R = rec_s[lists[i]];
    keys[i] = ((uint64_t)t << 32) | __float_as_uint(R.depth);
    values[i] = R.gid;
  }
}

}  // namespace

void launch_depth_sort(const SetDev& S, const Work& w, hipStream_t st) {
  const int64_t M = (int64_t)S.n * S.n_cams;
  if (M == 0) {
    launch_fill_u32(w.counters, 0u, 1, st);
    launch_fill_u32(w.vis_off, 0u, S.n_cams + 1, st);
    launch_fill_u32(w.tiles_s, 0u, 1, st);
    return;
  }
  scan_u32(w.vis, w.vis_scan, M, nullptr, w.scan_scratch, st);
  hipLaunchKernelGGL(k_vis_offsets, dim3((S.n_cams + 1 + 255) / 256), dim3(256), 0, st, w.vis_scan,
                     w.vis, S.n, S.n_cams, w.vis_off, w.counters);
  const unsigned gb = (unsigned)((M + 255) / 256);
  hipLaunchKernelGGL(k_compact, dim3(gb), dim3(256), 0, st, w.vis, w.vis_scan, w.dkey, M,
                     w.skey[0], w.sval[0]);
  int passes = 4;
  if (S.n_cams > 1) passes = S.n_cams > 256 ? 6 : 5;
  const int64_t nb = w.rs_blocks;
  int cur = 0;
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nb), dim3(RS_B), 0, st, w.skey[cur], w.sval[cur],
                       w.counters, p, S.n, nb, w.rs_hist);
    scan_u32(w.rs_hist, w.rs_hist, 256 * nb, nullptr, w.scan_scratch, st);
    hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nb), dim3(RS_B), 0, st, w.skey[cur],
                       w.sval[cur], w.skey[cur ^ 1], w.sval[cur ^ 1], w.counters, p, S.n, nb,
                       w.rs_hist);
    cur ^= 1;
  }
  hipLaunchKernelGGL(k_gather, dim3((unsigned)((M + 1 + 255) / 256)), dim3(256), 0, st,
                     w.sval[cur], w.counters, M, w.rec, w.rect, w.tiles, w.rec_s, w.rect_s,
                     w.tiles_s, w.item_s, w.rank_of);
}

void launch_binning(const SetDev& S, const Work& w, int n_cams, hr_outputs* out, hipStream_t st) {
  const int64_t M = (int64_t)S.n * S.n_cams;
  uint64_t* Ktot = reinterpret_cast<uint64_t*>(w.counters + 10);
  scan_u64(w.tiles_s, w.pair_off, M + 1, Ktot, w.scan_scratch, st);
  hipLaunchKernelGGL(k_pair_total, dim3(1), dim3(1), 0, st, Ktot, S.key_cap, w.counters);
  if (w.chunk_rows > 0)
    hipLaunchKernelGGL(k_chunk_count, dim3((unsigned)w.chunk_rows), dim3(256), 0, st, w.cams,
                       n_cams, w.vis_off, w.pair_off, w.rect_s, w.mat);
  hipLaunchKernelGGL(k_colscan, dim3((S.n_tiles + 255) / 256), dim3(256), 0, st, w.cams, n_cams,
                     S.n_tiles, w.vis_off, w.mat, w.tile_total);
  scan_u32(w.tile_total, w.tile_start, S.n_tiles, nullptr, w.scan_scratch, st);
  if (w.chunk_rows > 0)
    hipLaunchKernelGGL(k_chunk_scatter, dim3((unsigned)w.chunk_rows), dim3(256), 0, st, w.cams,
                       n_cams, w.vis_off, w.pair_off, w.rect_s, w.mat, w.tile_start, S.key_cap,
                       w.lists);
  hipLaunchKernelGGL(k_tile_sort, dim3(S.n_tiles), dim3(256), 0, st, w.cams, n_cams, S.n_tiles,
                     w.vis_off, w.mat, w.tile_start, w.tile_total, S.key_cap, w.lists);
  if (out && out->ranges)
    hipLaunchKernelGGL(k_ranges, dim3((S.n_tiles + 255) / 256), dim3(256), 0, st, S.n_tiles,
                       w.tile_start, w.tile_total, out->ranges);
  if (out && out->keys && out->values)
    hipLaunchKernelGGL(k_export_keys, dim3(S.n_tiles), dim3(256), 0, st, w.cams, n_cams, S.n_tiles,
                       w.tile_start, w.tile_total, w.lists, w.rec_s, S.key_cap, out->keys,
                       out->values);
}

}  // namespace hr
