// Depth ordering and tile binning (the "tile-wise sorting" of Sec. 1).
//
// Instead of radix-sorting one 64-bit (tile | depth) key per (tile, Gaussian)
// pair, the pairs are produced grouped by tile and ordered by depth rank up to
// small windows:
//  1. the visible (camera, Gaussian) items are radix-sorted once by
//     (camera, fp32 depth bits); stability keeps equal depths in index order,
//     so an item's position (its rank) orders it by (depth, index);
//  2. ranks are cut into chunks of CHUNK (the rows of a chunk x tile count
//     matrix); the work unit of both binning passes is one (chunk, tile row):
//     the chunk's Gaussians whose tile rectangle spans that row, each
//     contributing one run of tiles [x0, x1);
//  3. count pass: a run adds +1 at x0 and -1 at x1 of an LDS difference row,
//     whose prefix sum is the chunk's count for every tile of the row - two
//     LDS atomics per (Gaussian, row) however many tiles it covers; a column
//     scan turns the matrix into (chunk, tile) sub-segment starts, and the
//     per-tile totals and ranges;
//  4. scatter pass: the same unit writes every rank of its runs into the
//     sub-segments of its row, a cursor per tile in LDS. One workgroup owns
//     all of the (chunk, tile) sub-segments of its row, so its writes fill
//     whole cache lines before they leave L2.
// Chunk sub-segments follow each other in rank order, so ordering a tile's
// list only needs the small rank windows of window.hpp, which the blend
// kernels do in LDS for the windows they reach. The key traffic is one write
// of a 4-byte rank per pair and one read per pair the blend reaches.
#include <algorithm>
#include <cmath>

#include "kernels.hpp"
#include "window.hpp"

namespace hr {
namespace {

constexpr int RS_B = 256;             // radix-sort threads per block
constexpr int MAX_TX = MAX_TILE_COLS; // widest tile row of a camera
constexpr int NARROW_RUN = 4;         // runs up to this wide are written by one lane
constexpr int GROUP = 4;              // lanes that share one medium run in the scatter
constexpr int SCHED_BUCKETS = 33;     // schedule buckets: list length 0, then by bit length

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

// digit `pass` of an item's sort key: bytes 0-3 of the fp32 depth bits, then
// bytes of the camera index (several cameras)
__device__ __forceinline__ uint32_t rs_digit(uint32_t key, uint32_t val, int pass, int n) {
  if (pass < 4) return (key >> (8 * pass)) & 255u;
  const uint32_t cam = val / (uint32_t)n;
  return (cam >> (8 * (pass - 4))) & 255u;
}

// Compaction of the visible items into the first radix-sort buffers, CB_ITEMS
// items per workgroup; the first n_cams + 1 threads also write each camera's
// first rank and the total, and thread n_cams the binning items of every
// camera: (used chunk row, tile row) pairs, item_off[c] the first of camera c,
// item_off[n_cams] the total. It counts digit 0 of the visible keys into the
// global digit counts (the counts do not depend on the order; pass p counts
// digit p + 1) and clears the state the radix passes will use for this number
// of visible items.
constexpr int CB_ITEMS = 1024;

__global__ __launch_bounds__(256) void k_compact(const uint32_t* __restrict__ vis,
                                                 const uint32_t* __restrict__ vis_scan,
                                                 const uint32_t* __restrict__ dkey, int n,
                                                 int n_cams, const CamDev* __restrict__ cams,
                                                 uint32_t* __restrict__ skey,
                                                 uint32_t* __restrict__ sval,
                                                 uint32_t* __restrict__ vis_off,
                                                 uint32_t* __restrict__ item_off,
                                                 uint32_t* __restrict__ counters, int passes,
                                                 uint32_t kpb, uint32_t* __restrict__ ghist,
                                                 uint32_t* __restrict__ rs1, int64_t groups,
                                                 int64_t nb_max) {
  __shared__ uint32_t lh[256];
  lh[threadIdx.x] = 0u;
  const int64_t M = (int64_t)n * n_cams;
  const uint32_t nv = vis_scan[M - 1] + vis[M - 1];
  // the radix state of the passes: tickets and group counters whole, then per
  // pass the group and block counts of the blocks this many keys fill
  {
    const int64_t nbk = ((int64_t)nv + kpb - 1) / kpb;
    const int64_t gk = (nbk + RS_GROUP - 1) / RS_GROUP;
    const int64_t head = 8 + RS_MAX_PASSES * groups;
    const int64_t per = 256 * (gk + nbk);
    const int64_t total = head + passes * per;
    uint32_t* gpub = rs1 + head;
    uint32_t* pub = gpub + (int64_t)RS_MAX_PASSES * groups * 256;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
      if (q < head) {
        rs1[q] = 0u;
        continue;
      }
      const int64_t r = q - head, p = r / per, e = r - p * per;
      if (e < 256 * gk)
        gpub[p * groups * 256 + e] = 0u;
      else
        pub[p * nb_max * 256 + (e - 256 * gk)] = 0u;
    }
  }
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q <= n_cams;
       q += (int64_t)gridDim.x * blockDim.x) {
    if (q < n_cams) {
      vis_off[q] = vis_scan[q * n];
      continue;
    }
    vis_off[q] = nv;
    counters[0] = nv;
    uint32_t acc = 0;
    for (int c = 0; c < n_cams; ++c) {
      item_off[c] = acc;
      const uint32_t end = c + 1 < n_cams ? vis_scan[(int64_t)(c + 1) * n] : nv;
      const uint32_t rows = (end - vis_scan[(int64_t)c * n] + CHUNK - 1) / CHUNK;
      acc += rows * (uint32_t)cams[c].TY;
    }
    item_off[n_cams] = acc;
  }
  const int64_t i0 = (int64_t)blockIdx.x * CB_ITEMS + threadIdx.x;
  __syncthreads();
  uint32_t fl[CB_ITEMS / 256], sc[CB_ITEMS / 256], dk[CB_ITEMS / 256];
#pragma unroll
  for (int r = 0; r < CB_ITEMS / 256; ++r) {
    const int64_t i = i0 + 256 * r;
    fl[r] = i < M ? vis[i] : 0u;
    sc[r] = i < M ? vis_scan[i] : 0u;
    dk[r] = i < M ? dkey[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < CB_ITEMS / 256; ++r)
    if (fl[r]) {
      skey[sc[r]] = dk[r];
      sval[sc[r]] = (uint32_t)(i0 + 256 * r);
      atomicAdd(&lh[rs_digit(dk[r], (uint32_t)(i0 + 256 * r), 0, n)], 1u);
    }
  __syncthreads();
  const uint32_t c = lh[threadIdx.x];
  if (c) atomicAdd(&ghist[(blockIdx.x % RS_GHIST_COPIES) * 256 + threadIdx.x], c);
}

// One radix pass in one dispatch. Workgroups take block numbers from a ticket,
// so a workgroup only ever waits for blocks whose workgroups already run. Each
// counts the digits of its block of keys and publishes the counts at once
// (device-coherent words, flagged); the last block of each group of RS_GROUP
// to publish also publishes the group's sum. A block's offset for digit d is
// the global offset of d (the digit counts made before the pass) plus the
// counts of d in the groups and the blocks of its group before it; those
// published words are read 16 at a time, since each read crosses to another
// XCD's writes and costs a round trip to memory. The scatter is stable inside
// the block (lanes ranked by equal digits per wave, waves in order). Each
// block also counts the next pass's digit of its keys into that pass's global
// counts.
constexpr uint32_t RS_PUB = 0x80000000u;
constexpr uint32_t RS_SPIN_LIMIT = 1u << 16;
constexpr int RS_BATCH = 16;

__device__ __forceinline__ void rs_publish(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v | RS_PUB, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t rs_peek(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// sum of the published words p[q * 256] for q in [q0, q1), waiting for each
// (bounded: a give-up sets gave_up and counts the word as 0)
__device__ __forceinline__ uint32_t rs_sum_published(const uint32_t* p, uint32_t q0, uint32_t q1,
                                                     bool& gave_up) {
  uint32_t s = 0;
  for (uint32_t qb = q0; qb < q1; qb += RS_BATCH) {
    uint32_t v[RS_BATCH];
#pragma unroll
    for (int j = 0; j < RS_BATCH; ++j) {
      const uint32_t q = qb + j < q1 ? qb + j : q1 - 1;
      v[j] = rs_peek(p + (int64_t)q * 256);
    }
#pragma unroll
    for (int j = 0; j < RS_BATCH; ++j) {
      if (qb + j >= q1) continue;
      uint32_t x = v[j];
      for (uint32_t spins = 0; !(x & RS_PUB); ++spins) {
        if (spins >= RS_SPIN_LIMIT) {
          gave_up = true;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        x = rs_peek(p + (int64_t)(qb + j) * 256);
      }
      s += x & ~RS_PUB;
    }
  }
  return s;
}

template <int RS_ROUNDS>
__global__ __launch_bounds__(RS_B) void k_rs_onepass(const uint32_t* __restrict__ key,
                                                     const uint32_t* __restrict__ val,
                                                     uint32_t* __restrict__ key_out,
                                                     uint32_t* __restrict__ val_out,
                                                     const uint32_t* __restrict__ counters,
                                                     int pass, int passes, int n,
                                                     uint32_t* __restrict__ ghist_all,
                                                     uint32_t* __restrict__ rs1, int64_t groups,
                                                     int64_t nb_max,
                                                     uint32_t* __restrict__ wait_flag) {
  __shared__ uint32_t off[256];
  __shared__ uint32_t lh[256];
  __shared__ uint32_t nh[256];
  __shared__ uint32_t wcnt[RS_B / 64][256];
  __shared__ uint32_t red4[4];
  __shared__ uint32_t s_b, s_last;
  const int tid = threadIdx.x, w = tid >> 6;
  const uint32_t nv = counters[0];
  constexpr uint32_t KPB = RS_ROUNDS * RS_B;
  const uint32_t nbk = (nv + KPB - 1) / KPB;
  // the grid is sized for every item being visible: the surplus leaves at once
  if (blockIdx.x >= nbk) return;
  uint32_t* ticket = rs1 + pass;
  uint32_t* gcnt = rs1 + 8 + (int64_t)pass * groups;
  uint32_t* gpub = rs1 + 8 + RS_MAX_PASSES * groups + (int64_t)pass * groups * 256;
  uint32_t* pub = rs1 + 8 + RS_MAX_PASSES * groups + (int64_t)RS_MAX_PASSES * groups * 256 +
                  (int64_t)pass * nb_max * 256;
  const uint32_t* ghist = ghist_all + (int64_t)pass * RS_GHIST_COPIES * 256;
  const bool count_next = pass + 1 < passes;
  if (tid == 0) s_b = atomicAdd(ticket, 1u);
  lh[tid] = 0u;
  nh[tid] = 0u;
#pragma unroll
  for (int k = 0; k < RS_B / 64; ++k) wcnt[k][tid] = 0u;
  // global counts of this thread's digit (the copies summed)
  uint32_t gd[RS_GHIST_COPIES];
#pragma unroll
  for (int c = 0; c < RS_GHIST_COPIES; ++c) gd[c] = ghist[c * 256 + tid];
  __syncthreads();
  const uint32_t b = s_b;
  const int64_t base = (int64_t)b * KPB;
  // every round's keys are loaded up front, so the loads overlap
  uint32_t kr[RS_ROUNDS], vr[RS_ROUNDS];
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = base + r * RS_B + tid;
    kr[r] = i < nv ? key[i] : 0u;
    vr[r] = i < nv ? val[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r)
    if (base + r * RS_B + tid < nv) atomicAdd(&lh[rs_digit(kr[r], vr[r], pass, n)], 1u);
  __syncthreads();
  rs_publish(&pub[(int64_t)b * 256 + tid], lh[tid]);
  if (count_next) {
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r)
      if (base + r * RS_B + tid < nv) atomicAdd(&nh[rs_digit(kr[r], vr[r], pass + 1, n)], 1u);
  }
  uint32_t gsum = 0;
#pragma unroll
  for (int c = 0; c < RS_GHIST_COPIES; ++c) gsum += gd[c];
  uint32_t total;
  const uint32_t gex = group_excl_scan(gsum, red4, total);  // has barriers
  if (count_next && nh[tid])
    atomicAdd(&ghist_all[((int64_t)(pass + 1) * RS_GHIST_COPIES + b % RS_GHIST_COPIES) * 256 + tid],
              nh[tid]);
  const uint32_t g = b / RS_GROUP, g0 = g * RS_GROUP;
  const uint32_t gsize = nbk - g0 < (uint32_t)RS_GROUP ? nbk - g0 : (uint32_t)RS_GROUP;
  if (tid == 0) s_last = atomicAdd(&gcnt[g], 1u) == gsize - 1 ? 1u : 0u;
  __syncthreads();
  bool gave_up = false;
  // the last of the group to arrive publishes the group's sum
  if (s_last)
    rs_publish(&gpub[(int64_t)g * 256 + tid],
               rs_sum_published(pub + tid, g0, g0 + gsize, gave_up));
  // the counts of this digit before the block: whole groups, then blocks
  const uint32_t pre = rs_sum_published(gpub + tid, 0, g, gave_up) +
                       rs_sum_published(pub + tid, g0, b, gave_up);
  if (gave_up) atomicOr(wait_flag, 1u);
  off[tid] = gex + pre;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = base + r * RS_B + tid;
    const bool valid = i < nv;
    const uint32_t kk = kr[r], vv = vr[r];
    const uint32_t d = valid ? rs_digit(kk, vv, pass, n) : 0u;
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
    uint32_t sum = 0;
    for (int k = 0; k < RS_B / 64; ++k) {
      sum += wcnt[k][tid];
      wcnt[k][tid] = 0;
    }
    off[tid] += sum;
    __syncthreads();
  }
}

// All passes of the radix sort in one dispatch of a few 1024-thread
// workgroups (at most RSC_MAX_BLOCKS, so that all of them are resident at
// once) that meet at grid barriers. In pass p each workgroup owns a slice of
// ceil(nv / grid) consecutive positions: it counts digit p over its slice and
// stores the counts, the workgroups meet, each sums every workgroup's counts
// (digit totals, and the counts of the workgroups before it) into its digit
// offsets, scatters its slice stably, and the workgroups meet again before
// the next pass reads the scattered keys. No workgroup waits on another's
// prefix, so a pass costs two barrier round trips instead of a look-back
// chain. The waits are bounded: a give-up sets wait_flag, every wave still
// leaves.
constexpr int RSC_T = 1024;             // threads per workgroup
constexpr int RSC_W = RSC_T / 64;       // waves per workgroup

// grid barrier number k (1, 2, ...) of a dispatch: arrive, then wait until
// every workgroup has arrived k times; the fences make the workgroup's global
// writes before the barrier visible to every workgroup after it
__device__ __forceinline__ void rsc_barrier(uint32_t* ctr, uint32_t k, uint32_t* wait_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(ctr, 1u);
    const uint32_t target = k * gridDim.x;
    uint32_t spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++spins >= RS_SPIN_LIMIT) {
        atomicOr(wait_flag, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
  }
  __syncthreads();
}

// exclusive scan of one value per thread over the RSC_T-thread workgroup
__device__ __forceinline__ uint32_t rsc_excl_scan(uint32_t v, uint32_t* lds) {
  const int w = threadIdx.x >> 6, l = __lane_id();
  uint32_t inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(inc, o, 64);
    if (l >= o) inc += u;
  }
  if (l == 63) lds[w] = inc;
  __syncthreads();
  uint32_t base = 0;
  for (int k = 0; k < w; ++k) base += lds[k];
  __syncthreads();
  return base + inc - v;
}

__global__ __launch_bounds__(RSC_T) void k_rs_coop(uint32_t* __restrict__ key0,
                                                   uint32_t* __restrict__ val0,
                                                   uint32_t* __restrict__ key1,
                                                   uint32_t* __restrict__ val1,
                                                   const uint32_t* __restrict__ counters,
                                                   int passes, int n, uint32_t* __restrict__ hist,
                                                   uint32_t* __restrict__ bar,
                                                   uint32_t* __restrict__ wait_flag) {
  __shared__ uint32_t lh[256];             // this slice's digit counts, then digit totals
  __shared__ uint32_t part[4][256];        // partial sums over workgroup ranges
  __shared__ uint32_t off[256];            // next position of each digit
  __shared__ uint32_t wc[2][RSC_W][256];   // a round's counts per wave, then positions
  __shared__ uint32_t red16[RSC_W];
  constexpr int QK = RSC_MAX_BLOCKS / 4;
  const int tid = threadIdx.x, w = tid >> 6;
  const uint32_t G = gridDim.x, b = blockIdx.x;
  const uint32_t nv = counters[0];
  const uint32_t S = (nv + G - 1) / G;
  const uint32_t lo = min(b * S, nv), hi = min(lo + S, nv);
  uint32_t nbar = 0;
  for (int p = 0; p < passes; ++p) {
    const uint32_t* ks = (p & 1) ? key1 : key0;
    const uint32_t* vs = (p & 1) ? val1 : val0;
    uint32_t* kd = (p & 1) ? key0 : key1;
    uint32_t* vd = (p & 1) ? val0 : val1;
    uint32_t* H = hist + (int64_t)p * RSC_MAX_BLOCKS * 256;
    if (tid < 256) lh[tid] = 0u;
    for (int k = tid; k < 2 * RSC_W * 256; k += RSC_T) (&wc[0][0][0])[k] = 0u;
    __syncthreads();
    for (uint32_t i = lo + tid; i < hi; i += RSC_T) atomicAdd(&lh[rs_digit(ks[i], vs[i], p, n)], 1u);
    __syncthreads();
    if (tid < 256) H[(int64_t)b * 256 + tid] = lh[tid];
    rsc_barrier(bar, ++nbar, wait_flag);
    // digit d = tid & 255: quarter q sums the counts of workgroups q, q + 4,
    // ... (all loads in flight at once)
    {
      const int d = tid & 255, q = tid >> 8;
      uint32_t c[QK];
#pragma unroll
      for (int k = 0; k < QK; ++k) {
        const uint32_t g = (uint32_t)(q + 4 * k);
        c[k] = g < G ? H[(int64_t)g * 256 + d] : 0u;
      }
      uint32_t before = 0, all = 0;
#pragma unroll
      for (int k = 0; k < QK; ++k) {
        all += c[k];
        if ((uint32_t)(q + 4 * k) < b) before += c[k];
      }
      part[q][d] = all;
      wc[0][q][d] = before;  // wc is free until the first round
    }
    __syncthreads();
    if (tid < 256) {
      lh[tid] = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
      off[tid] = wc[0][0][tid] + wc[0][1][tid] + wc[0][2][tid] + wc[0][3][tid];
    }
    __syncthreads();
    {
      // exclusive scan of the digit totals (threads past 256 add zeros)
      const uint32_t v = tid < 256 ? lh[tid] : 0u;
      const uint32_t gex = rsc_excl_scan(v, red16);
      if (tid < 256) off[tid] += gex;
    }
    for (int k = tid; k < RSC_W * 256; k += RSC_T) (&wc[0][0][0])[k] = 0u;
    __syncthreads();
    // stable scatter in rounds of RSC_T positions: wave w holds positions
    // [64 w, 64 w + 64) of the round, so (round, wave, lane) is position
    // order. The two count buffers alternate: a round clears the one the
    // next round fills, two barriers per round.
    int cb = 0;
    for (uint32_t r0 = lo; r0 < hi; r0 += RSC_T, cb ^= 1) {
      const uint32_t i = r0 + tid;
      const bool valid = i < hi;
      const uint32_t kk = valid ? ks[i] : 0u, vv = valid ? vs[i] : 0u;
      const uint32_t d = valid ? rs_digit(kk, vv, p, n) : 0u;
      const uint64_t m = match_digit(d, valid);
      const uint32_t below = (uint32_t)__popcll(m & lanemask_lt());
      if (valid && below == 0) wc[cb][w][d] = (uint32_t)__popcll(m);
      __syncthreads();
      if (tid < 256) {  // first position of each (wave, digit), in place
        uint32_t s = off[tid];
#pragma unroll
        for (int k = 0; k < RSC_W; ++k) {
          const uint32_t c = wc[cb][k][tid];
          wc[cb][k][tid] = s;
          s += c;
        }
        off[tid] = s;
      }
      for (int k = tid; k < RSC_W * 256; k += RSC_T) (&wc[cb ^ 1][0][0])[k] = 0u;
      __syncthreads();
      if (valid) {
        const uint32_t pos = wc[cb][w][d] + below;
        kd[pos] = kk;
        vd[pos] = vv;
      }
    }
    if (p + 1 < passes) rsc_barrier(bar, ++nbar, wait_flag);
  }
}

// The per-rank part of the tile-ellipse test (see ellipse_cut), FP64.
__device__ __forceinline__ EllP ell_params(const GRec& R, const uint2 rc, double ln_amin) {
  const double a = R.ca, b = R.cb, c = R.cc;
  EllP e;
  e.det = a * c - b * b;
  e.dymax = e.sc = 0.0;
  if (!(a > 0.0 && c > 0.0 && e.det > 0.0)) {
    e.rp = INFINITY;  // keep the rectangle run
  } else {
    const double rr = 2.0 * (log((double)R.op) - ln_amin);
    if (!(rr > 0.0)) {
      e.rp = -1.0;  // alpha never reaches alpha_min
    } else {
      const int w = (int)(rc.x >> 16) - (int)(rc.x & 0xffffu);
      const int h = (int)(rc.y >> 16) - (int)(rc.y & 0xffffu);
      const double ext = 16.0 * (double)max(w, h);
      e.rp = 1.01 * rr + 0.1 + 1e-5 * (a + c) * ext * ext;
      e.dymax = sqrt(a * e.rp / e.det);
      e.sc = sqrt(e.rp / (c * e.det));
    }
  }
  return e;
}

__global__ __launch_bounds__(256) void k_gather(const uint32_t* __restrict__ sval,
                                                const uint32_t* __restrict__ counters, int64_t M,
                                                const GRec* __restrict__ rec,
                                                const uint2* __restrict__ rect,
                                                GRec* __restrict__ rec_s, uint2* __restrict__ rect_s,
                                                uint32_t* __restrict__ item_s,
                                                int32_t* __restrict__ rank_of, double ln_amin,
                                                EllP* __restrict__ ell) {
  const int64_t nv = std::min<int64_t>(M, (int64_t)counters[0]);
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nv;
       r += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t it = sval[r];
    const GRec R = rec[it];
    const uint2 rc = rect[it];
    rec_s[r] = R;
    rect_s[r] = rc;
    item_s[r] = it;
    rank_of[it] = (int32_t)r;
    if (ell) ell[r] = ell_params(R, rc, ln_amin);
  }
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

struct BinItem {
  int cam, y, TX, ntl;
  int64_t chunk, r0, r1;  // chunk index in the camera; its ranks [r0, r1)
};

__device__ __forceinline__ BinItem bin_item(const CamDev* cams, int n_cams,
                                            const uint32_t* vis_off, const uint32_t* item_off,
                                            uint32_t item) {
  int lo = 0, hi = n_cams - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (item_off[mid] <= item) lo = mid; else hi = mid - 1;
  }
  BinItem b;
  b.cam = lo;
  const CamDev& cam = cams[lo];
  const uint32_t li = item - item_off[lo];
  b.chunk = li / (uint32_t)cam.TY;
  b.y = (int)(li - (uint32_t)b.chunk * (uint32_t)cam.TY);
  b.TX = cam.TX;
  b.ntl = cam.TX * cam.TY;
  b.r0 = (int64_t)vis_off[lo] + b.chunk * CHUNK;
  const int64_t e = vis_off[lo + 1];
  b.r1 = b.r0 + CHUNK < e ? b.r0 + CHUNK : e;
  return b;
}

// The run of rank k in tile row y, or an empty one.
__device__ __forceinline__ bool row_run(const uint2 rc, int y, int& x0, int& x1) {
  x0 = (int)(rc.x & 0xffffu);
  x1 = (int)(rc.x >> 16);
  return y >= (int)(rc.y & 0xffffu) && y < (int)(rc.y >> 16);
}

// With the tile-ellipse option, the run is cut to the tiles whose pixel
// centres can reach alpha >= alpha_min: outside the ellipse
// d^T Q d <= 2 ln(opacity / alpha_min) (conic Q of the record) every pixel
// skips the Gaussian, so those pairs change no output. The ellipse is grown
// (1.01 R + 0.1, plus a term for the magnitude of the quadratic form over the
// rectangle) to cover the FP32 evaluation of the blend's test. An opacity at
// or below alpha_min empties the row. FP64; the per-rank part is computed
// once (ell_params, in the gather), the per-row part in both passes by the
// same steps.
// g = (u, v, conic a, conic b), the first 16 bytes of the record
__device__ __forceinline__ bool ellipse_cut(const float4 g, const EllP& e, int y, int& x0,
                                            int& x1) {
  if (e.rp < 0.0) return false;
  if (isinf(e.rp)) return true;
  const double a = g.z, b = g.w;
  const double lo = fmax((double)y * TILE + 0.5 - (double)g.y, -e.dymax);
  const double hi = fmin((double)y * TILE + (TILE - 0.5) - (double)g.y, e.dymax);
  if (lo > hi) return false;
  const double ys = fmin(fmax(-b * e.sc, lo), hi), yn = fmin(fmax(b * e.sc, lo), hi);
  const double xmax = (-b * ys + sqrt(fmax(a * e.rp - e.det * ys * ys, 0.0))) / a;
  const double xmin = (-b * yn - sqrt(fmax(a * e.rp - e.det * yn * yn, 0.0))) / a;
  const int ex0 = (int)ceil(((double)g.x + xmin - (TILE - 0.5)) / TILE);
  const int ex1 = (int)floor(((double)g.x + xmax - 0.5) / TILE) + 1;
  x0 = max(x0, ex0);
  x1 = min(x1, ex1);
  return x1 > x0;
}

// The runs in row B.y of this thread's ranks k0 + 256 j, j < RUNS (x1 <= x0:
// none). All rectangles are loaded first, then the ellipse data of the ranks
// whose rectangle spans the row, so the loads of a thread overlap.
constexpr int RUNS = 2;
__device__ __forceinline__ void item_runs(const BinItem& B, int64_t k0,
                                          const uint2* __restrict__ rect_s,
                                          const GRec* __restrict__ rec_s,
                                          const EllP* __restrict__ ell, int x0[RUNS],
                                          int x1[RUNS]) {
  uint2 rc[RUNS];
#pragma unroll
  for (int j = 0; j < RUNS; ++j) {
    const int64_t k = k0 + 256 * j;
    rc[j] = k < B.r1 ? rect_s[k] : make_uint2(0u, 0u);  // rows [0, 0): no run
  }
  bool on[RUNS];
#pragma unroll
  for (int j = 0; j < RUNS; ++j) on[j] = row_run(rc[j], B.y, x0[j], x1[j]);
  if (ell) {
    float4 g[RUNS];
    EllP e[RUNS];
#pragma unroll
    for (int j = 0; j < RUNS; ++j)
      if (on[j]) {
        const int64_t k = k0 + 256 * j;
        g[j] = *reinterpret_cast<const float4*>(rec_s + k);
        e[j] = ell[k];
      }
#pragma unroll
    for (int j = 0; j < RUNS; ++j)
      if (on[j]) on[j] = ellipse_cut(g[j], e[j], B.y, x0[j], x1[j]);
  }
#pragma unroll
  for (int j = 0; j < RUNS; ++j)
    if (!on[j]) x1[j] = x0[j];
}

// Count pass: per (chunk, tile row), the chunk's pair count of every tile of
// the row, written to the chunk's row of the count matrix.
__global__ __launch_bounds__(256) void k_bin_count(const CamDev* __restrict__ cams, int n_cams,
                                                   const uint32_t* __restrict__ vis_off,
                                                   const uint32_t* __restrict__ item_off,
                                                   const uint2* __restrict__ rect_s,
                                                   const GRec* __restrict__ rec_s,
                                                   const uint32_t* __restrict__ tile_dmax,
                                                   const EllP* __restrict__ ell,
                                                   uint32_t* __restrict__ mat,
                                                   uint32_t* __restrict__ counters,
                                                   uint32_t* __restrict__ runs,
                                                   uint2* __restrict__ unit_runs,
                                                   int64_t key_cap) {
  __shared__ int32_t diff[MAX_TX + 1];
  __shared__ uint32_t red4[4];
  __shared__ uint32_t lr[CHUNK];  // the unit's runs: x0 | x1 << 10 | rank offset << 21
  __shared__ uint32_t nlr, lbase, lkeep;
  const uint32_t n_items = item_off[n_cams];
  for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const BinItem B = bin_item(cams, n_cams, vis_off, item_off, it);
    const CamDev& cam = cams[B.cam];
    for (int x = threadIdx.x; x <= B.TX; x += 256) diff[x] = 0;
    if (threadIdx.x == 0) nlr = 0;
    __syncthreads();
    const uint32_t* tdm = tile_dmax ? tile_dmax + cam.tile_off + B.y * B.TX : nullptr;
    for (int64_t k0 = B.r0 + threadIdx.x; k0 < B.r1; k0 += 256 * RUNS) {
      int rx0[RUNS], rx1[RUNS];
      item_runs(B, k0, rect_s, rec_s, ell, rx0, rx1);
#pragma unroll
      for (int j = 0; j < RUNS; ++j) {
        const int x0 = rx0[j], x1 = rx1[j];
        if (x1 <= x0) continue;
        lr[atomicAdd(&nlr, 1u)] =
            (uint32_t)x0 | ((uint32_t)x1 << 10) | ((uint32_t)(k0 + 256 * j - B.r0) << 21);
        if (!tdm) {
          atomicAdd(&diff[x0], 1);
          atomicSub(&diff[x1], 1);
        } else {
          const uint32_t dep = __float_as_uint(rec_s[k0 + 256 * j].depth);
          for (int x = x0; x < x1; ++x)
            if (dep < tdm[x]) {
              atomicAdd(&diff[x], 1);
              atomicSub(&diff[x + 1], 1);
            }
        }
      }
    }
    __syncthreads();
    // inclusive prefix of the difference row: 4 consecutive entries per thread
    const int x0 = 4 * threadIdx.x;
    int32_t v[4], s4 = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q] = x0 + q < B.TX ? diff[x0 + q] : 0;
      s4 += v[q];
    }
    uint32_t total;
    int32_t run = (int32_t)group_excl_scan((uint32_t)s4, red4, total);
    uint32_t* row = mat + cam.mat_off + B.chunk * B.ntl + (int64_t)B.y * B.TX;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      run += v[q];
      if (x0 + q < B.TX) row[x0 + q] = (uint32_t)run;
    }
    // the runs go to the scatter pass: one reservation per unit (there are no
    // more runs than pairs, so key_cap entries hold them unless the pairs
    // overflow, which the capacity check reports)
    if (threadIdx.x == 0) {
      const uint32_t nr = nlr;
      const uint32_t base = nr ? atomicAdd(&counters[RUN_ALLOC], nr) : 0u;
      const uint32_t keep = (int64_t)base >= key_cap ? 0u
                            : (uint32_t)min((int64_t)nr, key_cap - (int64_t)base);
      lbase = base;
      lkeep = keep;
      unit_runs[it] = make_uint2(base, keep);
    }
    __syncthreads();
    const uint32_t nr = lkeep, base = lbase;
    for (uint32_t q = threadIdx.x; q < nr; q += 256) runs[base + q] = lr[q];
    __syncthreads();
  }
}

// Scatter pass: per (chunk, tile row), every rank of the row's runs goes to
// the next free entry of its tile's sub-segment; afterwards the matrix entry
// holds the end of that sub-segment (relative to the tile start). Runs are
// written three ways by width: short ones (at most NARROW_RUN tiles) by one
// lane each, medium ones by groups of GROUP lanes (one LDS cursor atomic per
// tile in both), and runs over more than half of the row tile-major: each
// thread owns the cursors of its tiles in registers and walks those ranks in
// order, without atomics, its stores running along its own sub-segment.
__global__ __launch_bounds__(256) void k_bin_scatter(const CamDev* __restrict__ cams, int n_cams,
                                                     const uint32_t* __restrict__ vis_off,
                                                     const uint32_t* __restrict__ item_off,
                                                     const uint32_t* __restrict__ runs,
                                                     const uint2* __restrict__ unit_runs,
                                                     const GRec* __restrict__ rec_s,
                                                     const uint32_t* __restrict__ tile_dmax,
                                                     uint32_t* __restrict__ mat,
                                                     const uint32_t* __restrict__ tile_start,
                                                     int64_t key_cap, uint32_t* __restrict__ lists) {
  __shared__ uint32_t cur[MAX_TX];
  __shared__ uint32_t wide[CHUNK];      // x0 | x1 << 10 | rank offset << 21
  __shared__ uint32_t wide_dep[CHUNK];  // depth bits (culling only)
  __shared__ uint32_t mid[CHUNK];       // medium runs, same packing
  __shared__ uint32_t nwide, nmid;
  static_assert(MAX_TX <= 1024 && CHUNK <= 2048, "run packing");
  const uint32_t n_items = item_off[n_cams];
  for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const BinItem B = bin_item(cams, n_cams, vis_off, item_off, it);
    const CamDev& cam = cams[B.cam];
    const int trow = cam.tile_off + B.y * B.TX;
    uint32_t* row = mat + cam.mat_off + B.chunk * B.ntl + (int64_t)B.y * B.TX;
    for (int x = threadIdx.x; x < B.TX; x += 256) cur[x] = tile_start[trow + x] + row[x];
    if (threadIdx.x == 0) nwide = nmid = 0;
    __syncthreads();
    const uint32_t* tdm = tile_dmax ? tile_dmax + trow : nullptr;
    auto put = [&](uint32_t k, int x) {
      const uint32_t pos = atomicAdd(&cur[x], 1u);
      if ((int64_t)pos < key_cap) lists[pos] = k;
    };
    const int half = B.TX / 2;
    // the unit's runs from the count pass: short ones by one lane; the others
    // are sorted into the two lists
    const uint2 ur = unit_runs[it];
    for (uint32_t q = threadIdx.x; q < ur.y; q += 256) {
      const uint32_t packed = runs[ur.x + q];
      const int x0 = (int)(packed & 1023u), x1 = (int)((packed >> 10) & 2047u);
      const int64_t k = B.r0 + (packed >> 21);
      const int w = x1 - x0;
      if (w > NARROW_RUN && w > half) {
        const uint32_t qw = atomicAdd(&nwide, 1u);
        wide[qw] = packed;
        if (tdm) wide_dep[qw] = __float_as_uint(rec_s[k].depth);
      } else if (w > NARROW_RUN) {
        mid[atomicAdd(&nmid, 1u)] = packed;
      } else {
        const uint32_t dep = tdm ? __float_as_uint(rec_s[k].depth) : 0u;
        for (int x = x0; x < x1; ++x)
          if (!tdm || dep < tdm[x]) put((uint32_t)k, x);
      }
    }
    __syncthreads();
    // medium runs: groups of GROUP lanes take one rank each
    const uint32_t nm = nmid;
    const int grp = (int)threadIdx.x / GROUP, sub = (int)threadIdx.x % GROUP;
    for (uint32_t i = (uint32_t)grp; i < nm; i += 256 / GROUP) {
      const uint32_t wr = mid[i];
      const uint32_t k = (uint32_t)B.r0 + (wr >> 21);
      const int x1 = (int)((wr >> 10) & 2047u);
      const uint32_t dep = tdm ? __float_as_uint(rec_s[k].depth) : 0u;
      for (int x = (int)(wr & 1023u) + sub; x < x1; x += GROUP)
        if (!tdm || dep < tdm[x]) put(k, x);
    }
    __syncthreads();
    // wide runs, tile-major
    const uint32_t nw = nwide;
    for (int x = threadIdx.x; x < B.TX; x += 256) {
      uint32_t c = cur[x];
      const uint32_t tx = (uint32_t)x, lim = tdm ? tdm[x] : 0u;
      for (uint32_t i = 0; i < nw; ++i) {
        const uint32_t wr = wide[i];
        const bool in = tx >= (wr & 1023u) && tx < ((wr >> 10) & 2047u) &&
                        (!tdm || wide_dep[i] < lim);
        if (in) {
          if ((int64_t)c < key_cap) lists[c] = (uint32_t)B.r0 + (wr >> 21);
          ++c;
        }
      }
      row[x] = c - tile_start[trow + x];
    }
    __syncthreads();
  }
}

// per global tile: exclusive prefix over its camera's used chunk rows, and the
// tile total; per block of 256 tiles: the schedule bucket counts, the pairs,
// and the block-local part of the list starts
__global__ __launch_bounds__(256) void k_colscan(const CamDev* __restrict__ cams, int n_cams,
                                                 int n_tiles, const uint32_t* __restrict__ vis_off,
                                                 uint32_t* __restrict__ mat,
                                                 uint32_t* __restrict__ tile_total,
                                                 uint32_t* __restrict__ tile_start,
                                                 uint32_t* __restrict__ sched_cnt,
                                                 unsigned long long* __restrict__ sched_sum) {
  __shared__ uint32_t hist[SCHED_BUCKETS];
  __shared__ uint32_t wsum[4];
  if (threadIdx.x < SCHED_BUCKETS) hist[threadIdx.x] = 0;
  __syncthreads();
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  if (t < n_tiles) {
    const int c = find_cam_by_tile(cams, n_cams, t);
    const CamDev& cam = cams[c];
    const int ntl = cam.TX * cam.TY;
    const int tl = t - cam.tile_off;
    const int64_t nvc = (int64_t)vis_off[c + 1] - vis_off[c];
    const int64_t rows = (nvc + CHUNK - 1) / CHUNK;
    uint32_t* col = mat + cam.mat_off + tl;
    // 8 rows at a time: the loads of a group are in flight together
    for (int64_t r0 = 0; r0 < rows; r0 += 8) {
      uint32_t v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = r0 + q < rows ? col[(r0 + q) * ntl] : 0u;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (r0 + q < rows) col[(r0 + q) * ntl] = acc;
        acc += v[q];
      }
    }
    tile_total[t] = acc;
    atomicAdd(&hist[acc ? 32 - __clz(acc) : 0], 1u);
  }
  // the block's part of the list starts (the schedule adds the blocks before)
  uint32_t total;
  const uint32_t ex = group_excl_scan(acc, wsum, total);
  if (t < n_tiles) tile_start[t] = ex;
  __syncthreads();
  if (threadIdx.x < SCHED_BUCKETS) sched_cnt[blockIdx.x * SCHED_BUCKETS + threadIdx.x] = hist[threadIdx.x];
  if (threadIdx.x == 0) sched_sum[blockIdx.x] = total;
}

// Blend schedule: tiles by decreasing list length (buckets of log2 length),
// so the longest lists start first and the short ones fill in at the end.
// Each block of 256 tiles places its tiles after every tile of a longer
// bucket and after its bucket's tiles in earlier blocks; it also finishes
// the list starts, and block 0 the key count and the capacity check.
__global__ __launch_bounds__(256) void k_tile_schedule(int n_tiles, int64_t key_cap,
                                                       const uint32_t* __restrict__ tile_total,
                                                       const uint32_t* __restrict__ sched_cnt,
                                                       const unsigned long long* __restrict__ sched_sum,
                                                       uint32_t* __restrict__ tile_start,
                                                       uint32_t* __restrict__ order,
                                                       uint32_t* __restrict__ counters) {
  __shared__ uint32_t tot[SCHED_BUCKETS];
  __shared__ uint32_t off[SCHED_BUCKETS];
  __shared__ unsigned long long red[4];
  const int b = blockIdx.x;
  const int nb = gridDim.x;
  // sums over blocks: before this one (list starts), all (block 0: key count)
  unsigned long long pre = 0, all = 0;
  for (int q = threadIdx.x; q < nb; q += blockDim.x) {
    const unsigned long long v = sched_sum[q];
    if (q < b) pre += v;
    all += v;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    pre += __shfl_xor(pre, o, 64);
    all += __shfl_xor(all, o, 64);
  }
  if (__lane_id() == 0) red[threadIdx.x >> 6] = pre;
  __syncthreads();
  pre = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  if (b == 0) {
    if (__lane_id() == 0) red[threadIdx.x >> 6] = all;
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned long long K = red[0] + red[1] + red[2] + red[3];
      counters[2] = (uint32_t)K;
      counters[3] = (uint32_t)(K >> 32);
      counters[1] = K > (unsigned long long)key_cap ? 1u : 0u;
    }
  }
  // bucket k: tiles of every block, and of the blocks before this one (wave
  // w sums buckets w, w + 4, ..., a lane per block of tiles)
  const int wv = threadIdx.x >> 6, ln = __lane_id();
  for (int k = wv; k < SCHED_BUCKETS; k += 4) {
    uint32_t s_all = 0, s_pre = 0;
    for (int q = ln; q < nb; q += 64) {
      const uint32_t v = sched_cnt[q * SCHED_BUCKETS + k];
      s_all += v;
      if (q < b) s_pre += v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      s_all += __shfl_xor(s_all, o, 64);
      s_pre += __shfl_xor(s_pre, o, 64);
    }
    if (ln == 0) {
      tot[k] = s_all;
      off[k] = s_pre;
    }
  }
  __syncthreads();
  if (threadIdx.x < SCHED_BUCKETS) {
    uint32_t longer = 0;
    for (int k2 = threadIdx.x + 1; k2 < SCHED_BUCKETS; ++k2) longer += tot[k2];
    off[threadIdx.x] += longer;
  }
  __syncthreads();
  const int t = b * blockDim.x + threadIdx.x;
  if (t < n_tiles) {
    tile_start[t] += (uint32_t)pre;
    const uint32_t L = tile_total[t];
    order[atomicAdd(&off[L ? 32 - __clz(L) : 0], 1u)] = (uint32_t)t;
  }
}

__global__ __launch_bounds__(256) void k_ranges(int n_tiles, const uint32_t* __restrict__ tile_start,
                                                const uint32_t* __restrict__ tile_total,
                                                uint32_t* __restrict__ ranges) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  ranges[2 * t] = tile_start[t];
  ranges[2 * t + 1] = tile_start[t] + tile_total[t];
}

// Orders every window of every tile in place (only for exporting the keys;
// the blend kernels order the windows they reach themselves).
__global__ __launch_bounds__(256) void k_tile_order(const CamDev* __restrict__ cams, int n_cams,
                                                    const uint32_t* __restrict__ vis_off,
                                                    const uint32_t* __restrict__ mat,
                                                    const uint32_t* __restrict__ tile_start,
                                                    const uint32_t* __restrict__ tile_total,
                                                    int64_t key_cap, uint32_t* __restrict__ lists) {
  __shared__ uint32_t bitmap[WIN_WORDS];
  __shared__ uint32_t red[4];
  const int t = blockIdx.x;
  const int c = find_cam_by_tile(cams, n_cams, t);
  const WinCtx W = win_ctx(cams[c], c, t, vis_off, mat, tile_start, tile_total, key_cap);
  for (int w = 0; w < W.nwin; ++w) {
    int64_t a, b;
    win_range(W, w, a, b);
    if (a >= b) continue;
    const uint32_t wbase = W.rbase + (uint32_t)w * WIN;
    bitmap[threadIdx.x] = 0;
    __syncthreads();
    win_mark(lists, W, a, b, wbase, bitmap);
    __syncthreads();
    const uint32_t word = bitmap[threadIdx.x];
    uint32_t total;
    const uint32_t pre = group_excl_scan((uint32_t)__popc(word), red, total);
    uint32_t wv = word, idx = pre;
    while (wv) {
      const uint32_t bit = __ffs(wv) - 1;
      wv &= wv - 1;
      lists[W.s + a + idx] = wbase + 32u * threadIdx.x + bit;
      ++idx;
    }
    __syncthreads();
  }
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

void launch_depth_sort(const SetDev& S, const Work& w, bool ell, hipStream_t st) {
  const int64_t M = (int64_t)S.n * S.n_cams;
  if (M == 0) {
    launch_fill_u32(w.counters, 0u, 1, st);
    launch_fill_u32(w.vis_off, 0u, S.n_cams + 1, st);
    launch_fill_u32(w.item_off, 0u, S.n_cams + 1, st);
    return;
  }
  scan_u32(w.vis, w.vis_scan, M, nullptr, w.scan_scratch, st);
  int passes = 4;
  if (S.n_cams > 1) passes = S.n_cams > 256 ? 6 : 5;
  const int64_t nb = w.rs_blocks;
  const int kpb = rs_keys_for(M);
  const unsigned gb = (unsigned)((std::max<int64_t>(M, S.n_cams + 1) + CB_ITEMS - 1) / CB_ITEMS);
  hipLaunchKernelGGL(k_compact, dim3(gb), dim3(256), 0, st, w.vis, w.vis_scan, w.dkey, S.n,
                     S.n_cams, w.cams, w.skey[0], w.sval[0], w.vis_off, w.item_off, w.counters,
                     passes, (uint32_t)kpb, w.rs_ghist, w.rs1, w.rs_groups, nb);
  uint32_t* wait_flag = (uint32_t*)w.scan_scratch + 2;  // reported with the scans' flag
  if (kpb > 1024) {
    // many items (several cameras): the look-back of the one-dispatch passes
    // would chain over hundreds of blocks, the grid-barrier sort waits only
    // for its RSC_MAX_BLOCKS workgroups
    hipLaunchKernelGGL(k_rs_coop, dim3(RSC_MAX_BLOCKS), dim3(RSC_T), 0, st, w.skey[0],
                       w.sval[0], w.skey[1], w.sval[1], w.counters, passes, S.n, w.rs_hist,
                       w.rs1 + 7, wait_flag);
  } else {
    for (int p = 0; p < passes; ++p)
      hipLaunchKernelGGL(k_rs_onepass<4>, dim3((unsigned)nb), dim3(RS_B), 0, st,
                         w.skey[p & 1], w.sval[p & 1], w.skey[(p & 1) ^ 1], w.sval[(p & 1) ^ 1],
                         w.counters, p, passes, S.n, w.rs_ghist, w.rs1, w.rs_groups, nb,
                         wait_flag);
  }
  const int cur = passes & 1;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)std::min<int64_t>(4096, (M + 255) / 256)), dim3(256), 0, st,
                     w.sval[cur], w.counters, M, w.rec, w.rect, w.rec_s, w.rect_s,
                     w.item_s, w.rank_of, std::log((double)S.alpha_min),
                     ell ? w.ell_s : nullptr);
}

void launch_binning(const SetDev& S, const Work& w, int n_cams, bool cull, bool ell,
                    hr_outputs* out, hipStream_t st) {
  const uint32_t* tdm = cull ? w.tile_dmax : nullptr;
  const EllP* ellp = ell ? w.ell_s : nullptr;
  // one workgroup per (chunk, tile row) the cameras could use (the unused ones
  // exit at once): the dispatcher balances the uneven rows, nearest chunks first
  // at most 8192 workgroups, each taking units it, it + grid, ...: the bound
  // counts every chunk the cameras could fill, and with several cameras most
  // of those units do not exist, so a workgroup per unit of the bound would
  // mostly start only to leave
  const unsigned grid = (unsigned)std::min<int64_t>(8192, std::max<int64_t>(1, w.bin_items_max));
  if (w.bin_items_max > 0)
    hipLaunchKernelGGL(k_bin_count, dim3(grid), dim3(256), 0, st, w.cams, n_cams, w.vis_off,
                       w.item_off, w.rect_s, w.rec_s, tdm, ellp, w.mat, w.counters, w.runs,
                       w.unit_runs, S.key_cap);
  const unsigned tb = (unsigned)((S.n_tiles + 255) / 256);
  hipLaunchKernelGGL(k_colscan, dim3(tb), dim3(256), 0, st, w.cams, n_cams, S.n_tiles, w.vis_off,
                     w.mat, w.tile_total, w.tile_start, w.sched_cnt, w.sched_sum);
  hipLaunchKernelGGL(k_tile_schedule, dim3(tb), dim3(256), 0, st, S.n_tiles, S.key_cap,
                     w.tile_total, w.sched_cnt, w.sched_sum, w.tile_start, w.tile_order,
                     w.counters);
  if (w.bin_items_max > 0)
    hipLaunchKernelGGL(k_bin_scatter, dim3(grid), dim3(256), 0, st, w.cams, n_cams, w.vis_off,
                       w.item_off, w.runs, w.unit_runs, w.rec_s, tdm, w.mat, w.tile_start,
                       S.key_cap, w.lists);
  if (out && out->ranges)
    hipLaunchKernelGGL(k_ranges, dim3((S.n_tiles + 255) / 256), dim3(256), 0, st, S.n_tiles,
                       w.tile_start, w.tile_total, out->ranges);
  if (out && out->keys && out->values) {
    hipLaunchKernelGGL(k_tile_order, dim3(S.n_tiles), dim3(256), 0, st, w.cams, n_cams, w.vis_off,
                       w.mat, w.tile_start, w.tile_total, S.key_cap, w.lists);
    hipLaunchKernelGGL(k_export_keys, dim3(S.n_tiles), dim3(256), 0, st, w.cams, n_cams, S.n_tiles,
                       w.tile_start, w.tile_total, w.lists, w.rec_s, S.key_cap, out->keys,
                       out->values);
  }
}

}  // namespace hr
