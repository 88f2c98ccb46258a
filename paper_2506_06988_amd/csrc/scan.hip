// Exclusive prefix sums over device arrays: one pass up to 192 tiles of 4096
// elements, a reduce and a down-sweep kernel beyond.
// Every size is a host-side maximum; entries past the used part must be zero,
// so data-dependent lengths need no host synchronisation. Inputs and outputs
// are 16-byte aligned (workspace regions).
//
// Workgroups take their tile index from a ticket counter, so a workgroup only
// ever waits for tiles whose workgroups are already running. Each publishes
// its tile total at once (it waits for nothing before), then adds up the
// published totals of all tiles before it, read in parallel by its threads,
// retrying until every one of them is there. The last workgroup to finish
// clears the tickets and the published words for the next scan; the forward
// also clears them first (they live in the scan scratch, which the caller's
// workspace holds).
#include <algorithm>

#include "common.hpp"

namespace hr {
namespace {

constexpr int SB = 256;        // threads per block
constexpr int SI = 16;         // elements per thread
constexpr int SE = SB * SI;    // elements per block
constexpr uint32_t SPIN_LIMIT = 1u << 16;  // bounded wait: a broken protocol cannot hang

constexpr unsigned long long ST_TOTAL = 1ull << 32;  // published word holds the tile total

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int l = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(v, o, 64);
    if (l >= o) v += u;
  }
  return v;
}

// exclusive scan of one value per thread over the 256-thread block; returns the block total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* lds4, uint32_t& total) {
  const int w = threadIdx.x >> 6, l = __lane_id();
  const uint32_t inc = wave_incl_scan(v);
  if (l == 63) lds4[w] = inc;
  __syncthreads();
  uint32_t base = 0;
  total = 0;
#pragma unroll
  for (int k = 0; k < SB / 64; ++k) {
    const uint32_t s = lds4[k];
    if (k < w) base += s;
    total += s;
  }
  __syncthreads();
  return base + inc - v;
}

// Published words carry their value, so no other write has to become visible
// with them: relaxed device-coherent stores and loads, no L2 write-back.
__device__ __forceinline__ void publish(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long peek(unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// state: [0] ticket, [1] finished workgroups, [2] wait-limit flag; words: [nb].
// `in` may equal `out` (each workgroup reads its own tile before writing it).
__global__ __launch_bounds__(SB) void k_scan(const uint32_t* in, uint32_t* out, int64_t n,
                                             uint32_t* __restrict__ total_out,
                                             uint32_t* __restrict__ state,
                                             unsigned long long* __restrict__ words) {
  __shared__ uint32_t lds[SB / 64];
  __shared__ uint32_t s_tile, s_excl, s_last;
  const uint32_t nb = gridDim.x;
  if (threadIdx.x == 0) s_tile = atomicAdd(&state[0], 1u);
  __syncthreads();
  const uint32_t b = s_tile;
  const int64_t base = (int64_t)b * SE + (int64_t)threadIdx.x * SI;
  uint32_t v[SI];
  uint32_t s = 0;
  const bool full = base + SI <= n;  // whole 64-byte runs load and store as 16-byte vectors
  if (full) {
#pragma unroll
    for (int i = 0; i < SI; i += 4) {
      const uint4 q = *reinterpret_cast<const uint4*>(in + base + i);
      v[i] = q.x; v[i + 1] = q.y; v[i + 2] = q.z; v[i + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < SI; ++i) v[i] = base + i < n ? in[base + i] : 0u;
  }
#pragma unroll
  for (int i = 0; i < SI; ++i) s += v[i];
  uint32_t agg;
  uint32_t ex = block_excl_scan(s, lds, agg);
  if (threadIdx.x == 0) publish(&words[b], ST_TOTAL | agg);
  // the totals of every earlier tile (published without waiting)
  uint32_t pre = 0;
  for (uint32_t spins = 0;; ++spins) {
    pre = 0;
    bool ok = true;
    for (uint32_t q = threadIdx.x; q < b; q += SB) {
      const unsigned long long w = peek(&words[q]);
      ok = ok && (w & ST_TOTAL) != 0;
      pre += (uint32_t)w;
    }
    if (__syncthreads_and(ok)) break;
    if (spins >= SPIN_LIMIT) {
      if (threadIdx.x == 0) atomicOr(&state[2], 1u);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  uint32_t excl;
  block_excl_scan(pre, lds, excl);
  if (threadIdx.x == 0) {
    s_excl = excl;
    if (b == nb - 1 && total_out) *total_out = excl + agg;
  }
  __syncthreads();
  ex += s_excl;
  uint32_t o[SI];
#pragma unroll
  for (int i = 0; i < SI; ++i) {
    o[i] = ex;
    ex += v[i];
  }
  if (full) {
#pragma unroll
    for (int i = 0; i < SI; i += 4)
      *reinterpret_cast<uint4*>(out + base + i) = make_uint4(o[i], o[i + 1], o[i + 2], o[i + 3]);
  } else {
#pragma unroll
    for (int i = 0; i < SI; ++i)
      if (base + i < n) out[base + i] = o[i];
  }
  // the last workgroup to finish leaves the state clear for the next scan
  // (every workgroup has read all the words it needs before it counts itself)
  if (threadIdx.x == 0) s_last = atomicAdd(&state[1], 1u) == nb - 1 ? 1u : 0u;
  __syncthreads();
  if (s_last) {
    for (uint32_t i = threadIdx.x; i < nb; i += SB) publish(&words[i], 0ull);
    if (threadIdx.x == 0) {
      state[0] = 0u;
      state[1] = 0u;
    }
  }
}

// Two-kernel form for long arrays (the single pass would make every
// workgroup read the totals of all before it): block totals, then a
// down-sweep in which each block first adds up the totals before it. Tiles
// of SB x LI elements (LI per thread, loaded as 16-byte vectors), so that
// the down-sweep's reads of earlier totals stay few.
constexpr int LI = 64;
constexpr int64_t LE = (int64_t)SB * LI;

__device__ __forceinline__ void load_run(const uint32_t* in, int64_t base, int64_t n, uint32_t* v) {
  if (base + LI <= n) {
#pragma unroll
    for (int i = 0; i < LI; i += 4) {
      const uint4 q = *reinterpret_cast<const uint4*>(in + base + i);
      v[i] = q.x; v[i + 1] = q.y; v[i + 2] = q.z; v[i + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < LI; ++i) v[i] = base + i < n ? in[base + i] : 0u;
  }
}

__global__ __launch_bounds__(SB) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                    uint32_t* __restrict__ partial) {
  __shared__ uint32_t lds[SB / 64];
  const int64_t base = (int64_t)blockIdx.x * LE + (int64_t)threadIdx.x * LI;
  uint32_t v[LI];
  load_run(in, base, n, v);
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < LI; ++i) s += v[i];
  uint32_t total;
  block_excl_scan(s, lds, total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

__global__ __launch_bounds__(SB) void k_scan_down(const uint32_t* in, uint32_t* out, int64_t n,
                                                  const uint32_t* __restrict__ partial,
                                                  uint32_t* __restrict__ total_out) {
  __shared__ uint32_t lds[SB / 64];
  uint32_t s = 0;
  for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += SB) s += partial[b];
  uint32_t pre;
  block_excl_scan(s, lds, pre);
  const int64_t base = (int64_t)blockIdx.x * LE + (int64_t)threadIdx.x * LI;
  uint32_t v[LI];
  load_run(in, base, n, v);
  s = 0;
#pragma unroll
  for (int i = 0; i < LI; ++i) s += v[i];
  uint32_t total;
  uint32_t ex = block_excl_scan(s, lds, total) + pre;
  if (base + LI <= n) {
#pragma unroll
    for (int i = 0; i < LI; i += 4) {
      uint4 q;
      q.x = ex; ex += v[i];
      q.y = ex; ex += v[i + 1];
      q.z = ex; ex += v[i + 2];
      q.w = ex; ex += v[i + 3];
      *reinterpret_cast<uint4*>(out + base + i) = q;
    }
  } else {
#pragma unroll
    for (int i = 0; i < LI; ++i) {
      if (base + i < n) out[base + i] = ex;
      ex += v[i];
    }
  }
  if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total_out = pre + total;
}

constexpr int64_t ONE_PASS_MAX_BLOCKS = 192;

}  // namespace

int64_t scan_blocks(int64_t n) { return (n + SE - 1) / SE; }

// state (16 bytes), one published word per tile of a single-pass scan, and
// the block totals of a two-kernel scan
size_t scan_scratch_bytes(int64_t n) {
  return 16 + (size_t)std::min<int64_t>(scan_blocks(n), ONE_PASS_MAX_BLOCKS) * 8 +
         (size_t)scan_blocks(n) * 4;
}

size_t scan_state_words(int64_t n) {
  return (16 + (size_t)std::min<int64_t>(scan_blocks(n), ONE_PASS_MAX_BLOCKS) * 8) / 4;
}

void scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, void* scratch,
              hipStream_t st) {
  if (n <= 0) return;
  const int64_t nb = scan_blocks(n);
  if (nb > ONE_PASS_MAX_BLOCKS) {
    // fewer, larger tiles: the totals array (sized for nb) has room for them
    const int64_t nl = (n + LE - 1) / LE;
    uint32_t* partial = (uint32_t*)((char*)scratch + 16 + ONE_PASS_MAX_BLOCKS * 8);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nl), dim3(SB), 0, st, in, n, partial);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nl), dim3(SB), 0, st, in, out, n,
                       (const uint32_t*)partial, total);
    return;
  }
  uint32_t* state = (uint32_t*)scratch;
  unsigned long long* words = (unsigned long long*)((char*)scratch + 16);
  hipLaunchKernelGGL(k_scan, dim3((unsigned)nb), dim3(SB), 0, st, in, out, n, total, state, words);
}

}  // namespace hr
