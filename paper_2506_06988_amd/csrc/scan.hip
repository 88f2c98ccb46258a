// Exclusive prefix sums over device arrays (reduce, scan of block sums, downsweep).
// Every size is a host-side maximum; entries past the used part must be zero,
// so data-dependent lengths need no host synchronisation.
#include "common.hpp"

namespace hr {
namespace {

constexpr int SB = 256;        // threads per block
constexpr int SI = 8;          // elements per thread
constexpr int SE = SB * SI;    // elements per block

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int l = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T u = __shfl_up(v, o, 64);
    if (l >= o) v += u;
  }
  return v;
}

// exclusive scan of one value per thread over the 256-thread block; returns the block total
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* lds4, T& total) {
  const int w = threadIdx.x >> 6, l = __lane_id();
  T inc = wave_incl_scan(v);
  if (l == 63) lds4[w] = inc;
  __syncthreads();
  T base = 0;
  total = 0;
#pragma unroll
  for (int k = 0; k < SB / 64; ++k) {
    T s = lds4[k];
    if (k < w) base += s;
    total += s;
  }
  __syncthreads();
  return base + inc - v;
}

template <typename T>
__global__ __launch_bounds__(SB) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                    T* __restrict__ partial) {
  __shared__ T lds[SB / 64];
  const int64_t base = (int64_t)blockIdx.x * SE + (int64_t)threadIdx.x * SI;
  T s = 0;
#pragma unroll
  for (int i = 0; i < SI; ++i)
    if (base + i < n) s += in[base + i];
  T total;
  block_excl_scan<T>(s, lds, total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Down-sweep: each block first sums the block totals before it (a few hundred
// at most, read cooperatively), then scans its own elements; the last block
// writes the grand total. With one block there is no partial array.
template <typename T>
__global__ __launch_bounds__(SB) void k_scan_down(const uint32_t* __restrict__ in, T* __restrict__ out,
                                                  int64_t n, const T* __restrict__ partial,
                                                  T* __restrict__ total_out) {
  __shared__ T lds[SB / 64];
  T pre = 0;
  if (partial) {
    T s = 0;
    for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += SB) s += partial[b];
    T tot;
    block_excl_scan<T>(s, lds, tot);
    pre = tot;
  }
  const int64_t base = (int64_t)blockIdx.x * SE + (int64_t)threadIdx.x * SI;
  uint32_t v[SI];
  T s = 0;
#pragma unroll
  for (int i = 0; i < SI; ++i) {
    v[i] = base + i < n ? in[base + i] : 0u;
    s += v[i];
  }
  T total;
  T ex = block_excl_scan<T>(s, lds, total) + pre;
#pragma unroll
  for (int i = 0; i < SI; ++i) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
  if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total_out = pre + total;
}

template <typename T>
void scan_impl(const uint32_t* in, T* out, int64_t n, T* total, void* scratch, hipStream_t st) {
  if (n <= 0) return;
  const int64_t nb = (n + SE - 1) / SE;
  T* partial = nb > 1 ? (T*)scratch : nullptr;
  if (partial)
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)nb), dim3(SB), 0, st, in, n, partial);
  hipLaunchKernelGGL(k_scan_down<T>, dim3((unsigned)nb), dim3(SB), 0, st, in, out, n,
                     (const T*)partial, total);
}

}  // namespace

size_t scan_scratch_bytes(int64_t n) {
  const int64_t nb = (n + SE - 1) / SE;
  return (size_t)(nb + 1) * sizeof(uint64_t);
}

void scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, void* scratch,
              hipStream_t st) {
  scan_impl<uint32_t>(in, out, n, total, scratch, st);
}

void scan_u64(const uint32_t* in, uint64_t* out, int64_t n, uint64_t* total, void* scratch,
              hipStream_t st) {
  scan_impl<uint64_t>(in, out, n, total, scratch, st);
}

}  // namespace hr
