// Small helper kernels of the host runtime: camera upload through kernel
// arguments, statistics export, accumulator clearing, output comparison.
#include "kernels.hpp"

namespace hr {

namespace {

// also clears the 64 forward counters, `n2` words of each of the two scan
// states and the radix sort's global digit counts when `clear` is given
__global__ __launch_bounds__(1024) void k_upload_cams(CamUpload u, CamDev* dst, uint32_t* clear, uint32_t* clear2,
                              uint32_t* clear3, int64_t n2, uint32_t* ghist) {
  const int k = threadIdx.x;
  if (k < u.count) dst[u.first + k] = u.c[k];
  if (!clear) return;
  if (k < 64) clear[k] = 0u;
  for (int64_t i = k; i < n2; i += blockDim.x) {
    clear2[i] = 0u;
    clear3[i] = 0u;
  }
  if (ghist)
    for (int i = k; i < 256 * RS_MAX_PASSES * RS_GHIST_COPIES; i += blockDim.x) ghist[i] = 0u;
}

// one group of 1024 threads: the counters, and the examined / blended pairs
// summed over the per-tile sums of the blend
__global__ __launch_bounds__(1024) void k_counters_to_stats(const uint32_t* __restrict__ c,
                                                            const uint64_t* __restrict__ tile_np,
                                                            int n_tiles,
                                                            const uint32_t* __restrict__ scan1,
                                                            const uint32_t* __restrict__ scan2,
                                                            hr_stats* __restrict__ s) {
  __shared__ unsigned long long part[2][16];
  // one 16-byte load per tile, four tiles in flight per thread
  const ulonglong2* __restrict__ np2 = reinterpret_cast<const ulonglong2*>(tile_np);
  unsigned long long sp = 0, sb = 0;
  const int step = (int)blockDim.x;
  int t = threadIdx.x;
  for (; t + 3 * step < n_tiles; t += 4 * step) {
    ulonglong2 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = np2[t + q * step];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sp += v[q].x;
      sb += v[q].y;
    }
  }
  for (; t < n_tiles; t += step) {
    const ulonglong2 v = np2[t];
    sp += v.x;
    sb += v.y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sp += __shfl_xor(sp, o, 64);
    sb += __shfl_xor(sb, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if (__lane_id() == 0) {
    part[0][w] = sp;
    part[1][w] = sb;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  sp = sb = 0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
    sp += part[0][k];
    sb += part[1][k];
  }
  s->n_visible = c[0];
  s->overflow = c[1];
  const uint64_t K = (uint64_t)c[2] | ((uint64_t)c[3] << 32);
  s->n_keys = K > 0xffffffffull ? 0xffffffffu : (uint32_t)K;
  s->n_tris = c[4];
  s->n_processed = sp;
  s->n_blended = sb;
  s->wait_limit = (scan1[2] | scan2[2]) != 0u ? 1u : 0u;
  s->reserved = 0u;
}

// clears the [n_visible][9] gradient accumulators
__global__ void k_zero_gacc(float* __restrict__ gacc, const uint32_t* __restrict__ counters) {
  const int64_t n = (int64_t)counters[0] * 9;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    gacc[i] = 0.f;
}

__global__ void k_count_mismatch(const float* __restrict__ a, const float* __restrict__ b,
                                 int64_t n, uint32_t* __restrict__ out) {
  uint32_t bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    bad += __float_as_uint(a[i]) != __float_as_uint(b[i]);
  if (bad) atomicAdd(out, bad);
}

// sums of (a - b)^2 and b^2 over n values (out[0], out[1]; cleared before)
__global__ void k_sq_diff(const float* __restrict__ a, const float* __restrict__ b, int64_t n,
                          double* __restrict__ out) {
  double d2 = 0.0, b2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double d = (double)a[i] - (double)b[i];
    d2 += d * d;
    b2 += (double)b[i] * (double)b[i];
  }
  for (int o = 32; o > 0; o >>= 1) {
    d2 += __shfl_xor(d2, o, 64);
    b2 += __shfl_xor(b2, o, 64);
  }
  if (__lane_id() == 0) {
    atomicAdd(&out[0], d2);
    atomicAdd(&out[1], b2);
  }
}

__global__ void k_copy_f32(const float* __restrict__ src, float* __restrict__ dst,
                           const uint32_t* __restrict__ count, int per) {
  const int64_t n = (int64_t)count[0] * per;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

}  // namespace

void launch_sq_diff(const float* a, const float* b, int64_t n, double* out, hipStream_t st) {
  launch_fill_u64((uint64_t*)out, 0ull, 2, st);
  if (n <= 0) return;
  int64_t g = (n + 255) / 256;
  if (g > 2048) g = 2048;
  hipLaunchKernelGGL(k_sq_diff, dim3((unsigned)g), dim3(256), 0, st, a, b, n, out);
}

void launch_copy_counted(const float* src, float* dst, const uint32_t* count, int per,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_copy_f32, dim3(2048), dim3(256), 0, st, src, dst, count, per);
}

void launch_upload_cams(const CamUpload& u, CamDev* dst, uint32_t* clear, uint32_t* clear2,
                        uint32_t* clear3, int64_t n2, uint32_t* ghist, hipStream_t st) {
  hipLaunchKernelGGL(k_upload_cams, dim3(1), dim3(1024), 0, st, u, dst, clear, clear2, clear3, n2,
                     ghist);
}

void launch_counters_to_stats(const uint32_t* counters, const uint64_t* tile_np, int n_tiles,
                              const uint32_t* scan1, const uint32_t* scan2, hr_stats* stats,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_counters_to_stats, dim3(1), dim3(1024), 0, st, counters, tile_np, n_tiles,
                     scan1, scan2, stats);
}

void launch_zero_gacc(float* gacc, const uint32_t* counters, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_gacc, dim3(2048), dim3(256), 0, st, gacc, counters);
}

void launch_count_mismatch(const float* a, const float* b, int64_t n, uint32_t* out,
                           hipStream_t st) {
  if (n <= 0) return;
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_count_mismatch, dim3((unsigned)g), dim3(256), 0, st, a, b, n, out);
}

}  // namespace hr
