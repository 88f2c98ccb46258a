// Internal definitions shared by the HIP translation units of libhybrid_raster.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hr.h"

namespace hr {

constexpr int TILE = 16;        // pixels per tile side
constexpr int TILE_PIX = 256;   // pixels per tile = threads per blend workgroup
constexpr int CHUNK = 2048;     // depth ranks per binning chunk
// keys per radix-sort workgroup (its histogram column): short sorts gain from
// more workgroups, long ones (several cameras) from fewer histogram columns
inline int rs_keys_for(int64_t n_items) { return n_items <= (int64_t)2 << 20 ? 1024 : 4096; }
constexpr int SORT_WIN = 8192;  // ranks one workgroup sorts in LDS at once
constexpr int SUBPIX = 256;     // fixed-point steps per pixel for mesh vertices
constexpr int64_t GUARD = (int64_t)1 << 29;  // |vertex| bound in fixed point (2^21 px)
constexpr int MAX_TILE_COLS = 1024;       // 16384 px / 16
constexpr int MAX_TILES_PER_CAM = 16384;     // LDS tile histogram of the binning kernels
constexpr float LOG2E = 1.4426950408889634f;

// Camera as the kernels see it.
// floor of the determinant ratio of the Mip-Splatting 2D filter
constexpr double MIP2D_FLOOR = 2.5e-5;
constexpr float LN2F = 0.69314718055994531f;

struct CamDev {
  double fx, fy, cx, cy;
  double R[9];
  double t[3];
  double C[3];       // camera centre in world space
  double limx, limy; // Jacobian clamp of x/z and y/z
  int32_t W, H, TX, TY;
  int32_t tile_off;  // first global tile id
  int32_t chunk_rows;// rows of this camera's chunk-count matrix (ceil(n / CHUNK))
  int64_t pix_off;   // first packed pixel
  int64_t row_off;   // first chunk row (global chunk index)
  int64_t mat_off;   // first entry of this camera's chunk-count matrix
};

struct SetDev {
  float bg[3];
  float low_pass, alpha_min, alpha_max, t_min, near_gs, near_mesh, clamp_fov;
  int32_t n, sh_degree, n_cams, n_faces, n_verts;
  int32_t n_tex, tex_h, tex_w;
  int32_t n_tiles;   // over all cameras
  int32_t max_tiles_cam;  // largest tile count of one camera
  int64_t n_pix;     // over all cameras
  int64_t key_cap;
  const float* filter3d;  // [n] Mip-Splatting 3D smoothing variance, or null
  int32_t mip2d;          // Mip-Splatting 2D filter with opacity compensation
};

// Projected Gaussian as the blend reads it (48 bytes, FP32).
struct alignas(16) GRec {
  float u, v, ca, cb;   // mean2D; conic [[ca, cb], [cb, cc]]
  float cc, op, depth, pad;
  float r, g, b;
  uint32_t gid;
};

// Clipped, snapped triangle of one camera.
struct alignas(16) TriRec {
  int32_t X[3], Y[3];   // vertices in 1/256 px, counter-clockwise (positive area)
  double iz[3];         // 1 / view depth of each vertex
  double uv[3][2];
  int32_t face, tex, cam, pad;
  int32_t bx0, by0, bx1, by1;  // raster blocks (RBLK x RBLK pixels) covered by the bbox (inclusive)
};

// ----------------------------------------------------------- wave tools --
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ uint32_t f2u(float f) { return __float_as_uint(f); }

// DPP lane move (row_mask/bank_mask select written rows/banks; lanes that have
// no source or are not written read 0)
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, true));
}

// Sum over the 64 lanes of a wave, complete in lane 63: shifts by 1, 2, 4, 8
// within each row of 16 lanes, then row 0 -> row 1 and row 2 -> row 3
// (broadcast of lane 15), then rows 0-1 -> rows 2-3 (broadcast of lane 31).
// Sum over each row of 16 lanes, complete in the row's last lane (15, 31, 47, 63).
__device__ __forceinline__ float row_sum_to_last(float v) {
  v += dpp_f<0x111>(v);
  v += dpp_f<0x112>(v);
  v += dpp_f<0x114>(v);
  v += dpp_f<0x118>(v);
  return v;
}

__device__ __forceinline__ float wave_sum_to_last(float v) {
  v += dpp_f<0x111>(v);
  v += dpp_f<0x112>(v);
  v += dpp_f<0x114>(v);
  v += dpp_f<0x118>(v);
  v += dpp_f<0x142, 0xa>(v);
  v += dpp_f<0x143, 0xc>(v);
  return v;
}

}  // namespace hr

// Launch wrappers implemented in the .hip files (host side).
namespace hr {

// generic exclusive scan over n elements (n may exceed what is used; the tail
// must be 0); the scratch holds its state, which must be zero before the first
// scan (the forward's camera upload clears scan_state_words of it)
size_t scan_scratch_bytes(int64_t n);
size_t scan_state_words(int64_t n);
void scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, void* scratch,
              hipStream_t st);

}  // namespace hr
