// Workspace view and launch wrappers of the HIP kernels (host side).
#pragma once

#include "common.hpp"

namespace hr {

// Per-rank part of the tile-ellipse test: determinant of the conic, grown
// radius^2 rp (+inf keeps the rectangle, < 0 empties it), half-height of the
// ellipse and the scale of its x-extreme points.
struct EllP {
  double det, rp, dymax, sc;
};

// Device pointers into the caller's workspace (see plan.cpp for the layout).
struct Work {
  CamDev* cams;          // [n_cams]
  // per (camera, Gaussian) item, M = n_cams * n
  uint32_t* vis;         // [M] 1 = visible
  uint32_t* vis_scan;    // [M] exclusive scan of vis
  uint32_t* dkey;        // [M] fp32 depth bits
  GRec* rec;             // [M]
  uint2* rect;           // [M] packed tile rectangle
  int32_t* rank_of;      // [M] depth rank, -1 = culled
  // depth sort (radix, ping-pong; rs_blocks blocks of keys) and per-rank arrays
  uint32_t* skey[2];     // [M]
  uint32_t* sval[2];     // [M]
  int64_t rs_blocks;
  // one-dispatch radix passes: per pass a ticket, the global digit counts
  // (digit 0 from the compaction, digit p + 1 from pass p), and the published
  // digit counts of every block and of every group of RS_GROUP blocks; the
  // compaction clears the part of rs1 the passes use, the camera upload
  // clears rs_ghist
  uint32_t* rs1;         // [rs1_words]: tickets | group counters | group counts | block counts
  int64_t rs1_words;
  uint32_t* rs_ghist;    // [RS_MAX_PASSES][RS_GHIST_COPIES][256]
  uint32_t* rs_hist;     // [RS_MAX_PASSES][RSC_MAX_BLOCKS][256] slice counts of the grid-barrier sort
  int64_t rs_groups;     // ceil(rs_blocks / RS_GROUP)
  uint32_t* vis_off;     // [n_cams + 1] first rank of each camera
  GRec* rec_s;           // [M] by rank
  uint2* rect_s;         // [M] by rank
  uint32_t* item_s;      // [M] item of each rank
  EllP* ell_s;           // [M] by rank; shares the memory of gacc (forward only)
  // tile binning
  uint32_t* mat;         // chunk x tile counts, then column prefixes
  int64_t chunk_rows;    // total chunk rows
  int64_t bin_items_max; // (chunk, tile row) binning items if every chunk were used
  uint32_t* item_off;    // [n_cams + 1] first binning item of each camera, then the total
  uint32_t* tile_total;  // [n_tiles]
  uint32_t* tile_start;  // [n_tiles]
  uint32_t* tile_order;  // [n_tiles] blend schedule, longest lists first
  uint32_t* sched_cnt;   // [ceil(n_tiles / 256)][33] schedule bucket counts per block of tiles
  unsigned long long* sched_sum;  // [ceil(n_tiles / 256)] pairs per block of tiles
  uint32_t* tile_dmax;   // [n_tiles] largest mesh depth bits over the tile (culling)
  uint64_t* tile_np;     // [2 * n_tiles] examined and blended pairs of each tile (forward)
  uint32_t* lists;       // [key_cap] ranks grouped by tile, chunk sub-segments in chunk order
  uint32_t* runs;        // [key_cap] the count pass's tile runs, packed, unit after unit
  uint2* unit_runs;      // [bin_items_max] first run and run count of each binning unit
  // counters: [0] n_vis, [1] overflow, [2..3] K = pairs in the tile lists (u64),
  // [4] n_tris, [5] n_blocks, [14] tile queue
  uint32_t* counters;
  // mesh
  uint64_t* zbuf;        // [P] fp32 depth bits << 32 | triangle index
  uint32_t* tri_cnt;     // [n_cams * F]
  uint32_t* blk_cnt;     // [n_cams * F]
  uint32_t* tri_off;     // [n_cams * F]
  uint32_t* blk_off;     // [n_cams * F + 1]
  TriRec* tris;          // [2 * n_cams * F]
  // per pixel, kept for the backward
  float* final_T;        // [P]
  int32_t* n_contrib;    // [P]
  float* mesh_rgb;       // [3P]
  uint4* taps;           // [P] bilinear footprint of each mesh pixel (pack_taps)
  // backward accumulators, [M][9] by rank: u, v, conic a b c, opacity, r g b
  float* gacc;
  // scratch of the scans (its first scan_words words are the scan state)
  void* scan_scratch;
  void* scan_scratch2;  // the same for the mesh pass on the second stream
  int64_t scan_words;
};

constexpr int RUN_ALLOC = 24;     // counters slot: runs handed out to the binning units
constexpr int RS_MAX_PASSES = 6;  // 4 depth bytes, up to 2 camera bytes
constexpr int RS_GROUP = 32;      // blocks per published group total
constexpr int RSC_MAX_BLOCKS = 64;  // workgroups of the grid-barrier sort (all resident)
// copies of the global digit counts: workgroup w adds into copy w % 16, so
// that the few digits every workgroup holds (the exponent byte of the depths)
// do not serialise all of their atomics on one address
constexpr int RS_GHIST_COPIES = 16;
// words of the one-dispatch radix state for rs_blocks blocks of keys
inline int64_t rs1_words_for(int64_t rs_blocks) {
  const int64_t groups = (rs_blocks + RS_GROUP - 1) / RS_GROUP;
  return 8 + RS_MAX_PASSES * groups + (int64_t)RS_MAX_PASSES * 256 * (groups + rs_blocks);
}

// host launch wrappers (all asynchronous on `st`)
void launch_project(const SetDev& S, const CamDev* cams, const hr_gaussians& g, const Work& w,
                    int32_t* radii, hipStream_t st);
void launch_depth_sort(const SetDev& S, const Work& w, bool ell, hipStream_t st);
void launch_binning(const SetDev& S, const Work& w, int n_cams, bool cull, bool ell,
                    hr_outputs* out, hipStream_t st);
void launch_tile_dmax(const SetDev& S, const Work& w, hipStream_t st);
void launch_mesh(const SetDev& S, const hr_mesh& m, const Work& w, hr_outputs* out,
                 hipStream_t st);
void launch_blend_forward(const SetDev& S, const Work& w, hr_outputs* out, int batch, int variant,
                          hipStream_t st, bool shade = false, const float* tex = nullptr);
void launch_blend_backward(const SetDev& S, const Work& w, const float* grad_image,
                           const float* grad_T, int batch, int variant, hipStream_t st);
void launch_project_backward(const SetDev& S, const CamDev* cams, const hr_gaussians& g,
                             const Work& w, hr_grads* grads, hipStream_t st);
void launch_texture_backward(const SetDev& S, const hr_mesh& m, const Work& w,
                             const float* grad_image, const float* grad_mesh_rgb, float* grad_tex,
                             hipStream_t st);
// loss over n_img packed planar images of img_pix[i] pixels each (host array)
size_t loss_scratch_bytes(int64_t n_pix, int32_t n_img);
void launch_loss(const float* image, const float* T, const float* mesh_rgb, const int32_t* tri,
                 const float* target, const int64_t* img_pix, int32_t n_img, float lambda_t,
                 float k, bool detach, float* loss, float* g_image, float* g_T, float* g_mesh,
                 void* scratch, hipStream_t st);
// device address of the library's static loss scratch on the current device
// (looked up once per device); its size in bytes
hr_status loss_static_scratch_ptr(void** out);
size_t loss_static_scratch_bytes();
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
void launch_adam(const hr_adam_group* groups, int n_groups, double b1, double b2, double eps,
                 int step, hipStream_t st);
size_t full_loss_scratch_bytes(int64_t n_pix, int64_t n_tiles, int32_t n_imgs);
void launch_full_loss(const float* image, const float* T, const float* mesh, const int32_t* tri,
                      const float* target, const int32_t* sizes, int32_t n_imgs, float lambda_c,
                      float lambda_t, float k, int mask_mode, bool detach, float* loss,
                      float* g_image, float* g_T, float* g_mesh, void* scratch, hipStream_t st);

// camera upload by kernel argument (graph-capturable, no host staging buffer)
constexpr int CAMS_PER_UPLOAD = 16;
struct CamUpload {
  CamDev c[CAMS_PER_UPLOAD];
  int32_t first, count;
};
static_assert(sizeof(CamUpload) + 8 <= 4096, "camera upload must fit in kernel arguments");
void launch_upload_cams(const CamUpload& u, CamDev* dst, uint32_t* clear, uint32_t* clear2,
                        uint32_t* clear3, int64_t n2, uint32_t* ghist, hipStream_t st);
void launch_mip_filter3d(const float* means, int n, const CamDev* cams, int n_cams, float near,
                         double scale, float* f3, hipStream_t st);
// scan1, scan2: the two scan scratch states (word 2 = bounded wait gave up)
void launch_counters_to_stats(const uint32_t* counters, const uint64_t* tile_np, int n_tiles,
                              const uint32_t* scan1, const uint32_t* scan2, hr_stats* stats,
                              hipStream_t st);
void launch_zero_gacc(float* gacc, const uint32_t* counters, hipStream_t st);
void launch_count_mismatch(const float* a, const float* b, int64_t n, uint32_t* out,
                           hipStream_t st);
void launch_fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t st);
// out[0] = sum (a - b)^2, out[1] = sum b^2 (FP64 device scalars)
void launch_sq_diff(const float* a, const float* b, int64_t n, double* out, hipStream_t st);
// dst[i] = src[i] for i < count[0] * per (count on the device)
void launch_copy_counted(const float* src, float* dst, const uint32_t* count, int per,
                         hipStream_t st);

}  // namespace hr
