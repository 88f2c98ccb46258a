/*
 * hr.h - C ABI of the MI355X hybrid mesh-Gaussian rasterizer (libhybrid_raster.so).
 *
 * The library renders the hybrid representation of "Hybrid Mesh-Gaussian
 * Representation for Efficient Indoor Scene Reconstruction" (arXiv 2506.06988):
 *   - 3D Gaussians: centre, opacity, rotation, scale and SH colour, with
 *     Sigma = R S S^T R^T projected to Sigma' = J W Sigma W^T J^T      (Sec. 3.1, Eq. 1)
 *   - front-to-back alpha blending over depth-sorted Gaussians        (Sec. 3.1, Eq. 2)
 *   - an opaque textured mesh rendered with barycentric UVs           (Sec. 3.1 "Textured mesh")
 *   - joint rasterization: the mesh gives I_m and D_m, only Gaussians
 *     with D_gs < D_m are blended and the residual transmittance T
 *     weights I_m (or the background)                                  (Sec. 3.4 "Joint optimization", paragraph "Joint rasterization")
 *   - gradients to every Gaussian parameter and to the texture map,
 *     none to mesh vertices                                            (Sec. 3.4)
 *   - the loss L1 + lambda * M_T * ||I~ - I~_m||^2                     (Sec. 3.4, transmittance-aware supervision)
 *
 * Conventions the paper inherits from its 3DGS code base without stating
 * them are fields of hr_settings: 16x16 pixel tiles, 3-sigma extent, the
 * 0.3 px^2 low-pass, alpha in [1/255, 0.99], the 1e-4 transmittance stop,
 * the 0.2 Gaussian near plane, the 1.3 x FOV clamp of the Jacobian and the
 * SH colour offset of 0.5 clamped at 0.
 *
 * Geometry: world and camera axes are x right, y down, z forward;
 * p_cam = R p_world + t; the pixel (i, j) is sampled at (i + 1/2, j + 1/2).
 *
 * Memory and ownership
 *   - Every array pointer is DEVICE memory owned by the caller, except the
 *     hr_camera array, which is host memory read during the call.
 *   - The library never allocates or frees device memory except inside
 *     hr_batch_create/hr_batch_destroy (documented there), and keeps no state
 *     between calls other than one internal stream and two events per device,
 *     created on first use and kept until the process ends. All intermediate
 *     state lives in the caller's workspace, sized by hr_query_workspace. The
 *     forward's workspace contents are the saved context of the matching
 *     backward call.
 *   - All work is ordered on the given stream (hipStream_t passed as void*;
 *     NULL = the null stream); calls return before the GPU finishes. The
 *     forward and backward fork independent parts onto the internal stream
 *     (after an event recorded on the given stream) and join them back (the
 *     given stream waits on an event) before their last kernels, so work
 *     enqueued later on the given stream sees every result; a graph capture
 *     of the given stream includes both branches. Calls that share a device
 *     share the internal stream, which serialises their forked parts.
 *   - Several cameras are rendered by one call. Their pixels are packed one
 *     camera after another: camera c starts at pixel offset
 *     P_c = sum_{c'<c} W_c' H_c'; images are planar [3, H_c, W_c] at 3 P_c.
 *
 * Errors
 *   - Every entry point returns hr_status and never aborts or throws.
 *   - Arguments are checked before anything is enqueued; on
 *     HR_ERR_INVALID_ARGUMENT nothing is written. hr_last_error() returns a
 *     thread-local description of the last failure.
 *   - When the pair count exceeds the workspace's key capacity the outputs
 *     are undefined (no write leaves the workspace or the outputs), the
 *     device flag hr_stats.overflow is set and, unless HR_FLAG_NO_SYNC is
 *     given, the call synchronises the stream once and returns
 *     HR_ERR_CAPACITY with hr_stats.n_keys holding the needed count. The same
 *     synchronisation reports HR_ERR_INTERNAL when hr_stats.wait_limit is set.
 *     A replayed graph (hr_batch_launch) never synchronises: hr_batch_status
 *     reads both flags after the replay.
 *   - Non-finite Gaussian parameters cull that Gaussian; degenerate triangles
 *     are skipped; n = 0 and n_faces = 0 are legal.
 */
#ifndef HR_H_
#define HR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HR_ABI_VERSION 2

typedef enum {
  HR_OK = 0,
  HR_ERR_INVALID_ARGUMENT = 1,
  HR_ERR_CAPACITY = 2,
  HR_ERR_HIP = 3,
  HR_ERR_UNSUPPORTED = 4,
  HR_ERR_INTERNAL = 5
} hr_status;

/* Gaussian set (Sec. 3.1): n Gaussians, structure of arrays, FP32. */
typedef struct {
  int32_t n;               /* >= 0 */
  int32_t sh_degree;       /* 0..3; K = (sh_degree + 1)^2 coefficients */
  const float* means;      /* [n,3] world centre u */
  const float* log_scales; /* [n,3] S = diag(exp(log_scales)) */
  const float* quats;      /* [n,4] (w,x,y,z), normalised by the library */
  const float* opacity_logits; /* [n] opacity = sigmoid(logit) */
  const float* sh;         /* [n,K,3] real SH coefficients per channel */
  /* [n] Mip-Splatting 3D smoothing variance (world units^2), or null for none:
   * Sigma + f3 I, opacity scaled by prod_i s_i / sqrt(s_i^2 + f3). A negative
   * or non-finite entry culls its Gaussian. See hr_mip_filter3d. */
  const float* filter3d;
} hr_gaussians;

/* Textured triangle mesh (Sec. 3.1 "Textured mesh"). Each face corner has
 * its own UV; texel (i, j) of a W x H texture is centred at
 * ((i + 1/2)/W, (j + 1/2)/H), row 0 at V = 0, clamped at the edges. */
typedef struct {
  int32_t n_verts, n_faces; /* n_faces = 0: no mesh (Gaussians over bg) */
  int32_t n_tex, tex_h, tex_w;
  const float* verts;      /* [n_verts,3] */
  const int32_t* faces;    /* [n_faces,3] vertex indices */
  const float* uvs;        /* [n_faces,3,2] */
  const int32_t* face_tex; /* [n_faces] texture index in [0, n_tex) */
  const float* tex;        /* [n_tex,tex_h,tex_w,3] RGB, FP32 */
} hr_mesh;

/* Pinhole camera, host memory. */
typedef struct {
  int32_t width, height;
  double fx, fy, cx, cy;
  double R[9]; /* world -> camera rotation, row-major */
  double t[3];
} hr_camera;

enum {
  HR_FLAG_NO_SYNC = 1u << 0,      /* never synchronise to check the capacity */
  HR_FLAG_DETACH_MASK = 1u << 1,  /* loss: no gradient through M_T */
  HR_FLAG_EXPORT_KEYS = 1u << 2,  /* forward: fill hr_outputs.keys/values/ranges */
  /* forward: leave out of the tile lists every (Gaussian, tile) pair whose
   * fp32 depth is >= the largest mesh depth over the tile's pixels (only
   * tiles whose pixels all have a face). Such a Gaussian reaches the depth
   * stop of Sec. 3.4 in every pixel of the tile, so images, T, n_contrib and
   * n_blended are unchanged; n_processed loses the one stopping candidate
   * where it was dropped; keys/ranges, n_keys and the capacity requirement
   * count the kept pairs only. */
  HR_FLAG_CULL_BEHIND_MESH = 1u << 3,
  /* Mip-Splatting 2D filter (the anti-aliased host method of Table 1):
   * low_pass is the pixel filter variance (0.1 for that method) and the
   * opacity is scaled by sqrt(det Sigma' / det(Sigma' + low_pass I)), the
   * ratio floored at 2.5e-5. Forward and backward must agree on it. */
  HR_FLAG_MIP_2D = 1u << 4,
  /* forward: keep a (Gaussian, tile) pair only if the tile's pixel centres
   * meet the ellipse where alpha = opacity * G can reach alpha_min (grown by
   * a margin that covers FP32 evaluation), instead of the whole 3-sigma
   * tile rectangle. The dropped pairs are skipped by every pixel anyway, so
   * images, T and n_blended are unchanged; n_contrib and n_processed are
   * positions in the kept lists; keys/ranges, n_keys and the capacity
   * requirement count the kept pairs. */
  HR_FLAG_TILE_ELLIPSE = 1u << 5,
  /* forward: skip the mesh pass and use the z-buffer, mesh colour and texel
   * footprints the workspace already holds from a forward of the same
   * cameras and mesh (for renders of the Gaussians alone over an unchanged
   * mesh view). The outputs mesh_rgb, mesh_depth and tri_id are not written
   * and hr_stats.n_tris is 0. */
  HR_FLAG_MESH_REUSED = 1u << 6
};

typedef struct {
  float bg[3];        /* I_bg, Sec. 3.4 (default 0) */
  float low_pass;     /* added to the diagonal of Sigma' (0.3) */
  float alpha_min;    /* Gaussians with alpha below are skipped (1/255) */
  float alpha_max;    /* alpha clamp (0.99) */
  float t_min;        /* a pixel stops before T would drop below (1e-4) */
  float near_gs;      /* Gaussians with view z <= near_gs are culled (0.2) */
  float near_mesh;    /* triangles are clipped at view z = near_mesh (0.05) */
  float clamp_fov;    /* Jacobian direction clamp in units of tan(fov/2) (1.3) */
  uint32_t flags;     /* HR_FLAG_* */
  int32_t batch;      /* Gaussians staged in LDS per batch: 32,64,128,256 (0 = tuned default) */
  int32_t variant;    /* blend variant: bit 0 two-deep LDS staging, bit 1 persistent
                         workgroups on a tile queue, bit 2 one 64-lane wave per tile with
                         four pixels per lane (batch 64 or 128; bits 0-1 ignored) - these
                         three chosen by hr_autotune; bit 3 the backward in one wave per
                         tile (chosen by hr_autotune_backward). 0 = default */
  int32_t batch_bwd;  /* Gaussians staged per batch by the backward: 0 (= batch), 32, 64,
                         128, 256 */
} hr_settings;

/* Counters written by the forward (device memory). */
typedef struct {
  uint32_t n_visible;  /* visible (camera, Gaussian) pairs */
  uint32_t n_keys;     /* (tile, Gaussian) pairs, needed key capacity */
  uint32_t overflow;   /* 1 when n_keys exceeded the capacity */
  uint32_t n_tris;     /* visible clipped triangles */
  uint64_t n_processed;/* sum over pixels of list entries examined */
  uint64_t n_blended;  /* sum over pixels of Gaussians blended */
  uint32_t wait_limit; /* 1 when a one-pass prefix sum gave up waiting for another
                          workgroup (a bounded wait that should never end this way):
                          the outputs are undefined; reported as HR_ERR_INTERNAL */
  uint32_t reserved;   /* 0 */
} hr_stats;

/* Outputs of the forward; every pointer is device memory, sized over the
 * packed pixels of all cameras (P = sum W_c H_c) unless stated. */
typedef struct {
  float* image;          /* [3P] planar per camera: I_h, Sec. 3.4 */
  float* final_T;        /* [P]  residual transmittance T */
  float* mesh_rgb;       /* [3P] I_m (0 where no triangle), nullable */
  float* mesh_depth;     /* [P]  D_m, view z of the mesh (+inf where none), nullable */
  int32_t* tri_id;       /* [P]  covering face, -1 where none, nullable */
  int32_t* n_contrib;    /* [P]  1-based list index of the last blended Gaussian, nullable */
  int32_t* n_blended;    /* [P]  Gaussians blended, nullable */
  int32_t* n_processed;  /* [P]  list entries examined incl. the terminating one, nullable */
  int32_t* radii;        /* [n_cams*n] integer 3-sigma radius, 0 = culled, nullable */
  uint64_t* keys;        /* [key_capacity] (global tile << 32 | fp32 depth bits), with EXPORT_KEYS */
  uint32_t* values;      /* [key_capacity] Gaussian index, with EXPORT_KEYS */
  uint32_t* ranges;      /* [n_tiles,2] [start,end) per global tile, with EXPORT_KEYS */
  hr_stats* stats;       /* nullable */
} hr_outputs;

/* Gradients, accumulated (+=) into caller-zeroed device arrays; any may be
 * NULL to skip it. Shapes match hr_gaussians / hr_mesh.tex. */
typedef struct {
  float* means;
  float* log_scales;
  float* quats;
  float* opacity_logits;
  float* sh;
  float* tex;
  /* densification statistics (3DGS-style, in pixel units): for every camera
   * where the Gaussian is visible, |dL/d mean2D| is added to mean2d_norm and
   * 1 to mean2d_count (both [n], nullable) */
  float* mean2d_norm;
  int32_t* mean2d_count;
} hr_grads;

/* hr_settings with the defaults listed above. */
hr_settings hr_default_settings(void);

/* Bytes of workspace the forward/backward pair needs for these inputs and a
 * key capacity (maximum number of (tile, Gaussian) pairs); 0 on invalid
 * arguments. The global tile id of camera c's tile (tx, ty) is
 * T_c + ty * ceil(W_c/16) + tx with T_c the tiles of the cameras before c. */
size_t hr_query_workspace(const hr_gaussians* g, const hr_mesh* mesh, const hr_camera* cams,
                          int32_t n_cams, const hr_settings* s, int64_t key_capacity);

/* Forward joint rasterization (Sec. 3.4) of n_cams cameras:
 * mesh raster -> I_m, D_m; Gaussian projection -> tile binning and depth
 * sort -> per-pixel blend stopping at D_m; I_h = C + T * (I_m or I_bg).
 * `workspace` (workspace_bytes >= hr_query_workspace(...)) keeps the
 * context for hr_render_hybrid_backward. */
hr_status hr_render_hybrid(const hr_gaussians* g, const hr_mesh* mesh, const hr_camera* cams,
                           int32_t n_cams, const hr_settings* s, int64_t key_capacity,
                           void* workspace, size_t workspace_bytes, hr_outputs* out,
                           void* stream);

/* hr_render_hybrid that also times its stages with events, synchronising the
 * stream before it returns (not for graph capture). stage_ms (host,
 * HR_N_STAGES floats) receives milliseconds: on the given stream 0 camera
 * upload and projection, 1 depth sort (visibility scan, compaction, radix
 * passes, gather), 2 tile binning (with the mesh-depth bound when culling,
 * which waits for the mesh), 3 blend (with the shading of the mesh pixels
 * unless the mesh is reused), 4 statistics export; 5 the mesh pass up to the
 * z-buffer on the internal stream (concurrent with 1-2; 0 with
 * HR_FLAG_MESH_REUSED); 6 the
 * whole forward on the given stream. Errors as hr_render_hybrid (the capacity
 * check is always made). */
#define HR_N_STAGES 7
hr_status hr_render_hybrid_timed(const hr_gaussians* g, const hr_mesh* mesh, const hr_camera* cams,
                                 int32_t n_cams, const hr_settings* s, int64_t key_capacity,
                                 void* workspace, size_t workspace_bytes, hr_outputs* out,
                                 void* stream, float* stage_ms);

/* Backward of hr_render_hybrid given upstream gradients of I_h, T and I_m
 * (grad_final_T and grad_mesh_rgb nullable). Blends in reverse order,
 * recovering each T from the stored final T by division, and accumulates
 * gradients to the Gaussian parameters and the texture (Sec. 3.4). Every
 * argument except the gradients must equal the forward's. */
hr_status hr_render_hybrid_backward(const hr_gaussians* g, const hr_mesh* mesh,
                                    const hr_camera* cams, int32_t n_cams, const hr_settings* s,
                                    int64_t key_capacity, void* workspace, size_t workspace_bytes,
                                    const float* grad_image, const float* grad_final_T,
                                    const float* grad_mesh_rgb, hr_grads* grads, void* stream);

/* hr_render_hybrid_backward that also times its stages with events,
 * synchronising the stream before it returns (not for graph capture).
 * stage_ms (host, HR_N_BWD_STAGES floats) receives milliseconds: 0 the blend
 * backward (clearing the accumulators included), 1 the projection backward,
 * 2 the texture backward, 3 the whole backward on the given stream. With
 * serial = 0 the texture backward runs beside the blend backward on the
 * library's second stream, as in hr_render_hybrid_backward; with serial != 0 it
 * runs on the given stream after the projection backward, so that each stage is
 * timed alone. Errors as hr_render_hybrid_backward, plus HR_ERR_INVALID_ARGUMENT
 * for a null stage_ms. */
#define HR_N_BWD_STAGES 4
hr_status hr_render_hybrid_backward_timed(const hr_gaussians* g, const hr_mesh* mesh,
                                          const hr_camera* cams, int32_t n_cams,
                                          const hr_settings* s, int64_t key_capacity,
                                          void* workspace, size_t workspace_bytes,
                                          const float* grad_image, const float* grad_final_T,
                                          const float* grad_mesh_rgb, hr_grads* grads,
                                          void* stream, int32_t serial, float* stage_ms);

/* Re-runs only the per-tile blend and composite of the forward that last
 * filled this workspace (all arguments equal to that forward's), rewriting
 * the same image, T and counts; the mesh colour is the one that forward's
 * shading left in the workspace (mesh_rgb, mesh_depth and tri_id are not
 * written). Used to time the blend kernel on its own and by the autotuner. */
hr_status hr_blend_forward(const hr_gaussians* g, const hr_mesh* mesh, const hr_camera* cams,
                           int32_t n_cams, const hr_settings* s, int64_t key_capacity,
                           void* workspace, size_t workspace_bytes, hr_outputs* out,
                           void* stream);

/* Loss of Sec. 3.4 ("transmittance-aware supervision") over n_images images
 * packed like the renderer's outputs: image i is sizes[2i] wide and
 * sizes[2i+1] high (`sizes` is host memory), its pixels start at
 * P_i = sum_{i'<i} W_i' H_i' in final_T and tri_id and its planar [3, H_i, W_i]
 * colours at 3 P_i in image, mesh_rgb and target. With P = sum W_i H_i:
 *   L = mean_{p,c} |I_h - I| + lambda_t * mean_{p,c} M_T(p) (I~ - I~_m)^2,
 *   M_T = 1 / (1 + exp(-k (T - 1/2))), I~ = I and I~_m = I_m where
 *   tri_id >= 0, else 0 (the means run over 3P values).
 * Writes the loss (device scalar, deterministic reduction) and dL/dI_h,
 * dL/dT (0 with HR_FLAG_DETACH_MASK) and dL/dI_m, laid out like their inputs.
 * One image of n pixels may be given as sizes = {n, 1}. `scratch` holds
 * hr_loss_scratch_bytes(sizes, n_images) bytes of device memory (0 = invalid
 * sizes); its contents need no clearing. Errors: HR_ERR_INVALID_ARGUMENT
 * (null pointer, n_images < 1, a size < 1, more than 2^40 pixels). */
size_t hr_loss_scratch_bytes(const int32_t* sizes, int32_t n_images);
hr_status hr_hybrid_loss(const float* image, const float* final_T, const float* mesh_rgb,
                         const int32_t* tri_id, const float* target, const int32_t* sizes,
                         int32_t n_images, float lambda_t, float k, uint32_t flags,
                         float* loss_out, float* grad_image, float* grad_final_T,
                         float* grad_mesh_rgb, void* scratch, void* stream);

/* hr_hybrid_loss for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid allocation):
 * the same loss, gradients and layout, with the scratch taken from a static
 * device array of the library instead of a caller buffer. At most
 * HR_LOSS_NOALLOC_MAX_IMAGES images and HR_LOSS_NOALLOC_MAX_PIXELS pixels in
 * all (about 0.53 MB of scratch, one copy per GPU, held until the process
 * ends); larger inputs return HR_ERR_INVALID_ARGUMENT. The call allocates and
 * frees nothing. Every call on a GPU uses that GPU's one array: calls that
 * overlap on one GPU (different streams or threads without ordering) race and
 * their results are undefined; calls ordered on one stream are safe. The
 * first call on a device looks up the array's device address (HR_ERR_HIP if
 * that fails). */
#define HR_LOSS_NOALLOC_MAX_IMAGES 256
#define HR_LOSS_NOALLOC_MAX_PIXELS (1 << 26)
hr_status hr_hybrid_loss_noalloc(const float* image, const float* final_T, const float* mesh_rgb,
                                 const int32_t* tri_id, const float* target, const int32_t* sizes,
                                 int32_t n_images, float lambda_t, float k, uint32_t flags,
                                 float* loss_out, float* grad_image, float* grad_final_T,
                                 float* grad_mesh_rgb, void* stream);

/* Mip-Splatting 3D smoothing variance of every Gaussian for a set of
 * training views: scale / nu^2, nu the highest sampling rate fx / z over the
 * views that see the centre beyond settings->near_gs and inside the image
 * widened by 15% on each side; Gaussians no view sees take the largest
 * variance of the seen ones (0 when none is seen). scale is 0.2 for that
 * method. filter3d_out: device [n], written. Any number of cameras. */
hr_status hr_mip_filter3d(const hr_gaussians* gaussians, const hr_camera* cams, int32_t n_cams,
                          const hr_settings* settings, double scale, float* filter3d_out,
                          void* stream);

/* One Adam step (Kingma and Ba, with bias correction) over several parameter
 * groups: the joint optimisation of Sec. 3.4 / Alg. 1 updates the Gaussians and
 * the texture map together. Per element, with g the gradient:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).
 * lr is per group; when row > 0, elements whose index modulo row is below
 * head use lr_head instead (the SH array: the degree-0 coefficients, 3 floats
 * of every row of 3(d+1)^2, take a larger rate than the higher orders).
 * The betas come in double so that 1-b1, 1-b2 and the bias corrections are
 * formed before rounding to FP32 (1-0.999 rounded from an FP32 0.999 is off
 * by 1.3e-5 relative).
 * `groups` is host memory (at most HR_ADAM_MAX_GROUPS); every array is device
 * memory of n floats, updated in place; grad is only read. Groups must not
 * overlap. Errors: HR_ERR_INVALID_ARGUMENT (null array with n > 0, n < 0,
 * step < 1, betas outside [0,1), eps <= 0, head > row). */
#define HR_ADAM_MAX_GROUPS 8
typedef struct {
  float* param;
  const float* grad;
  float* m;
  float* v;
  int64_t n;
  float lr;
  float lr_head;
  int32_t head;
  int32_t row;
} hr_adam_group;
hr_status hr_adam_step(const hr_adam_group* groups, int32_t n_groups, double beta1, double beta2,
                       double eps, int32_t step, void* stream);

/* Photometric loss of Eq. 3 with the transmittance-aware term of Sec. 3.4,
 * over n_images images packed like the renderer's outputs (image i is
 * sizes[2i] wide and sizes[2i+1] high; `sizes` is host memory):
 *   L = (1 - lambda_c) mean|I_h - I| + lambda_c (1 - mean SSIM(I_h, I))
 *       + lambda_t mean_{p,c} M_T(p) (I~ - I~_m)^2
 * SSIM per channel with an 11x11 Gaussian window (sigma 1.5) over zero-padded
 * images, C1 = 0.01^2, C2 = 0.03^2 (the paper's lambda_c is 0.2). mask_mode
 * selects M_T as in the ablation of Table 3: 0 no L_t term, 1 M_T = 1,
 * 2 M_T = T, 3 M_T = 1 / (1 + exp(-k (T - 1/2))). Writes the loss (device
 * scalar) and dL/dI_h, dL/dT, dL/dI_m. `scratch` holds
 * hr_full_loss_scratch_bytes(sizes, n_images) bytes (0 on invalid sizes). */
size_t hr_full_loss_scratch_bytes(const int32_t* sizes, int32_t n_images);
hr_status hr_full_loss(const float* image, const float* final_T, const float* mesh_rgb,
                       const int32_t* tri_id, const float* target, const int32_t* sizes,
                       int32_t n_images, float lambda_c, float lambda_t, float k,
                       int32_t mask_mode, uint32_t flags, float* loss_out, float* grad_image,
                       float* grad_final_T, float* grad_mesh_rgb, void* scratch, void* stream);

/* Backward autotuner: with the workspace of a forward just run on the same
 * arguments, times the backward blend (256-thread and one-wave kernels, LDS
 * batch 64 and 128) on the given upstream gradients and writes the fastest
 * choice to s->batch_bwd and bit 3 of s->variant. Every candidate's
 * accumulated record gradients must match those of the 256-thread kernel at
 * batch 64 to 1e-4 relative (2-norm; float atomics sum in any order), else
 * HR_ERR_INTERNAL. No gradient output is touched. Synchronises the stream.
 * HR_AUTOTUNE_CACHE is honoured as by hr_autotune. */
hr_status hr_autotune_backward(const hr_gaussians* gaussians, const hr_mesh* mesh,
                               const hr_camera* cams, int32_t n_cams, hr_settings* s,
                               int64_t key_capacity, void* workspace, size_t workspace_bytes,
                               const float* grad_image, const float* grad_final_T,
                               int32_t repeats, void* stream);

/* Autotuner: times the blend variants (LDS batch size and staging depth) on
 * the inputs of a forward that has just run with this workspace, checks that
 * every variant's outputs (image, T, n_contrib and, when exported, n_blended
 * and n_processed) are bit-identical, and writes the fastest choice to
 * s->batch and s->variant (HR_ERR_INTERNAL if a variant differs).
 * Synchronises the stream.
 * With the environment variable HR_AUTOTUNE_CACHE naming a file, a choice
 * cached there for the same workload class (hr_autotune_key) is used without
 * timing, and a newly timed choice is added to the file. HR_LOG (not "" or
 * "0") prints the decisions and every failure to stderr. */
hr_status hr_autotune(const hr_gaussians* g, const hr_mesh* mesh, const hr_camera* cams,
                      int32_t n_cams, hr_settings* s, int64_t key_capacity, void* workspace,
                      size_t workspace_bytes, hr_outputs* out, int32_t repeats, void* stream);

/* Autotuner cache. A tuned choice is kept for a workload class: the key
 * "fwd|" or "bwd|" (backward != 0), the architecture name and compute-unit
 * count of the device, then the powers of two at or below the total pixel
 * count, the Gaussian count and the camera count, the SH degree, whether a
 * mesh is present, and the flags that change the lists (CULL_BEHIND_MESH,
 * MIP_2D, TILE_ELLIPSE), e.g. "fwd|gfx950|cu256|px2^20|n2^19|cams2^0|sh3|mesh1|flags32".
 * hr_autotune_key writes it to buf (cap bytes, truncated, NUL-terminated) and
 * returns the bytes it needs (0 on invalid arguments); host only.
 * The cache file is a JSON object {"hr_autotune_cache": 1, "entries": {key:
 * [batch, variant], ...}} with one entry per line.
 * hr_autotune_cache_lookup returns 1 and fills batch and variant when the file
 * holds the key, else 0. hr_autotune_cache_store adds or replaces the key
 * (written to a temporary file, then renamed over the cache);
 * HR_ERR_INVALID_ARGUMENT for a null path, a key not starting with "fwd|" or
 * "bwd|" or holding a quote, backslash or newline; HR_ERR_INTERNAL when the
 * file cannot be written. Both are host only. */
size_t hr_autotune_key(const char* arch, int32_t compute_units, const hr_gaussians* g,
                       const hr_mesh* mesh, const hr_camera* cams, int32_t n_cams,
                       const hr_settings* s, int32_t backward, char* buf, size_t cap);
int32_t hr_autotune_cache_lookup(const char* path, const char* key, int32_t* batch,
                                 int32_t* variant);
hr_status hr_autotune_cache_store(const char* path, const char* key, int32_t batch,
                                  int32_t variant);

/* Batched training step captured in a hipGraph: forward of all cameras,
 * loss against `target` (planar, packed like the image), backward into
 * `grads`. The graph is recorded once for fixed shapes and pointers; every
 * hr_batch_launch replays it. hr_batch_create allocates nothing on the
 * device; the graph object itself is host state freed by hr_batch_destroy.
 * loss_scratch holds hr_loss_scratch_bytes() of the cameras' sizes. */
typedef struct hr_batch hr_batch;
hr_status hr_batch_create(const hr_gaussians* g, const hr_mesh* mesh, const hr_camera* cams,
                          int32_t n_cams, const hr_settings* s, int64_t key_capacity,
                          void* workspace, size_t workspace_bytes, hr_outputs* out,
                          const float* target, float lambda_t, float k, float* loss_out,
                          float* grad_image, float* grad_final_T, float* grad_mesh_rgb,
                          void* loss_scratch, hr_grads* grads, void* stream, hr_batch** batch);
hr_status hr_batch_launch(hr_batch* batch, void* stream);
/* Outcome of the replays enqueued so far: synchronises `stream` (the one the
 * graph was launched on), then reads the forward's device flags. Returns
 * HR_ERR_CAPACITY when the pair count exceeded the key capacity (the step's
 * outputs and gradients are undefined; stats->n_keys is the needed count:
 * create the batch again over a workspace with that capacity),
 * HR_ERR_INTERNAL when a prefix sum's bounded wait gave up, else HR_OK.
 * `stats` (host memory, nullable) receives the counters of the last replay
 * (n_processed and n_blended are 0: they are not summed by a replay). */
hr_status hr_batch_status(hr_batch* batch, hr_stats* stats, void* stream);
void hr_batch_destroy(hr_batch* batch);

const char* hr_status_string(hr_status s);
const char* hr_last_error(void);
int32_t hr_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HR_H_ */
