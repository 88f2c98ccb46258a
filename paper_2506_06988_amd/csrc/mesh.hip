// Z-buffered rasterization of the textured mesh for every camera (Sec. 3.4:
// the mesh is rendered first, giving I_m and D_m).
//   k_mesh_count   per (camera, face): clip, snap, count kept triangles and
//                  RBLK x RBLK pixel blocks of their bounding boxes
//   k_mesh_setup   per (camera, face): write the kept triangles compactly
//   k_mesh_raster  (triangle, block) work items, a contiguous run per group
//                  of RBLK^2 lanes (one pixel each) that test integer edge
//                  functions and atomicMin a 64-bit key
//                  (fp32 depth bits << 32 | triangle index) into the z-buffer.
//                  Triangle indices increase with face id, so equal depths
//                  resolve to the lower face whatever the launch order.
//   the shading of each pixel (perspective-correct UV, bilinear texture fetch,
//   mesh_math.hpp) runs in the blend's epilogue, beside the composite
#include "kernels.hpp"
#include "mesh_math.hpp"

namespace hr {
namespace {

__global__ __launch_bounds__(256) void k_mesh_count(SetDev S, const CamDev* __restrict__ cams,
                                                    const float* __restrict__ verts,
                                                    const int32_t* __restrict__ faces,
                                                    const float* __restrict__ uvs,
                                                    uint32_t* __restrict__ tri_cnt,
                                                    uint32_t* __restrict__ blk_cnt) {
  const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t MF = (int64_t)S.n_faces * S.n_cams;
  if (item >= MF) {
    if (item == MF) blk_cnt[MF] = 0;
    return;
  }
  const int cam = (int)(item / S.n_faces);
  const int f = (int)(item - (int64_t)cam * S.n_faces);
  const CamDev& C = cams[cam];
  CV poly[4];
  const int np = clip_face(C, (double)S.near_mesh, S.n_verts, verts, faces, uvs, f, poly);
  uint32_t nt = 0, nb = 0;
  for (int s = 0; s + 2 < np; ++s) {
    TriRec T;
    if (setup_tri(C, poly, s, T)) {
      ++nt;
      nb += (uint32_t)tri_blocks(T);
    }
  }
  tri_cnt[item] = nt;
  blk_cnt[item] = nb;
}

__global__ __launch_bounds__(256) void k_mesh_setup(SetDev S, const CamDev* __restrict__ cams,
                                                    const float* __restrict__ verts,
                                                    const int32_t* __restrict__ faces,
                                                    const float* __restrict__ uvs,
                                                    const int32_t* __restrict__ face_tex,
                                                    const uint32_t* __restrict__ tri_cnt,
                                                    const uint32_t* __restrict__ tri_off,
                                                    TriRec* __restrict__ tris) {
  const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t MF = (int64_t)S.n_faces * S.n_cams;
  if (item >= MF || tri_cnt[item] == 0) return;
  const int cam = (int)(item / S.n_faces);
  const int f = (int)(item - (int64_t)cam * S.n_faces);
  const CamDev& C = cams[cam];
  CV poly[4];
  const int np = clip_face(C, (double)S.near_mesh, S.n_verts, verts, faces, uvs, f, poly);
  uint32_t o = tri_off[item];
  for (int s = 0; s + 2 < np; ++s) {
    TriRec T;
    if (setup_tri(C, poly, s, T)) {
      T.face = f;
      const int tx = face_tex[f];  // out-of-range texture ids are clamped
      T.tex = tx < 0 ? 0 : (tx >= S.n_tex ? S.n_tex - 1 : tx);
      T.cam = cam;
      T.pad = 0;
      tris[o++] = T;
    }
  }
}

__global__ __launch_bounds__(256) void k_mesh_raster(SetDev S, const CamDev* __restrict__ cams,
                                                     const uint32_t* __restrict__ tri_off,
                                                     const uint32_t* __restrict__ blk_off,
                                                     const TriRec* __restrict__ tris,
                                                     unsigned long long* __restrict__ zbuf) {
  const int64_t MF = (int64_t)S.n_faces * S.n_cams;
  const uint32_t nblk = blk_off[MF];
  // a group of RBLK^2 lanes takes one block; each group rasterizes a
  // contiguous run of blocks: one search, then a walk
  constexpr int GL = RBLK * RBLK;
  const int lane = (int)threadIdx.x % GL;
  const uint32_t groups = gridDim.x * (blockDim.x / GL);
  const uint32_t gid = blockIdx.x * (blockDim.x / GL) + threadIdx.x / GL;
  const uint32_t per = (nblk + groups - 1) / groups;
  const uint32_t b0 = gid * per;
  if (b0 >= nblk) return;
  const uint32_t b1 = b0 + per < nblk ? b0 + per : nblk;
  int64_t lo = 0, hi = MF - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (blk_off[mid] <= b0) lo = mid; else hi = mid - 1;
  }
  uint32_t t = tri_off[lo];
  int lb = (int)(b0 - blk_off[lo]);
  int nbt = tri_blocks(tris[t]);
  if (lb >= nbt) {
    lb -= nbt;
    ++t;
    nbt = tri_blocks(tris[t]);
  }
  for (uint32_t b = b0; b < b1; ++b) {
    const TriRec& T = tris[t];
    const CamDev& C = cams[T.cam];
    const int nbx = T.bx1 - T.bx0 + 1;
    const int bx = T.bx0 + lb % nbx, by = T.by0 + lb / nbx;
    const int i = bx * RBLK + (lane % RBLK), j = by * RBLK + (lane / RBLK);
    int64_t e[3];
    if (i < C.W && j < C.H && tri_cover(T, i, j, e)) {
      const double z = tri_interp(T, e, nullptr);
      const unsigned long long key =
          ((unsigned long long)__float_as_uint(__double2float_rn(z)) << 32) | t;
      atomicMin(&zbuf[C.pix_off + (int64_t)j * C.W + i], key);
    }
    if (++lb >= nbt && b + 1 < b1) {
      lb = 0;
      ++t;
      nbt = tri_blocks(tris[t]);
    }
  }
}

__device__ __forceinline__ int find_cam_by_pix(const CamDev* cams, int n_cams, int64_t p) {
  int lo = 0, hi = n_cams - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cams[mid].pix_off <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int find_cam_by_tile_m(const CamDev* cams, int n_cams, int tile) {
  int lo = 0, hi = n_cams - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cams[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Per tile: the largest fp32 mesh depth over its pixels inside the image, as
// bits (depths are positive, so bit order is value order); a pixel without a
// face makes it 0xffffffff, above every finite or infinite depth. One
// workgroup per tile, one thread per pixel.
__global__ __launch_bounds__(256) void k_tile_dmax(SetDev S, const CamDev* __restrict__ cams,
                                                   const unsigned long long* __restrict__ zbuf,
                                                   uint32_t* __restrict__ tile_dmax) {
  __shared__ uint32_t red;
  const int t = blockIdx.x;
  const int c = find_cam_by_tile_m(cams, S.n_cams, t);
  const CamDev& C = cams[c];
  const int tl = t - C.tile_off;
  const int i = (tl % C.TX) * TILE + (int)(threadIdx.x % TILE);
  const int j = (tl / C.TX) * TILE + (int)(threadIdx.x / TILE);
  uint32_t v = 0;
  if (i < C.W && j < C.H) v = (uint32_t)(zbuf[C.pix_off + (int64_t)j * C.W + i] >> 32);
  if (threadIdx.x == 0) red = 0;
  __syncthreads();
  atomicMax(&red, v);
  __syncthreads();
  if (threadIdx.x == 0) tile_dmax[t] = red;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u64(uint64_t* p, uint64_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

unsigned fill_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid(n)), dim3(256), 0, st, p, v, n);
}

void launch_fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(n)), dim3(256), 0, st, p, v, n);
}

void launch_mesh(const SetDev& S, const hr_mesh& m, const Work& w, hr_outputs* out,
                 hipStream_t st) {
  launch_fill_u64(w.zbuf, ~0ull, S.n_pix, st);
  const int64_t MF = (int64_t)S.n_faces * S.n_cams;
  if (MF > 0) {
    hipLaunchKernelGGL(k_mesh_count, dim3((unsigned)((MF + 1 + 255) / 256)), dim3(256), 0, st, S,
                       w.cams, m.verts, m.faces, m.uvs, w.tri_cnt, w.blk_cnt);
    scan_u32(w.tri_cnt, w.tri_off, MF, w.counters + 4, w.scan_scratch, st);
    scan_u32(w.blk_cnt, w.blk_off, MF + 1, w.counters + 5, w.scan_scratch, st);
    hipLaunchKernelGGL(k_mesh_setup, dim3((unsigned)((MF + 255) / 256)), dim3(256), 0, st, S,
                       w.cams, m.verts, m.faces, m.uvs, m.face_tex, w.tri_cnt, w.tri_off, w.tris);
    hipLaunchKernelGGL(k_mesh_raster, dim3(2048), dim3(256), 0, st, S, w.cams, w.tri_off,
                       w.blk_off, w.tris, (unsigned long long*)w.zbuf);
  }
  // the shading of every pixel (mesh_shade) is done by the blend, once the
  // z-buffer is complete
  (void)out;
}

void launch_tile_dmax(const SetDev& S, const Work& w, hipStream_t st) {
  if (S.n_tiles == 0) return;
  hipLaunchKernelGGL(k_tile_dmax, dim3((unsigned)S.n_tiles), dim3(256), 0, st, S, w.cams,
                     (const unsigned long long*)w.zbuf, w.tile_dmax);
}

}  // namespace hr
