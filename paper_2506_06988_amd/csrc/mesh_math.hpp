// Device-side triangle setup and per-pixel interpolation of the textured mesh
// (Sec. 3.1 "Textured mesh": barycentric UVs select the texture colour).
// Triangles are clipped at view z = near_mesh, their vertices snapped to
// 1/256 px, and coverage is decided by exact integer edge functions.
#pragma once

#include "common.hpp"

namespace hr {

struct CV {
  double p[3];   // camera space
  double uv[2];
  double w[3];   // world position (orders clip edges canonically)
};

__device__ __forceinline__ bool lex_less(const double* a, const double* b) {
  if (a[0] != b[0]) return a[0] < b[0];
  if (a[1] != b[1]) return a[1] < b[1];
  return a[2] < b[2];
}

// Polygon of face f clipped to z >= zn: 0, 3 or 4 vertices.
__device__ __forceinline__ int clip_face(const CamDev& cam, double zn, int n_verts,
                                         const float* __restrict__ verts,
                                         const int32_t* __restrict__ faces,
                                         const float* __restrict__ uvs, int f, CV out[4]) {
  CV v[3];
  const int i0 = faces[3 * f], i1 = faces[3 * f + 1], i2 = faces[3 * f + 2];
  if (i0 < 0 || i1 < 0 || i2 < 0 || i0 >= n_verts || i1 >= n_verts || i2 >= n_verts) return 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int vi = faces[3 * f + k];
    const double x = verts[3 * vi], y = verts[3 * vi + 1], z = verts[3 * vi + 2];
    v[k].w[0] = x; v[k].w[1] = y; v[k].w[2] = z;
#pragma unroll
    for (int i = 0; i < 3; ++i)
      v[k].p[i] = cam.R[3 * i] * x + cam.R[3 * i + 1] * y + cam.R[3 * i + 2] * z + cam.t[i];
    v[k].uv[0] = uvs[6 * f + 2 * k];
    v[k].uv[1] = uvs[6 * f + 2 * k + 1];
  }
  int n = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const CV& a = v[i];
    const CV& b = v[(i + 1) % 3];
    const bool ain = a.p[2] >= zn, bin = b.p[2] >= zn;
    if (ain) out[n++] = a;
    if (ain != bin) {
      const bool sw = lex_less(b.w, a.w);
      const CV& e0 = sw ? b : a;
      const CV& e1 = sw ? a : b;
      const double t = (zn - e0.p[2]) / (e1.p[2] - e0.p[2]);
      CV c;
      c.p[0] = e0.p[0] + t * (e1.p[0] - e0.p[0]);
      c.p[1] = e0.p[1] + t * (e1.p[1] - e0.p[1]);
      c.p[2] = zn;
      c.uv[0] = e0.uv[0] + t * (e1.uv[0] - e0.uv[0]);
      c.uv[1] = e0.uv[1] + t * (e1.uv[1] - e0.uv[1]);
      c.w[0] = c.w[1] = c.w[2] = 0.0;
      out[n++] = c;
    }
  }
  return n;
}

__device__ __forceinline__ int64_t edge_i64(int64_t ax, int64_t ay, int64_t bx, int64_t by,
                                            int64_t px, int64_t py) {
  return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}

// edge a->b owns samples exactly on it when it runs down the screen, or left
__device__ __forceinline__ bool edge_owns(int64_t ax, int64_t ay, int64_t bx, int64_t by) {
  const int64_t dy = by - ay, dx = bx - ax;
  return dy > 0 || (dy == 0 && dx < 0);
}

// Raster blocks: RBLK x RBLK pixels, one group of RBLK^2 lanes each (the
// room's triangles cover a few pixels at 1080p, so small blocks keep most
// lanes on covered pixels).
constexpr int RBLK_LOG = 2;
constexpr int RBLK = 1 << RBLK_LOG;

// Sub-triangle `sub` (fan 0, sub+1, sub+2) of a clipped polygon, snapped and
// oriented; false when degenerate, outside the guard band or off screen.
__device__ __forceinline__ bool setup_tri(const CamDev& cam, const CV poly[4], int sub, TriRec& T) {
  const CV* tv[3] = {&poly[0], &poly[sub + 1], &poly[sub + 2]};
  int64_t X[3], Y[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double u = cam.fx * tv[k]->p[0] / tv[k]->p[2] + cam.cx;
    const double v = cam.fy * tv[k]->p[1] / tv[k]->p[2] + cam.cy;
    const double su = u * SUBPIX, sv = v * SUBPIX;
    if (!(fabs(su) <= (double)GUARD && fabs(sv) <= (double)GUARD)) return false;
    X[k] = (int64_t)rint(su);
    Y[k] = (int64_t)rint(sv);
  }
  int64_t A = edge_i64(X[0], Y[0], X[1], Y[1], X[2], Y[2]);
  if (A == 0) return false;
  int o1 = 1, o2 = 2;
  if (A < 0) { o1 = 2; o2 = 1; }
  const int ord[3] = {0, o1, o2};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T.X[k] = (int32_t)X[ord[k]];
    T.Y[k] = (int32_t)Y[ord[k]];
    T.iz[k] = 1.0 / tv[ord[k]]->p[2];
    T.uv[k][0] = tv[ord[k]]->uv[0];
    T.uv[k][1] = tv[ord[k]]->uv[1];
  }
  const int64_t minx = min(X[0], min(X[1], X[2])), maxx = max(X[0], max(X[1], X[2]));
  const int64_t miny = min(Y[0], min(Y[1], Y[2])), maxy = max(Y[0], max(Y[1], Y[2]));
  int i0 = (int)fmax(0.0, ceil((double)(minx - SUBPIX / 2) / SUBPIX));
  int i1 = (int)fmin((double)(cam.W - 1), floor((double)(maxx - SUBPIX / 2) / SUBPIX));
  int j0 = (int)fmax(0.0, ceil((double)(miny - SUBPIX / 2) / SUBPIX));
  int j1 = (int)fmin((double)(cam.H - 1), floor((double)(maxy - SUBPIX / 2) / SUBPIX));
  if (i0 > i1 || j0 > j1) return false;
  T.bx0 = i0 >> RBLK_LOG; T.bx1 = i1 >> RBLK_LOG;
  T.by0 = j0 >> RBLK_LOG; T.by1 = j1 >> RBLK_LOG;
  return true;
}

__device__ __forceinline__ int tri_blocks(const TriRec& T) {
  return (T.bx1 - T.bx0 + 1) * (T.by1 - T.by0 + 1);
}

// Coverage of pixel (i, j): edge values e[k] (the weight of vertex k). The
// vertices are within 2^29 in fixed point, so every difference fits 32 bits
// and each edge value is two 32 x 32 -> 64-bit products.
__device__ __forceinline__ int64_t edge_at(int32_t ax, int32_t ay, int32_t bx, int32_t by,
                                           int32_t px, int32_t py) {
  return (int64_t)(bx - ax) * (int64_t)(py - ay) - (int64_t)(by - ay) * (int64_t)(px - ax);
}

__device__ __forceinline__ bool tri_cover(const TriRec& T, int i, int j, int64_t e[3]) {
  const int32_t px = SUBPIX * i + SUBPIX / 2, py = SUBPIX * j + SUBPIX / 2;
  const int32_t X0 = T.X[0], Y0 = T.Y[0], X1 = T.X[1], Y1 = T.Y[1], X2 = T.X[2], Y2 = T.Y[2];
  e[0] = edge_at(X1, Y1, X2, Y2, px, py);
  e[1] = edge_at(X2, Y2, X0, Y0, px, py);
  e[2] = edge_at(X0, Y0, X1, Y1, px, py);
  const bool in0 = e[0] > 0 || (e[0] == 0 && edge_owns(X1, Y1, X2, Y2));
  const bool in1 = e[1] > 0 || (e[1] == 0 && edge_owns(X2, Y2, X0, Y0));
  const bool in2 = e[2] > 0 || (e[2] == 0 && edge_owns(X0, Y0, X1, Y1));
  return in0 && in1 && in2;
}

// Perspective-correct depth and UV from the edge values: with s_k = e_k / z_k,
// the depth is (e_0 + e_1 + e_2) / (s_0 + s_1 + s_2) and the perspective
// weights are s_k / (s_0 + s_1 + s_2). One FP64 reciprocal per pixel.
__device__ __forceinline__ double tri_interp(const TriRec& T, const int64_t e[3], double uv[2]) {
  const double s0 = (double)e[0] * T.iz[0];
  const double s1 = (double)e[1] * T.iz[1];
  const double s2 = (double)e[2] * T.iz[2];
  const double inv = 1.0 / (s0 + s1 + s2);
  const double z = (double)(e[0] + e[1] + e[2]) * inv;
  if (uv) {
    uv[0] = (s0 * T.uv[0][0] + s1 * T.uv[1][0] + s2 * T.uv[2][0]) * inv;
    uv[1] = (s0 * T.uv[0][1] + s1 * T.uv[1][1] + s2 * T.uv[2][1]) * inv;
  }
  return z;
}

struct Taps {
  int64_t o00, o10, o01, o11;  // element offsets of the 4 texels (RGB follows)
  float fx, fy;
  int i0, j0, di, dj;          // first texel; steps to the second column / row (0 or 1)
};

// The footprint of a pixel as the backward reads it (16 bytes): x = i0 | j0 << 16,
// y = texture | di << 30 | dj << 31, z and w the bits of fx and fy; x = ~0 for
// a pixel without a face.
__device__ __forceinline__ uint4 pack_taps(int tex, const Taps& t) {
  return make_uint4((uint32_t)t.i0 | ((uint32_t)t.j0 << 16),
                    (uint32_t)tex | ((uint32_t)t.di << 30) | ((uint32_t)t.dj << 31),
                    __float_as_uint(t.fx), __float_as_uint(t.fy));
}

// bilinear footprint: texel (i, j) centred at ((i+1/2)/W, (j+1/2)/H), clamp to edge
__device__ __forceinline__ Taps bilinear_taps(int tex, int H, int W, const double uv[2]) {
  const double x = uv[0] * W - 0.5, y = uv[1] * H - 0.5;
  const double fx0 = floor(x), fy0 = floor(y);
  Taps t;
  t.fx = (float)(x - fx0);
  t.fy = (float)(y - fy0);
  const int i0 = (int)fmin((double)(W - 1), fmax(0.0, fx0));
  const int i1 = (int)fmin((double)(W - 1), fmax(0.0, fx0 + 1.0));
  const int j0 = (int)fmin((double)(H - 1), fmax(0.0, fy0));
  const int j1 = (int)fmin((double)(H - 1), fmax(0.0, fy0 + 1.0));
  const int64_t b = (int64_t)tex * H * W;
  t.o00 = (b + (int64_t)j0 * W + i0) * 3;
  t.o10 = (b + (int64_t)j0 * W + i1) * 3;
  t.o01 = (b + (int64_t)j1 * W + i0) * 3;
  t.o11 = (b + (int64_t)j1 * W + i1) * 3;
  t.i0 = i0;
  t.j0 = j0;
  t.di = i1 - i0;
  t.dj = j1 - j0;
  return t;
}

// Where the shading of a mesh pixel goes: the workspace copies the blend and
// the backward read (colour, footprint) and the exported outputs (any of
// colour, depth, face may be null).
struct MeshOut {
  float* rgb_ws;
  uint4* taps;
  float* rgb;
  float* depth;
  int32_t* tri_id;
};

// Shading of pixel (i, j) of camera C (packed index p) from its z-buffer key:
// perspective-correct UV, bilinear texture colour, footprint, depth and face;
// a pixel without a face gets colour 0, depth +inf, face -1 and an empty
// footprint. Writes all of them and returns the colour.
__device__ __forceinline__ void mesh_shade(const SetDev& S, const CamDev& C, int i, int j,
                                           int64_t p, unsigned long long key,
                                           const TriRec* __restrict__ tris,
                                           const float* __restrict__ tex, const MeshOut& o,
                                           float rgb[3]) {
  rgb[0] = rgb[1] = rgb[2] = 0.f;
  float depth = __int_as_float(0x7f800000);
  int face = -1;
  uint4 tq = make_uint4(~0u, 0u, 0u, 0u);
  if (key != ~0ull) {
    const TriRec& T = tris[(uint32_t)key];
    int64_t e[3];
    tri_cover(T, i, j, e);
    double uv[2];
    tri_interp(T, e, uv);
    const Taps tp = bilinear_taps(T.tex, S.tex_h, S.tex_w, uv);
    tq = pack_taps(T.tex, tp);
    const float wx = tp.fx, wy = tp.fy;
    const float w00 = (1.f - wx) * (1.f - wy), w10 = wx * (1.f - wy), w01 = (1.f - wx) * wy,
                w11 = wx * wy;
    // one 12-byte load per texel
    float3 t00, t10, t01, t11;
    __builtin_memcpy(&t00, tex + tp.o00, 12);
    __builtin_memcpy(&t10, tex + tp.o10, 12);
    __builtin_memcpy(&t01, tex + tp.o01, 12);
    __builtin_memcpy(&t11, tex + tp.o11, 12);
    rgb[0] = w00 * t00.x + w10 * t10.x + w01 * t01.x + w11 * t11.x;
    rgb[1] = w00 * t00.y + w10 * t10.y + w01 * t01.y + w11 * t11.y;
    rgb[2] = w00 * t00.z + w10 * t10.z + w01 * t01.z + w11 * t11.z;
    depth = __uint_as_float((uint32_t)(key >> 32));
    face = T.face;
  }
  const int64_t hw = (int64_t)C.W * C.H;
  const int64_t pl = 3 * C.pix_off + (p - C.pix_off);
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    o.rgb_ws[pl + ch * hw] = rgb[ch];
    if (o.rgb) o.rgb[pl + ch * hw] = rgb[ch];
  }
  o.taps[p] = tq;
  if (o.depth) o.depth[p] = depth;
  if (o.tri_id) o.tri_id[p] = face;
}

}  // namespace hr
