// CPU FP64 oracle of the hybrid mesh-Gaussian rasterizer.
//
// TEST INFRASTRUCTURE ONLY: only tests/, the smoke entry point and the
// benchmark's CPU-baseline leg may load this library. It shares no code,
// header or table with the HIP implementation.
//
// What it computes, and where the paper defines it:
//   * Gaussian primitive: centre u, opacity, rotation R, scale S, SH colour;
//     density exp(-1/2 (x-u)^T Sigma^-1 (x-u))                 (Sec. 3.1, Eq. 1)
//   * Sigma = R S S^T R^T;  Sigma' = J W Sigma W^T J^T           (Sec. 3.1)
//   * front-to-back alpha blending over depth-sorted Gaussians (Sec. 3.1, Eq. 2)
//   * textured mesh rendered by barycentric UV interpolation     (Sec. 3.1 "Textured mesh")
//   * joint rasterization: mesh gives I_m and D_m; only Gaussians with
//     D_gs < D_m are blended; the residual transmittance T weights the mesh
//     colour, else the background colour                         (Sec. 3.4 "Joint optimization", paragraph "Joint rasterization")
//   * gradients to Gaussians and texture (texture optimisable, no vertex
//     optimisation)                                              (Sec. 3.4)
// Conventions the paper leaves to its 3DGS code base (16 px tiles, 3 sigma
// extent, 0.3 px^2 low-pass, alpha in [1/255, 0.99], T stop 1e-4, 0.2 near
// plane, 1.3 x FOV clamp of the Jacobian, SH colour + 0.5 clamped at 0) are
// inputs (or_params), not constants.
//
// Decisions of the blend that an FP32 evaluation cannot be sure of (alpha
// within a relative slack of alpha_min, T(1 - alpha) within one of t_min) are
// tagged; or_render can also list the outcome of every path through them,
// taken either way, so that a kernel's result can be matched against one of
// them instead of being left unchecked.
//
// Everything is FP64 except where the method's definition rounds: the sort key
// and the depth test use fp32(z); the blend reads the projected record rounded
// to FP32 (the record precision of the kernel) unless OR_FP64_RECORDS is set,
// which the finite-difference tests use.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include <omp.h>

extern "C" {

typedef struct {
  int32_t n, sh_degree;
  const double* means;           // [n,3]
  const double* log_scales;      // [n,3]
  const double* quats;           // [n,4] (w,x,y,z)
  const double* opacity_logits;  // [n]
  const double* sh;              // [n,(d+1)^2,3]
  int32_t n_verts, n_faces, n_tex, tex_h, tex_w;
  const double* verts;     // [V,3]
  const int32_t* faces;    // [F,3]
  const double* uvs;       // [F,3,2]
  const int32_t* face_tex; // [F]
  const float* tex;        // [n_tex,tex_h,tex_w,3]
  const double* filter3d;  // [n] Mip-Splatting 3D smoothing variance, or null
} or_scene;

typedef struct {
  int32_t width, height;
  double fx, fy, cx, cy;
  double R[9];  // world -> camera, row-major
  double t[3];
} or_camera;

typedef struct {
  double bg[3];
  double low_pass, alpha_min, alpha_max, t_min, near_gs, near_mesh, clamp_fov;
  int32_t tile, flags;
  double amb_alpha, amb_t;  // relative slack under which a decision is tagged
} or_params;

enum { OR_FP64_RECORDS = 1, OR_CULL_MESH = 2, OR_MIP_2D = 4, OR_TILE_ELLIPSE = 8 };

// per-Gaussian record export
typedef struct {
  double* mean2d;      // [n,2]
  double* conic;       // [n,3]
  double* cov2d;       // [n,3]
  double* opacity;     // [n]
  double* rgb;         // [n,3]
  double* depth;       // [n]
  uint32_t* depth_bits;// [n]
  int32_t* radius;     // [n]   0 = culled
  int32_t* rect;       // [n,4] x0,x1,y0,y1 in tiles (exclusive ends)
  int32_t* tiles;      // [n]
  uint8_t* amb;        // [n]
} or_proj_out;

typedef struct {
  double* image;        // [3,h,w]  window
  double* final_T;      // [h,w]
  int32_t* n_contrib;   // [h,w]
  int32_t* n_blended;   // [h,w]
  int32_t* n_processed; // [h,w]
  uint8_t* amb;         // [h,w]  bit0 alpha slack, bit1 T slack, bit2 projection, bit4 mesh
  int32_t* tri_id;      // [h,w]
  float* mesh_depth;    // [h,w]
  double* mesh_rgb;     // [3,h,w]
  uint64_t* trace;      // [1] hash of every decision taken
  // Every pixel with an alpha-skip or T-stop decision inside the ambiguity
  // slack (amb bits 0-1) gets the outcome of each path through its ambiguous
  // decisions, either way at each: n_alt[h,w] paths (1 elsewhere, at most
  // OR_MAX_ALT; amb bit 5 set when more exist), alts[h,w,OR_MAX_ALT,7] =
  // (r, g, b, T, n_contrib, n_blended, n_processed). Both nullable.
  int32_t* n_alt;
  double* alts;
} or_render_out;

#define OR_MAX_ALT 16

typedef struct {
  double* means;     // [n,3]
  double* log_scales;
  double* quats;     // [n,4]
  double* opacity_logits;
  double* sh;        // [n,K,3]
  double* tex;       // [n_tex,H,W,3]
  double* mean2d;    // [n,2] gradient w.r.t. the projected mean (u, v), in pixels
} or_grads;
}

namespace {

constexpr double PI = 3.14159265358979323846;
constexpr double MIP2D_FLOOR = 2.5e-5;  // lower bound of the 2D filter's determinant ratio

struct Rec {
  bool vis = false, amb = false;
  double pc[3];
  double u, v;
  double cov[3];
  double con[3];
  double op, logit;
  double rgb[3];
  bool clamped[3];
  double dir[3], dnorm;
  int r, x0, x1, y0, y1;
  uint32_t dbits;
  double zf;  // fp32(z) as double
  // values the blend uses (FP32-rounded unless OR_FP64_RECORDS)
  double bu, bv, bcon[3], bop, brgb[3];
  // Mip-Splatting: 3D smoothing variance f3 and its opacity factor c3; 2D
  // filter opacity factor c2 (c2lo: at its floor); opr = op c3 c2
  double f3 = 0.0, c3 = 1.0, c2 = 1.0, opr;
  bool c2lo = false;
  // backward intermediates
  double s[3], qn[4], qnorm, Rq[9], Sc[9], J[6];
  bool clx, cly;
  double xc, yc;
};

inline uint32_t f32bits(float f) {
  uint32_t b;
  std::memcpy(&b, &f, 4);
  return b;
}

inline double r32(double x) { return (double)(float)x; }

bool near_int(double x, double rel) {
  double d = std::fabs(x - std::nearbyint(x));
  return d <= rel * std::max(1.0, std::fabs(x));
}

// FP64 results of two implementations differ by ~1e-15 relative; a rounding
// or integer decision closer than that to its boundary may go either way.
bool f32_boundary(double x) {
  double e = std::fabs(x) * 1e-14;
  return (float)(x + e) != (float)(x - e);
}

// Real spherical harmonics, orthonormal on the unit sphere, without the
// Condon-Shortley phase; index k = l*l + l + m, m = -l..l.
void sh_basis(const double d[3], double* Y, int deg) {
  const double x = d[0], y = d[1], z = d[2];
  Y[0] = 0.5 * std::sqrt(1.0 / PI);
  if (deg < 1) return;
  const double c1 = std::sqrt(3.0 / (4.0 * PI));
  Y[1] = c1 * y;
  Y[2] = c1 * z;
  Y[3] = c1 * x;
  if (deg < 2) return;
  const double a2 = 0.5 * std::sqrt(15.0 / PI), b2 = 0.25 * std::sqrt(5.0 / PI),
               d2 = 0.25 * std::sqrt(15.0 / PI);
  Y[4] = a2 * x * y;
  Y[5] = a2 * y * z;
  Y[6] = b2 * (3.0 * z * z - 1.0);
  Y[7] = a2 * x * z;
  Y[8] = d2 * (x * x - y * y);
  if (deg < 3) return;
  const double e3 = 0.25 * std::sqrt(35.0 / (2.0 * PI)), f3 = 0.5 * std::sqrt(105.0 / PI),
               g3 = 0.25 * std::sqrt(21.0 / (2.0 * PI)), h3 = 0.25 * std::sqrt(7.0 / PI),
               k3 = 0.25 * std::sqrt(105.0 / PI);
  Y[9] = e3 * y * (3.0 * x * x - y * y);
  Y[10] = f3 * x * y * z;
  Y[11] = g3 * y * (5.0 * z * z - 1.0);
  Y[12] = h3 * z * (5.0 * z * z - 3.0);
  Y[13] = g3 * x * (5.0 * z * z - 1.0);
  Y[14] = k3 * z * (x * x - y * y);
  Y[15] = e3 * x * (x * x - 3.0 * y * y);
}

// gradient of each basis polynomial above with respect to (x, y, z)
void sh_basis_grad(const double d[3], double (*G)[3], int deg) {
  const double x = d[0], y = d[1], z = d[2];
  for (int k = 0; k < 16; ++k) G[k][0] = G[k][1] = G[k][2] = 0.0;
  if (deg < 1) return;
  const double c1 = std::sqrt(3.0 / (4.0 * PI));
  G[1][1] = c1;
  G[2][2] = c1;
  G[3][0] = c1;
  if (deg < 2) return;
  const double a2 = 0.5 * std::sqrt(15.0 / PI), b2 = 0.25 * std::sqrt(5.0 / PI),
               d2 = 0.25 * std::sqrt(15.0 / PI);
  G[4][0] = a2 * y; G[4][1] = a2 * x;
  G[5][1] = a2 * z; G[5][2] = a2 * y;
  G[6][2] = 6.0 * b2 * z;
  G[7][0] = a2 * z; G[7][2] = a2 * x;
  G[8][0] = 2.0 * d2 * x; G[8][1] = -2.0 * d2 * y;
  if (deg < 3) return;
  const double e3 = 0.25 * std::sqrt(35.0 / (2.0 * PI)), f3 = 0.5 * std::sqrt(105.0 / PI),
               g3 = 0.25 * std::sqrt(21.0 / (2.0 * PI)), h3 = 0.25 * std::sqrt(7.0 / PI),
               k3 = 0.25 * std::sqrt(105.0 / PI);
  G[9][0] = 6.0 * e3 * x * y; G[9][1] = e3 * (3.0 * x * x - 3.0 * y * y);
  G[10][0] = f3 * y * z; G[10][1] = f3 * x * z; G[10][2] = f3 * x * y;
  G[11][1] = g3 * (5.0 * z * z - 1.0); G[11][2] = 10.0 * g3 * y * z;
  G[12][2] = h3 * (15.0 * z * z - 3.0);
  G[13][0] = g3 * (5.0 * z * z - 1.0); G[13][2] = 10.0 * g3 * x * z;
  G[14][0] = 2.0 * k3 * x * z; G[14][1] = -2.0 * k3 * y * z; G[14][2] = k3 * (x * x - y * y);
  G[15][0] = e3 * (3.0 * x * x - 3.0 * y * y); G[15][1] = -6.0 * e3 * x * y;
}

// unit quaternion (w,x,y,z) -> rotation matrix, row-major
void quat_to_rot(const double q[4], double* R) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

int tiles_x(const or_camera& c, const or_params& p) { return (c.width + p.tile - 1) / p.tile; }
int tiles_y(const or_camera& c, const or_params& p) { return (c.height + p.tile - 1) / p.tile; }

// Sec. 3.1: Sigma = R S S^T R^T, Sigma' = J W Sigma W^T J^T (+ low-pass), conic,
// 3-sigma radius and tile rectangle, SH colour, depth key.
Rec project(const or_scene& sc, const or_camera& cam, const or_params& p, int g) {
  Rec r;
  const int K = (sc.sh_degree + 1) * (sc.sh_degree + 1);
  const double* mu = sc.means + 3 * (size_t)g;
  const double* ls = sc.log_scales + 3 * (size_t)g;
  const double* q = sc.quats + 4 * (size_t)g;
  const double* shc = sc.sh + (size_t)g * K * 3;
  bool fin = std::isfinite(sc.opacity_logits[g]);
  for (int i = 0; i < 3; ++i) fin = fin && std::isfinite(mu[i]) && std::isfinite(ls[i]);
  for (int i = 0; i < 4; ++i) fin = fin && std::isfinite(q[i]);
  for (int i = 0; i < K * 3; ++i) fin = fin && std::isfinite(shc[i]);
  if (!fin) return r;

  const double* W = cam.R;
  for (int i = 0; i < 3; ++i)
    r.pc[i] = W[3 * i] * mu[0] + W[3 * i + 1] * mu[1] + W[3 * i + 2] * mu[2] + cam.t[i];
  const double x = r.pc[0], y = r.pc[1], z = r.pc[2];
  if (std::fabs(z - p.near_gs) <= 1e-14 * p.near_gs) r.amb = true;
  if (!(z > p.near_gs)) return r;

  r.logit = sc.opacity_logits[g];
  r.op = 1.0 / (1.0 + std::exp(-r.logit));
  for (int i = 0; i < 3; ++i) r.s[i] = std::exp(ls[i]);
  r.qnorm = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  if (!(r.qnorm > 0)) return r;
  for (int i = 0; i < 4; ++i) r.qn[i] = q[i] / r.qnorm;
  quat_to_rot(r.qn, r.Rq);
  double M[9], Sig[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[3 * i + j] = r.Rq[3 * i + j] * r.s[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double a = 0;
      for (int k = 0; k < 3; ++k) a += M[3 * i + k] * M[3 * j + k];
      Sig[3 * i + j] = a;
    }
  // Mip-Splatting 3D smoothing: Sigma + f3 I, opacity scaled by
  // sqrt(det Sigma / det(Sigma + f3 I)) = prod_i s_i / sqrt(s_i^2 + f3)
  if (sc.filter3d) {
    r.f3 = sc.filter3d[g];
    if (!(std::isfinite(r.f3) && r.f3 >= 0.0)) return r;
    for (int i = 0; i < 3; ++i) {
      Sig[4 * i] += r.f3;
      r.c3 *= r.s[i] / std::sqrt(r.s[i] * r.s[i] + r.f3);
    }
  }
  double WS[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double a = 0;
      for (int k = 0; k < 3; ++k) a += W[3 * i + k] * Sig[3 * k + j];
      WS[3 * i + j] = a;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double a = 0;
      for (int k = 0; k < 3; ++k) a += WS[3 * i + k] * W[3 * j + k];
      r.Sc[3 * i + j] = a;
    }
  const double limx = p.clamp_fov * cam.width / (2.0 * cam.fx);
  const double limy = p.clamp_fov * cam.height / (2.0 * cam.fy);
  const double xz = x / z, yz = y / z;
  r.xc = std::min(limx, std::max(-limx, xz));
  r.yc = std::min(limy, std::max(-limy, yz));
  r.clx = (xz < -limx) || (xz > limx);
  r.cly = (yz < -limy) || (yz > limy);
  r.J[0] = cam.fx / z; r.J[1] = 0.0; r.J[2] = -cam.fx * r.xc / z;
  r.J[3] = 0.0; r.J[4] = cam.fy / z; r.J[5] = -cam.fy * r.yc / z;
  double JS[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double a = 0;
      for (int k = 0; k < 3; ++k) a += r.J[3 * i + k] * r.Sc[3 * k + j];
      JS[3 * i + j] = a;
    }
  double C2[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double a = 0;
      for (int k = 0; k < 3; ++k) a += JS[3 * i + k] * r.J[3 * j + k];
      C2[2 * i + j] = a;
    }
  r.cov[0] = C2[0] + p.low_pass;
  r.cov[1] = 0.5 * (C2[1] + C2[2]);
  r.cov[2] = C2[3] + p.low_pass;
  const double det = r.cov[0] * r.cov[2] - r.cov[1] * r.cov[1];
  if (!(det > 0)) return r;
  // Mip-Splatting 2D filter: the low-pass variance is the pixel filter, and the
  // opacity is scaled by sqrt(det(Sigma') / det(Sigma' + low_pass I)), the ratio
  // floored at MIP2D_FLOOR
  if (p.flags & OR_MIP_2D) {
    const double d0 = (r.cov[0] - p.low_pass) * (r.cov[2] - p.low_pass) - r.cov[1] * r.cov[1];
    const double ratio = d0 / det;
    r.c2lo = !(ratio > MIP2D_FLOOR);
    r.c2 = std::sqrt(r.c2lo ? MIP2D_FLOOR : ratio);
  }
  r.opr = r.op * r.c3 * r.c2;
  r.con[0] = r.cov[2] / det;
  r.con[1] = -r.cov[1] / det;
  r.con[2] = r.cov[0] / det;
  r.u = cam.fx * x / z + cam.cx;
  r.v = cam.fy * y / z + cam.cy;
  const double m = 0.5 * (r.cov[0] + r.cov[2]);
  const double lam = m + std::sqrt(std::max(0.1, m * m - det));
  const double r3 = 3.0 * std::sqrt(lam);
  r.r = (int)std::ceil(r3);
  if (near_int(r3, 1e-13)) r.amb = true;
  const int TX = tiles_x(cam, p), TY = tiles_y(cam, p);
  const double T = (double)p.tile;
  const double ex0 = (r.u - r.r) / T, ex1 = (r.u + r.r) / T;
  const double ey0 = (r.v - r.r) / T, ey1 = (r.v + r.r) / T;
  if (near_int(ex0, 1e-13) || near_int(ex1, 1e-13) || near_int(ey0, 1e-13) ||
      near_int(ey1, 1e-13))
    r.amb = true;
  auto clampi = [](double v, int hi) {
    if (!(v > 0)) return 0;  // also catches NaN
    if (v > hi) return hi;
    return (int)v;
  };
  r.x0 = clampi(std::floor(ex0), TX);
  r.x1 = clampi(std::floor(ex1) + 1, TX);
  r.y0 = clampi(std::floor(ey0), TY);
  r.y1 = clampi(std::floor(ey1) + 1, TY);
  if ((r.x1 - r.x0) * (r.y1 - r.y0) <= 0) return r;

  // view-dependent colour from SH toward normalize(u - camera centre)
  double C[3];
  for (int i = 0; i < 3; ++i)
    C[i] = -(W[i] * cam.t[0] + W[3 + i] * cam.t[1] + W[6 + i] * cam.t[2]);
  double d[3] = {mu[0] - C[0], mu[1] - C[1], mu[2] - C[2]};
  r.dnorm = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  for (int i = 0; i < 3; ++i) r.dir[i] = d[i] / r.dnorm;
  double Y[16];
  sh_basis(r.dir, Y, sc.sh_degree);
  for (int c = 0; c < 3; ++c) {
    double a = 0.5;
    for (int k = 0; k < K; ++k) a += Y[k] * shc[3 * k + c];
    r.clamped[c] = a < 0.0;
    r.rgb[c] = r.clamped[c] ? 0.0 : a;
  }
  const float zf = (float)z;
  r.dbits = f32bits(zf);
  r.zf = zf;
  if (f32_boundary(z)) r.amb = true;
  r.vis = true;
  if (p.flags & OR_FP64_RECORDS) {
    r.bu = r.u; r.bv = r.v; r.bop = r.opr;
    for (int i = 0; i < 3; ++i) { r.bcon[i] = r.con[i]; r.brgb[i] = r.rgb[i]; }
  } else {
    r.bu = r32(r.u); r.bv = r32(r.v); r.bop = r32(r.opr);
    for (int i = 0; i < 3; ++i) { r.bcon[i] = r32(r.con[i]); r.brgb[i] = r32(r.rgb[i]); }
  }
  return r;
}

std::vector<Rec> project_all(const or_scene& sc, const or_camera& cam, const or_params& p) {
  std::vector<Rec> recs(sc.n);
#pragma omp parallel for schedule(static)
  for (int g = 0; g < sc.n; ++g) recs[g] = project(sc, cam, p, g);
  return recs;
}

// ------------------------------------------------------------------ mesh --
struct MeshPix {
  uint64_t key = ~0ull;  // fp32 depth bits << 32 | (2 * face + sub)
  double z, uv[2];
  bool amb = false;
};

struct CVert {
  double p[3];
  double uv[2];
  double w[3];  // world position, used to order clip edges canonically
};

// Sutherland-Hodgman against z >= zn. The crossing of an edge is computed
// from the lexicographically smaller world endpoint so that an edge shared by
// two faces gives the same clip point in both.
int clip_near(const CVert in[3], double zn, CVert out[4], bool* amb) {
  int n = 0;
  for (int i = 0; i < 3; ++i) {
    const CVert& a = in[i];
    const CVert& b = in[(i + 1) % 3];
    if (std::fabs(a.p[2] - zn) <= 1e-12 * zn) *amb = true;
    const bool ain = a.p[2] >= zn, bin = b.p[2] >= zn;
    if (ain) out[n++] = a;
    if (ain != bin) {
      bool swap = std::lexicographical_compare(b.w, b.w + 3, a.w, a.w + 3);
      const CVert& e0 = swap ? b : a;
      const CVert& e1 = swap ? a : b;
      const double t = (zn - e0.p[2]) / (e1.p[2] - e0.p[2]);
      CVert c;
      for (int k = 0; k < 3; ++k) c.p[k] = e0.p[k] + t * (e1.p[k] - e0.p[k]);
      c.p[2] = zn;
      for (int k = 0; k < 2; ++k) c.uv[k] = e0.uv[k] + t * (e1.uv[k] - e0.uv[k]);
      for (int k = 0; k < 3; ++k) c.w[k] = 0;
      out[n++] = c;
    }
  }
  return n;
}

inline int64_t edge_fn(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t px, int64_t py) {
  return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}

// an edge a->b owns the samples lying exactly on it when it points down the
// screen, or exactly left; the reverse edge of a neighbour then does not
inline bool owns(int64_t ax, int64_t ay, int64_t bx, int64_t by) {
  const int64_t dx = bx - ax, dy = by - ay;
  return dy > 0 || (dy == 0 && dx < 0);
}

constexpr int64_t SUBPIX = 256;
constexpr int64_t GUARD = (int64_t)1 << 29;

// Z-buffered rasterization of the textured mesh over window [wx0,wx1)x[wy0,wy1).
void mesh_pass(const or_scene& sc, const or_camera& cam, const or_params& p, int wx0, int wy0,
               int wx1, int wy1, std::vector<MeshPix>& pix) {
  const int ww = wx1 - wx0, wh = wy1 - wy0;
  pix.assign((size_t)ww * wh, MeshPix());
  const double* W = cam.R;
  for (int f = 0; f < sc.n_faces; ++f) {
    CVert cv[3];
    for (int k = 0; k < 3; ++k) {
      const int vi = sc.faces[3 * f + k];
      const double* v = sc.verts + 3 * (size_t)vi;
      for (int i = 0; i < 3; ++i) {
        cv[k].p[i] = W[3 * i] * v[0] + W[3 * i + 1] * v[1] + W[3 * i + 2] * v[2] + cam.t[i];
        cv[k].w[i] = v[i];
      }
      cv[k].uv[0] = sc.uvs[6 * (size_t)f + 2 * k];
      cv[k].uv[1] = sc.uvs[6 * (size_t)f + 2 * k + 1];
    }
    bool famb = false;
    CVert poly[4];
    const int np = clip_near(cv, p.near_mesh, poly, &famb);
    if (np < 3) continue;
    for (int sub = 0; sub < np - 2; ++sub) {
      CVert tv[3] = {poly[0], poly[sub + 1], poly[sub + 2]};
      int64_t X[3], Yv[3];
      bool skip = false, amb = famb;
      for (int k = 0; k < 3; ++k) {
        const double u = cam.fx * tv[k].p[0] / tv[k].p[2] + cam.cx;
        const double v = cam.fy * tv[k].p[1] / tv[k].p[2] + cam.cy;
        const double su = u * SUBPIX, sv = v * SUBPIX;
        if (!(std::fabs(su) <= (double)GUARD && std::fabs(sv) <= (double)GUARD)) skip = true;
        // two FP64 evaluations of the projection differ by ~1e-15 relative;
        // a snap within 1e-13 of a rounding midpoint may round either way
        if (std::fabs(std::fabs(su - std::floor(su)) - 0.5) <= 1e-13 * std::max(1.0, std::fabs(su)) ||
            std::fabs(std::fabs(sv - std::floor(sv)) - 0.5) <= 1e-13 * std::max(1.0, std::fabs(sv)))
          amb = true;
        X[k] = skip ? 0 : (int64_t)std::nearbyint(su);
        Yv[k] = skip ? 0 : (int64_t)std::nearbyint(sv);
      }
      if (skip) continue;
      int64_t A = edge_fn(X[0], Yv[0], X[1], Yv[1], X[2], Yv[2]);
      if (A == 0) continue;
      if (A < 0) {
        std::swap(X[1], X[2]);
        std::swap(Yv[1], Yv[2]);
        std::swap(tv[1], tv[2]);
        A = -A;
      }
      const int64_t minx = std::min(X[0], std::min(X[1], X[2]));
      const int64_t maxx = std::max(X[0], std::max(X[1], X[2]));
      const int64_t miny = std::min(Yv[0], std::min(Yv[1], Yv[2]));
      const int64_t maxy = std::max(Yv[0], std::max(Yv[1], Yv[2]));
      // pixel i samples at 256 i + 128
      int64_t i0 = (int64_t)std::floor((minx - 128) / 256.0), i1 = (int64_t)std::ceil((maxx - 128) / 256.0);
      int64_t j0 = (int64_t)std::floor((miny - 128) / 256.0), j1 = (int64_t)std::ceil((maxy - 128) / 256.0);
      i0 = std::max<int64_t>(i0, wx0); i1 = std::min<int64_t>(i1, wx1 - 1);
      j0 = std::max<int64_t>(j0, wy0); j1 = std::min<int64_t>(j1, wy1 - 1);
      const bool o0 = owns(X[1], Yv[1], X[2], Yv[2]);
      const bool o1 = owns(X[2], Yv[2], X[0], Yv[0]);
      const bool o2 = owns(X[0], Yv[0], X[1], Yv[1]);
      const uint64_t uid = 2ull * (uint64_t)f + (uint64_t)sub;
      for (int64_t j = j0; j <= j1; ++j)
        for (int64_t i = i0; i <= i1; ++i) {
          const int64_t px = SUBPIX * i + SUBPIX / 2, py = SUBPIX * j + SUBPIX / 2;
          const int64_t e0 = edge_fn(X[1], Yv[1], X[2], Yv[2], px, py);
          const int64_t e1 = edge_fn(X[2], Yv[2], X[0], Yv[0], px, py);
          const int64_t e2 = edge_fn(X[0], Yv[0], X[1], Yv[1], px, py);
          const bool in0 = e0 > 0 || (e0 == 0 && o0);
          const bool in1 = e1 > 0 || (e1 == 0 && o1);
          const bool in2 = e2 > 0 || (e2 == 0 && o2);
          if (!(in0 && in1 && in2)) continue;
          // screen barycentrics, then perspective-correct weights
          const double b0 = (double)e0 / (double)A, b1 = (double)e1 / (double)A,
                       b2 = (double)e2 / (double)A;
          const double q0 = b0 / tv[0].p[2], q1 = b1 / tv[1].p[2], q2 = b2 / tv[2].p[2];
          const double s = q0 + q1 + q2;
          const double z = 1.0 / s;
          const float zf = (float)z;
          const uint64_t key = ((uint64_t)f32bits(zf) << 32) | uid;
          MeshPix& mp = pix[(size_t)(j - wy0) * ww + (i - wx0)];
          if (key < mp.key) {
            mp.key = key;
            mp.z = z;
            const double w0 = q0 * z, w1 = q1 * z, w2 = q2 * z;
            for (int k = 0; k < 2; ++k) mp.uv[k] = w0 * tv[0].uv[k] + w1 * tv[1].uv[k] + w2 * tv[2].uv[k];
            mp.amb = amb || f32_boundary(z);
          }
        }
    }
  }
}

struct Bilin {
  int tex, i0, i1, j0, j1;
  double fx, fy;
};

// bilinear texel addressing: texel (i, j) centred at ((i+0.5)/W, (j+0.5)/H),
// row 0 at V = 0, clamp to edge
Bilin bilinear(const or_scene& sc, int face, const double uv[2]) {
  Bilin b;
  b.tex = sc.face_tex[face];
  const double x = uv[0] * sc.tex_w - 0.5, y = uv[1] * sc.tex_h - 0.5;
  const double fx0 = std::floor(x), fy0 = std::floor(y);
  b.fx = x - fx0;
  b.fy = y - fy0;
  auto cl = [](double v, int hi) { return (int)std::min<double>(hi, std::max<double>(0.0, v)); };
  b.i0 = cl(fx0, sc.tex_w - 1);
  b.i1 = cl(fx0 + 1, sc.tex_w - 1);
  b.j0 = cl(fy0, sc.tex_h - 1);
  b.j1 = cl(fy0 + 1, sc.tex_h - 1);
  return b;
}

double texel(const or_scene& sc, int t, int j, int i, int c) {
  return (double)sc.tex[(((size_t)t * sc.tex_h + j) * sc.tex_w + i) * 3 + c];
}

// --------------------------------------------------------------- binning --
struct Cand {
  uint32_t dbits;
  int32_t g;
};

// Tile-ellipse option: in tile row ty, the tiles whose pixel centres meet
// the ellipse d^T Q d <= 2 ln(opacity / alpha_min) of the record (where
// alpha = opacity G reaches alpha_min), grown to 1.01 R + 0.1 plus a term
// for the magnitude of the form over the rectangle; outside it every pixel
// skips the Gaussian (alpha < alpha_min). Returns false for an empty run.
bool ellipse_run(const Rec& r, int ty, double ln_amin, int tile, int* x0, int* x1) {
  *x0 = r.x0;
  *x1 = r.x1;
  const double a = r.bcon[0], b = r.bcon[1], c = r.bcon[2];
  const double det = a * c - b * b;
  if (!(a > 0.0 && c > 0.0 && det > 0.0)) return true;
  const double rr = 2.0 * (std::log(r.bop) - ln_amin);
  if (!(rr > 0.0)) return false;
  const double ext = (double)tile * std::max(r.x1 - r.x0, r.y1 - r.y0);
  const double rp = 1.01 * rr + 0.1 + 1e-5 * (a + c) * ext * ext;
  const double dymax = std::sqrt(a * rp / det);
  const double lo = std::max((double)ty * tile + 0.5 - r.bv, -dymax);
  const double hi = std::min((double)ty * tile + (tile - 0.5) - r.bv, dymax);
  if (lo > hi) return false;
  const double sc = std::sqrt(rp / (c * det));
  const double ys = std::min(std::max(-b * sc, lo), hi), yn = std::min(std::max(b * sc, lo), hi);
  const double xmax = (-b * ys + std::sqrt(std::max(a * rp - det * ys * ys, 0.0))) / a;
  const double xmin = (-b * yn - std::sqrt(std::max(a * rp - det * yn * yn, 0.0))) / a;
  *x0 = std::max(*x0, (int)std::ceil((r.bu + xmin - (tile - 0.5)) / tile));
  *x1 = std::min(*x1, (int)std::floor((r.bu + xmax - 0.5) / tile) + 1);
  return *x1 > *x0;
}

// For every tile overlapping the window: all Gaussians whose tile rectangle
// holds it (and, with OR_TILE_ELLIPSE, whose ellipse run holds it), ordered
// by (fp32 depth bits, index).
std::vector<std::vector<Cand>> tile_lists(const std::vector<Rec>& recs, const or_params& p,
                                          int tx0, int ty0, int tx1, int ty1) {
  const int ntx = tx1 - tx0, nty = ty1 - ty0;
  const bool ell = (p.flags & OR_TILE_ELLIPSE) != 0;
  const double ln_amin = std::log(p.alpha_min);
  std::vector<std::vector<Cand>> lists((size_t)ntx * nty);
  for (int g = 0; g < (int)recs.size(); ++g) {
    const Rec& r = recs[g];
    if (!r.vis) continue;
    for (int ty = std::max(r.y0, ty0); ty < std::min(r.y1, ty1); ++ty) {
      int x0 = r.x0, x1 = r.x1;
      if (ell && !ellipse_run(r, ty, ln_amin, p.tile, &x0, &x1)) continue;
      for (int tx = std::max(x0, tx0); tx < std::min(x1, tx1); ++tx)
        lists[(size_t)(ty - ty0) * ntx + (tx - tx0)].push_back({r.dbits, g});
    }
  }
#pragma omp parallel for schedule(dynamic)
  for (int t = 0; t < ntx * nty; ++t)
    std::sort(lists[t].begin(), lists[t].end(), [](const Cand& a, const Cand& b) {
      return a.dbits != b.dbits ? a.dbits < b.dbits : a.g < b.g;
    });
  return lists;
}

inline uint64_t mix(uint64_t h, uint64_t v) {
  h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
  return h;
}

struct Step {
  int g;
  double alpha, G, T;  // T before this Gaussian
  bool clamped;
};

// A floating-point decision of the blend taken too close to its threshold for
// an FP32 evaluation to be sure of it: the alpha-skip (kind 0) or the
// transmittance stop (kind 1) at list entry k.
struct Decision {
  int k, kind;
  bool operator<(const Decision& o) const { return k != o.k ? k < o.k : kind < o.kind; }
  bool operator==(const Decision& o) const { return k == o.k && kind == o.kind; }
};

// Sec. 3.1 Eq. 2 with the joint-rasterization depth stop of Sec. 3.4.
// Returns the steps that blended (the tape) and fills the pixel outputs.
// `flip` lists decisions to take the other way; `near` (nullable) receives
// every decision met within the ambiguity slack, in list order.
void blend_pixel(const std::vector<Rec>& recs, const std::vector<Cand>& list, const or_params& p,
                 double px, double py, float Dm, std::vector<Step>* tape, double C[3], double* Tout,
                 int* nc, int* nb, int* npro, uint8_t* amb, uint64_t* hash,
                 const std::vector<Decision>* flip = nullptr, std::vector<Decision>* near = nullptr) {
  double T = 1.0;
  C[0] = C[1] = C[2] = 0.0;
  *nc = 0; *nb = 0; *npro = (int)list.size();
  uint64_t h = 0;
  auto flipped = [&](int k, int kind) {
    return flip && std::find(flip->begin(), flip->end(), Decision{k, kind}) != flip->end();
  };
  for (size_t k = 0; k < list.size(); ++k) {
    const Rec& r = recs[list[k].g];
    if (r.amb) *amb |= 4;
    if ((float)r.zf >= Dm) {
      *npro = (int)k + 1;
      h = mix(h, 3);
      break;
    }
    const double dx = px - r.bu, dy = py - r.bv;
    const double power = -0.5 * (r.bcon[0] * dx * dx + r.bcon[2] * dy * dy) - r.bcon[1] * dx * dy;
    const double G = std::exp(power);
    const double a = r.bop * G;
    const bool clamped = a >= p.alpha_max;
    const double alpha = clamped ? p.alpha_max : a;
    if (std::fabs(alpha - p.alpha_min) <= p.amb_alpha * p.alpha_min) {
      *amb |= 1;
      if (near) near->push_back({(int)k, 0});
    }
    if ((alpha < p.alpha_min) != flipped((int)k, 0)) {
      h = mix(h, 1);
      continue;
    }
    const double Tn = T * (1.0 - alpha);
    if (std::fabs(Tn - p.t_min) <= p.amb_t * p.t_min) {
      *amb |= 2;
      if (near) near->push_back({(int)k, 1});
    }
    if ((Tn < p.t_min) != flipped((int)k, 1)) {
      *npro = (int)k + 1;
      h = mix(h, 2);
      break;
    }
    if (tape) tape->push_back({list[k].g, alpha, G, T, clamped});
    for (int c = 0; c < 3; ++c) C[c] += r.brgb[c] * alpha * T;
    T = Tn;
    *nc = (int)k + 1;
    *nb += 1;
    h = mix(h, ((uint64_t)list[k].g << 3) | (clamped ? 5 : 4));
  }
  *Tout = T;
  *hash = h;
}

// Joint rasterization (Sec. 3.4): each pixel stops at the first Gaussian
// whose fp32 depth is not below its fp32 mesh depth. A Gaussian at or beyond
// the largest mesh depth of every pixel of a tile therefore stops every pixel
// there, and with OR_CULL_MESH it is removed from that tile's list (tiles with
// a pixel that has no face keep their lists). The tile's pixels are those of
// the image, whatever the window.
void cull_behind_mesh(const or_scene& sc, const or_camera& cam, const or_params& p,
                      const std::vector<Rec>& recs, int tx0, int ty0, int tx1, int ty1,
                      std::vector<std::vector<Cand>>& lists) {
  if (sc.n_faces == 0) return;
  const int x0 = tx0 * p.tile, y0 = ty0 * p.tile;
  const int x1 = std::min(tx1 * p.tile, cam.width), y1 = std::min(ty1 * p.tile, cam.height);
  std::vector<MeshPix> pix;
  mesh_pass(sc, cam, p, x0, y0, x1, y1, pix);
  const int ww = x1 - x0, ntx = tx1 - tx0;
  for (int ty = ty0; ty < ty1; ++ty)
    for (int tx = tx0; tx < tx1; ++tx) {
      bool covered = true;
      float dmax = 0.f;
      for (int j = ty * p.tile; j < std::min((ty + 1) * p.tile, cam.height) && covered; ++j)
        for (int i = tx * p.tile; i < std::min((tx + 1) * p.tile, cam.width); ++i) {
          const MeshPix& mp = pix[(size_t)(j - y0) * ww + (i - x0)];
          if (mp.key == ~0ull) {
            covered = false;
            break;
          }
          dmax = std::max(dmax, (float)mp.z);
        }
      if (!covered) continue;
      auto& l = lists[(size_t)(ty - ty0) * ntx + (tx - tx0)];
      std::vector<Cand> kept;
      for (const Cand& c : l)
        if ((float)recs[c.g].zf < dmax) kept.push_back(c);
      l.swap(kept);
    }
}

struct Frame {
  std::vector<Rec> recs;
  std::vector<MeshPix> mesh;
  std::vector<std::vector<Cand>> lists;
  int tx0, ty0, tx1, ty1;
};

Frame prepare(const or_scene& sc, const or_camera& cam, const or_params& p, int wx0, int wy0,
              int wx1, int wy1) {
  Frame f;
  f.recs = project_all(sc, cam, p);
  mesh_pass(sc, cam, p, wx0, wy0, wx1, wy1, f.mesh);
  f.tx0 = wx0 / p.tile;
  f.ty0 = wy0 / p.tile;
  f.tx1 = (wx1 + p.tile - 1) / p.tile;
  f.ty1 = (wy1 + p.tile - 1) / p.tile;
  f.lists = tile_lists(f.recs, p, f.tx0, f.ty0, f.tx1, f.ty1);
  if (p.flags & OR_CULL_MESH) cull_behind_mesh(sc, cam, p, f.recs, f.tx0, f.ty0, f.tx1, f.ty1, f.lists);
  return f;
}

}  // namespace

extern "C" {

int or_abi_version(void) { return 1; }

// Threads an OpenMP loop of the oracle runs on (the timing harness reports it).
int or_max_threads(void) {
  int n = 1;
#pragma omp parallel
  {
#pragma omp single
    n = omp_get_num_threads();
  }
  return n;
}

// Per-Gaussian projected records for one camera.
int or_project(const or_scene* sc, const or_camera* cam, const or_params* p, or_proj_out* o) {
  if (!sc || !cam || !p || !o || p->tile <= 0) return 1;
  std::vector<Rec> recs = project_all(*sc, *cam, *p);
  for (int g = 0; g < sc->n; ++g) {
    const Rec& r = recs[g];
    if (o->amb) o->amb[g] = r.amb;
    if (o->radius) o->radius[g] = r.vis ? r.r : 0;
    if (o->tiles) o->tiles[g] = r.vis ? (r.x1 - r.x0) * (r.y1 - r.y0) : 0;
    if (!r.vis) continue;
    if (o->mean2d) { o->mean2d[2 * g] = r.u; o->mean2d[2 * g + 1] = r.v; }
    for (int i = 0; i < 3; ++i) {
      if (o->conic) o->conic[3 * g + i] = r.con[i];
      if (o->cov2d) o->cov2d[3 * g + i] = r.cov[i];
      if (o->rgb) o->rgb[3 * g + i] = r.rgb[i];
    }
    if (o->opacity) o->opacity[g] = r.opr;  // the record's opacity (Mip factors included)
    if (o->depth) o->depth[g] = r.pc[2];
    if (o->depth_bits) o->depth_bits[g] = r.dbits;
    if (o->rect) {
      o->rect[4 * g] = r.x0; o->rect[4 * g + 1] = r.x1;
      o->rect[4 * g + 2] = r.y0; o->rect[4 * g + 3] = r.y1;
    }
  }
  return 0;
}

// Mip-Splatting 3D smoothing variance of every Gaussian: s / nu^2, with nu
// the highest sampling rate fx / z over the cameras that see the centre in
// front of the near plane inside the view widened by 15% on each side.
// Gaussians no camera sees take the largest variance of the seen ones (0
// when none is seen).
int or_mip_filter3d(const or_scene* sc, const or_camera* cams, int n_cams, const or_params* p,
                    double s, double* out) {
  if (!sc || !cams || !p || !out || n_cams < 1) return 1;
  double vmax = 0.0;
  std::vector<char> seen(sc->n, 0);
  for (int g = 0; g < sc->n; ++g) {
    const double* mu = sc->means + 3 * (size_t)g;
    double nu = 0.0;
    for (int c = 0; c < n_cams; ++c) {
      const or_camera& cam = cams[c];
      double pc[3];
      for (int i = 0; i < 3; ++i)
        pc[i] = cam.R[3 * i] * mu[0] + cam.R[3 * i + 1] * mu[1] + cam.R[3 * i + 2] * mu[2] + cam.t[i];
      if (!(pc[2] > p->near_gs)) continue;
      const double u = cam.fx * pc[0] / pc[2] + cam.cx, v = cam.fy * pc[1] / pc[2] + cam.cy;
      if (u < -0.15 * cam.width || u > 1.15 * cam.width || v < -0.15 * cam.height ||
          v > 1.15 * cam.height)
        continue;
      nu = std::max(nu, cam.fx / pc[2]);
    }
    if (nu > 0.0) {
      seen[g] = 1;
      out[g] = s / (nu * nu);
      vmax = std::max(vmax, out[g]);
    }
  }
  for (int g = 0; g < sc->n; ++g)
    if (!seen[g]) out[g] = vmax;
  return 0;
}

// Sorted (tile << 32 | depth bits, index) pairs and per-tile [start, end).
// Returns the pair count; arrays are filled when capacity allows.
int64_t or_keys(const or_scene* sc, const or_camera* cam, const or_params* p, uint64_t* keys,
                uint32_t* values, uint32_t* ranges, int64_t capacity) {
  if (!sc || !cam || !p || p->tile <= 0) return -1;
  std::vector<Rec> recs = project_all(*sc, *cam, *p);
  const int TX = tiles_x(*cam, *p), TY = tiles_y(*cam, *p);
  auto lists = tile_lists(recs, *p, 0, 0, TX, TY);
  if (p->flags & OR_CULL_MESH) cull_behind_mesh(*sc, *cam, *p, recs, 0, 0, TX, TY, lists);
  int64_t K = 0;
  for (auto& l : lists) K += (int64_t)l.size();
  if (keys && values && ranges && capacity >= K) {
    int64_t o = 0;
    for (int t = 0; t < TX * TY; ++t) {
      ranges[2 * t] = (uint32_t)o;
      for (const Cand& c : lists[t]) {
        keys[o] = ((uint64_t)t << 32) | c.dbits;
        values[o] = (uint32_t)c.g;
        ++o;
      }
      ranges[2 * t + 1] = (uint32_t)o;
    }
  }
  return K;
}

// Forward render of the pixels in window [wx0,wx1) x [wy0,wy1).
int or_render(const or_scene* sc, const or_camera* cam, const or_params* p, int wx0, int wy0,
              int wx1, int wy1, or_render_out* o) {
  if (!sc || !cam || !p || !o || p->tile <= 0) return 1;
  if (wx0 < 0 || wy0 < 0 || wx1 > cam->width || wy1 > cam->height || wx0 >= wx1 || wy0 >= wy1)
    return 1;
  Frame f = prepare(*sc, *cam, *p, wx0, wy0, wx1, wy1);
  const int ww = wx1 - wx0, wh = wy1 - wy0;
  const int ntx = f.tx1 - f.tx0;
  std::vector<uint64_t> hashes((size_t)ww * wh);
#pragma omp parallel for schedule(dynamic, 16)
  for (int idx = 0; idx < ww * wh; ++idx) {
    const int i = wx0 + idx % ww, j = wy0 + idx / ww;
    const MeshPix& mp = f.mesh[idx];
    const bool has = mp.key != ~0ull;
    const int face = has ? (int)((mp.key & 0xffffffffull) >> 1) : -1;
    const float Dm = has ? (float)mp.z : std::numeric_limits<float>::infinity();
    double Im[3] = {0, 0, 0};
    if (has) {
      Bilin b = bilinear(*sc, face, mp.uv);
      for (int c = 0; c < 3; ++c)
        Im[c] = (1 - b.fx) * (1 - b.fy) * texel(*sc, b.tex, b.j0, b.i0, c) +
                b.fx * (1 - b.fy) * texel(*sc, b.tex, b.j0, b.i1, c) +
                (1 - b.fx) * b.fy * texel(*sc, b.tex, b.j1, b.i0, c) +
                b.fx * b.fy * texel(*sc, b.tex, b.j1, b.i1, c);
    }
    const auto& list = f.lists[(size_t)(j / p->tile - f.ty0) * ntx + (i / p->tile - f.tx0)];
    double C[3], T;
    int nc, nb, npro;
    uint8_t amb = has && mp.amb ? 16 : 0;
    uint64_t h;
    std::vector<Decision> near;
    blend_pixel(f.recs, list, *p, i + 0.5, j + 0.5, Dm, nullptr, C, &T, &nc, &nb, &npro, &amb, &h,
                nullptr, &near);
    const size_t hw = (size_t)ww * wh;
    double B[3];
    for (int c = 0; c < 3; ++c) {
      B[c] = has ? Im[c] : p->bg[c];
      if (o->image) o->image[c * hw + idx] = C[c] + T * B[c];
      if (o->mesh_rgb) o->mesh_rgb[c * hw + idx] = Im[c];
    }
    if (o->n_alt && o->alts) {
      // depth-first over the ambiguous decisions: a path flips a set of them,
      // each later in the list than the previous flip and met (within the
      // slack) on the path so far; every path is one possible FP32 outcome
      double* al = o->alts + (size_t)idx * OR_MAX_ALT * 7;
      int n_alt = 0;
      auto put = [&](const double* Cc, double Tt, int a, int b, int c) {
        double* q = al + (size_t)n_alt * 7;
        for (int ch = 0; ch < 3; ++ch) q[ch] = Cc[ch] + Tt * B[ch];
        q[3] = Tt; q[4] = a; q[5] = b; q[6] = c;
        ++n_alt;
      };
      put(C, T, nc, nb, npro);
      std::vector<std::pair<std::vector<Decision>, std::vector<Decision>>> stack;
      stack.push_back({{}, near});
      while (!stack.empty()) {
        auto [flips, met] = stack.back();
        stack.pop_back();
        for (const Decision& d : met) {
          if (!flips.empty() && !(flips.back() < d)) continue;
          if (n_alt == OR_MAX_ALT) {
            amb |= 32;
            break;
          }
          std::vector<Decision> f2 = flips;
          f2.push_back(d);
          std::vector<Decision> met2;
          double C2[3], T2;
          int nc2, nb2, np2;
          uint8_t amb2 = 0;
          uint64_t h2;
          blend_pixel(f.recs, list, *p, i + 0.5, j + 0.5, Dm, nullptr, C2, &T2, &nc2, &nb2, &np2,
                      &amb2, &h2, &f2, &met2);
          put(C2, T2, nc2, nb2, np2);
          stack.push_back({f2, met2});
        }
      }
      o->n_alt[idx] = n_alt;
    }
    if (o->final_T) o->final_T[idx] = T;
    if (o->n_contrib) o->n_contrib[idx] = nc;
    if (o->n_blended) o->n_blended[idx] = nb;
    if (o->n_processed) o->n_processed[idx] = npro;
    if (o->amb) o->amb[idx] = amb;
    if (o->tri_id) o->tri_id[idx] = face;
    if (o->mesh_depth) o->mesh_depth[idx] = Dm;
    hashes[idx] = mix(h, (uint64_t)face + 7);
  }
  if (o->trace) {
    uint64_t h = 0;
    for (uint64_t v : hashes) h = mix(h, v);
    for (const Rec& r : f.recs) {
      h = mix(h, r.vis ? ((uint64_t)r.r << 40 | (uint64_t)r.x0 << 30 | (uint64_t)r.x1 << 20 |
                          (uint64_t)r.y0 << 10 | (uint64_t)r.y1)
                       : 1);
      if (r.vis) h = mix(h, (uint64_t)r.clamped[0] | (uint64_t)r.clamped[1] << 1 |
                                (uint64_t)r.clamped[2] << 2 | (uint64_t)r.clx << 3 |
                                (uint64_t)r.cly << 4);
    }
    *o->trace = h;
  }
  return 0;
}

// Reverse mode over a stored tape: the gradient of
//   F = sum(g_image * I_h) + sum(g_T * T) + sum(g_mesh_rgb * I_m)
// over the window, with respect to all Gaussian parameters and the texture.
// Gradients are accumulated (+=) into `o` (any pointer may be null).
int or_backward(const or_scene* sc, const or_camera* cam, const or_params* p, int wx0, int wy0,
                int wx1, int wy1, const double* g_image, const double* g_T,
                const double* g_mesh_rgb, or_grads* o) {
  if (!sc || !cam || !p || !o || p->tile <= 0) return 1;
  if (wx0 < 0 || wy0 < 0 || wx1 > cam->width || wy1 > cam->height || wx0 >= wx1 || wy0 >= wy1)
    return 1;
  Frame f = prepare(*sc, *cam, *p, wx0, wy0, wx1, wy1);
  const int ww = wx1 - wx0, wh = wy1 - wy0;
  const int ntx = f.tx1 - f.tx0;
  const size_t hw = (size_t)ww * wh;
  const int n = sc->n;
  // per-Gaussian gradient of the record: u, v, conic[3], opacity, rgb[3]
  std::vector<double> grec((size_t)n * 9, 0.0);
  std::vector<double> gtex;
  if (o->tex) gtex.assign((size_t)sc->n_tex * sc->tex_h * sc->tex_w * 3, 0.0);
  // pixels are processed sequentially so that the accumulation order is fixed
  std::vector<Step> tape;
  for (size_t idx = 0; idx < hw; ++idx) {
    const int i = wx0 + (int)(idx % ww), j = wy0 + (int)(idx / ww);
    const MeshPix& mp = f.mesh[idx];
    const bool has = mp.key != ~0ull;
    const int face = has ? (int)((mp.key & 0xffffffffull) >> 1) : -1;
    const float Dm = has ? (float)mp.z : std::numeric_limits<float>::infinity();
    Bilin b{};
    double B[3];
    for (int c = 0; c < 3; ++c) B[c] = p->bg[c];
    if (has) {
      b = bilinear(*sc, face, mp.uv);
      for (int c = 0; c < 3; ++c)
        B[c] = (1 - b.fx) * (1 - b.fy) * texel(*sc, b.tex, b.j0, b.i0, c) +
               b.fx * (1 - b.fy) * texel(*sc, b.tex, b.j0, b.i1, c) +
               (1 - b.fx) * b.fy * texel(*sc, b.tex, b.j1, b.i0, c) +
               b.fx * b.fy * texel(*sc, b.tex, b.j1, b.i1, c);
    }
    const auto& list = f.lists[(size_t)(j / p->tile - f.ty0) * ntx + (i / p->tile - f.tx0)];
    tape.clear();
    double C[3], Tf;
    int nc, nb, npro;
    uint8_t amb = 0;
    uint64_t h;
    blend_pixel(f.recs, list, *p, i + 0.5, j + 0.5, Dm, &tape, C, &Tf, &nc, &nb, &npro, &amb, &h);
    double gC[3], gT = g_T ? g_T[idx] : 0.0;
    for (int c = 0; c < 3; ++c) {
      gC[c] = g_image ? g_image[c * hw + idx] : 0.0;
      gT += gC[c] * B[c];
    }
    if (has && !gtex.empty()) {
      for (int c = 0; c < 3; ++c) {
        const double gm = Tf * gC[c] + (g_mesh_rgb ? g_mesh_rgb[c * hw + idx] : 0.0);
        auto add = [&](int jj, int ii, double w) {
          gtex[(((size_t)b.tex * sc->tex_h + jj) * sc->tex_w + ii) * 3 + c] += w * gm;
        };
        add(b.j0, b.i0, (1 - b.fx) * (1 - b.fy));
        add(b.j0, b.i1, b.fx * (1 - b.fy));
        add(b.j1, b.i0, (1 - b.fx) * b.fy);
        add(b.j1, b.i1, b.fx * b.fy);
      }
    }
    // reverse sweep: S = colour accumulated behind step k (from T = 1 after it),
    // P = product of (1 - alpha) behind step k
    double S[3] = {0, 0, 0}, P = 1.0;
    for (int k = (int)tape.size() - 1; k >= 0; --k) {
      const Step& st = tape[k];
      const Rec& r = f.recs[st.g];
      double* gr = &grec[(size_t)st.g * 9];
      double galpha = 0.0;
      for (int c = 0; c < 3; ++c) {
        gr[6 + c] += st.alpha * st.T * gC[c];
        galpha += st.T * (r.brgb[c] - S[c]) * gC[c];
      }
      galpha += gT * (-st.T * P);  // dT_final / dalpha_k = -T_k * prod_{j>k} (1 - alpha_j)
      for (int c = 0; c < 3; ++c) S[c] = st.alpha * r.brgb[c] + (1.0 - st.alpha) * S[c];
      P *= (1.0 - st.alpha);
      if (st.clamped) continue;
      gr[5] += galpha * st.G;  // d alpha / d opacity
      const double gpow = galpha * r.bop * st.G;
      const double dx = (i + 0.5) - r.bu, dy = (j + 0.5) - r.bv;
      // power = -1/2 (a dx^2 + c dy^2) - b dx dy,  dx = px - u
      gr[0] += gpow * (r.bcon[0] * dx + r.bcon[1] * dy);
      gr[1] += gpow * (r.bcon[2] * dy + r.bcon[1] * dx);
      gr[2] += gpow * (-0.5 * dx * dx);
      gr[3] += gpow * (-dx * dy);
      gr[4] += gpow * (-0.5 * dy * dy);
    }
  }
  if (o->tex)
    for (size_t k = 0; k < gtex.size(); ++k) o->tex[k] += gtex[k];

  // chain rule from records to parameters
  const int K = (sc->sh_degree + 1) * (sc->sh_degree + 1);
  const double* W = cam->R;
#pragma omp parallel for schedule(static)
  for (int g = 0; g < n; ++g) {
    const double* gr = &grec[(size_t)g * 9];
    if (o->mean2d) {
      o->mean2d[2 * g] += gr[0];
      o->mean2d[2 * g + 1] += gr[1];
    }
    bool any = false;
    for (int k = 0; k < 9; ++k) any = any || gr[k] != 0.0;
    if (!any) continue;
    const Rec& r = f.recs[g];
    double gpc[3] = {0, 0, 0}, gmu[3] = {0, 0, 0};
    // opacity: the record holds op c3 c2
    if (o->opacity_logits) o->opacity_logits[g] += gr[5] * r.c3 * r.c2 * r.op * (1.0 - r.op);
    // c3 = prod s_i / sqrt(s_i^2 + f3):  d c3 / d log s_i = c3 f3 / (s_i^2 + f3)
    double gls_mip[3] = {0, 0, 0};
    if (r.f3 > 0.0)
      for (int i = 0; i < 3; ++i)
        gls_mip[i] = gr[5] * r.op * r.c2 * r.c3 * r.f3 / (r.s[i] * r.s[i] + r.f3);
    // c2 = sqrt(D0 / D1), D1 = det(cov), D0 = det(cov - low_pass I):
    // d c2 = c2 / 2 (dD0 / D0 - dD1 / D1), as a gradient on (a, b, c) of cov
    double gcov_mip[3] = {0, 0, 0};
    if ((p->flags & OR_MIP_2D) && !r.c2lo) {
      const double a = r.cov[0], b = r.cov[1], c = r.cov[2], k = p->low_pass;
      const double D1 = a * c - b * b, D0 = (a - k) * (c - k) - b * b;
      const double gc2 = gr[5] * r.op * r.c3 * 0.5 * r.c2;
      gcov_mip[0] = gc2 * ((c - k) / D0 - c / D1);
      gcov_mip[1] = gc2 * (-2.0 * b / D0 + 2.0 * b / D1);
      gcov_mip[2] = gc2 * ((a - k) / D0 - a / D1);
    }
    // colour
    {
      double Y[16], GY[16][3];
      sh_basis(r.dir, Y, sc->sh_degree);
      sh_basis_grad(r.dir, GY, sc->sh_degree);
      const double* shc = sc->sh + (size_t)g * K * 3;
      double gdir[3] = {0, 0, 0};
      for (int c = 0; c < 3; ++c) {
        if (r.clamped[c]) continue;
        for (int k = 0; k < K; ++k) {
          if (o->sh) o->sh[((size_t)g * K + k) * 3 + c] += Y[k] * gr[6 + c];
          for (int a = 0; a < 3; ++a) gdir[a] += GY[k][a] * shc[3 * k + c] * gr[6 + c];
        }
      }
      const double dd = gdir[0] * r.dir[0] + gdir[1] * r.dir[1] + gdir[2] * r.dir[2];
      for (int a = 0; a < 3; ++a) gmu[a] += (gdir[a] - r.dir[a] * dd) / r.dnorm;
    }
    // conic -> 2D covariance: G = [[ga, gb/2],[gb/2, gc]], H = -Q G Q
    const double Q[4] = {r.con[0], r.con[1], r.con[1], r.con[2]};
    const double Gm[4] = {gr[2], 0.5 * gr[3], 0.5 * gr[3], gr[4]};
    double QG[4], H[4];
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 2; ++c) QG[2 * a + c] = Q[2 * a] * Gm[c] + Q[2 * a + 1] * Gm[2 + c];
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 2; ++c) H[2 * a + c] = -(QG[2 * a] * Q[c] + QG[2 * a + 1] * Q[2 + c]);
    // the off-diagonal b of cov sits in two entries of the symmetric matrix
    H[0] += gcov_mip[0];
    H[1] += 0.5 * gcov_mip[1];
    H[2] += 0.5 * gcov_mip[1];
    H[3] += gcov_mip[2];
    // Sigma' = J Sc J^T + lp I:  dSc = J^T H J,  dJ = 2 H J Sc
    double gSc[9], HJ[6], gJ[6];
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 3; ++c) HJ[3 * a + c] = H[2 * a] * r.J[c] + H[2 * a + 1] * r.J[3 + c];
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) gSc[3 * a + c] = r.J[a] * HJ[c] + r.J[3 + a] * HJ[3 + c];
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 3; ++c) {
        double s = 0;
        for (int k = 0; k < 3; ++k) s += HJ[3 * a + k] * r.Sc[3 * k + c];
        gJ[3 * a + c] = 2.0 * s;
      }
    const double x = r.pc[0], y = r.pc[1], z = r.pc[2];
    const double fx = cam->fx, fy = cam->fy;
    // J00 = fx/z, J02 = -fx xc / z (xc = x/z unless clamped), same for row 1
    gpc[2] += gJ[0] * (-fx / (z * z)) + gJ[4] * (-fy / (z * z));
    if (r.clx) {
      gpc[2] += gJ[2] * (fx * r.xc / (z * z));
    } else {
      gpc[0] += gJ[2] * (-fx / (z * z));
      gpc[2] += gJ[2] * (2.0 * fx * x / (z * z * z));
    }
    if (r.cly) {
      gpc[2] += gJ[5] * (fy * r.yc / (z * z));
    } else {
      gpc[1] += gJ[5] * (-fy / (z * z));
      gpc[2] += gJ[5] * (2.0 * fy * y / (z * z * z));
    }
    // mean2D
    gpc[0] += gr[0] * fx / z;
    gpc[1] += gr[1] * fy / z;
    gpc[2] += gr[0] * (-fx * x / (z * z)) + gr[1] * (-fy * y / (z * z));
    for (int a = 0; a < 3; ++a)
      gmu[a] += W[a] * gpc[0] + W[3 + a] * gpc[1] + W[6 + a] * gpc[2];
    if (o->means)
      for (int a = 0; a < 3; ++a) o->means[3 * g + a] += gmu[a];
    // Sc = W Sig W^T -> gSig = W^T gSc W
    double tmp[9], gSig[9];
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) {
        double s = 0;
        for (int k = 0; k < 3; ++k) s += W[3 * k + a] * gSc[3 * k + c];
        tmp[3 * a + c] = s;
      }
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) {
        double s = 0;
        for (int k = 0; k < 3; ++k) s += tmp[3 * a + k] * W[3 * k + c];
        gSig[3 * a + c] = s;
      }
    // Sig = M M^T, M = Rq diag(s): gM = (gSig + gSig^T) M
    double M[9], gM[9];
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) M[3 * a + c] = r.Rq[3 * a + c] * r.s[c];
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) {
        double s = 0;
        for (int k = 0; k < 3; ++k) s += (gSig[3 * a + k] + gSig[3 * k + a]) * M[3 * k + c];
        gM[3 * a + c] = s;
      }
    double gR[9];
    for (int c = 0; c < 3; ++c) {
      double gs = 0;
      for (int a = 0; a < 3; ++a) {
        gs += gM[3 * a + c] * r.Rq[3 * a + c];
        gR[3 * a + c] = gM[3 * a + c] * r.s[c];
      }
      if (o->log_scales) o->log_scales[3 * g + c] += gs * r.s[c] + gls_mip[c];
    }
    const double w = r.qn[0], qx = r.qn[1], qy = r.qn[2], qz = r.qn[3];
    double gq[4];
    gq[0] = 2 * (-qz * gR[1] + qy * gR[2] + qz * gR[3] - qx * gR[5] - qy * gR[6] + qx * gR[7]);
    gq[1] = 2 * (qy * gR[1] + qz * gR[2] + qy * gR[3] - 2 * qx * gR[4] - w * gR[5] + qz * gR[6] +
                 w * gR[7] - 2 * qx * gR[8]);
    gq[2] = 2 * (-2 * qy * gR[0] + qx * gR[1] + w * gR[2] + qx * gR[3] + qz * gR[5] - w * gR[6] +
                 qz * gR[7] - 2 * qy * gR[8]);
    gq[3] = 2 * (-2 * qz * gR[0] - w * gR[1] + qx * gR[2] + w * gR[3] - 2 * qz * gR[4] +
                 qy * gR[5] + qx * gR[6] + qy * gR[7]);
    const double dq = gq[0] * r.qn[0] + gq[1] * r.qn[1] + gq[2] * r.qn[2] + gq[3] * r.qn[3];
    if (o->quats)
      for (int a = 0; a < 4; ++a) o->quats[4 * g + a] += (gq[a] - r.qn[a] * dq) / r.qnorm;
  }
  return 0;
}

// SH basis at unit directions (used by the orthonormality pins)
void or_sh_basis(int deg, int n, const double* dirs, double* out) {
  const int K = (deg + 1) * (deg + 1);
  for (int i = 0; i < n; ++i) {
    double Y[16];
    sh_basis(dirs + 3 * i, Y, deg);
    for (int k = 0; k < K; ++k) out[(size_t)i * K + k] = Y[k];
  }
}

void or_quat_to_rot(const double* q, double* R) {
  double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double qn[4] = {q[0] / n, q[1] / n, q[2] / n, q[3] / n};
  quat_to_rot(qn, R);
}

}  // extern "C"
