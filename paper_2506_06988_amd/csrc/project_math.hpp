// Device-side projection of one Gaussian into one camera, in FP64 (Sec. 3.1):
// opacity, Sigma = R S S^T R^T, Sigma' = J W Sigma W^T J^T + low-pass, conic,
// 3-sigma radius and tile rectangle, view-dependent SH colour, depth key.
// Shared by the forward projection and its backward (which recomputes it).
#pragma once

#include "common.hpp"

namespace hr {

struct Proj {
  bool vis;
  double pc[3];      // camera-space centre
  double op;         // opacity
  double s[3];       // scales
  double qn[4];      // normalised quaternion
  double qnorm;
  double Rq[9];      // rotation of the Gaussian
  double N[9];       // W Rq S, so that Sigma_cam = N N^T
  double J[4];       // j00, j02, j11, j12 of the 2x3 Jacobian
  bool clx, cly;     // direction clamped in x / y
  double xc, yc;     // (clamped) x/z and y/z
  double Sc[6];      // camera-space covariance, xx xy xz yy yz zz
  double cov[3];     // Sigma' (a, b, c)
  double con[3];     // conic
  double u, v;       // mean2D
  int r, x0, x1, y0, y1;
  double dir[3], dnorm;
  double rgb[3];
  bool clamped[3];
  float zf;
  // Mip-Splatting: 3D variance f3 and opacity factor c3, 2D factor c2 (c2lo:
  // at its floor); opr = op c3 c2 is the record's opacity
  double f3, c3, c2, opr;
  bool c2lo;
};

// Real spherical harmonics without the Condon-Shortley phase, orthonormal on
// the sphere, index l*l + l + m. Constants are sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!)
// times the normalisation of the cos/sin combination, written out in closed
// form (computed in FP64, then rounded to T).
template <typename T>
__device__ __forceinline__ void sh_eval(const T d[3], int deg, T* Y) {
  constexpr double PI = 3.14159265358979323846;
  const T x = d[0], y = d[1], z = d[2];
  Y[0] = T(0.5 * sqrt(1.0 / PI));
  if (deg < 1) return;
  const T c1 = T(sqrt(3.0 / (4.0 * PI)));
  Y[1] = c1 * y;
  Y[2] = c1 * z;
  Y[3] = c1 * x;
  if (deg < 2) return;
  const T a2 = T(0.5 * sqrt(15.0 / PI)), b2 = T(0.25 * sqrt(5.0 / PI)),
          d2 = T(0.25 * sqrt(15.0 / PI));
  const T xx = x * x, yy = y * y, zz = z * z;
  Y[4] = a2 * x * y;
  Y[5] = a2 * y * z;
  Y[6] = b2 * (T(3) * zz - T(1));
  Y[7] = a2 * x * z;
  Y[8] = d2 * (xx - yy);
  if (deg < 3) return;
  const T e3 = T(0.25 * sqrt(35.0 / (2.0 * PI))), f3 = T(0.5 * sqrt(105.0 / PI)),
          g3 = T(0.25 * sqrt(21.0 / (2.0 * PI))), h3 = T(0.25 * sqrt(7.0 / PI)),
          k3 = T(0.25 * sqrt(105.0 / PI));
  Y[9] = e3 * y * (T(3) * xx - yy);
  Y[10] = f3 * x * y * z;
  Y[11] = g3 * y * (T(5) * zz - T(1));
  Y[12] = h3 * z * (T(5) * zz - T(3));
  Y[13] = g3 * x * (T(5) * zz - T(1));
  Y[14] = k3 * z * (xx - yy);
  Y[15] = e3 * x * (xx - T(3) * yy);
}

// d/d(x,y,z) of each polynomial of sh_eval, accumulated against weights w[k]:
// g += sum_k w[k] grad Y_k
template <typename T>
__device__ __forceinline__ void sh_grad_acc(const T d[3], int deg, const T* w, T g[3]) {
  constexpr double PI = 3.14159265358979323846;
  const T x = d[0], y = d[1], z = d[2];
  if (deg < 1) return;
  const T c1 = T(sqrt(3.0 / (4.0 * PI)));
  g[1] += c1 * w[1];
  g[2] += c1 * w[2];
  g[0] += c1 * w[3];
  if (deg < 2) return;
  const T a2 = T(0.5 * sqrt(15.0 / PI)), b2 = T(0.25 * sqrt(5.0 / PI)),
          d2 = T(0.25 * sqrt(15.0 / PI));
  g[0] += a2 * (y * w[4] + z * w[7]) + T(2) * d2 * x * w[8];
  g[1] += a2 * (x * w[4] + z * w[5]) - T(2) * d2 * y * w[8];
  g[2] += a2 * (y * w[5] + x * w[7]) + T(6) * b2 * z * w[6];
  if (deg < 3) return;
  const T e3 = T(0.25 * sqrt(35.0 / (2.0 * PI))), f3 = T(0.5 * sqrt(105.0 / PI)),
          g3 = T(0.25 * sqrt(21.0 / (2.0 * PI))), h3 = T(0.25 * sqrt(7.0 / PI)),
          k3 = T(0.25 * sqrt(105.0 / PI));
  const T xx = x * x, yy = y * y, zz = z * z;
  g[0] += e3 * T(6) * x * y * w[9] + f3 * y * z * w[10] + g3 * (T(5) * zz - T(1)) * w[13] +
          T(2) * k3 * x * z * w[14] + e3 * T(3) * (xx - yy) * w[15];
  g[1] += e3 * T(3) * (xx - yy) * w[9] + f3 * x * z * w[10] + g3 * (T(5) * zz - T(1)) * w[11] -
          T(2) * k3 * y * z * w[14] - e3 * T(6) * x * y * w[15];
  g[2] += f3 * x * y * w[10] + T(10) * g3 * y * z * w[11] + h3 * (T(15) * zz - T(3)) * w[12] +
          T(10) * g3 * x * z * w[13] + k3 * (xx - yy) * w[14];
}

// View-dependent colour before the clamp, in FP64: acc[ch] = 1/2 + sum_k
// Y_k(dir) sh[k][ch], each channel summed in increasing k (the forward's and
// the backward's clamp decisions come from this one function).
__device__ __forceinline__ void sh_colour64(const float* __restrict__ shg, int deg,
                                            const double dir[3], double acc[3]) {
  const int K = (deg + 1) * (deg + 1);
  double Y[16];
  sh_eval(dir, deg, Y);
  acc[0] = acc[1] = acc[2] = 0.5;
  if ((((uintptr_t)shg) & 15u) == 0 && (3 * K) % 4 == 0) {
    // 3K floats as 16-byte vectors (K = 4, 16 give 12 and 48 floats)
    const float4* v4 = reinterpret_cast<const float4*>(shg);
    for (int i = 0; i < (3 * K) / 4; ++i) {
      const float4 f = v4[i];
      const float e[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int idx = 4 * i + k;
        acc[idx % 3] += Y[idx / 3] * (double)e[k];
      }
    }
  } else {
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) acc[ch] += Y[k] * (double)shg[3 * k + ch];
  }
}

__device__ __forceinline__ int clamp_tile(double v, int hi) {
  if (!(v > 0.0)) return 0;
  if (v > (double)hi) return hi;
  return (int)v;
}

__device__ __forceinline__ bool finite_f(float v) { return isfinite(v); }

// full projection; `need_colour` false skips the SH evaluation
__device__ __forceinline__ void project_gaussian(const SetDev& S, const CamDev& cam,
                                                 const float* __restrict__ means,
                                                 const float* __restrict__ log_scales,
                                                 const float* __restrict__ quats,
                                                 const float* __restrict__ logits,
                                                 const float* __restrict__ sh, int g, Proj& P,
                                                 bool need_colour = true) {
  P.vis = false;
  const int K = (S.sh_degree + 1) * (S.sh_degree + 1);
  const float m0 = means[3 * g], m1 = means[3 * g + 1], m2 = means[3 * g + 2];
  const float l0 = log_scales[3 * g], l1 = log_scales[3 * g + 1], l2 = log_scales[3 * g + 2];
  const float4 q4 = *reinterpret_cast<const float4*>(quats + 4 * (size_t)g);
  const float lg = logits[g];
  // non-finite SH coefficients give a non-finite colour, which culls below
  const bool fin = finite_f(m0) && finite_f(m1) && finite_f(m2) && finite_f(l0) &&
                   finite_f(l1) && finite_f(l2) && finite_f(q4.x) && finite_f(q4.y) &&
                   finite_f(q4.z) && finite_f(q4.w) && finite_f(lg);
  if (!fin) return;
  const float* shg = sh + (size_t)g * K * 3;

  const double mu[3] = {m0, m1, m2};
  for (int i = 0; i < 3; ++i)
    P.pc[i] = cam.R[3 * i] * mu[0] + cam.R[3 * i + 1] * mu[1] + cam.R[3 * i + 2] * mu[2] + cam.t[i];
  const double x = P.pc[0], y = P.pc[1], z = P.pc[2];
  if (!(z > (double)S.near_gs)) return;

  P.op = 1.0 / (1.0 + exp(-(double)lg));
  P.s[0] = exp((double)l0);
  P.s[1] = exp((double)l1);
  P.s[2] = exp((double)l2);
  const double qw = q4.x, qx = q4.y, qy = q4.z, qz = q4.w;
  P.qnorm = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  if (!(P.qnorm > 0.0)) return;
  const double inv = 1.0 / P.qnorm;
  const double w = qw * inv, a = qx * inv, b = qy * inv, c = qz * inv;
  P.qn[0] = w; P.qn[1] = a; P.qn[2] = b; P.qn[3] = c;
  double* R = P.Rq;
  R[0] = 1.0 - 2.0 * (b * b + c * c); R[1] = 2.0 * (a * b - w * c); R[2] = 2.0 * (a * c + w * b);
  R[3] = 2.0 * (a * b + w * c); R[4] = 1.0 - 2.0 * (a * a + c * c); R[5] = 2.0 * (b * c - w * a);
  R[6] = 2.0 * (a * c - w * b); R[7] = 2.0 * (b * c + w * a); R[8] = 1.0 - 2.0 * (a * a + b * b);
  // N = W Rq S; Sigma_cam = N N^T
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      P.N[3 * i + j] = (cam.R[3 * i] * R[j] + cam.R[3 * i + 1] * R[3 + j] + cam.R[3 * i + 2] * R[6 + j]) * P.s[j];
  const double* N = P.N;
  auto dot3 = [&](int i, int k) { return N[3 * i] * N[3 * k] + N[3 * i + 1] * N[3 * k + 1] + N[3 * i + 2] * N[3 * k + 2]; };
  P.Sc[0] = dot3(0, 0); P.Sc[1] = dot3(0, 1); P.Sc[2] = dot3(0, 2);
  P.Sc[3] = dot3(1, 1); P.Sc[4] = dot3(1, 2); P.Sc[5] = dot3(2, 2);
  // Mip-Splatting 3D smoothing: W (Sigma + f3 I) W^T = N N^T + f3 I
  P.f3 = 0.0;
  P.c3 = 1.0;
  if (S.filter3d) {
    const float f = S.filter3d[g];
    if (!(isfinite(f) && f >= 0.f)) return;
    P.f3 = (double)f;
    P.Sc[0] += P.f3;
    P.Sc[3] += P.f3;
    P.Sc[5] += P.f3;
#pragma unroll
    for (int i = 0; i < 3; ++i) P.c3 *= P.s[i] / sqrt(P.s[i] * P.s[i] + P.f3);
  }

  const double xz = x / z, yz = y / z;
  P.clx = xz < -cam.limx || xz > cam.limx;
  P.cly = yz < -cam.limy || yz > cam.limy;
  P.xc = fmin(cam.limx, fmax(-cam.limx, xz));
  P.yc = fmin(cam.limy, fmax(-cam.limy, yz));
  const double j00 = cam.fx / z, j02 = -cam.fx * P.xc / z;
  const double j11 = cam.fy / z, j12 = -cam.fy * P.yc / z;
  P.J[0] = j00; P.J[1] = j02; P.J[2] = j11; P.J[3] = j12;
  const double* Sc = P.Sc;
  // T = J Sc (rows 0 and 1)
  const double t00 = j00 * Sc[0] + j02 * Sc[2], t01 = j00 * Sc[1] + j02 * Sc[4], t02 = j00 * Sc[2] + j02 * Sc[5];
  const double t11 = j11 * Sc[3] + j12 * Sc[4], t12 = j11 * Sc[4] + j12 * Sc[5];
  P.cov[0] = t00 * j00 + t02 * j02 + (double)S.low_pass;
  P.cov[1] = t01 * j11 + t02 * j12;
  P.cov[2] = t11 * j11 + t12 * j12 + (double)S.low_pass;
  const double det = P.cov[0] * P.cov[2] - P.cov[1] * P.cov[1];
  if (!(det > 0.0)) return;
  // Mip-Splatting 2D filter: opacity times sqrt(det(Sigma') / det(Sigma' + lp I))
  P.c2 = 1.0;
  P.c2lo = false;
  if (S.mip2d) {
    const double lp = (double)S.low_pass;
    const double ratio = ((P.cov[0] - lp) * (P.cov[2] - lp) - P.cov[1] * P.cov[1]) / det;
    P.c2lo = !(ratio > MIP2D_FLOOR);
    P.c2 = sqrt(P.c2lo ? MIP2D_FLOOR : ratio);
  }
  P.opr = P.op * P.c3 * P.c2;
  const double idet = 1.0 / det;
  P.con[0] = P.cov[2] * idet;
  P.con[1] = -P.cov[1] * idet;
  P.con[2] = P.cov[0] * idet;
  P.u = cam.fx * x / z + cam.cx;
  P.v = cam.fy * y / z + cam.cy;
  const double mid = 0.5 * (P.cov[0] + P.cov[2]);
  const double lam = mid + sqrt(fmax(0.1, mid * mid - det));
  P.r = (int)ceil(3.0 * sqrt(lam));
  const double rr = (double)P.r;
  P.x0 = clamp_tile(floor((P.u - rr) / TILE), cam.TX);
  P.x1 = clamp_tile(floor((P.u + rr) / TILE) + 1.0, cam.TX);
  P.y0 = clamp_tile(floor((P.v - rr) / TILE), cam.TY);
  P.y1 = clamp_tile(floor((P.v + rr) / TILE) + 1.0, cam.TY);
  if ((P.x1 - P.x0) * (P.y1 - P.y0) <= 0) return;
  P.zf = __double2float_rn(z);
  if (!need_colour) {
    P.vis = true;
    return;
  }
  const double d0 = mu[0] - cam.C[0], d1 = mu[1] - cam.C[1], d2 = mu[2] - cam.C[2];
  P.dnorm = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  P.dir[0] = d0 / P.dnorm; P.dir[1] = d1 / P.dnorm; P.dir[2] = d2 / P.dnorm;
  double acc[3];
  sh_colour64(shg, S.sh_degree, P.dir, acc);
  bool finite_rgb = true;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    finite_rgb = finite_rgb && isfinite(acc[ch]);
    P.clamped[ch] = acc[ch] < 0.0;
    P.rgb[ch] = P.clamped[ch] ? 0.0 : acc[ch];
  }
  P.vis = finite_rgb;
}

}  // namespace hr
