// The trust region of Algorithm 1, shared by the parameter-update kernels
// and the fused projection backward: the per-Gaussian radius eta =
// SHD(x, eps) and the update of one parameter row.
//
// Paper: Algorithm 1 and Methodology ("Algorithm Design"; "Trust-Region
// Based on Squared Hellinger Distance"; appendix derivations of the bounds).
// Per Gaussian, with alpha = sigmoid(logit), s = exp(log-scale), R from the
// quaternion and L = -ln(1 - eps/alpha) (infinite when eps >= alpha):
//   mean_c      eta = sqrt(8 Sigma_cc L)                     (printed bound)
//   log-scale   eta = sqrt(2 s_c^2 eps / alpha) / s_c = sqrt(2 eps / alpha)
//   quaternion  eta = sqrt(8 L / beta_c),  beta_c = T''(0) of the appendix
//   logit       eta = sqrt(4 alpha eps) / (alpha (1 - alpha))
//   SH (k, c)   eta = sqrt(4 max(C_c, 1/255) eps / alpha) / C0, C_c the base colour
// Readings: the clip acts on raw parameters through the first-order chain
// rule; every SH coefficient of a channel shares the base colour's radius.
// Variants: the mean radius may use 1 / (Sigma^-1)_cc, the exact radius along
// axis c for any rotation (the printed Sigma_cc is exact only for an
// axis-aligned Sigma); and the scale, quaternion, opacity and colour radii
// may use the constants 8/3, 16, 8, 8 instead of 2, 8, 4, 4, with which each
// class spends the whole budget to second order (the printed Taylor steps
// give 0.75, 0.5, 0.5 and 0.5 of it).  The view-dependent SH coefficients
// may share eta_C / S_d (S_d = max over directions of sum_{k>=1} |Y_k| at
// degree d), which bounds the colour change of moving all of them at once.
// beta_c in closed form: R^T dR/dq_c is the skew matrix of the body-frame
// angular velocity w_c = (2/|q|^2) vec(conj(q) e_c), and
//   beta_c = 2 sum_{i<j} A_ij^2 (s_i/s_j - s_j/s_i)^2,
// with A_01 = -w_2, A_02 = w_1, A_12 = -w_0; it vanishes for isotropic s.
//
#pragma once
#include "gs3_internal.h"
#include "gs3tr.h"

namespace gs3trust {

constexpr float SH_C0 = 0.28209479177387814f;

struct Radius {
  float mu[3], ls, q[4], logit, col[3], rest[3];
};

// max over unit directions of sum_{1 <= k < (d+1)^2} |Y_k|, by degree d:
// sqrt(9 / (4 pi)) at d = 1; the others by numerical maximisation
__device__ __forceinline__ float sh_rest_abs_max(int deg) {
  return deg == 1 ? 0.8462843753216346f : (deg == 2 ? 2.145449272073426f : 3.926815898482296f);
}

// Opacity of the radius: the same expression wherever a radius is formed.
__device__ __forceinline__ float radius_alpha(const float* __restrict__ x, int64_t n, int64_t g) {
  return 1.f / (1.f + expf(-x[10 * n + g]));
}

// Mean, log-scale, quaternion and opacity-logit radii of Gaussian g.
__device__ __forceinline__ void radius_geo(const float* __restrict__ x, int64_t n, int64_t g, float eps,
                                           uint32_t variant, float alpha, Radius& o) {
#pragma clang fp contract(off)  // the same rounding in every translation unit that uses it
  const bool second = variant & GS3_TR_SECOND_ORDER;
  const float k_s = second ? 8.f / 3.f : 2.f, k_q = second ? 16.f : 8.f, k_a = second ? 8.f : 4.f;
  const float s0 = expf(x[3 * n + g]), s1 = expf(x[4 * n + g]), s2 = expf(x[5 * n + g]);
  const float qx = x[6 * n + g], qy = x[7 * n + g], qz = x[8 * n + g], qw = x[9 * n + g];
  const float r2 = qx * qx + qy * qy + qz * qz + qw * qw;
  const float ir2 = 1.f / r2;
  // rows of R (normalised), Sigma_cc = sum_k R_ck^2 s_k^2
  const float R00 = 1.f - 2.f * (qy * qy + qz * qz) * ir2, R01 = 2.f * (qx * qy - qw * qz) * ir2,
              R02 = 2.f * (qx * qz + qw * qy) * ir2;
  const float R10 = 2.f * (qx * qy + qw * qz) * ir2, R11 = 1.f - 2.f * (qz * qz + qx * qx) * ir2,
              R12 = 2.f * (qy * qz - qw * qx) * ir2;
  const float R20 = 2.f * (qx * qz - qw * qy) * ir2, R21 = 2.f * (qy * qz + qw * qx) * ir2,
              R22 = 1.f - 2.f * (qx * qx + qy * qy) * ir2;
  const float v0 = s0 * s0, v1 = s1 * s1, v2 = s2 * s2;
  const float L = eps < alpha ? -log1pf(-eps / alpha) : INFINITY;
  if (variant & GS3_TR_MEAN_EXACT) {
    // (Sigma^-1)_cc = sum_k R_ck^2 / s_k^2
    const float w0 = 1.f / v0, w1 = 1.f / v1, w2 = 1.f / v2;
    o.mu[0] = sqrtf(8.f * L / (R00 * R00 * w0 + R01 * R01 * w1 + R02 * R02 * w2));
    o.mu[1] = sqrtf(8.f * L / (R10 * R10 * w0 + R11 * R11 * w1 + R12 * R12 * w2));
    o.mu[2] = sqrtf(8.f * L / (R20 * R20 * w0 + R21 * R21 * w1 + R22 * R22 * w2));
  } else {
    const float Sxx = R00 * R00 * v0 + R01 * R01 * v1 + R02 * R02 * v2;
    const float Syy = R10 * R10 * v0 + R11 * R11 * v1 + R12 * R12 * v2;
    const float Szz = R20 * R20 * v0 + R21 * R21 * v1 + R22 * R22 * v2;
    o.mu[0] = sqrtf(8.f * Sxx * L);
    o.mu[1] = sqrtf(8.f * Syy * L);
    o.mu[2] = sqrtf(8.f * Szz * L);
  }
  o.ls = sqrtf(k_s * eps / alpha);
  const float p01 = s0 / s1 - s1 / s0, p02 = s0 / s2 - s2 / s0, p12 = s1 / s2 - s2 / s1;
  const float e01 = p01 * p01, e02 = p02 * p02, e12 = p12 * p12;
  // vec(conj(q) e_c) for c = x, y, z, w
  const float wv[4][3] = {{qw, -qz, qy}, {qz, qw, -qx}, {-qy, qx, qw}, {-qx, -qy, -qz}};
  const float k2 = 4.f * ir2 * ir2;  // (2 / |q|^2)^2
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float beta = 2.f * k2 * (wv[c][2] * wv[c][2] * e01 + wv[c][1] * wv[c][1] * e02 + wv[c][0] * wv[c][0] * e12);
    o.q[c] = beta > 0.f ? sqrtf(k_q * L / beta) : INFINITY;
  }
  o.logit = sqrtf(k_a * alpha * eps) / (alpha * (1.f - alpha));
}

// Colour radii of Gaussian g: the DC coefficient's (col) and the
// view-dependent coefficients' (rest) per channel.
__device__ __forceinline__ void radius_colour(const float* __restrict__ x, int64_t n, int64_t g, float eps,
                                              uint32_t variant, int deg, float alpha, Radius& o) {
#pragma clang fp contract(off)
  const float k_c = (variant & GS3_TR_SECOND_ORDER) ? 8.f : 4.f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float base = 0.5f + SH_C0 * x[(int64_t)(11 + c) * n + g];
    const float eta_c = sqrtf(k_c * fmaxf(base, GS3_COLOUR_FLOOR) * eps / alpha);
    o.col[c] = eta_c / SH_C0;
    o.rest[c] = (variant & GS3_TR_SH_JOINT) && deg > 0 ? eta_c / sh_rest_abs_max(deg) : o.col[c];
  }
}

__device__ __forceinline__ Radius trust_radius(const float* __restrict__ x, int64_t n, int64_t g, float eps,
                                               uint32_t variant, int deg) {
  Radius o;
  const float alpha = radius_alpha(x, n, g);
  radius_geo(x, n, g, eps, variant, alpha, o);
  radius_colour(x, n, g, eps, variant, deg, alpha, o);
  return o;
}

__device__ __forceinline__ float row_radius(const Radius& r, int row) {
  if (row < 3) return r.mu[row];
  if (row < 6) return r.ls;
  if (row < 10) return r.q[row - 6];
  if (row == 10) return r.logit;
  if (row < 14) return r.col[row - 11];
  return r.rest[(row - 11) % 3];
}

__device__ __forceinline__ float sgnf(float v) { return v > 0.f ? 1.f : (v < 0.f ? -1.f : 0.f); }

// One row of the update of Algorithm 1 from its loaded state: the EMAs (D
// only on a Hutchinson step), dx = -ghat / Dhat where Dhat > 0 (else
// -sign(ghat) eta, or 0 if eta is infinite), clipped to [-eta, eta].
// gh_io / dh_io hold the old EMAs on entry and the new ones on return.
__device__ __forceinline__ float tr_row(float g, float& gh_io, float& dh_io, float D, float eta, const TrArgs& a) {
#pragma clang fp contract(off)
  const float gh = a.theta1 * gh_io + (1.f - a.theta1) * g;
  float dh = dh_io;
  if (a.hutch) dh = a.theta2 * dh + (1.f - a.theta2) * D;
  gh_io = gh;
  dh_io = dh;
  const float newton = -gh / dh;
  const float dx = (dh > 0.f && isfinite(dh) && isfinite(newton)) ? newton : (isfinite(eta) ? -sgnf(gh) * eta : 0.f);
  return fminf(fmaxf(dx, -eta), eta);
}

// The same for entry k of the state arrays, loading and storing in place
// (nontemporal: each entry is touched once per launch).
__device__ __forceinline__ float tr_update(float* __restrict__ ghat, float* __restrict__ dhat,
                                           const float* __restrict__ D, int64_t k, float g, float eta,
                                           const TrArgs& a) {
  float gh = __builtin_nontemporal_load(&ghat[k]), dh = __builtin_nontemporal_load(&dhat[k]);
  const float step = tr_row(g, gh, dh, a.hutch ? __builtin_nontemporal_load(&D[k]) : 0.f, eta, a);
  __builtin_nontemporal_store(gh, &ghat[k]);
  if (a.hutch) __builtin_nontemporal_store(dh, &dhat[k]);
  return step;
}

__host__ __device__ constexpr int degree_of_rows(int P) { return P == 14 ? 0 : (P == 23 ? 1 : (P == 38 ? 2 : 3)); }

}  // namespace gs3trust
