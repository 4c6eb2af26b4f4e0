// Projection of 3D Gaussians to screen-space splats, its tangent (JVP) and
// its gradient (VJP), for gfx950.
//
// Paper: Background, "Review of Gaussian Splatting" -- each Gaussian
// G(z) = alpha C exp(-1/2 (z-mu)^T Sigma^-1 (z-mu)) is projected to a 2D splat
// before alpha blending; Sigma is built from a scale and a rotation given by
// an unnormalised quaternion (appendix, "Bound on the rotation R"), and the
// colour is a view-dependent spherical-harmonic expansion of order 3.
// Sigma = R diag(s)^2 R^T (the form the rotation derivation composes with).
//
// One generic routine, templated on the scalar, serves three purposes:
//  * float: the forward pass.  This file is compiled with -ffp-contract=off
//    and correctly rounded division and square root, and the
//    key-determining expressions are written in a fixed evaluation order, so
//    depths, radii and tile rectangles are reproducible bit for bit by any
//    IEEE float32 evaluation of the same expressions;
//  * Dual (value, tangent): the Jacobian-vector product along a Rademacher
//    probe or a caller tangent;
//  * Dual with one-hot tangents: the backward pass, one forward-mode sweep
//    per geometric parameter (mean, log-scale, quaternion) -- exact and
//    cheap next to the blend, and it keeps a single source for the
//    projection's derivative.  Opacity and SH rows have closed forms.
#include "gs3_trust.h"

namespace {

struct Dual {
  float v, t;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.t + b.t}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.t - b.t}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.t}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.t * b.v + a.v * b.t}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  float q = a.v / b.v;
  return {q, (a.t - q * b.t) / b.v};
}
__device__ __forceinline__ Dual operator*(float a, Dual b) { return {a * b.v, a * b.t}; }
__device__ __forceinline__ Dual operator*(Dual a, float b) { return {a.v * b, a.t * b}; }
__device__ __forceinline__ Dual operator+(Dual a, float b) { return {a.v + b, a.t}; }
__device__ __forceinline__ Dual operator-(Dual a, float b) { return {a.v - b, a.t}; }
__device__ __forceinline__ Dual operator-(float a, Dual b) { return {a - b.v, -b.t}; }
__device__ __forceinline__ Dual operator/(float a, Dual b) {
  float q = a / b.v;
  return {q, -q * b.t / b.v};
}

__device__ __forceinline__ float val(float a) { return a; }
__device__ __forceinline__ float val(Dual a) { return a.v; }
__device__ __forceinline__ float sqrt_(float a) { return sqrtf(a); }
__device__ __forceinline__ Dual sqrt_(Dual a) {
  float s = sqrtf(a.v);
  return {s, s > 0.f ? 0.5f * a.t / s : 0.f};
}
// exp of a log-scale, evaluated in double and rounded once: reproducible in
// float32 by any correctly rounded double exp.
__device__ __forceinline__ float exp_ls(float a) { return (float)exp((double)a); }
__device__ __forceinline__ Dual exp_ls(Dual a) {
  float e = exp_ls(a.v);
  return {e, e * a.t};
}
__device__ __forceinline__ float sigmoid_(float a) { return 1.f / (1.f + expf(-a)); }
__device__ __forceinline__ Dual sigmoid_(Dual a) {
  float s = sigmoid_(a.v);
  return {s, a.t * s * (1.f - s)};
}
__device__ __forceinline__ float min_(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ float max_(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ Dual min_(Dual a, float b) { return a.v <= b ? a : Dual{b, 0.f}; }
__device__ __forceinline__ Dual max_(Dual a, float b) { return a.v >= b ? a : Dual{b, 0.f}; }

template <class T>
__device__ __forceinline__ T cst(float v);
template <>
__device__ __forceinline__ float cst<float>(float v) {
  return v;
}
template <>
__device__ __forceinline__ Dual cst<Dual>(float v) {
  return Dual{v, 0.f};
}

template <class T>
struct Proj {
  T u, v, ca, cb, cc;
  float depth, radius;
  bool ok;  // in front of the near plane and a positive-definite screen covariance
};

// s = exp(log-scale) with its tangent, from a value computed once per Gaussian.
__device__ __forceinline__ float scale_of(float, float sval) { return sval; }
__device__ __forceinline__ Dual scale_of(Dual ls, float sval) { return Dual{sval, sval * ls.t}; }

// Screen-space centre, conic, depth and radius of one Gaussian.  `src(r)`
// returns row r of the raw parameters (as float or Dual); sv[i] is
// exp_ls(log-scale i) evaluated once by the caller.
template <class T, class Src>
__device__ __forceinline__ void project_geo(const Src& src, const float sv[3], const CamDev& cam, Proj<T>& o) {
  const T mu0 = src(0), mu1 = src(1), mu2 = src(2);
  const T s0 = scale_of(src(3), sv[0]), s1 = scale_of(src(4), sv[1]), s2 = scale_of(src(5), sv[2]);
  const T qx = src(6), qy = src(7), qz = src(8), qw = src(9);
  const float two = 2.f;
  const T r2 = ((qx * qx + qy * qy) + qz * qz) + qw * qw;
  const T R00 = (((qw * qw + qx * qx) - qy * qy) - qz * qz) / r2;
  const T R01 = (two * (qx * qy - qw * qz)) / r2;
  const T R02 = (two * (qx * qz + qw * qy)) / r2;
  const T R10 = (two * (qx * qy + qw * qz)) / r2;
  const T R11 = (((qw * qw - qx * qx) + qy * qy) - qz * qz) / r2;
  const T R12 = (two * (qy * qz - qw * qx)) / r2;
  const T R20 = (two * (qx * qz - qw * qy)) / r2;
  const T R21 = (two * (qy * qz + qw * qx)) / r2;
  const T R22 = (((qw * qw - qx * qx) - qy * qy) + qz * qz) / r2;
  // M = R diag(s): Sigma = M M^T
  const T M00 = R00 * s0, M01 = R01 * s1, M02 = R02 * s2;
  const T M10 = R10 * s0, M11 = R11 * s1, M12 = R12 * s2;
  const T M20 = R20 * s0, M21 = R21 * s1, M22 = R22 * s2;
  const float* W = cam.W;
  const T p0 = ((W[0] * mu0 + W[1] * mu1) + W[2] * mu2) + cam.t[0];
  const T p1 = ((W[3] * mu0 + W[4] * mu1) + W[5] * mu2) + cam.t[1];
  const T p2 = ((W[6] * mu0 + W[7] * mu1) + W[8] * mu2) + cam.t[2];
  const T txtz = min_(max_(p0 / p2, -cam.limx), cam.limx);
  const T tytz = min_(max_(p1 / p2, -cam.limy), cam.limy);
  const T j00 = cam.fx / p2;
  const T j02 = -(cam.fx * txtz) / p2;
  const T j11 = cam.fy / p2;
  const T j12 = -(cam.fy * tytz) / p2;
  // T = J W (2x3), V = T M (2x3), screen covariance V V^T + dilation
  const T T00 = j00 * W[0] + j02 * W[6], T01 = j00 * W[1] + j02 * W[7], T02 = j00 * W[2] + j02 * W[8];
  const T T10 = j11 * W[3] + j12 * W[6], T11 = j11 * W[4] + j12 * W[7], T12 = j11 * W[5] + j12 * W[8];
  const T V00 = (T00 * M00 + T01 * M10) + T02 * M20;
  const T V01 = (T00 * M01 + T01 * M11) + T02 * M21;
  const T V02 = (T00 * M02 + T01 * M12) + T02 * M22;
  const T V10 = (T10 * M00 + T11 * M10) + T12 * M20;
  const T V11 = (T10 * M01 + T11 * M11) + T12 * M21;
  const T V12 = (T10 * M02 + T11 * M12) + T12 * M22;
  const T a = ((V00 * V00 + V01 * V01) + V02 * V02) + GS3_DILATION;
  const T b = (V00 * V10 + V01 * V11) + V02 * V12;
  const T c = ((V10 * V10 + V11 * V11) + V12 * V12) + GS3_DILATION;
  const T det = a * c - b * b;
  const float mid = 0.5f * (val(a) + val(c));
  const float lam = mid + sqrtf(fmaxf(mid * mid - val(det), 0.f));
  o.radius = ceilf(3.f * sqrtf(lam));
  o.u = (cam.fx * p0) / p2 + cam.cx;
  o.v = (cam.fy * p1) / p2 + cam.cy;
  o.ca = c / det;
  o.cb = -b / det;
  o.cc = a / det;
  o.depth = val(p2);
  o.ok = val(p2) > GS3_NEAR && val(det) > 0.f;
}

// Real spherical harmonics up to degree 3 (orthonormal on the sphere).
#define SH_C0 0.28209479177387814f
#define SH_C1 0.4886025119029199f
__constant__ float kSH2[5] = {1.0925484305920792f, -1.0925484305920792f, 0.31539156525252005f,
                              -1.0925484305920792f, 0.5462742152960396f};
__constant__ float kSH3[7] = {-0.5900435899266435f, 2.890611442640554f, -0.4570457994644658f,
                              0.3731763325901154f, -0.4570457994644658f, 1.445305721320277f,
                              -0.5900435899266435f};

template <class T, int DEG>
__device__ __forceinline__ void sh_basis(T x, T y, T z, T* Y) {
  Y[0] = cst<T>(SH_C0);
  if (DEG < 1) return;
  Y[1] = (-SH_C1) * y;
  Y[2] = SH_C1 * z;
  Y[3] = (-SH_C1) * x;
  if (DEG < 2) return;
  const T xx = x * x, yy = y * y, zz = z * z, xy = x * y, yz = y * z, xz = x * z;
  Y[4] = kSH2[0] * xy;
  Y[5] = kSH2[1] * yz;
  Y[6] = kSH2[2] * ((2.f * zz - xx) - yy);
  Y[7] = kSH2[3] * xz;
  Y[8] = kSH2[4] * (xx - yy);
  if (DEG < 3) return;
  Y[9] = kSH3[0] * y * (3.f * xx - yy);
  Y[10] = kSH3[1] * xy * z;
  Y[11] = kSH3[2] * y * ((4.f * zz - xx) - yy);
  Y[12] = kSH3[3] * z * ((2.f * zz - 3.f * xx) - 3.f * yy);
  Y[13] = kSH3[4] * x * ((4.f * zz - xx) - yy);
  Y[14] = kSH3[5] * z * (xx - yy);
  Y[15] = kSH3[6] * x * (xx - 3.f * yy);
}

// RGB = sum_k Y_k(dir) f_k + 0.5, clamped at 0; raw_pos[c] tells whether the
// clamp is inactive (its derivative is then 1).
template <class T, int DEG, class Src>
__device__ __forceinline__ void colour(const Src& src, const CamDev& cam, T rgb[3], bool raw_pos[3],
                                       float* Yout = nullptr) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const T dx = src(0) - cam.campos[0], dy = src(1) - cam.campos[1], dz = src(2) - cam.campos[2];
  const T inv = cst<T>(1.f) / sqrt_((dx * dx + dy * dy) + dz * dz);
  T Y[K];
  sh_basis<T, DEG>(dx * inv, dy * inv, dz * inv, Y);
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    T acc = cst<T>(0.5f);
#pragma unroll
    for (int k = 0; k < K; ++k) acc = acc + Y[k] * src(11 + 3 * k + ch);
    raw_pos[ch] = val(acc) >= 0.f;
    rgb[ch] = max_(acc, 0.f);
  }
  if (Yout) {
#pragma unroll
    for (int k = 0; k < K; ++k) Yout[k] = val(Y[k]);
  }
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t v) {
  uint64_t z = v + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// Rademacher entry k of probe i: +1 when the top bit of the hash is clear.
__device__ __forceinline__ float probe_sign(uint64_t inner, uint64_t k) {
  return (splitmix64(inner ^ k) >> 63) ? -1.f : 1.f;
}

// Opacity and skip threshold, each evaluated in double and rounded once so
// that any float32 reproduction of the skip decision agrees bit for bit.
__device__ __forceinline__ float opacity_of(float logit) { return (float)(1.0 / (1.0 + exp(-(double)logit))); }
__device__ __forceinline__ float skip_threshold(float op) { return (float)(-log(255.0 * (double)op)); }

template <int DEG>
__global__ __launch_bounds__(256) void k_project_fwd(const float* __restrict__ x, int64_t n, CamDev cam,
                                                      Rec* __restrict__ rec, uint2* __restrict__ rect,
                                                      uint32_t* __restrict__ depth_key,
                                                      uint32_t* __restrict__ tiles) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  auto src = [&](int r) { return x[(int64_t)r * n + g]; };
  const float sv[3] = {exp_ls(src(3)), exp_ls(src(4)), exp_ls(src(5))};
  Proj<float> p;
  project_geo<float>(src, sv, cam, p);
  const float inv = 0.0625f;
  const float txf = (float)cam.tiles_x, tyf = (float)cam.tiles_y;
  const float x0 = fminf(fmaxf(floorf((p.u - p.radius) * inv), 0.f), txf);
  const float x1 = fminf(fmaxf(floorf((p.u + p.radius) * inv) + 1.f, 0.f), txf);
  const float y0 = fminf(fmaxf(floorf((p.v - p.radius) * inv), 0.f), tyf);
  const float y1 = fminf(fmaxf(floorf((p.v + p.radius) * inv) + 1.f, 0.f), tyf);
  bool vis = p.ok && isfinite(p.u) && isfinite(p.v) && isfinite(p.radius);
  const int ix0 = vis ? (int)x0 : 0, ix1 = vis ? (int)x1 : 0, iy0 = vis ? (int)y0 : 0, iy1 = vis ? (int)y1 : 0;
  const int touched = max(ix1 - ix0, 0) * max(iy1 - iy0, 0);
  vis = vis && touched > 0;
  if (!vis) {
    depth_key[g] = 0xffffffffu;
    tiles[g] = 0u;
    return;
  }
  float rgb[3];
  bool pos[3];
  colour<float, DEG>(src, cam, rgb, pos);
  const float op = opacity_of(src(10));
  Rec r;
  r.a = make_float4(p.u, p.v, -0.5f * p.ca, -p.cb);
  r.b = make_float4(-0.5f * p.cc, op, rgb[0], rgb[1]);
  // spare word: which colour channels are unclamped (bit c), for the backward
  const uint32_t posm = (pos[0] ? 1u : 0u) | (pos[1] ? 2u : 0u) | (pos[2] ? 4u : 0u);
  r.c = make_float4(rgb[2], skip_threshold(op), 0.f, __uint_as_float(posm));
  rec[g] = r;
  rect[g] = make_uint2((uint32_t)ix0 | ((uint32_t)iy0 << 16), (uint32_t)ix1 | ((uint32_t)iy1 << 16));
  depth_key[g] = __float_as_uint(p.depth);
  tiles[g] = (uint32_t)touched;
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project_jvp(const float* __restrict__ x, int64_t n, CamDev cam,
                                                      const Rec* __restrict__ rec, const uint32_t* __restrict__ tiles,
                                                      int kind, uint64_t inner, const float* __restrict__ tangent,
                                                      TRec* __restrict__ trec) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  if (tiles[g] == 0u) return;
  auto src = [&](int r) {
    const int64_t k = (int64_t)r * n + g;
    float t = kind == PROBE_HASH ? probe_sign(inner, (uint64_t)k) : tangent[k];
    return Dual{x[k], t};
  };
  const float sv[3] = {exp_ls(x[3 * n + g]), exp_ls(x[4 * n + g]), exp_ls(x[5 * n + g])};
  Proj<Dual> p;
  project_geo<Dual>(src, sv, cam, p);
  Dual rgb[3];
  bool pos[3];
  colour<Dual, DEG>(src, cam, rgb, pos);
  const Dual op = sigmoid_(src(10));
  TRec t;
  t.a = make_float4(p.u.t, p.v.t, p.ca.t, p.cb.t);
  t.b = make_float4(p.cc.t, op.t, rgb[0].t, rgb[1].t);
  t.c = make_float4(rgb[2].t, 0.f, 0.f, 0.f);
  trec[g] = t;
}

// Sum of each Gaussian's per-(Gaussian, tile) partials, which sit in the
// contiguous slots [offsets[i], offsets[i] + counts[i]) of the Gaussian of
// depth rank i (order[i]): G[k][order[i]], k < 9, summed in slot order.  A
// workgroup takes 28 consecutive depth ranks, whose slots form one contiguous
// run; the run is streamed through LDS in chunks with coalesced loads, and
// thread (j, k) adds component k of rank j's slots in order.  Invisible
// Gaussians (count 0) get zeros.
constexpr int kSumRanks = 28;      // 28 x 9 = 252 of the 256 threads
constexpr int kSumChunk = 4096;    // floats per LDS chunk

__global__ __launch_bounds__(256) void k_sum_pair_partials(const uint32_t* __restrict__ order,
                                                            const uint32_t* __restrict__ offsets,
                                                            const uint32_t* __restrict__ counts,
                                                            const float* __restrict__ partials, int64_t n,
                                                            float* __restrict__ G) {
  __shared__ float buf[kSumChunk];
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * kSumRanks;
  const int64_t i1 = i0 + kSumRanks < n ? i0 + kSumRanks : n;
  const int j = tid / 9, k = tid % 9;
  const int64_t i = i0 + j;
  const bool mine = tid < 9 * kSumRanks && i < i1;
  const int64_t lo = (int64_t)offsets[i0] * 9;
  const int64_t hi = ((int64_t)offsets[i1 - 1] + counts[i1 - 1]) * 9;
  int64_t first = 0, last = 0;  // my float indices: first, first + 9, ..., < last
  if (mine) {
    first = (int64_t)offsets[i] * 9 + k;
    last = ((int64_t)offsets[i] + counts[i]) * 9;
  }
  float acc = 0.f;
  for (int64_t base = lo; base < hi; base += kSumChunk) {
    const int64_t end = base + kSumChunk < hi ? base + kSumChunk : hi;
    for (int64_t f = base + tid; f < end; f += 256) buf[f - base] = partials[f];
    __syncthreads();
    for (; first < last && first < end; first += 9) acc += buf[first - base];
    __syncthreads();
  }
  if (mine) G[(int64_t)k * n + order[i]] = acc;
}

// Trust-region radius of every Gaussian from the parameters before the
// update, for the fused update: rad[c][g] for the 15 components of
// gs3trust::Radius (mu 0-2, log-scale 3, quaternion 4-7, logit 8, colour
// 9-11, view-dependent SH 12-14).
template <int DEG>
__global__ __launch_bounds__(256) void k_trust_radius(const float* __restrict__ x, int64_t n, float eps,
                                                       uint32_t variant, float* __restrict__ rad) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const gs3trust::Radius r = gs3trust::trust_radius(x, n, g, eps, variant, DEG);
  const float v[15] = {r.mu[0], r.mu[1], r.mu[2], r.ls, r.q[0], r.q[1], r.q[2], r.q[3],
                       r.logit, r.col[0], r.col[1], r.col[2], r.rest[0], r.rest[1], r.rest[2]};
#pragma unroll
  for (int c = 0; c < 15; ++c) rad[(int64_t)c * n + g] = v[c];
}

__device__ __forceinline__ int radius_component(int row) {
  if (row < 3) return row;
  if (row < 6) return 3;
  if (row < 10) return row - 2;
  if (row == 10) return 8;
  if (row < 14) return row - 2;
  return 12 + (row - 11) % 3;
}

// SH coefficients per role of the projection backward
constexpr int kShPerRole = 4;
template <int DEG>
constexpr int bwd_roles() {
  return 11 + ((DEG + 1) * (DEG + 1) + kShPerRole - 1) / kShPerRole;
}

// Chain rule from the summed screen-space partials G (d/du, d/dv, d/dconic
// a, b, c, d/dalpha, d/drgb) to the raw parameters.  blockIdx.y picks the
// work of a thread: 0..9 one forward-mode sweep along geometric row y (mean,
// log-scale, quaternion; the mean rows also move the SH view direction), 10
// the opacity logit, 11.. four SH coefficients each, d rgb_c / d f_kc =
// Y_k(dir) where the colour clamp is inactive.  One thread per (Gaussian,
// role) keeps many more waves in flight than one thread per Gaussian walking
// every row.
template <int DEG>
__global__ __launch_bounds__(256) void k_project_bwd(const float* __restrict__ x, int64_t n, CamDev cam,
                                                      const Rec* __restrict__ rec, const uint32_t* __restrict__ tiles,
                                                      const float* __restrict__ G, int mode, int accumulate,
                                                      uint64_t inner, float scale, float* __restrict__ out,
                                                      FusedTr ft) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int role = blockIdx.y;
  // this role's rows: [r0, r1)
  const int r0 = role <= 10 ? role : 11 + 3 * kShPerRole * (role - 11);
  const int r1 = role <= 10 ? role + 1 : min(11 + 3 * K, r0 + 3 * kShPerRole);
  auto emit = [&](int r, float v) {
    const int64_t k = (int64_t)r * n + g;
    if (mode == 0) {
      out[k] = accumulate ? out[k] + v : v;
    } else if (mode == 1) {
      out[k] += scale * probe_sign(inner, (uint64_t)k) * v;
    } else {
      // the update of Algorithm 1; x is only read, the update goes to x_out
      const float gk = ft.gacc ? ft.gacc[k] + v : v;
      const float eta = ft.rad[(int64_t)radius_component(r) * n + g];
      ft.x_out[k] = x[k] + gs3trust::tr_update(ft.ghat, ft.dhat, ft.D, k, gk, eta, ft.a);
    }
  };
  if (tiles[g] == 0u) {  // no gradient from this view
    if (mode == 2 || (mode == 0 && !accumulate))
      for (int r = r0; r < r1; ++r) emit(r, 0.f);
    return;
  }
  auto Gk = [&](int k) { return G[(int64_t)k * n + g]; };
  if (role < 10) {
    const float sv[3] = {exp_ls(x[3 * n + g]), exp_ls(x[4 * n + g]), exp_ls(x[5 * n + g])};
    auto src = [&](int r) { return Dual{x[(int64_t)r * n + g], r == role ? 1.f : 0.f}; };
    Proj<Dual> p;
    project_geo<Dual>(src, sv, cam, p);
    float d = Gk(0) * p.u.t + Gk(1) * p.v.t + Gk(2) * p.ca.t + Gk(3) * p.cb.t + Gk(4) * p.cc.t;
    if (role < 3) {
      Dual rgb[3];
      bool pos[3];
      colour<Dual, DEG>(src, cam, rgb, pos);
      d += Gk(6) * rgb[0].t + Gk(7) * rgb[1].t + Gk(8) * rgb[2].t;
    }
    emit(role, d);
    return;
  }
  if (role == 10) {
    const float s = sigmoid_(x[10 * n + g]);
    emit(10, Gk(5) * s * (1.f - s));
    return;
  }
  // the SH basis at the view direction (same expressions as the forward's
  // colour) and the forward's clamp mask: no SH coefficient is read
  float Y[K];
  {
    const float dx = x[g] - cam.campos[0], dy = x[n + g] - cam.campos[1], dz = x[2 * n + g] - cam.campos[2];
    const float inv = 1.f / sqrtf((dx * dx + dy * dy) + dz * dz);
    sh_basis<float, DEG>(dx * inv, dy * inv, dz * inv, Y);
  }
  const uint32_t posm = __float_as_uint(rec[g].c.w);
  const bool pos[3] = {(posm & 1u) != 0u, (posm & 2u) != 0u, (posm & 4u) != 0u};
  const float G6 = Gk(6), G7 = Gk(7), G8 = Gk(8);
  const int k0 = kShPerRole * (role - 11);
#pragma unroll
  for (int kk = 0; kk < kShPerRole; ++kk) {
    const int k = k0 + kk;
    if (k >= K) break;
    emit(11 + 3 * k, pos[0] ? Y[k] * G6 : 0.f);
    emit(12 + 3 * k, pos[1] ? Y[k] * G7 : 0.f);
    emit(13 + 3 * k, pos[2] ? Y[k] * G8 : 0.f);
  }
}

uint64_t probe_inner(uint64_t seed, uint32_t i) {
  uint64_t z = (seed ^ (uint64_t)i) + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

#define GS3_DEG_DISPATCH(deg, KERNEL, ...)                                                        \
  switch (deg) {                                                                                  \
    case 0: hipLaunchKernelGGL(KERNEL<0>, __VA_ARGS__); break;                                    \
    case 1: hipLaunchKernelGGL(KERNEL<1>, __VA_ARGS__); break;                                    \
    case 2: hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__); break;                                    \
    default: hipLaunchKernelGGL(KERNEL<3>, __VA_ARGS__); break;                                   \
  }

void launch_project_fwd(const float* x, int64_t n, int deg, const CamDev& cam, Rec* rec, uint2* rect,
                        uint32_t* depth_key, uint32_t* tiles, hipStream_t st) {
  GS3_DEG_DISPATCH(deg, k_project_fwd, dim3(blocks_for(n, 256)), dim3(256), 0, st, x, n, cam, rec, rect, depth_key,
                   tiles);
}

void launch_project_jvp(const float* x, int64_t n, int deg, const CamDev& cam, const Rec* rec,
                        const uint32_t* tiles, int probe_kind, uint64_t seed, uint32_t probe_index,
                        const float* tangent, TRec* trec, hipStream_t st) {
  GS3_DEG_DISPATCH(deg, k_project_jvp, dim3(blocks_for(n, 256)), dim3(256), 0, st, x, n, cam, rec, tiles, probe_kind,
                   probe_inner(seed, probe_index), tangent, trec);
}

void launch_project_bwd(const float* x, int64_t n, int deg, const CamDev& cam, const Rec* rec, const uint32_t* order,
                        const uint32_t* offsets, const uint32_t* counts, const uint32_t* tiles,
                        const float* partials, float* gsum, int mode, int accumulate, uint64_t seed,
                        uint32_t probe_index, float scale, float* out, const FusedTr& ft, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_pair_partials, dim3(blocks_for(n, kSumRanks)), dim3(256), 0, st, order, offsets, counts,
                     partials, n, gsum);
  if (mode == 2)
    GS3_DEG_DISPATCH(deg, k_trust_radius, dim3(blocks_for(n, 256)), dim3(256), 0, st, x, n, ft.a.epsilon,
                     ft.a.variant, ft.rad);
  const unsigned roles = deg == 0 ? bwd_roles<0>() : (deg == 1 ? bwd_roles<1>() : (deg == 2 ? bwd_roles<2>()
                                                                                            : bwd_roles<3>()));
  GS3_DEG_DISPATCH(deg, k_project_bwd, dim3(blocks_for(n, 256), roles), dim3(256), 0, st, x, n, cam, rec, tiles,
                   gsum, mode, accumulate, probe_inner(seed, probe_index), scale, out, ft);
}
