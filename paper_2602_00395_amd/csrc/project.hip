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
//    probe or a caller tangent.
// The backward pass is the same chain written out in reverse (adjoint) mode,
// one pass per Gaussian for the mean, log-scale, quaternion and opacity rows
// (the view direction of the SH colour included); SH rows have closed forms.
#include <type_traits>

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

// A workgroup takes 256 consecutive Gaussians.  First each thread projects
// one of them (screen centre, conic, depth, tile rectangle) and the
// Gaussians whose rectangle is not empty are listed in LDS with what the
// rest needs; the others are culled at once.  Then thread j takes listed
// Gaussian j: opacity and skip threshold and the exact tile count of its
// tile list (a splat that reaches no tile is culled), and for a visible
// splat its record, tile rectangle, depth key and tile count.  Last the
// colour: one thread per (channel, listed visible splat), each loading its
// 16 SH coefficients before the sum, and the clamp bits.  The per-splat work
// thus runs on dense lists (with a Gaussian per thread throughout, most
// lanes idled behind the few visible splats of a wave: at city scale most
// Gaussians are outside the view), and an invisible Gaussian's SH rows are
// never read.  vis_count receives the visible count of every 64 consecutive
// Gaussians.
constexpr int kFwdGauss = 256;

template <int DEG>
__global__ __launch_bounds__(256) void k_project_fwd(const float* __restrict__ x, int64_t n, CamDev cam,
                                                      Rec* __restrict__ rec, uint2* __restrict__ rect,
                                                      uint32_t* __restrict__ depth_key,
                                                      uint32_t* __restrict__ tiles,
                                                      uint32_t* __restrict__ vis_count) {
  // the listed Gaussians (structure of arrays)
  __shared__ float l_u[kFwdGauss], l_v[kFwdGauss], l_qa[kFwdGauss], l_qb[kFwdGauss], l_qc[kFwdGauss];
  __shared__ float l_depth[kFwdGauss], l_dir[3][kFwdGauss];
  __shared__ uint32_t l_lo[kFwdGauss], l_hi[kFwdGauss], l_off[kFwdGauss];
  __shared__ uint32_t l_clamp[kFwdGauss];  // bit c: channel c unclamped; bit 3: the splat is visible
  __shared__ uint32_t listed;
  __shared__ uint32_t vis_bits[kFwdGauss / 32];  // bit o: Gaussian g0 + o is visible
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t g0 = (int64_t)blockIdx.x * kFwdGauss;
  if (tid == 0) listed = 0u;
  if (tid < kFwdGauss / 32) vis_bits[tid] = 0u;
  __syncthreads();
  {
    const int64_t g = g0 + tid;
    auto src = [&](int r) { return x[(int64_t)r * n + g]; };
    bool cand = false;
    Proj<float> p;
    int ix0 = 0, ix1 = 0, iy0 = 0, iy1 = 0;
    if (g < n) {
      const float sv[3] = {exp_ls(src(3)), exp_ls(src(4)), exp_ls(src(5))};
      project_geo<float>(src, sv, cam, p);
      const float inv = 0.0625f;
      const float txf = (float)cam.tiles_x, tyf = (float)cam.tiles_y;
      const float x0 = fminf(fmaxf(floorf((p.u - p.radius) * inv), 0.f), txf);
      const float x1 = fminf(fmaxf(floorf((p.u + p.radius) * inv) + 1.f, 0.f), txf);
      const float y0 = fminf(fmaxf(floorf((p.v - p.radius) * inv), 0.f), tyf);
      const float y1 = fminf(fmaxf(floorf((p.v + p.radius) * inv) + 1.f, 0.f), tyf);
      cand = p.ok && isfinite(p.u) && isfinite(p.v) && isfinite(p.radius);
      if (cand) {
        ix0 = (int)x0;
        ix1 = (int)x1;
        iy0 = (int)y0;
        iy1 = (int)y1;
      }
      cand = cand && ix1 > ix0 && iy1 > iy0;
    }
    const uint64_t b = __ballot(cand);
    uint32_t base = 0u;
    if (lane == 0 && b) base = atomicAdd(&listed, (uint32_t)__popcll(b));
    base = __shfl(base, 0, 64);
    if (cand) {
      const int j = (int)base + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
      l_u[j] = p.u;
      l_v[j] = p.v;
      l_qa[j] = -0.5f * p.ca;
      l_qb[j] = -p.cb;
      l_qc[j] = -0.5f * p.cc;
      l_depth[j] = p.depth;
      // view direction for the colour
      const float dx = src(0) - cam.campos[0], dy = src(1) - cam.campos[1], dz = src(2) - cam.campos[2];
      const float inv = 1.f / sqrtf((dx * dx + dy * dy) + dz * dz);
      l_dir[0][j] = dx * inv;
      l_dir[1][j] = dy * inv;
      l_dir[2][j] = dz * inv;
      l_lo[j] = (uint32_t)ix0 | ((uint32_t)iy0 << 16);
      l_hi[j] = (uint32_t)ix1 | ((uint32_t)iy1 << 16);
      l_off[j] = (uint32_t)tid;
    } else if (g < n) {
      depth_key[g] = 0xffffffffu;
      tiles[g] = 0u;
    }
  }
  __syncthreads();
  const int m = (int)listed;
  if (tid < m) {
    const int j = tid, o = (int)l_off[j];
    const int64_t g = g0 + o;
    const float u = l_u[j], v = l_v[j], qa = l_qa[j], qb = l_qb[j], qc = l_qc[j];
    const uint32_t lo = l_lo[j], hi = l_hi[j];
    const float op = opacity_of(x[10 * n + g]);
    const float tau = skip_threshold(op);
    // the rectangle's tiles the splat can reach (the tile list, see
    // SplatRows); the stored rectangle is the bounding box of the listed
    // tiles, so the emission and the backward walk no rows without tiles
    int bx0, by0, bx1, by1;
    const uint32_t touched = splat_tile_bounds(
        splat_rows(u, v, qa, qb, qc, tau, (int)(lo & 0xffffu), (int)(lo >> 16), (int)(hi & 0xffffu), (int)(hi >> 16)),
        bx0, by0, bx1, by1);
    l_clamp[j] = touched ? 8u : 0u;
    if (touched == 0u) {
      depth_key[g] = 0xffffffffu;
      tiles[g] = 0u;
    } else {
      float* rw = reinterpret_cast<float*>(rec + g);
      *reinterpret_cast<float4*>(rw) = make_float4(u, v, qa, qb);
      rw[4] = qc;
      rw[5] = op;
      rw[9] = tau;
      rw[10] = 0.f;  // filled later (the splat's first pair)
      rect[g] = make_uint2((uint32_t)bx0 | ((uint32_t)by0 << 16), (uint32_t)bx1 | ((uint32_t)by1 << 16));
      depth_key[g] = __float_as_uint(l_depth[j]);
      tiles[g] = touched;
      atomicOr(&vis_bits[o >> 5], 1u << (o & 31));
    }
  }
  __syncthreads();
  // colour channel c of listed splat j, for the visible ones:
  // RGB_c = sum_k Y_k(dir) f_kc + 0.5, clamped at 0 (as colour<>)
  for (int i = tid; i < 3 * m; i += 256) {
    const int c = i / m, j = i - c * m;
    if (!(l_clamp[j] & 8u)) continue;
    const int64_t g = g0 + l_off[j];
    constexpr int K = (DEG + 1) * (DEG + 1);
    float f[K];
#pragma unroll
    for (int k = 0; k < K; ++k) f[k] = x[(int64_t)(11 + 3 * k + c) * n + g];
    float Y[K];
    sh_basis<float, DEG>(l_dir[0][j], l_dir[1][j], l_dir[2][j], Y);
    float acc = 0.5f;
#pragma unroll
    for (int k = 0; k < K; ++k) acc = acc + Y[k] * f[k];
    reinterpret_cast<float*>(rec + g)[6 + c] = fmaxf(acc, 0.f);
    if (acc >= 0.f) atomicOr(&l_clamp[j], 1u << c);
  }
  __syncthreads();
  // spare word: which colour channels are unclamped (bit c), for the backward
  if (tid < m && (l_clamp[tid] & 8u)) reinterpret_cast<float*>(rec + g0 + l_off[tid])[11] = __uint_as_float(l_clamp[tid] & 7u);
  const int64_t q = (int64_t)blockIdx.x * (kFwdGauss / 64) + w;  // this wave's 64 Gaussians
  if (lane == 0 && q * 64 < n) vis_count[q] = (uint32_t)(__popc(vis_bits[2 * w]) + __popc(vis_bits[2 * w + 1]));
}

// Tangent records of the visible Gaussians (tiles != 0).  A workgroup takes
// kJvpChunk consecutive Gaussians, lists its visible ones in LDS (order
// within the list is immaterial: each Gaussian's record is computed on its
// own), and its threads walk the list, so a wave's lanes all carry visible
// Gaussians (one thread per Gaussian left most lanes idle: 13% lane use at
// the city scale).
constexpr int kJvpChunk = 1024;

template <int DEG>
__global__ __launch_bounds__(256) void k_project_jvp(const float* __restrict__ x, int64_t n, CamDev cam,
                                                      const uint32_t* __restrict__ tiles, int kind, uint64_t inner,
                                                      const float* __restrict__ tangent, TRec* __restrict__ trec) {
  __shared__ uint32_t list[kJvpChunk];
  __shared__ uint32_t listed;
  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t g0 = (int64_t)blockIdx.x * kJvpChunk;
  if (tid == 0) listed = 0u;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kJvpChunk / 256; ++j) {
    const int o = j * 256 + tid;
    const bool vis = g0 + o < n && tiles[g0 + o] != 0u;
    const uint64_t b = __ballot(vis);
    uint32_t base = 0u;
    if (lane == 0 && b) base = atomicAdd(&listed, (uint32_t)__popcll(b));
    base = __shfl(base, 0, 64);
    if (vis) list[base + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u))] = o;
  }
  __syncthreads();
  const int m = (int)listed;
  for (int i = tid; i < m; i += 256) {
    const int64_t g = g0 + list[i];
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
}

// Sum of each Gaussian's per-(Gaussian, tile) partials, which sit in the
// contiguous slots [offsets[i], offsets[i] + counts[i]) of the Gaussian of
// depth rank i (order[i]): G[order[i]][k], k < 9.  A workgroup takes 28
// consecutive depth ranks.  Thread (j, k) sums component k of rank j when
// the rank has at most kSumLong slots, in rounds of 16 loads issued together,
// with four interleaved partial sums
// (slot t goes to sum t mod 4 in slot order, combined as (s0 + s1) +
// (s2 + s3)); a rank
// with more slots (a splat covering many tiles, which would hold its wave
// for hundreds of serial steps) is summed by the whole workgroup: thread t
// takes slots t, t + 256, ... and the 256 partial sums are combined in a
// fixed tree.  Every order is fixed, so the result is deterministic.
// Invisible Gaussians (count 0) sort last and get nothing: their rows of G
// are never read (the chain rule skips them), so a workgroup whose first
// rank is invisible returns at once.
constexpr int kSumRanks = 28;  // 28 x 9 = 252 of the 256 threads
constexpr uint32_t kSumLong = 48;

__device__ __forceinline__ float wave_sum_xor(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__global__ __launch_bounds__(256) void k_sum_pair_partials(const uint32_t* __restrict__ order,
                                                            const uint32_t* __restrict__ offsets,
                                                            const uint32_t* __restrict__ counts,
                                                            const float* __restrict__ partials,
                                                            const uint32_t* __restrict__ valid, int64_t n,
                                                            const uint32_t* __restrict__ n_dev,
                                                            float* __restrict__ G) {
  // slot j holds partials where its valid bit is set, else it counts as zero
  auto set = [&](uint64_t j) { return (valid[j >> 5] >> (j & 31)) & 1u; };
  __shared__ float wsum[4][9];
  __shared__ uint32_t long_ranks;  // bit j: rank i0 + j is summed by the workgroup
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * kSumRanks;
  const int nr = (int)(i0 + kSumRanks < n ? kSumRanks : n - i0);
  if (n_dev) n = *n_dev;  // the visible ranks, when the count is on the device
  if (i0 >= n || counts[i0] == 0u) return;  // this rank and every later one is invisible
  const int j = tid / 9, k = tid % 9;
  if (tid == 0) long_ranks = 0u;
  __syncthreads();
  if (tid < 9 * kSumRanks && j < nr) {
    const int64_t i = i0 + j;
    const uint32_t c = counts[i];
    if (c == 0u) {
      // invisible: nothing to sum
    } else if (c <= kSumLong) {
      const uint64_t o = offsets[i];
      const float* p = partials + (int64_t)o * 9 + k;
      float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
      // rounds of 16 slots, all loads of a round issued before any is added
      // (one round for nine Gaussians in ten).  A round's slot loads and
      // its one or two valid-bit words are issued together: a slot without
      // partials is read (its contents are stale) and replaced by an exact
      // zero, so no load waits on a valid bit; slots past c read nothing.
      for (uint32_t t = 0; t < c; t += 16) {
        const uint64_t s = o + t;
        const uint32_t last = (uint32_t)((s + (c - t < 16u ? c - t : 16u) - 1u) >> 5);
        const uint64_t w0 = valid[s >> 5];
        const uint64_t w1 = last != (uint32_t)(s >> 5) ? valid[last] : 0u;
        const uint64_t bits = (w0 | (w1 << 32)) >> (s & 31);
        float v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = t + q < c ? p[9 * (t + q)] : 0.f;
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = (bits >> q) & 1u ? v[q] : 0.f;
#pragma unroll
        for (int q = 0; q < 16; q += 4) {
          s0 += v[q];
          s1 += v[q + 1];
          s2 += v[q + 2];
          s3 += v[q + 3];
        }
      }
      G[(int64_t)order[i] * 9 + k] = (s0 + s1) + (s2 + s3);
    } else if (k == 0) {
      atomicOr(&long_ranks, 1u << j);
    }
  }
  __syncthreads();
  // long ranks, one at a time, by the whole workgroup
  for (uint32_t m = long_ranks; m != 0u; m &= m - 1u) {
    const int64_t i = i0 + __builtin_ctz(m);
    const uint32_t c = counts[i];
    const uint64_t o = offsets[i];
    const float* p = partials + (int64_t)o * 9;
    float acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = 0.f;
    for (uint32_t t = tid; t < c; t += 256) {
      if (!set(o + t)) continue;
#pragma unroll
      for (int q = 0; q < 9; ++q) acc[q] += p[(int64_t)t * 9 + q];
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = wave_sum_xor(acc[q]);
    if ((tid & 63) == 0) {
#pragma unroll
      for (int q = 0; q < 9; ++q) wsum[tid >> 6][q] = acc[q];
    }
    __syncthreads();
    if (tid < 9) G[(int64_t)order[i] * 9 + tid] = ((wsum[0][tid] + wsum[1][tid]) + wsum[2][tid]) + wsum[3][tid];
    __syncthreads();
  }
}

// Reverse-mode derivative of project_geo: from the summed screen-space
// partials G[0..4] (d/du, d/dv, d/dconic a, b, c) to the mean (3),
// log-scale (3) and quaternion (4) rows, out[0..9].  Every intermediate is
// recomputed in float32 as in the forward; the adjoints are the transposed
// local derivatives of each step (conic = inverse of the screen covariance,
// V = T M, T = J W with the clamped Jacobian, M = R diag(s), R = Rn(q) /
// |q|^2, p = W mu + t), so the result is the Jacobian a forward-mode sweep
// per row would give, up to float32 rounding.
__device__ __forceinline__ void geo_vjp(const float* __restrict__ x, int64_t n, int64_t g, const CamDev& cam,
                                        const float G[5], float out[10]) {
  auto xr = [&](int r) { return x[(int64_t)r * n + g]; };
  const float mu[3] = {xr(0), xr(1), xr(2)};
  const float sv[3] = {exp_ls(xr(3)), exp_ls(xr(4)), exp_ls(xr(5))};
  const float qx = xr(6), qy = xr(7), qz = xr(8), qw = xr(9);
  // ---- forward recomputation
  const float r2 = ((qx * qx + qy * qy) + qz * qz) + qw * qw;
  const float ir2 = 1.f / r2;
  float Rn[3][3];
  Rn[0][0] = ((qw * qw + qx * qx) - qy * qy) - qz * qz;
  Rn[0][1] = 2.f * (qx * qy - qw * qz);
  Rn[0][2] = 2.f * (qx * qz + qw * qy);
  Rn[1][0] = 2.f * (qx * qy + qw * qz);
  Rn[1][1] = ((qw * qw - qx * qx) + qy * qy) - qz * qz;
  Rn[1][2] = 2.f * (qy * qz - qw * qx);
  Rn[2][0] = 2.f * (qx * qz - qw * qy);
  Rn[2][1] = 2.f * (qy * qz + qw * qx);
  Rn[2][2] = ((qw * qw - qx * qx) - qy * qy) + qz * qz;
  float R[3][3], M[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      R[i][j] = Rn[i][j] * ir2;
      M[i][j] = R[i][j] * sv[j];
    }
  const float* W = cam.W;
  float p[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) p[i] = ((W[3 * i] * mu[0] + W[3 * i + 1] * mu[1]) + W[3 * i + 2] * mu[2]) + cam.t[i];
  const float ip2 = 1.f / p[2];
  const float rx = p[0] * ip2, ry = p[1] * ip2;
  const bool inx = rx >= -cam.limx && rx <= cam.limx, iny = ry >= -cam.limy && ry <= cam.limy;
  const float txtz = fminf(fmaxf(rx, -cam.limx), cam.limx), tytz = fminf(fmaxf(ry, -cam.limy), cam.limy);
  const float j00 = cam.fx * ip2, j02 = -(cam.fx * txtz) * ip2;
  const float j11 = cam.fy * ip2, j12 = -(cam.fy * tytz) * ip2;
  float Tm[2][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    Tm[0][k] = j00 * W[k] + j02 * W[6 + k];
    Tm[1][k] = j11 * W[3 + k] + j12 * W[6 + k];
  }
  float V[2][3];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) V[i][j] = (Tm[i][0] * M[0][j] + Tm[i][1] * M[1][j]) + Tm[i][2] * M[2][j];
  const float a = ((V[0][0] * V[0][0] + V[0][1] * V[0][1]) + V[0][2] * V[0][2]) + GS3_DILATION;
  const float b = (V[0][0] * V[1][0] + V[0][1] * V[1][1]) + V[0][2] * V[1][2];
  const float c = ((V[1][0] * V[1][0] + V[1][1] * V[1][1]) + V[1][2] * V[1][2]) + GS3_DILATION;
  const float idet = 1.f / (a * c - b * b);
  // ---- adjoints: conic (c, -b, a) / det
  const float ca = c * idet, cb = -b * idet, cc = a * idet;
  const float gdet = -((G[2] * ca + G[3] * cb) + G[4] * cc) * idet;
  const float ga = G[4] * idet + gdet * c;
  const float gcv = G[2] * idet + gdet * a;
  const float gb = -G[3] * idet - 2.f * gdet * b;
  float gV[2][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    gV[0][k] = 2.f * ga * V[0][k] + gb * V[1][k];
    gV[1][k] = gb * V[0][k] + 2.f * gcv * V[1][k];
  }
  // V = Tm M
  float gT[2][3], gM[3][3];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) gT[i][k] = (gV[i][0] * M[k][0] + gV[i][1] * M[k][1]) + gV[i][2] * M[k][2];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < 3; ++j) gM[k][j] = Tm[0][k] * gV[0][j] + Tm[1][k] * gV[1][j];
  // Tm = J W
  const float gj00 = (gT[0][0] * W[0] + gT[0][1] * W[1]) + gT[0][2] * W[2];
  const float gj02 = (gT[0][0] * W[6] + gT[0][1] * W[7]) + gT[0][2] * W[8];
  const float gj11 = (gT[1][0] * W[3] + gT[1][1] * W[4]) + gT[1][2] * W[5];
  const float gj12 = (gT[1][0] * W[6] + gT[1][1] * W[7]) + gT[1][2] * W[8];
  // J entries and the screen centre as functions of p
  float gp0 = G[0] * cam.fx * ip2, gp1 = G[1] * cam.fy * ip2;
  float gp2 = -((G[0] * cam.fx) * p[0] + (G[1] * cam.fy) * p[1]) * ip2 * ip2;
  gp2 -= (((gj00 * j00 + gj02 * j02) + gj11 * j11) + gj12 * j12) * ip2;
  const float gtx = -gj02 * cam.fx * ip2, gty = -gj12 * cam.fy * ip2;
  if (inx) {
    gp0 += gtx * ip2;
    gp2 -= gtx * rx * ip2;
  }
  if (iny) {
    gp1 += gty * ip2;
    gp2 -= gty * ry * ip2;
  }
  float gmu[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) gmu[k] = (W[k] * gp0 + W[3 + k] * gp1) + W[6 + k] * gp2;
  // M = R diag(s), R = Rn / r2
  float A[3][3], gr2 = 0.f;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    float gs = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float gR = gM[k][j] * sv[j];
      gs += gM[k][j] * R[k][j];
      gr2 -= gR * R[k][j];
      A[k][j] = gR * ir2;
    }
    out[3 + j] = gs * sv[j];  // d/d log-scale
  }
  gr2 *= ir2;
  out[6] = 2.f * (((qx * ((A[0][0] - A[1][1]) - A[2][2]) + qy * (A[0][1] + A[1][0])) + qz * (A[0][2] + A[2][0])) +
                  qw * (A[2][1] - A[1][2])) + 2.f * qx * gr2;
  out[7] = 2.f * (((qy * ((A[1][1] - A[0][0]) - A[2][2]) + qx * (A[0][1] + A[1][0])) + qz * (A[1][2] + A[2][1])) +
                  qw * (A[0][2] - A[2][0])) + 2.f * qy * gr2;
  out[8] = 2.f * (((qz * ((A[2][2] - A[0][0]) - A[1][1]) + qx * (A[0][2] + A[2][0])) + qy * (A[1][2] + A[2][1])) +
                  qw * (A[1][0] - A[0][1])) + 2.f * qz * gr2;
  out[9] = 2.f * (((qw * ((A[0][0] + A[1][1]) + A[2][2]) + qz * (A[1][0] - A[0][1])) + qy * (A[0][2] - A[2][0])) +
                  qx * (A[2][1] - A[1][2])) + 2.f * qw * gr2;
  out[0] = gmu[0];
  out[1] = gmu[1];
  out[2] = gmu[2];
}

// Gradient of the basis polynomial Y_k (sh_basis) in its three arguments.
__device__ __forceinline__ void sh_grad(int k, float x, float y, float z, float gr[3]) {
  float a = 0.f, b = 0.f, c = 0.f;
  switch (k) {
    case 1: b = -SH_C1; break;
    case 2: c = SH_C1; break;
    case 3: a = -SH_C1; break;
    case 4: a = kSH2[0] * y; b = kSH2[0] * x; break;
    case 5: b = kSH2[1] * z; c = kSH2[1] * y; break;
    case 6: a = -2.f * kSH2[2] * x; b = -2.f * kSH2[2] * y; c = 4.f * kSH2[2] * z; break;
    case 7: a = kSH2[3] * z; c = kSH2[3] * x; break;
    case 8: a = 2.f * kSH2[4] * x; b = -2.f * kSH2[4] * y; break;
    case 9: a = 6.f * kSH3[0] * x * y; b = 3.f * kSH3[0] * (x * x - y * y); break;
    case 10: a = kSH3[1] * y * z; b = kSH3[1] * x * z; c = kSH3[1] * x * y; break;
    case 11:
      a = -2.f * kSH3[2] * x * y;
      b = kSH3[2] * ((4.f * z * z - x * x) - 3.f * y * y);
      c = 8.f * kSH3[2] * y * z;
      break;
    case 12:
      a = -6.f * kSH3[3] * x * z;
      b = -6.f * kSH3[3] * y * z;
      c = kSH3[3] * ((6.f * z * z - 3.f * x * x) - 3.f * y * y);
      break;
    case 13:
      a = kSH3[4] * ((4.f * z * z - 3.f * x * x) - y * y);
      b = -2.f * kSH3[4] * x * y;
      c = 8.f * kSH3[4] * x * z;
      break;
    case 14: a = 2.f * kSH3[5] * x * z; b = -2.f * kSH3[5] * y * z; c = kSH3[5] * (x * x - y * y); break;
    case 15: a = 3.f * kSH3[6] * (x * x - y * y); b = -6.f * kSH3[6] * x * y; break;
    default: break;
  }
  gr[0] = a;
  gr[1] = b;
  gr[2] = c;
}

// Rows of the projection backward per wave: a workgroup takes 64 consecutive
// Gaussians (lane = Gaussian, so every row access of a wave is one coalesced
// 256-byte transaction) and its four waves split the rows of those
// Gaussians: wave 0 the mean, log-scale, quaternion and opacity rows (0..10),
// waves 1..3 the SH coefficients [sh_lo(w), sh_lo(w + 1)) in three near-equal
// runs (K = 16 at degree 3: 6, 5, 5 coefficients, 18, 15, 15 rows).
constexpr int kBwdGauss = 64;
template <int DEG>
__host__ __device__ constexpr int sh_lo(int w) {
  return w >= 4 ? (DEG + 1) * (DEG + 1) : ((w - 1) * (DEG + 1) * (DEG + 1) + 2) / 3;
}

// What a wave does with the summed value v of each of its rows (see
// launch_project_bwd; `have` false: no view of the batch sees the Gaussian):
// mode 0 writes (or adds to) out, mode 1 adds v to out (v already holds the
// probes' signs and the scale), mode 2 applies the update of Algorithm 1,
// with D_t read from ft.D, or (HUT) taken from dval_of: the batch's own
// Hutchinson entries, summed in registers.
// Rows go in chunks of kChunk: every load of a chunk is issued before any of
// its stores (the state arrays may alias as far as the compiler knows, so
// loads would otherwise wait for the previous row's stores), which keeps up
// to 5 x kChunk loads in flight per wave without the registers of all rows
// at once.  The optimizer state (ghat, Dhat, D) and the new parameters are each
// touched once per launch: their loads and stores are nontemporal, so they
// do not evict the parameter rows the chain rule reads twice (1.47 -> 1.38 ms
// per city update).
constexpr int kChunk = 6;

template <int R, bool HUT, class RowOf, class ValOf, class DValOf, class EtaOf>
__device__ __forceinline__ void emit_rows(const float* __restrict__ x, int64_t n, int64_t g, int mode, int accumulate,
                                          bool have, float* __restrict__ out, const FusedTr& ft, const RowOf& row_of,
                                          const ValOf& val_of, const DValOf& dval_of, const EtaOf& eta_of) {
#pragma unroll
  for (int c0 = 0; c0 < R; c0 += kChunk) {
    constexpr int C = kChunk;
    if (mode == 0) {
      float o[C];
#pragma unroll
      for (int j = 0; j < C; ++j)
        if (c0 + j < R) o[j] = accumulate ? out[(int64_t)row_of(c0 + j) * n + g] : 0.f;
#pragma unroll
      for (int j = 0; j < C; ++j)
        if (c0 + j < R) out[(int64_t)row_of(c0 + j) * n + g] = accumulate ? o[j] + val_of(c0 + j) : val_of(c0 + j);
    } else if (mode == 1) {
      float o[C];
#pragma unroll
      for (int j = 0; j < C; ++j)
        if (c0 + j < R) o[j] = out[(int64_t)row_of(c0 + j) * n + g];
#pragma unroll
      for (int j = 0; j < C; ++j)
        if (c0 + j < R) out[(int64_t)row_of(c0 + j) * n + g] = o[j] + val_of(c0 + j);
    } else {
      const TrArgs& a = ft.a;
      float xv[C], gh[C], dh[C], dv[C], ga[C];
#pragma unroll
      for (int j = 0; j < C; ++j)
        if (c0 + j < R) {
          const int64_t k = (int64_t)row_of(c0 + j) * n + g;
          xv[j] = x[k];
          gh[j] = __builtin_nontemporal_load(&ft.ghat[k]);
          dh[j] = __builtin_nontemporal_load(&ft.dhat[k]);
          if constexpr (HUT) dv[j] = dval_of(c0 + j);
          else dv[j] = a.hutch ? __builtin_nontemporal_load(&ft.D[k]) : 0.f;
          ga[j] = ft.gacc ? ft.gacc[k] : 0.f;
        }
#pragma unroll
      for (int j = 0; j < C; ++j)
        if (c0 + j < R) {
          const int64_t k = (int64_t)row_of(c0 + j) * n + g;
          // this batch's part added to the earlier batches' sum, as the
          // separate gradient accumulates it
          const float v = have ? val_of(c0 + j) : 0.f;
          const float gk = ft.gacc ? (have ? ga[j] + v : ga[j]) : v;
          const float xn = xv[j] + gs3trust::tr_row(gk, gh[j], dh[j], dv[j], eta_of(c0 + j), a);
          __builtin_nontemporal_store(xn, &ft.x_out[k]);
          __builtin_nontemporal_store(gh[j], &ft.ghat[k]);
          if (a.hutch) __builtin_nontemporal_store(dh[j], &ft.dhat[k]);
          note_nonfinite(ft.nonfinite, gk, xn);
        }
    }
  }
}

// Chain rule from the summed screen-space partials G (d/du, d/dv, d/dconic
// a, b, c, d/dalpha, d/drgb) of every view of a batch to the raw
// parameters, summed over the views in batch order.  Wave 0: per view the
// reverse-mode pass through the projection (geo_vjp), d alpha / d logit =
// s (1 - s), and the colour's dependence on the mean through the view
// direction dir = (mu - campos) / |mu - campos|: sum_k (sum_c g_c f_kc)
// grad Y_k(dir), projected on the plane normal to dir and divided by
// |mu - campos|.  Waves 1..3: d rgb_c / d f_kc = Y_k(dir) where the colour
// clamp is inactive, and their coefficients' share of the direction term,
// passed to wave 0 through LDS and summed in wave order.  A view adds
// nothing for a Gaussian it does not see.  In mode 1 each batch entry is a
// probe of a view, and its part is multiplied by the scale and the probe's
// sign before the sum.  In mode 2 each wave forms the trust-region radii of
// its rows from the parameters before the update (the same expressions as
// the separate update kernel); with HUT the batch's last B.n_probe entries
// are Hutchinson probes, summed as in mode 1 (scale B.probe_scale) into a
// second set of registers that stands in for D_t.
template <int DEG, int mode, bool HUT = false>
__device__ __forceinline__ void project_bwd_body(const float* __restrict__ x, int64_t n, const BwdBatch& B,
                                                 int accumulate, float scale, float* __restrict__ out,
                                                 const FusedTr& ft) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  __shared__ float gdir_part[GS3_MAX_VIEWS][3][3][kBwdGauss];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t g = (int64_t)blockIdx.x * kBwdGauss + lane;
  const bool live = g < n;
  auto xr = [&](int r) { return x[(int64_t)r * n + g]; };
  const float mu[3] = {live ? xr(0) : 0.f, live ? xr(1) : 0.f, live ? xr(2) : 0.f};
  // view direction of the Gaussian in view v
  auto direction = [&](const CamDev& cam, float e[3], float& inv) {
    const float dx = mu[0] - cam.campos[0], dy = mu[1] - cam.campos[1], dz = mu[2] - cam.campos[2];
    inv = 1.f / sqrtf((dx * dx + dy * dy) + dz * dz);
    e[0] = dx * inv;
    e[1] = dy * inv;
    e[2] = dz * inv;
  };
  // the unclamped colour cotangents of view v
  auto colour_cot = [&](const BwdView& V, float gc[3]) {
    const uint32_t posm = __float_as_uint(V.rec[g].c.w);
    const float* Gg = V.G + g * 9;
    gc[0] = (posm & 1u) ? Gg[6] : 0.f;
    gc[1] = (posm & 2u) ? Gg[7] : 0.f;
    gc[2] = (posm & 4u) ? Gg[8] : 0.f;
  };
  // entry v is a Hutchinson probe (mode 1, or the tail of a HUT batch)
  const int first_probe = HUT ? B.n - B.n_probe : (mode == 1 ? 0 : B.n);
  // the weight of entry v's part of row r: the scaled probe sign for a probe
  auto weight = [&](const BwdView& V, int v, int r) {
    if (mode == 1) return scale * probe_sign(V.inner, (uint64_t)((int64_t)r * n + g));
    if (HUT && v >= first_probe) return B.probe_scale * probe_sign(V.inner, (uint64_t)((int64_t)r * n + g));
    return 1.f;
  };
  const float eps = ft.a.epsilon;
  const uint32_t variant = ft.a.variant;
  bool have = false;   // some view of the batch sees the Gaussian
  bool haveh = false;  // HUT: some probe entry sees it
  if (w > 0) {
    // the wave's coefficient run as compile-time indices, so the basis
    // values, row sums and radii stay in registers
    auto run = [&](auto wave) {
      constexpr int W = decltype(wave)::value;
      constexpr int k0 = sh_lo<DEG>(W), k1 = sh_lo<DEG>(W + 1);
      constexpr int NR = 3 * (k1 - k0) > 0 ? 3 * (k1 - k0) : 1;
      float val[NR], dvl[HUT ? NR : 1];
#pragma unroll
      for (int i = 0; i < NR; ++i) val[i] = 0.f;
#pragma unroll
      for (int i = 0; i < (HUT ? NR : 1); ++i) dvl[i] = 0.f;
      for (int v = 0; v < B.n; ++v) {
        const BwdView& V = B.v[v];
        const bool vis = live && V.tiles[g] != 0u;
        const bool pr = HUT && v >= first_probe;
        float part[3] = {0.f, 0.f, 0.f};
        if (vis) {
          float gc[3], e[3], inv;
          colour_cot(V, gc);
          direction(V.cam, e, inv);
          float Y[K];
          sh_basis<float, DEG>(e[0], e[1], e[2], Y);
#pragma unroll
          for (int k = k0; k < k1; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const int i = 3 * (k - k0) + c;
              const float pv = weight(V, v, 11 + 3 * k + c) * (gc[c] * Y[k]);
              if constexpr (HUT) {
                if (pr) dvl[i] = haveh ? dvl[i] + pv : pv;
                else val[i] = have ? val[i] + pv : pv;
              } else {
                val[i] = have ? val[i] + pv : pv;
              }
            }
            if (k == 0) continue;
            // this wave's share of the direction term, coefficients in order
            const float gy = (gc[0] * xr(11 + 3 * k) + gc[1] * xr(12 + 3 * k)) + gc[2] * xr(13 + 3 * k);
            float gr[3];
            sh_grad(k, e[0], e[1], e[2], gr);
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) part[ax] += gy * gr[ax];
          }
          // value updates (a branch on which flag to set becomes a store
          // through a selected private address)
          haveh = haveh || pr;
          have = have || !pr;
        }
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) gdir_part[v][W - 1][ax][lane] = part[ax];
      }
      __syncthreads();
      // an invisible Gaussian adds nothing to an accumulated output
      if (!live || (!have && (mode == 1 || (mode == 0 && accumulate)))) return;
      if constexpr (k1 > k0) {
        gs3trust::Radius rad;
        if (mode == 2) gs3trust::radius_colour(x, n, g, eps, variant, DEG, gs3trust::radius_alpha(x, n, g), rad);
        emit_rows<3 * (k1 - k0), HUT>(
            x, n, g, mode, accumulate, have, out, ft, [&](int i) { return 11 + 3 * k0 + i; },
            [&](int i) { return val[i]; },
            [&](int i) {
              if constexpr (HUT) return dvl[i];
              else return 0.f;
            },
            [&](int i) { return k0 + i / 3 == 0 ? rad.col[i % 3] : rad.rest[i % 3]; });
      }
    };
    if (w == 1) run(std::integral_constant<int, 1>{});
    else if (w == 2) run(std::integral_constant<int, 2>{});
    else run(std::integral_constant<int, 3>{});
    return;
  }
  // wave 0: geometry and opacity
  float d[11], dd[HUT ? 11 : 1];
#pragma unroll
  for (int r = 0; r < 11; ++r) d[r] = 0.f;
#pragma unroll
  for (int r = 0; r < (HUT ? 11 : 1); ++r) dd[r] = 0.f;
  for (int v = 0; v < B.n; ++v) {
    const BwdView& V = B.v[v];
    if (!(live && V.tiles[g] != 0u)) continue;
    const float* Gg = V.G + g * 9;
    const float Gs[5] = {Gg[0], Gg[1], Gg[2], Gg[3], Gg[4]};
    float dv[11];
    geo_vjp(x, n, g, V.cam, Gs, dv);
    const float s = sigmoid_(xr(10));
    dv[10] = Gg[5] * s * (1.f - s);
    const bool pr = HUT && v >= first_probe;
#pragma unroll
    for (int r = 0; r < 11; ++r) {
      const float pv = weight(V, v, r) * dv[r];
      if constexpr (HUT) {
        if (pr) dd[r] = haveh ? dd[r] + pv : pv;
        else d[r] = have ? d[r] + pv : pv;
      } else {
        d[r] = have ? d[r] + pv : pv;
      }
    }
    haveh = haveh || pr;
    have = have || !pr;
  }
  __syncthreads();
  if (DEG > 0) {
    for (int v = 0; v < B.n; ++v) {
      const BwdView& V = B.v[v];
      if (!(live && V.tiles[g] != 0u)) continue;
      float e[3], inv, gdir[3];
      direction(V.cam, e, inv);
#pragma unroll
      for (int ax = 0; ax < 3; ++ax)
        gdir[ax] = (gdir_part[v][0][ax][lane] + gdir_part[v][1][ax][lane]) + gdir_part[v][2][ax][lane];
      const float ed = (e[0] * gdir[0] + e[1] * gdir[1]) + e[2] * gdir[2];
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const float t = weight(V, v, ax) * ((gdir[ax] - e[ax] * ed) * inv);
        if constexpr (HUT) {
          if (v >= first_probe) dd[ax] += t;
          else d[ax] += t;
        } else {
          d[ax] += t;
        }
      }
    }
  }
  if (!live || (!have && (mode == 1 || (mode == 0 && accumulate)))) return;
  gs3trust::Radius rad;
  if (mode == 2) gs3trust::radius_geo(x, n, g, eps, variant, gs3trust::radius_alpha(x, n, g), rad);
  emit_rows<11, HUT>(
      x, n, g, mode, accumulate, have, out, ft, [](int i) { return i; }, [&](int i) { return d[i]; },
      [&](int i) {
        if constexpr (HUT) return dd[i];
        else return 0.f;
      },
      [&](int i) { return gs3trust::row_radius(rad, i); });
}

// The chain rule into a gradient (MODE 0) or a Hutchinson diagonal (MODE 1).
template <int DEG, int MODE>
__global__ __launch_bounds__(256) void k_project_bwd(const float* __restrict__ x, int64_t n, BwdBatch B,
                                                      int accumulate, float scale, float* __restrict__ out) {
  project_bwd_body<DEG, MODE>(x, n, B, accumulate, scale, out, FusedTr{});
}

// The chain rule fused with the update of Algorithm 1 (mode 2): a kernel of
// its own name, so profiles tell it from the gradient launches.
template <int DEG, bool HUT>
__global__ __launch_bounds__(256) void k_tr_update(const float* __restrict__ x, int64_t n, BwdBatch B, FusedTr ft) {
  project_bwd_body<DEG, 2, HUT>(x, n, B, 0, 0.f, nullptr, ft);
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
                        uint32_t* depth_key, uint32_t* tiles, uint32_t* vis_count, hipStream_t st) {
  GS3_DEG_DISPATCH(deg, k_project_fwd, dim3(blocks_for(n, kFwdGauss)), dim3(256), 0, st, x, n, cam, rec, rect,
                   depth_key, tiles, vis_count);
}

void launch_project_jvp(const float* x, int64_t n, int deg, const CamDev& cam, const Rec* rec,
                        const uint32_t* tiles, int probe_kind, uint64_t seed, uint32_t probe_index,
                        const float* tangent, TRec* trec, hipStream_t st) {
  (void)rec;
  GS3_DEG_DISPATCH(deg, k_project_jvp, dim3(blocks_for(n, kJvpChunk)), dim3(256), 0, st, x, n, cam, tiles, probe_kind,
                   probe_inner(seed, probe_index), tangent, trec);
}

void launch_pair_sums(const uint32_t* order, const uint32_t* offsets, const uint32_t* counts, const float* partials,
                      const uint32_t* valid, int64_t n, const uint32_t* n_dev, float* gsum, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_pair_partials, dim3(blocks_for(n, kSumRanks)), dim3(256), 0, st, order, offsets, counts,
                     partials, valid, n, n_dev, gsum);
}

void launch_project_bwd(const float* x, int64_t n, int deg, const BwdBatch& B, int mode, int accumulate, float scale,
                        float* out, const FusedTr& ft, hipStream_t st) {
  if (B.n < 1) return;
  if (mode == 2) {
    auto kernel = [&](auto d, auto h) {
      hipLaunchKernelGGL((k_tr_update<decltype(d)::value, decltype(h)::value>), dim3(blocks_for(n, kBwdGauss)),
                         dim3(256), 0, st, x, n, B, ft);
    };
    auto by_probe = [&](auto d) {
      if (B.n_probe > 0) kernel(d, std::true_type{});
      else kernel(d, std::false_type{});
    };
    switch (deg) {
      case 0: by_probe(std::integral_constant<int, 0>{}); break;
      case 1: by_probe(std::integral_constant<int, 1>{}); break;
      case 2: by_probe(std::integral_constant<int, 2>{}); break;
      default: by_probe(std::integral_constant<int, 3>{}); break;
    }
  } else {
    auto kernel = [&](auto d, auto m) {
      hipLaunchKernelGGL((k_project_bwd<decltype(d)::value, decltype(m)::value>), dim3(blocks_for(n, kBwdGauss)),
                         dim3(256), 0, st, x, n, B, accumulate, scale, out);
    };
    auto by_mode = [&](auto d) {
      if (mode == 1) kernel(d, std::integral_constant<int, 1>{});
      else kernel(d, std::integral_constant<int, 0>{});
    };
    switch (deg) {
      case 0: by_mode(std::integral_constant<int, 0>{}); break;
      case 1: by_mode(std::integral_constant<int, 1>{}); break;
      case 2: by_mode(std::integral_constant<int, 2>{}); break;
      default: by_mode(std::integral_constant<int, 3>{}); break;
    }
  }
}

uint64_t probe_key(uint64_t seed, uint32_t probe_index) { return probe_inner(seed, probe_index); }
