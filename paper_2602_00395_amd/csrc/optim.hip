// Parameter updates for gfx950: the trust-region step of Algorithm 1 and the
// Adam baseline (optionally clipped by the same trust region, ADAM-TR).  The
// radius and the row update are in gs3_trust.h.
#include <type_traits>

#include "gs3_trust.h"

namespace {

using namespace gs3trust;

// The gradient and the optimizer state are each read and written once per
// launch: those accesses are nontemporal (they would only evict the rows the
// radius reads).
// Work split: a workgroup takes 64 consecutive Gaussians and its four waves
// take a quarter of the rows each (wave w: rows [w R, (w+1) R), R = ceil(P/4)),
// so every row access of a wave is one coalesced 256-byte transaction and four
// times more waves keep HBM busy than with one thread per Gaussian.  Every
// thread evaluates its Gaussian's radius from the parameters before the
// update; the barrier keeps the rows the radius reads unchanged until all
// four waves have read them.
constexpr int kGaussPerBlock = 64;

template <int P>
__global__ __launch_bounds__(256) void k_tr_step(float* __restrict__ x, const float* __restrict__ grad,
                                                  float* __restrict__ ghat, float* __restrict__ dhat,
                                                  const float* __restrict__ D, int64_t n, TrArgs a,
                                                  float* __restrict__ eta_out, float* __restrict__ dx_out,
                                                  uint32_t* nonfinite) {
  constexpr int R = (P + 3) / 4;
  const int64_t g = (int64_t)blockIdx.x * kGaussPerBlock + (threadIdx.x & 63);
  const int r0 = (threadIdx.x >> 6) * R;
  const bool live = g < n;
  Radius rad;
  if (live) rad = trust_radius(x, n, g, a.epsilon, a.variant, degree_of_rows(P));
  __syncthreads();
  if (!live) return;
  // the wave's rows as compile-time indices, so the radius components stay
  // in registers (a run-time row index would place them in private memory)
  auto rows = [&](auto wave) {
    constexpr int W = decltype(wave)::value;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int r = W * R + rr;
      if (r >= P) break;
      const int64_t k = (int64_t)r * n + g;
      const float eta = row_radius(rad, r);
      const float gk = __builtin_nontemporal_load(&grad[k]);
      const float step = tr_update(ghat, dhat, D, k, gk, eta, a);
      const float xn = x[k] + step;
      x[k] = xn;
      note_nonfinite(nonfinite, gk, xn);
      if (eta_out) eta_out[k] = eta;
      if (dx_out) dx_out[k] = step;
    }
  };
  switch (r0 / R) {
    case 0: rows(std::integral_constant<int, 0>{}); break;
    case 1: rows(std::integral_constant<int, 1>{}); break;
    case 2: rows(std::integral_constant<int, 2>{}); break;
    default: rows(std::integral_constant<int, 3>{}); break;
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_adam_step(float* __restrict__ x, const float* __restrict__ grad,
                                                    float* __restrict__ m, float* __restrict__ v, int64_t n,
                                                    AdamArgs a, uint32_t* nonfinite) {
  constexpr int R = (P + 3) / 4;
  const int64_t g = (int64_t)blockIdx.x * kGaussPerBlock + (threadIdx.x & 63);
  const int r0 = (threadIdx.x >> 6) * R;
  const bool live = g < n;
  const bool clip = a.epsilon > 0.f;
  Radius rad;
  if (clip) {
    if (live) rad = trust_radius(x, n, g, a.epsilon, 0u, 0);
    __syncthreads();
  }
  if (!live) return;
  // compile-time rows per wave, as in the trust-region step
  auto rows = [&](auto wave) {
    constexpr int W = decltype(wave)::value;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int r = W * R + rr;
      if (r >= P) break;
      const int64_t k = (int64_t)r * n + g;
      const float gr = __builtin_nontemporal_load(&grad[k]);
      const float mm = a.b1 * __builtin_nontemporal_load(&m[k]) + (1.f - a.b1) * gr;
      const float vv = a.b2 * __builtin_nontemporal_load(&v[k]) + (1.f - a.b2) * gr * gr;
      __builtin_nontemporal_store(mm, &m[k]);
      __builtin_nontemporal_store(vv, &v[k]);
      float step = -a.lr_row[r] * (mm / a.bc1) / (sqrtf(vv / a.bc2) + a.eps);
      if (clip) {
        const float eta = row_radius(rad, r);
        step = fminf(fmaxf(step, -eta), eta);
      }
      const float xn = x[k] + step;
      __builtin_nontemporal_store(xn, &x[k]);
      note_nonfinite(nonfinite, gr, xn);
    }
  };
  switch (r0 / R) {
    case 0: rows(std::integral_constant<int, 0>{}); break;
    case 1: rows(std::integral_constant<int, 1>{}); break;
    case 2: rows(std::integral_constant<int, 2>{}); break;
    default: rows(std::integral_constant<int, 3>{}); break;
  }
}

}  // namespace

#define GS3_P_DISPATCH(deg, KERNEL, ...)                   \
  switch (deg) {                                           \
    case 0: hipLaunchKernelGGL(KERNEL<14>, __VA_ARGS__); break; \
    case 1: hipLaunchKernelGGL(KERNEL<23>, __VA_ARGS__); break; \
    case 2: hipLaunchKernelGGL(KERNEL<38>, __VA_ARGS__); break; \
    default: hipLaunchKernelGGL(KERNEL<59>, __VA_ARGS__); break; \
  }

void launch_tr_step(float* x, const float* grad, float* ghat, float* dhat, const float* D, int64_t n, int deg,
                    TrArgs a, float* eta_out, float* dx_out, uint32_t* nonfinite, hipStream_t st) {
  const dim3 grid((unsigned)((n + kGaussPerBlock - 1) / kGaussPerBlock));
  GS3_P_DISPATCH(deg, k_tr_step, grid, dim3(256), 0, st, x, grad, ghat, dhat, D, n, a, eta_out, dx_out, nonfinite);
}

void launch_adam_step(float* x, const float* grad, float* m, float* v, int64_t n, int deg, const AdamArgs& a,
                      uint32_t* nonfinite, hipStream_t st) {
  const dim3 grid((unsigned)((n + kGaussPerBlock - 1) / kGaussPerBlock));
  GS3_P_DISPATCH(deg, k_adam_step, grid, dim3(256), 0, st, x, grad, m, v, n, a, nonfinite);
}
