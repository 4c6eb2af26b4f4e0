// Image-space loss kernels for gfx950: the L1 / D-SSIM components of
// Eq. pixel_loss, their gradient cotangent and the Gauss-Newton cotangent.
//
// Paper: Background, Eq. pixel_loss (L = (1-lambda) L1 + lambda D-SSIM, one
// component per RGB channel) and Eq. objective (F = square roots of the
// components).  With l1 = (1-lambda)|r| and ls = lambda (1 - SSIM):
//  * gradient mode writes  cot = scale * d(sum_k l_k)/dC;
//  * Gauss-Newton mode, given the image tangent u = J_img z, writes
//      cot = scale * sum_k (dl_k/dC)^T (dl_k/dC . u) / (4 max(l_k, 1e-6)),
//    i.e. J_F^T J_F z pulled back to image space (J_F = dl/dC / (2 sqrt(l))).
// SSIM (Wang et al.): 11x11 Gaussian window, sigma 1.5, zero-padded "same"
// filtering, C1 = 0.01^2, C2 = 0.03^2.  SSIM is a function of five filtered
// maps (x, y, x^2, y^2, xy); its VJP filters three coefficient maps with the
// same symmetric window (the adjoint of zero-padded filtering).  Each
// 256-thread workgroup owns a 16x16 output tile and stages a 26x26 halo
// region per channel in LDS, filtering separably (rows, then columns).
#include "gs3_internal.h"

namespace {

constexpr int R = 5;                 // window radius
constexpr int HW = GS3_TILE + 2 * R; // halo width 26
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct Win {
  float w[11];
};

__device__ __forceinline__ float sgn(float r) { return r > 0.f ? 1.f : (r < 0.f ? -1.f : 0.f); }

// Workgroup barrier that orders LDS accesses only: outstanding global loads
// (a prefetch) stay in flight across it.  For kernels whose threads share
// data through LDS alone.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Output tile of this workgroup on a gx-wide grid of nt tiles.  Workgroups
// go to the 8 XCDs round robin and each XCD has its own L2, so workgroup b
// takes tile (b mod 8) ceil(nt / 8) + b / 8: every XCD works through one
// contiguous band of tiles and neighbouring tiles read their shared halo
// rows through the same L2.  False for the padding workgroups past nt.
__device__ __forceinline__ bool ssim_tile(int gx, int nt, int& bx, int& by, int& t) {
  const int per = (nt + 7) / 8;
  t = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
  bx = t % gx;
  by = t / gx;
  return t < nt;
}

__device__ __forceinline__ double block_sum_d(double v) {
  __shared__ double ws[4];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = ((ws[0] + ws[1]) + ws[2]) + ws[3];
  __syncthreads();
  return r;
}

// Gradient (GN = false) or Gauss-Newton (GN = true) coefficient maps of the
// SSIM term, and (gradient mode) per-block loss sums.  The 26x26 halo region
// of all three channels is loaded in one pass (each region row is 78
// consecutive floats); coefficient maps are stored planar, map m of channel c
// at coef[(3 m + c) npix + pixel], so the combine pass reads whole rows.
template <bool GN>
__global__ __launch_bounds__(GS3_BLOCK) void k_ssim_coef(const float* __restrict__ img, const float* __restrict__ tgt,
                                                          const float* __restrict__ u, int W, int H, float lam,
                                                          float scale, Win win, float* __restrict__ coef,
                                                          double* __restrict__ loss_partials, int gx, int nt) {
  int bx, by, t;
  if (!ssim_tile(gx, nt, bx, by, t)) return;
  __shared__ float sx[3][HW][HW + 1], sy[3][HW][HW + 1], su[GN ? 3 : 1][GN ? HW : 1][HW + 1];
  constexpr int NM = GN ? 8 : 5;
  __shared__ float hb[NM][HW][GS3_TILE];
  const int tid = threadIdx.x;
  const int ox = bx * GS3_TILE - R, oy = by * GS3_TILE - R;
  const int i = tid >> 4, j = tid & 15;
  const int px = bx * GS3_TILE + j, py = by * GS3_TILE + i;
  const bool inside = px < W && py < H;
  const int64_t npix = (int64_t)W * H;
  {
    // element e = tid + 256 k of the region (row r, column qq, channel c);
    // 256 = 3 rows of 78 + 22 = 3 rows + 7 columns + 1 channel, so the
    // indices advance by additions instead of divisions per element
    int r = tid / (HW * 3), qq = (tid % (HW * 3)) / 3, c = tid % 3;
    for (int e = tid; e < HW * HW * 3; e += GS3_BLOCK) {
      const int gx = ox + qq, gy = oy + r;
      const bool ok = gx >= 0 && gy >= 0 && gx < W && gy < H;
      const int64_t o = ((int64_t)gy * W + gx) * 3 + c;
      sx[c][r][qq] = ok ? img[o] : 0.f;
      sy[c][r][qq] = ok ? tgt[o] : 0.f;
      if (GN) su[c][r][qq] = ok ? u[o] : 0.f;
      r += GS3_BLOCK / (HW * 3);
      qq += (GS3_BLOCK % (HW * 3)) / 3;
      c += GS3_BLOCK % 3;
      if (c >= 3) {
        c -= 3;
        ++qq;
      }
      if (qq >= HW) {
        qq -= HW;
        ++r;
      }
    }
  }
  __syncthreads();
  double lsum = 0.0;
  for (int c = 0; c < 3; ++c) {
    // horizontal pass: a thread filters two adjacent outputs of a row, q0
    // and q0 + 1, from one window of 12 inputs, so every product is formed
    // once for both (same terms in the same order as one output at a time)
    for (int e = tid; e < HW * (GS3_TILE / 2); e += GS3_BLOCK) {
      const int r = e / (GS3_TILE / 2), q0 = 2 * (e % (GS3_TILE / 2));
      float m0[NM], m1[NM];
#pragma unroll
      for (int k = 0; k < NM; ++k) m0[k] = m1[k] = 0.f;
#pragma unroll
      for (int t = 0; t < 12; ++t) {
        const float xv = sx[c][r][q0 + t], yv = sy[c][r][q0 + t];
        float pr[NM];
        pr[0] = xv;
        pr[1] = yv;
        pr[2] = xv * xv;
        pr[3] = yv * yv;
        pr[4] = xv * yv;
        if (GN) {
          const float uv = su[c][r][q0 + t];
          pr[5] = uv;
          pr[6] = 2.f * xv * uv;
          pr[7] = yv * uv;
        }
        if (t < 11) {
          const float wk = win.w[t];
#pragma unroll
          for (int k = 0; k < NM; ++k) m0[k] += wk * pr[k];
        }
        if (t >= 1) {
          const float wk = win.w[t - 1];
#pragma unroll
          for (int k = 0; k < NM; ++k) m1[k] += wk * pr[k];
        }
      }
#pragma unroll
      for (int k = 0; k < NM; ++k) {
        hb[k][r][q0] = m0[k];
        hb[k][r][q0 + 1] = m1[k];
      }
    }
    __syncthreads();
    float f[NM];
#pragma unroll
    for (int k = 0; k < NM; ++k) f[k] = 0.f;
#pragma unroll
    for (int k = 0; k < 11; ++k) {
      const float wk = win.w[k];
#pragma unroll
      for (int m = 0; m < NM; ++m) f[m] += wk * hb[m][i + k][j];
    }
    const float A = f[0], B = f[1];
    const float sxx = f[2] - A * A, syy = f[3] - B * B, sxy = f[4] - A * B;
    const float n1 = 2.f * A * B + kC1, n2 = 2.f * sxy + kC2;
    const float d1 = A * A + B * B + kC1, d2 = sxx + syy + kC2;
    // one division: 1 / d2 = d1 / (d1 d2)
    const float inv = 1.f / (d1 * d2);
    const float S = (n1 * n2) * inv;
    const float dS_dA = (2.f * B * (n2 - n1) - S * 2.f * A * (d2 - d1)) * inv;
    const float dS_dXX = -S * (d1 * inv);
    const float dS_dXY = 2.f * n1 * inv;
    float wgt;
    if (GN) {
      const float dS = dS_dA * f[5] + dS_dXX * f[6] + dS_dXY * f[7];
      const float ls = lam * (1.f - S);
      wgt = scale * (lam * lam * dS) / (4.f * fmaxf(ls, GS3_GN_FLOOR));
    } else {
      wgt = -lam * scale;
      if (inside) {
        const float xv = sx[c][i + R][j + R], yv = sy[c][i + R][j + R];
        lsum += (double)((1.f - lam) * fabsf(xv - yv)) + (double)(lam * (1.f - S));
      }
    }
    if (inside) {
      const int64_t o = (int64_t)py * W + px;
      coef[(0 * 3 + c) * npix + o] = wgt * dS_dA;
      coef[(1 * 3 + c) * npix + o] = wgt * dS_dXX;
      coef[(2 * 3 + c) * npix + o] = wgt * dS_dXY;
    }
    __syncthreads();
  }
  if (!GN) {
    const double tot = block_sum_d(lsum);
    if (tid == 0) loss_partials[t] = tot;
  }
}

// Filter the three coefficient maps and add the L1 term: the final cotangent.
template <bool GN>
__global__ __launch_bounds__(GS3_BLOCK) void k_ssim_combine(const float* __restrict__ img,
                                                             const float* __restrict__ tgt,
                                                             const float* __restrict__ u,
                                                             const float* __restrict__ coef, int W, int H, float lam,
                                                             float scale, Win win, float* __restrict__ cot, int gx,
                                                             int nt) {
  int bx, by, t;
  if (!ssim_tile(gx, nt, bx, by, t)) return;
  __shared__ float sc[3][HW][HW + 1];
  __shared__ float hb[3][HW][GS3_TILE];
  const int tid = threadIdx.x;
  const int ox = bx * GS3_TILE - R, oy = by * GS3_TILE - R;
  const int i = tid >> 4, j = tid & 15;
  const int px = bx * GS3_TILE + j, py = by * GS3_TILE + i;
  const bool inside = px < W && py < H;
  const int64_t npix = (int64_t)W * H;
  const int64_t o3 = ((int64_t)py * W + px) * 3;
  float xv[3] = {0.f, 0.f, 0.f}, yv[3] = {0.f, 0.f, 0.f}, uv[3] = {0.f, 0.f, 0.f}, out[3];
  if (inside) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xv[c] = img[o3 + c];
      yv[c] = tgt[o3 + c];
      if (GN) uv[c] = u[o3 + c];
    }
  }
  // the next channel's halo of the three maps is loaded into registers
  // while this channel is filtered; the barriers inside order LDS only, so
  // those loads stay in flight across them
  constexpr int kPer = (HW * HW + GS3_BLOCK - 1) / GS3_BLOCK;
  float pre[kPer][3];
  auto load = [&](int c) {
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int e = tid + t * GS3_BLOCK;
      const int r = e / HW, q = e % HW;
      const int gx = ox + q, gy = oy + r;
      const bool ok = e < HW * HW && gx >= 0 && gy >= 0 && gx < W && gy < H;
      const int64_t o = (int64_t)gy * W + gx;
#pragma unroll
      for (int m = 0; m < 3; ++m) pre[t][m] = ok ? coef[(m * 3 + c) * npix + o] : 0.f;
    }
  };
  load(0);
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int e = tid + t * GS3_BLOCK;
      if (e < HW * HW) {
#pragma unroll
        for (int m = 0; m < 3; ++m) sc[m][e / HW][e % HW] = pre[t][m];
      }
    }
    lds_barrier();
    if (c < 2) load(c + 1);
    for (int e = tid; e < HW * GS3_TILE; e += GS3_BLOCK) {
      const int r = e / GS3_TILE, q = e % GS3_TILE;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < 11; ++k) acc += win.w[k] * sc[m][r][q + k];
        hb[m][r][q] = acc;
      }
    }
    lds_barrier();
    float bA = 0.f, bXX = 0.f, bXY = 0.f;
#pragma unroll
    for (int k = 0; k < 11; ++k) {
      bA += win.w[k] * hb[0][i + k][j];
      bXX += win.w[k] * hb[1][i + k][j];
      bXY += win.w[k] * hb[2][i + k][j];
    }
    const float r = xv[c] - yv[c], sg = sgn(r);
    float l1term;
    if (GN) {
      const float l1 = (1.f - lam) * fabsf(r);
      const float w1 = (1.f - lam) * sg * uv[c] / (4.f * fmaxf(l1, GS3_GN_FLOOR));
      l1term = scale * (1.f - lam) * sg * w1;
    } else {
      l1term = scale * (1.f - lam) * sg;
    }
    out[c] = l1term + (bA + 2.f * xv[c] * bXX + yv[c] * bXY);
    lds_barrier();
  }
  if (inside) {
#pragma unroll
    for (int c = 0; c < 3; ++c) cot[o3 + c] = out[c];
  }
}

// lambda = 0: the L1 term only.
template <bool GN>
__global__ __launch_bounds__(256) void k_l1_only(const float* __restrict__ img, const float* __restrict__ tgt,
                                                  const float* __restrict__ u, int64_t n, float scale,
                                                  float* __restrict__ cot, double* __restrict__ loss_partials) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (o < n) {
    const float r = img[o] - tgt[o], s = sgn(r);
    if (GN) {
      const float l1 = fabsf(r);
      cot[o] = scale * s * (s * u[o] / (4.f * fmaxf(l1, GS3_GN_FLOOR)));
    } else {
      cot[o] = scale * s;
      l = (double)fabsf(r);
    }
  }
  if (!GN) {
    const double tot = block_sum_d(l);
    if (threadIdx.x == 0) loss_partials[blockIdx.x] = tot;
  }
}

__global__ __launch_bounds__(256) void k_sq_err(const float* __restrict__ img, const float* __restrict__ tgt,
                                                 int64_t n, double* __restrict__ partials) {
  double acc = 0.0;
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n; o += (int64_t)gridDim.x * blockDim.x) {
    const double d = (double)img[o] - (double)tgt[o];
    acc += d * d;
  }
  const double tot = block_sum_d(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ p, int n, double* __restrict__ out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += p[i];
  const double tot = block_sum_d(acc);
  if (threadIdx.x == 0) *out = tot;
}

Win make_window() {
  Win w;
  double s = 0.0, v[11];
  for (int k = 0; k < 11; ++k) {
    const double d = k - 5;
    v[k] = exp(-(d * d) / (2.0 * 1.5 * 1.5));
    s += v[k];
  }
  for (int k = 0; k < 11; ++k) w.w[k] = (float)(v[k] / s);
  return w;
}

}  // namespace

size_t ssim_tmp_floats(int w, int h) { return (size_t)3 * 3 * w * h; }

void launch_loss_grad(const float* img, const float* tgt, int w, int h, float lam, float scale, float* cot,
                      float* ssim_tmp, double* loss_partials, int* n_partials, hipStream_t st) {
  const int64_t n = (int64_t)w * h * 3;
  if (lam == 0.f) {
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_l1_only<false>, dim3(nb), dim3(256), 0, st, img, tgt, nullptr, n, scale, cot,
                       loss_partials);
    *n_partials = (int)nb;
    return;
  }
  const int gx = (w + GS3_TILE - 1) / GS3_TILE, nt = gx * ((h + GS3_TILE - 1) / GS3_TILE);
  const dim3 grid((unsigned)(8 * ((nt + 7) / 8)));
  const Win win = make_window();
  hipLaunchKernelGGL(k_ssim_coef<false>, grid, dim3(GS3_BLOCK), 0, st, img, tgt, nullptr, w, h, lam, scale, win,
                     ssim_tmp, loss_partials, gx, nt);
  hipLaunchKernelGGL(k_ssim_combine<false>, grid, dim3(GS3_BLOCK), 0, st, img, tgt, nullptr, ssim_tmp, w, h, lam,
                     scale, win, cot, gx, nt);
  *n_partials = nt;
}

void launch_loss_gn(const float* img, const float* tgt, const float* u, int w, int h, float lam, float scale,
                    float* cot, float* ssim_tmp, hipStream_t st) {
  const int64_t n = (int64_t)w * h * 3;
  if (lam == 0.f) {
    hipLaunchKernelGGL(k_l1_only<true>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, img, tgt, u, n, scale,
                       cot, nullptr);
    return;
  }
  const int gx = (w + GS3_TILE - 1) / GS3_TILE, nt = gx * ((h + GS3_TILE - 1) / GS3_TILE);
  const dim3 grid((unsigned)(8 * ((nt + 7) / 8)));
  const Win win = make_window();
  hipLaunchKernelGGL(k_ssim_coef<true>, grid, dim3(GS3_BLOCK), 0, st, img, tgt, u, w, h, lam, scale, win, ssim_tmp,
                     nullptr, gx, nt);
  hipLaunchKernelGGL(k_ssim_combine<true>, grid, dim3(GS3_BLOCK), 0, st, img, tgt, u, ssim_tmp, w, h, lam, scale,
                     win, cot, gx, nt);
}

void launch_sq_err(const float* img, const float* tgt, int64_t n, double* partials, int* n_partials, hipStream_t st) {
  const unsigned nb = 256;
  hipLaunchKernelGGL(k_sq_err, dim3(nb), dim3(256), 0, st, img, tgt, n, partials);
  *n_partials = (int)nb;
}

void launch_sum_partials(const double* partials, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, partials, n, out);
}
