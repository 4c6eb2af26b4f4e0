// Alpha blending of depth-sorted splats (front to back), its JVP and its VJP
// (back to front), for gfx950.
//
// Paper: Background, "Review of Gaussian Splatting": C = sum_i c_i abar_i T_i
// with T_i = prod_{j<i} (1 - abar_j) over the splats of the pixel's tile in
// depth order.  Rasteriser readings (the paper names none): abar =
// min(0.99, alpha exp(power)), power = -1/2 d^T conic d; power > 0 or
// abar < 1/255 is skipped; a pixel stops before the splat that would take T
// below 1e-4; the output adds T_final times the background colour.
// The skip test is taken as power < tau with tau = float32(-ln(255 alpha)),
// power evaluated in float32 in a fixed order without contraction: the
// decision which splats contribute is then a reproducible float32 function
// of the splat record, not a side effect of exp's rounding.
//
// Layout: one 256-thread workgroup per 16x16 tile, one pixel per thread,
// each wave64 an 8x8 block of the tile; records of a batch of splats are
// staged in LDS together with, per wave, a bit mask of the splats whose
// skip test can pass somewhere in its block (the skip ellipse, widened by its
// float32 rounding, against the block's rectangle of pixel centres), and
// every wave walks only the set bits (the forward and the JVP compact those
// splats to the front of their slice and walk them in order).  In the forward and the JVP each wave
// stages its own batches in a private LDS slice and never waits for the
// other three (they differ in how far their pixels blend); the backward
// stages per workgroup.  Culled
// evaluations are exactly the ones the skip test would reject, so the
// result is the same bit for bit.  Workgroups take tiles longest list first
// (a pixel's walk is serial, so the tiles with the longest lists bound the
// kernel unless they start early); without that order each of the 8 XCDs
// gets a contiguous band of tiles (neighbouring tiles share splats, and each
// XCD has its own L2).
//
// The backward cuts each tile's list into depth segments of GS3_SEG pairs and
// runs one workgroup per (tile, segment), longest first: a few hundred tiles
// hold most of the pairs, and whole tiles would leave some SIMDs with one
// long walk more than others.  For tiles of more than one segment the
// forward (and the JVP) store, at every segment boundary a pixel reaches, its
// transmittance and the colour the segment added; the backward of segment m
// starts from the transmittance after m and the colour of the later segments
// up to the pixel's last contribution.
//
// The backward pass walks each tile back to front: the forward stores, per
// pixel, its final transmittance and the last splat that contributed; the
// backward starts there, recovers T in front of each splat as T / (1 - abar)
// and accumulates (sum over the splats behind of c w + T_final bg) . dL/dC
// from zero, so no term comes from cancelling two large sums (a deep splat's
// gradient keeps its relative precision).  Which splats contribute is taken
// from the same float32 skip test and the stored last index, so the set is
// exactly the forward's.  Per pixel it reduces dL/dopacity times dx, dy,
// dx^2, dx dy and dy^2 (dL/dpower is the opacity times dL/dopacity); the
// opacity and the conic coefficients are constant over the splat, so the
// derivatives along u, v and the conic are formed once per splat.  Gradients
// of each (splat, tile) pair are reduced over the workgroup (a transposed
// wave64 reduction with permlane swaps and DPP row scans, then the four waves
// in LDS in a fixed order) and written to the pair's own slot: no float
// atomics, so the backward is deterministic.
#include <algorithm>

#include "gs3_internal.h"

namespace {

// Tile of workgroup b: the longest-list-first order when given, else each of
// the 8 XCDs (which receive workgroups round robin) gets a contiguous band.
__device__ __forceinline__ int tile_of_block(int b, const uint32_t* order, int n_tiles, int chunk) {
  if (order) return b < n_tiles ? (int)order[b] : n_tiles;
  return (b & 7) * chunk + (b >> 3);
}

// Measurement hook of the COUNT instances: adds this wave's number of
// (pixel, splat) evaluations and of contributing evaluations to one of the
// launch's GS3_PROF_SUB counter pairs (ctr[2 s], ctr[2 s + 1]).  The
// instances launched without counters carry no counting instructions.
template <bool COUNT>
__device__ __forceinline__ void count_evals(unsigned long long* ctr, uint32_t nev, uint32_t ncon) {
  if (!COUNT) return;
  unsigned long long a = nev, b = ncon;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    a += __shfl_xor(a, m, 64);
    b += __shfl_xor(b, m, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    const int sub = (int)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % GS3_PROF_SUB);
    atomicAdd(ctr + 2 * sub, a);
    atomicAdd(ctr + 2 * sub + 1, b);
  }
}

// -1/2 d^T conic d in float32 from the pre-scaled conic (qa, qb, qc) =
// (-a/2, -b, -c/2), rounded exactly as written: equal bit for bit to
// -1/2 ((a dx) dx + (c dy) dy) - (b dx) dy.
__device__ __forceinline__ float splat_power(float qa, float qb, float qc, float dx, float dy) {
#pragma clang fp contract(off)
  return ((qa * dx) * dx + (qc * dy) * dy) + (qb * dx) * dy;
}


// Pixel of thread `tid` in tile (tx, ty): wave w = tid / 64 covers the 8x8
// block (w & 1, w >> 1), lane l its pixel (l & 7, l >> 3).
__device__ __forceinline__ int pixel_x(int tx, int tid) { return tx * GS3_TILE + ((tid >> 6) & 1) * 8 + (tid & 7); }
__device__ __forceinline__ int pixel_y(int ty, int tid) { return ty * GS3_TILE + (tid >> 7) * 8 + ((tid >> 3) & 7); }

// Minimum of q(x, y) = a x^2 + 2 b x y + c y^2 (positive definite) over the
// rectangle [x0, x1] x [y0, y1]: 0 if the rectangle holds the origin, else
// the least of the four edges' minima (each a 1D quadratic, its minimiser
// clamped to the edge).  sx = -b / c and sy = -b / a give the minimisers
// y = sx x on a vertical edge and x = sy y on a horizontal one.
__device__ __forceinline__ double quad_rect_min(double a, double b, double c, double sx, double sy, double x0,
                                                double x1, double y0, double y1) {
  if (x0 <= 0.0 && x1 >= 0.0 && y0 <= 0.0 && y1 >= 0.0) return 0.0;
  auto q = [&](double x, double y) { return (a * x + 2.0 * b * y) * x + c * y * y; };
  auto on_x = [&](double x) { return q(x, fmin(fmax(sx * x, y0), y1)); };
  auto on_y = [&](double y) { return q(fmin(fmax(sy * y, x0), x1), y); };
  return fmin(fmin(on_x(x0), on_x(x1)), fmin(on_y(y0), on_y(y1)));
}

// Which of the four 8x8 blocks of tile (tx, ty) may hold a pixel whose skip
// test passes for the splat (u, v, pre-scaled conic qa, qb, qc, threshold
// tau); bit b for block b.  With the plain conic Q = (a, b; b, c) =
// (-2 qa, -qb; -qb, -2 qc), the test asks p >= tau for the float32 power p of
// -1/2 d^T Q d, so it can pass only where d^T Q d <= k (1 + r) with k = -2 tau
// and r the relative rounding error of p: with rho^2 = b^2 / (a c), r is at
// most 4 u (1 + rho) / (1 - rho), below 1e-3 for rho^2 <= 0.999 (u = 2^-24).
// A block is kept when the minimum of d^T Q d over the rectangle spanned by
// its pixel centres is at most 1.002 k + 1e-4, evaluated in double (det Q of
// the float32 entries is then exact up to one rounding; a minimiser off by a
// few double roundings is still a point of the rectangle, and raises q by a
// second-order amount far inside the 1e-4).  Splats with
// rho^2 > 0.999 or non-finite entries are never culled; tau > 0 passes
// nowhere.
struct Cull {
  int all;  // -1: no pixel passes, 1: never culled, 0: test each block
  double a, b, c, sx, sy, k, x0, y0;
};
__device__ __forceinline__ Cull cull_setup(float4 A, float4 B, float tau, int tx, int ty) {
  Cull q{};
  if (tau > 0.f) {
    q.all = -1;
    return q;
  }
  q.a = -2.0 * (double)A.z;
  q.b = -(double)A.w;
  q.c = -2.0 * (double)B.x;
  const double det = q.a * q.c - q.b * q.b;
  q.all = (q.a > 0.0 && q.c > 0.0 && det * 1000.0 >= q.a * q.c && det < INFINITY) ? 0 : 1;
  q.k = -2.004 * (double)tau + 1e-4;
  q.x0 = tx * GS3_TILE + 0.5 - (double)A.x;
  q.y0 = ty * GS3_TILE + 0.5 - (double)A.y;
  q.sx = -q.b / q.c;
  q.sy = -q.b / q.a;
  return q;
}
__device__ __forceinline__ bool cull_keep(const Cull& q, int blk) {
  if (q.all != 0) return q.all > 0;
  const double bx = q.x0 + 8 * (blk & 1), by = q.y0 + 8 * (blk >> 1);
  return quad_rect_min(q.a, q.b, q.c, q.sx, q.sy, bx, bx + 7.0, by, by + 7.0) <= q.k;
}
// all four blocks: bit b for block b
__device__ __forceinline__ uint32_t block_mask(float4 A, float4 B, float tau, int tx, int ty) {
  const Cull q = cull_setup(A, B, tau, tx, ty);
  uint32_t m = 0u;
#pragma unroll
  for (int blk = 0; blk < 4; ++blk) m |= cull_keep(q, blk) ? (1u << blk) : 0u;
  return m;
}

// Orders this wave's LDS writes before its later LDS reads and the reads
// before later writes (its lanes exchange data through a wave-private slice).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Publish the block masks of the splats staged by this wave (one splat per
// lane, `m` = 0 for empty slots): bits[b][wave] gets bit l for lane l.  Every
// lane of the wave must call it.
template <int NW>
__device__ __forceinline__ void publish_masks(uint64_t (*bits)[NW], uint32_t m, int tid) {
  const uint64_t b0 = __ballot(m & 1u), b1 = __ballot(m & 2u), b2 = __ballot(m & 4u), b3 = __ballot(m & 8u);
  if ((tid & 63) == 0) {
    const int sw = tid >> 6;
    bits[0][sw] = b0;
    bits[1][sw] = b1;
    bits[2][sw] = b2;
    bits[3][sw] = b3;
  }
}

// The tile's pair range, held in scalar registers (one value per workgroup),
// so that the batch loops and the bit walks derived from it stay scalar.
__device__ __forceinline__ uint2 uniform_range(const uint2* ranges, int t) {
  const uint2 r = ranges[t];
  return make_uint2(__builtin_amdgcn_readfirstlane(r.x), __builtin_amdgcn_readfirstlane(r.y));
}

// A wave-uniform copy of a 64-bit LDS word (held in scalar registers).
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// One wave's batch of 64 splats (the forward's waves never wait for each
// other: each stages, culls for its own 8x8 block and walks on its own).
struct StageW {
  float4 a[64];
  float4 b[64];
  float4 c[64];  // b, tau, 1 + pair index (as bits), unused
};

template <bool COUNT>
__device__ __forceinline__ void blend_fwd_body(const Rec* __restrict__ rec, const uint32_t* __restrict__ pair_gid,
                                               const uint2* __restrict__ ranges, const uint32_t* __restrict__ order,
                                               const CamDev& cam, float bg0, float bg1, float bg2,
                                               float* __restrict__ img, uint32_t* __restrict__ pix_last,
                                               float* __restrict__ pix_T, float4* __restrict__ seg, int n_tiles,
                                               int chunk, int bid, unsigned long long* __restrict__ ctr) {
  const int t = tile_of_block(bid, order, n_tiles, chunk);
  if (t >= n_tiles) return;
  __shared__ StageW stage[4];
  uint32_t nev = 0, ncon = 0;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  StageW& s = stage[w];
  const int tx = t % cam.tiles_x, ty = t / cam.tiles_x;
  const int px = pixel_x(tx, tid), py = pixel_y(ty, tid);
  const bool inside = px < cam.width && py < cam.height;
  const float pxf = (float)px + 0.5f, pyf = (float)py + 0.5f;
  const uint2 range = uniform_range(ranges, t);
  // C: colour added by the current depth segment, E: by the finished ones
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, E0 = 0.f, E1 = 0.f, E2 = 0.f;
  // 1 while the pixel still blends; an integer rather than a bool, so the
  // loop carries it in a vector register instead of a scalar lane mask
  uint32_t live = inside ? 1u : 0u;
  uint32_t lastp = 0u;  // 1 + pair index of the last contributing splat (0: none)
  const bool split = range.y - range.x > GS3_SEG;
  float4* seg_px = seg + ((int64_t)t + range.x / GS3_SEG) * GS3_BLOCK + tid;
  uint32_t cur = 0;  // depth segment of the batch being walked
  // this lane's pair id of the batch about to be staged, loaded one batch
  // ahead so that staging waits for one dependent load, not two
  uint32_t g_next = range.x + lane < range.y ? pair_gid[range.x + lane] : 0u;
  for (uint32_t start = range.x; start < range.y; start += 64) {
    // every pixel of the block has stopped: the rest is never read
    if (__ballot(live) == 0ull) break;
    if (split && start != range.x && (start - range.x) % GS3_SEG == 0) {
      seg_px[(int64_t)cur * GS3_BLOCK] = make_float4(T, C0, C1, C2);
      E0 += C0;
      E1 += C1;
      E2 += C2;
      C0 = C1 = C2 = 0.f;
      ++cur;
    }
    const uint32_t i = start + lane;
    // the splats this wave's block keeps are compacted to the front of its
    // slice, in pair order, so the walk below steps through consecutive
    // records with a counter instead of scanning a bit mask
    bool keep = false;
    Rec r;
    if (i < range.y) {
      r = rec[g_next];
      keep = cull_keep(cull_setup(r.a, r.b, r.c.y, tx, ty), w);
    }
    if (i + 64 < range.y) g_next = pair_gid[i + 64];
    const uint64_t kb = __ballot(keep);
    const int cnt = __builtin_popcountll(kb);
    if (keep) {
      const int pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(kb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)kb, 0u));
      s.a[pos] = r.a;
      s.b[pos] = r.b;
      s.c[pos] = make_float4(r.c.x, r.c.y, __uint_as_float(i + 1u), 0.f);
    }
    wave_lds_sync();
    // one walked splat; `valid` false: no splat (the odd slot of a pair)
    auto walk = [&](const float4 A, const float4 B, const float4 Cc, const bool valid) {
      if (COUNT) nev += valid ? live : 0u;
      const float dx = A.x - pxf, dy = A.y - pyf;
      const float power = splat_power(A.z, A.w, B.x, dx, dy);
      // predicated rather than branched: nearly every wave has a lane
      // that contributes, so a branch would only add mask bookkeeping
      const bool pass = valid && live && power <= 0.f && power >= Cc.y;
      const float a = fminf(GS3_ALPHA_MAX, B.y * __expf(power));
      const float Tn = T * (1.f - a);
      const bool stop = pass && Tn < GS3_T_STOP;
      const bool use = pass && !stop;
      live = stop ? 0u : live;
      if (COUNT) ncon += use ? 1u : 0u;
      const float w8 = use ? a * T : 0.f;
      C0 += B.z * w8;
      C1 += B.w * w8;
      C2 += Cc.x * w8;
      T = use ? Tn : T;
      lastp = use ? __float_as_uint(Cc.z) : lastp;
    };
    // splats are walked in pairs: both walks of a pair sit in one scheduling
    // region, so the second's transmittance-free part (offset, power, alpha)
    // overlaps the first's transmittance update, and the stop test runs once
    // per pair.  The records of the next pair are read from LDS one pair
    // ahead, into the other of two register sets.  Every slot read is one
    // of this batch's records (indices clamped to the count): the idle
    // second walk of an odd count multiplies its colour by a zero weight,
    // and a stale slot could hold an infinity.
    if (cnt > 0) {
      const int f1 = min(1, cnt - 1);
      float4 A0 = s.a[0], B0 = s.b[0], D0 = s.c[0], A1 = s.a[f1], B1 = s.b[f1], D1 = s.c[f1];
      float4 A2, B2, D2, A3, B3, D3;
      for (int j = 0;;) {
        const int n2 = min(j + 2, cnt - 1), n3 = min(j + 3, cnt - 1);
        A2 = s.a[n2];
        B2 = s.b[n2];
        D2 = s.c[n2];
        A3 = s.a[n3];
        B3 = s.b[n3];
        D3 = s.c[n3];
        __builtin_amdgcn_sched_barrier(0);
        walk(A0, B0, D0, true);
        walk(A1, B1, D1, j + 1 < cnt);
        j += 2;
        if (j >= cnt || __ballot(live) == 0ull) break;
        const int n0 = min(j + 2, cnt - 1), n1 = min(j + 3, cnt - 1);
        A0 = s.a[n0];
        B0 = s.b[n0];
        D0 = s.c[n0];
        A1 = s.a[n1];
        B1 = s.b[n1];
        D1 = s.c[n1];
        __builtin_amdgcn_sched_barrier(0);
        walk(A2, B2, D2, true);
        walk(A3, B3, D3, j + 1 < cnt);
        j += 2;
        if (j >= cnt || __ballot(live) == 0ull) break;
      }
    }
    wave_lds_sync();
  }
  if (split) seg_px[(int64_t)cur * GS3_BLOCK] = make_float4(T, C0, C1, C2);
  if (inside) {
    const int64_t pix = (int64_t)py * cam.width + px;
    float* o = img + pix * 3;
    o[0] = (E0 + C0) + T * bg0;
    o[1] = (E1 + C1) + T * bg1;
    o[2] = (E2 + C2) + T * bg2;
    pix_last[pix] = lastp;
    pix_T[pix] = T;
  }
  count_evals<COUNT>(ctr, nev, ncon);
}

// One wave's batch of 64 splats with their tangent records (the JVP's
// waves, like the forward's, never wait for each other).
struct StageJW {
  float4 a[64];
  float4 b[64];
  float4 ta[64];
  float4 tb[64];
  float4 c[64];  // b, tau, tangent of b, 1 + pair index (as bits)
};

template <bool COUNT>
__device__ __forceinline__ void blend_jvp_body(const Rec* __restrict__ rec, const TRec* __restrict__ trec,
                                               const uint32_t* __restrict__ pair_gid,
                                               const uint2* __restrict__ ranges, const uint32_t* __restrict__ order,
                                               const CamDev& cam, float bg0, float bg1, float bg2,
                                               float* __restrict__ img, float* __restrict__ tan_img,
                                               uint32_t* __restrict__ pix_last, float* __restrict__ pix_T,
                                               float4* __restrict__ seg, int n_tiles, int chunk, int bid,
                                               unsigned long long* __restrict__ ctr) {
  const int t = tile_of_block(bid, order, n_tiles, chunk);
  if (t >= n_tiles) return;
  __shared__ StageJW stage[4];
  uint32_t nev = 0, ncon = 0;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  StageJW& s = stage[w];
  const int tx = t % cam.tiles_x, ty = t / cam.tiles_x;
  const int px = pixel_x(tx, tid), py = pixel_y(ty, tid);
  const bool inside = px < cam.width && py < cam.height;
  const float pxf = (float)px + 0.5f, pyf = (float)py + 0.5f;
  const uint2 range = uniform_range(ranges, t);
  float T = 1.f, dT = 0.f;
  float C0 = 0.f, C1 = 0.f, C2 = 0.f, D0 = 0.f, D1 = 0.f, D2 = 0.f, E0 = 0.f, E1 = 0.f, E2 = 0.f;
  uint32_t live = inside ? 1u : 0u;  // as in the forward
  uint32_t lastp = 0u;
  // depth segments of long tiles, as in the forward
  const bool split = range.y - range.x > GS3_SEG;
  float4* seg_px = seg + ((int64_t)t + range.x / GS3_SEG) * GS3_BLOCK + tid;
  uint32_t cur = 0;
  // this lane's pair id of the batch about to be staged, loaded one batch ahead
  uint32_t g_next = range.x + lane < range.y ? pair_gid[range.x + lane] : 0u;
  for (uint32_t start = range.x; start < range.y; start += 64) {
    if (__ballot(live) == 0ull) break;
    if (split && start != range.x && (start - range.x) % GS3_SEG == 0) {
      seg_px[(int64_t)cur * GS3_BLOCK] = make_float4(T, C0, C1, C2);
      E0 += C0;
      E1 += C1;
      E2 += C2;
      C0 = C1 = C2 = 0.f;
      ++cur;
    }
    const uint32_t i = start + lane;
    // kept splats compacted to the front of the slice, as in the forward
    bool keep = false;
    float4 ra = make_float4(0.f, 0.f, 0.f, 0.f), rb = ra, rc = ra, qa = ra, qb = ra;
    float qc = 0.f;
    if (i < range.y) {
      const Rec r = rec[g_next];
      const TRec q = trec[g_next];
      ra = r.a;
      rb = r.b;
      rc = r.c;
      qa = q.a;
      qb = q.b;
      qc = q.c.x;
      keep = cull_keep(cull_setup(r.a, r.b, r.c.y, tx, ty), w);
    }
    if (i + 64 < range.y) g_next = pair_gid[i + 64];
    const uint64_t kb = __ballot(keep);
    const int cnt = __builtin_popcountll(kb);
    if (keep) {
      const int pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(kb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)kb, 0u));
      s.a[pos] = ra;
      s.b[pos] = rb;
      s.ta[pos] = qa;
      s.tb[pos] = qb;
      s.c[pos] = make_float4(rc.x, rc.y, qc, __uint_as_float(i + 1u));
    }
    wave_lds_sync();
    // one walked splat; `valid` false: no splat (the odd slot of a pair)
    auto walk = [&](const float4 A, const float4 B, const float4 Cc, const float4 TA, const float4 TB,
                    const bool valid) {
      if (COUNT) nev += valid ? live : 0u;
      const float dx = A.x - pxf, dy = A.y - pyf;
      const float power = splat_power(A.z, A.w, B.x, dx, dy);
      const bool pass = valid && live && power <= 0.f && power >= Cc.y;
      const float G = __expf(power);
      const float araw = B.y * G;
      const float a = fminf(GS3_ALPHA_MAX, araw);
      const float Tn = T * (1.f - a);
      const bool stop = pass && Tn < GS3_T_STOP;
      const bool use = pass && !stop;
      live = stop ? 0u : live;
      if (COUNT) ncon += use ? 1u : 0u;
      // d power along the tangent: d = (u - px, v - py), dd = (du, dv); the
      // record holds the pre-scaled conic, the tangent record the plain one
      const float dpow = 2.f * (A.z * dx * TA.x + B.x * dy * TA.y) + A.w * (TA.x * dy + dx * TA.y) -
                         0.5f * (TA.z * dx * dx + TB.x * dy * dy) - TA.w * dx * dy;
      const float da = araw > GS3_ALPHA_MAX ? 0.f : (TB.y * G + B.y * G * dpow);
      const float wt = use ? a * T : 0.f;
      const float dw = use ? da * T + a * dT : 0.f;
      C0 += B.z * wt;
      C1 += B.w * wt;
      C2 += Cc.x * wt;
      D0 += TB.z * wt + B.z * dw;
      D1 += TB.w * wt + B.w * dw;
      D2 += Cc.z * wt + Cc.x * dw;
      dT = use ? dT * (1.f - a) - T * da : dT;
      T = use ? Tn : T;
      lastp = use ? __float_as_uint(Cc.w) : lastp;
    };
    // walked in pairs, the next pair's records read one pair ahead (as in
    // the forward)
    if (cnt > 0) {
      float4 A0 = s.a[0], B0 = s.b[0], D0r = s.c[0], P0 = s.ta[0], Q0 = s.tb[0];
      const int f1 = min(1, cnt - 1);
      float4 A1 = s.a[f1], B1 = s.b[f1], D1r = s.c[f1], P1 = s.ta[f1], Q1 = s.tb[f1];
      float4 A2, B2, D2r, P2, Q2, A3, B3, D3r, P3, Q3;
      for (int j = 0;;) {
        const int n2 = min(j + 2, cnt - 1), n3 = min(j + 3, cnt - 1);
        A2 = s.a[n2];
        B2 = s.b[n2];
        D2r = s.c[n2];
        P2 = s.ta[n2];
        Q2 = s.tb[n2];
        A3 = s.a[n3];
        B3 = s.b[n3];
        D3r = s.c[n3];
        P3 = s.ta[n3];
        Q3 = s.tb[n3];
        __builtin_amdgcn_sched_barrier(0);
        walk(A0, B0, D0r, P0, Q0, true);
        walk(A1, B1, D1r, P1, Q1, j + 1 < cnt);
        j += 2;
        if (j >= cnt || __ballot(live) == 0ull) break;
        const int n0 = min(j + 2, cnt - 1), n1 = min(j + 3, cnt - 1);
        A0 = s.a[n0];
        B0 = s.b[n0];
        D0r = s.c[n0];
        P0 = s.ta[n0];
        Q0 = s.tb[n0];
        A1 = s.a[n1];
        B1 = s.b[n1];
        D1r = s.c[n1];
        P1 = s.ta[n1];
        Q1 = s.tb[n1];
        __builtin_amdgcn_sched_barrier(0);
        walk(A2, B2, D2r, P2, Q2, true);
        walk(A3, B3, D3r, P3, Q3, j + 1 < cnt);
        j += 2;
        if (j >= cnt || __ballot(live) == 0ull) break;
      }
    }
    wave_lds_sync();
  }
  if (split) seg_px[(int64_t)cur * GS3_BLOCK] = make_float4(T, C0, C1, C2);
  if (inside) {
    pix_last[(int64_t)py * cam.width + px] = lastp;
    pix_T[(int64_t)py * cam.width + px] = T;
    const int64_t o = ((int64_t)py * cam.width + px) * 3;
    img[o + 0] = (E0 + C0) + T * bg0;
    img[o + 1] = (E1 + C1) + T * bg1;
    img[o + 2] = (E2 + C2) + T * bg2;
    tan_img[o + 0] = D0 + dT * bg0;
    tan_img[o + 1] = D1 + dT * bg1;
    tan_img[o + 2] = D2 + dT * bg2;
  }
  count_evals<COUNT>(ctr, nev, ncon);
}

// Data-parallel-primitive (DPP) move: lane i reads `v` from the lane selected
// by CTRL; lanes without a source read 0.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}

// Transposed reduction helpers (gfx950 permlane swaps).  fold32(a, b): lane
// i < 32 gets a[i] + a[i+32], lane i >= 32 gets b[i-32] + b[i].  fold16(a, b):
// with rows of 16 lanes, row pairs (0,1) and (2,3) are summed and the result
// rows are [a01, b01, a23, b23].
__device__ __forceinline__ float fold32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float fold16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// fold8(a, b): within each 16-lane row, lanes 0-7 get a[l] + a[l+8] and
// lanes 8-15 get b[l-8] + b[l] (a rotation by 8 within the row, then a
// select on lane bit 3).
__device__ __forceinline__ float fold8(float a, float b, bool hi8) {
  const float ra = a + dpp_move<0x128>(a), rb = b + dpp_move<0x128>(b);
  return hi8 ? rb : ra;
}
// Inclusive scan over 8 lanes within each 16-lane row (row_shr 1, 2, 4;
// lanes shifted in from below the row read 0): lane 7 of a row holds the sum
// of its lanes 0-7, lane 15 the sum of its lanes 8-15.
__device__ __forceinline__ float half_row_sum(float v) {
  v += dpp_move<0x111>(v);
  v += dpp_move<0x112>(v);
  v += dpp_move<0x114>(v);
  return v;
}

// The backward stages 128 splats per batch: with the per-wave partial sums
// this keeps the workgroup at ~24 KB of LDS (six workgroups per CU).
constexpr int kBwdBatch = 128;
struct StageB {
  float4 a[kBwdBatch];
  float4 b[kBwdBatch];
  float2 c[kBwdBatch];  // b, tau
  uint32_t first[kBwdBatch];  // the Gaussian's first pair
  uint32_t cnt[kBwdBatch];    // its tile count
  uint2 rc[kBwdBatch];        // its tile rectangle
  float red[4][9][kBwdBatch];
  uint64_t bits[4][kBwdBatch / 64];
};


template <bool COUNT>
__device__ __forceinline__ void blend_bwd_body(const Rec* __restrict__ rec, const uint2* __restrict__ rect,
                                               const uint32_t* __restrict__ tiles,
                                               const uint32_t* __restrict__ rowtab,
                                               const uint32_t* __restrict__ pair_gid,
                                               const uint2* __restrict__ ranges, const uint2* __restrict__ units,
                                               const CamDev& cam, const uint32_t* __restrict__ pix_last,
                                               const float* __restrict__ pix_T, const float4* __restrict__ seg,
                                               float bg0, float bg1, float bg2, const float* __restrict__ cot,
                                               float* __restrict__ partials, uint32_t* __restrict__ valid,
                                               int n_tiles, int bid, unsigned long long* __restrict__ ctr) {
  const uint2 unit = units[bid];
  const int t = (int)__builtin_amdgcn_readfirstlane(unit.x);
  if (t >= n_tiles) return;
  const uint32_t m = __builtin_amdgcn_readfirstlane(unit.y);  // depth segment of the tile's list
  __shared__ StageB s;
  __shared__ uint32_t tile_end;
  uint32_t nev = 0, ncon = 0;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int tx = t % cam.tiles_x, ty = t / cam.tiles_x;
  const int px = pixel_x(tx, tid), py = pixel_y(ty, tid);
  const bool inside = px < cam.width && py < cam.height;
  const float pxf = (float)px + 0.5f, pyf = (float)py + 0.5f;
  const uint2 range = uniform_range(ranges, t);
  // this workgroup's pairs [lo, hi): segment m of the tile's list
  const uint32_t lo = range.x + m * GS3_SEG, hi = min(range.y, lo + GS3_SEG);
  float g0 = 0.f, g1 = 0.f, g2 = 0.f, T = 1.f, acc = 0.f;
  uint32_t last = 0u;  // 1 + pair index of the pixel's last contributing splat (0: none)
  if (inside) {
    const int64_t pix = (int64_t)py * cam.width + px;
    g0 = cot[pix * 3 + 0];
    g1 = cot[pix * 3 + 1];
    g2 = cot[pix * 3 + 2];
    last = pix_last[pix];
    T = pix_T[pix];
    // (sum over the contributing splats behind the current one of c w +
    // T_final bg) . dL/dC, accumulated from the back
    acc = T * (bg0 * g0 + bg1 * g1 + bg2 * g2);
    // the pixel's last contribution lies in a later segment k: start from
    // the transmittance after segment m and add the colour of segments
    // m+1..k (segments after k add nothing for this pixel)
    const uint32_t k = last > range.x ? (last - 1u - range.x) / GS3_SEG : 0u;
    if (range.y - range.x > GS3_SEG && k > m) {
      const float4* sp = seg + ((int64_t)t + range.x / GS3_SEG) * GS3_BLOCK + tid;
      T = sp[(int64_t)m * GS3_BLOCK].x;
      for (uint32_t q = m + 1u; q <= k; ++q) {
        const float4 v = sp[(int64_t)q * GS3_BLOCK];
        acc += v.y * g0 + v.z * g1 + v.w * g2;
      }
    }
  }
  if (tid == 0) tile_end = 0u;
  __syncthreads();
  if (last > 0u) atomicMax(&tile_end, last);
  __syncthreads();
  // pairs at or after the tile's last contribution get no partials (their
  // valid bits stay clear) and are not staged at all; at city scale most
  // pairs of a tile lie behind its last contribution
  const uint32_t end = min(max(tile_end, lo), hi);
  // where this lane's wave sums land in the reduction rows (lanes 7 and 15
  // of each 16-lane row; see the reduction in the walk)
  const bool hi8 = (lane & 8) != 0;
  float* red_w = &s.red[w][0][0];
  const int red_lane = (((lane >> 4) & 1) * 2 + (lane >> 5) + (hi8 ? 4 : 0)) * kBwdBatch;
  // the wave's own last contribution bounds the splats it walks
  uint32_t wave_end = last;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) wave_end = max(wave_end, (uint32_t)__shfl_xor((int)wave_end, m, 64));
  wave_end = __builtin_amdgcn_readfirstlane(wave_end);
  if (end > lo) {
    for (int64_t bstart = lo + (int64_t)((end - 1 - lo) / kBwdBatch) * kBwdBatch; bstart >= lo;
         bstart -= kBwdBatch) {
      const int cnt = (int)min((int64_t)kBwdBatch, (int64_t)end - bstart);
      const int64_t i = bstart + tid;
      if (tid < kBwdBatch) {
        uint32_t m = 0u;
        if (tid < cnt) {
          const uint32_t g = pair_gid[i];
          const Rec r = rec[g];
          s.a[tid] = r.a;
          s.b[tid] = r.b;
          s.c[tid] = make_float2(r.c.x, r.c.y);
          s.first[tid] = __float_as_uint(r.c.z);
          s.cnt[tid] = tiles[g];
          s.rc[tid] = rect[g];
          m = block_mask(r.a, r.b, r.c.y, tx, ty);
        }
        publish_masks(s.bits, m, tid);
      }
      __syncthreads();
      const int nwords = (cnt + 63) >> 6;
      // splats of this batch at or after the wave's last contribution add nothing for it
      const int64_t lim = (int64_t)wave_end - bstart;  // walk j < lim
      for (int q = nwords - 1; q >= 0; --q) {
        const int64_t lq = lim - 64 * q;
        const uint64_t keep = lq >= 64 ? ~0ull : (lq <= 0 ? 0ull : ((1ull << lq) - 1ull));
        const uint64_t word = uniform64(s.bits[w][q]);
        uint64_t bits = word & keep;
        uint64_t reduced = bits;  // less the splats no lane of the wave uses
        // one walked splat: j its index in the batch, hi its bit in the word
        auto walk = [&](const float4 A, const float4 B, const float2 Cc, const int hi) {
          const int j = (q << 6) + hi;
          const uint32_t pi = (uint32_t)bstart + (uint32_t)j;
          const float dx = A.x - pxf, dy = A.y - pyf;
          const float power = splat_power(A.z, A.w, B.x, dx, dy);
          // predicated like the forward: lanes that do not contribute end
          // with zero partials and unchanged T and acc
          const bool use = pi < last && power <= 0.f && power >= Cc.y;
          if (COUNT) {
            nev += pi < last ? 1u : 0u;
            ncon += use ? 1u : 0u;
          }
          const float G = __expf(power);
          const float araw = B.y * G;
          const float a = fminf(GS3_ALPHA_MAX, araw);
          const float r1 = __builtin_amdgcn_rcpf(1.f - a);
          const float Tb = T * r1;  // transmittance in front of this splat
          const float cdot = B.z * g0 + B.w * g1 + Cc.x * g2;
          const float wgt = use ? a * Tb : 0.f;
          const float dL_da = Tb * cdot - acc * r1;
          const bool open = use && araw <= GS3_ALPHA_MAX;  // the 0.99 clamp passes no gradient
          // dL/dopacity; dL/dpower is opacity times it, and that factor is
          // applied once per splat after the reduction
          const float h = open ? G * dL_da : 0.f;
          const float pt = h * dx, pu = h * dy;
          float gr[9];
          gr[0] = pt;
          gr[1] = pu;
          gr[2] = pt * dx;
          gr[3] = pt * dy;
          gr[4] = pu * dy;
          gr[5] = h;
          gr[6] = wgt * g0;
          gr[7] = wgt * g1;
          gr[8] = wgt * g2;
          acc += wgt * cdot;
          T = use ? Tb : T;
          // wave sums of the 9 partial derivatives, transposed: values 0-7
          // are folded in pairs across half-waves, row pairs and half-rows,
          // leaving in row r value k(r) = {0,2,1,3}[r] in lanes 0-7 and value
          // 4 + k(r) in lanes 8-15, each then summed into lane 7 and lane 15;
          // value 8 (folded with zeros) ends summed in lane 7 of row 0.
          if (__ballot(use) != 0ull) {
            const float E = fold16(fold32(gr[0], gr[1]), fold32(gr[2], gr[3]));
            const float F = fold16(fold32(gr[4], gr[5]), fold32(gr[6], gr[7]));
            const float M = half_row_sum(fold8(E, F, hi8));
            const float H = half_row_sum(fold8(fold16(fold32(gr[8], 0.f), 0.f), 0.f, false));
            if ((lane & 7) == 7) {
              red_w[red_lane + j] = M;
              if (lane == 7) s.red[w][8][j] = H;
            }
          } else {
            reduced &= ~(1ull << hi);
          }
        };
        // each splat's record is read from LDS one step ahead, into the other
        // of two register sets
        if (bits) {
          int h0 = 63 - __builtin_clzll(bits), h1 = 0;
          float4 A0 = s.a[(q << 6) + h0], B0 = s.b[(q << 6) + h0], A1, B1;
          float2 C0 = s.c[(q << 6) + h0], C1;
          while (true) {
            bits &= ~(1ull << h0);
            h1 = bits ? 63 - __builtin_clzll(bits) : h0;
            A1 = s.a[(q << 6) + h1];
            B1 = s.b[(q << 6) + h1];
            C1 = s.c[(q << 6) + h1];
            walk(A0, B0, C0, h0);
            if (!bits) break;
            bits &= ~(1ull << h1);
            h0 = bits ? 63 - __builtin_clzll(bits) : h1;
            A0 = s.a[(q << 6) + h0];
            B0 = s.b[(q << 6) + h0];
            C0 = s.c[(q << 6) + h0];
            walk(A1, B1, C1, h1);
            if (!bits) break;
          }
        }
        // the epilogue counts the splats this wave did not reduce as zero
        if (reduced != word && lane == 0) s.bits[w][q] = reduced;
      }
      __syncthreads();
      const uint64_t bit = 1ull << (tid & 63);
      const bool h0 = tid < cnt && (s.bits[0][tid >> 6] & bit), h1 = tid < cnt && (s.bits[1][tid >> 6] & bit);
      const bool h2 = tid < cnt && (s.bits[2][tid >> 6] & bit), h3 = tid < cnt && (s.bits[3][tid >> 6] & bit);
      // a pair no wave used keeps no partials: its valid bit stays clear and
      // the pair sums skip it (every other pair's bit is set with its store)
      if (h0 || h1 || h2 || h3) {
        // the pair's slot in the Gaussian-contiguous partials: the
        // Gaussian's first pair plus the tile's index in its tile list,
        // from the row's entry (or, without one, a walk over the rows)
        const uint32_t first = s.first[tid];
        const uint2 rc = s.rc[tid];
        const int row_off = ty - (int)(rc.x >> 16);
        uint32_t idx;
        if (row_entry_kept(row_off, s.cnt[tid])) {
          const uint32_t e = rowtab[first + (uint32_t)row_off];
          idx = (e & 0xffffu) + (uint32_t)(tx - (int)(e >> 16));
        } else {
          const Rec rr{s.a[tid], s.b[tid], make_float4(s.c[tid].x, s.c[tid].y, 0.f, 0.f)};
          idx = splat_tile_index(splat_rows_of(rr, rc), tx, ty);
        }
        const uint32_t slot = first + idx;
        // a wave that skipped the splat contributes exactly zero
        float* dst = partials + (int64_t)slot * 9;
        atomicOr(valid + (slot >> 5), 1u << (slot & 31));
        float R[9];
#pragma unroll
        for (int k = 0; k < 9; ++k)
          R[k] = (((h0 ? s.red[0][k][tid] : 0.f) + (h1 ? s.red[1][k][tid] : 0.f)) + (h2 ? s.red[2][k][tid] : 0.f)) +
                 (h3 ? s.red[3][k][tid] : 0.f);
        // power = qa dx^2 + qc dy^2 + qb dx dy, (qa, qb, qc) = (-a/2, -b, -c/2),
        // dx = u - px, dy = v - py; R[0..4] still lack the opacity factor
        const float qa = s.a[tid].z, qb = s.a[tid].w, qc = s.b[tid].x, op = s.b[tid].y;
        const float R0 = op * R[0], R1 = op * R[1];
        dst[0] = 2.f * qa * R0 + qb * R1;
        dst[1] = 2.f * qc * R1 + qb * R0;
        dst[2] = (-0.5f * op) * R[2];
        dst[3] = -op * R[3];
        dst[4] = (-0.5f * op) * R[4];
#pragma unroll
        for (int k = 5; k < 9; ++k) dst[k] = R[k];
      }
      __syncthreads();
    }
  }
  count_evals<COUNT>(ctr, nev, ncon);
}

// Views of one launch: workgroup b works for view b mod n on that view's
// block b / n (views interleaved, so every view's longest tiles start early),
// and returns at once past the view's own block count.
__device__ __forceinline__ bool view_of_block(const BlendBatch& B, int& v, int& local) {
  v = (int)(blockIdx.x % (unsigned)B.n);
  local = (int)(blockIdx.x / (unsigned)B.n);
  return local < B.v[v].blocks;
}

template <bool COUNT>
__global__ __launch_bounds__(GS3_BLOCK) void k_blend_fwd(BlendBatch B, float bg0, float bg1, float bg2,
                                                          unsigned long long* __restrict__ ctr) {
  int v, b;
  if (!view_of_block(B, v, b)) return;
  const BlendView& V = B.v[v];
  blend_fwd_body<COUNT>(V.rec, V.pair_gid, V.ranges, V.order, V.cam, bg0, bg1, bg2, V.img, V.pix_last, V.pix_T,
                        V.seg, V.n_tiles, V.chunk, b, ctr);
}

template <bool COUNT>
__global__ __launch_bounds__(GS3_BLOCK) void k_blend_jvp(BlendBatch B, float bg0, float bg1, float bg2,
                                                          unsigned long long* __restrict__ ctr) {
  int v, b;
  if (!view_of_block(B, v, b)) return;
  const BlendView& V = B.v[v];
  blend_jvp_body<COUNT>(V.rec, V.trec, V.pair_gid, V.ranges, V.order, V.cam, bg0, bg1, bg2, V.img, V.tan_img,
                        V.pix_last, V.pix_T, V.seg, V.n_tiles, V.chunk, b, ctr);
}

template <bool COUNT>
__global__ __launch_bounds__(GS3_BLOCK) void k_blend_bwd(BlendBatch B, float bg0, float bg1, float bg2,
                                                          unsigned long long* __restrict__ ctr) {
  int v, b;
  if (!view_of_block(B, v, b)) return;
  const BlendView& V = B.v[v];
  blend_bwd_body<COUNT>(V.rec, V.rect, V.tiles, V.rowtab, V.pair_gid, V.ranges, V.units, V.cam, V.pix_last, V.pix_T,
                        V.seg, bg0, bg1, bg2, V.cot, V.partials, V.valid, V.n_tiles, b, ctr);
}

inline int chunk_for(int n_tiles) { return (n_tiles + 7) / 8; }

// Fills the per-launch fields of each view (block counts) and the grid.
unsigned batch_grid(BlendBatch& B, int kind) {
  int span = 0;
  for (int v = 0; v < B.n; ++v) {
    BlendView& V = B.v[v];
    V.chunk = chunk_for(V.n_tiles);
    V.blocks = kind == 2 ? (int)V.n_units : (V.order ? V.n_tiles : 8 * V.chunk);
    span = std::max(span, V.blocks);
  }
  return (unsigned)span * (unsigned)B.n;
}

}  // namespace

void launch_blend_fwd(BlendBatch B, const float* bg, hipStream_t st, unsigned long long* ctr) {
  const unsigned grid = batch_grid(B, 0);
  if (grid == 0) return;
  auto kernel = ctr ? k_blend_fwd<true> : k_blend_fwd<false>;
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(GS3_BLOCK), 0, st, B, bg[0], bg[1], bg[2], ctr);
}

void launch_blend_jvp(BlendBatch B, const float* bg, hipStream_t st, unsigned long long* ctr) {
  const unsigned grid = batch_grid(B, 1);
  if (grid == 0) return;
  auto kernel = ctr ? k_blend_jvp<true> : k_blend_jvp<false>;
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(GS3_BLOCK), 0, st, B, bg[0], bg[1], bg[2], ctr);
}

void launch_blend_bwd(BlendBatch B, const float* bg, hipStream_t st, unsigned long long* ctr) {
  const unsigned grid = batch_grid(B, 2);
  if (grid == 0) return;
  auto kernel = ctr ? k_blend_bwd<true> : k_blend_bwd<false>;
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(GS3_BLOCK), 0, st, B, bg[0], bg[1], bg[2], ctr);
}
