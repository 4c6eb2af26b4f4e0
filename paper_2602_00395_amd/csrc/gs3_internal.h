// Internal declarations shared by the gfx950 kernels and the host library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GS3_TILE 16
// measurement counters of one profiled launch are spread over this many
// (evaluations, contributions) pairs, so the waves' atomics do not all hit
// one address
#define GS3_PROF_SUB 64
#define GS3_BLOCK (GS3_TILE * GS3_TILE)
// depth segment of a tile's pair list processed by one backward workgroup
// (a multiple of the backward's 128-splat batch)
#define GS3_SEG 256
// views (or probes) one blend or projection-backward launch covers
#define GS3_MAX_VIEWS 8

// Rasteriser constants of the original 3DGS design (the paper states only the
// blend equation): near plane, screen-space dilation, frustum clamp of the
// EWA Jacobian, opacity clamp and skip threshold, transmittance stop.
#define GS3_NEAR 0.2f
#define GS3_DILATION 0.3f
#define GS3_FOV_CLAMP 1.3f
#define GS3_ALPHA_MAX 0.99f
#define GS3_ALPHA_MIN (1.0f / 255.0f)
#define GS3_T_STOP 1e-4f
// Gauss-Newton weight floor and colour floor of the trust region.
#define GS3_GN_FLOOR 1e-6f
#define GS3_COLOUR_FLOOR (1.0f / 255.0f)

struct CamDev {
  float W[9];
  float t[3];
  float fx, fy, cx, cy;
  float limx, limy;
  float campos[3];
  int width, height, tiles_x, tiles_y;
};

// Per-Gaussian screen-space record, 12 words (three float4):
//   {u, v, qa, qb}, {qc, opacity, r, g}, {b, tau, pair_off, clamp}
// clamp: bit c set where colour channel c is unclamped (its bits, not a float)
// with the conic stored pre-scaled, qa = -a/2, qb = -b, qc = -c/2, so that
// power = (qa dx) dx + (qc dy) dy + (qb dx) dy -- bit for bit the float32
// value of -1/2 ((a dx) dx + (c dy) dy) - (b dx) dy, since scaling by powers of
// two commutes with rounding.
// tau = float32(-ln(255 opacity)): a splat is skipped at a pixel where its
// float32 power is below tau (equivalently opacity exp(power) < 1/255).
// The tile rectangle lives in a separate uint2 array:
//   x = x0 | y0 << 16, y = x1 | y1 << 16 (half-open).
struct __align__(16) Rec {
  float4 a, b, c;
};

// Tile list of a splat.  A splat is paired with the tiles of its rectangle
// whose 16x16 block of pixel centres meets the widened skip ellipse
//   E = {d : d^T Q d <= k},  Q = (a, b; b, c) = (-2 qa, -qb; -qb, -2 qc),
//   k = 2.02 (-tau) + 1e-3,
// from the float32 conic and threshold of its record.  The skip test can
// pass only where d^T Q d <= -2 tau (1 + r), r <= 1e-3 the relative rounding
// error of the float32 power for rho^2 = b^2 / (a c) <= 0.999; the further
// 0.9% of k and a 0.01-pixel margin on every edge below cover the rounding
// of the float32 evaluation of the extent (relative errors of a few 1e-4 at
// most near the top and bottom of E).  So every pixel the splat reaches lies
// in a listed tile, and the render and its derivatives are those of the
// whole rectangle.  A splat with rho^2 > 0.999 or a conic that is not
// positive definite or finite keeps its whole rectangle; tau > 0 passes
// nowhere (no tiles).  Row ty of the rectangle holds the columns [lo, hi) of
// tiles that meet E within the band of pixel-centre rows 16 ty + 1/2 ..
// 16 ty + 15.5: the band cuts E in a convex set whose x-extent runs from the
// left end of E at the band's row nearest E's leftmost point to the right
// end at the row nearest its rightmost point.  Every evaluation is in
// float32 without contraction, in one fixed order, so the projection (the
// counts), the emission and the backward (the partials slot) get the same
// spans.  Pairs of a splat go row by row, columns in order.
struct SplatRows {
  int mode;  // 0: no tile, 1: the whole rectangle, 2: the ellipse rows
  int x0, y0, x1, y1;
  float u, v, b, det, ka, inv_a, ymax, yr;
};

__device__ __forceinline__ SplatRows splat_rows(float u, float v, float qa, float qb, float qc, float tau, int x0,
                                                int y0, int x1, int y1) {
#pragma clang fp contract(off)
  SplatRows s;
  s.x0 = x0;
  s.y0 = y0;
  s.x1 = x1;
  s.y1 = y1;
  s.u = u;
  s.v = v;
  if (tau > 0.f) {
    s.mode = 0;
    return s;
  }
  const float a = -2.f * qa, b = -qb, c = -2.f * qc;
  const float det = a * c - b * b;
  s.mode = (a > 0.f && c > 0.f && det * 1000.f >= a * c && det < INFINITY) ? 2 : 1;
  const float k = -2.02f * tau + 1e-3f;
  s.b = b;
  s.det = det;
  s.ka = k * a;
  s.inv_a = 1.f / a;
  s.ymax = sqrtf(s.ka / det);
  // the rightmost point of E is (xm, yr), xm = sqrt(k c / det), yr = -b xm / c;
  // the leftmost is (-xm, -yr)
  s.yr = -b * sqrtf((k * c) / det) / c;
  return s;
}

// Columns [lo, hi) of row ty (lo >= hi: none).
__device__ __forceinline__ void splat_row_span(const SplatRows& s, int ty, int& lo, int& hi) {
#pragma clang fp contract(off)
  if (s.mode != 2) {
    lo = s.x0;
    hi = s.mode == 1 ? s.x1 : s.x0;
    return;
  }
  const float row = 16.f * (float)ty;
  const float ya = fmaxf((row + 0.49f) - s.v, -s.ymax), yb = fminf((row + 15.51f) - s.v, s.ymax);
  if (!(ya <= yb)) {
    lo = hi = s.x0;
    return;
  }
  const float y_r = fminf(fmaxf(s.yr, ya), yb), y_l = fminf(fmaxf(-s.yr, ya), yb);
  const float xr = (-s.b * y_r + sqrtf(fmaxf(s.ka - (s.det * y_r) * y_r, 0.f))) * s.inv_a;
  const float xl = (-s.b * y_l - sqrtf(fmaxf(s.ka - (s.det * y_l) * y_l, 0.f))) * s.inv_a;
  const float clo = ceilf(((s.u + xl) - 15.51f) * 0.0625f), chi = floorf(((s.u + xr) - 0.49f) * 0.0625f) + 1.f;
  lo = (int)fminf(fmaxf(clo, (float)s.x0), (float)s.x1);
  hi = (int)fmaxf(fminf(chi, (float)s.x1), (float)s.x0);
}

// Number of tiles of the splat and the bounding rectangle of its listed
// tiles [tx0, tx1) x [ty0, ty1) (the splat's own rectangle when every tile is
// listed; empty when none is).  Clipping the rows to that rectangle leaves
// every row's span as it is, so the spans may be taken from either.
__device__ __forceinline__ uint32_t splat_tile_bounds(const SplatRows& s, int& tx0, int& ty0, int& tx1, int& ty1) {
  tx0 = s.x0;
  ty0 = s.y0;
  tx1 = s.x1;
  ty1 = s.y1;
  if (s.mode != 2) return s.mode == 1 ? (uint32_t)((s.x1 - s.x0) * (s.y1 - s.y0)) : 0u;
  uint32_t n = 0;
  int xa = s.x1, xb = s.x0, ya = s.y1, yb = s.y0;
  for (int ty = s.y0; ty < s.y1; ++ty) {
    int lo, hi;
    splat_row_span(s, ty, lo, hi);
    if (hi > lo) {
      n += (uint32_t)(hi - lo);
      xa = min(xa, lo);
      xb = max(xb, hi);
      ya = min(ya, ty);
      yb = ty + 1;
    }
  }
  if (n) {
    tx0 = xa;
    tx1 = xb;
    ty0 = ya;
    ty1 = yb;
  }
  return n;
}

// Index of tile (tx, ty) among the splat's tiles (the tile is listed).
__device__ __forceinline__ uint32_t splat_tile_index(const SplatRows& s, int tx, int ty) {
  if (s.mode != 2) return (uint32_t)((ty - s.y0) * (s.x1 - s.x0) + (tx - s.x0));
  uint32_t n = 0;
  for (int r = s.y0; r < ty; ++r) {
    int lo, hi;
    splat_row_span(s, r, lo, hi);
    n += hi > lo ? (uint32_t)(hi - lo) : 0u;
  }
  int lo, hi;
  splat_row_span(s, ty, lo, hi);
  return n + (uint32_t)(tx - lo);
}

// Row entries of the tile lists, written by the emission and read by the
// backward in place of a row walk.  A Gaussian whose pairs take the slots
// [first, first + count) and whose stored rectangle starts at row y0 has, at
// rowtab[first + ty - y0], for each row ty of its list with pairs: the
// number of its pairs in the rows before ty (low 16 bits) and the row's
// first column (high 16 bits) -- kept only where ty - y0 < count and count
// fits 16 bits, so an entry stays inside the Gaussian's own slots (the rows
// of a list are the rows a convex ellipse reaches, contiguous in practice,
// but a float32 row span might still come out empty).
__device__ __forceinline__ bool row_entry_kept(int row_off, uint32_t count) {
  return row_off >= 0 && (uint32_t)row_off < count && count <= 0xffffu;
}
__device__ __forceinline__ uint32_t row_entry(uint32_t before, int first_col) {
  return before | ((uint32_t)first_col << 16);
}

__device__ __forceinline__ SplatRows splat_rows_of(const Rec& r, uint2 rc) {
  return splat_rows(r.a.x, r.a.y, r.a.z, r.a.w, r.b.x, r.c.y, (int)(rc.x & 0xffff), (int)(rc.x >> 16),
                    (int)(rc.y & 0xffff), (int)(rc.y >> 16));
}

// Tangent of the record under a parameter-space direction, 12 words:
//   {du, dv, dconic_a, dconic_b}, {dconic_c, dopacity, dr, dg}, {db, 0, 0, 0}
struct __align__(16) TRec {
  float4 a, b, c;
};

enum ProbeKind { PROBE_NONE = 0, PROBE_HASH = 1, PROBE_ARRAY = 2 };

// --------------------------------------------------------------------------
// launchers (all asynchronous on `st`)

// projection: records + depth keys + tiles touched; culled Gaussians get
// key 0xffffffff and zero tiles; vis_count[b] = the number of visible
// Gaussians among 64 b .. 64 b + 63.
void launch_project_fwd(const float* x, int64_t n, int deg, const CamDev& cam, Rec* rec, uint2* rect,
                        uint32_t* depth_key, uint32_t* tiles, uint32_t* vis_count, hipStream_t st);
// tangent records for a probe (hash) or a caller tangent array.
void launch_project_jvp(const float* x, int64_t n, int deg, const CamDev& cam, const Rec* rec,
                        const uint32_t* tiles, int probe_kind, uint64_t seed, uint32_t probe_index,
                        const float* tangent, TRec* trec, hipStream_t st);
// the update of Algorithm 1: EMA decays, budget, whether this is a
// Hutchinson iteration, radius variant
struct TrArgs {
  float theta1, theta2, epsilon;
  int hutch;
  uint32_t variant;  // GS3_TR_* bits
};
// the trust-region update fused into the projection backward (mode 2): the
// summed gradient of a row is gacc (nullable) plus this view's part; the
// update of Algorithm 1 writes x_out (x itself is only read), ghat, dhat
struct FusedTr {
  float* x_out = nullptr;
  float* ghat = nullptr;
  float* dhat = nullptr;
  const float* D = nullptr;
  const float* gacc = nullptr;
  uint32_t* nonfinite = nullptr;  // pinned host word set to 1 by a non-finite gradient or parameter
  TrArgs a{};
};
// Sum of each Gaussian's per-(Gaussian, tile) backward partials: order /
// offsets / counts are the view's depth order, first pair and tile count per
// depth rank; gsum: float[n][9] (a Gaussian's nine values contiguous).
// valid: bit per slot, set where the backward wrote the slot's partials
// (the others count as zeros and are never read).
void launch_pair_sums(const uint32_t* order, const uint32_t* offsets, const uint32_t* counts, const float* partials,
                      const uint32_t* valid, int64_t n, const uint32_t* n_dev, float* gsum, hipStream_t st);
// One view (or one probe of a view) of a projection-backward batch: its
// records, tile counts (0: the view does not see the Gaussian), summed
// partials and camera; `inner` is the probe's key (probe_key) in mode 1.
struct BwdView {
  const Rec* rec = nullptr;
  const uint32_t* tiles = nullptr;
  const float* G = nullptr;
  CamDev cam{};
  uint64_t inner = 0;
};
struct BwdBatch {
  BwdView v[GS3_MAX_VIEWS];
  int n = 0;
  // mode 2: the last n_probe entries are Hutchinson probes whose D_t (scale
  // probe_scale) the update takes in place of FusedTr::D
  int n_probe = 0;
  float probe_scale = 0.f;
};
// Key of probe i of `seed` (the inner SplitMix64 of the probe definition).
uint64_t probe_key(uint64_t seed, uint32_t probe_index);
// Chain rule from each view's gsum to the raw parameters, summed over the
// views of B.  mode 0: out = (accumulate ? out : 0) + dL/dx; mode 1: out +=
// scale sum_i z_i dL_i/dx for the probes of B's entries (Gaussians no entry
// sees untouched); mode 2: the fused update described by ft, its gradient
// from the first B.n - B.n_probe entries and, when B.n_probe > 0, its D_t
// from the rest (ft.D unused).
void launch_project_bwd(const float* x, int64_t n, int deg, const BwdBatch& B, int mode, int accumulate, float scale,
                        float* out, const FusedTr& ft, hipStream_t st);

// sorting and binning
size_t radix_temp_bytes(int64_t n);
// Stable LSD radix sort of n (key, value) pairs on the low `bits` key bits
// (8 per pass).  The first pass reads (keys_in, vals_in) -- vals_in null means
// value = index -- and passes alternate between (ka, va) and (kb, vb), so
// keys_in must not alias ka; *keys_out / *vals_out name the result buffers.
void radix_sort_u32(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* ka, uint32_t* va, uint32_t* kb,
                    uint32_t* vb, int64_t n, int bits, void* temp, hipStream_t st, uint32_t** keys_out,
                    uint32_t** vals_out);
// Depth order of a view's n Gaussians: the visible ones (key not
// 0xffffffff) stably sorted by depth key, then the culled ones in index order
// -- the order a stable sort of all n keys gives -- with only the visible
// ones sorted.  vis_count: the projection's per-64 visible counts; vis_off
// (ceil(n / 64) entries) and *visible (their total) are written; scan_temp
// as for scan_exclusive_u32 over ceil(n / 64) items; (ka, va), (kb, vb):
// n-element scratch; radix_temp: radix_temp_bytes(n).  *order names the
// buffer holding the order (vb).
void depth_order(const uint32_t* depth_key, int64_t n, const uint32_t* vis_count, uint32_t* vis_off,
                 uint32_t* visible, void* scan_temp, uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb,
                 void* radix_temp, hipStream_t st, uint32_t** order);
size_t scan_temp_bytes(int64_t n);
// owner (nullable): owner[b] = the item whose output range holds element
// 256 b of the expanded sequence, for b < owner_blocks.  total_host
// (nullable): pinned host word that receives the total as soon as it is
// known (before the last kernel of the scan ends)
// n_dev (nullable): the item count is *n_dev <= n, known on the device only.
void scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, void* temp, hipStream_t st,
                        uint32_t* owner = nullptr, int64_t owner_blocks = 0, uint32_t* total_host = nullptr,
                        const uint32_t* n_dev = nullptr);
// counts_sorted[i] = tiles[order[i]] for i < n (or *n_dev)
void launch_gather_counts(const uint32_t* order, const uint32_t* tiles, int64_t n, const uint32_t* n_dev,
                          uint32_t* counts_sorted, hipStream_t st);
// writes each visible Gaussian's pair offset into its record (rec.c.z);
// owner (nullable, from scan_exclusive_u32) names the first pair's item of
// each 256-pair block b < owner_blocks, the others search the offsets
// rowtab: the row entries of the tile lists (row_entry), n_pairs words
void launch_emit_pairs(const uint32_t* order, const uint32_t* offsets_sorted, const uint32_t* owner,
                       int64_t owner_blocks, Rec* rec, const uint2* rect, int64_t n, const uint32_t* n_dev,
                       int64_t n_pairs, int tiles_x, uint32_t* pair_tile, uint32_t* pair_gid, uint32_t* rowtab,
                       hipStream_t st);
void launch_tile_ranges(const uint32_t* pair_tile, int64_t n_pairs, uint2* ranges, int n_tiles, hipStream_t st);
// Tile ids in (approximately) descending order of their pair count, and the
// backward's work units: each non-empty tile's list cut into depth segments
// of GS3_SEG pairs, unit = (tile, segment), also longest first; entries from
// the unit count up to n_units hold (n_tiles, 0).  n_units must be at least
// n_tiles + n_pairs / GS3_SEG + 1.
bool launch_tile_order(const uint2* ranges, int n_tiles, uint32_t* order, uint2* units, int64_t n_units,
                       hipStream_t st);
void launch_make_keys(const uint32_t* pair_tile, const uint32_t* pair_gid, const uint32_t* depth_key,
                      int64_t n_pairs, uint64_t* keys, hipStream_t st);

// blending
// A blend launch covers up to GS3_MAX_VIEWS views (several views of a
// mini-batch, or several Hutchinson probes of one view, in one launch).  Per
// view:
// order (nullable): tile processed by the view's workgroup b is order[b]
// (longest list first); NULL = XCD-banded order.
// pix_last / pix_T (float[H][W] each): 1 + pair index of each pixel's last
// contributing splat (0: none) and its final transmittance, written by the
// forward (or the JVP) and read by the backward.
// seg (float4[seg_slots(n_tiles, n_pairs)][256]): for tiles of more than
// GS3_SEG pairs, per depth segment m and pixel of the tile, the transmittance
// after the segment and the colour the segment added, at row
// t + ranges[t].x / GS3_SEG + m; written by the forward (or the JVP) for the
// segments its pixels reach, read by the backward's segment units.
// units / n_units: the backward's (tile, segment) units from
// launch_tile_order (one workgroup per unit).
// ctr (nullable): two u64 counters receiving the number of (pixel, splat)
// evaluations and of contributing evaluations (measurement only).
inline int64_t seg_slots(int64_t n_tiles, int64_t n_pairs) { return n_tiles + n_pairs / GS3_SEG + 1; }
struct BlendView {
  const Rec* rec = nullptr;
  const TRec* trec = nullptr;  // JVP
  const uint32_t* pair_gid = nullptr;
  const uint2* ranges = nullptr;
  const uint32_t* order = nullptr;
  const uint2* rect = nullptr;    // backward
  const uint32_t* tiles = nullptr;   // backward: tile count per Gaussian
  const uint32_t* rowtab = nullptr;  // backward: row entries of the tile lists (row_entry)
  const uint2* units = nullptr;   // backward
  int64_t n_units = 0;            // backward
  const float* cot = nullptr;     // backward
  float* partials = nullptr;      // backward
  uint32_t* valid = nullptr;      // backward: bit per partials slot, set where the slot was written
  float* img = nullptr;           // forward, JVP
  float* tan_img = nullptr;       // JVP
  uint32_t* pix_last = nullptr;
  float* pix_T = nullptr;
  float4* seg = nullptr;
  CamDev cam{};
  int n_tiles = 0;
  int chunk = 0, blocks = 0;  // set by the launcher
};
struct BlendBatch {
  BlendView v[GS3_MAX_VIEWS];
  int n = 0;
};
void launch_blend_fwd(BlendBatch views, const float* bg, hipStream_t st, unsigned long long* ctr = nullptr);
void launch_blend_jvp(BlendBatch views, const float* bg, hipStream_t st, unsigned long long* ctr = nullptr);
void launch_blend_bwd(BlendBatch views, const float* bg, hipStream_t st, unsigned long long* ctr = nullptr);

// loss
// cot = scale * d(sum_k l_k)/dC; optional per-block loss partial sums (double).
void launch_loss_grad(const float* img, const float* tgt, int w, int h, float lam, float scale, float* cot,
                      float* ssim_tmp, double* loss_partials, int* n_partials, hipStream_t st);
// cot = scale * sum_k (dl_k/dC)^T w_k, w_k = (dl_k/dC . u) / (4 max(l_k, floor)).
void launch_loss_gn(const float* img, const float* tgt, const float* u, int w, int h, float lam, float scale,
                    float* cot, float* ssim_tmp, hipStream_t st);
size_t ssim_tmp_floats(int w, int h);
void launch_sq_err(const float* img, const float* tgt, int64_t n, double* partials, int* n_partials, hipStream_t st);
void launch_sum_partials(const double* partials, int n, double* out, hipStream_t st);

// optimizer
// nonfinite (nullable): pinned host word that receives 1 where a gradient
// entry or an updated parameter is not finite
void launch_tr_step(float* x, const float* grad, float* ghat, float* dhat, const float* D, int64_t n, int deg,
                    TrArgs a, float* eta_out, float* dx_out, uint32_t* nonfinite, hipStream_t st);
struct AdamArgs {
  float lr_row[64];
  float b1, b2, eps, bc1, bc2;
  float epsilon;  // > 0: clip by the trust-region radius (ADAM-TR)
};
void launch_adam_step(float* x, const float* grad, float* m, float* v, int64_t n, int deg, const AdamArgs& a,
                      uint32_t* nonfinite, hipStream_t st);

// Marks a non-finite value for the host: a system-scope store to a pinned
// host word (several lanes storing the same 1 is harmless).
__device__ __forceinline__ void note_nonfinite(uint32_t* word, float g, float x_new) {
  if (word && !(isfinite(g) && isfinite(x_new))) __hip_atomic_store(word, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
void launch_fill_f32(float* p, int64_t n, float v, hipStream_t st);
void launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);
