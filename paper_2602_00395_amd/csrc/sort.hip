// Tile binning for gfx950: exclusive scan, stable LSD radix sort of 32-bit
// keys with 32-bit values, pair emission and per-tile ranges.
//
// Paper: Background ("Review of Gaussian Splatting") -- splats are bucketed
// per screen tile and blended in depth order; the Introduction notes that this
// order changes discontinuously with the positions.  The required order is
// lexicographic in (tile, float bits of depth, Gaussian index).  Instead of
// one radix sort over 64-bit (tile, depth) keys of every pair, the visible
// Gaussians are sorted once by depth (N elements, 32 key bits), pairs are
// emitted in that order, and the pairs are then stably sorted by tile id
// (ceil(log2 tiles) key bits).  Stability makes the two orders identical and
// moves far fewer bytes: the pair sort needs 2 passes instead of 6.
//
// Radix pass = upsweep (per-block digit histograms), per-digit scan across
// blocks (one workgroup per digit), scatter.  In the scatter each wave64
// ranks its own contiguous run of 256 keys: lanes holding the same digit are
// found with 8 ballots, and a per-wave running count per digit in LDS gives
// each key its rank without any workgroup barrier inside the run; one barrier
// then turns the four waves' counts into output offsets.  No workgroup ever
// waits on another: every kernel is a plain data-parallel launch.  The first
// pass may take its values implicitly as the key's index.
#include <algorithm>

#include "gs3_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;  // scan: items per thread per block
constexpr int kTileItems = kThreads * kItems;
// radix passes: keys per thread (per lane and round) per block -- 4 (1,024
// keys per workgroup) up to kRsBigFrom keys, 16 (4,096) above: large inputs
// then write four times fewer per-block digit counts, and each digit's run
// of a block's output spans about 64 contiguous bytes instead of 16
constexpr int kRsItems = 4;
constexpr int kRsItemsBig = 16;
constexpr int64_t kRsBigFrom = (int64_t)1 << 21;
constexpr int kRsTile = kThreads * kRsItems;
// workgroups per radix launch when the element count is on the device
constexpr int kRsDevGrid = 2048;
constexpr int kRadix = 256;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(v, d, 64);
    if (lane >= d) v += y;
  }
  return v;
}

// Exclusive scan across a 256-thread block; returns the block total in *total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    off += (i < w) ? wsum[i] : 0u;
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

// ---------------------------------------------------------------- scan

// The scan kernels take the item count from n, or from *n_dev when it is not
// null (then blocks past the count return at once).
__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                           const uint32_t* __restrict__ n_dev,
                                                           uint32_t* __restrict__ block_sums) {
  if (n_dev) n = *n_dev;
  if ((int64_t)blockIdx.x * kTileItems >= n) return;
  const int64_t base = (int64_t)blockIdx.x * kTileItems + (int64_t)threadIdx.x * kItems;
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i)
    if (base + i < n) s += in[base + i];
  uint32_t tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// total_host (nullable): pinned host word that also receives the total, with
// a system-scope store (written through to memory; nothing else needs to be
// visible with it), so the host can read it while the rest of
// the scan still runs.  The total is summed in 64 bits (each block sum fits
// 32 bits: a view has fewer than 2^20 tiles); a total of 0xfffffffe or more
// is reported as 0xfffffffe in both words, and the host refuses the view.
__global__ __launch_bounds__(kThreads) void k_scan_top(uint32_t* __restrict__ block_sums, int nb,
                                                        const uint32_t* __restrict__ n_dev,
                                                        uint32_t* __restrict__ total, uint32_t* total_host) {
  if (n_dev) nb = (int)(((int64_t)*n_dev + kTileItems - 1) / kTileItems);
  __shared__ unsigned long long sum64;
  if (threadIdx.x == 0) sum64 = 0ull;
  uint32_t running = 0;
  uint64_t mine = 0;
  for (int base = 0; base < nb; base += kThreads) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < nb ? block_sums[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan(v, &tot);
    if (i < nb) block_sums[i] = running + ex;
    running += tot;
    mine += v;
  }
  atomicAdd(&sum64, (unsigned long long)mine);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t t = sum64 >= 0xfffffffeull ? 0xfffffffeu : (uint32_t)sum64;
    *total = t;
    if (total_host) __hip_atomic_store(total_host, t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// owner (nullable): for every b < owner_blocks with 256 b inside an item's
// output range [out[i], out[i] + in[i]), owner[b] = i -- the item that owns
// element 256 b of the expanded sequence
__global__ __launch_bounds__(kThreads) void k_scan_down(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                         int64_t n, const uint32_t* __restrict__ n_dev,
                                                         const uint32_t* __restrict__ block_sums,
                                                         uint32_t* __restrict__ owner, int64_t owner_blocks) {
  if (n_dev) n = *n_dev;
  if ((int64_t)blockIdx.x * kTileItems >= n) return;
  const int64_t base = (int64_t)blockIdx.x * kTileItems + (int64_t)threadIdx.x * kItems;
  uint32_t v[kItems];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0u;
    s += v[i];
  }
  uint32_t tot;
  uint32_t run = block_excl_scan(s, &tot) + block_sums[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    if (base + i < n) {
      out[base + i] = run;
      if (owner)
        for (int64_t b = ((int64_t)run + 255) >> 8; b < owner_blocks && (b << 8) < (int64_t)run + v[i]; ++b)
          owner[b] = (uint32_t)(base + i);
    }
    run += v[i];
  }
}

// ---------------------------------------------------------------- radix sort

// The radix kernels take the element count from n, or from the device word
// *n_dev when it is not null (a count produced on the device, e.g. the
// visible Gaussians of a view); then the grid may be smaller than the number
// of blocks and each workgroup takes blocks blockIdx.x, + gridDim.x, ...
__device__ __forceinline__ int64_t rs_count(int64_t n, const uint32_t* n_dev) { return n_dev ? (int64_t)*n_dev : n; }

template <int ITEMS>
__global__ __launch_bounds__(kThreads) void k_rs_upsweep(const uint32_t* __restrict__ keys, int64_t n,
                                                          const uint32_t* __restrict__ n_dev, int shift,
                                                          uint32_t* __restrict__ hist, int nb) {
  __shared__ uint32_t h[kRadix];
  n = rs_count(n, n_dev);
  const int live = (int)((n + kThreads * ITEMS - 1) / (kThreads * ITEMS));
  for (int blk = blockIdx.x; blk < live; blk += gridDim.x) {
    // a thread clears its bin only after reading it out for the previous
    // block, and no thread counts into the bins before all have cleared
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blk * (kThreads * ITEMS);
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int64_t i = base + r * kThreads + threadIdx.x;
      if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xffu], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blk] = h[threadIdx.x];
  }
}

// One workgroup per digit: exclusive scan of hist[d][0..nb) in place, 2048
// entries per round (8 consecutive per thread, all loaded before the scan).
constexpr int kRsScanPer = 8;
// With n_dev, only the live blocks' entries of each row (stride nb) count.
__global__ __launch_bounds__(kThreads) void k_rs_scan(uint32_t* __restrict__ hist, int nb,
                                                       const uint32_t* __restrict__ n_dev, int tile,
                                                       uint32_t* __restrict__ digit_total) {
  uint32_t* row = hist + (int64_t)blockIdx.x * nb;
  if (n_dev) nb = (int)(((int64_t)*n_dev + tile - 1) / tile);
  uint32_t running = 0;
  for (int base = 0; base < nb; base += kThreads * kRsScanPer) {
    const int i0 = base + (int)threadIdx.x * kRsScanPer;
    uint32_t v[kRsScanPer], s = 0;
#pragma unroll
    for (int q = 0; q < kRsScanPer; ++q) {
      v[q] = i0 + q < nb ? row[i0 + q] : 0u;
      s += v[q];
    }
    uint32_t tot;
    uint32_t r = running + block_excl_scan(s, &tot);
#pragma unroll
    for (int q = 0; q < kRsScanPer; ++q) {
      if (i0 + q < nb) row[i0 + q] = r;
      r += v[q];
    }
    running += tot;
  }
  if (threadIdx.x == 0) digit_total[blockIdx.x] = running;
}

// Keys [blk + w * kWaveItems, + kWaveItems) belong to wave w of block blk,
// 64 per round; `vals` null means value = index.  A key's position in the
// block's stable order by digit is the block's count of smaller digits, the
// counts of its digit in earlier waves and its rank among its wave's keys of
// that digit.  The block's keys and values are first placed in that order in
// LDS, then thread e writes element e to the digit's global run (element e
// minus the digit's block-local start, plus its global start): a wave's 64
// writes fall into a few contiguous runs, where writing each key from its
// own lane scattered them over up to 64 short runs (with 256 digits a
// block's run of a digit averages 16 keys, and its partial lines went to
// memory separately: 2.3x the bytes written at city scale).
template <int ITEMS>
__global__ __launch_bounds__(kThreads) void k_rs_scatter(const uint32_t* __restrict__ keys,
                                                          const uint32_t* __restrict__ vals,
                                                          uint32_t* __restrict__ keys_out,
                                                          uint32_t* __restrict__ vals_out, int64_t n,
                                                          const uint32_t* __restrict__ n_dev, int shift,
                                                          const uint32_t* __restrict__ hist, int nb,
                                                          const uint32_t* __restrict__ digit_total) {
  constexpr int kBlockItems = kThreads * ITEMS;
  __shared__ uint32_t cnt[4][kRadix];
  __shared__ uint32_t gshift[kRadix];  // global start - block-local start of each digit
  __shared__ uint32_t lk[kBlockItems], lv[kBlockItems];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  constexpr int kWaveItems = ITEMS * 64;
  n = rs_count(n, n_dev);
  const int live = (int)((n + kBlockItems - 1) / kBlockItems);
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int blk = blockIdx.x; blk < live; blk += gridDim.x) {
    const int64_t wbase = (int64_t)blk * kBlockItems + (int64_t)w * kWaveItems;
    const int in_block = (int)min((int64_t)kBlockItems, n - (int64_t)blk * kBlockItems);
    // the keys and values are read first, so their latency overlaps that of
    // the digit offsets below
    uint32_t k[ITEMS], v[ITEMS], rk[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int64_t i = wbase + r * 64 + lane;
      const bool valid = i < n;
      k[r] = valid ? keys[i] : 0u;
      v[r] = valid ? (vals ? vals[i] : (uint32_t)i) : 0u;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) cnt[q][tid] = 0u;
    uint32_t base;
    {
      uint32_t tot;
      base = block_excl_scan(digit_total[tid], &tot) + hist[(int64_t)tid * nb + blk];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int64_t i = wbase + r * 64 + lane;
      const bool valid = i < n;
      const uint32_t d = (k[r] >> shift) & 0xffu;
      uint64_t same = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(bit);
        same &= bit ? m : ~m;
      }
      const uint32_t below = (uint32_t)__popcll(same & lt_mask);
      uint32_t prior = 0u;
      if (valid) prior = cnt[w][d];
      // the lowest lane of each digit group advances the wave's running
      // count; LDS accesses of one wave complete in order, so the next round
      // reads it
      if (valid && below == 0u) cnt[w][d] = prior + (uint32_t)__popcll(same);
      rk[r] = prior + below;
    }
    __syncthreads();
    {
      // digit tid: its block-local start (a scan over the digits) and the
      // start of each wave's keys of it
      const uint32_t c0 = cnt[0][tid], c1 = cnt[1][tid], c2 = cnt[2][tid], c3 = cnt[3][tid];
      uint32_t tot;
      const uint32_t local = block_excl_scan(((c0 + c1) + c2) + c3, &tot);
      cnt[0][tid] = local;
      cnt[1][tid] = local + c0;
      cnt[2][tid] = local + c0 + c1;
      cnt[3][tid] = local + c0 + c1 + c2;
      gshift[tid] = base - local;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int64_t i = wbase + r * 64 + lane;
      if (i < n) {
        const uint32_t lp = cnt[w][(k[r] >> shift) & 0xffu] + rk[r];
        lk[lp] = k[r];
        lv[lp] = v[r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int e = r * kThreads + tid;
      if (e < in_block) {
        const uint32_t kk = lk[e];
        const uint32_t pos = (uint32_t)e + gshift[(kk >> shift) & 0xffu];
        keys_out[pos] = kk;
        vals_out[pos] = lv[e];
      }
    }
    // the next block clears the counts and refills LDS only after every
    // wave has read them
    __syncthreads();
  }
}

// Visible Gaussians first: one wave per 64 consecutive Gaussians (the
// projection's workgroup b, whose visible count the scan turned into
// vis_off[b]).  A visible Gaussian's (key, index) goes to position
// vis_off[b] + (visible lanes below it); a culled one's index goes to
// tail[V + (culled Gaussians before it)], V = *visible.  Both keep index
// order, so a stable sort of the first V entries by key gives the same
// order as a stable sort of all n keys with the culled ones' key 0xffffffff.
__global__ __launch_bounds__(256) void k_compact_visible(const uint32_t* __restrict__ depth_key, int64_t n,
                                                          const uint32_t* __restrict__ vis_off,
                                                          const uint32_t* __restrict__ visible,
                                                          uint32_t* __restrict__ keys_out,
                                                          uint32_t* __restrict__ vals_out,
                                                          uint32_t* __restrict__ tail) {
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t g = b * 64 + lane;
  if (b * 64 >= n) return;
  const bool live = g < n;
  const uint32_t key = live ? depth_key[g] : 0xffffffffu;
  const bool vis = key != 0xffffffffu;
  const uint64_t m = __ballot(vis);
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const uint32_t before = vis_off[b];
  if (vis) {
    const uint32_t pos = before + (uint32_t)__popcll(m & below);
    keys_out[pos] = key;
    vals_out[pos] = (uint32_t)g;
  } else if (live) {
    // every lane below a live lane is live: the culled ones below are the
    // unset bits below
    const uint64_t culled_before = (uint64_t)(b * 64) - before;
    tail[*visible + culled_before + (uint64_t)__popcll(~m & below)] = (uint32_t)g;
  }
}

// ---------------------------------------------------------------- binning

__global__ __launch_bounds__(256) void k_gather_counts(const uint32_t* __restrict__ order,
                                                        const uint32_t* __restrict__ tiles, int64_t n,
                                                        const uint32_t* __restrict__ n_dev,
                                                        uint32_t* __restrict__ counts) {
  if (n_dev) n = *n_dev;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) counts[i] = tiles[order[i]];
}

// The owning Gaussian of pair index `target` (in depth order): the last
// entry whose exclusive offset is <= target (a zero-count entry shares its
// offset with the next one, so the last such entry is the owner).
__device__ __forceinline__ int64_t last_le(const uint32_t* __restrict__ offsets, int64_t n, uint32_t target) {
  int64_t lo = 0, hi = n;  // the first index with offsets[idx] > target is in (lo, hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (offsets[mid] <= target) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int wave_incl_max(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(v, d, 64);
    if (lane >= d) v = max(v, y);
  }
  return v;
}

// A workgroup writes the window of kEmitWin consecutive pairs [p0, p1).
// Every Gaussian (in depth order, count >= 1 up to the visible count) with
// pairs in the window is walked once, by one thread: its tile list row by
// row (SplatRows) up to the window's end, marking for each row the window
// position of the row's first pair in the window with that pair's tile and
// the Gaussian.  Then pair q takes the last mark at or before q (a
// workgroup max-scan): its tile is the marked tile plus the distance, since
// the pairs of a row are its tiles left to right.  Walking each Gaussian's
// rows once per window, instead of once per pair up to the pair's row, cuts
// the row evaluations of a splat of R rows from about pairs x (R + 1) / 2 to
// R.  The owners span at most kEmitWin consecutive entries from the owner of
// p0 (each has a pair), found from the scan's owner table (one entry per 256
// pairs) or by a binary search.  The thread of a Gaussian whose first pair
// lies in the window also records that pair in the splat record, and each
// row's entry (row_entry) is written by the window that holds the row's
// first pair.  A window holds four pairs per thread: the kernel is bound by
// the latency of its dependent loads and barriers (a city view took 0.160 ms
// with a workgroup per 256 pairs and 0.115 per 512; 1,024 take 15-24 us less
// than 512).  Pair writes are contiguous.
constexpr int kEmitWin = 1024;

__global__ __launch_bounds__(256) void k_emit_pairs(const uint32_t* __restrict__ order,
                                                     const uint32_t* __restrict__ offsets,
                                                     const uint32_t* __restrict__ owner, int64_t owner_blocks,
                                                     Rec* __restrict__ rec, const uint2* __restrict__ rect, int64_t n,
                                                     const uint32_t* __restrict__ n_dev, int64_t n_pairs, int tiles_x,
                                                     uint32_t* __restrict__ pair_tile, uint32_t* __restrict__ pair_gid,
                                                     uint32_t* __restrict__ rowtab) {
  if (n_dev) n = *n_dev;
  constexpr int kPer = kEmitWin / 256;
  __shared__ int64_t bounds[2];
  __shared__ int mark[kEmitWin];            // q where a row's first pair in the window sits at q, else -1
  __shared__ uint32_t run_tile[kEmitWin];   // at a mark: that pair's tile
  __shared__ uint32_t run_g[kEmitWin];      // at a mark: the Gaussian
  __shared__ int wmax[4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t p0 = (int64_t)blockIdx.x * kEmitWin;
  const int64_t p1 = p0 + kEmitWin < n_pairs ? p0 + kEmitWin : n_pairs;
  const int64_t ob = (int64_t)blockIdx.x * kPer;  // the owner table's 256-pair block of p0
  if (ob < owner_blocks) {
    if (tid == 0) {
      bounds[0] = owner[ob];
      bounds[1] = min(bounds[0] + kEmitWin - 1, n - 1);
    }
  } else if (tid < 2) {
    bounds[tid] = last_le(offsets, n, (uint32_t)(tid == 0 ? p0 : p1 - 1));
  }
#pragma unroll
  for (int h = 0; h < kPer; ++h) mark[h * 256 + tid] = -1;
  __syncthreads();
  const int64_t first = bounds[0];
#pragma unroll
  for (int h = 0; h < kPer; ++h) {
    const int64_t j = h * 256 + tid;
    if (j > bounds[1] - first) break;
    const int64_t rank = first + j;
    const int64_t off = offsets[rank];
    const int64_t end = rank + 1 < n ? (int64_t)offsets[rank + 1] : n_pairs;
    // the Gaussian's pairs k in [k_lo, k_hi) lie in the window
    const int64_t k_lo = p0 > off ? p0 - off : 0, k_hi = (p1 < end ? p1 : end) - off;
    if (k_lo < k_hi) {
      const uint32_t g = order[rank];
      const SplatRows sr = splat_rows_of(rec[g], rect[g]);
      if (k_lo == 0) rec[g].c.z = __uint_as_float((uint32_t)off);
      int64_t c = 0;  // pairs in the rows before row ty
      for (int ty = sr.y0; ty < sr.y1 && c < k_hi; ++ty) {
        int lo, hi;
        splat_row_span(sr, ty, lo, hi);
        const int64_t m = hi > lo ? hi - lo : 0;
        if (c + m > k_lo) {
          const int64_t kk = c > k_lo ? c : k_lo;
          const int q = (int)(off + kk - p0);
          mark[q] = q;
          run_tile[q] = (uint32_t)(ty * tiles_x + lo + (int)(kk - c));
          run_g[q] = g;
          // the row's entry, written by the window that holds its first pair
          if (kk == c && row_entry_kept(ty - sr.y0, (uint32_t)(end - off)))
            rowtab[off + (ty - sr.y0)] = row_entry((uint32_t)c, lo);
        }
        c += m;
      }
    }
  }
  __syncthreads();
  // the last mark at or before each position, over the window in quarters
  // of 256 positions carried in order (position 0 is always marked: the
  // owner of p0 marks the row of its pair k_lo)
  int carry = -1;
#pragma unroll
  for (int h = 0; h < kPer; ++h) {
    int s = wave_incl_max(mark[h * 256 + tid]);
    if (lane == 63) wmax[w] = s;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 3; ++i) s = i < w ? max(s, wmax[i]) : s;
    s = max(s, carry);
    carry = max(carry, max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3])));
    __syncthreads();
    const int q = h * 256 + tid;
    const int64_t i = p0 + q;
    if (i < p1) {
      pair_tile[i] = run_tile[s] + (uint32_t)(q - s);
      pair_gid[i] = run_g[s];
    }
  }
}

// Four consecutive sorted pairs per thread (one 16-byte load, the
// neighbours on either side from the adjacent words): a tile's range starts
// where the tile id differs from the previous pair's and ends where it
// differs from the next one's.
__global__ __launch_bounds__(256) void k_tile_ranges(const uint32_t* __restrict__ tile, int64_t n,
                                                      uint2* __restrict__ ranges) {
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= n) return;
  constexpr uint32_t kNone = 0xffffffffu;  // no tile id takes this value
  uint32_t t[6];
  t[0] = i0 > 0 ? tile[i0 - 1] : kNone;
  if (i0 + 4 <= n) {
    const uint4 q = *reinterpret_cast<const uint4*>(tile + i0);
    t[1] = q.x;
    t[2] = q.y;
    t[3] = q.z;
    t[4] = q.w;
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) t[1 + j] = i0 + j < n ? tile[i0 + j] : kNone;
  }
  t[5] = i0 + 4 < n ? tile[i0 + 4] : kNone;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t i = i0 + j;
    if (i >= n) break;
    if (t[j] != t[j + 1]) ranges[t[j + 1]].x = (uint32_t)i;
    if (t[j + 2] != t[j + 1]) ranges[t[j + 1]].y = (uint32_t)(i + 1);
  }
}

// Longest-list-first schedule of the tiles (approximate): one workgroup
// buckets the tiles by pair count on a quarter-octave scale, scans the bucket
// sizes from the longest down and scatters the tile ids.  The order inside a
// bucket is whatever the LDS atomics give -- each tile's result does not
// depend on when it runs, only the kernel's makespan does.  A second
// workgroup orders the backward's units the same way: a non-empty tile of c
// pairs gives c / GS3_SEG full depth segments and, if c is not a multiple,
// one shorter last segment, each bucketed by its own pair count.
constexpr int kOrderBuckets = 128;
__device__ __forceinline__ int count_bucket(uint32_t c) {
  return min(kOrderBuckets - 1, (int)(4.f * log2f((float)c + 1.f)));
}
// Exclusive scan of the bucket sizes from the longest bucket down, by the
// first wave (two buckets per lane): cur[b] becomes the number of entries in
// buckets above b; *total gets the sum.  The caller synchronises.
__device__ __forceinline__ void scan_buckets_desc(uint32_t* cur, uint32_t* total) {
  if (threadIdx.x < 64) {
    const int l = threadIdx.x;
    const uint32_t c0 = cur[kOrderBuckets - 1 - 2 * l], c1 = cur[kOrderBuckets - 2 - 2 * l];
    const uint32_t inc = wave_incl_scan(c0 + c1);
    const uint32_t ex = inc - (c0 + c1);
    cur[kOrderBuckets - 1 - 2 * l] = ex;
    cur[kOrderBuckets - 2 - 2 * l] = ex + c0;
    if (l == 63) *total = inc;
  }
}
// Workgroup 0 orders the tiles, workgroup 1 the units (independent, so the
// two run side by side).  The full segments all share one bucket; their
// counts are summed per wave first, so that bucket takes one LDS atomic per
// wave instead of one per tile.
__global__ __launch_bounds__(1024) void k_tile_order(const uint2* __restrict__ ranges, int n_tiles,
                                                      uint32_t* __restrict__ order, uint2* __restrict__ units,
                                                      int64_t n_units) {
  __shared__ uint32_t cursor[kOrderBuckets];
  __shared__ uint32_t total;
  const bool by_unit = blockIdx.x == 1;
  const int lane = threadIdx.x & 63;
  if (threadIdx.x < kOrderBuckets) cursor[threadIdx.x] = 0u;
  __syncthreads();
  const int full_bucket = count_bucket(GS3_SEG);
  for (int b0 = 0; b0 < n_tiles; b0 += blockDim.x) {
    const int i = b0 + (int)threadIdx.x;
    const uint2 r = i < n_tiles ? ranges[i] : make_uint2(0u, 0u);
    const uint32_t c = r.y - r.x;
    if (!by_unit) {
      if (i < n_tiles) atomicAdd(&cursor[count_bucket(c)], 1u);
    } else {
      const uint32_t nfull = wave_incl_scan(c / GS3_SEG);
      if (lane == 63 && nfull) atomicAdd(&cursor[full_bucket], nfull);
      if (c % GS3_SEG) atomicAdd(&cursor[count_bucket(c % GS3_SEG)], 1u);
    }
  }
  __syncthreads();
  scan_buckets_desc(cursor, &total);
  __syncthreads();
  for (int b0 = 0; b0 < n_tiles; b0 += blockDim.x) {
    const int i = b0 + (int)threadIdx.x;
    const uint2 r = i < n_tiles ? ranges[i] : make_uint2(0u, 0u);
    const uint32_t c = r.y - r.x, nfull = c / GS3_SEG, rem = c % GS3_SEG;
    if (!by_unit) {
      if (i < n_tiles) order[atomicAdd(&cursor[count_bucket(c)], 1u)] = (uint32_t)i;
    } else {
      // this lane's full segments follow those of the lanes below it
      const uint32_t inc = wave_incl_scan(nfull);
      uint32_t p = 0u;
      if (lane == 63 && inc) p = atomicAdd(&cursor[full_bucket], inc);
      p = (uint32_t)__shfl((int)p, 63, 64) + inc - nfull;
      for (uint32_t m = 0; m < nfull; ++m) units[p + m] = make_uint2((uint32_t)i, m);
      if (rem) units[atomicAdd(&cursor[count_bucket(rem)], 1u)] = make_uint2((uint32_t)i, nfull);
    }
  }
  if (by_unit)
    for (int64_t j = (int64_t)total + threadIdx.x; j < n_units; j += blockDim.x)
      units[j] = make_uint2((uint32_t)n_tiles, 0u);
}

__global__ __launch_bounds__(256) void k_make_keys(const uint32_t* __restrict__ tile, const uint32_t* __restrict__ gid,
                                                    const uint32_t* __restrict__ depth_key, int64_t n,
                                                    uint64_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) keys[i] = ((uint64_t)tile[i] << 32) | (uint64_t)depth_key[gid[i]];
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_fill_f32(float* __restrict__ p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

size_t scan_temp_bytes(int64_t n) { return (size_t)(nblk(n, kTileItems) + 1) * sizeof(uint32_t); }

void scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, void* temp, hipStream_t st,
                        uint32_t* owner, int64_t owner_blocks, uint32_t* total_host, const uint32_t* n_dev) {
  const int nb = (int)nblk(n, kTileItems);
  uint32_t* sums = (uint32_t*)temp;
  if (n <= 0) {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, total, (int64_t)1, 0u);
    if (total_host) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, total_host, (int64_t)1, 0u);
    return;
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kThreads), 0, st, in, n, n_dev, sums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kThreads), 0, st, sums, nb, n_dev, total, total_host);
  hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kThreads), 0, st, in, out, n, n_dev, sums, owner, owner_blocks);
}

size_t radix_temp_bytes(int64_t n) {
  const int64_t nb = nblk(n > 0 ? n : 1, kRsTile);
  return (size_t)(kRadix * nb + kRadix) * sizeof(uint32_t);
}

namespace {
// passes of `bits` key bits; with n_dev the element count is *n_dev <= n
void radix_passes(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* ka, uint32_t* va, uint32_t* kb,
                  uint32_t* vb, int64_t n, const uint32_t* n_dev, int bits, void* temp, hipStream_t st,
                  uint32_t** keys_out, uint32_t** vals_out) {
  *keys_out = ka;
  *vals_out = va;
  if (n <= 0) return;
  // a count known only on the device takes the small blocks (it is usually
  // far below its bound n) and at most kRsDevGrid workgroups per launch
  const bool big = !n_dev && n >= kRsBigFrom;
  const int tile = big ? kThreads * kRsItemsBig : kRsTile;
  const int nb = (int)nblk(n, tile);
  const dim3 grid(n_dev ? std::min(nb, kRsDevGrid) : nb);
  uint32_t* hist = (uint32_t*)temp;
  uint32_t* dtot = hist + (size_t)kRadix * nb;
  const uint32_t *kin = keys_in, *vin = vals_in;
  const int passes = std::max(1, (bits + 7) / 8);
  for (int p = 0; p < passes; ++p) {
    uint32_t* ko = (p & 1) ? kb : ka;
    uint32_t* vo = (p & 1) ? vb : va;
    if (big)
      hipLaunchKernelGGL(k_rs_upsweep<kRsItemsBig>, grid, dim3(kThreads), 0, st, kin, n, n_dev, 8 * p, hist, nb);
    else
      hipLaunchKernelGGL(k_rs_upsweep<kRsItems>, grid, dim3(kThreads), 0, st, kin, n, n_dev, 8 * p, hist, nb);
    hipLaunchKernelGGL(k_rs_scan, dim3(kRadix), dim3(kThreads), 0, st, hist, nb, n_dev, tile, dtot);
    if (big)
      hipLaunchKernelGGL(k_rs_scatter<kRsItemsBig>, grid, dim3(kThreads), 0, st, kin, vin, ko, vo, n, n_dev, 8 * p,
                         hist, nb, dtot);
    else
      hipLaunchKernelGGL(k_rs_scatter<kRsItems>, grid, dim3(kThreads), 0, st, kin, vin, ko, vo, n, n_dev, 8 * p,
                         hist, nb, dtot);
    kin = ko;
    vin = vo;
    *keys_out = ko;
    *vals_out = vo;
  }
}
}  // namespace

void radix_sort_u32(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* ka, uint32_t* va, uint32_t* kb,
                    uint32_t* vb, int64_t n, int bits, void* temp, hipStream_t st, uint32_t** keys_out,
                    uint32_t** vals_out) {
  radix_passes(keys_in, vals_in, ka, va, kb, vb, n, nullptr, bits, temp, st, keys_out, vals_out);
}

void depth_order(const uint32_t* depth_key, int64_t n, const uint32_t* vis_count, uint32_t* vis_off,
                 uint32_t* visible, void* scan_temp, uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb,
                 void* radix_temp, hipStream_t st, uint32_t** order) {
  *order = vb;
  if (n <= 0) return;
  const int64_t groups = (n + 63) / 64;
  scan_exclusive_u32(vis_count, vis_off, groups, visible, scan_temp, st);
  // visible (key, index) into (kb, vb)[0, V), culled indices into vb[V, n);
  // four passes then go kb -> ka -> kb -> ka -> kb over [0, V) only
  hipLaunchKernelGGL(k_compact_visible, dim3(nblk(groups, 4)), dim3(256), 0, st, depth_key, n, vis_off, visible, kb,
                     vb, vb);
  uint32_t* keys_out;
  radix_passes(kb, vb, ka, va, kb, vb, n, visible, 32, radix_temp, st, &keys_out, order);
}

void launch_gather_counts(const uint32_t* order, const uint32_t* tiles, int64_t n, const uint32_t* n_dev,
                          uint32_t* counts_sorted, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_gather_counts, dim3(nblk(n, 256)), dim3(256), 0, st, order, tiles, n, n_dev, counts_sorted);
}

void launch_emit_pairs(const uint32_t* order, const uint32_t* offsets_sorted, const uint32_t* owner,
                       int64_t owner_blocks, Rec* rec, const uint2* rect, int64_t n, const uint32_t* n_dev,
                       int64_t n_pairs, int tiles_x, uint32_t* pair_tile, uint32_t* pair_gid, uint32_t* rowtab,
                       hipStream_t st) {
  if (n > 0 && n_pairs > 0)
    hipLaunchKernelGGL(k_emit_pairs, dim3(nblk(n_pairs, kEmitWin)), dim3(256), 0, st, order, offsets_sorted, owner,
                       owner ? owner_blocks : (int64_t)0, rec, rect, n, n_dev, n_pairs, tiles_x, pair_tile, pair_gid,
                       rowtab);
}

void launch_tile_ranges(const uint32_t* pair_tile, int64_t n_pairs, uint2* ranges, int n_tiles, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u32, dim3(nblk(2 * (int64_t)n_tiles, 256)), dim3(256), 0, st, (uint32_t*)ranges,
                     2 * (int64_t)n_tiles, 0u);
  if (n_pairs > 0)
    hipLaunchKernelGGL(k_tile_ranges, dim3(nblk(n_pairs, 1024)), dim3(256), 0, st, pair_tile, n_pairs, ranges);
}

void launch_make_keys(const uint32_t* pair_tile, const uint32_t* pair_gid, const uint32_t* depth_key,
                      int64_t n_pairs, uint64_t* keys, hipStream_t st) {
  if (n_pairs > 0)
    hipLaunchKernelGGL(k_make_keys, dim3(nblk(n_pairs, 256)), dim3(256), 0, st, pair_tile, pair_gid, depth_key,
                       n_pairs, keys);
}

bool launch_tile_order(const uint2* ranges, int n_tiles, uint32_t* order, uint2* units, int64_t n_units,
                       hipStream_t st) {
  if (n_tiles < 1) return false;
  hipLaunchKernelGGL(k_tile_order, dim3(2), dim3(1024), 0, st, ranges, n_tiles, order, units, n_units);
  return true;
}

void launch_fill_f32(float* p, int64_t n, float v, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_fill_f32, dim3(nblk(n, 256)), dim3(256), 0, st, p, n, v);
}

void launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_fill_u32, dim3(nblk(n, 256)), dim3(256), 0, st, p, n, v);
}
