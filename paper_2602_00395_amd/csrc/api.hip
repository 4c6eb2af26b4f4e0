// Host side of the C ABI declared in include/gs3tr.h: scene ownership,
// argument validation, per-view binning and the orchestration of one
// optimizer iteration of 3DGS^2-TR (Algorithm 1) on a caller stream.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <utility>
#include <type_traits>
#include <vector>

#include "gs3_internal.h"
#include "gs3tr.h"

namespace {

thread_local std::string g_err;

gs3_status fail(gs3_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define GS3_HIP(call)                                                                                 \
  do {                                                                                               \
    hipError_t e_ = (call);                                                                          \
    if (e_ != hipSuccess) return fail(GS3_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define GS3_LAUNCHED() GS3_HIP(hipGetLastError())
#define GS3_TRY(expr)              \
  do {                             \
    gs3_status s_ = (expr);        \
    if (s_ != GS3_OK) return s_;   \
  } while (0)

constexpr int kMaxLossViews = 4096;
// pinned host words of a scene: [0] the pair count of the view being binned,
// [1] set by the update kernels when a gradient entry or an updated
// parameter is not finite
constexpr int kHostWords = 16;
// Largest image side: fewer than 2^20 tiles per view, so that a scan block of
// 4,096 Gaussians never sums to 2^32 tiles.
constexpr int kMaxSide = 16368;

// ---------------------------------------------------------------- profiler
// HIP events around named stages, plus device work counters for the blends.
namespace prof {
std::mutex mu;
std::atomic<bool> active{false};
bool counting = true;  // blend stages launch their counting instances
std::string names;  // ",name,name," or ",all,"
struct Entry {
  std::string name;
  hipEvent_t a = nullptr, b = nullptr;
  int slot = -1;
  int64_t w0 = 0, w1 = 0;
};
std::vector<Entry> entries;
constexpr int kSlots = 1 << 12;
constexpr size_t kSlotWords = 2 * GS3_PROF_SUB;
unsigned long long* ctr = nullptr;
int slots_used = 0;

struct Scope {
  int idx = -1;
  unsigned long long* c = nullptr;
};

Scope begin(const char* name, hipStream_t st, bool counted = false) {
  Scope sc;
  if (!active.load(std::memory_order_relaxed)) return sc;
  std::lock_guard<std::mutex> lk(mu);
  if (names.find(",all,") == std::string::npos && names.find("," + std::string(name) + ",") == std::string::npos)
    return sc;
  Entry e;
  e.name = name;
  if (hipEventCreate(&e.a) != hipSuccess || hipEventCreate(&e.b) != hipSuccess) return sc;
  (void)hipEventRecord(e.a, st);
  if (counted && counting && ctr && slots_used < kSlots) {
    e.slot = slots_used++;
    sc.c = ctr + kSlotWords * e.slot;
  }
  entries.push_back(e);
  sc.idx = (int)entries.size() - 1;
  return sc;
}

void end(const Scope& sc, hipStream_t st, int64_t w0 = 0, int64_t w1 = 0) {
  if (sc.idx < 0) return;
  std::lock_guard<std::mutex> lk(mu);
  Entry& e = entries[sc.idx];
  (void)hipEventRecord(e.b, st);
  e.w0 += w0;
  e.w1 += w1;
}

void clear_locked() {
  for (auto& e : entries) {
    if (e.a) (void)hipEventDestroy(e.a);
    if (e.b) (void)hipEventDestroy(e.b);
  }
  entries.clear();
  slots_used = 0;
}
}  // namespace prof

}  // namespace

// Buffers of one slot of a batch: the binning of a view (the slot of the
// view's first entry) and one entry's blend state, backward partials and
// image scratch (an entry is a view of a gradient batch, or one probe of a
// view of a Hutchinson batch).  Slot 0 is created with the scene, the others
// on the first batch that needs them.
struct ViewBufs {
  bool ready = false;
  // per-Gaussian binning scratch
  Rec* rec = nullptr;
  uint2* rect = nullptr;
  uint32_t *depth_key = nullptr, *tiles = nullptr, *ka = nullptr, *va = nullptr, *kb = nullptr, *vb = nullptr;
  uint32_t *counts = nullptr, *offsets = nullptr, *total_dev = nullptr;
  void* stmp = nullptr;
  void* rtmp = nullptr;
  size_t rtmp_bytes = 0;
  // per-pair binning scratch
  int64_t pair_cap = 0;
  uint32_t *pt = nullptr, *pg = nullptr, *pt2 = nullptr, *pg2 = nullptr;
  uint32_t* rowtab = nullptr;  // per-row entries of the tile lists (k_emit_pairs)
  // depth rank owning pair 256 b, written by the offsets scan for the
  // emission; sized from the pair capacity of earlier views
  uint32_t* block_owner = nullptr;
  int64_t owner_blocks = 0;
  // the backward's (tile, depth segment) units, seg_slots(max_tiles,
  // pair_cap) entries
  uint2* units = nullptr;
  uint2* ranges = nullptr;
  uint32_t* tile_order = nullptr;
  bool have_order = false;
  // state of the binned view
  const uint32_t* sorted_gid = nullptr;
  const uint32_t* order = nullptr;  // Gaussians in depth order
  const uint32_t* sorted_tile = nullptr;
  int64_t n_pairs = 0;
  int cam = -1;  // camera index of the binned view (-1: a camera given directly)
  CamDev cd{};   // its device camera
  // the entry's blend state: the long tiles' segment states
  // (seg_slots(max_tiles, blend_cap) rows) and the backward partials
  int64_t blend_cap = 0;
  float4* seg = nullptr;
  float* partials = nullptr;
  uint32_t* valid = nullptr;  // bit per partials slot: written by the last backward
  float* gsum = nullptr;  // float[N][9]: each Gaussian's summed partials
  TRec* trec = nullptr;
  // per-pixel image scratch
  float *img = nullptr, *cot = nullptr, *tan_img = nullptr, *ssim_tmp = nullptr;
  uint32_t* pix_last = nullptr;  // per pixel: 1 + pair index of the last contributing splat
  float* pix_T = nullptr;        // per pixel: final transmittance
  double* dpart = nullptr;
};

struct aux_stream_t {
  hipStream_t st = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

struct gs3_scene {
  int64_t N = 0;
  int deg = 0, K = 1, P = 14, n_cams = 0, n_train = 0;
  std::vector<gs3_camera> cams;
  std::vector<uint8_t> train;
  std::vector<int64_t> tgt_off;
  float bg[3] = {0, 0, 0};
  float lam = 0.f;
  uint32_t flags = 0;
  int64_t m_comp = 0;  // m = 6 * sum over training views of H W
  int64_t max_px = 0;
  int max_tiles = 0;
  // resident state
  float *x = nullptr, *targets = nullptr, *ghat = nullptr, *dhat = nullptr, *am = nullptr, *av = nullptr;
  // gs3_tr_iteration: the fused update writes x_alt (then the two swap); its
  // Hutchinson diagonal and the gradient of the views of earlier batches
  float *x_alt = nullptr, *dbuf = nullptr, *gacc = nullptr;
  ViewBufs vb[GS3_MAX_VIEWS];
  double* dsum = nullptr;
  uint32_t* host_u32 = nullptr;
  double* host_f64 = nullptr;
  hipEvent_t done_ev = nullptr;
  // gs3_tr_iteration: a second stream (default priority) for the probe
  // entries of a Hutchinson batch, forked from and joined to the caller's
  aux_stream_t aux{};
  // every buffer carved from the static scratch: nothing may be allocated
  bool fixed_scratch = false;
};

namespace {

int params_for(int deg) { return (deg < 0 || deg > 3) ? -1 : 11 + 3 * (deg + 1) * (deg + 1); }

CamDev make_cam(const gs3_camera& c) {
  CamDev d;
  for (int i = 0; i < 9; ++i) d.W[i] = c.R[i];
  for (int i = 0; i < 3; ++i) d.t[i] = c.t[i];
  d.fx = c.fx;
  d.fy = c.fy;
  d.cx = c.cx;
  d.cy = c.cy;
  const float hw = (float)c.width * 0.5f, hh = (float)c.height * 0.5f;
  const float tx = hw / c.fx, ty = hh / c.fy;
  d.limx = GS3_FOV_CLAMP * tx;
  d.limy = GS3_FOV_CLAMP * ty;
  for (int i = 0; i < 3; ++i) {
    double acc = 0.0;
    for (int k = 0; k < 3; ++k) acc -= (double)c.R[k * 3 + i] * (double)c.t[k];
    d.campos[i] = (float)acc;
  }
  d.width = c.width;
  d.height = c.height;
  d.tiles_x = (c.width + GS3_TILE - 1) / GS3_TILE;
  d.tiles_y = (c.height + GS3_TILE - 1) / GS3_TILE;
  return d;
}

// ---------------------------------------------------------------- memory
// Device blocks that a scene gives back (its teardown, pair scratch it has
// outgrown) stay in a process-wide cache instead of going back to the
// runtime, whose free waits for every stream of the device; a block is handed
// out again, to any scene, once the event recorded on the stream that last
// used it has completed.  So neither a scene's teardown nor its growth waits
// for another scene's stream.  The cache holds at most kCacheCap bytes (larger
// surpluses are returned to the runtime at once) and gs3_trim_cache empties it.
namespace mem {
struct Block {
  void* p;
  size_t bytes;
  int dev;
  hipEvent_t ready;  // completed once the last user's work is done; NULL: ready
};
std::mutex mu;
std::vector<Block> cached;
size_t cached_bytes = 0;
size_t cache_cap = (size_t)16 << 30;
std::vector<std::pair<void*, size_t>> sizes;  // live block -> bytes

size_t& live_size(void* p) {
  for (auto& e : sizes)
    if (e.first == p) return e.second;
  sizes.emplace_back(p, 0);
  return sizes.back().second;
}

bool is_ready(const Block& b) { return !b.ready || hipEventQuery(b.ready) == hipSuccess; }

void drop(Block& b) {
  if (b.ready) {
    (void)hipEventSynchronize(b.ready);
    (void)hipEventDestroy(b.ready);
  }
  (void)hipFree(b.p);
}

// smallest ready cached block of this device with bytes <= size <= 2 bytes
void* take(size_t bytes, int dev) {
  int best = -1;
  for (int i = 0; i < (int)cached.size(); ++i) {
    const Block& b = cached[i];
    if (b.dev != dev || b.bytes < bytes || b.bytes > 2 * bytes) continue;
    if (best >= 0 && cached[best].bytes <= b.bytes) continue;
    if (!is_ready(b)) continue;
    best = i;
  }
  if (best < 0) return nullptr;
  Block b = cached[best];
  cached.erase(cached.begin() + best);
  cached_bytes -= b.bytes;
  if (b.ready) (void)hipEventDestroy(b.ready);
  live_size(b.p) = b.bytes;
  return b.p;
}

void trim_locked(int dev) {
  for (size_t i = 0; i < cached.size();) {
    if (dev < 0 || cached[i].dev == dev) {
      cached_bytes -= cached[i].bytes;
      drop(cached[i]);
      cached.erase(cached.begin() + i);
    } else {
      ++i;
    }
  }
}

gs3_status alloc(void** p, size_t bytes) {
  *p = nullptr;
  bytes = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(GS3_EDEVICE, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(mu);
  if ((*p = take(bytes, dev))) return GS3_OK;
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    trim_locked(dev);  // the runtime may find room once the cache is empty
    if (hipMalloc(p, bytes) != hipSuccess) {
      *p = nullptr;
      (void)hipGetLastError();
      return fail(GS3_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
  }
  live_size(*p) = bytes;
  return GS3_OK;
}

// gives p back; `last_use` is the stream whose queued work may still use it
// (NULL pointer: nothing in flight uses it any more)
void release(void* p, const hipStream_t* last_use) {
  if (!p) return;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(mu);
  size_t bytes = 0;
  for (size_t i = 0; i < sizes.size(); ++i)
    if (sizes[i].first == p) {
      bytes = sizes[i].second;
      sizes.erase(sizes.begin() + i);
      break;
    }
  Block b{p, bytes, dev, nullptr};
  if (last_use) {
    if (hipEventCreateWithFlags(&b.ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(b.ready, *last_use) != hipSuccess) {
      if (b.ready) (void)hipEventDestroy(b.ready);
      b.ready = nullptr;
      (void)hipStreamSynchronize(*last_use);
    }
  }
  if (bytes == 0 || cached_bytes + bytes > cache_cap) {
    drop(b);
    return;
  }
  cached.push_back(b);
  cached_bytes += bytes;
}
// Pinned host buffers (the pair-count and non-finite words, loss sums) are
// small; they are pooled by size and kept for the life of the process, since
// freeing pinned memory can wait for the device as well.
std::vector<std::pair<void*, size_t>> host_pool;

gs3_status host_alloc(void** p, size_t bytes) {
  std::lock_guard<std::mutex> lk(mu);
  for (size_t i = 0; i < host_pool.size(); ++i)
    if (host_pool[i].second == bytes) {
      *p = host_pool[i].first;
      host_pool.erase(host_pool.begin() + i);
      return GS3_OK;
    }
  if (hipHostMalloc(p, bytes, hipHostMallocDefault) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(GS3_ENOMEM, "hipHostMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return GS3_OK;
}

void host_release(void* p, size_t bytes) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(mu);
  host_pool.emplace_back(p, bytes);
}
}  // namespace mem

template <class T>
gs3_status dalloc(T** p, size_t count) {
  void* v = nullptr;
  const gs3_status rc = mem::alloc(&v, std::max<size_t>(count, 1) * sizeof(T));
  *p = (T*)v;
  return rc;
}

// frees p; st: the stream whose queued work may still read or write it
template <class T>
void dfree(T*& p, const hipStream_t* st = nullptr) {
  mem::release((void*)p, st);
  p = nullptr;
}

void free_slot(ViewBufs& v) {
  dfree(v.rec);
  dfree(v.rect);
  dfree(v.trec);
  dfree(v.depth_key);
  dfree(v.tiles);
  dfree(v.ka);
  dfree(v.va);
  dfree(v.kb);
  dfree(v.vb);
  dfree(v.counts);
  dfree(v.offsets);
  dfree(v.total_dev);
  dfree(v.stmp);
  dfree(v.rtmp);
  dfree(v.pt);
  dfree(v.pg);
  dfree(v.pt2);
  dfree(v.pg2);
  dfree(v.rowtab);
  dfree(v.partials);
  dfree(v.valid);
  dfree(v.block_owner);
  dfree(v.units);
  dfree(v.seg);
  dfree(v.gsum);
  dfree(v.ranges);
  dfree(v.tile_order);
  dfree(v.img);
  dfree(v.cot);
  dfree(v.tan_img);
  dfree(v.pix_last);
  dfree(v.pix_T);
  dfree(v.ssim_tmp);
  dfree(v.dpart);
  v = ViewBufs{};
}

void free_all(gs3_scene* s) {
  dfree(s->x);
  dfree(s->x_alt);
  dfree(s->dbuf);
  dfree(s->gacc);
  dfree(s->targets);
  dfree(s->ghat);
  dfree(s->dhat);
  dfree(s->am);
  dfree(s->av);
  for (auto& v : s->vb)
    if (v.ready) free_slot(v);
  dfree(s->dsum);
  mem::host_release(s->host_u32, kHostWords * sizeof(uint32_t));
  mem::host_release(s->host_f64, sizeof(double) * kMaxLossViews);
  s->host_u32 = nullptr;
  s->host_f64 = nullptr;
  if (s->done_ev) (void)hipEventDestroy(s->done_ev);
  s->done_ev = nullptr;
  // every use of the second stream precedes a join the caller's stream
  // waited for, so the completion event above covered it
  if (s->aux.fork) (void)hipEventDestroy(s->aux.fork);
  if (s->aux.join) (void)hipEventDestroy(s->aux.join);
  if (s->aux.st) (void)hipStreamDestroy(s->aux.st);
  s->aux = aux_stream_t{};
}

// Optimizer state is allocated (and zeroed) on first use, so a scene holds
// only what its method needs: the trust-region EMAs on the first TR call,
// the Adam moments on the first Adam call, the fused iteration's second
// parameter buffer, D_t, gradient accumulator and radius on the first
// gs3_tr_iteration.
gs3_status zeroed(float** p, int64_t count, hipStream_t st) {
  if (*p) return GS3_OK;
  GS3_TRY(dalloc(p, (size_t)count));
  launch_fill_f32(*p, count, 0.f, st);
  return GS3_OK;
}
gs3_status need_tr_state(gs3_scene* s, hipStream_t st) {
  const int64_t PN = (int64_t)s->P * s->N;
  GS3_TRY(zeroed(&s->ghat, PN, st));
  return zeroed(&s->dhat, PN, st);
}
gs3_status need_adam_state(gs3_scene* s, hipStream_t st) {
  const int64_t PN = (int64_t)s->P * s->N;
  GS3_TRY(zeroed(&s->am, PN, st));
  return zeroed(&s->av, PN, st);
}
gs3_status need_aux(gs3_scene* s) {
  if (s->aux.st) return GS3_OK;
  GS3_HIP(hipStreamCreateWithFlags(&s->aux.st, hipStreamNonBlocking));
  GS3_HIP(hipEventCreateWithFlags(&s->aux.fork, hipEventDisableTiming));
  GS3_HIP(hipEventCreateWithFlags(&s->aux.join, hipEventDisableTiming));
  return GS3_OK;
}

gs3_status need_fused_state(gs3_scene* s, hipStream_t st) {
  const int64_t PN = (int64_t)s->P * s->N;
  GS3_TRY(need_tr_state(s, st));
  if (!s->x_alt) GS3_TRY(dalloc(&s->x_alt, (size_t)PN));
  if (!s->gacc) GS3_TRY(dalloc(&s->gacc, (size_t)PN));
  return GS3_OK;
}

// Pair scratch reserved at scene creation: kPairsPerGaussian pairs per
// Gaussian (the same estimate gs3_scene_bytes reports; object-scale views
// of 800x800 hold about 11).  A view with more
// pairs grows it; the outgrown blocks go back to the cache stream-ordered
// (on `st`, behind the work that still reads them), so growing never waits
// for the device.
constexpr int64_t kPairsPerGaussian = 12;

int64_t reserved_pairs(int64_t n) { return kPairsPerGaussian * n; }

// bytes of pair scratch for a capacity of `cap` pairs on views of up to
// max_tiles tiles: tile ids and Gaussian ids double-buffered, the tile
// lists' row entries, nine partials per pair, the backward's units and
// segment states, the radix histograms
int64_t pair_bytes(int64_t cap, int64_t max_tiles, int64_t n) {
  return cap * (20 + 36) + cap / 8 + seg_slots(max_tiles, cap) * (8 + 16 * GS3_BLOCK) +
         (int64_t)radix_temp_bytes(std::max<int64_t>(cap, n)) + 4 * (cap / 256 + 1);
}


// capacity allocated for a view of n pairs: 25% slack
int64_t pair_capacity(int64_t n_pairs) { return n_pairs + n_pairs / 4 + 4096; }

// per-Gaussian and per-pixel scratch of one slot (slot 0 is allocated at
// scene creation)
int64_t view_scratch_bytes(int64_t n, int64_t max_px, int64_t max_tiles) {
  return 172 * n + (int64_t)scan_temp_bytes(n) + 16 + 12 * max_tiles + 44 * max_px +
         4 * (int64_t)ssim_tmp_floats(1, (int)max_px) + 8 * (max_px * 3 / 256 + max_tiles + 1024);
}

// Binning buffers of a slot for a view of n_pairs pairs.
gs3_status ensure_pairs(gs3_scene* s, ViewBufs& v, int64_t n_pairs, const hipStream_t* st) {
  if (n_pairs <= v.pair_cap && v.rtmp) return GS3_OK;
  if (s->fixed_scratch)
    return fail(GS3_EINVAL, "the view has " + std::to_string(n_pairs) + " (Gaussian, tile) pairs; the static scratch holds " +
                                std::to_string(v.pair_cap));
  const int64_t cap = std::max<int64_t>(pair_capacity(n_pairs), v.pair_cap);
  dfree(v.pt, st);
  dfree(v.pg, st);
  dfree(v.pt2, st);
  dfree(v.pg2, st);
  dfree(v.rowtab, st);
  dfree(v.rtmp, st);
  dfree(v.units, st);
  v.pair_cap = 0;
  GS3_TRY(dalloc(&v.pt, cap));
  GS3_TRY(dalloc(&v.pg, cap));
  GS3_TRY(dalloc(&v.pt2, cap));
  GS3_TRY(dalloc(&v.pg2, cap));
  GS3_TRY(dalloc(&v.rowtab, cap));
  GS3_TRY(dalloc(&v.units, (size_t)seg_slots(s->max_tiles, cap)));
  v.rtmp_bytes = radix_temp_bytes(std::max<int64_t>(cap, s->N));
  GS3_TRY(dalloc((char**)&v.rtmp, v.rtmp_bytes));
  v.pair_cap = cap;
  return GS3_OK;
}

// Blend state of a slot for an entry of a view of n_pairs pairs: the
// backward partials and the long tiles' segment states.
// (the allocation-free render has segment states only: no backward)
gs3_status ensure_blend(gs3_scene* s, ViewBufs& v, int64_t n_pairs, const hipStream_t* st) {
  if (n_pairs <= v.blend_cap && v.seg && (v.partials || s->fixed_scratch)) return GS3_OK;
  if (s->fixed_scratch)
    return fail(GS3_EINVAL, "the view has " + std::to_string(n_pairs) + " (Gaussian, tile) pairs; the static scratch holds " +
                                std::to_string(v.blend_cap));
  const int64_t cap = std::max<int64_t>(pair_capacity(n_pairs), v.blend_cap);
  dfree(v.partials, st);
  dfree(v.valid, st);
  dfree(v.seg, st);
  v.blend_cap = 0;
  GS3_TRY(dalloc(&v.partials, (size_t)cap * 9));
  GS3_TRY(dalloc(&v.valid, (size_t)(cap / 32 + 1)));
  GS3_TRY(dalloc(&v.seg, (size_t)seg_slots(s->max_tiles, cap) * GS3_BLOCK));
  v.blend_cap = cap;
  return GS3_OK;
}

// The offsets scan records the owner of every 256-pair block of the pair
// capacity known before the view (the emission searches for the owners of
// blocks beyond it), so this array follows the capacity one view later.
gs3_status ensure_owner_blocks(gs3_scene* s, ViewBufs& v, const hipStream_t* st) {
  if (v.owner_blocks >= v.pair_cap / 256 + 1 || s->fixed_scratch) return GS3_OK;
  dfree(v.block_owner, st);
  v.owner_blocks = 0;
  GS3_TRY(dalloc(&v.block_owner, (size_t)(v.pair_cap / 256 + 1)));
  v.owner_blocks = v.pair_cap / 256 + 1;
  return GS3_OK;
}

// Per-Gaussian and per-pixel buffers of a slot, and its pair buffers for
// `pairs` pairs.
gs3_status alloc_slot(gs3_scene* s, ViewBufs& v, int64_t pairs) {
  if (v.ready) return GS3_OK;
  const int64_t N = s->N;
  gs3_status rc = GS3_OK;
  auto step = [&](gs3_status r) {
    if (rc == GS3_OK) rc = r;
  };
  step(dalloc(&v.rec, N));
  step(dalloc(&v.rect, N));
  step(dalloc(&v.trec, N));
  step(dalloc(&v.depth_key, N));
  step(dalloc(&v.tiles, N));
  step(dalloc(&v.ka, N));
  step(dalloc(&v.va, N));
  step(dalloc(&v.kb, N));
  step(dalloc(&v.vb, N));
  step(dalloc(&v.counts, N));
  step(dalloc(&v.gsum, 9 * N));
  step(dalloc(&v.offsets, N));
  step(dalloc(&v.total_dev, 4));
  step(dalloc((char**)&v.stmp, scan_temp_bytes(N)));
  step(dalloc(&v.ranges, s->max_tiles));
  step(dalloc(&v.tile_order, s->max_tiles));
  step(dalloc(&v.img, s->max_px * 3));
  step(dalloc(&v.cot, s->max_px * 3));
  step(dalloc(&v.tan_img, s->max_px * 3));
  step(dalloc(&v.pix_last, s->max_px));
  step(dalloc(&v.pix_T, s->max_px));
  step(dalloc(&v.ssim_tmp, ssim_tmp_floats(1, (int)s->max_px)));
  step(dalloc(&v.dpart, s->max_px * 3 / 256 + s->max_tiles + 1024));
  if (rc == GS3_OK) rc = ensure_pairs(s, v, pairs, nullptr);
  if (rc == GS3_OK) rc = ensure_blend(s, v, pairs, nullptr);
  if (rc == GS3_OK) rc = ensure_owner_blocks(s, v, nullptr);
  if (rc != GS3_OK) {
    free_slot(v);
    return rc;
  }
  v.ready = true;
  return GS3_OK;
}

// Slots 0..n-1 ready (new ones sized like slot 0's current pair capacity).
gs3_status need_slots(gs3_scene* s, int n) {
  if (n > GS3_MAX_VIEWS) return fail(GS3_EINVAL, "batch of more than GS3_MAX_VIEWS entries");
  for (int k = 1; k < n; ++k)
    GS3_TRY(alloc_slot(s, s->vb[k], std::max<int64_t>(s->vb[0].n_pairs, 4096)));
  return GS3_OK;
}

gs3_status check_scene(gs3_scene* s) {
  if (!s) return fail(GS3_EINVAL, "scene is NULL");
  if (!s->x) return fail(GS3_ESTATE, "scene has been destroyed");
  return GS3_OK;
}

gs3_status check_cam(gs3_scene* s, int32_t cam) {
  if (cam < 0 || cam >= s->n_cams)
    return fail(GS3_EINVAL, "camera index " + std::to_string(cam) + " out of range [0, " + std::to_string(s->n_cams) + ")");
  return GS3_OK;
}

// Value of the pinned pair-count word until the scan has written it (a pair
// count never reaches it: pair indices are 32-bit).
constexpr uint32_t kCountPending = 0xffffffffu;
// Value the scan writes when the view's pair count does not fit 32 bits.
constexpr uint32_t kCountOverflow = 0xfffffffeu;

// Waits until the scan has written the pinned word: a short busy poll, then
// polls that yield the thread; after 10 s, or if the stream reports an
// error, the stream is synchronised and its status returned.
gs3_status wait_count(volatile uint32_t* word, hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  for (uint64_t k = 0; *word == kCountPending; ++k) {
    if ((k & 1023u) == 1023u) {
      const hipError_t q = hipStreamQuery(st);
      if (q != hipErrorNotReady && q != hipSuccess) break;
      if (q == hipSuccess && *word == kCountPending) break;  // stream done, word never written
      if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(10)) break;
      if (k > (1u << 16)) std::this_thread::yield();
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  if (*word == kCountPending) {
    GS3_HIP(hipStreamSynchronize(st));
    if (*word == kCountPending) return fail(GS3_EDEVICE, "pair count was not written by the scan");
  }
  return GS3_OK;
}

int bits_for(int n_tiles) {
  int b = 1;
  while ((1 << b) < n_tiles) ++b;
  return b;
}

// Project, sort by depth, emit pairs, sort pairs by tile, per-tile ranges.
// Waits once for the pair count (see wait_count), not for the whole stream.
gs3_status bin_camera(gs3_scene* s, ViewBufs& v, const gs3_camera& camera, int cam, hipStream_t st) {
  const CamDev cd = make_cam(camera);
  v.cd = cd;
  const int64_t N = s->N;
  GS3_TRY(ensure_owner_blocks(s, v, &st));
  auto p0 = prof::begin("project_fwd", st);
  // the per-64 visible counts go to v.counts and their offsets to
  // v.offsets, both free until the pair-count scan below
  launch_project_fwd(s->x, N, s->deg, cd, v.rec, v.rect, v.depth_key, v.tiles, v.counts, st);
  prof::end(p0, st);
  GS3_LAUNCHED();
  auto p1 = prof::begin("depth_sort", st);
  uint32_t* order;
  depth_order(v.depth_key, N, v.counts, v.offsets, v.total_dev + 1, v.stmp, v.ka, v.va, v.kb, v.vb, v.rtmp, st,
              &order);
  prof::end(p1, st);
  auto p2 = prof::begin("scan", st);
  // ranks past the visible count V = v.total_dev[1] hold culled Gaussians:
  // the counts, their scan, the emission and the pair sums stop at V
  launch_gather_counts(order, v.tiles, N, v.total_dev + 1, v.counts, st);
  // the scan stores the pair count into a pinned host word as soon as it is
  // known; the host waits for that word (not for the stream), so the
  // launches below are queued while the scan's last kernel still runs
  // (without a pinned word -- the allocation-free render -- the count is
  // copied back and the stream synchronised)
  uint32_t copied = kCountPending;
  volatile uint32_t* count_word = s->host_u32 ? s->host_u32 : &copied;
  *count_word = kCountPending;
  std::atomic_thread_fence(std::memory_order_seq_cst);
  scan_exclusive_u32(v.counts, v.offsets, N, v.total_dev, v.stmp, st, v.block_owner, v.owner_blocks,
                     s->host_u32, v.total_dev + 1);
  prof::end(p2, st);
  GS3_LAUNCHED();
  if (s->host_u32) {
    GS3_TRY(wait_count(count_word, st));
  } else {
    GS3_HIP(hipMemcpyAsync(&copied, v.total_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    GS3_HIP(hipStreamSynchronize(st));
  }
  if (*count_word == kCountOverflow)
    return fail(GS3_EINVAL, "camera " + std::to_string(cam) + ": the view has 2^32 - 2 or more (Gaussian, tile) pairs");
  const int64_t n_pairs = *count_word;
  GS3_TRY(ensure_pairs(s, v, n_pairs, &st));
  GS3_TRY(ensure_blend(s, v, n_pairs, &st));
  auto p3 = prof::begin("emit_pairs", st);
  launch_emit_pairs(order, v.offsets, v.block_owner, v.owner_blocks, v.rec, v.rect, N, v.total_dev + 1, n_pairs,
                    cd.tiles_x, v.pt, v.pg, v.rowtab, st);
  prof::end(p3, st, N, n_pairs);
  const int n_tiles = cd.tiles_x * cd.tiles_y;
  uint32_t *tk, *tv;
  auto p4 = prof::begin("pair_sort", st);
  radix_sort_u32(v.pt, v.pg, v.pt2, v.pg2, v.pt, v.pg, n_pairs, bits_for(n_tiles), v.rtmp, st, &tk, &tv);
  launch_tile_ranges(tk, n_pairs, v.ranges, n_tiles, st);
  v.have_order = launch_tile_order(v.ranges, n_tiles, v.tile_order, v.units, seg_slots(n_tiles, n_pairs), st);
  prof::end(p4, st, n_pairs, bits_for(n_tiles));
  GS3_LAUNCHED();
  v.sorted_gid = tv;
  v.sorted_tile = tk;
  v.order = order;
  v.n_pairs = n_pairs;
  return GS3_OK;
}

gs3_status bin_view(gs3_scene* s, ViewBufs& v, int cam, hipStream_t st) {
  v.cam = cam;
  return bin_camera(s, v, s->cams[cam], cam, st);
}

gs3_status finish(gs3_scene* s, hipStream_t st) {
  (void)s;
  (void)st;
  GS3_LAUNCHED();
  return GS3_OK;
}

// Records the scene's completion event on the call's stream when an entry
// point returns, whether it succeeded or failed after enqueuing work, so
// that gs3_scene_sync and gs3_scene_destroy wait for everything the scene
// has enqueued (and for nothing else).
struct CallEnd {
  gs3_scene* s;
  hipStream_t st;
  ~CallEnd() {
    if (s && s->done_ev) (void)hipEventRecord(s->done_ev, st);
  }
};

const float* target_of(gs3_scene* s, int cam) { return s->targets + s->tgt_off[cam]; }

// Entry k of a batch: its view's binning is in slot b[k], its blend state
// in slot e[k] (equal for the views of a gradient batch; the probes of one
// view in a Hutchinson batch share the binning of the view's first slot).
struct Entries {
  int n = 0;
  int b[GS3_MAX_VIEWS] = {}, e[GS3_MAX_VIEWS] = {};
  uint32_t probe[GS3_MAX_VIEWS] = {};
};

BlendView blend_view(const ViewBufs& b, ViewBufs& e) {
  BlendView V;
  V.rec = b.rec;
  V.trec = e.trec;
  V.pair_gid = b.sorted_gid;
  V.ranges = b.ranges;
  V.order = b.have_order ? b.tile_order : nullptr;
  V.rect = b.rect;
  V.tiles = b.tiles;
  V.rowtab = b.rowtab;
  V.units = b.units;
  V.cam = b.cd;
  V.n_tiles = b.cd.tiles_x * b.cd.tiles_y;
  V.n_units = b.have_order ? seg_slots(V.n_tiles, b.n_pairs) : 0;
  V.cot = e.cot;
  V.partials = e.partials;
  V.valid = e.valid;
  V.img = e.img;
  V.tan_img = e.tan_img;
  V.pix_last = e.pix_last;
  V.pix_T = e.pix_T;
  V.seg = e.seg;
  return V;
}

BlendBatch blend_batch(gs3_scene* s, const Entries& E) {
  BlendBatch B;
  B.n = E.n;
  for (int k = 0; k < E.n; ++k) B.v[k] = blend_view(s->vb[E.b[k]], s->vb[E.e[k]]);
  return B;
}

// out (nullable): the image of a single-entry batch goes there instead of
// the slot's image buffer
void blend_fwd(gs3_scene* s, const Entries& E, hipStream_t st, float* out = nullptr) {
  BlendBatch B = blend_batch(s, E);
  if (out) B.v[0].img = out;
  auto p = prof::begin("blend_fwd", st, true);
  launch_blend_fwd(B, s->bg, st, p.c);
  prof::end(p, st);
}

void blend_jvp(gs3_scene* s, const Entries& E, hipStream_t st, float* out = nullptr, float* tan = nullptr) {
  BlendBatch B = blend_batch(s, E);
  if (out) B.v[0].img = out;
  if (tan) B.v[0].tan_img = tan;
  auto p = prof::begin("blend_jvp", st, true);
  launch_blend_jvp(B, s->bg, st, p.c);
  prof::end(p, st);
}

// cot (nullable): the cotangent of a single-entry batch, in place of the slot's
void blend_bwd(gs3_scene* s, const Entries& E, hipStream_t st, const float* cot = nullptr) {
  BlendBatch B = blend_batch(s, E);
  if (cot) B.v[0].cot = cot;
  auto p = prof::begin("blend_bwd", st, true);
  // the backward writes the partials of the pairs some wave used and sets
  // their bits; every other slot (behind each tile's last contribution, or
  // culled for every wave) counts as zero without being written
  for (int k = 0; k < E.n; ++k) launch_fill_u32(s->vb[E.e[k]].valid, s->vb[E.b[k]].n_pairs / 32 + 1, 0u, st);
  launch_blend_bwd(B, s->bg, st, p.c);
  prof::end(p, st);
}

// Pair sums of every entry, then the chain rule over the batch (modes as
// launch_project_bwd; mode 1 takes each entry's probe of `seed`, and so do
// the last n_probe entries of a mode-2 batch).
void project_bwd(gs3_scene* s, const Entries& E, int mode, int acc, uint64_t seed, float scale, float* out,
                 hipStream_t st, const FusedTr& ft = FusedTr{}, int n_probe = 0, float probe_scale = 0.f) {
  BwdBatch B;
  B.n = E.n;
  B.n_probe = n_probe;
  B.probe_scale = probe_scale;
  auto ps = prof::begin("pair_sums", st);
  int64_t pairs = 0;
  for (int k = 0; k < E.n; ++k) {
    const ViewBufs& b = s->vb[E.b[k]];
    ViewBufs& e = s->vb[E.e[k]];
    launch_pair_sums(b.order, b.offsets, b.counts, e.partials, e.valid, s->N, b.total_dev + 1, e.gsum, st);
    B.v[k].rec = b.rec;
    B.v[k].tiles = b.tiles;
    B.v[k].G = e.gsum;
    B.v[k].cam = b.cd;
    B.v[k].inner = mode == 1 || k >= E.n - n_probe ? probe_key(seed, E.probe[k]) : 0ull;
    pairs += b.n_pairs;
  }
  prof::end(ps, st, s->N, pairs);
  auto p = prof::begin(mode == 2 ? "tr_update" : "project_bwd", st);
  launch_project_bwd(s->x, s->N, s->deg, B, mode, acc, scale, out, ft, st);
  prof::end(p, st, s->N, 0);
}

void project_jvp(gs3_scene* s, const ViewBufs& b, ViewBufs& e, int kind, uint64_t seed, uint32_t i,
                 const float* tangent, hipStream_t st) {
  auto p = prof::begin("project_jvp", st);
  launch_project_jvp(s->x, s->N, s->deg, b.cd, b.rec, b.tiles, kind, seed, i, tangent, e.trec, st);
  prof::end(p, st, s->N, 0);
}

Entries single() {
  Entries E;
  E.n = 1;
  return E;
}

gs3_status validate_desc(const gs3_scene_desc* d) {
  if (!d) return fail(GS3_EINVAL, "desc is NULL");
  if (d->n_gaussians < 1 || d->n_gaussians > 0x7fffffffLL) return fail(GS3_EINVAL, "n_gaussians must be in [1, 2^31)");
  if (params_for(d->sh_degree) < 0) return fail(GS3_EINVAL, "sh_degree must be 0..3");
  if (d->n_cameras < 1 || !d->cameras) return fail(GS3_EINVAL, "need at least one camera");
  if (!(d->lambda_dssim >= 0.f && d->lambda_dssim <= 1.f)) return fail(GS3_EINVAL, "lambda_dssim must be in [0, 1]");
  if (d->flags != GS3_FLAG_NONE) return fail(GS3_EINVAL, "flags is reserved and must be 0");
  int n_train = 0;
  for (int j = 0; j < d->n_cameras; ++j) {
    const gs3_camera& c = d->cameras[j];
    if (c.width < 1 || c.height < 1 || c.width > kMaxSide || c.height > kMaxSide)
      return fail(GS3_EINVAL, "camera " + std::to_string(j) + " has an invalid size");
    if (!(c.fx > 0.f) || !(c.fy > 0.f)) return fail(GS3_EINVAL, "camera " + std::to_string(j) + " has fx/fy <= 0");
    n_train += (!d->train_mask || d->train_mask[j]) ? 1 : 0;
  }
  if (n_train < 1) return fail(GS3_EINVAL, "no training camera");
  return GS3_OK;
}

}  // namespace

// ---------------------------------------------------------------- static scratch
// Device scratch of gs3_render_noalloc, the render for callers that cannot
// allocate: one array per GPU, created with the code object and held until
// the process ends.  Host code never takes the array's name as an address:
// each device's address comes from hipGetSymbolAddress on the first call on
// that device (with that device current) and is kept per device.
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

namespace statics {
std::mutex mu;
constexpr int kMaxDevices = 64;
void* addr[kMaxDevices] = {};
}  // namespace statics

gs3_status static_scratch(void** out) {
  int dev = 0;
  GS3_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= statics::kMaxDevices) return fail(GS3_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(statics::mu);
  if (!statics::addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(GS3_EDEVICE, std::string("hipGetSymbolAddress of the static scratch failed: ") + hipGetErrorString(e));
    }
    statics::addr[dev] = p;
  }
  *out = statics::addr[dev];
  return GS3_OK;
}

// Consecutive 256-byte aligned pieces of one buffer.
struct Carver {
  char* base;
  size_t size, used = 0;
  template <class T>
  T* take(size_t count) {
    const size_t at = (used + 255) & ~(size_t)255;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (at + bytes > size) return nullptr;
    used = at + bytes;
    return reinterpret_cast<T*>(base + at);
  }
  // bytes the same takes would need, for the size check before any work
  template <class T>
  void need(size_t count) {
    used = ((used + 255) & ~(size_t)255) + std::max<size_t>(count, 1) * sizeof(T);
  }
};

// The render's buffers for n Gaussians and one camera, laid out by `c`;
// `pairs` is the pair capacity.  With take == false only sizes are summed.
template <bool Take>
void carve_render(Carver& c, ViewBufs& t, int64_t n, int64_t px, int64_t tiles, int64_t pairs) {
  auto get = [&](auto** p, size_t count) {
    using T = std::remove_pointer_t<std::remove_reference_t<decltype(p)>>;
    if constexpr (Take) {
      *p = c.template take<std::remove_pointer_t<T>>(count);
    } else {
      c.template need<std::remove_pointer_t<T>>(count);
    }
  };
  get(&t.rec, n);
  get(&t.rect, n);
  get(&t.depth_key, n);
  get(&t.tiles, n);
  get(&t.ka, n);
  get(&t.va, n);
  get(&t.kb, n);
  get(&t.vb, n);
  get(&t.counts, n);
  get(&t.offsets, n);
  get(&t.total_dev, 4);
  get((char**)&t.stmp, scan_temp_bytes(n));
  get(&t.ranges, tiles);
  get(&t.tile_order, tiles);
  get(&t.pix_last, px);
  get(&t.pix_T, px);
  get(&t.pt, pairs);
  get(&t.pg, pairs);
  get(&t.pt2, pairs);
  get(&t.pg2, pairs);
  get(&t.rowtab, pairs);
  get(&t.units, seg_slots(tiles, pairs));
  get(&t.seg, seg_slots(tiles, pairs) * GS3_BLOCK);
  get((char**)&t.rtmp, radix_temp_bytes(std::max<int64_t>(pairs, n)));
  get(&t.block_owner, pairs / 256 + 1);
}

size_t render_bytes(int64_t n, int64_t px, int64_t tiles, int64_t pairs) {
  ViewBufs t;
  Carver c{nullptr, 0};
  carve_render<false>(c, t, n, px, tiles, pairs);
  return c.used;
}

}  // namespace

extern "C" {

int32_t gs3_n_params(int32_t sh_degree) { return params_for(sh_degree); }

const char* gs3_version(void) { return "gs3tr 0.1 gfx950"; }

const char* gs3_last_error(void) { return g_err.c_str(); }

gs3_status gs3_scene_bytes(const gs3_scene_desc* d, int64_t* resident, int64_t* peak_scratch) {
  GS3_TRY(validate_desc(d));
  if (!resident || !peak_scratch) return fail(GS3_EINVAL, "output pointers must not be NULL");
  const int64_t N = d->n_gaussians, P = params_for(d->sh_degree);
  int64_t px_total = 0, max_px = 0, max_tiles = 0;
  for (int j = 0; j < d->n_cameras; ++j) {
    const int64_t px = (int64_t)d->cameras[j].width * d->cameras[j].height;
    px_total += px;
    max_px = std::max(max_px, px);
    max_tiles = std::max<int64_t>(max_tiles, (int64_t)((d->cameras[j].width + GS3_TILE - 1) / GS3_TILE) *
                                                 ((d->cameras[j].height + GS3_TILE - 1) / GS3_TILE));
  }
  // the targets, the parameters, both buffers of the fused iteration, the
  // EMAs, D_t and the gradient accumulator of the trust-region method (Adam
  // instead holds two moments)
  *resident = 12 * px_total + 4 * P * N * 6;
  // slot 0 at creation, and the slot of the probe entry of a trust-region
  // iteration with one Hutchinson view and probe
  *peak_scratch =
      2 * (view_scratch_bytes(N, max_px, max_tiles) + pair_bytes(pair_capacity(reserved_pairs(N)), max_tiles, N));
  return GS3_OK;
}

gs3_status gs3_scene_create(const gs3_scene_desc* d, const float* params_dev, const float* targets_dev,
                            hipStream_t st, gs3_scene** out) {
  if (!out) return fail(GS3_EINVAL, "out is NULL");
  *out = nullptr;
  GS3_TRY(validate_desc(d));
  if (!params_dev || !targets_dev) return fail(GS3_EINVAL, "params_dev and targets_dev must not be NULL");
  gs3_scene* s = new gs3_scene();
  s->N = d->n_gaussians;
  s->deg = d->sh_degree;
  s->K = (d->sh_degree + 1) * (d->sh_degree + 1);
  s->P = params_for(d->sh_degree);
  s->n_cams = d->n_cameras;
  s->cams.assign(d->cameras, d->cameras + d->n_cameras);
  s->train.resize(d->n_cameras);
  s->tgt_off.resize(d->n_cameras);
  int64_t off = 0;
  for (int j = 0; j < d->n_cameras; ++j) {
    s->train[j] = (!d->train_mask || d->train_mask[j]) ? 1 : 0;
    const int64_t px = (int64_t)s->cams[j].width * s->cams[j].height;
    s->tgt_off[j] = off;
    off += px * 3;
    s->max_px = std::max(s->max_px, px);
    const CamDev cd = make_cam(s->cams[j]);
    s->max_tiles = std::max(s->max_tiles, cd.tiles_x * cd.tiles_y);
    if (s->train[j]) {
      s->n_train += 1;
      s->m_comp += 6 * px;
    }
  }
  for (int c = 0; c < 3; ++c) s->bg[c] = d->background[c];
  s->lam = d->lambda_dssim;
  s->flags = d->flags;
  const int64_t PN = (int64_t)s->P * s->N;
  gs3_status rc = GS3_OK;
  auto step = [&](gs3_status r) {
    if (rc == GS3_OK) rc = r;
  };
  step(dalloc(&s->x, PN));
  step(dalloc(&s->targets, off));
  step(dalloc(&s->dsum, kMaxLossViews));
  if (rc == GS3_OK) rc = mem::host_alloc((void**)&s->host_u32, kHostWords * sizeof(uint32_t));
  if (rc == GS3_OK) rc = mem::host_alloc((void**)&s->host_f64, sizeof(double) * kMaxLossViews);
  if (rc == GS3_OK) s->host_u32[1] = 0u;
  if (rc == GS3_OK && hipEventCreateWithFlags(&s->done_ev, hipEventDisableTiming) != hipSuccess)
    rc = fail(GS3_EDEVICE, "hipEventCreate failed");
  if (rc == GS3_OK) rc = alloc_slot(s, s->vb[0], reserved_pairs(s->N));
  if (rc != GS3_OK) {
    free_all(s);
    delete s;
    return rc;
  }
  auto copy = [&](void* dst, const void* src, size_t bytes) -> gs3_status {
    GS3_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
    return GS3_OK;
  };
  rc = copy(s->x, params_dev, PN * sizeof(float));
  if (rc == GS3_OK) rc = copy(s->targets, targets_dev, off * sizeof(float));
  if (rc == GS3_OK) rc = finish(s, st);
  if (rc == GS3_OK && hipEventRecord(s->done_ev, st) != hipSuccess) rc = fail(GS3_EDEVICE, "hipEventRecord failed");
  if (rc != GS3_OK) {
    (void)hipStreamSynchronize(st);
    free_all(s);
    delete s;
    return rc;
  }
  *out = s;
  return GS3_OK;
}

gs3_status gs3_scene_destroy(gs3_scene* s) {
  if (!s) return fail(GS3_EINVAL, "scene is NULL");
  // everything this scene enqueued precedes its completion event; its
  // blocks go back to the cache, so nothing here waits for other streams
  if (s->done_ev) (void)hipEventSynchronize(s->done_ev);
  free_all(s);
  delete s;
  return GS3_OK;
}

gs3_status gs3_scene_device_bytes(gs3_scene* s, int64_t* bytes) {
  GS3_TRY(check_scene(s));
  if (!bytes) return fail(GS3_EINVAL, "bytes is NULL");
  const int64_t PN = (int64_t)s->P * s->N;
  int64_t px_total = 0;
  for (const auto& c : s->cams) px_total += (int64_t)c.width * c.height;
  const float* state[7] = {s->ghat, s->dhat, s->am, s->av, s->x_alt, s->dbuf, s->gacc};
  int64_t b = 12 * px_total + 4 * PN + 8 * kMaxLossViews;
  for (const float* v : state) b += v ? 4 * PN : 0;
  for (const auto& v : s->vb)
    if (v.ready)
      b += view_scratch_bytes(s->N, s->max_px, s->max_tiles) + pair_bytes(v.pair_cap, s->max_tiles, s->N) +
           (v.blend_cap - v.pair_cap) * (36 + 16);
  *bytes = b;
  return GS3_OK;
}

gs3_status gs3_trim_cache(void) {
  std::lock_guard<std::mutex> lk(mem::mu);
  mem::trim_locked(-1);
  return GS3_OK;
}

gs3_status gs3_scene_params(gs3_scene* s, float** p) {
  GS3_TRY(check_scene(s));
  if (!p) return fail(GS3_EINVAL, "output pointer is NULL");
  *p = s->x;
  return GS3_OK;
}

gs3_status gs3_scene_set_params(gs3_scene* s, const float* params_dev, hipStream_t st) {
  GS3_TRY(check_scene(s));
  CallEnd end_{s, st};
  if (!params_dev) return fail(GS3_EINVAL, "params_dev is NULL");
  GS3_HIP(hipMemcpyAsync(s->x, params_dev, (size_t)s->P * s->N * sizeof(float), hipMemcpyDeviceToDevice, st));
  return finish(s, st);
}

gs3_status gs3_scene_sync(gs3_scene* s) {
  GS3_TRY(check_scene(s));
  GS3_HIP(hipEventSynchronize(s->done_ev));
  GS3_HIP(hipGetLastError());
  volatile uint32_t* flag = s->host_u32 + 1;
  if (*flag) {
    *flag = 0u;
    return fail(GS3_ENONFINITE, "a gradient entry or an updated parameter was not finite since the last sync");
  }
  return GS3_OK;
}

gs3_status gs3_render(gs3_scene* s, int32_t cam, float* rgb, hipStream_t st) {
  GS3_TRY(check_scene(s));
  CallEnd end_{s, st};
  GS3_TRY(check_cam(s, cam));
  if (!rgb) return fail(GS3_EINVAL, "rgb_dev is NULL");
  GS3_TRY(bin_view(s, s->vb[0], cam, st));
  blend_fwd(s, single(), st, rgb);
  return finish(s, st);
}

gs3_status gs3_render_noalloc(int64_t n_gaussians, int32_t sh_degree, const float* params_dev,
                              const gs3_camera* camera, const float background[3], float* rgb_dev, hipStream_t st) {
  if (n_gaussians < 1 || n_gaussians > 0x7fffffffLL) return fail(GS3_EINVAL, "n_gaussians must be in [1, 2^31)");
  if (params_for(sh_degree) < 0) return fail(GS3_EINVAL, "sh_degree must be 0..3");
  if (!params_dev || !camera || !rgb_dev) return fail(GS3_EINVAL, "params_dev, camera and rgb_dev must not be NULL");
  const gs3_camera& c = *camera;
  if (c.width < 1 || c.height < 1 || c.width > kMaxSide || c.height > kMaxSide)
    return fail(GS3_EINVAL, "camera has an invalid size");
  if (!(c.fx > 0.f) || !(c.fy > 0.f)) return fail(GS3_EINVAL, "camera has fx/fy <= 0");
  const CamDev cd = make_cam(c);
  const int64_t px = (int64_t)c.width * c.height, tiles = (int64_t)cd.tiles_x * cd.tiles_y;
  // the largest pair capacity whose buffers fit beside the per-Gaussian and
  // per-pixel ones (none when even those do not fit)
  if (render_bytes(n_gaussians, px, tiles, 0) > kStaticScratchBytes)
    return fail(GS3_EINVAL, std::to_string(n_gaussians) + " Gaussians at " + std::to_string(c.width) + "x" +
                                std::to_string(c.height) + " do not fit the " + std::to_string(kStaticScratchBytes >> 20) +
                                " MiB static scratch");
  int64_t lo = 0, hi = (int64_t)(kStaticScratchBytes / 16);
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (render_bytes(n_gaussians, px, tiles, mid) <= kStaticScratchBytes) lo = mid;
    else hi = mid - 1;
  }
  void* base = nullptr;
  GS3_TRY(static_scratch(&base));
  gs3_scene t;
  t.N = n_gaussians;
  t.deg = sh_degree;
  t.K = (sh_degree + 1) * (sh_degree + 1);
  t.P = params_for(sh_degree);
  t.n_cams = 1;
  t.max_px = px;
  t.max_tiles = (int)tiles;
  t.x = const_cast<float*>(params_dev);  // only read by the projection
  for (int k = 0; k < 3; ++k) t.bg[k] = background ? background[k] : 0.f;
  t.fixed_scratch = true;
  ViewBufs& v = t.vb[0];
  Carver carver{(char*)base, kStaticScratchBytes};
  carve_render<true>(carver, v, n_gaussians, px, tiles, lo);
  v.pair_cap = lo;
  v.blend_cap = lo;
  v.rtmp_bytes = radix_temp_bytes(std::max<int64_t>(lo, n_gaussians));
  v.owner_blocks = lo / 256 + 1;
  v.ready = true;
  GS3_TRY(bin_camera(&t, v, c, -1, st));
  blend_fwd(&t, single(), st, rgb_dev);
  GS3_LAUNCHED();
  return GS3_OK;
}

gs3_status gs3_bin(gs3_scene* s, int32_t cam, uint64_t* keys, uint32_t* gids, uint32_t* ranges, int64_t capacity,
                   int64_t* n_pairs, hipStream_t st) {
  GS3_TRY(check_scene(s));
  CallEnd end_{s, st};
  GS3_TRY(check_cam(s, cam));
  if (!n_pairs) return fail(GS3_EINVAL, "n_pairs is NULL");
  ViewBufs& v = s->vb[0];
  GS3_TRY(bin_view(s, v, cam, st));
  *n_pairs = v.n_pairs;
  if ((keys || gids) && v.n_pairs > capacity)
    return fail(GS3_EINVAL, "pair count " + std::to_string(v.n_pairs) + " exceeds capacity");
  if (keys) launch_make_keys(v.sorted_tile, v.sorted_gid, v.depth_key, v.n_pairs, keys, st);
  if (gids && v.n_pairs > 0)
    GS3_HIP(hipMemcpyAsync(gids, v.sorted_gid, v.n_pairs * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
  if (ranges) {
    const CamDev cd = make_cam(s->cams[cam]);
    GS3_HIP(hipMemcpyAsync(ranges, v.ranges, (size_t)cd.tiles_x * cd.tiles_y * sizeof(uint2),
                           hipMemcpyDeviceToDevice, st));
  }
  GS3_TRY(finish(s, st));
  GS3_HIP(hipStreamSynchronize(st));
  return GS3_OK;
}

namespace {

// The gradient of Eq. objective over views cams[0..n) into grad (mode 0);
// with `fuse` set, the last batch's projection backward applies the update
// of Algorithm 1 instead of writing its gradient (the earlier batches' sum
// is in grad, passed to the update as the accumulated part).  Views go in
// batches of up to GS3_MAX_VIEWS: each view is binned into a slot of its
// own, then one blend launch, one backward launch and one projection
// backward cover the whole batch.
// Views cams[c0 .. c0 + count) as one batch in slots [base, base + count):
// binning, render, loss cotangent (scale: the loss weight of one view) and
// backward, leaving the partials for the chain rule; each view's loss goes to
// s->dsum[c0 + k] when `loss` is set.
gs3_status grad_batch(gs3_scene* s, const int32_t* cams, int c0, int count, int base, float scale, bool loss,
                      Entries& E, hipStream_t st) {
  E.n = count;
  for (int k = 0; k < count; ++k) {
    E.b[k] = E.e[k] = base + k;
    GS3_TRY(bin_view(s, s->vb[base + k], cams[c0 + k], st));
  }
  blend_fwd(s, E, st);
  for (int k = 0; k < count; ++k) {
    ViewBufs& v = s->vb[base + k];
    int np = 0;
    auto pl = prof::begin("loss", st);
    launch_loss_grad(v.img, target_of(s, v.cam), v.cd.width, v.cd.height, s->lam, scale, v.cot, v.ssim_tmp, v.dpart,
                     &np, st);
    prof::end(pl, st);
    if (loss) launch_sum_partials(v.dpart, np, s->dsum + c0 + k, st);
  }
  blend_bwd(s, E, st);
  return GS3_OK;
}

// The loss of n_cams views whose per-view sums grad_batch left in s->dsum.
gs3_status read_loss(gs3_scene* s, int32_t n_cams, double* loss_out, hipStream_t st) {
  GS3_HIP(hipMemcpyAsync(s->host_f64, s->dsum, sizeof(double) * n_cams, hipMemcpyDeviceToHost, st));
  GS3_HIP(hipStreamSynchronize(st));
  double tot = 0.0;
  for (int k = 0; k < n_cams; ++k) tot += s->host_f64[k];
  *loss_out = tot / (2.0 * (double)s->m_comp);
  return GS3_OK;
}

float grad_scale(const gs3_scene* s, int32_t n_cams) {
  return (float)((double)s->n_train / (2.0 * (double)s->m_comp * n_cams));
}
float hvp_scale(const gs3_scene* s, int32_t n_cams, int32_t nu) {
  return (float)((double)s->n_train / ((double)s->m_comp * n_cams * nu));
}

gs3_status grad_views(gs3_scene* s, const int32_t* cams, int32_t n_cams, float* grad, double* loss_out,
                      const FusedTr* fuse, hipStream_t st) {
  const float scale = grad_scale(s, n_cams);
  GS3_TRY(need_slots(s, std::min<int>(n_cams, GS3_MAX_VIEWS)));
  for (int c0 = 0; c0 < n_cams; c0 += GS3_MAX_VIEWS) {
    Entries E;
    GS3_TRY(grad_batch(s, cams, c0, std::min<int>(GS3_MAX_VIEWS, n_cams - c0), 0, scale, loss_out != nullptr, E, st));
    if (fuse && c0 + E.n == n_cams) {
      FusedTr ft = *fuse;
      ft.gacc = c0 > 0 ? grad : nullptr;
      project_bwd(s, E, 2, 0, 0, 0.f, nullptr, st, ft);
    } else {
      project_bwd(s, E, 0, c0 > 0, 0, 0.f, grad, st);
    }
    GS3_LAUNCHED();
  }
  if (loss_out) GS3_TRY(read_loss(s, n_cams, loss_out, st));
  return GS3_OK;
}

// Hutchinson entries q0 .. q0 + count (entry q: probe q mod nu of view
// cams[q / nu]) as one batch in slots [base, base + count): a view is binned
// once per batch (into the slot of its first probe), every entry gets its
// own tangent records, images and partials, and one JVP blend launch and
// one backward launch cover the batch; the pair sums and the chain rule are
// left to the caller.
gs3_status hvp_batch(gs3_scene* s, const int32_t* cams, int32_t nu, uint64_t seed, int64_t q0, int count, int base,
                     Entries& E, hipStream_t st) {
  E.n = count;
  for (int k = 0; k < count; ++k) {
    const int64_t q = q0 + k;
    const int j = (int)(q / nu);
    E.e[k] = base + k;
    E.probe[k] = (uint32_t)(q % nu);
    // the view's binning: in this batch's slot of its first entry
    const int first = (int)(std::max<int64_t>(q0, (int64_t)j * nu) - q0);
    E.b[k] = base + first;
    if (first == k) {
      GS3_TRY(bin_view(s, s->vb[base + k], cams[j], st));
    } else {
      GS3_TRY(ensure_blend(s, s->vb[base + k], s->vb[base + first].n_pairs, &st));
    }
  }
  for (int k = 0; k < count; ++k)
    project_jvp(s, s->vb[E.b[k]], s->vb[E.e[k]], PROBE_HASH, seed, E.probe[k], nullptr, st);
  blend_jvp(s, E, st);
  for (int k = 0; k < count; ++k) {
    ViewBufs& v = s->vb[E.e[k]];
    const ViewBufs& b = s->vb[E.b[k]];
    auto pl = prof::begin("loss", st);
    launch_loss_gn(v.img, target_of(s, b.cam), v.tan_img, b.cd.width, b.cd.height, s->lam, 1.f, v.cot, v.ssim_tmp, st);
    prof::end(pl, st);
  }
  blend_bwd(s, E, st);
  return GS3_OK;
}

// D_t of Hutchinson over views cams[0..n) and nu probes, in batches of up to
// GS3_MAX_VIEWS entries, each closed by one projection backward (mode 1).
gs3_status hvp_views(gs3_scene* s, const int32_t* cams, int32_t n_cams, int32_t nu, uint64_t seed, float* D,
                     hipStream_t st) {
  launch_fill_f32(D, (int64_t)s->P * s->N, 0.f, st);
  const float scale = hvp_scale(s, n_cams, nu);
  const int64_t total = (int64_t)n_cams * nu;
  GS3_TRY(need_slots(s, (int)std::min<int64_t>(total, GS3_MAX_VIEWS)));
  for (int64_t q0 = 0; q0 < total; q0 += GS3_MAX_VIEWS) {
    Entries E;
    GS3_TRY(hvp_batch(s, cams, nu, seed, q0, (int)std::min<int64_t>(GS3_MAX_VIEWS, total - q0), 0, E, st));
    project_bwd(s, E, 1, 0, seed, scale, D, st);
    GS3_LAUNCHED();
  }
  return GS3_OK;
}

gs3_status check_views(gs3_scene* s, const int32_t* cams, int32_t n_cams) {
  if (!cams || n_cams < 1 || n_cams > kMaxLossViews) return fail(GS3_EINVAL, "need 1..4096 camera indices");
  for (int k = 0; k < n_cams; ++k) GS3_TRY(check_cam(s, cams[k]));
  return GS3_OK;
}

gs3_status check_hparams(const gs3_tr_hparams* hp) {
  if (!hp) return fail(GS3_EINVAL, "hp must not be NULL");
  if (!(hp->theta1 >= 0.f && hp->theta1 < 1.f && hp->theta2 >= 0.f && hp->theta2 < 1.f))
    return fail(GS3_EINVAL, "theta1 and theta2 must be in [0, 1)");
  if (!(hp->epsilon > 0.f) || !std::isfinite(hp->epsilon)) return fail(GS3_EINVAL, "epsilon must be > 0 and finite");
  if (hp->variant & ~(GS3_TR_MEAN_EXACT | GS3_TR_SECOND_ORDER | GS3_TR_SH_JOINT))
    return fail(GS3_EINVAL, "unknown variant bits");
  return GS3_OK;
}

}  // namespace

gs3_status gs3_grad(gs3_scene* s, const int32_t* cams, int32_t n_cams, float* grad, double* loss_out,
                    hipStream_t st) {
  GS3_TRY(check_scene(s));
  CallEnd end_{s, st};
  GS3_TRY(check_views(s, cams, n_cams));
  if (!grad) return fail(GS3_EINVAL, "grad_dev is NULL");
  GS3_TRY(grad_views(s, cams, n_cams, grad, loss_out, nullptr, st));
  return finish(s, st);
}

gs3_status gs3_hvp_diag(gs3_scene* s, const int32_t* cams, int32_t n_cams, int32_t nu, uint64_t seed, float* D,
                        hipStream_t st) {
  GS3_TRY(check_scene(s));
  CallEnd end_{s, st};
  GS3_TRY(check_views(s, cams, n_cams));
  if (nu < 1) return fail(GS3_EINVAL, "nu must be >= 1");
  if (!D) return fail(GS3_EINVAL, "D_dev is NULL");
  GS3_TRY(hvp_views(s, cams, n_cams, nu, seed, D, st));
  return finish(s, st);
}

gs3_status gs3_tr_iteration(gs3_scene* s, const int32_t* cams1, int32_t n1, const int32_t* cams2, int32_t n2,
                            int32_t nu, uint64_t seed, const gs3_tr_hparams* hp, double* loss_out, hipStream_t st) {
  GS3_TRY(check_scene(s));
  CallEnd end_{s, st};
  GS3_TRY(check_views(s, cams1, n1));
  if (n2 < 0 || (n2 > 0 && nu < 1)) return fail(GS3_EINVAL, "n2 must be >= 0 and nu >= 1 when n2 > 0");
  if (n2 > 0) GS3_TRY(check_views(s, cams2, n2));
  GS3_TRY(check_hparams(hp));
  GS3_TRY(need_fused_state(s, st));
  FusedTr ft;
  ft.x_out = s->x_alt;
  ft.ghat = s->ghat;
  ft.dhat = s->dhat;
  ft.nonfinite = s->host_u32 + 1;
  ft.a = TrArgs{hp->theta1, hp->theta2, hp->epsilon, n2 > 0, hp->variant};
  const int64_t nh = n2 > 0 ? (int64_t)n2 * nu : 0;
  if (n2 > 0 && nh + n1 <= GS3_MAX_VIEWS) {
    // one batch: the Hutchinson entries in slots [0, nh), the gradient views
    // after them, and one update launch that sums D_t in registers (D_t never
    // goes through device memory).  The two parts share no buffer until the
    // update, so the probe entries run on the second stream beside the
    // gradient views (much of either part is latency-bound: pair sums,
    // emission, radix passes), forked after the caller's earlier work and
    // joined before the update.
    GS3_TRY(need_slots(s, (int)(nh + n1)));
    GS3_TRY(need_aux(s));
    GS3_HIP(hipEventRecord(s->aux.fork, st));
    GS3_HIP(hipStreamWaitEvent(s->aux.st, s->aux.fork, 0));
    // on every exit from here the caller's stream waits for the second one,
    // so the scene's completion event covers the probe work
    struct Join {
      gs3_scene* s;
      hipStream_t st;
      ~Join() {
        (void)hipEventRecord(s->aux.join, s->aux.st);
        (void)hipStreamWaitEvent(st, s->aux.join, 0);
      }
    };
    Entries H, C;
    {
      Join join_{s, st};
      GS3_TRY(hvp_batch(s, cams2, nu, seed, 0, (int)nh, 0, H, s->aux.st));
      GS3_TRY(grad_batch(s, cams1, 0, n1, (int)nh, grad_scale(s, n1), loss_out != nullptr, C, st));
    }
    for (int k = 0; k < H.n; ++k) {
      C.b[C.n + k] = H.b[k];
      C.e[C.n + k] = H.e[k];
      C.probe[C.n + k] = H.probe[k];
    }
    C.n += H.n;
    project_bwd(s, C, 2, 0, seed, 0.f, nullptr, st, ft, H.n, hvp_scale(s, n2, nu));
    GS3_LAUNCHED();
    if (loss_out) GS3_TRY(read_loss(s, n1, loss_out, st));
  } else {
    if (n2 > 0) {
      if (!s->dbuf) GS3_TRY(dalloc(&s->dbuf, (size_t)s->P * s->N));
      GS3_TRY(hvp_views(s, cams2, n2, nu, seed, s->dbuf, st));
      ft.D = s->dbuf;
    }
    GS3_TRY(grad_views(s, cams1, n1, s->gacc, loss_out, &ft, st));
  }
  std::swap(s->x, s->x_alt);
  return finish(s, st);
}

gs3_status gs3_tr_step(gs3_scene* s, const float* grad, const float* D, const gs3_tr_hparams* hp, float* eta_out,
                       float* dx_out, hipStream_t st) {
  GS3_TRY(check_scene(s));
  CallEnd end_{s, st};
  if (!grad) return fail(GS3_EINVAL, "grad_dev must not be NULL");
  GS3_TRY(check_hparams(hp));
  GS3_TRY(need_tr_state(s, st));
  TrArgs a{hp->theta1, hp->theta2, hp->epsilon, D != nullptr, hp->variant};
  auto p = prof::begin("tr_step", st);
  launch_tr_step(s->x, grad, s->ghat, s->dhat, D, s->N, s->deg, a, eta_out, dx_out, s->host_u32 + 1, st);
  prof::end(p, st, s->N, (int64_t)s->P * s->N);
  return finish(s, st);
}

static gs3_status adam_common(gs3_scene* s, const float* grad, const float* lr, int32_t step, float epsilon,
                              hipStream_t st) {
  GS3_TRY(check_scene(s));
  CallEnd end_{s, st};
  if (!grad || !lr) return fail(GS3_EINVAL, "grad_dev and lr_per_group must not be NULL");
  if (step < 1) return fail(GS3_EINVAL, "step is 1-based");
  AdamArgs a;
  for (int r = 0; r < 64; ++r) a.lr_row[r] = 0.f;
  for (int r = 0; r < s->P; ++r) {
    int grp;
    if (r < 3) grp = 0;          // mean
    else if (r < 6) grp = 4;     // scale
    else if (r < 10) grp = 5;    // rotation
    else if (r == 10) grp = 3;   // opacity
    else if (r < 14) grp = 1;    // SH DC
    else grp = 2;                // SH rest
    a.lr_row[r] = lr[grp];
  }
  a.b1 = 0.9f;
  a.b2 = 0.999f;
  a.eps = 1e-15f;
  a.bc1 = (float)(1.0 - std::pow(0.9, step));
  a.bc2 = (float)(1.0 - std::pow(0.999, step));
  a.epsilon = epsilon;
  auto p = prof::begin("adam_step", st);
  GS3_TRY(need_adam_state(s, st));
  launch_adam_step(s->x, grad, s->am, s->av, s->N, s->deg, a, s->host_u32 + 1, st);
  prof::end(p, st, s->N, (int64_t)s->P * s->N);
  return finish(s, st);
}

gs3_status gs3_adam_step(gs3_scene* s, const float* grad, const float* lr, int32_t step, hipStream_t st) {
  return adam_common(s, grad, lr, step, 0.f, st);
}

gs3_status gs3_adam_tr_step(gs3_scene* s, const float* grad, const float* lr, int32_t step, float epsilon,
                            hipStream_t st) {
  if (!(epsilon > 0.f)) return fail(GS3_EINVAL, "epsilon must be > 0");
  return adam_common(s, grad, lr, step, epsilon, st);
}

gs3_status gs3_psnr(gs3_scene* s, int32_t cam, double* out, hipStream_t st) {
  GS3_TRY(check_scene(s));
  CallEnd end_{s, st};
  GS3_TRY(check_cam(s, cam));
  if (!out) return fail(GS3_EINVAL, "psnr_out is NULL");
  ViewBufs& v = s->vb[0];
  GS3_TRY(bin_view(s, v, cam, st));
  blend_fwd(s, single(), st);
  int np = 0;
  const int64_t n = (int64_t)v.cd.width * v.cd.height * 3;
  launch_sq_err(v.img, target_of(s, cam), n, v.dpart, &np, st);
  launch_sum_partials(v.dpart, np, s->dsum, st);
  GS3_HIP(hipMemcpyAsync(s->host_f64, s->dsum, sizeof(double), hipMemcpyDeviceToHost, st));
  GS3_HIP(hipStreamSynchronize(st));
  const double mse = s->host_f64[0] / (double)n;
  *out = mse > 0.0 ? 10.0 * std::log10(1.0 / mse) : INFINITY;
  return finish(s, st);
}

gs3_status gs3_render_vjp(gs3_scene* s, int32_t cam, const float* cot, float* grad, hipStream_t st) {
  GS3_TRY(check_scene(s));
  CallEnd end_{s, st};
  GS3_TRY(check_cam(s, cam));
  if (!cot || !grad) return fail(GS3_EINVAL, "cot_dev and grad_dev must not be NULL");
  GS3_TRY(bin_view(s, s->vb[0], cam, st));
  blend_fwd(s, single(), st);
  blend_bwd(s, single(), st, cot);
  project_bwd(s, single(), 0, 0, 0, 0.f, grad, st);
  return finish(s, st);
}

gs3_status gs3_render_jvp(gs3_scene* s, int32_t cam, const float* tangent, float* rgb, float* tan, hipStream_t st) {
  GS3_TRY(check_scene(s));
  CallEnd end_{s, st};
  GS3_TRY(check_cam(s, cam));
  if (!tangent || !rgb || !tan) return fail(GS3_EINVAL, "tangent_dev, rgb_dev and tan_dev must not be NULL");
  ViewBufs& v = s->vb[0];
  GS3_TRY(bin_view(s, v, cam, st));
  project_jvp(s, v, v, PROBE_ARRAY, 0, 0, tangent, st);
  blend_jvp(s, single(), st, rgb, tan);
  return finish(s, st);
}

gs3_status gs3_scene_export(gs3_scene* s, float* x, float* ghat, float* dhat, float* m, float* v, hipStream_t st) {
  GS3_TRY(check_scene(s));
  CallEnd end_{s, st};
  const size_t bytes = (size_t)s->P * s->N * sizeof(float);
  const float* src[5] = {s->x, s->ghat, s->dhat, s->am, s->av};
  float* dst[5] = {x, ghat, dhat, m, v};
  for (int i = 0; i < 5; ++i) {
    if (!dst[i]) continue;
    if (src[i]) {
      GS3_HIP(hipMemcpyAsync(dst[i], src[i], bytes, hipMemcpyDeviceToDevice, st));
    } else {
      launch_fill_f32(dst[i], (int64_t)s->P * s->N, 0.f, st);  // state not created yet: zero
    }
  }
  return finish(s, st);
}

gs3_status gs3_scene_import(gs3_scene* s, const float* x, const float* ghat, const float* dhat, const float* m,
                            const float* v, hipStream_t st) {
  GS3_TRY(check_scene(s));
  CallEnd end_{s, st};
  const size_t bytes = (size_t)s->P * s->N * sizeof(float);
  if (ghat || dhat) GS3_TRY(need_tr_state(s, st));
  if (m || v) GS3_TRY(need_adam_state(s, st));
  float* dst[5] = {s->x, s->ghat, s->dhat, s->am, s->av};
  const float* src[5] = {x, ghat, dhat, m, v};
  for (int i = 0; i < 5; ++i)
    if (src[i]) GS3_HIP(hipMemcpyAsync(dst[i], src[i], bytes, hipMemcpyDeviceToDevice, st));
  return finish(s, st);
}

gs3_status gs3_profile_enable(const char* names) {
  std::lock_guard<std::mutex> lk(prof::mu);
  if (!names || !*names) {
    prof::active.store(false);
    prof::names.clear();
    return GS3_OK;
  }
  if (!prof::ctr) {
    if (hipMalloc((void**)&prof::ctr, sizeof(unsigned long long) * prof::kSlotWords * prof::kSlots) != hipSuccess) {
      prof::ctr = nullptr;
      return fail(GS3_ENOMEM, "profiler counter allocation failed");
    }
    GS3_HIP(hipMemset(prof::ctr, 0, sizeof(unsigned long long) * prof::kSlotWords * prof::kSlots));
  }
  prof::names = "," + std::string(names) + ",";
  prof::active.store(true);
  return GS3_OK;
}

gs3_status gs3_profile_count(int32_t on) {
  std::lock_guard<std::mutex> lk(prof::mu);
  prof::counting = on != 0;
  return GS3_OK;
}

gs3_status gs3_profile_reset(void) {
  std::lock_guard<std::mutex> lk(prof::mu);
  for (auto& e : prof::entries)
    if (e.b) (void)hipEventSynchronize(e.b);
  prof::clear_locked();
  if (prof::ctr) GS3_HIP(hipMemset(prof::ctr, 0, sizeof(unsigned long long) * prof::kSlotWords * prof::kSlots));
  return GS3_OK;
}

gs3_status gs3_profile_read(const char* name, int64_t* launches, double* total_ms, int64_t* work0, int64_t* work1) {
  if (!name) return fail(GS3_EINVAL, "name is NULL");
  std::lock_guard<std::mutex> lk(prof::mu);
  int64_t n = 0, w0 = 0, w1 = 0;
  double ms = 0.0;
  std::vector<unsigned long long> host;
  bool need_ctr = false;
  for (auto& e : prof::entries)
    if (e.name == name) {
      GS3_HIP(hipEventSynchronize(e.b));
      float t = 0.f;
      GS3_HIP(hipEventElapsedTime(&t, e.a, e.b));
      ms += t;
      ++n;
      w0 += e.w0;
      w1 += e.w1;
      need_ctr |= e.slot >= 0;
    }
  if (need_ctr) {
    host.resize(prof::kSlotWords * (size_t)prof::slots_used);
    if (!host.empty())
      GS3_HIP(hipMemcpy(host.data(), prof::ctr, host.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    for (auto& e : prof::entries)
      if (e.name == name && e.slot >= 0)
        for (int k = 0; k < GS3_PROF_SUB; ++k) {
          w0 += (int64_t)host[prof::kSlotWords * e.slot + 2 * k];
          w1 += (int64_t)host[prof::kSlotWords * e.slot + 2 * k + 1];
        }
  }
  if (launches) *launches = n;
  if (total_ms) *total_ms = ms;
  if (work0) *work0 = w0;
  if (work1) *work1 = w1;
  return GS3_OK;
}

}  // extern "C"
