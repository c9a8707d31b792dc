// C-ABI of the SGM library (declared in include/sgm.h): argument validation,
// context and scratch management, stage calls, and the batched
// sgm_submit / sgm_poll path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/sgm.h"
#include "sgm_kernels.h"

using namespace sgmk;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(SGM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int popcount8(uint32_t m) { return __builtin_popcount(m & 0xFFu); }

// Horizontal cost source of shapes without a tuned or context schedule:
// Census windows where a 64-lane row holds four disparities per lane
// (D in (192, 256]; measured faster on MI355X), the cost volume elsewhere
// (with one disparity pair per lane the window costs more time on the row's
// dependent chain than the volume reads it saves).
int default_hcosts(const sgm_params &p, int hlps) {
  return hlps == 64 && 16 * agg_k(p.max_disp) / hlps == 4 ? SGM_HCOSTS_CODES : SGM_HCOSTS_VOLUME;
}

int validate(const sgm_params *p) {
  if (!p) return fail(SGM_EINVAL, "params is null");
  if (p->width < 1 || p->height < 1 || p->width > 16384 || p->height > 16384)
    return fail(SGM_EINVAL, "width/height must be in [1, 16384] (got %d x %d)", p->width, p->height);
  if (p->max_disp < 1 || p->max_disp > 256)
    return fail(SGM_EINVAL, "max_disp must be in [1, 256] (got %d)", p->max_disp);
  if (p->census_w < 1 || p->census_h < 1 || !(p->census_w & 1) || !(p->census_h & 1))
    return fail(SGM_EINVAL, "census window must have odd sides >= 1 (got %d x %d)", p->census_w,
                p->census_h);
  if (p->cost != SGM_COST_CENSUS && p->cost != SGM_COST_SAD)
    return fail(SGM_EINVAL, "cost must be SGM_COST_CENSUS or SGM_COST_SAD (got %u)", p->cost);
  const long nb = (long)p->census_w * p->census_h - 1;
  if (p->cost == SGM_COST_CENSUS && (nb < 1 || nb > 64))
    return fail(SGM_EINVAL, "census_w*census_h-1 must be in [1, 64] (got %ld)", nb);
  if (p->cost == SGM_COST_SAD && (nb + 1) * 255 > 65535)
    return fail(SGM_EINVAL, "SAD window too large: census_w*census_h*255 must be <= 65535");
  if (p->path_mask == 0 || (p->path_mask & ~0xFFu))
    return fail(SGM_EINVAL, "path_mask must be a nonzero subset of the 8 directions (got 0x%x)",
                p->path_mask);
  if (p->p1 > p->p2) return fail(SGM_EINVAL, "p1 must be <= p2 (got %u > %u)", p->p1, p->p2);
  const long cmax = p->cost == SGM_COST_SAD ? (nb + 1) * 255 : nb;
  if ((long)popcount8(p->path_mask) * (cmax + p->p2) > 65535)
    return fail(SGM_EINVAL, "paths*(Cmax+p2) = %ld exceeds 65535: S could overflow 16 bits",
                (long)popcount8(p->path_mask) * (cmax + p->p2));
  if (p->lr_check != 0 && p->lr_check != 1) return fail(SGM_EINVAL, "lr_check must be 0 or 1");
  if (p->lr_max_diff < 0) return fail(SGM_EINVAL, "lr_max_diff must be >= 0");
  if (p->median != 0 && p->median != 3 && p->median != 5)
    return fail(SGM_EINVAL, "median must be 0, 3 or 5 (got %d)", p->median);
  if (p->invalid < p->max_disp)
    return fail(SGM_EINVAL, "invalid (%u) must be >= max_disp (%d)", p->invalid, p->max_disp);
  // the kernels address one path-cost volume (padded disparity stride, up to
  // 2 bytes per cell) with 32-bit offsets
  const int64_t dp = 16 * (int64_t)agg_k(p->max_disp);
  if ((int64_t)p->width * p->height * dp * 2 >= (int64_t)1 << 32)
    return fail(SGM_EINVAL, "image too large: width*height*%lld*2 bytes must stay below 4 GiB",
                (long long)dp);
  return SGM_OK;
}

int nbits_of(const sgm_params &p) { return p.census_w * p.census_h - 1; }
bool is_sad(const sgm_params &p) { return p.cost == SGM_COST_SAD; }
// Largest matching cost: N_b for Census/Hamming, window * 255 for SAD.
int cmax_of(const sgm_params &p) { return is_sad(p) ? p.census_w * p.census_h * 255 : nbits_of(p); }
// Disparities per lane of the aggregation / selection kernels, and the
// padded disparity stride of the internal volumes.
int k_of(const sgm_params &p) { return agg_k(p.max_disp); }
int dp_of(const sgm_params &p) { return 16 * k_of(p); }
// Path costs fit in 8 bits when Cmax + P2 <= 255 (L_r <= C + P2).
int lr_bytes_of(const sgm_params &p) { return cmax_of(p) + p.p2 <= 255 ? 1 : 2; }

int fill_dirs(uint32_t mask, int *dirs) {
  int n = 0;
  for (int d = 0; d < 8; ++d)
    if (mask & (1u << d)) dirs[n++] = d;
  return n;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Device scratch held by a context: one growable buffer for stage calls and
// a cache of idle batch blocks.
struct Block {
  void *ptr = nullptr;
  size_t bytes = 0;
};

struct StageEvents {
  int stage;
  int launches;
  hipEvent_t begin, end;
};

// Polls (each a device-scope load after a short sleep, ~1-2 us) before a
// stripe's wait for its neighbour's edge gives up: seconds, far beyond any
// legitimate wait.
constexpr int kStripePolls = 1 << 22;

// Bounds of the stripe passes' waits for a neighbour's edge (sgm_set_stripe_wait).
struct StripeWait {
  int max_polls = kStripePolls;
  int withhold = 0;
};

struct Batch {
  hipEvent_t done = nullptr;
  Block mem;
  int stream = 0;
  int sync_frames = 0;  // frames with stripe sync words at the start of mem (two-pass frames' slots)
  uint32_t *sync_host = nullptr;  // pinned copy of those words, written by the batch's last copy
  std::vector<StageEvents> prof;  // empty unless profiling
  std::vector<hipEvent_t> joins;  // fork / join events of a batch split over streams
};

}  // namespace

struct ShapeKey {
  int W, H, D;
  uint32_t mask;
  int lb;
  bool operator<(const ShapeKey &o) const {
    return std::tie(W, H, D, mask, lb) < std::tie(o.W, o.H, o.D, o.mask, o.lb);
  }
};

struct sgm_ctx {
  int device = 0;
  size_t budget = 0;
  std::mutex mu;
  Block stage;                  // stage-call scratch
  std::vector<Block> idle;      // finished batch blocks kept for reuse
  std::map<uint64_t, Batch> inflight;
  uint64_t next_ticket = 1;
  static constexpr int kStreams = 8;
  hipStream_t streams[kStreams] = {};
  int nstreams = 4;  // streams in use (round robin)
  int next_stream = 0;
  int split = 4;     // streams a batch's frames are spread over when no other batch is in flight
  bool profiling = false;
  bool graphs = false;
  std::map<std::string, hipGraphExec_t> graph_cache;  // by batch composition
  uint64_t graph_hits = 0, graph_misses = 0;
  sgm_schedule dflt{};                     // h_lanes 0: library default
  std::map<ShapeKey, sgm_schedule> tuned;  // per-shape schedules (sgm_set_schedule / autotune)
  double stage_ms[SGM_NSTAGES] = {};
  uint64_t stage_count[SGM_NSTAGES] = {};
  void *static_scratch = nullptr;  // device address of `scratch` on this device
  StripeWait stripe_wait;          // sgm_set_stripe_wait
  // pinned host blocks of kSyncHostBytes for batches' sync words (reused)
  std::vector<uint32_t *> sync_pool;

  size_t held() const {
    size_t s = stage.bytes;
    for (auto &b : idle) s += b.bytes;
    for (auto &kv : inflight) s += kv.second.mem.bytes;
    return s;
  }
  size_t inflight_bytes() const {
    size_t s = 0;
    for (auto &kv : inflight) s += kv.second.mem.bytes;
    return s;
  }
};

// Fixed scratch of the allocation-free entry point (sgm_disparity_noalloc):
// one array per GPU, in the code object's device memory, held until the
// process ends.  Host code never passes `scratch` itself (on the host it is
// only a stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_addr;  // device -> address of `scratch` there

// Device address of `scratch` on `device` (which must be current), looked up
// once per device.
int static_scratch_of(int device, void **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it == g_scratch_addr.end()) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(SGM_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    it = g_scratch_addr.emplace(device, ptr).first;
  }
  *out = it->second;
  return SGM_OK;
}

size_t disparity_scratch_bytes(const sgm_params &p);
int enqueue_disparity(const sgm_params *p, const uint16_t *aggr, uint16_t *disp, void *v, hipStream_t s);

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Free idle batch blocks until `need` more bytes fit in the budget.
int make_room(sgm_ctx *c, size_t need) {
  while (c->held() + need > c->budget && !c->idle.empty()) {
    HIP_TRY(hipFree(c->idle.back().ptr));
    c->idle.pop_back();
  }
  return SGM_OK;
}

// Ensure the stage scratch holds `bytes`; work already enqueued on `s` may
// still use the old buffer, so the stream is drained before freeing it.
int stage_scratch(sgm_ctx *c, size_t bytes, hipStream_t s, void **out) {
  bytes = align256(bytes);
  if (c->stage.bytes < bytes) {
    const size_t old = c->stage.bytes;
    int rc = make_room(c, bytes - old);
    if (rc) return rc;
    if (c->held() - old + bytes > c->budget)
      return fail(SGM_ENOMEM, "stage scratch of %zu bytes exceeds the budget (%zu held of %zu)",
                  bytes, c->held(), c->budget);
    if (c->stage.ptr) {
      HIP_TRY(hipStreamSynchronize(s));
      HIP_TRY(hipFree(c->stage.ptr));
      c->stage = Block{};
    }
    HIP_TRY(hipMalloc(&c->stage.ptr, bytes));
    c->stage.bytes = bytes;
  }
  *out = c->stage.ptr;
  return SGM_OK;
}

int check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SGM_EHIP, "kernel launch: %s", hipGetErrorString(e));
  return SGM_OK;
}

// Check that a pointer is device memory of this device (or managed memory).
int check_dev_ptr(const void *ptr, int dev, const char *name) {
  if (!ptr) return fail(SGM_EINVAL, "%s is null", name);
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SGM_EINVAL, "%s is not a HIP allocation", name);
  }
  if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
    return fail(SGM_EINVAL, "%s is not device memory", name);
  if (a.type == hipMemoryTypeDevice && a.device != dev)
    return fail(SGM_EINVAL, "%s lives on device %d, context is on device %d", name, a.device, dev);
  return SGM_OK;
}

#define CHECK(expr)       \
  do {                    \
    int rc_ = (expr);     \
    if (rc_) return rc_;  \
  } while (0)

// ------------------------------------------------------ whole-frame plan

constexpr size_t kNoSync = ~(size_t)0;  // FramePlan::off_sync of a batch without a sync header
constexpr size_t kSyncHostBytes = 4096;  // pinned block of a batch's sync words (256 frames; larger batches get their own)

struct FramePlan {
  size_t off_cost, off_lr, off_dlr, off_dl, off_part, off_codes, bytes;
  // two-pass frames: S_D after the four path-cost slots, the stripes' edge
  // words and the frame's sync words
  size_t off_sd, off_bnd, off_sync;
};

// Scratch of one frame of a batch: the padded uint8 cost volume, the P
// padded path-cost volumes and the LR-checked map before the median.
// Bytes of the Census code records of sliding horizontal windows: 16 per
// pixel plus Dp records of padding before the first.
size_t code_records_bytes(const sgm_params &p) { return ((size_t)p.width * p.height + dp_of(p)) * 16; }

// Stripe columns of the two-pass schedule with `waves` waves per workgroup.
int stripe_cols(int waves) { return 4 * waves; }
int stripes_of(const sgm_params &p, int waves) { return (p.width + stripe_cols(waves) - 1) / stripe_cols(waves); }
size_t stripe_part_bytes(const sgm_params &p, int waves) {
  return (size_t)p.height * stripes_of(p, waves) * (stripe_cols(waves) + p.max_disp - 1) * 4;
}

FramePlan plan_frame(const sgm_params &p, size_t base, bool sweep, bool codes, int tp_waves = 0) {
  const size_t px = (size_t)p.width * p.height;
  const size_t dp = (size_t)dp_of(p);
  FramePlan f;
  f.off_cost = base;
  f.off_codes = 0;
  f.off_sd = f.off_bnd = f.off_sync = 0;
  if (sweep) {
    // Census codes of both views; D_L and D_R; the band-boundary carry rows;
    // the LR-checked map before the median
    f.off_lr = f.off_cost + align256(2 * px * 8);
    f.off_dlr = f.off_lr + align256(2 * px * 2) + align256((size_t)2 * (p.width + 2) * kSweepCarry);
    f.off_dl = f.off_part = 0;
    f.bytes = f.off_dlr + align256(px * 2) - base;
    return f;
  }
  // Census costs: padded uint8 [H][W][Dp]; SAD costs: padded uint16 [H][W][Dp]
  f.off_lr = f.off_cost + align256(is_sad(p) ? px * dp * 2 : px * dp);
  f.off_dlr = f.off_lr + align256(px * dp * (size_t)popcount8(p.path_mask) * lr_bytes_of(p));
  // D_L and the row segments' right-view keys (left-right check)
  f.off_dl = f.off_dlr + align256(px * 2);
  f.off_part = f.off_dl + align256(px * 2);
  size_t part = disp_part_bytes(p.width, p.height, p.max_disp);
  if (tp_waves) part = std::max(part, stripe_part_bytes(p, tp_waves));
  f.bytes = f.off_part + align256(part) - base;
  if (codes) {
    f.off_codes = base + f.bytes;
    f.bytes += align256(code_records_bytes(p));
  }
  if (tp_waves) {
    // the 8 path-cost slots' room holds the 4 slots and S_D (uint16)
    f.off_sd = f.off_lr + align256(px * dp * 4);
    f.off_bnd = base + f.bytes;
    f.bytes += align256((size_t)stripes_of(p, tp_waves) * p.height * dp * 4);
    // the sync words live in the batch's header (submit_impl sets off_sync)
  }
  return f;
}

// Enqueue census -> aggregation (costs recomputed from the Census codes) ->
// disparity selection -> median -> U/V maps for `n` frames on `s`, with the
// frames' scratch at `mem` laid out by plan_frame.
ShapeKey shape_key(const sgm_params &p) {
  return ShapeKey{p.width, p.height, p.max_disp, p.path_mask, lr_bytes_of(p)};
}

// Lanes per horizontal scanline for a frame: the tuned entry for its shape,
// else the context default, else a width rule measured on MI355X (wide
// lane groups pay off on long rows, where the horizontal paths' dependent
// chain is the critical path): 64 from 1024 columns, 32 from 400, else 16,
// stepping down to a layout that fits the disparity count.
int resolve_hlps(const sgm_ctx *c, const sgm_params &p) {
  int h = 0;
  auto it = c->tuned.find(shape_key(p));
  if (it != c->tuned.end()) h = it->second.h_lanes;
  if (h == 0) h = c->dflt.h_lanes;
  if (h == 0) h = p.width >= 1024 ? 64 : p.width >= 400 ? 32 : 16;
  const int K = k_of(p);
  for (int cand : {64, 32, 16})
    if (cand <= h && agg_hlps_ok(K, cand)) return cand;
  return 16;
}

// Frames the single-pass sweep handles: Census costs with codes of at most
// 32 bits, at most 64 disparities (16 lanes x 4), only forward paths, and
// path costs that fit 8 bits.
bool sweep_ok(const sgm_params &p) {
  return !is_sad(p) && nbits_of(p) <= 32 && p.max_disp <= 64 && (p.path_mask & ~0x55u) == 0 &&
         lr_bytes_of(p) == 1;
}

int resolve_sweep(const sgm_ctx *c, const sgm_params &p) {
  auto it = c->tuned.find(shape_key(p));
  const int want = it != c->tuned.end() ? it->second.sweep : c->dflt.sweep;
  return want && sweep_ok(p) ? 1 : 0;
}

// Horizontal costs from sliding Census windows: Census cost with uint8
// volumes, a 64-lane horizontal layout of 2 or 4 disparities per lane, and
// code records whose byte offsets fit 31 bits.
bool hcodes_ok(const sgm_params &p, int hlps) {
  return !is_sad(p) && lr_bytes_of(p) == 1 && agg_slide_ok(k_of(p), hlps) &&
         code_records_bytes(p) < ((size_t)1 << 31);
}

// SGM_HCOSTS_CODES or SGM_HCOSTS_VOLUME for a frame with `hlps` horizontal
// lanes: the tuned entry for its shape, else the context default, else the
// library's default.
int resolve_hcosts(const sgm_ctx *c, const sgm_params &p, int hlps) {
  auto it = c->tuned.find(shape_key(p));
  int want = it != c->tuned.end() ? it->second.h_costs : SGM_HCOSTS_DEFAULT;
  if (want == SGM_HCOSTS_DEFAULT) want = c->dflt.h_costs;
  if (want == SGM_HCOSTS_DEFAULT) want = default_hcosts(p, hlps);
  return want == SGM_HCOSTS_CODES && hcodes_ok(p, hlps) ? SGM_HCOSTS_CODES : SGM_HCOSTS_VOLUME;
}

// Frames the two-pass schedule handles: Census costs, all 8 paths, uint8
// path costs (the four per-direction slots and S_D share the room of eight
// uint8 slots).
bool twopass_ok(const sgm_params &p) { return !is_sad(p) && p.path_mask == 0xFF && lr_bytes_of(p) == 1; }

// Waves per stripe workgroup of the two-pass schedule for a frame, 0 when it
// does not run it: the tuned entry for its shape, else the context default,
// else the per-direction kernels.
int resolve_twopass(const sgm_ctx *c, const sgm_params &p) {
  auto it = c->tuned.find(shape_key(p));
  int want = it != c->tuned.end() ? it->second.two_pass : SGM_TWOPASS_DEFAULT;
  if (want == SGM_TWOPASS_DEFAULT) want = c->dflt.two_pass;
  if (!twopass_ok(p) || resolve_sweep(c, p)) return 0;
  return want == SGM_TWOPASS_WIDE ? 16 : want == SGM_TWOPASS_NARROW ? 8 : 0;
}

// Fewest stripes (workgroups of a stripe pass) in a batch for its two-pass
// frames to run as such: half the CUs of an MI355X.
constexpr int kMinStripes = 128;

// A fresh nonzero tag for a stripe launch's edge words.
uint32_t next_epoch() {
  static std::atomic<uint32_t> e{0};
  uint32_t v;
  do v = e.fetch_add(1) + 1; while (v == 0);
  return v;
}

// Disparity-selection block size for a frame (0: by the launch's block count).
int resolve_disp_threads(const sgm_ctx *c, const sgm_params &p) {
  auto it = c->tuned.find(shape_key(p));
  const int t = it != c->tuned.end() ? it->second.disp_threads : 0;
  return t ? t : c->dflt.disp_threads;
}

// Check one sgm_remap (sizes, pitches, device pointers) and build its job.
int check_remap(const sgm_remap &r, int i, int dev, RemapJob *out) {
  if (r.w < 1 || r.h < 1 || r.w > 16384 || r.h > 16384)
    return fail(SGM_EINVAL, "job %d: rectified size %dx%d outside 1..16384", i, r.w, r.h);
  if (r.src_w < 1 || r.src_h < 1 || r.src_w > 65535 || r.src_h > 65535)
    return fail(SGM_EINVAL, "job %d: raw size %dx%d outside 1..65535", i, r.src_w, r.src_h);
  if (r.src_pitch < r.src_w) return fail(SGM_EINVAL, "job %d: src_pitch < src_w", i);
  if (r.out_pitch < r.w) return fail(SGM_EINVAL, "job %d: out_pitch < w", i);
  const void *ptrs[4] = {r.src, r.map_x, r.map_y, r.out};
  const char *names[4] = {"src", "map_x", "map_y", "out"};
  char name[32];
  for (int k = 0; k < 4; ++k) {
    snprintf(name, sizeof(name), "job %d: %s", i, names[k]);
    CHECK(check_dev_ptr(ptrs[k], dev, name));
  }
  RemapJob j{};
  j.src = r.src;
  j.mx = r.map_x;
  j.my = r.map_y;
  j.out = r.out;
  j.src_pitch = r.src_pitch;
  j.out_pitch = r.out_pitch;
  j.src_w = r.src_w;
  j.src_h = r.src_h;
  j.w = r.w;
  j.h = r.h;
  j.vec = ((reinterpret_cast<uintptr_t>(r.map_x) | reinterpret_cast<uintptr_t>(r.map_y)) & 15) == 0;
  *out = j;
  return SGM_OK;
}

// Everything that decides a batch's launch sequence (kernels, grids, LDS):
// the frames' parameters and schedules, in order.
std::string composition_key(const sgm_frame *fr, int n, const std::vector<int> &hlps,
                            const std::vector<int> &sweep, const std::vector<RemapJob> &rect) {
  std::string k;
  char buf[160];
  for (const RemapJob &r : rect) {
    snprintf(buf, sizeof buf, "R%d,%d,%d,%d,%d;", r.w, r.h, r.src_w, r.src_h, r.vec);
    k += buf;
  }
  for (int i = 0; i < n; ++i) {
    const sgm_params &p = fr[i].p;
    // the cost kind and the path-cost width select other kernels and
    // argument layouts
    snprintf(buf, sizeof buf, "%d,%d,%d,%d,%d,%u,%u,%u,%d,%d,%d,%u,%u,%d,%d,%d;", p.width, p.height,
             p.max_disp, p.census_w, p.census_h, p.path_mask, p.p1, p.p2, p.lr_check, p.lr_max_diff,
             p.median, p.invalid, p.cost, lr_bytes_of(p), hlps[i] | sweep[i] << 12, fr[i].umap ? 1 : 0);
    // (hlps carries the horizontal cost source and the disparity block size)
    k += buf;
  }
  return k;
}

int check_schedule(const sgm_schedule *s) {
  if (!s) return fail(SGM_EINVAL, "schedule is null");
  if (s->h_lanes != 0 && s->h_lanes != 16 && s->h_lanes != 32 && s->h_lanes != 64)
    return fail(SGM_EINVAL, "h_lanes must be 0, 16, 32 or 64 (got %d)", s->h_lanes);
  if (s->sweep != 0 && s->sweep != 1) return fail(SGM_EINVAL, "sweep must be 0 or 1 (got %d)", s->sweep);
  if (s->disp_threads != 0 && s->disp_threads != 256 && s->disp_threads != 512 && s->disp_threads != 1024)
    return fail(SGM_EINVAL, "disp_threads must be 0, 256, 512 or 1024 (got %d)", s->disp_threads);
  if (s->h_costs < SGM_HCOSTS_DEFAULT || s->h_costs > SGM_HCOSTS_CODES)
    return fail(SGM_EINVAL, "h_costs must be 0, 1 or 2 (got %d)", s->h_costs);
  if (s->two_pass < SGM_TWOPASS_DEFAULT || s->two_pass > SGM_TWOPASS_NARROW)
    return fail(SGM_EINVAL, "two_pass must be 0, 1, 2 or 3 (got %d)", s->two_pass);
  return SGM_OK;
}

// Brackets the launches of one stage with timing events when profiling.
struct StageMark {
  std::vector<StageEvents> *out;
  hipStream_t s;
  StageEvents cur{};
  int begin(int stage) {
    if (!out) return SGM_OK;
    cur = StageEvents{stage, 0, nullptr, nullptr};
    HIP_TRY(hipEventCreate(&cur.begin));
    HIP_TRY(hipEventCreate(&cur.end));
    HIP_TRY(hipEventRecord(cur.begin, s));
    return SGM_OK;
  }
  int end(int launches) {
    if (!out) return SGM_OK;
    cur.launches = launches;
    HIP_TRY(hipEventRecord(cur.end, s));
    out->push_back(cur);
    return SGM_OK;
  }
};

int enqueue_frames(const sgm_frame *fr, int n, const std::vector<FramePlan> &plans,
                   const std::vector<int> &hlps, const std::vector<int> &sweep,
                   const std::vector<RemapJob> &rect, char *mem, hipStream_t s,
                   std::vector<StageEvents> *prof, hipEvent_t census_done = nullptr,
                   StripeWait wait = StripeWait{}) {
  StageMark mark{prof, s};
  // rectification of the raw views into the frames' input buffers (one
  // launch for every view of the batch)
  if (!rect.empty()) {
    CHECK(mark.begin(SGM_STAGE_RECTIFY));
    launch_rectify(rect, s);
    CHECK(check_launch());
    CHECK(mark.end((int)((rect.size() + kMaxJobs - 1) / kMaxJobs)));
  }
  // Census of both views + padded uint8 costs (one launch for all Census
  // frames); SAD costs (one launch for all SAD frames, U-maps cleared apart)
  std::vector<FusedCostJob> fj;
  std::vector<SadJob> sj;
  std::vector<CensusJob> cj;  // sweep frames: Census codes of both views
  for (int i = 0; i < n; ++i) {
    const sgm_params &p = fr[i].p;
    if (sweep[i]) {
      const size_t px = (size_t)p.width * p.height;
      for (int v = 0; v < 2; ++v) {
        CensusJob j{};
        j.img = v ? fr[i].right : fr[i].left;
        j.pitch = fr[i].pitch;
        j.out = reinterpret_cast<uint64_t *>(mem + plans[i].off_cost) + v * px;
        j.W = p.width;
        j.H = p.height;
        j.cw = p.census_w;
        j.ch = p.census_h;
        j.ostride = p.width;
        cj.push_back(j);
      }
      continue;
    }
    if (is_sad(p)) {
      SadJob j{};
      j.left = fr[i].left;
      j.right = fr[i].right;
      j.pitch = fr[i].pitch;
      j.out = reinterpret_cast<uint16_t *>(mem + plans[i].off_cost);
      j.W = p.width;
      j.H = p.height;
      j.D = p.max_disp;
      j.ww = p.census_w;
      j.wh = p.census_h;
      j.ostride = dp_of(p);
      sj.push_back(j);
      continue;
    }
    FusedCostJob j{};
    j.left = fr[i].left;
    j.right = fr[i].right;
    j.pitch = fr[i].pitch;
    j.out8 = reinterpret_cast<uint8_t *>(mem + plans[i].off_cost);
    j.W = p.width;
    j.H = p.height;
    j.D = p.max_disp;
    j.Dp = dp_of(p);
    j.nbits = nbits_of(p);
    j.cw = p.census_w;
    j.ch = p.census_h;
    if (hlps[i] & (1 << 8))  // the records start after Dp padding records
      j.codes = reinterpret_cast<uint64_t *>(mem + plans[i].off_codes) + 2 * (size_t)dp_of(p);
    fj.push_back(j);
  }
  CHECK(mark.begin(SGM_STAGE_CENSUS));
  int launches = 0;
  if (!fj.empty()) {
    launch_census_cost(fj, s);
    CHECK(check_launch());
    ++launches;
  }
  if (!sj.empty()) {
    launch_sad(sj, s);
    CHECK(check_launch());
    ++launches;
  }
  if (!cj.empty()) {
    launch_census(cj, s);
    CHECK(check_launch());
    ++launches;
  }
  CHECK(mark.end(launches));
  if (census_done) HIP_TRY(hipEventRecord(census_done, s));
  // two-pass frames: waves per stripe (0: per-direction kernels only)
  auto tp_waves = [&](int i) { return (hlps[i] >> 9) & 1 ? ((hlps[i] >> 10) & 1 ? 16 : 8) : 0; };
  {  // the stripes' ticket counters and error flags start at zero (outside
     // the stages: a few words)
    std::vector<SyncZeroJob> zj;
    for (int i = 0; i < n; ++i)
      if (plans[i].off_sync != kNoSync)  // every frame's words of the batch header
        zj.push_back(SyncZeroJob{reinterpret_cast<uint32_t *>(mem + plans[i].off_sync), kSyncWords, 0});
    if (!zj.empty()) {
      launch_zero_sync(zj, s);
      CHECK(check_launch());
    }
  }
  // aggregation, one launch per (disparities per lane, path-cost width); the
  // two-pass frames' stripe passes belong to the disparity stage
  CHECK(mark.begin(SGM_STAGE_AGGREGATE));
  int groups = 0;
  for (int sad = 0; sad <= 1; ++sad)
  for (int K : {4, 8, 12, 16})
    for (int lb = 1; lb <= 2; ++lb)
    for (int c_hlps : {16, 32, 64})
    for (int slide = 0; slide <= 1; ++slide) {
      std::vector<AggJob> aj;
      for (int i = 0; i < n; ++i) {
        const sgm_params &p = fr[i].p;
        if (sweep[i] || (int)is_sad(p) != sad || k_of(p) != K || lr_bytes_of(p) != lb) continue;
        if ((hlps[i] & 0xFF) != c_hlps || ((hlps[i] >> 8) & 1) != slide) continue;
        AggJob j{};
        if (slide) {
          j.codes = reinterpret_cast<const uint64_t *>(mem + plans[i].off_codes) + 2 * (size_t)dp_of(p);
          j.nbits = nbits_of(p);
        }
        if (sad) j.cost16 = reinterpret_cast<const uint16_t *>(mem + plans[i].off_cost);
        else j.cost8 = reinterpret_cast<const uint8_t *>(mem + plans[i].off_cost);
        j.lr = mem + plans[i].off_lr;
        j.W = p.width;
        j.H = p.height;
        j.D = p.max_disp;
        j.Dp = dp_of(p);
        j.p1 = p.p1;
        j.p2 = p.p2;
        // two-pass frames: L->R, R->L, TR->BL, BL->TR here, the others in stripes
        j.ndirs = fill_dirs(tp_waves(i) ? 0xC3u : p.path_mask, j.dirs);
        aj.push_back(j);
      }
      if (!aj.empty()) {
        launch_aggregate(aj, sad != 0, K, c_hlps, lb, slide != 0, s);
        CHECK(check_launch());
        ++groups;
      }
    }
  {
    std::vector<SweepJob> wj;
    for (int i = 0; i < n; ++i) {
      if (!sweep[i]) continue;
      const sgm_params &p = fr[i].p;
      const size_t px = (size_t)p.width * p.height;
      SweepJob j{};
      j.cl = reinterpret_cast<const uint64_t *>(mem + plans[i].off_cost);
      j.cr = j.cl + px;
      j.dl = reinterpret_cast<uint16_t *>(mem + plans[i].off_lr);
      j.dr = j.dl + px;
      j.carry = reinterpret_cast<uint8_t *>(mem + plans[i].off_lr + align256(2 * px * 2));
      j.W = p.width;
      j.H = p.height;
      j.D = p.max_disp;
      j.nbits = nbits_of(p);
      j.p1 = p.p1;
      j.p2 = p.p2;
      j.mask = p.path_mask;
      j.count = 1;
      j.stride = 0;
      // frames with the same parameters whose scratch follows at a fixed
      // distance share one entry (a launch holds any number of them)
      if (!wj.empty()) {
        SweepJob &q = wj.back();
        const int64_t step = reinterpret_cast<const char *>(j.cl) - reinterpret_cast<const char *>(q.cl);
        const bool same = q.W == j.W && q.H == j.H && q.D == j.D && q.nbits == j.nbits && q.p1 == j.p1 &&
                          q.p2 == j.p2 && q.mask == j.mask;
        if (same && (q.count == 1 ? step > 0 : step == (int64_t)q.count * q.stride)) {
          if (q.count == 1) q.stride = step;
          ++q.count;
          continue;
        }
      }
      wj.push_back(j);
    }
    if (!wj.empty()) {
      launch_sweep(wj, s);
      CHECK(check_launch());
      ++groups;
    }
  }
  // the stripe passes, one launch per (disparities per lane, stripe width)
  // frames with Census code records (bit 8: horizontal costs from codes)
  // form their stripe passes' costs from the codes, the others read the
  // cost volume: separate launches
  auto stripe_jobs = [&](int K, int waves, bool codes, uint32_t epoch) {
    std::vector<StripeJob> sj;
    for (int i = 0; i < n; ++i) {
      const sgm_params &p = fr[i].p;
      const bool has_codes = ((hlps[i] >> 8) & 1) && (K == 8 || K == 16);
      if (tp_waves(i) != waves || k_of(p) != K || has_codes != codes) continue;
      StripeJob j{};
      j.cost = reinterpret_cast<const uint8_t *>(mem + plans[i].off_cost);
      if (has_codes)  // the records start after Dp padding records
        j.codes = reinterpret_cast<const uint64_t *>(mem + plans[i].off_codes) + 2 * (size_t)dp_of(p);
      j.nbits = nbits_of(p);
      j.sd = reinterpret_cast<uint16_t *>(mem + plans[i].off_sd);
      j.lr4 = reinterpret_cast<const uint8_t *>(mem + plans[i].off_lr);
      j.bnd = reinterpret_cast<uint64_t *>(mem + plans[i].off_bnd);
      j.sync = reinterpret_cast<uint32_t *>(mem + plans[i].off_sync);
      uint16_t *final_map = p.median ? reinterpret_cast<uint16_t *>(mem + plans[i].off_dlr) : fr[i].disp;
      j.dl = p.lr_check ? reinterpret_cast<uint16_t *>(mem + plans[i].off_dl) : final_map;
      j.part = reinterpret_cast<uint32_t *>(mem + plans[i].off_part);
      j.W = p.width;
      j.H = p.height;
      j.D = p.max_disp;
      j.Dp = dp_of(p);
      j.p1 = p.p1;
      j.p2 = p.p2;
      j.lr_check = p.lr_check;
      j.epoch = epoch;
      j.max_polls = wait.max_polls;
      j.withhold = wait.withhold;
      sj.push_back(j);
    }
    return sj;
  };
  const uint32_t epoch_down = next_epoch(), epoch_up = next_epoch();
  CHECK(mark.end(groups));
  CHECK(mark.begin(SGM_STAGE_DISPARITY));
  groups = 0;
  // two-pass frames: the top-down stripe pass (then, below, the bottom-up
  // pass with the selection)
  for (int K : {4, 8, 12, 16})
    for (int waves : {8, 16})
      for (bool codes : {false, true}) {
        std::vector<StripeJob> sj = stripe_jobs(K, waves, codes, epoch_down);
        if (sj.empty()) continue;
        launch_stripes(sj, K, false, waves, codes, s);
        CHECK(check_launch());
        ++groups;
      }
  // split image rows across blocks only when the batch's rows are too few to
  // fill the chip on their own
  int disp_rows = 0;
  for (int i = 0; i < n; ++i)
    if (!sweep[i]) disp_rows += fr[i].p.height;
  const bool split = disp_rows < kDispSplitRows;
  {
    std::vector<LRJob> lj;
    for (int i = 0; i < n; ++i) {
      if (!sweep[i]) continue;
      const sgm_params &p = fr[i].p;
      const size_t px = (size_t)p.width * p.height;
      LRJob j{};
      j.dl = reinterpret_cast<const uint16_t *>(mem + plans[i].off_lr);
      j.dr = j.dl + px;
      j.out = p.median ? reinterpret_cast<uint16_t *>(mem + plans[i].off_dlr) : fr[i].disp;
      j.W = p.width;
      j.H = p.height;
      j.lr_check = p.lr_check;
      j.max_diff = p.lr_max_diff;
      j.invalid = p.invalid;
      lj.push_back(j);
    }
    if (!lj.empty()) {
      launch_lr(lj, s);
      CHECK(check_launch());
      ++groups;
    }
  }
  for (int K : {4, 8, 12, 16})
    for (int waves : {8, 16})
      for (bool codes : {false, true}) {
        std::vector<StripeJob> sj = stripe_jobs(K, waves, codes, epoch_up);
        if (sj.empty()) continue;
        launch_stripes(sj, K, true, waves, codes, s);
        CHECK(check_launch());
        ++groups;
      }
  // row segments of a frame's right-view keys: the stripes of two-pass
  // frames, else those of the disparity kernel
  auto segments = [&](int i, int *nseg, int *seglen) {
    const sgm_params &p = fr[i].p;
    if (tp_waves(i)) {
      *nseg = stripes_of(p, tp_waves(i));
      *seglen = stripe_cols(tp_waves(i));
    } else {
      disp_segments(p.width, p.max_disp, split, nseg, seglen);
    }
  };
  for (int lb = 1; lb <= 2; ++lb) {
    std::vector<DispJob> dj;
    for (int i = 0; i < n; ++i) {
      const sgm_params &p = fr[i].p;
      if (sweep[i] || tp_waves(i) || lr_bytes_of(p) != lb) continue;
      DispJob j{};
      j.lr = mem + plans[i].off_lr;
      j.P = popcount8(p.path_mask);
      uint16_t *final_map = p.median ? reinterpret_cast<uint16_t *>(mem + plans[i].off_dlr) : fr[i].disp;
      j.out = p.lr_check ? reinterpret_cast<uint16_t *>(mem + plans[i].off_dl) : final_map;
      j.part = reinterpret_cast<uint32_t *>(mem + plans[i].off_part);
      j.W = p.width;
      j.H = p.height;
      j.D = p.max_disp;
      j.Dp = dp_of(p);
      j.lr_check = p.lr_check;
      j.threads = hlps[i] >> 16;
      disp_segments(p.width, p.max_disp, split, &j.nseg, &j.seglen);
      dj.push_back(j);
    }
    if (!dj.empty()) {
      launch_disparity(dj, lb, s);
      CHECK(check_launch());
      ++groups;
    }
  }
  {
    std::vector<LRSegJob> lj;
    for (int i = 0; i < n; ++i) {
      const sgm_params &p = fr[i].p;
      // with a median, the median kernel forms the LR check itself
      if (sweep[i] || !p.lr_check || p.median) continue;
      LRSegJob j{};
      j.dl = reinterpret_cast<const uint16_t *>(mem + plans[i].off_dl);
      j.part = reinterpret_cast<const uint32_t *>(mem + plans[i].off_part);
      j.out = fr[i].disp;
      j.W = p.width;
      j.H = p.height;
      j.D = p.max_disp;
      segments(i, &j.nseg, &j.seglen);
      j.max_diff = p.lr_max_diff;
      j.invalid = p.invalid;
      lj.push_back(j);
    }
    if (!lj.empty()) {
      launch_lr_seg(lj, s);
      CHECK(check_launch());
      ++groups;
    }
  }
  CHECK(mark.end(groups));
  std::vector<MedianJob> mj;
  for (int i = 0; i < n; ++i) {
    const sgm_params &p = fr[i].p;
    if (!p.median) continue;
    MedianJob j{};
    j.in = reinterpret_cast<const uint16_t *>(mem + plans[i].off_dlr);
    j.out = fr[i].disp;
    j.W = p.width;
    j.H = p.height;
    j.k = p.median;
    if (!sweep[i] && p.lr_check) {  // D_L and the segments' keys from the disparity stage
      j.lr = 1;
      j.dl = reinterpret_cast<const uint16_t *>(mem + plans[i].off_dl);
      j.part = reinterpret_cast<const uint32_t *>(mem + plans[i].off_part);
      j.D = p.max_disp;
      segments(i, &j.nseg, &j.seglen);
      j.max_diff = p.lr_max_diff;
      j.invalid = p.invalid;
    }
    mj.push_back(j);
  }
  if (!mj.empty()) {
    CHECK(mark.begin(SGM_STAGE_MEDIAN));
    launch_median(mj, s);
    CHECK(check_launch());
    CHECK(mark.end(1));
  }
  std::vector<UVJob> uj;
  for (int i = 0; i < n; ++i) {
    if (!fr[i].umap || !fr[i].vmap) continue;
    UVJob j{};
    j.disp = fr[i].disp;
    j.U = fr[i].umap;
    j.V = fr[i].vmap;
    j.W = fr[i].p.width;
    j.H = fr[i].p.height;
    j.D = fr[i].p.max_disp;
    uj.push_back(j);
  }
  if (!uj.empty()) {
    CHECK(mark.begin(SGM_STAGE_UV));
    launch_uv(uj, s);
    CHECK(check_launch());
    CHECK(mark.end(1));
  }
  return SGM_OK;
}

void destroy_events(Batch &b) {
  for (auto &e : b.prof) {
    if (e.begin) (void)hipEventDestroy(e.begin);
    if (e.end) (void)hipEventDestroy(e.end);
  }
  b.prof.clear();
  for (hipEvent_t e : b.joins) (void)hipEventDestroy(e);
  b.joins.clear();
  if (b.done) (void)hipEventDestroy(b.done);
  b.done = nullptr;
}

// Spread the frames of one batch over `groups` of the context's streams --
// largest frames first, each to the group with the least work so far -- so
// that the stages of different frames overlap on the GPU.  Group g starts
// when group g - 1 has finished its Census stage, so its Census (bound by
// the ALUs) runs next to the previous group's aggregation and disparity
// selection (bound by HBM) rather than next to the other groups' Census.
// The batch's own stream waits for every group before its done event.
// Results do not depend on the split.
int enqueue_split(sgm_ctx *c, Batch &b, const sgm_frame *fr, int n, const std::vector<FramePlan> &plans,
                  const std::vector<int> &hl, const std::vector<int> &sw, const std::vector<RemapJob> &rect,
                  char *mem, int groups, std::vector<StageEvents> *prof) {
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  auto work = [&](int i) {
    const sgm_params &p = fr[i].p;
    return (double)p.width * p.height * p.max_disp * popcount8(p.path_mask);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b2) { return work(a) > work(b2); });
  std::vector<std::vector<int>> part(groups);
  std::vector<double> load(groups, 0.0);
  for (int i : order) {
    int g = 0;
    for (int k = 1; k < groups; ++k)
      if (load[k] < load[g]) g = k;
    part[g].push_back(i);
    load[g] += work(i);
  }
  hipStream_t s0 = c->streams[b.stream];
  hipEvent_t fork = nullptr;  // where the next group may start
  HIP_TRY(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
  b.joins.push_back(fork);
  HIP_TRY(hipEventRecord(fork, s0));
  for (int g = 0; g < groups; ++g) {
    if (part[g].empty()) continue;
    std::sort(part[g].begin(), part[g].end());  // frames keep their batch order
    hipStream_t sg = c->streams[(b.stream + g) % c->nstreams];
    HIP_TRY(hipStreamWaitEvent(sg, fork, 0));
    hipEvent_t next = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&next, hipEventDisableTiming));
    b.joins.push_back(next);
    fork = next;
    std::vector<sgm_frame> f;
    std::vector<FramePlan> pl;
    std::vector<int> h, w;
    std::vector<RemapJob> r;
    for (int i : part[g]) {
      f.push_back(fr[i]);
      pl.push_back(plans[i]);
      h.push_back(hl[i]);
      w.push_back(sw[i]);
      if (!rect.empty()) {
        r.push_back(rect[2 * i]);
        r.push_back(rect[2 * i + 1]);
      }
    }
    CHECK(enqueue_frames(f.data(), (int)f.size(), pl, h, w, r, mem, sg, prof, fork, c->stripe_wait));
    if (sg != s0) {
      hipEvent_t join = nullptr;
      HIP_TRY(hipEventCreateWithFlags(&join, hipEventDisableTiming));
      b.joins.push_back(join);
      HIP_TRY(hipEventRecord(join, sg));
      HIP_TRY(hipStreamWaitEvent(s0, join, 0));
    }
  }
  return SGM_OK;
}

// Capture the batch's launches on `s` into a graph, then replay it through
// the cached executable graph of the same composition (updated with this
// batch's buffers), instantiating one on a miss.
int enqueue_graph(sgm_ctx *c, const sgm_frame *fr, int n, const std::vector<FramePlan> &plans,
                  const std::vector<int> &hlps, const std::vector<int> &sweep,
                  const std::vector<RemapJob> &rect, char *mem, hipStream_t s) {
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
  int rc = enqueue_frames(fr, n, plans, hlps, sweep, rect, mem, s, nullptr, nullptr, c->stripe_wait);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  if (rc != SGM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(SGM_EHIP, "graph capture: %s", hipGetErrorString(e));
  const std::string key = composition_key(fr, n, hlps, sweep, rect);
  auto it = c->graph_cache.find(key);
  hipGraphExec_t ex = nullptr;
  if (it != c->graph_cache.end()) {
    hipGraphExecUpdateResult res;
    hipGraphNode_t bad = nullptr;
    if (hipGraphExecUpdate(it->second, g, &bad, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
      ex = it->second;
      ++c->graph_hits;
    } else {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(it->second);
      c->graph_cache.erase(it);
    }
  }
  if (!ex) {
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return fail(SGM_EHIP, "graph instantiate: %s", hipGetErrorString(e));
    }
    c->graph_cache[key] = ex;
    ++c->graph_misses;
  }
  e = hipGraphLaunch(ex, s);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(SGM_EHIP, "graph launch: %s", hipGetErrorString(e));
  return SGM_OK;
}

}  // namespace

extern "C" {

const char *sgm_last_error(void) { return g_err.c_str(); }

int sgm_validate(const sgm_params *p) { return validate(p); }

int sgm_create(sgm_ctx **ctx, int device, size_t hbm_budget_bytes) {
  if (!ctx) return fail(SGM_EINVAL, "ctx is null");
  *ctx = nullptr;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev)
    return fail(SGM_EINVAL, "device %d out of range (%d devices)", device, ndev);
  DeviceGuard g(device);
  if (!g.ok) return fail(SGM_EHIP, "hipSetDevice(%d) failed", device);
  size_t freeb = 0, total = 0;
  HIP_TRY(hipMemGetInfo(&freeb, &total));
  void *fixed = nullptr;
  CHECK(static_scratch_of(device, &fixed));
  auto *c = new sgm_ctx();
  c->device = device;
  c->static_scratch = fixed;
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : freeb / 2;
  for (int i = 0; i < sgm_ctx::kStreams; ++i) {
    if (hipStreamCreateWithFlags(&c->streams[i], hipStreamNonBlocking) != hipSuccess) {
      for (int k = 0; k < i; ++k) (void)hipStreamDestroy(c->streams[k]);
      delete c;
      return fail(SGM_EHIP, "hipStreamCreate failed");
    }
  }
  *ctx = c;
  return SGM_OK;
}

int sgm_destroy(sgm_ctx *c) {
  if (!c) return SGM_OK;
  int rc = SGM_OK;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (hipDeviceSynchronize() != hipSuccess) rc = fail(SGM_EHIP, "device fault before destroy");
    for (auto &kv : c->inflight) {
      destroy_events(kv.second);
      (void)hipFree(kv.second.mem.ptr);
      if (kv.second.sync_host) (void)hipHostFree(kv.second.sync_host);
    }
    for (uint32_t *h : c->sync_pool) (void)hipHostFree(h);
    for (auto &b : c->idle) (void)hipFree(b.ptr);
    for (auto &kv : c->graph_cache) (void)hipGraphExecDestroy(kv.second);
    if (c->stage.ptr) (void)hipFree(c->stage.ptr);
    for (auto &s : c->streams) (void)hipStreamDestroy(s);
  }
  delete c;
  return rc;
}

int sgm_rectify(sgm_ctx *c, const sgm_remap *jobs, int n, void *stream) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  if (n < 0) return fail(SGM_EINVAL, "n = %d < 0", n);
  if (n > 0 && !jobs) return fail(SGM_EINVAL, "jobs is null");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  std::vector<RemapJob> rj(n);
  for (int i = 0; i < n; ++i) CHECK(check_remap(jobs[i], i, c->device, &rj[i]));
  if (rj.empty()) return SGM_OK;
  launch_rectify(rj, (hipStream_t)stream);
  return check_launch();
}

int sgm_census(sgm_ctx *c, const sgm_params *p, const uint8_t *img, int64_t pitch, uint64_t *census,
               void *stream) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  CHECK(validate(p));
  if (is_sad(*p)) return fail(SGM_EINVAL, "sgm_census needs p->cost == SGM_COST_CENSUS");
  if (pitch < p->width) return fail(SGM_EINVAL, "pitch %lld < width %d", (long long)pitch, p->width);
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  CHECK(check_dev_ptr(img, c->device, "img"));
  CHECK(check_dev_ptr(census, c->device, "census"));
  CensusJob j{};
  j.img = img;
  j.pitch = pitch;
  j.out = census;
  j.W = p->width;
  j.H = p->height;
  j.cw = p->census_w;
  j.ch = p->census_h;
  j.ostride = p->width;
  launch_census({j}, (hipStream_t)stream);
  return check_launch();
}

int sgm_cost(sgm_ctx *c, const sgm_params *p, const uint64_t *cl, const uint64_t *cr, uint16_t *cost,
             void *stream) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  CHECK(validate(p));
  if (is_sad(*p)) return fail(SGM_EINVAL, "sgm_cost takes Census codes: use sgm_cost_sad for SAD");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  CHECK(check_dev_ptr(cl, c->device, "cl"));
  CHECK(check_dev_ptr(cr, c->device, "cr"));
  CHECK(check_dev_ptr(cost, c->device, "cost"));
  CostJob j{};
  j.cl = cl;
  j.cr = cr;
  j.out16 = cost;
  j.W = p->width;
  j.H = p->height;
  j.D = p->max_disp;
  j.Dp = dp_of(*p);
  j.nbits = nbits_of(*p);
  launch_cost({j}, (hipStream_t)stream);
  return check_launch();
}

int sgm_cost_sad(sgm_ctx *c, const sgm_params *p, const uint8_t *left, const uint8_t *right,
                 int64_t pitch, uint16_t *cost, void *stream) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  CHECK(validate(p));
  if (!is_sad(*p)) return fail(SGM_EINVAL, "sgm_cost_sad needs p->cost == SGM_COST_SAD");
  if (pitch < p->width) return fail(SGM_EINVAL, "pitch %lld < width %d", (long long)pitch, p->width);
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  CHECK(check_dev_ptr(left, c->device, "left"));
  CHECK(check_dev_ptr(right, c->device, "right"));
  CHECK(check_dev_ptr(cost, c->device, "cost"));
  SadJob j{};
  j.left = left;
  j.right = right;
  j.pitch = pitch;
  j.out = cost;
  j.W = p->width;
  j.H = p->height;
  j.D = p->max_disp;
  j.ww = p->census_w;
  j.wh = p->census_h;
  j.ostride = p->max_disp;
  launch_sad({j}, (hipStream_t)stream);
  return check_launch();
}

int sgm_aggregate(sgm_ctx *c, const sgm_params *p, const uint16_t *cost, uint16_t *aggr,
                  void *stream) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  CHECK(validate(p));
  if ((const void *)cost == (const void *)aggr) return fail(SGM_EINVAL, "cost and aggr alias");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  CHECK(check_dev_ptr(cost, c->device, "cost"));
  CHECK(check_dev_ptr(aggr, c->device, "aggr"));
  hipStream_t s = (hipStream_t)stream;
  const int lb = lr_bytes_of(*p);
  const int P = popcount8(p->path_mask);
  const int Dp = dp_of(*p);
  const int64_t px = (int64_t)p->width * p->height;
  // scratch: the costs repacked with the padded disparity stride, then the
  // P path-cost volumes
  void *mem = nullptr;
  const size_t cbytes = align256((size_t)px * Dp * 2);
  CHECK(stage_scratch(c, cbytes + (size_t)px * Dp * P * lb, s, &mem));
  uint16_t *cpad = reinterpret_cast<uint16_t *>(mem);
  void *lr = reinterpret_cast<char *>(mem) + cbytes;
  launch_pad16(cost, cpad, px, p->max_disp, Dp, s);
  CHECK(check_launch());
  AggJob j{};
  j.cost16 = cpad;
  j.lr = lr;
  j.W = p->width;
  j.H = p->height;
  j.D = p->max_disp;
  j.Dp = Dp;
  j.p1 = p->p1;
  j.p2 = p->p2;
  j.ndirs = fill_dirs(p->path_mask, j.dirs);
  launch_aggregate({j}, true, k_of(*p), resolve_hlps(c, *p), lb, false, s);
  CHECK(check_launch());
  SumJob sj{};
  sj.lr = lr;
  sj.S = aggr;
  sj.cells = px * p->max_disp;
  sj.D = p->max_disp;
  sj.Dp = Dp;
  sj.P = P;
  launch_sum({sj}, lb, s);
  return check_launch();
}

int sgm_disparity(sgm_ctx *c, const sgm_params *p, const uint16_t *aggr, uint16_t *disp,
                  void *stream) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  CHECK(validate(p));
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  CHECK(check_dev_ptr(aggr, c->device, "aggr"));
  CHECK(check_dev_ptr(disp, c->device, "disp"));
  hipStream_t s = (hipStream_t)stream;
  void *v = nullptr;
  CHECK(stage_scratch(c, disparity_scratch_bytes(*p), s, &v));
  return enqueue_disparity(p, aggr, disp, v, s);
}

int sgm_disparity_noalloc(sgm_ctx *c, const sgm_params *p, const uint16_t *aggr, uint16_t *disp,
                          void *stream) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  CHECK(validate(p));
  const size_t need = disparity_scratch_bytes(*p);
  if (need > kStaticScratchBytes)
    return fail(SGM_ENOMEM, "sgm_disparity_noalloc: a %dx%d D=%d frame needs %zu bytes of scratch, "
                "the library's fixed scratch holds %zu", p->width, p->height, p->max_disp, need,
                kStaticScratchBytes);
  std::lock_guard<std::mutex> lk(c->mu);
  if (!c->static_scratch) return fail(SGM_EHIP, "the fixed scratch of device %d is not mapped", c->device);
  DeviceGuard g(c->device);
  CHECK(check_dev_ptr(aggr, c->device, "aggr"));
  CHECK(check_dev_ptr(disp, c->device, "disp"));
  return enqueue_disparity(p, aggr, disp, c->static_scratch, (hipStream_t)stream);
}

}  // extern "C"

namespace {

// Scratch of disparity selection: the pre-median map, D_L and the row
// segments' right-view keys.
size_t disparity_scratch_bytes(const sgm_params &p) {
  const size_t m2 = align256((size_t)p.width * p.height * 2);
  return 2 * m2 + disp_part_bytes(p.width, p.height, p.max_disp);
}

// WTA + right-view keys, LR check and median of one frame from the caller's
// S, with its scratch at `v` (disparity_scratch_bytes).
int enqueue_disparity(const sgm_params *p, const uint16_t *aggr, uint16_t *disp, void *v, hipStream_t s) {
  const size_t px = (size_t)p->width * p->height;
  const size_t m2 = align256(px * 2);
  uint16_t *tmp = reinterpret_cast<uint16_t *>(v);
  uint16_t *dlmap = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(v) + m2);
  uint32_t *part = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(v) + 2 * m2);
  uint16_t *final_map = p->median ? tmp : disp;
  DispJob j{};
  j.S = aggr;
  j.P = popcount8(p->path_mask);
  j.out = p->lr_check ? dlmap : final_map;
  j.part = part;
  j.W = p->width;
  j.H = p->height;
  j.D = p->max_disp;
  j.Dp = dp_of(*p);
  j.lr_check = p->lr_check;
  const bool split = p->height < kDispSplitRows;
  disp_segments(p->width, p->max_disp, split, &j.nseg, &j.seglen);
  launch_disparity({j}, 0, s);
  CHECK(check_launch());
  if (p->lr_check) {
    LRSegJob l{};
    l.dl = dlmap;
    l.part = part;
    l.out = final_map;
    l.W = p->width;
    l.H = p->height;
    l.D = p->max_disp;
    disp_segments(p->width, p->max_disp, split, &l.nseg, &l.seglen);
    l.max_diff = p->lr_max_diff;
    l.invalid = p->invalid;
    launch_lr_seg({l}, s);
    CHECK(check_launch());
  }
  if (p->median) {
    MedianJob m{};
    m.in = tmp;
    m.out = disp;
    m.W = p->width;
    m.H = p->height;
    m.k = p->median;
    launch_median({m}, s);
    CHECK(check_launch());
  }
  return SGM_OK;
}

}  // namespace

extern "C" {

int uv_maps(sgm_ctx *c, const sgm_params *p, const uint16_t *disp, uint16_t *umap, uint16_t *vmap,
            void *stream) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  CHECK(validate(p));
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  CHECK(check_dev_ptr(disp, c->device, "disp"));
  CHECK(check_dev_ptr(umap, c->device, "umap"));
  CHECK(check_dev_ptr(vmap, c->device, "vmap"));
  UVJob j{};
  j.disp = disp;
  j.U = umap;
  j.V = vmap;
  j.W = p->width;
  j.H = p->height;
  j.D = p->max_disp;
  launch_uv({j}, (hipStream_t)stream);
  return check_launch();
}

static int submit_impl(sgm_ctx *c, const sgm_frame *frames, const sgm_remap *remaps, int n,
                       uint64_t *ticket, void *const *events = nullptr, int n_events = 0) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  if (!frames || n < 1 || !ticket) return fail(SGM_EINVAL, "need frames, n >= 1 and a ticket pointer");
  if (n_events < 0 || (n_events > 0 && !events)) return fail(SGM_EINVAL, "need n_events >= 0 events");
  for (int i = 0; i < n_events; ++i)
    if (!events[i]) return fail(SGM_EINVAL, "event %d is null", i);
  for (int i = 0; i < n; ++i) {
    int rc = validate(&frames[i].p);
    if (rc) return fail(rc, "frame %d: %s", i, g_err.c_str());
    if (frames[i].pitch < frames[i].p.width) return fail(SGM_EINVAL, "frame %d: pitch < width", i);
    if ((frames[i].umap == nullptr) != (frames[i].vmap == nullptr))
      return fail(SGM_EINVAL, "frame %d: give both umap and vmap, or neither", i);
  }
  std::lock_guard<std::mutex> lk(c->mu);
  std::vector<int> hl(n), sw(n);
  std::vector<FramePlan> plans(n);
  // The two-pass schedule runs one workgroup per stripe, each a chain of
  // the frame's rows: it needs a batch's stripes to fill the chip.  A batch
  // whose two-pass frames have fewer than kMinStripes stripes in all runs
  // them on the per-direction kernels (one 1920x1080 frame alone: 8.1 ms
  // against 2.6 ms).
  std::vector<int> tpw(n);
  int stripes = 0;
  for (int i = 0; i < n; ++i) {
    tpw[i] = resolve_twopass(c, frames[i].p);
    if (tpw[i]) stripes += stripes_of(frames[i].p, tpw[i]);
  }
  if (stripes < kMinStripes) std::fill(tpw.begin(), tpw.end(), 0);
  // a header of kSyncWords words per frame (the two-pass frames' ticket
  // counters and error flags), read back when the batch is done
  const bool any_tp = stripes >= kMinStripes;
  size_t total = any_tp ? align256((size_t)n * kSyncWords * 4) : 0;
  for (int i = 0; i < n; ++i) {
    // lanes per horizontal scanline (low byte), horizontal costs from codes
    // (bit 8), two-pass stripes (bit 9; bit 10: 16 waves per stripe, else
    // 8), the disparity block size (above bit 16)
    const int h = resolve_hlps(c, frames[i].p);
    sw[i] = resolve_sweep(c, frames[i].p);
    const bool codes = !sw[i] && resolve_hcosts(c, frames[i].p, h) == SGM_HCOSTS_CODES;
    const int tp = tpw[i];
    hl[i] = h | (codes ? 1 << 8 : 0) | (tp ? 1 << 9 : 0) | (tp == 16 ? 1 << 10 : 0) |
            resolve_disp_threads(c, frames[i].p) << 16;
    plans[i] = plan_frame(frames[i].p, total, sw[i] != 0, codes, tp);
    plans[i].off_sync = any_tp ? (size_t)i * kSyncWords * 4 : kNoSync;
    total += plans[i].bytes;
  }
  DeviceGuard g(c->device);
  for (int i = 0; i < n; ++i) {
    CHECK(check_dev_ptr(frames[i].left, c->device, "left"));
    CHECK(check_dev_ptr(frames[i].right, c->device, "right"));
    CHECK(check_dev_ptr(frames[i].disp, c->device, "disp"));
    if (frames[i].umap) {
      CHECK(check_dev_ptr(frames[i].umap, c->device, "umap"));
      CHECK(check_dev_ptr(frames[i].vmap, c->device, "vmap"));
    }
  }
  std::vector<RemapJob> rect;
  if (remaps) {
    rect.resize(2 * (size_t)n);
    for (int i = 0; i < 2 * n; ++i) {
      CHECK(check_remap(remaps[i], i, c->device, &rect[i]));
      const sgm_frame &f = frames[i / 2];
      const uint8_t *dst = (i & 1) ? f.right : f.left;
      if (remaps[i].out != dst || remaps[i].out_pitch != f.pitch || remaps[i].w != f.p.width ||
          remaps[i].h != f.p.height)
        return fail(SGM_EINVAL, "job %d: out, out_pitch, w, h must be frame %d's %s view, pitch and size", i,
                    i / 2, (i & 1) ? "right" : "left");
    }
  }
  total = align256(total);
  if (total + c->stage.bytes > c->budget)
    return fail(SGM_ENOMEM, "batch needs %zu bytes of scratch, budget is %zu", total, c->budget);
  // reuse the smallest idle block that is big enough
  Block blk;
  size_t bi = c->idle.size();
  for (size_t i = 0; i < c->idle.size(); ++i)
    if (c->idle[i].bytes >= total && (bi == c->idle.size() || c->idle[i].bytes < c->idle[bi].bytes))
      bi = i;
  if (bi < c->idle.size()) {  // already counted in held(): no admission change
    blk = c->idle[bi];
    c->idle.erase(c->idle.begin() + bi);
  }
  if (!blk.ptr) {
    CHECK(make_room(c, total));
    if (c->held() + total > c->budget)
      return fail(SGM_EBUSY, "batch needs %zu bytes, %zu of %zu held by batches in flight", total,
                  c->inflight_bytes(), c->budget);
    HIP_TRY(hipMalloc(&blk.ptr, total));
    blk.bytes = total;
  }
  Batch b;
  b.mem = blk;
  b.sync_frames = any_tp ? n : 0;
  b.stream = c->next_stream;
  c->next_stream = (c->next_stream + 1) % c->nstreams;
  hipStream_t s = c->streams[b.stream];
  int rc = SGM_OK;
  // the caller's events gate the batch's first launch (on the GPU)
  for (int i = 0; i < n_events && rc == SGM_OK; ++i)
    if (hipStreamWaitEvent(s, (hipEvent_t)events[i], 0) != hipSuccess)
      rc = fail(SGM_EHIP, "hipStreamWaitEvent on event %d failed", i);
  if (rc != SGM_OK) {
    c->idle.push_back(blk);
    return rc;
  }
  // a batch submitted while others run already overlaps with them on the
  // context's streams; one submitted to an idle context overlaps its own
  // frames' stages by the split
  const int groups = c->inflight.empty() ? std::min(std::min(c->split, c->nstreams), n) : 1;
  if (c->graphs && !c->profiling) {
    rc = enqueue_graph(c, frames, n, plans, hl, sw, rect, reinterpret_cast<char *>(blk.ptr), s);
  } else if (groups > 1) {
    rc = enqueue_split(c, b, frames, n, plans, hl, sw, rect, reinterpret_cast<char *>(blk.ptr), groups,
                       c->profiling ? &b.prof : nullptr);
  } else {
    rc = enqueue_frames(frames, n, plans, hl, sw, rect, reinterpret_cast<char *>(blk.ptr), s,
                        c->profiling ? &b.prof : nullptr, nullptr, c->stripe_wait);
  }
  if (rc == SGM_OK && b.sync_frames) {
    // the sync words (error flags) to pinned host memory, as the batch's
    // last step: once its done event has completed they are readable
    const size_t bytes = (size_t)n * kSyncWords * 4;
    if (bytes <= kSyncHostBytes && !c->sync_pool.empty()) {
      b.sync_host = c->sync_pool.back();
      c->sync_pool.pop_back();
    } else if (hipHostMalloc((void **)&b.sync_host, std::max(bytes, kSyncHostBytes), hipHostMallocDefault) !=
               hipSuccess) {
      b.sync_host = nullptr;
      rc = fail(SGM_EHIP, "hipHostMalloc of %zu bytes failed", bytes);
    }
    if (rc == SGM_OK && hipMemcpyAsync(b.sync_host, blk.ptr, bytes, hipMemcpyDeviceToHost, s) != hipSuccess)
      rc = fail(SGM_EHIP, "copy of the sync words failed");
  }
  if (rc == SGM_OK && hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess)
    rc = fail(SGM_EHIP, "hipEventCreate failed");
  if (rc == SGM_OK && hipEventRecord(b.done, s) != hipSuccess) rc = fail(SGM_EHIP, "hipEventRecord failed");
  if (rc != SGM_OK) {
    // work already enqueued (on every stream a split batch used) must end
    // before the block can be reused
    for (int g = 0; g < std::max(groups, 1); ++g) (void)hipStreamSynchronize(c->streams[(b.stream + g) % c->nstreams]);
    destroy_events(b);
    c->idle.push_back(blk);
    if (b.sync_host) c->sync_pool.push_back(b.sync_host);
    return rc;
  }
  *ticket = c->next_ticket++;
  c->inflight[*ticket] = b;
  return SGM_OK;
}

int uv_filter(sgm_ctx *c, const uv_filter_job *jobs, int n, void *stream) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  if (n < 0) return fail(SGM_EINVAL, "n = %d < 0", n);
  if (n > 0 && !jobs) return fail(SGM_EINVAL, "jobs is null");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  std::vector<UVFilterJob> fj(n);
  for (int i = 0; i < n; ++i) {
    const uv_filter_job &q = jobs[i];
    if (q.rows < 1 || q.cols < 1 || q.rows > 16384 || q.cols > 16384)
      return fail(SGM_EINVAL, "job %d: map size %d x %d outside 1..16384", i, q.rows, q.cols);
    if (q.dilate_r > kUVFMaxDil) return fail(SGM_EINVAL, "job %d: dilate_r %u > %d", i, q.dilate_r, kUVFMaxDil);
    if (q.blur_r > kUVFMaxBlur) return fail(SGM_EINVAL, "job %d: blur_r %u > %d", i, q.blur_r, kUVFMaxBlur);
    if (q.reserved) return fail(SGM_EINVAL, "job %d: reserved must be 0", i);
    if (q.roi_r0 < 0 || q.roi_r0 > q.roi_r1 || q.roi_r1 > q.rows || q.roi_c0 < 0 || q.roi_c0 > q.roi_c1 ||
        q.roi_c1 > q.cols)
      return fail(SGM_EINVAL, "job %d: region of interest rows [%d,%d) cols [%d,%d) outside the map", i,
                  q.roi_r0, q.roi_r1, q.roi_c0, q.roi_c1);
    char name[32];
    snprintf(name, sizeof(name), "job %d: map", i);
    CHECK(check_dev_ptr(q.map, c->device, name));
    snprintf(name, sizeof(name), "job %d: out", i);
    CHECK(check_dev_ptr(q.out, c->device, name));
    UVFilterJob &j = fj[i];
    j = UVFilterJob{};
    j.map = q.map;
    j.out = q.out;
    j.rows = q.rows;
    j.cols = q.cols;
    j.thr = q.threshold;
    j.dil = q.dilate_r;
    j.blur = q.blur_r;
    j.r0 = q.roi_r0;
    j.r1 = q.roi_r1;
    j.c0 = q.roi_c0;
    j.c1 = q.roi_c1;
  }
  if (fj.empty()) return SGM_OK;
  launch_uv_filter(fj, (hipStream_t)stream);
  return check_launch();
}

int sgm_submit(sgm_ctx *c, const sgm_frame *frames, int n, uint64_t *ticket) {
  return submit_impl(c, frames, nullptr, n, ticket);
}

int sgm_submit_after(sgm_ctx *c, const sgm_frame *frames, int n, void *const *events, int n_events,
                     uint64_t *ticket) {
  return submit_impl(c, frames, nullptr, n, ticket, events, n_events);
}

int sgm_submit_rectify(sgm_ctx *c, const sgm_frame *frames, const sgm_remap *remaps, int n,
                       uint64_t *ticket) {
  if (!remaps) return fail(SGM_EINVAL, "remaps is null");
  return submit_impl(c, frames, remaps, n, ticket);
}

static int poll_locked(sgm_ctx *c, uint64_t ticket, int *done) {
  auto it = c->inflight.find(ticket);
  if (it == c->inflight.end()) return fail(SGM_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  hipError_t e = hipEventQuery(it->second.done);
  if (e == hipErrorNotReady) {
    *done = 0;
    return SGM_OK;
  }
  if (e != hipSuccess) return fail(SGM_EHIP, "batch %llu: %s", (unsigned long long)ticket, hipGetErrorString(e));
  int bad = -1;  // a two-pass frame whose stripes gave up waiting for a neighbour
  if (it->second.sync_host) {
    const uint32_t *w = it->second.sync_host;
    for (int i = 0; i < it->second.sync_frames && bad == -1; ++i)
      if (w[(size_t)i * kSyncWords + 1]) bad = i;
    if ((size_t)it->second.sync_frames * kSyncWords * 4 <= kSyncHostBytes) c->sync_pool.push_back(it->second.sync_host);
    else (void)hipHostFree(it->second.sync_host);
    it->second.sync_host = nullptr;
  }
  for (auto &e : it->second.prof) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e.begin, e.end) == hipSuccess) {
      c->stage_ms[e.stage] += ms;
      c->stage_count[e.stage] += (uint64_t)e.launches;
    }
  }
  destroy_events(it->second);
  c->idle.push_back(it->second.mem);
  c->inflight.erase(it);
  *done = 1;
  if (bad >= 0)
    return fail(SGM_EHIP, "batch %llu, frame %d: a stripe pass gave up waiting for its neighbour stripe",
                (unsigned long long)ticket, bad);
  return SGM_OK;
}

int sgm_poll(sgm_ctx *c, uint64_t ticket, int *done) {
  if (!c || !done) return fail(SGM_EINVAL, "ctx and done must be non-null");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->device);
  return poll_locked(c, ticket, done);
}

int sgm_wait(sgm_ctx *c, uint64_t ticket) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  // Poll, releasing the context's lock between polls: a blocking wait under
  // the lock would hold up every other thread's submit and poll until this
  // batch is done.
  for (;;) {
    int done = 0;
    {
      std::lock_guard<std::mutex> lk(c->mu);
      DeviceGuard g(c->device);
      CHECK(poll_locked(c, ticket, &done));
    }
    if (done) return SGM_OK;
    std::this_thread::yield();
  }
}

int sgm_set_schedule(sgm_ctx *c, const sgm_params *shape, const sgm_schedule *sc) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  CHECK(check_schedule(sc));
  if (shape) CHECK(validate(shape));
  std::lock_guard<std::mutex> lk(c->mu);
  if (shape) c->tuned[shape_key(*shape)] = *sc;
  else c->dflt = *sc;
  return SGM_OK;
}

int sgm_get_schedule(sgm_ctx *c, const sgm_params *shape, sgm_schedule *sc) {
  if (!c || !sc) return fail(SGM_EINVAL, "ctx and schedule must be non-null");
  CHECK(validate(shape));
  std::lock_guard<std::mutex> lk(c->mu);
  *sc = sgm_schedule{};
  sc->h_lanes = resolve_hlps(c, *shape);
  sc->sweep = resolve_sweep(c, *shape);
  sc->disp_threads = resolve_disp_threads(c, *shape);
  sc->h_costs = sc->sweep ? SGM_HCOSTS_VOLUME : resolve_hcosts(c, *shape, sc->h_lanes);
  const int tp = resolve_twopass(c, *shape);
  sc->two_pass = tp == 16 ? SGM_TWOPASS_WIDE : tp == 8 ? SGM_TWOPASS_NARROW : SGM_TWOPASS_OFF;
  return SGM_OK;
}

// Milliseconds per submit of the n `samples` as one batch under schedule
// `sc` (set for their shape), measured as the context runs batches: `reps`
// warm-up submits back to back (they also leave the scratch blocks the
// timed submits in flight need, so that no allocation falls in the timed
// region), then twice `reps` submits back to back on the context's
// streams, wall clock from the first submit until all are done, the better
// of the two.
static int time_schedule(sgm_ctx *c, const sgm_frame *samples, int n, int reps, const sgm_schedule &sc,
                         float *out) {
  const sgm_frame *sample = samples;
  CHECK(sgm_set_schedule(c, &sample->p, &sc));
  auto run = [&]() -> int {
    std::vector<uint64_t> tk;
    int rc = SGM_OK;
    for (int r = 0; r < reps && rc == SGM_OK; ++r) {
      uint64_t t = 0;
      rc = sgm_submit(c, samples, n, &t);
      if (rc == SGM_OK) tk.push_back(t);
    }
    for (uint64_t k : tk) {
      const int r2 = sgm_wait(c, k);
      if (rc == SGM_OK) rc = r2;
    }
    return rc;
  };
  CHECK(run());  // warm-up
  double best = -1.0;
  for (int k = 0; k < 2; ++k) {  // the better of two timed runs
    const auto t0 = std::chrono::steady_clock::now();
    CHECK(run());
    const auto t1 = std::chrono::steady_clock::now();
    const double ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    if (best < 0.0 || ms < best) best = ms;
  }
  *out = (float)(best / reps);
  return SGM_OK;
}

int sgm_autotune(sgm_ctx *c, const sgm_frame *samples, int n, int reps, sgm_schedule *best, float *ms,
                 int n_ms) {
  if (!c || !samples || n < 1) return fail(SGM_EINVAL, "ctx, samples and n >= 1 are required");
  if (reps < 1) return fail(SGM_EINVAL, "reps must be >= 1");
  const sgm_frame *sample = samples;
  CHECK(validate(&sample->p));
  for (int i = 1; i < n; ++i) {
    CHECK(validate(&samples[i].p));
    const sgm_params &a = sample->p, &b = samples[i].p;
    if (b.width != a.width || b.height != a.height || b.max_disp != a.max_disp || b.path_mask != a.path_mask ||
        lr_bytes_of(b) != lr_bytes_of(a))
      return fail(SGM_EINVAL, "sample %d has another shape than sample 0", i);
  }
  // h_lanes 16, 32, 64; h_costs codes; two_pass wide, narrow; disp_threads
  // 256, 512, 1024; sweep
  constexpr int kCands = 10;
  float times[kCands];
  for (float &t : times) t = -1.f;
  sgm_schedule win{};
  float win_ms = -1.f;
  auto consider = [&](int slot, const sgm_schedule &sc) -> int {
    float t = 0.f;
    CHECK(time_schedule(c, samples, n, reps, sc, &t));
    times[slot] = t;
    if (win_ms < 0.f || t < win_ms) {
      win = sc;
      win_ms = t;
    }
    return SGM_OK;
  };
  // 1. lanes per horizontal scanline, horizontal costs from the volume; and
  //    64 lanes with the costs from sliding Census windows, where it applies
  //    (all with the per-direction kernels)
  const int lanes[3] = {16, 32, 64};
  for (int ci = 0; ci < 3; ++ci) {
    if (!agg_hlps_ok(k_of(sample->p), lanes[ci])) continue;
    sgm_schedule sc{};
    sc.h_lanes = lanes[ci];
    sc.h_costs = SGM_HCOSTS_VOLUME;
    sc.two_pass = SGM_TWOPASS_OFF;
    CHECK(consider(ci, sc));
  }
  if (hcodes_ok(sample->p, 64)) {
    sgm_schedule sc{};
    sc.h_lanes = 64;
    sc.h_costs = SGM_HCOSTS_CODES;
    sc.two_pass = SGM_TWOPASS_OFF;
    CHECK(consider(3, sc));
  }
  // 2. the two-pass schedule with wide and narrow stripes, where the sample
  //    batch has enough stripes to run it (a smaller one would time the
  //    per-direction kernels it falls back to)
  if (twopass_ok(sample->p)) {
    const sgm_schedule base = win;
    const int modes[2] = {SGM_TWOPASS_WIDE, SGM_TWOPASS_NARROW};
    const int waves[2] = {16, 8};
    for (int ci = 0; ci < 2; ++ci) {
      if (n * stripes_of(sample->p, waves[ci]) < kMinStripes) continue;
      sgm_schedule sc = base;
      sc.two_pass = modes[ci];
      CHECK(consider(4 + ci, sc));
    }
  }
  // 3. disparity-selection block size (the per-direction schedule's kernel)
  if (win.two_pass == SGM_TWOPASS_OFF) {
    const int threads[3] = {256, 512, 1024};
    const sgm_schedule base = win;
    for (int ci = 0; ci < 3; ++ci) {
      sgm_schedule sc = base;
      sc.disp_threads = threads[ci];
      CHECK(consider(6 + ci, sc));
    }
  }
  // 4. the single-pass sweep, for frames it can take
  if (sweep_ok(sample->p)) {
    sgm_schedule sc = win;
    sc.sweep = 1;
    CHECK(consider(9, sc));
  }
  CHECK(sgm_set_schedule(c, &sample->p, &win));
  if (best) *best = win;
  for (int i = 0; ms && i < n_ms && i < kCands; ++i) ms[i] = times[i];
  return SGM_OK;
}

int sgm_graph_stats(sgm_ctx *c, uint64_t *hits, uint64_t *misses) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  std::lock_guard<std::mutex> lk(c->mu);
  if (hits) *hits = c->graph_hits;
  if (misses) *misses = c->graph_misses;
  return SGM_OK;
}

int sgm_set_graphs(sgm_ctx *c, int on) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  std::lock_guard<std::mutex> lk(c->mu);
  c->graphs = on != 0;
  return SGM_OK;
}

int sgm_set_stripe_wait(sgm_ctx *c, int max_polls, int withhold_edges) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  if (max_polls < 0) return fail(SGM_EINVAL, "max_polls must be >= 0 (got %d)", max_polls);
  if (withhold_edges != 0 && withhold_edges != 1)
    return fail(SGM_EINVAL, "withhold_edges must be 0 or 1 (got %d)", withhold_edges);
  std::lock_guard<std::mutex> lk(c->mu);
  c->stripe_wait.max_polls = max_polls ? max_polls : kStripePolls;
  c->stripe_wait.withhold = withhold_edges;
  return SGM_OK;
}

int sgm_set_split(sgm_ctx *c, int n) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  if (n < 1 || n > sgm_ctx::kStreams) return fail(SGM_EINVAL, "split must be in [1, %d]", sgm_ctx::kStreams);
  std::lock_guard<std::mutex> lk(c->mu);
  c->split = n;
  return SGM_OK;
}

int sgm_set_streams(sgm_ctx *c, int n) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  if (n < 1 || n > sgm_ctx::kStreams) return fail(SGM_EINVAL, "streams must be in [1, %d]", sgm_ctx::kStreams);
  std::lock_guard<std::mutex> lk(c->mu);
  c->nstreams = n;
  c->next_stream = 0;
  return SGM_OK;
}

int sgm_profile(sgm_ctx *c, int enable) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  std::lock_guard<std::mutex> lk(c->mu);
  c->profiling = enable != 0;
  return SGM_OK;
}

int sgm_profile_read(sgm_ctx *c, double *ms, uint64_t *count, int reset) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  std::lock_guard<std::mutex> lk(c->mu);
  for (int i = 0; i < SGM_NSTAGES; ++i) {
    if (ms) ms[i] = c->stage_ms[i];
    if (count) count[i] = c->stage_count[i];
    if (reset) {
      c->stage_ms[i] = 0;
      c->stage_count[i] = 0;
    }
  }
  return SGM_OK;
}

int sgm_memory(sgm_ctx *c, size_t *in_flight_bytes, size_t *budget_bytes) {
  if (!c) return fail(SGM_EINVAL, "ctx is null");
  std::lock_guard<std::mutex> lk(c->mu);
  if (in_flight_bytes) *in_flight_bytes = c->inflight_bytes();
  if (budget_bytes) *budget_bytes = c->budget;
  return SGM_OK;
}

}  // extern "C"
