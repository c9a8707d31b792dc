/*
 * sgm.h -- C ABI of the MI355X (gfx950) semi-global-matching library.
 *
 * The library computes the stereo disparity path of Ruf et al., "Real-time
 * on-board obstacle avoidance for UAVs based on embedded stereo vision"
 * (arXiv 1807.06271): rectified 8-bit left/right images in, a disparity map
 * and its U-/V-map histograms out (section 3.1 and 3.2).  Every stage is a
 * hand-written HIP kernel; all arithmetic is integer.
 *
 * Conventions shared by every entry point
 *  - Pointers named as device buffers must point to device memory of the
 *    context's device (e.g. a torch CUDA tensor's data_ptr()).  The caller
 *    owns every input and output buffer; the library never frees them, and they
 *    must stay valid until the work enqueued on `stream` has finished (or, for
 *    sgm_submit, until sgm_poll reports the ticket done).
 *  - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *    Stage calls only enqueue work and return at once.
 *  - Every call returns an sgm_status.  Argument errors are reported before
 *    anything is enqueued.  An asynchronous device fault is reported as
 *    SGM_EHIP by the next call that notices it.  sgm_last_error() gives a
 *    thread-local text for the last failure of the calling thread.
 *  - A context may be used from several threads (calls are serialised by an
 *    internal lock), but the stage calls of one context share its scratch
 *    memory: work of two stage calls on different streams of the same context
 *    must not overlap in time (use one context per stream for that).
 *    sgm_submit batches use their own scratch and may overlap freely.
 *
 * Layouts (row-major, no padding unless a pitch is given)
 *  - image   uint8  [H][pitch]      pitch >= W bytes
 *  - census  uint64 [H][W]          N_b = census_w*census_h - 1 low bits used
 *  - cost    uint16 [H][W][D]       disparity fastest
 *  - aggr    uint16 [H][W][D]       S = sum of the selected path costs
 *  - disp    uint16 [H][W]          values < D, or `invalid`
 *  - umap    uint16 [D][W]          U[d][x] = #{y : disp(x,y) = d}
 *  - vmap    uint16 [H][D]          V[y][d] = #{x : disp(x,y) = d}
 */
#ifndef SGM_H
#define SGM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SGM_OK = 0,
  SGM_EINVAL = -1,    /* invalid argument (nothing was enqueued)            */
  SGM_ENOMEM = -2,    /* scratch would exceed the context's memory budget   */
  SGM_EHIP = -3,      /* HIP runtime error, including earlier async faults  */
  SGM_EBUSY = -4,     /* batch not admissible now; poll, then submit again  */
  SGM_ENOTFOUND = -5  /* unknown ticket                                     */
} sgm_status;

/* Aggregation path directions r = (dx, dy) (section 3.1.3).  Each path starts
 * at the image border and visits p - r before p. */
enum {
  SGM_PATH_L2R = 1u << 0,   /* (+1,  0) left to right                     */
  SGM_PATH_R2L = 1u << 1,   /* (-1,  0) right to left                     */
  SGM_PATH_T2B = 1u << 2,   /* ( 0, +1) top to bottom                     */
  SGM_PATH_B2T = 1u << 3,   /* ( 0, -1) bottom to top                     */
  SGM_PATH_TL2BR = 1u << 4, /* (+1, +1) diagonal to the bottom right      */
  SGM_PATH_BR2TL = 1u << 5, /* (-1, -1) diagonal to the top left          */
  SGM_PATH_TR2BL = 1u << 6, /* (-1, +1) diagonal to the bottom left       */
  SGM_PATH_BL2TR = 1u << 7  /* (+1, -1) diagonal to the top right         */
};
/* The paper's four streaming paths (figure 2: 0, 45, 90 and 135 degrees). */
#define SGM_PATHS_PAPER4 (SGM_PATH_L2R | SGM_PATH_TL2BR | SGM_PATH_T2B | SGM_PATH_TR2BL)
/* Horizontal and vertical paths in both senses. */
#define SGM_PATHS_HV4 (SGM_PATH_L2R | SGM_PATH_R2L | SGM_PATH_T2B | SGM_PATH_B2T)
#define SGM_PATHS_ALL8 0xFFu

/* Matching cost (section 3.1.2): Census transform + Hamming distance, or the
 * sum of absolute differences over the census_w x census_h support region. */
enum { SGM_COST_CENSUS = 0, SGM_COST_SAD = 1 };

/* Parameters of one frame.  Validated by every call:
 *   1 <= width, height <= 16384;  1 <= max_disp (D) <= 256;
 *   census_w, census_h odd and >= 1; the largest cost Cmax is N_b =
 *   census_w*census_h - 1 (Census, 1 <= N_b <= 64) or census_w*census_h*255
 *   (SAD, <= 65535);
 *   path_mask a nonzero subset of SGM_PATH_*;  p1 <= p2;
 *   popcount(path_mask) * (Cmax + p2) <= 65535 (no 16-bit overflow of S);
 *   lr_check 0 or 1, lr_max_diff >= 0;  median 0 (off), 3 or 5;
 *   invalid >= D (255 is the usual value for D <= 255, 65535 above);
 *   width * height * Dp * 2 < 4 GiB, with Dp = D rounded up to 64, 128, 192
 *   or 256 (the padded disparity stride of the internal volumes). */
typedef struct {
  int32_t width, height;
  int32_t max_disp;
  int32_t census_w, census_h;
  uint32_t path_mask;
  uint16_t p1, p2;
  int32_t lr_check;
  int32_t lr_max_diff;
  int32_t median;
  uint16_t invalid;
  uint16_t cost;     /* SGM_COST_CENSUS (0) or SGM_COST_SAD (1) */
} sgm_params;

typedef struct sgm_ctx sgm_ctx;

/* Check a parameter set without touching the GPU: SGM_OK, or SGM_EINVAL
 * with the reason in sgm_last_error().  Every other call runs the same
 * checks. */
int sgm_validate(const sgm_params *p);

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * scratch the context may hold (stage-call scratch plus in-flight batches);
 * 0 selects half of the device's free memory.  Returns SGM_EINVAL for a bad
 * device or null `ctx`. */
int sgm_create(sgm_ctx **ctx, int device, size_t hbm_budget_bytes);

/* Wait for all work the context enqueued, free its scratch, destroy it.
 * Outstanding tickets become unknown.  A null ctx is a no-op. */
int sgm_destroy(sgm_ctx *ctx);

/* Text of the calling thread's last failure ("" if none).  Owned by the
 * library, valid until the thread's next call. */
const char *sgm_last_error(void);

/* One image to rectify (section 3.1.1).  For each pixel p = (x, y) of the
 * w x h rectified image, out(p) = src(map_x(p), map_y(p)): the maps hold, per
 * rectified pixel, the integer column and row of the raw image pixel it shows
 * (maps precomputed once from the calibration).  An entry with map_x >= src_w
 * or map_y >= src_h (e.g. 65535) means "no source pixel" and gives 0.
 *   src:   device uint8  [src_h][src_pitch], src_pitch >= src_w
 *   map_x, map_y: device uint16 [h][w] (16-byte aligned maps are read with
 *          wider loads; any alignment is accepted)
 *   out:   device uint8  [h][out_pitch], out_pitch >= w; must not overlap
 *          src or the maps.
 * Limits: 1 <= w, h <= 16384; 1 <= src_w, src_h <= 65535. */
typedef struct {
  const uint8_t *src;
  const uint16_t *map_x;
  const uint16_t *map_y;
  uint8_t *out;
  int64_t src_pitch;
  int64_t out_pitch;
  int32_t src_w, src_h;
  int32_t w, h;
} sgm_remap;

/* Rectify n >= 0 images (e.g. the left and right raw images of several
 * frames, each with its own maps) with one kernel launch per 24 images,
 * enqueued on `stream`.  n = 0 enqueues nothing.  Every job is checked
 * before anything is enqueued; SGM_EINVAL names the first bad job.  Uses no
 * scratch memory, so calls on different streams may overlap. */
int sgm_rectify(sgm_ctx *ctx, const sgm_remap *jobs, int n, void *stream);

/* Census transform (section 3.1.2): for each pixel p, an N_b-bit code of the
 * comparisons [I(q) < I(p)] over the census_w x census_h window, neighbours in
 * raster order with the first one in bit N_b-1, coordinates clamped to the
 * image.  img: device uint8 [H][pitch]; census: device uint64 [H][W]. */
int sgm_census(sgm_ctx *ctx, const sgm_params *p, const uint8_t *img, int64_t pitch,
               uint64_t *census, void *stream);

/* SAD matching cost volume, equation (1) with the SAD similarity (p->cost
 * must be SGM_COST_SAD): cost(x,y,d) = sum over the census_w x census_h
 * window of |I_L(x+dx,y+dy) - I_R(x-d+dx,y+dy)|, every coordinate clamped
 * to the image, and census_w*census_h*255 where x < d.  left, right: device
 * uint8 [H][pitch]; cost: device uint16 [H][W][D]. */
int sgm_cost_sad(sgm_ctx *ctx, const sgm_params *p, const uint8_t *left, const uint8_t *right,
                 int64_t pitch, uint16_t *cost, void *stream);

/* Matching cost volume, equation (1) with the Census/Hamming similarity:
 * cost(x,y,d) = popcount(cl(x,y) XOR cr(x-d,y)) for x >= d, else N_b.
 * cl, cr: device uint64 [H][W]; cost: device uint16 [H][W][D]. */
int sgm_cost(sgm_ctx *ctx, const sgm_params *p, const uint64_t *cl, const uint64_t *cr,
             uint16_t *cost, void *stream);

/* Semi-global aggregation (section 3.1.3, equation (2) as Hirschmueller's
 * path recurrence): for each path r in path_mask,
 *   L_r(p,d) = C(p,d) + min(L_r(p-r,d), L_r(p-r,d+-1) + P1, m + P2) - m,
 *   m = min_k L_r(p-r,k);  L_r(p,d) = C(p,d) at the first pixel of a path;
 * and aggr = S = sum_r L_r.  cost values must be <= Cmax (as sgm_cost and
 * sgm_cost_sad make them); larger values give unspecified (but memory-safe)
 * results.
 * cost, aggr: device uint16 [H][W][D]; may not alias. */
int sgm_aggregate(sgm_ctx *ctx, const sgm_params *p, const uint16_t *cost, uint16_t *aggr,
                  void *stream);

/* Disparity selection (sections 3.1.3 to 3.1.5) from S:
 *   D_L(p) = smallest argmin_d S(p,d);
 *   if lr_check: D_R(x,y) = smallest argmin_{d < min(D, W-x)} S(x+d,y,d) and
 *     the pixel keeps D_L iff x - D_L >= 0 and |D_L - D_R(x-D_L,y)| <= lr_max_diff,
 *     else it becomes `invalid`;
 *   if median: k x k median (clamped borders) of that map.
 * aggr: device uint16 [H][W][D]; disp: device uint16 [H][W]. */
int sgm_disparity(sgm_ctx *ctx, const sgm_params *p, const uint16_t *aggr, uint16_t *disp,
                  void *stream);

/* sgm_disparity that allocates nothing, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, same results (bit for bit) as
 * sgm_disparity.  Its scratch (the map before the median, D_L and the row
 * segments' right-view keys: 2*align256(2*W*H) + 4*H*nseg*(seglen + D - 1)
 * bytes, nseg = max(1, W / max(256, 2*D)), seglen = ceil(W / nseg); 20 MiB
 * for 1920x1080, D = 256) lives in a fixed 32 MiB array in the library's
 * device memory: one per GPU, mapped by sgm_create, held until the process
 * ends.  Larger frames get SGM_ENOMEM before anything is enqueued.  Every
 * call on a GPU uses that GPU's one array and leaves its contents behind
 * (no call relies on them): calls on one GPU whose work overlaps in time --
 * other streams, other contexts, other threads -- race on it, so serialise
 * them (e.g. enqueue them all on one stream). */
int sgm_disparity_noalloc(sgm_ctx *ctx, const sgm_params *p, const uint16_t *aggr, uint16_t *disp,
                          void *stream);

/* U-/V-maps (section 3.2): per-column and per-row disparity histograms of
 * disp; values >= D (the invalid marker) are not counted.  disp: device
 * uint16 [H][W]; umap: device uint16 [D][W]; vmap: device uint16 [H][D].
 * Every count is written (the maps need no clearing beforehand). */
int uv_maps(sgm_ctx *ctx, const sgm_params *p, const uint16_t *disp, uint16_t *umap,
            uint16_t *vmap, void *stream);

/* Obstacle-map filtering of one U- or V-map (section 3.2), in the paper's
 * order; the paper names the steps but gives no sizes, so they are inputs:
 *  1. threshold:  a cell is an obstacle cell when its count >= threshold
 *                 (binary value 255, else 0);
 *  2. dilation:   the maximum over the (2*dilate_r+1)^2 square around each
 *                 cell, cells outside the map ignored;
 *  3. Gaussian:   the binomial kernel of size 2*blur_r+1 (weights
 *                 C(2*blur_r, blur_r+k)) along both axes, borders replicated,
 *                 the exact 2-D sum divided by 4^(2*blur_r) and rounded half up;
 *  4. region of interest: cells outside rows [roi_r0, roi_r1) and columns
 *                 [roi_c0, roi_c1) become 0 (e.g. V-map rows above the horizon).
 *   map: device uint16 [rows][cols] (a U-map [D][W] or a V-map [H][D]);
 *   out: device uint8  [rows][cols], must not overlap map.
 * Limits: 1 <= rows, cols <= 16384; dilate_r <= 8; blur_r <= 4;
 * 0 <= roi_r0 <= roi_r1 <= rows; 0 <= roi_c0 <= roi_c1 <= cols. */
typedef struct {
  const uint16_t *map;
  uint8_t *out;
  int32_t rows, cols;
  uint16_t threshold;
  uint16_t dilate_r;
  uint16_t blur_r;
  uint16_t reserved;  /* must be 0 */
  int32_t roi_r0, roi_r1, roi_c0, roi_c1;
} uv_filter_job;

/* Filter n >= 0 maps with one kernel launch per 24 maps, enqueued on
 * `stream`.  Every job is checked before anything is enqueued; SGM_EINVAL
 * names the first bad job.  Uses no scratch memory. */
int uv_filter(sgm_ctx *ctx, const uv_filter_job *jobs, int n, void *stream);

/* One frame of the whole path for sgm_submit.  left/right: device uint8
 * [H][pitch] sharing one pitch; disp, umap, vmap: device outputs as above
 * (umap and vmap may both be NULL to skip the histograms). */
typedef struct {
  const uint8_t *left, *right;
  int64_t pitch;
  sgm_params p;
  uint16_t *disp, *umap, *vmap;
} sgm_frame;

/* Enqueue the whole path (census .. U/V maps) for n >= 1 frames, which may
 * differ in size and parameters, as one batch on the context's own streams.
 * Results equal those of the stage calls on each frame alone.  The batch's
 * scratch is taken from the context's budget: if it does not fit next to the
 * batches still in flight, returns SGM_EBUSY (retry after sgm_poll); if it
 * can never fit, SGM_ENOMEM.  On success *ticket identifies the batch. */
int sgm_submit(sgm_ctx *ctx, const sgm_frame *frames, int n, uint64_t *ticket);

/* sgm_submit whose batch first waits, on the GPU, for `n_events` HIP events
 * (hipEvent_t passed as void*, recorded by the caller on any stream of the
 * context's device, e.g. after an asynchronous host-to-device copy of the
 * frames' inputs): the batch's stream waits for each event before its first
 * launch, so the caller need not block the host until its copies finish.
 * n_events = 0 (events may then be NULL) behaves as sgm_submit.  SGM_EINVAL
 * for n_events < 0 or a null event; everything else as for sgm_submit.
 * (Used by the request loop of section 3.2's real-time use: frames arrive
 * while earlier ones run.) */
int sgm_submit_after(sgm_ctx *ctx, const sgm_frame *frames, int n, void *const *events, int n_events,
                     uint64_t *ticket);

/* Number of internal streams that consecutive batches rotate over (1 to 8;
 * 4 after sgm_create).  With 1, batches run one after another on the GPU;
 * with more, a batch can start while earlier ones still run.  The streams
 * are created by sgm_create; the HIP runtime maps a process's streams onto a
 * few hardware queues (GPU_MAX_HW_QUEUES, 4 by default) in the order they
 * appear, so a context created after other streams of the process may get
 * two of its streams on one queue and overlap less: create it early, or
 * raise GPU_MAX_HW_QUEUES. */
int sgm_set_streams(sgm_ctx *ctx, int n);

/* Failure path of the two-pass schedule (sgm_schedule.two_pass), for tests
 * that force it from the host: a stripe waits for its neighbour stripe's
 * edge record of each row, and gives up after `max_polls` polls (0 = the
 * default, about 4 million: seconds), records an error and goes on, so the
 * kernel always ends; sgm_poll / sgm_wait then return SGM_EHIP for the batch
 * (its maps are unspecified).  withhold_edges = 1 makes the stripes publish
 * no edge records, so every such wait gives up.  For callers, leave both at
 * 0. */
int sgm_set_stripe_wait(sgm_ctx *ctx, int max_polls, int withhold_edges);
/* Number of the context's streams a batch's frames are spread over (1 to 8;
 * 4 after sgm_create) when it is submitted while no other batch of the
 * context is in flight: the batch is split into up to n groups of about
 * equal work (W*H*D*paths), each enqueued on its own stream and started
 * when the previous group has finished its Census stage, so that one
 * group's Census overlaps another's aggregation and disparity selection;
 * the ticket completes when every group has.  A batch submitted while
 * others are in flight is not split (it overlaps with them on the streams
 * already).  Limited by sgm_set_streams; results are identical.  Graph mode
 * captures batches on one stream and ignores the split; with stage
 * profiling on, stage times are summed over the groups. */
int sgm_set_split(sgm_ctx *ctx, int n);

/* sgm_submit with rectification (section 3.1.1) as the batch's first
 * stage: remaps[2i] and remaps[2i+1] turn frame i's raw left and right images
 * into frames[i].left and frames[i].right, on the batch's own stream, so raw
 * pairs go through the whole path without a host wait.  Each remap's out,
 * out_pitch, w and h must be the frame's view buffer, pitch, width and height
 * (SGM_EINVAL otherwise).  The raw images and the maps must stay valid until
 * the ticket is done; everything else is as for sgm_submit.  (sgm_submit
 * itself does not wait for work the caller enqueued on other streams:
 * results of sgm_rectify on a caller's stream must be complete before the
 * frames are submitted.) */
int sgm_submit_rectify(sgm_ctx *ctx, const sgm_frame *frames, const sgm_remap *remaps, int n,
                       uint64_t *ticket);

/* Graph mode for sgm_submit (0 = off, the default after sgm_create; 1 = on).
 * When on, a batch's launches are captured into a HIP graph; graphs are
 * cached by batch composition (frame shapes, parameters and schedules), and
 * a later batch of the same composition updates the cached executable graph
 * with its buffers and replays it instead of instantiating a new one.
 * Batches submitted while stage profiling is enabled are launched directly. */
int sgm_set_graphs(sgm_ctx *ctx, int on);
/* Batches replayed from the graph cache (hits) and newly instantiated graphs
 * (misses) since sgm_create; either pointer may be NULL. */
int sgm_graph_stats(sgm_ctx *ctx, uint64_t *hits, uint64_t *misses);

/* Non-blocking completion check: *done = 1 once every frame of the ticket's
 * batch is finished (its scratch is then returned to the budget and the
 * ticket forgotten), else 0.  SGM_ENOTFOUND for an unknown ticket. */
int sgm_poll(sgm_ctx *ctx, uint64_t ticket, int *done);

/* Block until the ticket's batch has finished, then behave as sgm_poll.  The
 * calling thread polls; the context stays usable by other threads meanwhile.
 * A ticket is consumed by the first sgm_poll / sgm_wait that finds it done
 * (a later call on it returns SGM_ENOTFOUND). */
int sgm_wait(sgm_ctx *ctx, uint64_t ticket);

/* Work schedule of the whole-path kernels for one frame shape.  Only the
 * speed depends on it; every schedule gives bit-identical results. */
typedef struct {
  /* lanes per horizontal (left-right) scanline in the aggregation: 16, 32 or
   * 64; 0 = the library's default for the shape.  Wider rows shorten the
   * dependent chain along the long image rows; other paths use 16 lanes. */
  int32_t h_lanes;
  /* 1: run eligible frames of the shape through the single-pass row sweep
   * (the paper's forward path set computed in one top-down pass per frame,
   * section 3.1.3, figure 2: one block per frame, nothing but the disparity
   * maps written).  Eligible: Census cost with N_b <= 32, max_disp <= 64,
   * path_mask within SGM_PATHS_PAPER4, N_b + p2 <= 255; other frames ignore
   * the flag.  Pays off on batches of many frames; 0 (default) = the
   * per-direction kernels. */
  int32_t sweep;
  /* threads per block of the disparity-selection kernel (one block per image
   * row or row segment): 256, 512 or 1024; 0 = chosen by the launch's block
   * count (small blocks when there are many rows, large when few). */
  int32_t disp_threads;
  /* Matching costs of the horizontal scanlines (left-right paths):
   * SGM_HCOSTS_DEFAULT (0) = the library's default for the shape;
   * SGM_HCOSTS_VOLUME (1) = read from the cost volume, like every other path;
   * SGM_HCOSTS_CODES (2) = formed in the aggregation from the Census codes:
   * a 64-lane row wave holds the right-view codes of all its disparities and
   * slides them one code per pixel, so the two horizontal paths read 16
   * bytes per pixel instead of D bytes of cost volume.  Applies to Census
   * frames with 64 lanes per horizontal scanline, D in (64, 128] or
   * (192, 256], N_b + p2 <= 255 and W * H * 16 bytes below 2 GiB; other
   * frames use the volume. */
  int32_t h_costs;
  /* The vertical and diagonal paths of 8-path frames (section 3.1.3: one
   * pass over the image, a second from back to front):
   * SGM_TWOPASS_DEFAULT (0) = the library's default for the shape;
   * SGM_TWOPASS_OFF (1) = per-direction kernels for all 8 paths, each path's
   * costs written to memory and summed by the disparity selection;
   * SGM_TWOPASS_WIDE (2) / SGM_TWOPASS_NARROW (3) = a top-down pass for
   * T->B and TL->BR writing their uint16 sum, then a bottom-up pass for B->T
   * and BR->TL that also sums S over all 8 paths and selects the
   * disparities; both passes walk the rows of 64-column (WIDE) or 32-column
   * (NARROW) stripes, one workgroup per stripe.  The four other paths run
   * as per-direction kernels; where the frame's horizontal costs come from
   * the Census codes (h_costs), the two passes form their costs from the
   * same code records instead of reading the cost volume.  Applies to
   * Census frames with all 8 paths and N_b + p2 <= 255 that do not use the
   * single-pass sweep; other frames use the per-direction kernels.  A stripe is one workgroup walking all
   * rows, so the schedule needs many of them: a batch whose two-pass frames
   * have fewer than 128 stripes in all (ceil(width / 64) or ceil(width / 32)
   * per frame) runs them on the per-direction kernels. */
  int32_t two_pass;
} sgm_schedule;
enum { SGM_HCOSTS_DEFAULT = 0, SGM_HCOSTS_VOLUME = 1, SGM_HCOSTS_CODES = 2 };
enum { SGM_TWOPASS_DEFAULT = 0, SGM_TWOPASS_OFF = 1, SGM_TWOPASS_WIDE = 2, SGM_TWOPASS_NARROW = 3 };

/* Set the schedule used by sgm_submit for frames of the shape of `shape`
 * (width, height, max_disp, path_mask and the path-cost width it implies);
 * with shape == NULL, set the default for shapes without an entry. */
int sgm_set_schedule(sgm_ctx *ctx, const sgm_params *shape, const sgm_schedule *s);
/* The schedule sgm_submit would use for `shape` (after defaults). */
int sgm_get_schedule(sgm_ctx *ctx, const sgm_params *shape, sgm_schedule *s);
/* Autotuner: time the n >= 1 frames `samples` (inputs and outputs as for
 * sgm_submit; all of one shape -- width, height, max_disp, path_mask and
 * path-cost width -- else SGM_EINVAL), submitted as one batch, under
 * candidate schedules as the context runs batches -- `reps` submits back
 * to back on its streams (sgm_set_streams, sgm_set_split), in flight
 * together, timed by wall clock until all are done (the better of two such
 * runs), after as many warm-up submits (which also allocate the scratch the
 * timed ones hold) -- and keep
 * the one with the least time per submit for their shape (as
 * sgm_set_schedule);
 * return it in *best (may be NULL).  A batch of the size the caller will
 * submit finds the schedule for that batch size.  The search is by
 * coordinates: h_lanes 16, 32, 64 with horizontal costs from the volume,
 * and 64 lanes with horizontal costs from the Census codes where that
 * applies (per-direction kernels, disp_threads 0); then, with the best of
 * these, the two-pass schedule with wide and with narrow stripes where it
 * applies and the sample has at least 128 stripes (a batch with fewer runs
 * its two-pass frames on the per-direction kernels); then, if the
 * per-direction kernels still win, disp_threads 256,
 * 512, 1024; then, for frames the single-pass sweep can take, the sweep.
 * Blocks until done.
 * `ms`, if non-NULL, receives per-candidate milliseconds for up to `n_ms`
 * candidates in the order h_lanes 16, 32, 64, h_costs codes, two_pass wide,
 * two_pass narrow, disp_threads 256, 512, 1024, sweep (-1 where a candidate
 * does not apply or was not reached).  Must not run concurrently with other
 * submissions on the same context. */
int sgm_autotune(sgm_ctx *ctx, const sgm_frame *samples, int n, int reps, sgm_schedule *best, float *ms,
                 int n_ms);

/* Stage timing of batches (sgm_submit).  While enabled, every stage of a
 * batch is bracketed by HIP events on the batch's stream; when the batch is
 * found done (sgm_poll / sgm_wait) the elapsed times are added per stage.
 * A stage is one kernel launch per group of frames with the same kernel
 * variant (a batch of uniform frames: one launch per stage), except that on
 * the two-pass schedule (sgm_schedule.two_pass) the aggregation stage is the
 * per-direction launch of the four paths run that way, and the disparity
 * stage holds both stripe passes (top-down, then bottom-up with the
 * selection). */
enum {
  SGM_STAGE_CENSUS = 0,
  SGM_STAGE_AGGREGATE = 1,
  SGM_STAGE_DISPARITY = 2,
  SGM_STAGE_MEDIAN = 3,
  SGM_STAGE_UV = 4,
  SGM_STAGE_RECTIFY = 5,  /* sgm_submit_rectify only */
  SGM_NSTAGES = 6
};
int sgm_profile(sgm_ctx *ctx, int enable);
/* ms[SGM_NSTAGES]: summed milliseconds; count[SGM_NSTAGES]: launches summed
 * (either may be NULL).  reset != 0 clears the sums after reading. */
int sgm_profile_read(sgm_ctx *ctx, double *ms, uint64_t *count, int reset);

/* Bytes of budget currently held by in-flight batches, and the budget. */
int sgm_memory(sgm_ctx *ctx, size_t *in_flight_bytes, size_t *budget_bytes);

#ifdef __cplusplus
}
#endif

#endif /* SGM_H */
