// Internal interface between the C-ABI layer (api.hip) and the HIP kernels.
//
// Every kernel takes a small table of "jobs" by value (one job = one frame's
// share of that stage) so that one launch can cover a whole batch of frames
// of different sizes; a single-frame call is a table of one.  A job records
// the first block index it owns (blk0); a block finds its job by scanning the
// table (at most kMaxJobs entries, all in the kernel-argument segment).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace sgmk {

constexpr int kMaxJobs = 24;  // jobs per launch (kernel arguments stay < 4 KB)

// ---------------------------------------------------------------- census
struct CensusJob {
  const uint8_t *img;
  int64_t pitch;
  uint64_t *out;  // [H][ostride], codes of a row at out + y * ostride
  int W, H, cw, ch;
  int ostride;    // codes per output row (>= W)
  int blk0, tiles_x;
};
void launch_census(std::vector<CensusJob> jobs, hipStream_t s);

// ------------------------------------------------------------------ cost
// Hamming costs of equation (1).  out16 != null: the caller's uint16
// [H][W][D] volume.  Otherwise out8: the internal uint8 [H][W][Dp] volume
// (Dp = 16 * agg_k(D); cells with d >= D hold N_b).
struct CostJob {
  const uint64_t *cl, *cr;
  uint16_t *out16;
  uint8_t *out8;
  int W, H, D, Dp, nbits;
  int blk0, chunks_x;
};
void launch_cost(std::vector<CostJob> jobs, hipStream_t s);

// Census of both views and the padded uint8 costs of one row segment per
// block (LDS holds the segment's codes and the image rows of the window).
struct FusedCostJob {
  const uint8_t *left, *right;
  int64_t pitch;
  uint8_t *out8;    // [H][W][Dp]
  uint64_t *codes;  // or null: the Census code records {left, right} per pixel [H][W]
  int W, H, D, Dp, nbits, cw, ch;
  int blk0;
};
// LDS bytes of the fused kernel (at most ~75 KiB for a 65-row window).
size_t fused_cost_lds(int D, int cw, int ch);
void launch_census_cost(std::vector<FusedCostJob> jobs, hipStream_t s);

// SAD costs over a ww x wh window into the uint16 [H][W][D] volume.
struct SadJob {
  const uint8_t *left, *right;
  int64_t pitch;
  uint16_t *out;       // [H][W][ostride], cells d < D written
  int W, H, D, ww, wh;
  int ostride;         // D (the caller's volume) or Dp (internal, padded)
  int blk0, chunks_x;
};
// LDS bytes of the SAD kernel (window rows of both views for one chunk).
size_t sad_lds(int D, int ww, int wh);
void launch_sad(std::vector<SadJob> jobs, hipStream_t s);

// ----------------------------------------------------------- aggregation
// Disparities per lane for D (16 lanes per scanline): 4, 8, 12 or 16.
int agg_k(int D);
// Number of scanlines of direction `dir` on a W x H image.
__host__ __device__ int agg_lines(int dir, int W, int H);

struct AggJob {
  const uint8_t *cost8;          // internal padded uint8 costs [H][W][Dp], or
  const uint16_t *cost16;        // internal padded uint16 costs [H][W][Dp]
  const uint64_t *codes;         // sliding horizontal windows: Census code records
                                 // {left, right} per pixel [H][W], Dp readable
                                 // records before the first one
  int nbits;                     // N_b (sliding windows)
  void *lr;                      // path costs [P][H][W][Dp], uint8 or uint16
  int W, H, D, Dp, p1, p2;
  int ndirs;                     // P = number of active directions
  int dirs[8];                   // direction index of each slot
  int line0[9];                  // first wave of each slot; line0[P] = waves of the job
  int blk0;                      // first global wave of this job
};
// K = agg_k(D) of every job; hlps: lanes per horizontal scanline (16, 32 or
// 64; falls back to 16 where the layout does not fit K); lr_bytes: 1 or 2;
// slide: the horizontal waves form their costs from the jobs' Census code
// records (where agg_slide_ok holds and the volumes are uint8; ignored
// elsewhere).
void launch_aggregate(std::vector<AggJob> jobs, bool from_cost16, int K, int hlps, int lr_bytes, bool slide,
                      hipStream_t s);
bool agg_hlps_ok(int K, int hlps);
bool agg_slide_ok(int K, int hlps);
// Copy uint16 costs [px][D] into the padded layout [px][Dp] (pad cells 0).
void launch_pad16(const uint16_t *src, uint16_t *dst, int64_t px, int D, int Dp, hipStream_t s);

// S (unpadded uint16 [H][W][D]) = sum over the P slots of the padded path costs.
struct SumJob {
  const void *lr;
  uint16_t *S;
  int64_t cells;  // H * W * D
  int D, Dp, P;
  int blk0;
};
void launch_sum(std::vector<SumJob> jobs, int lr_bytes, hipStream_t s);

// ------------------------------------------------ disparity selection
// WTA, right-view disparity and left-right check for one image row per
// block.  Input is either S (caller's unpadded uint16) or the P padded path
// cost volumes, summed on the fly.
struct DispJob {
  const uint16_t *S;  // [H][W][D] or null
  const void *lr;     // [P][H][W][Dp] or null
  int P;
  uint16_t *out;      // [H][W]: D_L (the LR pass's input when lr_check = 1)
  uint32_t *part;     // lr_check: per row segment, the right-view keys of its zone
  int W, H, D, Dp;
  int lr_check;
  int nseg, seglen;   // row segments (disp_segments)
  int threads;        // block size (256, 512, 1024), 0: chosen by the launch's block count
  int blk0;
};
// Row segments of the disparity kernel: with split, nseg segments of seglen
// pixels (seglen >= D - 1 unless one segment covers the row), so that a
// frame alone gives enough blocks; without, whole rows.  Batches whose rows
// already fill the chip use whole rows (fewer, longer blocks).
void disp_segments(int W, int D, bool split, int *nseg, int *seglen);
constexpr int kDispSplitRows = 1024;  // split rows when a launch has fewer
// Bytes of DispJob::part for a frame (enough for either choice).
size_t disp_part_bytes(int W, int H, int D);
// Left-right check from D_L and the segments' right-view keys.
struct LRSegJob {
  const uint16_t *dl;
  const uint32_t *part;
  uint16_t *out;
  int W, H, D, nseg, seglen, max_diff, invalid;
  int blk0;
};
void launch_lr_seg(std::vector<LRSegJob> jobs, hipStream_t s);
// in_kind: 0 = S, 1 = uint8 path costs, 2 = uint16 path costs
void launch_disparity(std::vector<DispJob> jobs, int in_kind, hipStream_t s);

struct MedianJob {
  const uint16_t *in;  // the map to filter (lr == 0)
  uint16_t *out;
  int W, H, k;
  // lr == 1: the input is the LR check of D_L against the segments' keys,
  // formed in the median kernel (the fields of LRSegJob)
  int lr;
  const uint16_t *dl;
  const uint32_t *part;
  int D, nseg, seglen, max_diff, invalid;
  int blk0, tiles_x;
};
void launch_median(std::vector<MedianJob> jobs, hipStream_t s);

// --------------------------------------------------------------- U/V maps
// Every count of U and V is written once (no zero fill needed).
struct UVJob {
  const uint16_t *disp;
  uint16_t *U, *V;  // [D][W], [H][D]
  int W, H, D;
  int blk0;         // first block; blocks [blk0, blk0+H) build V rows,
  int ublocks;      // then `ublocks` blocks build 16-column strips of U
};
void launch_uv(std::vector<UVJob> jobs, hipStream_t s);


// ------------------------------------------------- two-pass stripes
// The vertical and two diagonal paths of an 8-path frame (T->B and TL->BR in
// a top-down pass, B->T and BR->TL in a bottom-up pass), one workgroup per
// stripe of 4 * waves columns; the up pass also sums S over all 8 paths and
// selects D_L and the right-view keys (disparity kernel layout, segments of
// one stripe).  Eligible frames: Census costs (uint8 volume), uint8 path
// costs, all 8 paths.
struct StripeJob {
  const uint8_t *cost;  // [H][W][Dp] (launches without codes)
  const uint64_t *codes;  // launches with codes: Census code records {left, right} per pixel [H][W]
                          // (Dp zero records before pixel 0)
  int nbits;              // N_b: the cost where x - d < 0
  uint16_t *sd;         // S_D = L_TB + L_TLBR + L_LR + L_RL, uint16 [H][W][Dp] (down: written, up: read)
  const uint8_t *lr4;   // the uint8 path costs of L->R, R->L (read by the down pass), TR->BL, BL->TR
                        // (read by the up pass) [4][H][W][Dp]
  uint64_t *bnd;        // [nstripes][H][Dp / 2]: each stripe's published edge pixel per row
  uint32_t *sync;       // [0] down ticket counter, [1] error flag, [2] up ticket counter
  uint16_t *dl;         // up: D_L [H][W]
  uint32_t *part;       // up with lr_check: [H][nstripes][4 * waves + D - 1] zone keys
  int W, H, D, Dp, p1, p2, lr_check;
  int nstripes;         // set by launch_stripes
  uint32_t epoch;       // tag of this launch's edge words (never 0, new per launch)
  int max_polls;        // polls before a wait for a neighbour's edge gives up
  int withhold;         // 1: publish no edges (tests of the failure path only)
  int blk0;
};
constexpr int kSyncWords = 4;
// LDS bytes of a stripe workgroup (up: the bottom-up pass).
size_t stripe_lds(int K, int D, int waves, bool up, bool codes);
// One launch per job table; K = agg_k(D) of every job; waves: 8 or 16;
// codes: costs formed from every job's Census code records (K = 8 or 16)
// instead of read from the cost volume.
void launch_stripes(std::vector<StripeJob> jobs, int K, bool up, int waves, bool codes, hipStream_t s);
struct SyncZeroJob {
  uint32_t *p;
  int words;
  int blk0;
};
void launch_zero_sync(std::vector<SyncZeroJob> jobs, hipStream_t s);

// ----------------------------------------------------- single-pass sweep
// The forward path set {L2R, TL2BR, T2B, TR2BL} (all predecessors lie above
// or to the left) in one top-down sweep per frame: costs from the Census
// codes, S, D_L and D_R formed on chip; only the disparity maps are written.
// Eligible frames: Census cost with N_b <= 32, D <= 64, forward paths only,
// uint8 path costs (N_b + P2 <= 255).
constexpr int kSweepCarry = 256;  // bytes per pixel of a band-boundary row
struct SweepJob {
  const uint64_t *cl, *cr;  // Census codes [H][W]
  uint16_t *dl, *dr;        // D_L and D_R [H][W]
  uint8_t *carry;           // [2][W + 2][kSweepCarry]: columns for pixels -1 .. W
  int64_t stride;           // bytes between the buffers of consecutive frames
  int count;                // frames of this job (one block each)
  int W, H, D, nbits, p1, p2;
  uint32_t mask;
  int blk0;
};
void launch_sweep(std::vector<SweepJob> jobs, hipStream_t s);
// Left-right check of D_L against D_R (or D_L itself when lr_check = 0).
struct LRJob {
  const uint16_t *dl, *dr;
  uint16_t *out;
  int W, H, lr_check, max_diff, invalid;
  int blk0;
};
void launch_lr(std::vector<LRJob> jobs, hipStream_t s);

// -------------------------------------------------------- U/V filtering
// Threshold, dilation, binomial Gaussian and region of interest of one map
// (section 3.2), one block per 64 x 16 output tile.
constexpr int kUVFMaxDil = 8, kUVFMaxBlur = 4;
struct UVFilterJob {
  const uint16_t *map;
  uint8_t *out;
  int rows, cols, thr, dil, blur;
  int r0, r1, c0, c1;
  int tiles_x, blk0;
};
void launch_uv_filter(std::vector<UVFilterJob> jobs, hipStream_t s);

// ------------------------------------------------------------ rectify
// Gather through integer remap maps (section 3.1.1).  Pixels are taken in
// groups of kRectPx consecutive entries of the [h][w] maps.
constexpr int kRectPx = 8;
struct RemapJob {
  const uint8_t *src;
  const uint16_t *mx, *my;  // [h][w]
  uint8_t *out;             // [h][out_pitch]
  int64_t src_pitch, out_pitch;
  int src_w, src_h, w, h;
  int vec;                  // maps 16-byte aligned: 128-bit map loads
  int blk0;
};
void launch_rectify(std::vector<RemapJob> jobs, hipStream_t s);

}  // namespace sgmk
