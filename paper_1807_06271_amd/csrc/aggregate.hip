// Semi-global path aggregation (section 3.1.3; equation (2) read as
// Hirschmueller's per-path recurrence with the predecessor's minimum
// subtracted after every pixel):
//
//   L_r(p,d) = C(p,d) + min(L_r(p-r,d), L_r(p-r,d-1)+P1, L_r(p-r,d+1)+P1, m+P2) - m,
//   m = min_k L_r(p-r,k),   L_r(p,d) = C(p,d) at the first pixel of a path.
//
// Work decomposition: one 64-lane wavefront per scanline of one direction;
// the disparity axis is spread over the lanes, DPL contiguous disparities per
// lane (d = lane*DPL + k).  The d-1 / d+1 neighbours that live in the
// adjacent lane come over DPP (wave_shr / wave_shl by one lane); the per-step
// minimum over d is a DPP row reduction followed by row broadcasts and one
// readlane, so the whole recurrence stays in registers and the only memory
// traffic is reading C (or the two Census rows) and writing L_r.  All
// directions of all frames of a batch are waves of the same launch, so the
// many short diagonal scanlines fill the chip next to the long ones.
#include "device_util.h"

namespace sgmk {

__device__ __constant__ int kDirDx[8] = {+1, -1, 0, 0, +1, -1, -1, +1};
__device__ __constant__ int kDirDy[8] = {0, 0, +1, -1, +1, -1, +1, -1};

int agg_lines(int dir, int W, int H) {
  if (dir < 2) return H;
  if (dir < 4) return W;
  return W + H - 1;
}

// First pixel and length of scanline `line` of direction `dir`.
__device__ __forceinline__ void line_start(int dir, int line, int W, int H, int &sx, int &sy,
                                           int &len) {
  switch (dir) {
    case 0: sx = 0; sy = line; len = W; break;
    case 1: sx = W - 1; sy = line; len = W; break;
    case 2: sx = line; sy = 0; len = H; break;
    case 3: sx = line; sy = H - 1; len = H; break;
    case 4:  // (+1,+1): top row, then the left column below it
      if (line < W) { sx = line; sy = 0; } else { sx = 0; sy = line - W + 1; }
      len = min(W - sx, H - sy);
      break;
    case 5:  // (-1,-1): bottom row, then the right column above it
      if (line < W) { sx = line; sy = H - 1; } else { sx = W - 1; sy = line - W; }
      len = min(sx + 1, sy + 1);
      break;
    case 6:  // (-1,+1): top row, then the right column below it
      if (line < W) { sx = line; sy = 0; } else { sx = W - 1; sy = line - W + 1; }
      len = min(sx + 1, H - sy);
      break;
    default:  // 7, (+1,-1): bottom row, then the left column above it
      if (line < W) { sx = line; sy = H - 1; } else { sx = 0; sy = line - W; }
      len = min(W - sx, sy + 1);
      break;
  }
}

constexpr uint32_t kInf = 0x3FFFFFFFu;  // above any path cost, safe to add P1/P2 to

template <int DPL, int SRC>
__device__ __forceinline__ void load_costs(const AggJob &J, int x, int y, int dbase,
                                           uint32_t (&c)[DPL]) {
  const int64_t pix = (int64_t)y * J.W + x;
  if (SRC == kFromCost) {
    const uint16_t *row = J.cost + pix * J.D;
#pragma unroll
    for (int k = 0; k < DPL; ++k) c[k] = (dbase + k < J.D) ? row[dbase + k] : 0u;
  } else {
    const uint64_t cl = J.cl[pix];
    const uint64_t *cr = J.cr + pix;  // cr[-d] is the right code at x - d
#pragma unroll
    for (int k = 0; k < DPL; ++k) {
      const int d = dbase + k;
      const uint64_t r = cr[-min(d, x)];  // clamped index: never reads left of the row
      c[k] = (d < J.D && x >= d) ? (uint32_t)__popcll(cl ^ r) : (uint32_t)J.nbits;
    }
  }
}

template <int DPL, int SRC, typename LT>
__global__ __launch_bounds__(256) void agg_kernel(JobTable<AggJob> t) {
  const int gw = uniform((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  const int lane = (int)(threadIdx.x & 63);
  const int ji = find_job(t.j, t.n, gw);
  const AggJob &J = t.j[ji];
  const int w = gw - J.blk0;
  if (w >= J.line0[J.ndirs]) return;  // whole wave: tail of the grid
  int slot = 0;
  for (int k = 1; k < J.ndirs; ++k)
    if (w >= J.line0[k]) slot = k;
  const int dir = J.dirs[slot];
  int sx, sy, len;
  line_start(dir, w - J.line0[slot], J.W, J.H, sx, sy, len);
  const int dx = kDirDx[dir], dy = kDirDy[dir];
  const int D = J.D;
  const uint32_t p1 = (uint32_t)J.p1, p2 = (uint32_t)J.p2;
  LT *out = reinterpret_cast<LT *>(J.lr) + (int64_t)slot * J.H * J.W * D;
  const int dbase = lane * DPL;

  uint32_t Lp[DPL];
  uint32_t mp = 0;
  uint32_t c[DPL];
  int x = sx, y = sy;
  load_costs<DPL, SRC>(J, x, y, dbase, c);
  for (int i = 0; i < len; ++i) {
    // issue the next pixel's loads before this pixel's arithmetic
    uint32_t cn[DPL];
    const int xn = x + dx, yn = y + dy;
    if (i + 1 < len) load_costs<DPL, SRC>(J, xn, yn, dbase, cn);
    uint32_t Lc[DPL];
    if (i == 0) {
#pragma unroll
      for (int k = 0; k < DPL; ++k) Lc[k] = (dbase + k < D) ? c[k] : kInf;
    } else {
      const uint32_t lo = from_lower_lane(Lp[DPL - 1], kInf);  // L(d-1) for k = 0
      const uint32_t hi = from_upper_lane(Lp[0], kInf);        // L(d+1) for k = DPL-1
      const uint32_t mP2 = mp + p2;
#pragma unroll
      for (int k = 0; k < DPL; ++k) {
        const uint32_t l = (k == 0) ? lo : Lp[k - 1];
        const uint32_t r = (k == DPL - 1) ? hi : Lp[k + 1];
        const uint32_t best = min(min(Lp[k], min(l, r) + p1), mP2);
        Lc[k] = (dbase + k < D) ? c[k] + best - mp : kInf;
      }
    }
    LT *o = out + ((int64_t)y * J.W + x) * D + dbase;
    uint32_t lm = Lc[0];
#pragma unroll
    for (int k = 0; k < DPL; ++k) {
      if (dbase + k < D) o[k] = (LT)Lc[k];
      lm = min(lm, Lc[k]);
      Lp[k] = Lc[k];
    }
    mp = wave_min_u32(lm);
    x = xn;
    y = yn;
#pragma unroll
    for (int k = 0; k < DPL; ++k) c[k] = cn[k];
  }
}

template <int DPL, int SRC, typename LT>
static void launch_one(const JobTable<AggJob> &t, int waves, hipStream_t s) {
  const int blocks = (waves + 3) / 4;
  hipLaunchKernelGGL((agg_kernel<DPL, SRC, LT>), dim3(blocks), dim3(256), 0, s, t);
}

template <int SRC, typename LT>
static void launch_dpl(int dpl, const JobTable<AggJob> &t, int waves, hipStream_t s) {
  switch (dpl) {
    case 1: launch_one<1, SRC, LT>(t, waves, s); break;
    case 2: launch_one<2, SRC, LT>(t, waves, s); break;
    case 3: launch_one<3, SRC, LT>(t, waves, s); break;
    default: launch_one<4, SRC, LT>(t, waves, s); break;
  }
}

void launch_aggregate(std::vector<AggJob> jobs, AggSource src, int dpl, int lr_bytes,
                      hipStream_t s) {
  for (auto &j : jobs) {
    int total = 0;
    for (int k = 0; k < j.ndirs; ++k) {
      j.line0[k] = total;
      total += agg_lines(j.dirs[k], j.W, j.H);
    }
    j.line0[j.ndirs] = total;
  }
  for_each_table(
      jobs, [](const AggJob &j) { return (long)j.line0[j.ndirs]; },
      [&](const JobTable<AggJob> &t, int waves) {
        if (src == kFromCost) {
          if (lr_bytes == 1) launch_dpl<kFromCost, uint8_t>(dpl, t, waves, s);
          else launch_dpl<kFromCost, uint16_t>(dpl, t, waves, s);
        } else {
          if (lr_bytes == 1) launch_dpl<kFromCensus, uint8_t>(dpl, t, waves, s);
          else launch_dpl<kFromCensus, uint16_t>(dpl, t, waves, s);
        }
      });
}

// S = sum over the P slots of the path-cost volumes; 4 cells per thread.
template <typename LT>
__global__ __launch_bounds__(256) void sum_kernel(JobTable<SumJob> t) {
  const int ji = find_job(t.j, t.n, (int)blockIdx.x);
  const SumJob &J = t.j[ji];
  const int64_t base = ((int64_t)((int)blockIdx.x - J.blk0) * 256 + threadIdx.x) * 4;
  const LT *lr = reinterpret_cast<const LT *>(J.lr);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t i = base + q;
    if (i >= J.cells) break;
    uint32_t s = 0;
    for (int p = 0; p < J.P; ++p) s += lr[(int64_t)p * J.cells + i];
    J.S[i] = (uint16_t)s;
  }
}

void launch_sum(std::vector<SumJob> jobs, int lr_bytes, hipStream_t s) {
  for_each_table(
      jobs, [](const SumJob &j) { return (long)((j.cells + 1023) / 1024); },
      [&](const JobTable<SumJob> &t, int blocks) {
        if (lr_bytes == 1) hipLaunchKernelGGL(sum_kernel<uint8_t>, dim3(blocks), dim3(256), 0, s, t);
        else hipLaunchKernelGGL(sum_kernel<uint16_t>, dim3(blocks), dim3(256), 0, s, t);
      });
}

}  // namespace sgmk
