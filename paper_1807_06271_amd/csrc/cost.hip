// Matching cost volume of equation (1) with the Census/Hamming similarity:
// C(x,y,d) = popcount(cl(x,y) ^ cr(x-d,y)), or N_b where x - d < 0.
// One block per (row, 64-pixel chunk): the chunk's left codes and the right
// codes it can reach (64 + D - 1) are staged in LDS, then the block writes the
// chunk's cells contiguously -- uint16 one cell per thread for the caller's
// volume, or four uint8 cells per thread (one dword) for the internal padded
// volume that feeds the aggregation.
#include "device_util.h"

namespace sgmk {

constexpr int kCostChunk = 64;

__global__ __launch_bounds__(256) void cost_kernel(JobTable<CostJob> t) {
  __shared__ uint64_t sl[kCostChunk];
  __shared__ uint64_t sr[kCostChunk + 256];
  const int ji = find_job(t.j, t.n, (int)blockIdx.x);
  const CostJob &J = t.j[ji];
  const int tb = (int)blockIdx.x - J.blk0;
  const int y = tb / J.chunks_x;
  const int x0 = (tb % J.chunks_x) * kCostChunk;
  const int nx = min(kCostChunk, J.W - x0);
  const int D = J.D;
  const uint64_t *rl = J.cl + (int64_t)y * J.W;
  const uint64_t *rr = J.cr + (int64_t)y * J.W;
  for (int i = threadIdx.x; i < nx; i += blockDim.x) sl[i] = rl[x0 + i];
  // sr[i] holds cr(x0 - D + 1 + i); positions left of the image are never used
  for (int i = threadIdx.x; i < nx + D - 1; i += blockDim.x) {
    int x = x0 - D + 1 + i;
    sr[i] = x >= 0 ? rr[x] : 0;
  }
  __syncthreads();
  if (J.out16) {
    uint16_t *out = J.out16 + ((int64_t)y * J.W + x0) * D;
    const int total = nx * D;
    for (int c = threadIdx.x; c < total; c += blockDim.x) {
      const int xi = c / D;
      const int d = c - xi * D;
      const int v = (x0 + xi >= d) ? __popcll(sl[xi] ^ sr[xi - d + D - 1]) : J.nbits;
      out[c] = (uint16_t)v;
    }
  } else {
    const int qpp = J.Dp >> 2;  // dwords per pixel
    uint32_t *out = reinterpret_cast<uint32_t *>(J.out8 + ((int64_t)y * J.W + x0) * J.Dp);
    const int total = nx * qpp;
    for (int c = threadIdx.x; c < total; c += blockDim.x) {
      const int xi = c / qpp;
      const int d0 = (c - xi * qpp) * 4;
      uint32_t word = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int d = d0 + b;
        const int v = (d < D && x0 + xi >= d) ? __popcll(sl[xi] ^ sr[xi - d + D - 1]) : J.nbits;
        word |= (uint32_t)v << (8 * b);
      }
      out[c] = word;
    }
  }
}

// ------------------------------------------------- fused Census + cost
// One block per (row, 256-pixel segment).  The block stages the CH image rows
// around y of both views in LDS (clamped halo; the right view also D - 1
// pixels to the left, which the segment's costs reach), computes the Census
// codes of its pixels (left) and of the pixels its disparities reach (right)
// into LDS, then writes the segment's padded uint8 costs.  Saves the Census
// round trip through HBM and two launches per batch; the right-view codes of
// the D - 1 halo pixels are computed twice (by this and the previous
// segment).

constexpr int kSeg = 256;
// Right-view codes a segment reaches: kSeg + D - 1, plus up to 3 more because
// the first one is aligned down to a multiple of 4.  They are stored behind
// kFront unused slots, so that the cost loop may read the codes of pixels
// left of the image (index down to -255, for x = 0 and d0 = 252) from inside
// the array and mask their costs afterwards; LDS slots, swizzled:
// rslot(kRightMax - 1) + 1
constexpr int kRightMax = kSeg + 255 + 3;
constexpr int kFront = 256;  // a multiple of 4: keeps an index's residue mod 4

__host__ __device__ constexpr int swz(int i) { return i + (i >> 2); }
__host__ __device__ constexpr int rslot(int i) { return swz(i + kFront); }
constexpr int kCodeRSlots = swz(kRightMax - 1 + kFront) + 1;
// the lowest index the cost loop reads is x - d0 - 3 - xr0 >= -(256 - 4) - 3
static_assert(kFront % 4 == 0 && kFront - (256 - 4) - 3 >= 0, "front slots too few");

__global__ __launch_bounds__(256) void census_cost_kernel(JobTable<FusedCostJob> t) {
  extern __shared__ uint64_t lds64[];
  const int ji = find_job(t.j, t.n, (int)blockIdx.x);
  const FusedCostJob &J = t.j[ji];
  const int tb = (int)blockIdx.x - J.blk0;
  const int segs = (J.W + kSeg - 1) / kSeg;
  const int y = tb / segs;
  // Blocks are dealt to the 8 XCDs round robin, so with a multiple of 8
  // segments per row the same segment of every row would run on the same XCD
  // -- the first one, whose cells near the left edge take the slower checked
  // path, always on XCD 0.  Rotating the segment order by the row spreads it.
  const int x0 = ((tb - y * segs + y) % segs) * kSeg;
  const int W = J.W, H = J.H, D = J.D, Dp = J.Dp;
  const int nx = min(kSeg, W - x0);
  // first right-view pixel the segment reaches, aligned down to a multiple of
  // 4 so that the cost loop's code indices are 0 mod 4 (fixed LDS offsets)
  const int xr0 = max(0, x0 - D + 1) & ~3;
  const int nr = x0 + nx - xr0;         // right-view codes needed
  const int rx = J.cw / 2, ry = J.ch / 2;
  const int sl = nx + 2 * rx, sr = nr + 2 * rx;  // staged row lengths
  // right-view code i is stored at rslot(i) = swz(i + kFront), swz(i) = i +
  // i/4: the cost loop's lanes read codes 4 apart, and the padding spreads
  // them over all LDS banks
  uint64_t *codeL = lds64;            // [nx]   codes of x0 ..
  uint64_t *codeR = lds64 + kSeg;     // [rslot(nr)] codes of xr0 ..
  uint8_t *rowsL = reinterpret_cast<uint8_t *>(lds64 + kSeg + kCodeRSlots);  // [ch][sl]
  uint8_t *rowsR = rowsL + J.ch * (kSeg + 2 * rx);                       // [ch][sr]
  {
    // the window rows of both views, row by row (no index division); each
    // thread issues a row's loads of both views before storing them
    for (int r = 0; r < J.ch; ++r) {
      const int64_t gy = (int64_t)min(max(y - ry + r, 0), H - 1) * J.pitch;
      const uint8_t *li = J.left + gy, *ri = J.right + gy;
      for (int c0 = threadIdx.x; c0 < sr; c0 += 2 * blockDim.x) {
        const int c1 = c0 + blockDim.x;
        const uint8_t vr0 = ri[min(max(xr0 - rx + c0, 0), W - 1)];
        const uint8_t vr1 = c1 < sr ? ri[min(max(xr0 - rx + c1, 0), W - 1)] : 0;
        const uint8_t vl0 = c0 < sl ? li[min(max(x0 - rx + c0, 0), W - 1)] : 0;
        const uint8_t vl1 = c1 < sl ? li[min(max(x0 - rx + c1, 0), W - 1)] : 0;
        rowsR[r * sr + c0] = vr0;
        if (c1 < sr) rowsR[r * sr + c1] = vr1;
        if (c0 < sl) rowsL[r * sl + c0] = vl0;
        if (c1 < sl) rowsL[r * sl + c1] = vl1;
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nr; i += blockDim.x) {
    codeR[rslot(i)] = census_at(rowsR, sr, i, J.cw, J.ch);
    if (i < nx) codeL[i] = census_at(rowsL, sl, i, J.cw, J.ch);
  }
  __syncthreads();
  if (J.codes) {  // the segment's code records {left, right}, for sliding horizontal windows
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
      const uint64_t rec[2] = {codeL[i], codeR[rslot(x0 + i - xr0)]};
      *reinterpret_cast<U32N<4> *>(J.codes + 2 * ((int64_t)y * W + x0 + i)) = *reinterpret_cast<const U32N<4> *>(rec);
    }
  }
  // each thread keeps one 4-disparity group q of the padded row and walks
  // the segment 4 pixels at a time: the 16 cells of pixels x..x+3 and
  // disparities d0..d0+3 use the 7 right-view codes x-d0-3 .. x-d0+3
  const int qpp = Dp >> 2;               // dwords per pixel (16..64)
  const int groups = blockDim.x / qpp;   // 4-pixel groups per sweep
  const int q = threadIdx.x % qpp, g = threadIdx.x / qpp;
  if (g >= groups) return;
  const int d0 = q * 4;
  // the segment's cost rows through one buffer descriptor: a lane stores at
  // byte (xi + p) * Dp + 4q, the pixel term p * Dp a scalar offset
  const __amdgpu_buffer_rsrc_t orow = row_rsrc(J.out8 + ((int64_t)y * W + x0) * Dp, (uint32_t)(nx * Dp));
  // padded disparities d0 + b >= D cost N_b: byte b of every word is kept
  // (keep) or replaced (fill)
  const uint32_t nb = (uint32_t)J.nbits;
  uint32_t keep = 0, fill = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    if (d0 + b < D) keep |= 0xFFu << (8 * b);
    else fill |= nb << (8 * b);
  }
  for (int xi = 4 * g; xi < nx; xi += 4 * groups) {
    const int x = x0 + xi;
    const uint32_t vo = (uint32_t)(xi * Dp + 4 * q);
    if (xi + 3 < nx) {
      // codes x - d0 - 3 .. x - d0 + 3 at indices a .. a + 6, a = 1 (mod 4):
      // rslot(a + k) = rslot(a) + k + (1 + k) / 4, one base address.  Code k
      // serves the cells p - b = k - 3; it lies left of the image when
      // x - d0 + k - 3 < 0, possible only while x < d0 + 3 (left of Dp - 1):
      // the whole wave then takes the masked variant, one branch per wave
      const int a = x - d0 - xr0 - 3;
      const uint64_t *cb = codeR + rslot(a);
      uint64_t r[7];
#pragma unroll
      for (int k = 0; k < 7; ++k) r[k] = cb[k + ((1 + k) >> 2)];
      const int t = x - d0;
      // EDGE: merge N_b into the costs of codes left of the image; PAD: apply
      // keep / fill (frames with D < Dp)
      auto tile = [&](auto edge, auto pad) {
        constexpr bool EDGE = decltype(edge)::value, PAD = decltype(pad)::value;
        // left[k]: all ones when code k lies left of the image (merged
        // bitwise: a conditional expression here becomes a branch per cell)
        uint32_t left[7];
        if constexpr (EDGE) {
#pragma unroll
          for (int k = 0; k < 7; ++k) left[k] = (uint32_t)((t + k - 3) >> 31);
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const uint64_t cl = codeL[xi + p];
          uint32_t word = 0;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int k = p - b + 3;
            uint32_t c = (uint32_t)__popcll(cl ^ r[k]);
            if constexpr (EDGE) c = (left[k] & nb) | (~left[k] & c);
            word |= c << (8 * b);
          }
          if constexpr (PAD) word = (word & keep) | fill;
          __builtin_amdgcn_raw_buffer_store_b32(word, orow, vo, p * Dp, 0);
        }
      };
      using T = std::integral_constant<bool, true>;
      using F = std::integral_constant<bool, false>;
      if (__builtin_amdgcn_ballot_w64(t < 3) != 0) tile(T{}, T{});
      else if (D != Dp) tile(F{}, T{});
      else tile(F{}, F{});
    } else {
      for (int p = 0; p < 4 && xi + p < nx; ++p) {  // the segment's last < 4 pixels
        const int xp = x + p;
        const uint64_t cl = codeL[xi + p];
        uint32_t word = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int d = d0 + b;
          const int v = (d < D && xp >= d) ? __popcll(cl ^ codeR[rslot(max(xp - d - xr0, 0))]) : J.nbits;
          word |= (uint32_t)v << (8 * b);
        }
        __builtin_amdgcn_raw_buffer_store_b32(word, orow, vo, p * Dp, 0);
      }
    }
  }
}

size_t fused_cost_lds(int D, int cw, int ch) {
  (void)D;
  // codes: kSeg left + kCodeRSlots right; rows: ch x (kSeg + cw - 1) left and
  // ch x (kRightMax + cw - 1) right
  return (size_t)(kSeg + kCodeRSlots) * 8 + (size_t)ch * (kSeg + cw - 1) +
         (size_t)ch * (kRightMax + cw - 1);
}

void launch_census_cost(std::vector<FusedCostJob> jobs, hipStream_t s) {
  size_t lds = 0;
  for (auto &j : jobs) lds = std::max(lds, fused_cost_lds(j.D, j.cw, j.ch));
  for_each_table(
      jobs, [](const FusedCostJob &j) { return (long)j.H * ((j.W + kSeg - 1) / kSeg); },
      [&](const JobTable<FusedCostJob> &t, int blocks) {
        hipLaunchKernelGGL(census_cost_kernel, dim3(blocks), dim3(256), lds, s, t);
      });
}

// ------------------------------------------------------------ SAD cost
// One block per (row, 64-pixel chunk): the window rows of both views around
// y are staged in LDS (clamped; the right view D - 1 pixels further left).
//
// With u = x + dx the window column, the left pixel is clamp(u) and the right
// one clamp(u - d): both depend on u and d only.  So with the column sums
//   V_d(u) = sum_dy |I_L(clamp(u), y+dy) - I_R(clamp(u - d), y+dy)|
// the cost is the sum of V_d over the ww columns u = x-rx .. x+rx, and one
// thread per (d, run of kSadRun pixels) forms the run's column sums once and
// slides the window over them.  Output: a uint16 [H][W][stride] volume
// (stride D for the caller's volume, Dp for the padded internal one).
constexpr int kSadRun = 16;

__device__ __forceinline__ uint32_t absdiff(uint32_t a, uint32_t b) { return a > b ? a - b : b - a; }

template <int WW, int WH>
__device__ __forceinline__ void sad_run(const uint8_t *L, int sl, const uint8_t *R, int sr, int xs, int nrun,
                                        int d, int D, int os, int x0, uint32_t cmax, uint16_t *out) {
  uint32_t V[kSadRun + WW - 1];
#pragma unroll
  for (int c = 0; c < kSadRun + WW - 1; ++c) {
    uint32_t v = 0;
#pragma unroll
    for (int dy = 0; dy < WH; ++dy) v += absdiff(L[dy * sl + xs + c], R[dy * sr + xs + c - d + D - 1]);
    V[c] = v;
  }
  uint32_t acc = 0;
#pragma unroll
  for (int c = 0; c < WW - 1; ++c) acc += V[c];
#pragma unroll
  for (int k = 0; k < kSadRun; ++k) {
    acc += V[k + WW - 1];
    if (k < nrun) out[(int64_t)(xs + k) * os] = (uint16_t)(x0 + xs + k >= d ? acc : cmax);
    acc -= V[k];
  }
}

// Any window: the direct sum per cell.
__device__ __forceinline__ void sad_run_any(const uint8_t *L, int sl, const uint8_t *R, int sr, int xs,
                                            int nrun, int d, int D, int os, int x0, uint32_t cmax, int ww,
                                            int wh, uint16_t *out) {
  for (int k = 0; k < nrun; ++k) {
    uint32_t acc = cmax;
    if (x0 + xs + k >= d) {
      acc = 0;
      for (int dy = 0; dy < wh; ++dy)
        for (int dx = 0; dx < ww; ++dx)
          acc += absdiff(L[dy * sl + xs + k + dx], R[dy * sr + xs + k + dx - d + D - 1]);
    }
    out[(int64_t)(xs + k) * os] = (uint16_t)acc;
  }
}

__global__ __launch_bounds__(256) void sad_kernel(JobTable<SadJob> t) {
  extern __shared__ uint8_t srows[];
  const int ji = find_job(t.j, t.n, (int)blockIdx.x);
  const SadJob &J = t.j[ji];
  const int tb = (int)blockIdx.x - J.blk0;
  const int y = tb / J.chunks_x;
  const int x0 = (tb % J.chunks_x) * kCostChunk;
  const int W = J.W, H = J.H, D = J.D;
  const int nx = min(kCostChunk, W - x0);
  const int rx = J.ww / 2, ry = J.wh / 2;
  // rows of the full chunk width (clamped past the image), so that every
  // column a run touches is staged
  const int sl = kCostChunk + 2 * rx;          // left: pixels x0 - rx .. x0 + 63 + rx
  const int sr = kCostChunk + D - 1 + 2 * rx;  // right: pixels x0 - D + 1 - rx ..
  uint8_t *L = srows, *R = srows + J.wh * sl;
  for (int i = threadIdx.x; i < J.wh * sr; i += blockDim.x) {
    const int r = i / sr, c = i - r * sr;
    const int64_t gy = (int64_t)min(max(y - ry + r, 0), H - 1) * J.pitch;
    R[r * sr + c] = J.right[gy + min(max(x0 - D + 1 - rx + c, 0), W - 1)];
    if (c < sl) L[r * sl + c] = J.left[gy + min(max(x0 - rx + c, 0), W - 1)];
  }
  __syncthreads();
  const uint32_t cmax = (uint32_t)J.ww * J.wh * 255u;
  const int os = J.ostride;
  uint16_t *row = J.out + ((int64_t)y * W + x0) * os;
  const int nruns = (nx + kSadRun - 1) / kSadRun;
  // consecutive threads take consecutive d of one run: coalesced stores
  for (int task = threadIdx.x; task < nruns * D; task += blockDim.x) {
    const int run = task / D, d = task - run * D;
    const int xs = run * kSadRun, nrun = min(kSadRun, nx - xs);
    uint16_t *o = row + d;  // cell (x0 + xs + k, d) is o[(xs + k) * os]
    if (J.ww == 5 && J.wh == 5) sad_run<5, 5>(L, sl, R, sr, xs, nrun, d, D, os, x0, cmax, o);
    else if (J.ww == 3 && J.wh == 3) sad_run<3, 3>(L, sl, R, sr, xs, nrun, d, D, os, x0, cmax, o);
    else if (J.ww == 7 && J.wh == 7) sad_run<7, 7>(L, sl, R, sr, xs, nrun, d, D, os, x0, cmax, o);
    else if (J.ww == 9 && J.wh == 7) sad_run<9, 7>(L, sl, R, sr, xs, nrun, d, D, os, x0, cmax, o);
    else sad_run_any(L, sl, R, sr, xs, nrun, d, D, os, x0, cmax, J.ww, J.wh, o);
  }
}

size_t sad_lds(int D, int ww, int wh) {
  // each run reads up to kSadRun + ww - 1 columns from its start; the last
  // run starts at kCostChunk - kSadRun, so rows of kCostChunk + ww - 1 suffice
  return (size_t)wh * (kCostChunk + ww - 1) + (size_t)wh * (kCostChunk + D - 1 + ww - 1);
}

void launch_sad(std::vector<SadJob> jobs, hipStream_t s) {
  size_t lds = 0;
  for (auto &j : jobs) {
    j.chunks_x = (j.W + kCostChunk - 1) / kCostChunk;
    lds = std::max(lds, sad_lds(j.D, j.ww, j.wh));
  }
  for_each_table(
      jobs, [](const SadJob &j) { return (long)j.chunks_x * j.H; },
      [&](const JobTable<SadJob> &t, int blocks) {
        hipLaunchKernelGGL(sad_kernel, dim3(blocks), dim3(256), lds, s, t);
      });
}

void launch_cost(std::vector<CostJob> jobs, hipStream_t s) {
  for (auto &j : jobs) j.chunks_x = (j.W + kCostChunk - 1) / kCostChunk;
  for_each_table(
      jobs, [](const CostJob &j) { return (long)j.chunks_x * j.H; },
      [&](const JobTable<CostJob> &t, int blocks) {
        hipLaunchKernelGGL(cost_kernel, dim3(blocks), dim3(256), 0, s, t);
      });
}

}  // namespace sgmk
