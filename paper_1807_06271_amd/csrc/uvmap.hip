// U-/V-maps (section 3.2): per-column and per-row histograms of the final
// disparity map, each count written once with a plain store (no atomics in
// global memory, no zero fill beforehand):
//   blocks [0, H):     V row y from an LDS histogram [D];
//   following blocks:  U for one 16-column strip over all rows, from an LDS
//                      histogram [D][16] (counts <= H <= 16384).
// Disparity maps are piecewise smooth, so neighbouring pixels mostly share a
// bin; adding one per pixel would make the lanes of a wave queue on one LDS
// address.  Both halves add whole runs of equal values instead:
//   V: a wave takes 64 consecutive pixels of the row at a time, and only the
//      last lane of each run of equal values (found with a ballot) adds the
//      run's length, so one instruction's lanes meet on an address only when
//      a value recurs after another within 64 pixels;
//   U: each thread walks down a stretch of one column, adding each run of
//      equal values once; the 16 columns of a wave's row segment are read
//      together (32 contiguous bytes).
#include "device_util.h"

namespace sgmk {

constexpr int kUCols = 16;
constexpr int kUVThreads = 256;
constexpr int kUVWaves = kUVThreads / 64;
constexpr uint32_t kNoBin = 0xFFFFFFFFu;  // beyond the row: never counted

__global__ __launch_bounds__(kUVThreads) void uv_kernel(JobTable<UVJob> t) {
  extern __shared__ uint32_t hist[];
  const int ji = find_job(t.j, t.n, (int)blockIdx.x);
  const UVJob &J = t.j[ji];
  const int b = (int)blockIdx.x - J.blk0;
  const int W = J.W, H = J.H;
  const uint32_t D = (uint32_t)J.D;
  const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
  if (b < H) {
    const int y = b;
    for (int i = threadIdx.x; i < (int)D; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const uint16_t *row = J.disp + (int64_t)y * W;
    const uint64_t below = (1ull << lane) - 1;  // lanes under this one
    for (int c0 = wave * 64; c0 < W; c0 += kUVWaves * 64) {
      const int x = c0 + lane;
      const uint32_t v = x < W ? row[x] : kNoBin;
      // the next lane's value (lane 63's run always ends here)
      const uint32_t nx = (uint32_t)__builtin_amdgcn_update_dpp((int)~v, (int)v, kDppWaveShl1, 0xF, 0xF, false);
      const bool ends = v != nx;
      const uint64_t ends_mask = __builtin_amdgcn_ballot_w64(ends);
      const uint64_t prev = ends_mask & below;  // run ends before this lane
      const int start = prev ? 64 - __builtin_clzll(prev) : 0;
      if (ends && v < D) atomicAdd(&hist[v], (uint32_t)(lane + 1 - start));
    }
    __syncthreads();
    for (int d = threadIdx.x; d < (int)D; d += blockDim.x) J.V[(int64_t)y * D + d] = (uint16_t)hist[d];
  } else {
    const int x0 = (b - H) * kUCols;
    for (int i = threadIdx.x; i < (int)D * kUCols; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    // thread (xl, r) counts rows [r * c, (r + 1) * c) of column x0 + xl
    const int xl = threadIdx.x & (kUCols - 1);
    const int x = x0 + xl;
    constexpr int kGroups = kUVThreads / kUCols;
    const int c = (H + kGroups - 1) / kGroups;
    const int r = (int)threadIdx.x / kUCols;
    const int ya = r * c, ye = min(H, ya + c);
    if (x < W && ya < ye) {
      const uint16_t *p = J.disp + (int64_t)ya * W + x;
      const int n = ye - ya;
      uint32_t cur = kNoBin, cnt = 0;
      for (int i0 = 0; i0 < n; i0 += 8) {
        uint32_t v[8];  // eight rows' loads in flight
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = i0 + k < n ? p[(int64_t)(i0 + k) * W] : kNoBin;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          if (i0 + k >= n) break;
          if (v[k] != cur) {
            if (cur < D) atomicAdd(&hist[cur * kUCols + xl], cnt);
            cur = v[k];
            cnt = 0;
          }
          ++cnt;
        }
      }
      if (cur < D) atomicAdd(&hist[cur * kUCols + xl], cnt);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < (int)D * kUCols; i += blockDim.x) {
      const int xi = x0 + (i & (kUCols - 1));
      if (xi < W) J.U[(int64_t)(i / kUCols) * W + xi] = (uint16_t)hist[i];
    }
  }
}

void launch_uv(std::vector<UVJob> jobs, hipStream_t s) {
  int maxd = 1;
  for (auto &j : jobs) {
    j.ublocks = (j.W + kUCols - 1) / kUCols;
    maxd = std::max(maxd, j.D);
  }
  const size_t lds = (size_t)maxd * kUCols * sizeof(uint32_t);
  for_each_table(
      jobs, [](const UVJob &j) { return (long)j.H + j.ublocks; },
      [&](const JobTable<UVJob> &t, int blocks) {
        hipLaunchKernelGGL(uv_kernel, dim3(blocks), dim3(kUVThreads), lds, s, t);
      });
}

}  // namespace sgmk
