// U-/V-maps (section 3.2): per-column and per-row histograms of the final
// disparity map, each count written once with a plain store (no atomics in
// global memory, no zero fill beforehand):
//   blocks [0, H):     V row y from an LDS histogram [D];
//   following blocks:  U for one 16-column strip over all rows, from an LDS
//                      histogram [D][16] (counts <= H <= 16384 fit 16 bits).
// Each thread walks a contiguous run of pixels (along the row for V, down a
// column for U) and adds every stretch of equal disparities with one LDS
// atomic: disparity maps are piecewise smooth, so neighbouring pixels mostly
// share a bin, and one add per pixel would make the lanes of a wave queue on
// the same LDS address.
#include "device_util.h"

namespace sgmk {

constexpr int kUCols = 16;
constexpr int kUVThreads = 256;

// Adds the run lengths of a thread's n values p[0], p[step], ... (p[i *
// step] for i < n) to hist[v * hstride + hoff], one atomic per stretch of
// equal values; values >= D are not counted.  Eight values are loaded at a
// time so that the loads overlap.
__device__ __forceinline__ void count_runs(const uint16_t *p, int64_t step, int n, uint32_t *hist, int hstride,
                                           int hoff, uint32_t D) {
  uint32_t cur = 0xFFFFFFFFu, cnt = 0;
  for (int i0 = 0; i0 < n; i0 += 8) {
    uint32_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = i0 + k < n ? p[(int64_t)(i0 + k) * step] : 0xFFFFFFFFu;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (i0 + k >= n) break;
      if (v[k] != cur) {
        if (cur < D) atomicAdd(&hist[cur * hstride + hoff], cnt);
        cur = v[k];
        cnt = 0;
      }
      ++cnt;
    }
  }
  if (cur < D) atomicAdd(&hist[cur * hstride + hoff], cnt);
}

__global__ __launch_bounds__(kUVThreads) void uv_kernel(JobTable<UVJob> t) {
  extern __shared__ uint32_t hist[];
  const int ji = find_job(t.j, t.n, (int)blockIdx.x);
  const UVJob &J = t.j[ji];
  const int b = (int)blockIdx.x - J.blk0;
  const int W = J.W, H = J.H;
  const uint32_t D = (uint32_t)J.D;
  if (b < H) {
    const int y = b;
    for (int i = threadIdx.x; i < (int)D; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const uint16_t *row = J.disp + (int64_t)y * W;
    // thread t counts pixels [t * c, (t + 1) * c) of the row
    const int c = (W + kUVThreads - 1) / kUVThreads;
    const int xa = (int)threadIdx.x * c, xe = min(W, xa + c);
    if (xa < xe) count_runs(row + xa, 1, xe - xa, hist, 1, 0, D);
    __syncthreads();
    for (int d = threadIdx.x; d < (int)D; d += blockDim.x) J.V[(int64_t)y * D + d] = (uint16_t)hist[d];
  } else {
    const int x0 = (b - H) * kUCols;
    for (int i = threadIdx.x; i < (int)D * kUCols; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const int xl = threadIdx.x & (kUCols - 1);
    const int x = x0 + xl;
    // thread (xl, r) counts rows [r * c, (r + 1) * c) of column x0 + xl; the
    // 16 columns of a row segment are read together (32 contiguous bytes)
    constexpr int kGroups = kUVThreads / kUCols;
    const int c = (H + kGroups - 1) / kGroups;
    const int r = (int)threadIdx.x / kUCols;
    const int ya = r * c, ye = min(H, ya + c);
    if (x < W && ya < ye) count_runs(J.disp + (int64_t)ya * W + x, W, ye - ya, hist, kUCols, xl, D);
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
