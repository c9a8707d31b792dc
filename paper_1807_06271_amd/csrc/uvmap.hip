// U-/V-maps (section 3.2): per-column and per-row histograms of the final
// disparity map, each count written once with a plain store (no atomics in
// global memory, no zero fill beforehand):
//   blocks [0, H):     V row y from an LDS histogram [D];
//   following blocks:  U for one 16-column strip over all rows, from an LDS
//                      histogram [D][16] (counts <= H <= 16384 fit 16 bits).
#include "device_util.h"

namespace sgmk {

constexpr int kUCols = 16;

__global__ __launch_bounds__(256) void uv_kernel(JobTable<UVJob> t) {
  extern __shared__ uint32_t hist[];
  const int ji = find_job(t.j, t.n, (int)blockIdx.x);
  const UVJob &J = t.j[ji];
  const int b = (int)blockIdx.x - J.blk0;
  const int W = J.W, H = J.H, D = J.D;
  if (b < H) {
    const int y = b;
    for (int i = threadIdx.x; i < D; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const uint16_t *row = J.disp + (int64_t)y * W;
    for (int x = threadIdx.x; x < W; x += blockDim.x) {
      const int d = row[x];
      if (d < D) atomicAdd(&hist[d], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < D; d += blockDim.x) J.V[(int64_t)y * D + d] = (uint16_t)hist[d];
  } else {
    const int x0 = (b - H) * kUCols;
    for (int i = threadIdx.x; i < D * kUCols; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const int xl = threadIdx.x & (kUCols - 1);
    const int x = x0 + xl;
    constexpr int kRowsPerPass = 256 / kUCols;
    if (x < W) {
      // eight rows per thread in flight, then their LDS updates
      for (int y = (int)threadIdx.x / kUCols; y < H; y += 8 * kRowsPerPass) {
        uint32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int yy = y + k * kRowsPerPass;
          v[k] = yy < H ? J.disp[(int64_t)yy * W + x] : 0xFFFFu;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (v[k] < (uint32_t)D) atomicAdd(&hist[v[k] * kUCols + xl], 1u);
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < D * kUCols; i += blockDim.x) {
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
        hipLaunchKernelGGL(uv_kernel, dim3(blocks), dim3(256), lds, s, t);
      });
}

}  // namespace sgmk
