// U-/V-maps (section 3.2): per-column and per-row histograms of the final
// disparity map, built in LDS with atomic adds and written once.
//   blocks [0, H):          V row y      (hist[D])
//   blocks [H, H+ublocks):  U columns of one 64-wide strip (hist[D][64])
#include "device_util.h"

namespace sgmk {

constexpr int kUStrip = 64;

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
    const int x0 = (b - H) * kUStrip;
    for (int i = threadIdx.x; i < D * kUStrip; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const int xl = threadIdx.x & (kUStrip - 1);
    const int x = x0 + xl;
    if (x < W) {
      for (int y = threadIdx.x >> 6; y < H; y += 4) {
        const int d = J.disp[(int64_t)y * W + x];
        if (d < D) atomicAdd(&hist[d * kUStrip + xl], 1u);
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < D * kUStrip; i += blockDim.x) {
      const int d = i / kUStrip, xi = x0 + (i & (kUStrip - 1));
      if (xi < W) J.U[(int64_t)d * W + xi] = (uint16_t)hist[i];
    }
  }
}

void launch_uv(std::vector<UVJob> jobs, hipStream_t s) {
  int maxd = 1;
  for (auto &j : jobs) {
    j.ublocks = (j.W + kUStrip - 1) / kUStrip;
    maxd = std::max(maxd, j.D);
  }
  const size_t lds = (size_t)maxd * kUStrip * sizeof(uint32_t);
  for_each_table(
      jobs, [](const UVJob &j) { return (long)j.H + j.ublocks; },
      [&](const JobTable<UVJob> &t, int blocks) {
        hipLaunchKernelGGL(uv_kernel, dim3(blocks), dim3(256), lds, s, t);
      });
}

}  // namespace sgmk
