// U-/V-maps (section 3.2): per-column and per-row histograms of the final
// disparity map.
//   blocks [0, H):   V row y, built in an LDS histogram and written once;
//   following blocks: U for one 64-column strip over a chunk of 64 rows, built
//   in an LDS histogram [D][64] and added into the (zeroed) U-map with 32-bit
//   atomics on the word holding each 16-bit count (counts <= H <= 65535, so
//   a half never carries into its neighbour).
#include "device_util.h"

namespace sgmk {

constexpr int kUStrip = 64;
constexpr int kURows = 64;

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
    const int strips = (W + kUStrip - 1) / kUStrip;
    const int u = b - H;
    const int x0 = (u % strips) * kUStrip;
    const int y0 = (u / strips) * kURows;
    const int y1 = min(H, y0 + kURows);
    for (int i = threadIdx.x; i < D * kUStrip; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const int xl = threadIdx.x & (kUStrip - 1);
    const int x = x0 + xl;
    if (x < W) {
      for (int y = y0 + (int)(threadIdx.x >> 6); y < y1; y += 4) {
        const int d = J.disp[(int64_t)y * W + x];
        if (d < D) atomicAdd(&hist[d * kUStrip + xl], 1u);
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < D * kUStrip; i += blockDim.x) {
      const uint32_t n = hist[i];
      const int xi = x0 + (i & (kUStrip - 1));
      if (n == 0 || xi >= W) continue;
      uint16_t *cell = J.U + (int64_t)(i / kUStrip) * W + xi;
      const uintptr_t a = reinterpret_cast<uintptr_t>(cell);
      atomicAdd(reinterpret_cast<uint32_t *>(a & ~(uintptr_t)3), n << ((a & 2) ? 16 : 0));
    }
  }
}

void launch_uv(std::vector<UVJob> jobs, hipStream_t s) {
  int maxd = 1;
  for (auto &j : jobs) {
    j.ublocks = ((j.W + kUStrip - 1) / kUStrip) * ((j.H + kURows - 1) / kURows);
    maxd = std::max(maxd, j.D);
  }
  const size_t lds = (size_t)maxd * kUStrip * sizeof(uint32_t);
  for_each_table(
      jobs, [](const UVJob &j) { return (long)j.H + j.ublocks; },
      [&](const JobTable<UVJob> &t, int blocks) {
        hipLaunchKernelGGL(uv_kernel, dim3(blocks), dim3(256), lds, s, t);
      });
}

// Zero-fill of uint16 buffers (U-maps before accumulation).
__global__ __launch_bounds__(256) void zero_kernel(JobTable<ZeroJob> t) {
  const int ji = find_job(t.j, t.n, (int)blockIdx.x);
  const ZeroJob &J = t.j[ji];
  const int64_t i = (int64_t)((int)blockIdx.x - J.blk0) * 256 + threadIdx.x;
  if (i < J.n) J.p[i] = 0;
}

void launch_zero(std::vector<ZeroJob> jobs, hipStream_t s) {
  for_each_table(
      jobs, [](const ZeroJob &j) { return (long)((j.n + 255) / 256); },
      [&](const JobTable<ZeroJob> &t, int blocks) {
        hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, s, t);
      });
}

}  // namespace sgmk
