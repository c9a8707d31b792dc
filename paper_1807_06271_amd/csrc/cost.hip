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

void launch_cost(std::vector<CostJob> jobs, hipStream_t s) {
  for (auto &j : jobs) j.chunks_x = (j.W + kCostChunk - 1) / kCostChunk;
  for_each_table(
      jobs, [](const CostJob &j) { return (long)j.chunks_x * j.H; },
      [&](const JobTable<CostJob> &t, int blocks) {
        hipLaunchKernelGGL(cost_kernel, dim3(blocks), dim3(256), 0, s, t);
      });
}

}  // namespace sgmk
