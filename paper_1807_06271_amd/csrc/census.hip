// Census transform (section 3.1.2; Census with Hamming distance after Zabih
// and Woodfill): one thread per pixel, the tile and its clamped halo staged in
// LDS so each image byte is read from HBM about once.
#include "device_util.h"

namespace sgmk {

constexpr int kCTW = 64;  // tile width  (pixels)
constexpr int kCTH = 16;  // tile height (pixels)

__global__ __launch_bounds__(256) void census_kernel(JobTable<CensusJob> t) {
  extern __shared__ uint8_t tile[];
  const int ji = find_job(t.j, t.n, (int)blockIdx.x);
  const CensusJob &J = t.j[ji];
  const int tb = (int)blockIdx.x - J.blk0;
  const int x0 = (tb % J.tiles_x) * kCTW;
  const int y0 = (tb / J.tiles_x) * kCTH;
  const int rx = J.cw >> 1, ry = J.ch >> 1;
  const int tw = kCTW + 2 * rx, th = kCTH + 2 * ry;
  // stage the tile with a clamped halo (edge replicate)
  for (int i = threadIdx.x; i < tw * th; i += blockDim.x) {
    int lx = i % tw, ly = i / tw;
    int gx = min(max(x0 - rx + lx, 0), J.W - 1);
    int gy = min(max(y0 - ry + ly, 0), J.H - 1);
    tile[i] = J.img[(int64_t)gy * J.pitch + gx];
  }
  __syncthreads();
  const int tx = threadIdx.x & (kCTW - 1);
  const int x = x0 + tx;
  if (x >= J.W) return;
  for (int ty = threadIdx.x >> 6; ty < kCTH; ty += 4) {
    const int y = y0 + ty;
    if (y >= J.H) break;
    J.out[(int64_t)y * J.ostride + x] = census_at(tile + ty * tw, tw, tx, J.cw, J.ch);
  }
}

void launch_census(std::vector<CensusJob> jobs, hipStream_t s) {
  int maxlds = 0;
  for (auto &j : jobs) {
    j.tiles_x = (j.W + kCTW - 1) / kCTW;
    maxlds = std::max(maxlds, (kCTW + j.cw - 1) * (kCTH + j.ch - 1));
  }
  for_each_table(
      jobs, [](const CensusJob &j) { return (long)j.tiles_x * ((j.H + kCTH - 1) / kCTH); },
      [&](const JobTable<CensusJob> &t, int blocks) {
        hipLaunchKernelGGL(census_kernel, dim3(blocks), dim3(256), maxlds, s, t);
      });
}

}  // namespace sgmk
