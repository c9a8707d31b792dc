// Obstacle-map filtering of U-/V-maps (section 3.2): threshold -> dilation ->
// binomial Gaussian -> region of interest.  One block per 64 x 16 output
// tile: the binary tile with its halo (dilation radius + blur radius) is
// staged in LDS, the square dilation runs as a row max then a column max,
// the Gaussian as a row pass then a column pass with replicated borders, all
// in integers, so the result is exact.
#include "device_util.h"

namespace sgmk {

constexpr int kFTW = 64, kFTH = 16;                        // output tile
constexpr int kFHalo = kUVFMaxDil + kUVFMaxBlur;           // largest halo
constexpr int kFAW = kFTW + 2 * kFHalo, kFAH = kFTH + 2 * kFHalo;

// C(2b, b+k) for b = 0..4, k = -b..b (row b, entries 0..2b)
__device__ __constant__ uint32_t kBinom[kUVFMaxBlur + 1][2 * kUVFMaxBlur + 1] = {
    {1}, {1, 2, 1}, {1, 4, 6, 4, 1}, {1, 6, 15, 20, 15, 6, 1}, {1, 8, 28, 56, 70, 56, 28, 8, 1}};

__global__ __launch_bounds__(256) void uv_filter_kernel(JobTable<UVFilterJob> t) {
  __shared__ uint8_t A[kFAH * kFAW];                       // binary map + halo
  __shared__ uint8_t H1[kFAH * (kFTW + 2 * kUVFMaxBlur)];  // row max
  __shared__ uint8_t DL[(kFTH + 2 * kUVFMaxBlur) * (kFTW + 2 * kUVFMaxBlur)];  // dilated
  __shared__ uint32_t G1[(kFTH + 2 * kUVFMaxBlur) * kFTW];  // row blur
  const int ji = find_job(t.j, t.n, (int)blockIdx.x);
  const UVFilterJob &J = t.j[ji];
  const int tb = (int)blockIdx.x - J.blk0;
  const int x0 = (tb % J.tiles_x) * kFTW, y0 = (tb / J.tiles_x) * kFTH;
  const int R = J.dil, B = J.blur, h = R + B;
  const int aw = kFTW + 2 * h, ah = kFTH + 2 * h;  // A: rows y0-h.., cols x0-h..
  const int dw = kFTW + 2 * B, dh = kFTH + 2 * B;  // H1 cols / DL: rows y0-B.., cols x0-B..
  // 1. threshold (cells outside the map are 0: they never raise a maximum)
  for (int i = threadIdx.x; i < ah * aw; i += blockDim.x) {
    const int r = i / aw, c = i - r * aw;
    const int y = y0 - h + r, x = x0 - h + c;
    uint8_t b = 0;
    if (y >= 0 && y < J.rows && x >= 0 && x < J.cols) b = J.map[(int64_t)y * J.cols + x] >= J.thr;
    A[i] = b;
  }
  __syncthreads();
  // 2. dilation: max over columns x-R..x+R, then rows y-R..y+R
  for (int i = threadIdx.x; i < ah * dw; i += blockDim.x) {
    const int r = i / dw, c = i - r * dw;
    uint8_t m = 0;
    for (int k = 0; k <= 2 * R; ++k) m |= A[r * aw + c + k];
    H1[r * dw + c] = m;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < dh * dw; i += blockDim.x) {
    const int r = i / dw, c = i - r * dw;
    uint8_t m = 0;
    for (int k = 0; k <= 2 * R; ++k) m |= H1[(r + k) * dw + c];
    DL[i] = m;
  }
  __syncthreads();
  // 3. Gaussian along rows, neighbours clamped to the map's columns
  for (int i = threadIdx.x; i < dh * kFTW; i += blockDim.x) {
    const int r = i / kFTW, c = i - r * kFTW;
    uint32_t acc = 0;
    for (int k = -B; k <= B; ++k) {
      const int xc = min(max(x0 + c + k, 0), J.cols - 1);
      acc += kBinom[B][B + k] * DL[r * dw + xc - (x0 - B)];
    }
    G1[i] = acc;
  }
  __syncthreads();
  // ... then along columns, neighbours clamped to the map's rows; round and
  // apply the region of interest
  const int shift = 4 * B;
  for (int i = threadIdx.x; i < kFTH * kFTW; i += blockDim.x) {
    const int r = i / kFTW, c = i - r * kFTW;
    const int y = y0 + r, x = x0 + c;
    if (y >= J.rows || x >= J.cols) continue;
    uint32_t acc = 0;
    for (int k = -B; k <= B; ++k) {
      const int yc = min(max(y + k, 0), J.rows - 1);
      acc += kBinom[B][B + k] * G1[(yc - (y0 - B)) * kFTW + c];
    }
    acc *= 255u;
    const uint32_t g = shift ? (acc + (1u << (shift - 1))) >> shift : acc;
    const bool in = y >= J.r0 && y < J.r1 && x >= J.c0 && x < J.c1;
    J.out[(int64_t)y * J.cols + x] = in ? (uint8_t)g : (uint8_t)0;
  }
}

void launch_uv_filter(std::vector<UVFilterJob> jobs, hipStream_t s) {
  for (auto &j : jobs) j.tiles_x = (j.cols + kFTW - 1) / kFTW;
  for_each_table(
      jobs, [](const UVFilterJob &j) { return (long)j.tiles_x * ((j.rows + kFTH - 1) / kFTH); },
      [&](const JobTable<UVFilterJob> &t, int blocks) {
        hipLaunchKernelGGL(uv_filter_kernel, dim3(blocks), dim3(256), 0, s, t);
      });
}

}  // namespace sgmk
