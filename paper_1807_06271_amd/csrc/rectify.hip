// Rectification by precomputed maps (section 3.1.1): out(p) = src(Mx(p), My(p)),
// 0 where the map points outside the raw image.  Each thread gathers kRectPx
// consecutive map entries; the maps are read with 128-bit loads, the source
// bytes come through the caches (the maps of a real calibration are locally
// smooth, so neighbouring threads read neighbouring source rows), and a
// group that lies in one output row is written with one 64-bit store.
#include "device_util.h"

namespace sgmk {

__global__ __launch_bounds__(256) void rectify_kernel(JobTable<RemapJob> t) {
  const int ji = find_job(t.j, t.n, (int)blockIdx.x);
  const RemapJob &J = t.j[ji];
  const int64_t n = (int64_t)J.w * J.h;
  const int64_t p0 = ((int64_t)((int)blockIdx.x - J.blk0) * 256 + threadIdx.x) * kRectPx;
  if (p0 >= n) return;
  uint16_t mx[kRectPx], my[kRectPx];
  if (J.vec && p0 + kRectPx <= n) {
    const uint4 a = *reinterpret_cast<const uint4 *>(J.mx + p0);
    const uint4 b = *reinterpret_cast<const uint4 *>(J.my + p0);
    const uint32_t aw[4] = {a.x, a.y, a.z, a.w}, bw[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      mx[2 * k] = (uint16_t)aw[k];
      mx[2 * k + 1] = (uint16_t)(aw[k] >> 16);
      my[2 * k] = (uint16_t)bw[k];
      my[2 * k + 1] = (uint16_t)(bw[k] >> 16);
    }
  } else {
#pragma unroll
    for (int k = 0; k < kRectPx; ++k) {
      const bool in = p0 + k < n;
      mx[k] = in ? J.mx[p0 + k] : (uint16_t)0xFFFF;
      my[k] = in ? J.my[p0 + k] : (uint16_t)0xFFFF;
    }
  }
  uint8_t v[kRectPx];
#pragma unroll
  for (int k = 0; k < kRectPx; ++k) {
    const bool ok = (int)mx[k] < J.src_w && (int)my[k] < J.src_h;
    v[k] = ok ? J.src[(int64_t)my[k] * J.src_pitch + mx[k]] : (uint8_t)0;
  }
  int y = (int)(p0 / J.w), x = (int)(p0 - (int64_t)y * J.w);
  uint8_t *dst = J.out + (int64_t)y * J.out_pitch + x;
  if (x + kRectPx <= J.w && (reinterpret_cast<uintptr_t>(dst) & 7) == 0) {
    uint2 w;
    w.x = v[0] | (uint32_t)v[1] << 8 | (uint32_t)v[2] << 16 | (uint32_t)v[3] << 24;
    w.y = v[4] | (uint32_t)v[5] << 8 | (uint32_t)v[6] << 16 | (uint32_t)v[7] << 24;
    *reinterpret_cast<uint2 *>(dst) = w;
    return;
  }
#pragma unroll
  for (int k = 0; k < kRectPx; ++k) {
    if (p0 + k >= n) break;
    J.out[(int64_t)y * J.out_pitch + x] = v[k];
    if (++x == J.w) {
      x = 0;
      ++y;
    }
  }
}

void launch_rectify(std::vector<RemapJob> jobs, hipStream_t s) {
  for_each_table(
      jobs,
      [](const RemapJob &j) {
        const int64_t groups = ((int64_t)j.w * j.h + kRectPx - 1) / kRectPx;
        return (long)((groups + 255) / 256);
      },
      [&](const JobTable<RemapJob> &t, int blocks) {
        hipLaunchKernelGGL(rectify_kernel, dim3(blocks), dim3(256), 0, s, t);
      });
}

}  // namespace sgmk
