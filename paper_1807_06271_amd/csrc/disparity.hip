// Disparity selection from the aggregated volume (sections 3.1.3 to 3.1.5).
//
// disp_kernel: one block per (row, segment).  Each 16-lane DPP row takes one
// pixel at a time, lane j owning K contiguous disparities (the same lane
// layout as the aggregation).  With path-cost volumes as input the P uint8
// (or uint16) volumes are read with one vector load per slot and summed as
// packed 16-bit fields (two cells per 32-bit word, no carries: S <= 65535 by
// the parameter check).  A cell's 32-bit key (S << 8) | d orders by cost,
// then by disparity, so an unsigned minimum picks the smallest-d argmin: D_L
// is the minimum key over d (DPP row butterfly), and D_R(x_r) =
// argmin_d S(x_r + d, d) collects the same keys by LDS atomicMin into slot
// x - d.  A segment [x0, x0 + n) reaches the right-view pixels of its zone
// [x0 - D + 1, x0 + n); it writes its D_L and its zone's keys, and the LR
// check (lr_value) takes for each x_r the minimum over the segments whose
// zones hold it (at most two of this kernel's segments; up to
// (D - 1) / n + 1 of the two-pass schedule's stripes, which use the same
// layout), then checks left against right: in
// lr_seg_kernel, or inside median_kernel when a median follows.  Splitting
// rows keeps every CU busy on a single frame.
//
// median_kernel: k x k median with clamped borders by a pruned sorting
// network on k*k registers; with the LR check in front of it,
// it forms the checked values of its tile and halo itself.
#include <utility>

#include "device_util.h"

namespace sgmk {

// LDS slot of the right-view key of zone position i.  The 16 lanes of a
// 16-lane row update positions K apart (one disparity each) and the rows of
// a wave handle consecutive pixels, i.e. positions one apart.  With two
// padding slots after every K positions (K a power of two) the lanes of a
// row land on 16 banks that are all even or all odd, and the next row's on
// the other 16, so a half wave (two rows) updates 32 different banks; a K
// boundary between two rows' positions shifts by 2 and keeps the parity.
template <int K>
__host__ __device__ constexpr int kswz(int i) {
  if constexpr ((K & (K - 1)) == 0) return i + 2 * (i / K);
  else return i + (i >> 3);
}
// LDS slots for n zone positions.
template <int K>
__host__ __device__ constexpr int kswz_slots(int n) { return n > 0 ? kswz<K>(n - 1) + 1 : 1; }

// Raw words of one pixel for one lane: IN 0 = K values of the caller's S
// (one per word); IN 1 = K bytes of each of the P (<= 8) uint8 path-cost
// slots; IN 2 = K 16-bit values of each uint16 slot.  Loading and summing are
// separate so that a pixel's loads can be issued one sweep ahead.
template <int K, int IN>
struct RawSums {
  static constexpr int NW = IN == 0 ? K : IN == 1 ? 8 * (K / 4) : 8 * (K / 2);
  uint32_t w[NW];
};

template <int K, int IN>
__device__ __forceinline__ void load_raw(const DispJob &J, int64_t pix, int dbase, int dvalid,
                                         RawSums<K, IN> &r) {
  if (IN == 0) {
    const uint16_t *q = J.S + pix * J.D + dbase;
#pragma unroll
    for (int k = 0; k < K; ++k) r.w[k] = k < dvalid ? q[k] : 0u;
  } else {
    constexpr int WPS = IN == 1 ? K / 4 : K / 2;  // words per slot
    const int64_t slot = (int64_t)J.H * J.W * J.Dp * (IN == 1 ? 1 : 2);
    const char *b = reinterpret_cast<const char *>(J.lr) + (pix * J.Dp + dbase) * (IN == 1 ? 1 : 2);
#pragma unroll
    for (int p = 0; p < 8; ++p)
      if (p < J.P) {
        const U32N<WPS> v = load_nt<WPS>(b + p * slot);  // each path cost is read once
#pragma unroll
        for (int i = 0; i < WPS; ++i) r.w[p * WPS + i] = v.v[i];
      }
  }
}

// Summed costs S of the lane's K disparities (d >= D lanes get garbage that
// is never used).  Path-cost slots are summed as packed 16-bit fields (two
// cells per 32-bit word, no carries: S <= 65535 by the parameter check).
template <int K, int IN>
__device__ __forceinline__ void sum_raw(const DispJob &J, const RawSums<K, IN> &r, uint32_t (&S)[K]) {
  if (IN == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) S[k] = r.w[k];
  } else if (IN == 1) {
    uint32_t ev[K / 4], od[K / 4];
#pragma unroll
    for (int q = 0; q < K / 4; ++q) ev[q] = od[q] = 0;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      if (p >= J.P) break;
#pragma unroll
      for (int q = 0; q < K / 4; ++q) {
        const uint32_t v = r.w[p * (K / 4) + q];
        ev[q] += v & 0x00FF00FFu;         // d = 4q, 4q+2 in the low/high half
        od[q] += (v >> 8) & 0x00FF00FFu;  // d = 4q+1, 4q+3
      }
    }
#pragma unroll
    for (int q = 0; q < K / 4; ++q) {
      S[4 * q] = ev[q] & 0xFFFF;
      S[4 * q + 1] = od[q] & 0xFFFF;
      S[4 * q + 2] = ev[q] >> 16;
      S[4 * q + 3] = od[q] >> 16;
    }
  } else {
    uint32_t acc[K / 2];
#pragma unroll
    for (int q = 0; q < K / 2; ++q) acc[q] = 0;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      if (p >= J.P) break;
#pragma unroll
      for (int q = 0; q < K / 2; ++q) acc[q] += r.w[p * (K / 2) + q];  // two 16-bit sums per word
    }
#pragma unroll
    for (int q = 0; q < K / 2; ++q) {
      S[2 * q] = acc[q] & 0xFFFF;
      S[2 * q + 1] = acc[q] >> 16;
    }
  }
}

// Pixels per 16-lane row per sweep, sized so that the raw words of the
// current and the next sweep stay in registers.
template <int K, int IN>
struct DispShape {
  static constexpr int RAW = RawSums<K, IN>::NW;
  static constexpr int NPX = RAW <= 16 ? 2 : 1;
};

// Threads per block for a launch of `blocks` (row, segment) blocks: small
// blocks when there are many, so that several share a CU and one block's
// barrier and tail overlap another's loads; large ones when there are few, so
// that the launch still fills the chip.  Measured on MI355X: 1242x375 D=128
// (1 500 blocks) 43 / 45 / 54 us with 256 / 512 / 1024 threads, 640x360
// D=60 (720) 12.1 / 10.5 / 13.1 us, 320x240 D=64 (240) 18.1 / 11.8 /
// 10.2 us.
inline int disp_threads(long blocks) { return blocks >= 1024 ? 256 : blocks >= 512 ? 512 : 1024; }

void disp_segments(int W, int D, bool split, int *nseg, int *seglen) {
  const int target = std::max(256, 2 * D);
  const int n = split ? std::max(1, W / target) : 1;
  *nseg = n;
  *seglen = (W + n - 1) / n;
}

size_t disp_part_bytes(int W, int H, int D) {
  // H * nseg * (seglen + D - 1) grows with nseg: size for the split case
  int nseg, seglen;
  disp_segments(W, D, true, &nseg, &seglen);
  return (size_t)H * nseg * (seglen + D - 1) * 4;
}

template <int K, int IN, int THREADS>
__global__ __launch_bounds__(THREADS) void disp_kernel(JobTable<DispJob> t) {
  constexpr int NPX = DispShape<K, IN>::NPX;
  extern __shared__ uint32_t smem[];
  const int ji = find_job(t.j, t.n, (int)blockIdx.x);
  const DispJob &J = t.j[ji];
  const int b = (int)blockIdx.x - J.blk0;
  const int y = b / J.nseg, sgi = b - y * J.nseg;
  const int W = J.W, D = J.D;
  const int xa = sgi * J.seglen, xe = min(W, xa + J.seglen);  // the segment [xa, xe)
  const int zr = xa - D + 1, zn = xe - zr;                     // its right-view zone
  // D_R keys of zone position i live at kswz<K>(i)
  uint32_t *keyR = smem;  // [kswz_slots<K>(zn)]
  if (J.lr_check)
    for (int i = threadIdx.x; i < kswz_slots<K>(zn); i += blockDim.x) keyR[i] = 0xFFFFFFFFu;
  __syncthreads();
  const int j = threadIdx.x & 15;
  const int dbase = j * K;
  const int dvalid = min(K, max(0, D - dbase));
  // NPX pixels per 16-lane row per sweep, and the next sweep's loads are
  // issued before this sweep's keys are reduced (software pipeline)
  const int kRows = (int)blockDim.x / 16;
  const int xfirst = xa + (int)(threadIdx.x >> 4);
  RawSums<K, IN> raw[NPX], rawn[NPX];
#pragma unroll
  for (int h = 0; h < NPX; ++h)
    load_raw<K, IN>(J, (int64_t)y * W + min(xfirst + h * kRows, xe - 1), dbase, dvalid, raw[h]);
  for (int x0 = xfirst; x0 < xe; x0 += NPX * kRows) {
    const int xn = x0 + NPX * kRows;
    if (xn < xe) {
#pragma unroll
      for (int h = 0; h < NPX; ++h)
        load_raw<K, IN>(J, (int64_t)y * W + min(xn + h * kRows, xe - 1), dbase, dvalid, rawn[h]);
    }
#pragma unroll
    for (int h = 0; h < NPX; ++h) {
      const int x = x0 + h * kRows;
      if (x >= xe) break;  // uniform over the 16-lane row
      uint32_t S[K];
      sum_raw<K, IN>(J, raw[h], S);
      uint32_t best = 0xFFFFFFFFu;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (k < dvalid) {
          const int d = dbase + k;
          const uint32_t key = (S[k] << 8) | (uint32_t)d;
          best = min(best, key);
          if (J.lr_check && x >= d) atomicMin(&keyR[kswz<K>(x - d - zr)], key);
        }
      }
      best = row16_allmin_u32(best);
      if (j == 0) J.out[(int64_t)y * W + x] = (uint16_t)(best & 0xFF);
    }
#pragma unroll
    for (int h = 0; h < NPX; ++h) raw[h] = rawn[h];
  }
  if (!J.lr_check) return;
  __syncthreads();
  uint32_t *part = J.part + ((int64_t)y * J.nseg + sgi) * (J.seglen + D - 1);
  for (int i = threadIdx.x; i < zn; i += blockDim.x) part[i] = keyR[kswz<K>(i)];
}

// Left-right check (section 3.1.4): D_R(x_r) is the smallest key over the
// segments whose zones hold x_r.
// The LR-checked value at (x, y): D_L if the right view's disparity at
// x - D_L, the smallest key over the segments whose zones hold it, is within
// max_diff, else the invalid value.
__device__ __forceinline__ int lr_value(const uint16_t *dl_map, const uint32_t *part, int W, int D, int nseg,
                                        int seglen, int max_diff, int invalid, int x, int y) {
  const int dl = dl_map[(int64_t)y * W + x];
  const int xr = x - dl;
  if (xr < 0) return invalid;
  const int zs = seglen + D - 1;
  const int sa = xr / seglen, sb = min((xr + D - 1) / seglen, nseg - 1);
  const uint32_t *row = part + (int64_t)y * nseg * zs + xr + D - 1;  // segment sg's key at row[sg * (zs - seglen)]
  uint32_t key = 0xFFFFFFFFu;
  // the segments' loads issued together (indices clamped to the last
  // segment: a repeated load leaves the minimum unchanged): two where no
  // position lies in more than two zones, else eight and, if segments are
  // short, the rest one by one
  if ((D - 1) / seglen + 2 <= 2) {
    key = min(row[(int64_t)sa * (zs - seglen)], row[(int64_t)min(sa + 1, sb) * (zs - seglen)]);
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) key = min(key, row[(int64_t)min(sa + i, sb) * (zs - seglen)]);
    for (int sg = sa + 8; sg <= sb; ++sg) key = min(key, row[(int64_t)sg * (zs - seglen)]);
  }
  const int dr = (int)(key & 0xFF);
  return abs(dl - dr) <= max_diff ? dl : invalid;
}

__global__ __launch_bounds__(256) void lr_seg_kernel(JobTable<LRSegJob> t) {
  const int ji = find_job(t.j, t.n, (int)blockIdx.x);
  const LRSegJob &J = t.j[ji];
  const int64_t i = (int64_t)((int)blockIdx.x - J.blk0) * 256 + threadIdx.x;
  if (i >= (int64_t)J.W * J.H) return;
  const int y = (int)(i / J.W), x = (int)(i - (int64_t)y * J.W);
  J.out[i] = (uint16_t)lr_value(J.dl, J.part, J.W, J.D, J.nseg, J.seglen, J.max_diff, J.invalid, x, y);
}

void launch_lr_seg(std::vector<LRSegJob> jobs, hipStream_t s) {
  for_each_table(
      jobs, [](const LRSegJob &j) { return (long)(((int64_t)j.W * j.H + 255) / 256); },
      [&](const JobTable<LRSegJob> &t, int blocks) {
        hipLaunchKernelGGL(lr_seg_kernel, dim3(blocks), dim3(256), 0, s, t);
      });
}

template <int K, int IN>
static void launch_disp_ki(const JobTable<DispJob> &t, int blocks, int want, size_t lds, hipStream_t s) {
  // 1024 threads leave 128 registers per lane: too few for two sweeps of
  // raw words beyond 64 of them
  constexpr bool fits1024 = K < 16 && 2 * DispShape<K, IN>::NPX * DispShape<K, IN>::RAW <= 64;
  const int threads = want ? want : disp_threads(blocks);
  if (threads == 256) {
    hipLaunchKernelGGL((disp_kernel<K, IN, 256>), dim3(blocks), dim3(256), lds, s, t);
  } else if (threads == 512 || !fits1024) {
    hipLaunchKernelGGL((disp_kernel<K, IN, 512>), dim3(blocks), dim3(512), lds, s, t);
  } else if constexpr (fits1024) {
    hipLaunchKernelGGL((disp_kernel<K, IN, 1024>), dim3(blocks), dim3(1024), lds, s, t);
  }
}

template <int K>
static void launch_disp_k(int in_kind, const JobTable<DispJob> &t, int blocks, int want, size_t lds,
                          hipStream_t s) {
  switch (in_kind) {
    case 0: launch_disp_ki<K, 0>(t, blocks, want, lds, s); break;
    case 1: launch_disp_ki<K, 1>(t, blocks, want, lds, s); break;
    default: launch_disp_ki<K, 2>(t, blocks, want, lds, s); break;
  }
}

void launch_disparity(std::vector<DispJob> jobs, int in_kind, hipStream_t s) {
  // one launch per disparities-per-lane width K and requested block size
  for (int K : {4, 8, 12, 16})
    for (int want : {0, 256, 512, 1024}) {
      std::vector<DispJob> sub;
      int maxz = 0;
      for (auto &j : jobs)
        if (agg_k(j.D) == K && j.threads == want) {  // nseg / seglen chosen by the caller
          sub.push_back(j);
          maxz = std::max(maxz, std::min(j.W, j.seglen) + j.D - 1);
        }
      if (sub.empty()) continue;
      const int slots = K == 4 ? kswz_slots<4>(maxz) : K == 8 ? kswz_slots<8>(maxz)
                        : K == 12 ? kswz_slots<12>(maxz) : kswz_slots<16>(maxz);
      const size_t lds = (size_t)slots * 4;
      for_each_table(
          sub, [](const DispJob &j) { return (long)j.H * j.nseg; },
          [&](const JobTable<DispJob> &t, int blocks) {
            switch (K) {
              case 4: launch_disp_k<4>(in_kind, t, blocks, want, lds, s); break;
              case 8: launch_disp_k<8>(in_kind, t, blocks, want, lds, s); break;
              case 12: launch_disp_k<12>(in_kind, t, blocks, want, lds, s); break;
              default: launch_disp_k<16>(in_kind, t, blocks, want, lds, s); break;
            }
          });
    }
}

// ------------------------------------------------------------- median

constexpr int kMedTile = 16;

// Median of N values by a pruned sorting network: Batcher's odd-even merge
// sort on the next power of two P >= N, the inputs padded with +infinity on
// wires N .. P-1.  A compare-exchange that touches a padding wire leaves the
// real wires unchanged (the padding is never smaller), so only those between
// two real wires are kept (5x5: 140 instead of the 300 of an odd-even
// transposition sort); wire N/2 then holds the median, and the compiler drops
// every min or max whose result does not reach it.
struct CeNet {
  int n;
  unsigned char a[256], b[256];
};

constexpr CeNet batcher_net(int n) {
  CeNet r{};
  int P = 1;
  while (P < n) P <<= 1;
  for (int p = 1; p < P; p <<= 1)
    for (int k = p; k >= 1; k >>= 1)
      for (int j = k % p; j + k < P; j += 2 * k)
        for (int i = 0; i < k && i + j + k < P; ++i)
          if ((i + j) / (2 * p) == (i + j + k) / (2 * p) && i + j + k < n) {
            r.a[r.n] = (unsigned char)(i + j);
            r.b[r.n] = (unsigned char)(i + j + k);
            ++r.n;
          }
  return r;
}

__device__ __forceinline__ void compare_exchange(uint32_t &x, uint32_t &y) {
  const uint32_t lo = min(x, y), hi = max(x, y);
  x = lo;
  y = hi;
}

template <int N, int... I>
__device__ __forceinline__ void apply_net(uint32_t (&v)[N], std::integer_sequence<int, I...>) {
  constexpr CeNet net = batcher_net(N);
  (compare_exchange(v[net.a[I]], v[net.b[I]]), ...);
}

template <int N>
__device__ __forceinline__ uint32_t median_of(uint32_t (&v)[N]) {
  apply_net(v, std::make_integer_sequence<int, batcher_net(N).n>{});
  return v[N / 2];
}

// LR = false: the median of the map J.in.  LR = true: the LR check and the
// median in one pass; the block first forms the LR-checked values of its
// tile and clamped halo in LDS from D_L and the segments' right-view keys
// (as lr_seg_kernel does per pixel), so the checked map never goes through
// memory.
template <int KS, bool LR>
__global__ __launch_bounds__(256) void median_kernel(JobTable<MedianJob> t) {
  constexpr int R = KS / 2, TW = kMedTile + 2 * R;
  __shared__ uint16_t tile[LR ? TW * TW : 1];
  const int ji = find_job(t.j, t.n, (int)blockIdx.x);
  const MedianJob &J = t.j[ji];
  const int tb = (int)blockIdx.x - J.blk0;
  const int x0 = (tb % J.tiles_x) * kMedTile, y0 = (tb / J.tiles_x) * kMedTile;
  const int x = x0 + (int)(threadIdx.x & (kMedTile - 1));
  const int y = y0 + (int)(threadIdx.x >> 4);
  uint32_t v[KS * KS];
  if (LR) {
    for (int i = (int)threadIdx.x; i < TW * TW; i += 256) {
      const int xx = min(max(x0 - R + i % TW, 0), J.W - 1);
      const int yy = min(max(y0 - R + i / TW, 0), J.H - 1);
      tile[i] = (uint16_t)lr_value(J.dl, J.part, J.W, J.D, J.nseg, J.seglen, J.max_diff, J.invalid, xx, yy);
    }
    __syncthreads();
    if (x >= J.W || y >= J.H) return;
    const int tx = x - x0, ty = y - y0;
#pragma unroll
    for (int dy = 0; dy < KS; ++dy)
#pragma unroll
      for (int dx = 0; dx < KS; ++dx) v[dy * KS + dx] = tile[(ty + dy) * TW + tx + dx];
  } else {
    if (x >= J.W || y >= J.H) return;
#pragma unroll
    for (int dy = -R; dy <= R; ++dy) {
      const int yy = min(max(y + dy, 0), J.H - 1);
#pragma unroll
      for (int dx = -R; dx <= R; ++dx) {
        const int xx = min(max(x + dx, 0), J.W - 1);
        v[(dy + R) * KS + dx + R] = J.in[(int64_t)yy * J.W + xx];
      }
    }
  }
  J.out[(int64_t)y * J.W + x] = (uint16_t)median_of<KS * KS>(v);
}

void launch_median(std::vector<MedianJob> jobs, hipStream_t s) {
  for (int K : {3, 5})
    for (int lr : {0, 1}) {
      std::vector<MedianJob> sub;
      for (auto &j : jobs)
        if (j.k == K && (j.lr != 0) == (lr != 0)) {
          j.tiles_x = (j.W + kMedTile - 1) / kMedTile;
          sub.push_back(j);
        }
      if (sub.empty()) continue;
      for_each_table(
          sub, [](const MedianJob &j) { return (long)j.tiles_x * ((j.H + kMedTile - 1) / kMedTile); },
          [&](const JobTable<MedianJob> &t, int blocks) {
            if (K == 3 && lr) hipLaunchKernelGGL((median_kernel<3, true>), dim3(blocks), dim3(256), 0, s, t);
            else if (K == 3) hipLaunchKernelGGL((median_kernel<3, false>), dim3(blocks), dim3(256), 0, s, t);
            else if (lr) hipLaunchKernelGGL((median_kernel<5, true>), dim3(blocks), dim3(256), 0, s, t);
            else hipLaunchKernelGGL((median_kernel<5, false>), dim3(blocks), dim3(256), 0, s, t);
          });
    }
}

}  // namespace sgmk
