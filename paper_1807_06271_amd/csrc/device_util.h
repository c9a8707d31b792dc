// Device helpers shared by the kernels: job lookup, DPP cross-lane moves and
// reductions for 64-wide CDNA wavefronts, and batching of job tables into
// launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "sgm_kernels.h"

namespace sgmk {

// DPP control words (GCN/CDNA "dpp_ctrl" encodings).
enum : int {
  kDppRowShr1 = 0x111,   // lane i reads lane i-1 of its row (row start has no source)
  kDppRowShr2 = 0x112,
  kDppRowShr4 = 0x114,
  kDppRowShr8 = 0x118,
  kDppRowShl1 = 0x101,   // lane i reads lane i+1 of its row (row end has no source)
  kDppRowRor1 = 0x121,   // row_ror:n = 0x120 + n
  kDppRowRor2 = 0x122,
  kDppRowRor4 = 0x124,
  kDppRowRor8 = 0x128,
  kDppWaveShl1 = 0x130,  // lane i reads lane i+1 (lane 63 has no source)
  kDppWaveShr1 = 0x138,  // lane i reads lane i-1 (lane 0 has no source)
  kDppRowBcast15 = 0x142,
  kDppRowBcast31 = 0x143,
};

// A raw buffer descriptor over `bytes` bytes from `base`: loads and stores
// through it take one 32-bit offset (no 64-bit address per lane), and the
// hardware drops a store, or returns 0 for a load, whose offset lies beyond
// the size.
constexpr int kBufWord3 = 0x00020000;  // 32-bit data format (gfx9 descriptor word 3)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kBufWord3);
}

// Value of lane i-1 (lane 0 gets `edge`).
__device__ __forceinline__ uint32_t from_lower_lane(uint32_t v, uint32_t edge) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, kDppWaveShr1, 0xF, 0xF, false);
}
// Value of lane i+1 (lane 63 gets `edge`).
__device__ __forceinline__ uint32_t from_upper_lane(uint32_t v, uint32_t edge) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, kDppWaveShl1, 0xF, 0xF, false);
}

// Unsigned minimum over all 64 lanes, returned as a wave-uniform value.
// Rows of 16 lanes are reduced with row_shr (lanes whose source falls outside
// the row keep the identity), then rows are combined with row_bcast:15/31;
// lane 63 ends up with the full minimum.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  const int id = -1;  // 0xFFFFFFFF: identity of unsigned min
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, kDppRowShr1, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, kDppRowShr2, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, kDppRowShr4, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, kDppRowShr8, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, kDppRowBcast15, 0xA, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, kDppRowBcast31, 0xC, 0xF, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Unsigned minimum over each 16-lane DPP row, delivered to every lane of the
// row: a butterfly of row rotations by 8, 4, 2 and 1 lanes.
__device__ __forceinline__ uint32_t row16_allmin_u32(uint32_t v) {
  // every source lane of a rotation is valid, so bound_ctrl is irrelevant;
  // setting it lets the compiler fold each move into the v_min as a DPP operand
  v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppRowRor8, 0xF, 0xF, true));
  v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppRowRor4, 0xF, 0xF, true));
  v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppRowRor2, 0xF, 0xF, true));
  v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppRowRor1, 0xF, 0xF, true));
  return v;
}

// Same result through __shfl_xor within aligned 16-lane groups.
__device__ __forceinline__ uint32_t row16_min_u32(uint32_t v) {
  v = min(v, (uint32_t)__shfl_xor((int)v, 8, 16));
  v = min(v, (uint32_t)__shfl_xor((int)v, 4, 16));
  v = min(v, (uint32_t)__shfl_xor((int)v, 2, 16));
  v = min(v, (uint32_t)__shfl_xor((int)v, 1, 16));
  return v;
}

// N consecutive 32-bit words, loaded / stored as one vector access.
template <int N>
struct alignas(4) U32N {
  uint32_t v[N];
};

// Non-temporal (streaming) vector store / load of N consecutive words, for
// data written once and read once by a later kernel: the path-cost volumes
// then do not linger as dirty lines in the caches, whose write-back would
// compete with the next kernel's reads.  Word alignment is enough.
typedef uint32_t u32x2a __attribute__((ext_vector_type(2), aligned(4)));
typedef uint32_t u32x4a __attribute__((ext_vector_type(4), aligned(4)));

template <int N>
__device__ __forceinline__ void store_nt(void *p, const U32N<N> &v) {
  if constexpr (N == 2) {
    __builtin_nontemporal_store(u32x2a{v.v[0], v.v[1]}, reinterpret_cast<u32x2a *>(p));
  } else if constexpr (N == 4) {
    __builtin_nontemporal_store(u32x4a{v.v[0], v.v[1], v.v[2], v.v[3]}, reinterpret_cast<u32x4a *>(p));
  } else if constexpr (N % 4 == 0) {
#pragma unroll
    for (int i = 0; i < N; i += 4)
      __builtin_nontemporal_store(u32x4a{v.v[i], v.v[i + 1], v.v[i + 2], v.v[i + 3]},
                                  reinterpret_cast<u32x4a *>(p) + i / 4);
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) __builtin_nontemporal_store(v.v[i], reinterpret_cast<uint32_t *>(p) + i);
  }
}

template <int N>
__device__ __forceinline__ U32N<N> load_nt(const void *p) {
  U32N<N> r;
  if constexpr (N == 2) {
    const u32x2a a = __builtin_nontemporal_load(reinterpret_cast<const u32x2a *>(p));
    r.v[0] = a.x;
    r.v[1] = a.y;
  } else if constexpr (N % 4 == 0) {
#pragma unroll
    for (int i = 0; i < N; i += 4) {
      const u32x4a a = __builtin_nontemporal_load(reinterpret_cast<const u32x4a *>(p) + i / 4);
      r.v[i] = a.x;
      r.v[i + 1] = a.y;
      r.v[i + 2] = a.z;
      r.v[i + 3] = a.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) r.v[i] = __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(p) + i);
  }
  return r;
}

// Census code (section 3.1.2) of the pixel at column x of a window whose ch
// rows start at rows, rows + stride, ...: neighbour n of the raster order
// (centre skipped) goes to bit N_b - 1 - n, bit = [I(q) < I(p)].
template <int CW, int CH>
__device__ __forceinline__ uint64_t census_fixed(const uint8_t *rows, int stride, int x) {
  constexpr int RX = CW / 2, RY = CH / 2, NB = CW * CH - 1;
  const uint32_t c = rows[RY * stride + x + RX];
  // neighbour n (raster order, centre skipped) goes to bit NB - 1 - n, so
  // the bits enter MSB first: the first NB - 32 neighbours shift into the high
  // half, the last 32 (or all, for NB <= 32) into the low half.  n - c is
  // negative exactly when I(q) < I(p), and v_alignbit({half, n - c}, 31)
  // shifts the half left by one and appends that sign bit: one subtract and
  // one alignbit per neighbour.
  uint32_t lo = 0, hi = 0;
  int n = 0;
#pragma unroll
  for (int dy = 0; dy < CH; ++dy)
#pragma unroll
    for (int dx = 0; dx < CW; ++dx) {
      if (dy == RY && dx == RX) continue;
      const int bit = NB - 1 - n++;
      const uint32_t diff = (uint32_t)rows[dy * stride + x + dx] - c;
      if (bit >= 32) hi = __builtin_amdgcn_alignbit(hi, diff, 31);
      else lo = __builtin_amdgcn_alignbit(lo, diff, 31);
    }
  return (uint64_t)hi << 32 | lo;
}

__device__ __forceinline__ uint64_t census_any(const uint8_t *rows, int stride, int x, int cw, int ch) {
  const int rx = cw / 2, ry = ch / 2;
  const uint8_t c = rows[ry * stride + x + rx];
  uint64_t code = 0;
  for (int dy = 0; dy < ch; ++dy)
    for (int dx = 0; dx < cw; ++dx) {
      if (dy == ry && dx == rx) continue;
      code = (code << 1) | (uint64_t)(rows[dy * stride + x + dx] < c);
    }
  return code;
}

__device__ __forceinline__ uint64_t census_at(const uint8_t *rows, int stride, int x, int cw, int ch) {
  if (cw == 9 && ch == 7) return census_fixed<9, 7>(rows, stride, x);
  if (cw == 5 && ch == 5) return census_fixed<5, 5>(rows, stride, x);
  return census_any(rows, stride, x, cw, ch);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Index of the job owning global block (or wave) index `b`: the last job with
// start <= b.  Jobs are sorted by start.
template <class Job>
__device__ __forceinline__ int find_job(const Job *jobs, int n, int b) {
  int j = 0;
  for (int k = 1; k < n; ++k)
    if (b >= jobs[k].blk0) j = k;
  return j;
}

template <class Job>
struct JobTable {
  Job j[kMaxJobs];
  int n;
};

// Split `jobs` into tables of at most kMaxJobs entries, assign blk0 as the
// running block count (blocks_of(job) blocks each) and call
// launch(table, total_blocks) for each table.
template <class Job, class BlocksOf, class Launch>
void for_each_table(std::vector<Job> &jobs, BlocksOf blocks_of, Launch launch) {
  for (size_t i = 0; i < jobs.size(); i += kMaxJobs) {
    JobTable<Job> t;
    t.n = (int)std::min<size_t>(kMaxJobs, jobs.size() - i);
    long total = 0;
    for (int k = 0; k < t.n; ++k) {
      t.j[k] = jobs[i + k];
      t.j[k].blk0 = (int)total;
      total += blocks_of(t.j[k]);
    }
    if (total > 0) launch(t, (int)total);
  }
}

}  // namespace sgmk
