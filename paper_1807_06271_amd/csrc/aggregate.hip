// Semi-global path aggregation (section 3.1.3; equation (2) read as
// Hirschmueller's per-path recurrence with the predecessor's minimum
// subtracted after every pixel):
//
//   L_r(p,d) = C(p,d) + min(L_r(p-r,d), L_r(p-r,d-1)+P1, L_r(p-r,d+1)+P1, m+P2) - m,
//   m = min_k L_r(p-r,k),   L_r(p,d) = C(p,d) at the first pixel of a path.
//
// Work decomposition (CDNA wave64): a scanline of one direction belongs to
// one 16-lane DPP row, so a wavefront runs four scanlines side by side.  Lane
// j of a row owns the K contiguous disparities d = j*K .. j*K+K-1 (16*K >= D).
// The d-1 / d+1 neighbours held by the adjacent lane arrive by DPP row_shr /
// row_shl (the row ends feed "infinity"), and the per-pixel minimum over d is
// a 4-step DPP row_ror butterfly that leaves the minimum in every lane of the
// row: no LDS, no readlane, no barrier.  Costs stream through a register ring
// PF pixels ahead of the recurrence so that HBM latency overlaps the
// dependent chain.  All directions of all frames of a launch are waves of one
// grid, so the short diagonal scanlines run next to the long rows.
//
// Internal volumes (costs and path costs) are stored [H][W][Dp] with the
// disparity stride padded to Dp = 16*K; cells with d >= D are never read.
#include <type_traits>

#include "device_util.h"

namespace sgmk {

__device__ __constant__ int kDirDx[8] = {+1, -1, 0, 0, +1, -1, -1, +1};
__device__ __constant__ int kDirDy[8] = {0, 0, +1, -1, +1, -1, +1, -1};

__host__ __device__ int agg_lines(int dir, int W, int H) {
  if (dir < 2) return H;
  if (dir < 4) return W;
  return W + H - 1;
}

int agg_k(int D) { return D <= 64 ? 4 : D <= 128 ? 8 : D <= 192 ? 12 : 16; }

// First pixel and length of scanline `line` of direction `dir`.
__device__ __forceinline__ void line_start(int dir, int line, int W, int H, int &sx, int &sy,
                                           int &len) {
  switch (dir) {
    case 0: sx = 0; sy = line; len = W; break;
    case 1: sx = W - 1; sy = line; len = W; break;
    case 2: sx = line; sy = 0; len = H; break;
    case 3: sx = line; sy = H - 1; len = H; break;
    case 4:  // (+1,+1): top row, then the left column below it
      if (line < W) { sx = line; sy = 0; } else { sx = 0; sy = line - W + 1; }
      len = min(W - sx, H - sy);
      break;
    case 5:  // (-1,-1): bottom row, then the right column above it
      if (line < W) { sx = line; sy = H - 1; } else { sx = W - 1; sy = line - W; }
      len = min(sx + 1, sy + 1);
      break;
    case 6:  // (-1,+1): top row, then the right column below it
      if (line < W) { sx = line; sy = 0; } else { sx = W - 1; sy = line - W + 1; }
      len = min(sx + 1, H - sy);
      break;
    default:  // 7, (+1,-1): bottom row, then the left column above it
      if (line < W) { sx = line; sy = H - 1; } else { sx = 0; sy = line - W; }
      len = min(W - sx, sy + 1);
      break;
  }
}

// Path costs are carried as packed pairs of 16-bit values (disparities 2i and
// 2i+1 of the lane in one 32-bit register) so that every min / add of the
// recurrence is one v_pk_* instruction for two disparities.  Values never
// exceed N_b + P2 <= 65535 (parameter check); 0xFFFF stands for "no such
// disparity" and the additions that can meet it saturate.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as_pair(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ u16x2 pmin(u16x2 a, u16x2 b) { return __builtin_elementwise_min(a, b); }
__device__ __forceinline__ u16x2 padd_sat(u16x2 a, u16x2 b) { return __builtin_elementwise_add_sat(a, b); }

constexpr uint32_t kInfPair = 0xFFFFFFFFu;

// Cost words of one pixel for one lane: K values of a padded volume (the
// uint8 volume for SRC kCost8, four per word; the uint16 one for kCost16, two
// per word).  Every lane reads its K cells with one vector load; cells with
// d >= D hold unspecified values that the recurrence masks out.
//
// kSlide (horizontal scanlines of 64 lanes only): the costs are the Hamming
// distances of the Census codes (equation (1)), formed in the wave.  The
// wave holds the right-view codes x - d of all its disparities in registers
// (lane j: codes x - jK - k, k < K) and slides that window by one code per
// pixel, so a pixel needs only two codes from memory, the same for every
// lane: the left-view code of x and the right-view code entering the window.
// Its ring words are those two codes.
enum { kCost8 = 0, kCost16 = 1, kSlide = 2 };

template <int K, int SRC>
struct CostWords {
  static constexpr int N = SRC == kCost8 ? (K + 3) / 4 : SRC == kCost16 ? K / 2 : 4;
  uint32_t w[N];
};

// kSlide: p is the pixel's code record {left code, right code}; the code
// entering the window lies rdelta bytes from p.
template <int K, int SRC>
__device__ __forceinline__ void load_cost(CostWords<K, SRC> &cw, const char *p, int32_t rdelta = 0) {
  if constexpr (SRC == kSlide) {
    const U32N<2> l = *reinterpret_cast<const U32N<2> *>(p);
    const U32N<2> r = *reinterpret_cast<const U32N<2> *>(p + rdelta);
    cw.w[0] = l.v[0];
    cw.w[1] = l.v[1];
    cw.w[2] = r.v[0];
    cw.w[3] = r.v[1];
    return;
  }
  (void)rdelta;
  if (SRC == kCost8 && K % 4 != 0) {  // K = 2 or 6: 2-byte aligned, one 16-bit load per pair
    const uint16_t *q = reinterpret_cast<const uint16_t *>(p);
#pragma unroll
    for (int i = 0; i < (K + 3) / 4; ++i) {
      const uint32_t lo = q[2 * i];
      const uint32_t hi = 2 * i + 1 < K / 2 ? (uint32_t)q[2 * i + 1] : 0u;
      cw.w[i] = lo | hi << 16;
    }
  } else {  // dword-aligned: Dp and K are even, the volumes 256-byte aligned
    constexpr int N = CostWords<K, SRC>::N;
    const U32N<N> v = *reinterpret_cast<const U32N<N> *>(p);
#pragma unroll
    for (int i = 0; i < N; ++i) cw.w[i] = v.v[i];
  }
}

// Costs of disparities (2i, 2i+1) as a packed pair.
template <int K, int SRC>
__device__ __forceinline__ u16x2 cost_pair(const CostWords<K, SRC> &cw, int i) {
  if (SRC == kCost8) {
    // bytes 2i and 2i+1 of the lane's K bytes, zero-extended into 16-bit halves
    const uint32_t sel = (i & 1) ? 0x0c030c02u : 0x0c010c00u;
    return as_pair(__builtin_amdgcn_perm(0u, cw.w[i >> 1], sel));
  }
  return as_pair(cw.w[i]);
}

// Minimum over each group of LPS lanes (16, 32 or 64), delivered to every lane
// of the group: a DPP row butterfly, then permlane swaps across row pairs and
// wave halves.
template <int LPS>
__device__ __forceinline__ uint32_t group_allmin_u32(uint32_t v) {
  v = row16_allmin_u32(v);
  if (LPS >= 32) {
    // rows (0,1) and (2,3) exchange: each lane then sees both rows' minima
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    v = min((uint32_t)r[0], (uint32_t)r[1]);
  }
  if (LPS == 64) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    v = min((uint32_t)r[0], (uint32_t)r[1]);
  }
  return v;
}

// f(std::integral_constant<int, S>{}) for S = B .. E - 1: a loop whose index
// is a compile-time constant in every iteration.
template <int B, int E>
struct Unrolled {
  template <class F>
  __device__ __forceinline__ static void run(F &&f) {
    if constexpr (B < E) {
      f(std::integral_constant<int, B>{});
      Unrolled<B + 1, E>::run(f);
    }
  }
};

// One wave's share of one direction: 64/LPS scanlines side by side, LPS lanes
// per scanline, K disparities per lane (K * LPS = Dp).
// HS = +1 / -1: the wave runs a horizontal direction (L->R / R->L), whose
// pixel step is known at compile time, so that every address of an unrolled
// block is one base plus immediate offsets; HS = 0: any direction.
template <int K, int LPS, int SRC, typename LT, int PF, bool PAD, int HS>
__device__ __forceinline__ void agg_wave(const AggJob &J, int slot, int wave_in_slot) {
  constexpr int NP = K / 2;       // packed pairs per lane
  constexpr int SPW = 64 / LPS;   // scanlines per wave
  const int lane = (int)(threadIdx.x & 63);
  const int row = lane / LPS, j = lane % LPS;
  const int dir = J.dirs[slot];
  const int W = J.W, H = J.H, D = J.D, Dp = J.Dp;
  const int line = wave_in_slot * SPW + row;
  int sx = 0, sy = 0, len = 0;
  if (line < agg_lines(dir, W, H)) line_start(dir, line, W, H, sx, sy, len);
  // the wave runs until its longest scanline is done
  int maxlen = __builtin_amdgcn_readlane(len, 0), minlen = maxlen;
#pragma unroll
  for (int r = 1; r < SPW; ++r) {
    maxlen = max(maxlen, __builtin_amdgcn_readlane(len, r * LPS));
    minlen = min(minlen, __builtin_amdgcn_readlane(len, r * LPS));
  }
  const int64_t step = HS ? HS : (int64_t)kDirDy[dir] * W + kDirDx[dir];  // pixel index step (uniform)
  const int64_t pix0 = (int64_t)sy * W + sx;
  const int dbase = j * K;
  // disparities of this lane below D (all K unless the row is padded, PAD)
  const int dvalid = PAD ? min(K, max(0, D - dbase)) : K;
  // halves for d >= D are forced to 0xFFFF after every pixel
  uint32_t padmask[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i)
    padmask[i] = (2 * i < dvalid ? 0u : 0xFFFFu) | (2 * i + 1 < dvalid ? 0u : 0xFFFF0000u);
  const u16x2 P1 = {(unsigned short)J.p1, (unsigned short)J.p1};
  const u16x2 P2 = {(unsigned short)J.p2, (unsigned short)J.p2};
  // lanes at the ends of a scanline's lane group take "no such disparity"
  // from outside the group
  const bool first_lane = j == 0, last_lane = j == LPS - 1;

  // Addresses are a wave-uniform base that advances by a uniform step per
  // pixel plus a per-lane 32-bit offset that stays fixed along the scanline.
  constexpr int CB = SRC == kCost8 ? 1 : 2;  // bytes per cost element
  const int cpp = Dp;                        // cost elements per pixel (padded)
  const char *cbase = SRC == kCost8 ? reinterpret_cast<const char *>(J.cost8)
                                    : reinterpret_cast<const char *>(J.cost16);
  uint32_t coff = (uint32_t)((pix0 * cpp + dbase) * CB);
  int64_t cstep = HS ? (int64_t)HS * K * LPS * CB : step * cpp * CB;  // Dp = K * LPS
  // kSlide: the code records (16 bytes per pixel); the code entering the
  // window is x's own right-view code (L->R) or that of x - Dp + 1 (R->L,
  // which may lie left of the row: the records before row 0 are padding,
  // and such codes only meet disparities whose cost is N_b anyway)
  int32_t rdelta = 0;
  uint32_t sc[2 * K] = {};  // the lane's window: codes x - dbase - k, k < K (lo, hi)
  const uint32_t nbits = (uint32_t)J.nbits;
  if constexpr (SRC == kSlide) {
    static_assert(HS != 0 && LPS == 64, "sliding Census windows are for 64-lane horizontal scanlines");
    cbase = reinterpret_cast<const char *>(J.codes);
    coff = (uint32_t)(pix0 * 16);
    cstep = (int64_t)HS * 16;
    rdelta = HS > 0 ? 8 : -(Dp - 1) * 16 + 8;
    if (HS < 0 && len > 0) {
      // the window before the row's last pixel: codes W - dbase - k (the
      // first slide moves them to W - 1 - dbase - k)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int xr = min(max(W - dbase - k, 0), W - 1);
        const U32N<2> c = *reinterpret_cast<const U32N<2> *>(cbase + ((int64_t)sy * W + xr) * 16 + 8);
        sc[2 * k] = c.v[0];
        sc[2 * k + 1] = c.v[1];
      }
    }
  }
  (void)nbits;
  char *obase = reinterpret_cast<char *>(J.lr) + (int64_t)slot * H * W * Dp * (int64_t)sizeof(LT);
  const uint32_t ooff = (uint32_t)((pix0 * Dp + dbase) * (int64_t)sizeof(LT));
  const int64_t ostep = HS ? (int64_t)HS * K * LPS * (int64_t)sizeof(LT) : step * Dp * (int64_t)sizeof(LT);

  // Loads are unconditional (a lane past its scanline's end re-reads the
  // last pixel, a lane without a scanline pixel 0): a conditional load here
  // would make the compiler wait for every outstanding access in the loops.
  const int last = max(len - 1, 0);
  CostWords<K, SRC> ring[PF];
#pragma unroll
  for (int s = 0; s < PF; ++s) {  // in ring order, which the waits in the loop assume
    load_cost<K, SRC>(ring[s], cbase + min(s, last) * cstep + coff, rdelta);
    __builtin_amdgcn_sched_barrier(0);
  }

  // A path's first pixel behaves as if its predecessor had all-zero path
  // costs: then every candidate is >= 0 = m, so L = C.
  u16x2 Lp[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) Lp[i] = as_pair(padmask[i]);

  // GUARD = false: every scanline of the wave has pixels i and i + PF, so
  // the load needs no clamp and the store no per-lane test
  // rot: the window ring's rotation before this pixel (kSlide); edgy: the
  // pixel may reach right-view columns left of the image (kSlide)
  auto pixel = [&](auto guard, auto rot, auto edgy, int i, CostWords<K, SRC> &rs) {
    constexpr bool GUARD = decltype(guard)::value;
    constexpr int R = decltype(rot)::value;
    constexpr bool EDGE = decltype(edgy)::value;
    // keep each pixel's instructions together: hoisting the unpacking of
    // later pixels' costs would wait on loads issued one pixel ago
    __builtin_amdgcn_sched_barrier(0);
    u16x2 Cs[NP];  // kSlide: the pixel's cost pairs
    if constexpr (SRC == kSlide) {
      // slide the window one code along the row: every code moves one
      // disparity up (L->R) or down (R->L), across lanes by DPP, and the
      // code entering at the window's end comes in as the DPP's old value.
      // The window is a ring of K code pairs: the code of position k (right
      // view x - dbase - k) sits in slot (k - R) mod K (L->R) or (k + R) mod
      // K (R->L), R the pixels slid since the block of PF pixels began (a
      // multiple of K: each block begins at R = 0), so a slide overwrites
      // the leaving code's slot instead of moving the others.
      constexpr int OUT = HS > 0 ? (K - 1 - R % K) % K : R % K;  // the leaving code's slot
      sc[2 * OUT] = (uint32_t)__builtin_amdgcn_update_dpp((int)rs.w[2], (int)sc[2 * OUT],
                                                          HS > 0 ? kDppWaveShr1 : kDppWaveShl1, 0xF, 0xF, false);
      sc[2 * OUT + 1] = (uint32_t)__builtin_amdgcn_update_dpp((int)rs.w[3], (int)sc[2 * OUT + 1],
                                                              HS > 0 ? kDppWaveShr1 : kDppWaveShl1, 0xF, 0xF, false);
      // Hamming costs; right-view pixels left of the image cost N_b (only
      // while x < Dp - 1, the same x for the whole wave: blocks without such
      // pixels skip the test)
      uint32_t c[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int sl = HS > 0 ? (k + K - (R + 1) % K) % K : (k + R + 1) % K;  // after the slide
        c[k] = (uint32_t)__builtin_popcount(sc[2 * sl] ^ rs.w[0]) +
               (uint32_t)__builtin_popcount(sc[2 * sl + 1] ^ rs.w[1]);
        if constexpr (EDGE) {
          const int x = sx + (GUARD ? min(i, last) : i) * HS;
          if (x < Dp - 1) c[k] = x - dbase - k >= 0 ? c[k] : nbits;
        }
      }
#pragma unroll
      for (int q = 0; q < NP; ++q) Cs[q] = as_pair(c[2 * q] | c[2 * q + 1] << 16);
    }
    auto cost_of = [&](int q) -> u16x2 {
      if constexpr (SRC == kSlide) return Cs[q];
      else return cost_pair<K, SRC>(rs, q);
    };
    u16x2 Lc[NP];
    if constexpr (NP == 1 && LPS >= 32) {
      // One pair per lane (the wide horizontal layouts, whose scanlines are
      // the longest dependent chains).  The reduction of the predecessor's
      // minimum and the neighbour candidates are independent chains of
      // dependent instructions; they are issued alternately (the barriers fix
      // the order), so each DPP step's wait states hold the other chain's
      // instructions rather than idle cycles.
      const uint32_t l0 = as_u32(Lp[0]);
      uint32_t m = min(l0 & 0xFFFFu, l0 >> 16);
      uint32_t prev = (uint32_t)__builtin_amdgcn_update_dpp((int)kInfPair, (int)l0, kDppWaveShr1, 0xF, 0xF, false);
      uint32_t next = (uint32_t)__builtin_amdgcn_update_dpp((int)kInfPair, (int)l0, kDppWaveShl1, 0xF, 0xF, false);
      __builtin_amdgcn_sched_barrier(0);
      m = min(m, (uint32_t)__builtin_amdgcn_mov_dpp((int)m, kDppRowRor8, 0xF, 0xF, true));
      if (LPS < 64) {
        prev = first_lane ? kInfPair : prev;
        next = last_lane ? kInfPair : next;
      }
      const u16x2 nb0 = as_pair(__builtin_amdgcn_alignbit(l0, prev, 16));
      __builtin_amdgcn_sched_barrier(0);
      m = min(m, (uint32_t)__builtin_amdgcn_mov_dpp((int)m, kDppRowRor4, 0xF, 0xF, true));
      const u16x2 nb1 = as_pair(__builtin_amdgcn_alignbit(next, l0, 16));
      const u16x2 c0 = cost_of(0);
      __builtin_amdgcn_sched_barrier(0);
      m = min(m, (uint32_t)__builtin_amdgcn_mov_dpp((int)m, kDppRowRor2, 0xF, 0xF, true));
      u16x2 a = pmin(nb0, nb1);
      __builtin_amdgcn_sched_barrier(0);
      m = min(m, (uint32_t)__builtin_amdgcn_mov_dpp((int)m, kDppRowRor1, 0xF, 0xF, true));
      a = padd_sat(a, P1);
      __builtin_amdgcn_sched_barrier(0);
      {  // rows (0,1) and (2,3) exchange their minima
        const auto r = __builtin_amdgcn_permlane16_swap(m, m, false, false);
        m = min((uint32_t)r[0], (uint32_t)r[1]);
      }
      a = pmin(a, Lp[0]);
      if (LPS == 64) {  // and the two wave halves
        __builtin_amdgcn_sched_barrier(0);
        const auto r = __builtin_amdgcn_permlane32_swap(m, m, false, false);
        m = min((uint32_t)r[0], (uint32_t)r[1]);
      }
      const u16x2 M = {(unsigned short)m, (unsigned short)m};
      u16x2 v = pmin(a, padd_sat(M, P2)) - M + c0;
      if (PAD) v = as_pair(as_u32(v) | padmask[0]);
      Lc[0] = v;
    } else {
      // neighbour pairs: Nb[q] = (L[2q-1], L[2q]) for q = 0..NP, so that pair
      // q has its d-1 values in Nb[q] and its d+1 values in Nb[q+1]
      uint32_t prev, next;
      if (LPS == 16) {
        prev = (uint32_t)__builtin_amdgcn_update_dpp((int)kInfPair, (int)as_u32(Lp[NP - 1]), kDppRowShr1,
                                                     0xF, 0xF, false);
        next = (uint32_t)__builtin_amdgcn_update_dpp((int)kInfPair, (int)as_u32(Lp[0]), kDppRowShl1,
                                                     0xF, 0xF, false);
      } else {
        prev = (uint32_t)__builtin_amdgcn_update_dpp((int)kInfPair, (int)as_u32(Lp[NP - 1]), kDppWaveShr1,
                                                     0xF, 0xF, false);
        next = (uint32_t)__builtin_amdgcn_update_dpp((int)kInfPair, (int)as_u32(Lp[0]), kDppWaveShl1,
                                                     0xF, 0xF, false);
        if (LPS < 64) {
          prev = first_lane ? kInfPair : prev;
          next = last_lane ? kInfPair : next;
        }
      }
      u16x2 Nb[NP + 1];
      Nb[0] = as_pair(__builtin_amdgcn_alignbit(as_u32(Lp[0]), prev, 16));
#pragma unroll
      for (int q = 1; q < NP; ++q) Nb[q] = as_pair(__builtin_amdgcn_alignbit(as_u32(Lp[q]), as_u32(Lp[q - 1]), 16));
      Nb[NP] = as_pair(__builtin_amdgcn_alignbit(next, as_u32(Lp[NP - 1]), 16));
      // the candidates that do not involve the predecessor's minimum
      u16x2 A[NP];
#pragma unroll
      for (int q = 0; q < NP; ++q) A[q] = pmin(padd_sat(pmin(Nb[q], Nb[q + 1]), P1), Lp[q]);
      // the predecessor's minimum over d, reduced here rather than at the end
      // of the previous pixel: in the same scheduling region as the lines
      // above, its dependent DPP steps interleave with them instead of
      // running ahead of them in issue order
      u16x2 lm = Lp[0];
#pragma unroll
      for (int q = 1; q < NP; ++q) lm = pmin(lm, Lp[q]);
      const uint32_t mp = group_allmin_u32<LPS>(min((uint32_t)lm.x, (uint32_t)lm.y));
      const u16x2 M = {(unsigned short)mp, (unsigned short)mp};
      const u16x2 MP2 = padd_sat(M, P2);
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        u16x2 v = pmin(A[q], MP2) - M + cost_of(q);
        if (PAD) v = as_pair(as_u32(v) | padmask[q]);
        Lc[q] = v;
      }
    }
    // the slot's costs are used: refill it PF pixels ahead
    load_cost<K, SRC>(rs, cbase + (int64_t)(GUARD ? min(i + PF, last) : i + PF) * cstep + coff, rdelta);
    if (!GUARD || i < len) {
      char *o = obase + (int64_t)i * ostep + ooff;
      if (sizeof(LT) == 1) {
        if (K % 4 == 0) {
          U32N<K / 4> pk;
#pragma unroll
          for (int q = 0; q < K / 4; ++q)  // low bytes of the four 16-bit values
            pk.v[q] = __builtin_amdgcn_perm(as_u32(Lc[2 * q + 1]), as_u32(Lc[2 * q]), 0x06040200u);
          store_nt<K / 4>(o, pk);  // read once, by the disparity kernel
        } else {  // K = 2 or 6: 2-byte aligned, one non-temporal 16-bit store per pair
#pragma unroll
          for (int q = 0; q < NP; ++q)
            __builtin_nontemporal_store((uint16_t)__builtin_amdgcn_perm(0u, as_u32(Lc[q]), 0x0c0c0200u),
                                        reinterpret_cast<uint16_t *>(o) + q);
        }
      } else {
        U32N<NP> pk;
#pragma unroll
        for (int q = 0; q < NP; ++q) pk.v[q] = as_u32(Lc[q]);
        store_nt<NP>(o, pk);
      }
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) Lp[q] = Lc[q];
  };

  using Guarded = std::integral_constant<bool, true>;
  using Unguarded = std::integral_constant<bool, false>;
  using Edge = std::integral_constant<bool, true>;
  using NoEdge = std::integral_constant<bool, false>;
  static_assert(SRC != kSlide || PF % K == 0, "a block of PF pixels must turn the window ring back to its start");
  // PF pixels from b0 (tail: only those below maxlen), ring slot and window
  // rotation compile-time constants
  auto block = [&](auto guard, auto edgy, int b0, bool tail) {
    Unrolled<0, PF>::run([&](auto si) {
      constexpr int s = decltype(si)::value;
      if (!tail || b0 + s < maxlen) pixel(guard, std::integral_constant<int, s % K>{}, edgy, b0 + s, ring[s]);
    });
  };
  int i0 = 0;
  // whole blocks, all scanlines long enough.  On sliding windows (one
  // scanline per wave) the blocks whose columns all lie at x >= Dp - 1 need
  // no left-edge test: L->R they follow the first ones, R->L they precede
  // the last ones (two loops rather than a branch per block, which would
  // hold both variants' registers)
  if constexpr (SRC == kSlide && HS > 0) {
    for (; i0 + 2 * PF <= minlen && sx + i0 < Dp - 1; i0 += PF) block(Unguarded{}, Edge{}, i0, false);
    for (; i0 + 2 * PF <= minlen; i0 += PF) block(Unguarded{}, NoEdge{}, i0, false);
  } else if constexpr (SRC == kSlide) {
    for (; i0 + 2 * PF <= minlen && sx - (i0 + PF - 1) >= Dp - 1; i0 += PF) block(Unguarded{}, NoEdge{}, i0, false);
    for (; i0 + 2 * PF <= minlen; i0 += PF) block(Unguarded{}, Edge{}, i0, false);
  } else {
    for (; i0 + 2 * PF <= minlen; i0 += PF) block(Unguarded{}, NoEdge{}, i0, false);
  }
  for (; i0 + PF <= maxlen; i0 += PF) block(Guarded{}, Edge{}, i0, false);  // whole blocks of PF pixels
  block(Guarded{}, Edge{}, i0, true);  // remaining < PF pixels
}

// Scanlines per wave of direction `dir` under a schedule whose horizontal
// directions use `hlps` lanes per scanline (all others use 16).
__host__ __device__ inline int lanes_per_scanline(int dir, int hlps) { return dir < 2 ? hlps : 16; }

// Each wave finds its job and direction slot, then runs that direction's
// scanlines with the lane layout of the schedule: KH disparities per lane
// over HLPS lanes for horizontal paths, K over 16 lanes for the others.
// HSRC: the cost source of the horizontal waves (SRC, or kSlide with
// 64-lane horizontal scanlines).
template <int K, int KH, int HLPS, int SRC, typename LT, int PF, bool PAD, int HSRC = SRC>
__global__ __launch_bounds__(256) void agg_kernel(JobTable<AggJob> t) {
  const int gw = uniform((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));  // global wave
  const int ji = find_job(t.j, t.n, gw);
  const AggJob &J = t.j[ji];
  const int w = gw - J.blk0;
  if (w >= J.line0[J.ndirs]) return;  // whole wave: tail of the grid
  int slot = 0;
  for (int k = 1; k < J.ndirs; ++k)
    if (w >= J.line0[k]) slot = k;
  const int wave_in_slot = w - J.line0[slot];
  // Wider lane groups finish a pixel in fewer instructions, so they prefetch
  // proportionally further ahead to cover the same memory latency; a sliding
  // window's ring slot is four words, so it keeps eight pixels in flight.
  constexpr int PFH = HSRC == kSlide ? 8 : PF * HLPS / 16;
  const int dir = J.dirs[slot];
  if (dir == 0)
    agg_wave<KH, HLPS, HSRC, LT, PFH, PAD, +1>(J, slot, wave_in_slot);
  else if (dir == 1)
    agg_wave<KH, HLPS, HSRC, LT, PFH, PAD, -1>(J, slot, wave_in_slot);
  else
    agg_wave<K, 16, SRC, LT, PF, PAD, 0>(J, slot, wave_in_slot);
}

template <int K, int KH, int HLPS, int SRC, typename LT, int HSRC = SRC>
static void launch_one(const JobTable<AggJob> &t, int waves, hipStream_t s) {
  constexpr int PF = SRC == kCost8 || K <= 8 ? 8 : 4;
  const int blocks = (waves + 3) / 4;
  bool pad = false;  // some frame's D is not a multiple of 16*K: mask the tail lanes
  for (int i = 0; i < t.n; ++i) pad |= t.j[i].D != 16 * K;
  if (pad)
    hipLaunchKernelGGL((agg_kernel<K, KH, HLPS, SRC, LT, PF, true, HSRC>), dim3(blocks), dim3(256), 0, s, t);
  else
    hipLaunchKernelGGL((agg_kernel<K, KH, HLPS, SRC, LT, PF, false, HSRC>), dim3(blocks), dim3(256), 0, s, t);
}

// Lanes per horizontal scanline available for a disparity width K (16 lanes):
// the horizontal layout needs an even number of disparities per lane.
bool agg_hlps_ok(int K, int hlps) {
  if (hlps == 16) return true;
  const int kh = 16 * K / hlps;
  return (hlps == 32 || hlps == 64) && kh >= 2 && kh % 2 == 0;
}

// Horizontal costs from sliding Census windows: 64-lane rows with two or
// four disparities per lane (D in (64, 128] or (192, 256]), uint8 volumes.
bool agg_slide_ok(int K, int hlps) { return hlps == 64 && (K == 8 || K == 16); }

template <int SRC, typename LT>
static void launch_k(int K, int hlps, bool slide, const JobTable<AggJob> &t, int waves, hipStream_t s) {
  if constexpr (SRC == kCost8 && std::is_same<LT, uint8_t>::value) {
    if (slide && K == 8 && hlps == 64) return launch_one<8, 2, 64, SRC, LT, kSlide>(t, waves, s);
    if (slide && K == 16 && hlps == 64) return launch_one<16, 4, 64, SRC, LT, kSlide>(t, waves, s);
  }
  switch (K * 100 + hlps) {
    case 416: launch_one<4, 4, 16, SRC, LT>(t, waves, s); break;
    case 432: launch_one<4, 2, 32, SRC, LT>(t, waves, s); break;
    case 816: launch_one<8, 8, 16, SRC, LT>(t, waves, s); break;
    case 832: launch_one<8, 4, 32, SRC, LT>(t, waves, s); break;
    case 864: launch_one<8, 2, 64, SRC, LT>(t, waves, s); break;
    case 1216: launch_one<12, 12, 16, SRC, LT>(t, waves, s); break;
    case 1232: launch_one<12, 6, 32, SRC, LT>(t, waves, s); break;
    case 1616: launch_one<16, 16, 16, SRC, LT>(t, waves, s); break;
    case 1632: launch_one<16, 8, 32, SRC, LT>(t, waves, s); break;
    default: launch_one<16, 4, 64, SRC, LT>(t, waves, s); break;
  }
}

void launch_aggregate(std::vector<AggJob> jobs, bool from_cost16, int K, int hlps, int lr_bytes, bool slide,
                      hipStream_t s) {
  if (!agg_hlps_ok(K, hlps)) hlps = 16;
  slide = slide && !from_cost16 && lr_bytes == 1 && agg_slide_ok(K, hlps);
  for (auto &j : jobs) {
    int total = 0;
    for (int k = 0; k < j.ndirs; ++k) {
      j.line0[k] = total;
      const int spw = 64 / lanes_per_scanline(j.dirs[k], hlps);  // scanlines per wave
      total += (agg_lines(j.dirs[k], j.W, j.H) + spw - 1) / spw;
    }
    j.line0[j.ndirs] = total;
  }
  for_each_table(
      jobs, [](const AggJob &j) { return (long)j.line0[j.ndirs]; },
      [&](const JobTable<AggJob> &t, int waves) {
        if (!from_cost16) {
          if (lr_bytes == 1) launch_k<kCost8, uint8_t>(K, hlps, slide, t, waves, s);
          else launch_k<kCost8, uint16_t>(K, hlps, false, t, waves, s);
        } else {
          if (lr_bytes == 1) launch_k<kCost16, uint8_t>(K, hlps, false, t, waves, s);
          else launch_k<kCost16, uint16_t>(K, hlps, false, t, waves, s);
        }
      });
}

// S = sum over the P slots of the (padded) path-cost volumes, written
// unpadded: one thread per (pixel, 4 consecutive disparities); the P slot
// loads are issued together, summed as packed 16-bit fields.
template <typename LT>
__global__ __launch_bounds__(256) void sum_kernel(JobTable<SumJob> t) {
  const int ji = find_job(t.j, t.n, (int)blockIdx.x);
  const SumJob &J = t.j[ji];
  const int qpp = J.Dp / 4;  // 4-disparity groups per pixel (padded)
  const int64_t g = (int64_t)((int)blockIdx.x - J.blk0) * 256 + threadIdx.x;
  const int64_t npix = J.cells / J.D;
  if (g >= npix * qpp) return;
  const int64_t pix = g / qpp;
  const int d0 = (int)(g - pix * qpp) * 4;
  if (d0 >= J.D) return;
  const int64_t slot = npix * J.Dp;
  const LT *src = reinterpret_cast<const LT *>(J.lr) + pix * J.Dp + d0;
  uint32_t lo = 0, hi = 0;  // (d0, d0+2) and (d0+1, d0+3) as 16-bit pairs
  if (sizeof(LT) == 1) {
    uint32_t v[8];
#pragma unroll
    for (int p = 0; p < 8; ++p)
      if (p < J.P) v[p] = *reinterpret_cast<const uint32_t *>(src + p * slot);
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      if (p >= J.P) break;
      lo += v[p] & 0x00FF00FFu;
      hi += (v[p] >> 8) & 0x00FF00FFu;
    }
  } else {
    uint2 v[8];
#pragma unroll
    for (int p = 0; p < 8; ++p)
      if (p < J.P) v[p] = *reinterpret_cast<const uint2 *>(src + p * slot);
    uint32_t a = 0, b = 0;  // (d0, d0+1), (d0+2, d0+3)
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      if (p >= J.P) break;
      a += v[p].x;
      b += v[p].y;
    }
    lo = (a & 0xFFFF) | (b << 16);
    hi = (a >> 16) | (b & 0xFFFF0000u);
  }
  const uint32_t s4[4] = {lo & 0xFFFF, hi & 0xFFFF, lo >> 16, hi >> 16};
  uint16_t *dst = J.S + pix * J.D + d0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (d0 + k < J.D) dst[k] = (uint16_t)s4[k];
}

void launch_sum(std::vector<SumJob> jobs, int lr_bytes, hipStream_t s) {
  for_each_table(
      jobs, [](const SumJob &j) { return (long)((j.cells / j.D * (j.Dp / 4) + 255) / 256); },
      [&](const JobTable<SumJob> &t, int blocks) {
        if (lr_bytes == 1) hipLaunchKernelGGL(sum_kernel<uint8_t>, dim3(blocks), dim3(256), 0, s, t);
        else hipLaunchKernelGGL(sum_kernel<uint16_t>, dim3(blocks), dim3(256), 0, s, t);
      });
}

__global__ __launch_bounds__(256) void pad16_kernel(const uint16_t *src, uint16_t *dst, int64_t px, int D,
                                                    int Dp) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= px * Dp) return;
  const int64_t pix = i / Dp;
  const int d = (int)(i - pix * Dp);
  dst[i] = d < D ? src[pix * D + d] : (uint16_t)0;
}

void launch_pad16(const uint16_t *src, uint16_t *dst, int64_t px, int D, int Dp, hipStream_t s) {
  const int64_t n = px * Dp;
  hipLaunchKernelGGL(pad16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, px, D, Dp);
}

}  // namespace sgmk
