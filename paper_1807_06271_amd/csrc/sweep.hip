// Single-pass row sweep for the forward path set of the paper's design
// (section 3.1.3, figure 2: the paths at 0, 45, 90 and 135 degrees all take
// their predecessor from the current row's left or the row above, so one
// top-down sweep computes them together, as the FPGA pipeline does).
//
// One block of 1024 threads per frame.  Row groups of 16 lanes each own one
// image row at a time; lane j holds the disparities 4j .. 4j+3 (D <= 64).
// The 60 groups of waves 0-14 take rows y = 60k + g in bands of 60, and group
// g starts its row two steps after group g-1, so at step t group g works on
// pixel x = t - 2g - k*P of its row: it then finds
//   - its own L2R predecessor (x-1, y) in registers,
//   - the T2B, TL2BR and TR2BL predecessors (x, y-1), (x-1, y-1), (x+1, y-1)
//     in a 4-slot LDS ring that group g-1 wrote one to three steps earlier
//     (for group 0, in a carry row that the last group of the previous band
//     wrote to global memory),
// all separated from the writes by the per-step block barrier.  Costs come
// from the Census codes: the right-view codes for x-d slide through the
// lanes (each step shifts them one disparity up, DPP row_shr), and the
// codes are prefetched kPF steps ahead.  Each step forms S(x, y, .) = sum of
// the path costs, the winner-takes-all D_L(x, y), and advances a systolic
// argmin for the right view: the candidate for x_r moves one disparity per
// step, meets S(x_r + d, y, d) in the lane that holds d, and is final when d
// reaches D-1 (or the row ends).  Ties go to the smaller disparity, since
// candidates are compared as (S << 8 | d).  Nothing but D_L and D_R leaves
// the chip.
//
// The computing waves issue only loads (unconditionally, so the waits for a
// prefetched value never wait for later memory operations); their outputs
// go to LDS, and wave 15 writes them to global memory one step later.
#include <type_traits>

#include "device_util.h"

namespace sgmk {

namespace {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ u16x2 as_pair(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ u16x2 pmin(u16x2 a, u16x2 b) { return __builtin_elementwise_min(a, b); }
__device__ __forceinline__ u16x2 padd_sat(u16x2 a, u16x2 b) { return __builtin_elementwise_add_sat(a, b); }

constexpr int kG = 60;    // computing row groups per block (waves 0-14)
constexpr int kPF = 4;    // prefetch depth in steps
constexpr uint32_t kInf = 0xFFFFFFFFu;

// One step of the path recurrence for a 16-lane group (4 disparities per
// lane as two packed pairs): Lp = predecessor's path costs, mp its minimum.
// Cells with d >= D carry C = 0xFFFF, so the saturating final add keeps them
// at 0xFFFF (every candidate is >= mp, so best - mp does not wrap).
__device__ __forceinline__ void path_step(const u16x2 Lp[2], uint32_t mp, const u16x2 C[2], u16x2 P1, u16x2 P2,
                                          u16x2 Lc[2]) {
  const uint32_t prev =
      (uint32_t)__builtin_amdgcn_update_dpp((int)kInf, (int)as_u32(Lp[1]), kDppRowShr1, 0xF, 0xF, false);
  const uint32_t next =
      (uint32_t)__builtin_amdgcn_update_dpp((int)kInf, (int)as_u32(Lp[0]), kDppRowShl1, 0xF, 0xF, false);
  // Nb[q] = (L[2q-1], L[2q]) of the lane's disparities
  const u16x2 Nb0 = as_pair(__builtin_amdgcn_alignbit(as_u32(Lp[0]), prev, 16));
  const u16x2 Nb1 = as_pair(__builtin_amdgcn_alignbit(as_u32(Lp[1]), as_u32(Lp[0]), 16));
  const u16x2 Nb2 = as_pair(__builtin_amdgcn_alignbit(next, as_u32(Lp[1]), 16));
  const u16x2 M = {(unsigned short)mp, (unsigned short)mp};
  const u16x2 MP2 = padd_sat(M, P2);
  u16x2 b0 = pmin(pmin(padd_sat(pmin(Nb0, Nb1), P1), Lp[0]), MP2);
  u16x2 b1 = pmin(pmin(padd_sat(pmin(Nb1, Nb2), P1), Lp[1]), MP2);
  Lc[0] = padd_sat(b0 - M, C[0]);
  Lc[1] = padd_sat(b1 - M, C[1]);
}

__device__ __forceinline__ uint32_t pair_min(const u16x2 L[2]) {
  const u16x2 m = pmin(L[0], L[1]);
  return row16_allmin_u32(min((uint32_t)m.x, (uint32_t)m.y));
}

// four path-cost bytes of the lane (low bytes of the four 16-bit values)
__device__ __forceinline__ uint32_t pack_bytes(const u16x2 L[2]) {
  return __builtin_amdgcn_perm(as_u32(L[1]), as_u32(L[0]), 0x06040200u);
}
// and back: sel[] are the lane's byte selectors, whose high byte of a cell
// with d >= D is 0xFF (v_perm selector 13) so that the cell reads 0xFFFF
__device__ __forceinline__ void unpack_bytes(uint32_t b, const uint32_t sel[2], u16x2 L[2]) {
  L[0] = as_pair(__builtin_amdgcn_perm(0u, b, sel[0]));
  L[1] = as_pair(__builtin_amdgcn_perm(0u, b, sel[1]));
}

}  // namespace

__global__ __launch_bounds__(1024) void sweep_kernel(JobTable<SweepJob> t) {
  __shared__ uint32_t ring[kG][4][3][16];  // [group][x % 4][path][lane]: path-cost bytes
  __shared__ uint32_t rmin[kG][4][3];      // their minima over d
  // outputs of the last two steps (by step parity) for the writer wave:
  // D_L per group, the right-view candidates per group and disparity, and
  // the carry bytes of the band's last group
  __shared__ uint8_t st_dl[2][kG];
  __shared__ uint32_t st_dr[2][kG][16];
  __shared__ uint32_t st_carry[2][kSweepCarry / 4];
  // the job's fields in registers (the job table lives in the kernel
  // arguments; indexing it by block would reload them inside the loop)
  const SweepJob &JT = t.j[find_job(t.j, t.n, (int)blockIdx.x)];
  // frame (blockIdx.x - blk0) of the job: its buffers lie `stride` bytes apart
  const int64_t off = (int64_t)((int)blockIdx.x - JT.blk0) * JT.stride;
  const uint64_t *const Jcl = reinterpret_cast<const uint64_t *>(reinterpret_cast<const char *>(JT.cl) + off);
  const uint64_t *const Jcr = reinterpret_cast<const uint64_t *>(reinterpret_cast<const char *>(JT.cr) + off);
  uint16_t *const Jdl = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(JT.dl) + off);
  uint16_t *const Jdr = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(JT.dr) + off);
  uint8_t *const Jcarry = JT.carry + off;
  const int W = JT.W, H = JT.H, D = JT.D;
  const uint32_t nbits = (uint32_t)JT.nbits, mask = JT.mask;
  const int jp1 = JT.p1, jp2 = JT.p2;
  const int g = (int)threadIdx.x >> 4, j = (int)threadIdx.x & 15;
  const bool writer = threadIdx.x >= 64 * 15;  // wave 15 (wave-uniform)
  const bool wave0 = threadIdx.x < 64;          // groups 0-3 (wave-uniform)
  const int gsh = 2 * (g & 1);                  // -2g mod 4
  // steps between the rows of a group: the row (W), two steps so that group
  // g+1 has read the ring before group g refills it, and at least enough for
  // the 2-step skew of kG groups plus the writer's step and the carry
  // prefetch distance
  const int P = max(W + 2, 2 * kG + kPF + 2);
  // steps until the last row's last pixel, plus one for the writer
  const int T = 2 * ((H - 1) % kG) + P * ((H - 1) / kG) + W + 1;
  const int dbase = 4 * j;
  const int dvalid = min(4, max(0, D - dbase));
  uint32_t pad[2], usel[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    pad[q] = (2 * q < dvalid ? 0u : 0xFFFFu) | (2 * q + 1 < dvalid ? 0u : 0xFFFF0000u);
    // bytes 2q and 2q+1 into the low bytes of the two halves; high bytes 0x00,
    // or 0xFF for cells with d >= D
    usel[q] = (uint32_t)(2 * q) | (2 * q < dvalid ? 0x0Cu : 0x0Du) << 8 | (uint32_t)(2 * q + 1) << 16 |
              (2 * q + 1 < dvalid ? 0x0Cu : 0x0Du) << 24;
  }
  const u16x2 P1 = {(unsigned short)jp1, (unsigned short)jp1};
  const u16x2 P2 = {(unsigned short)jp2, (unsigned short)jp2};
  const bool pL = mask & 0x01, pT = mask & 0x04, pTL = mask & 0x10, pTR = mask & 0x40;
  const bool vert = pT || pTL || pTR;
  const int dlast = D - 1;  // the candidate holding d = D-1 is final

  // (band, x) of the step being processed and of the prefetch target
  // the writer's lane gg tracks group gg one step late
  int band = 0, x = writer ? -2 * ((int)threadIdx.x & 63) - 1 : -2 * g, bandf = 0, xf = -2 * g;
  auto advance = [&](int &b, int &xx) {
    if (++xx == P) {
      xx = 0;
      ++b;
    }
  };
  // prefetch ring: Census words at (x, y) and, for group 0, the carry row's
  // path bytes and minima of the three predecessors
  uint32_t rcl[kPF], rcr[kPF], rcv0[kPF], rcv1[kPF], rcv2[kPF], rcm0[kPF], rcm1[kPF], rcm2[kPF];
  // Loads are issued unconditionally by every wave (an out-of-image target
  // reads pixel 0), so the ring registers are plain loop-carried values and
  // the waits for them stay kPF steps behind the loads.
  auto prefetch = [&](auto stag, int b, int xx) {
    constexpr int S_ = decltype(stag)::value;
    // a target outside the image reads a clamped pixel, whose value the
    // step then ignores; byte offsets from block-uniform bases fit 32 bits
    // (W*H*8 < 2^28 for an eligible frame; the carry rows are 2*(W+2)*256
    // bytes)
    const int xc = min(max(xx, 0), W - 1);
    const int yc = min(b * kG + g, H - 1);
    const uint32_t o = (uint32_t)(yc * W + xc) * 8u;
    rcl[S_] = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(Jcl) + o);
    rcr[S_] = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(Jcr) + o);
    {  // only group 0 (wave 0) uses the carry row: the other waves skip the
       // address arithmetic (a uniform branch) and load from offset 0, but
       // every wave issues the loads, so that all paths through a step issue
       // the same ones
      uint32_t c0 = 0, cm = 0, cp = 0;
      if (wave0) {  // carry column i holds pixel i - 1 (columns 0 and W + 1 stay zero)
        const uint32_t cb = (uint32_t)((max(b, 1) - 1) & 1) * (uint32_t)(W + 2) * kSweepCarry;
        cm = cb + (uint32_t)xc * kSweepCarry;
        c0 = cm + kSweepCarry;
        cp = c0 + kSweepCarry;
      }
      rcv0[S_] = *reinterpret_cast<const uint32_t *>(Jcarry + (c0 + dbase));
      rcm0[S_] = *reinterpret_cast<const uint32_t *>(Jcarry + (c0 + 192));
      rcv1[S_] = *reinterpret_cast<const uint32_t *>(Jcarry + (cm + 64 + dbase));
      rcm1[S_] = *reinterpret_cast<const uint32_t *>(Jcarry + (cm + 196));
      rcv2[S_] = *reinterpret_cast<const uint32_t *>(Jcarry + (cp + 128 + dbase));
      rcm2[S_] = *reinterpret_cast<const uint32_t *>(Jcarry + (cp + 200));
    }
  };

  if (vert) {
    // The first band's carry row (buffer 0) and the border columns of buffer
    // 1 read as zero path costs (no predecessor); the scratch holds whatever
    // an earlier frame left.  The first prefetch below reads them.
    uint32_t *const c32 = reinterpret_cast<uint32_t *>(Jcarry);
    constexpr int kCol = kSweepCarry / 4;  // dwords per carry column
    const int n0 = (W + 2) * kCol;
    for (int i = (int)threadIdx.x; i < n0; i += (int)blockDim.x) c32[i] = 0u;
    for (int i = (int)threadIdx.x; i < 2 * kCol; i += (int)blockDim.x)
      c32[n0 + (i < kCol ? 0 : (W + 1) * kCol) + i % kCol] = 0u;
  }
  // Group 0 starts its first row at x = 0, so no step of it zeroes the ring
  // slot of position -1 that group 1 reads at its first pixel: start from a
  // zeroed ring.
  for (int i = (int)threadIdx.x; i < kG * 4 * 3 * 16; i += (int)blockDim.x) (&ring[0][0][0][0])[i] = 0u;
  for (int i = (int)threadIdx.x; i < kG * 4 * 3; i += (int)blockDim.x) (&rmin[0][0][0])[i] = 0u;
  // the stores complete before any wave reads the carry; an explicit wait
  // for every counter also tells the compiler that nothing is outstanding,
  // so that its waits in the loop still count only the prefetch loads
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < kPF; ++s) {
    rcl[s] = rcr[s] = rcv0[s] = rcv1[s] = rcv2[s] = rcm0[s] = rcm1[s] = rcm2[s] = 0;
  }
  prefetch(std::integral_constant<int, 0>{}, bandf, xf);
  advance(bandf, xf);
  prefetch(std::integral_constant<int, 1>{}, bandf, xf);
  advance(bandf, xf);
  prefetch(std::integral_constant<int, 2>{}, bandf, xf);
  advance(bandf, xf);
  prefetch(std::integral_constant<int, 3>{}, bandf, xf);
  advance(bandf, xf);
  u16x2 Lh[2] = {as_pair(pad[0]), as_pair(pad[1])};
  uint32_t mh = 0;
  uint32_t crs[4] = {0u, 0u, 0u, 0u};           // cr(x - 4j - k), renamed per step
  uint32_t cand[4] = {kInf, kInf, kInf, kInf};  // right-view candidate of x - 4j - k, likewise

  static_assert(kPF == 4, "the prefetch slots below are spelled out for kPF = 4");
  auto step = [&](auto stag) {
      constexpr int S_ = decltype(stag)::value;
      const uint32_t ccl = rcl[S_], ccr = rcr[S_];
      const uint32_t cv0 = rcv0[S_], cv1 = rcv1[S_], cv2 = rcv2[S_];
      const uint32_t cm0 = rcm0[S_], cm1 = rcm1[S_], cm2 = rcm2[S_];
      constexpr int buf = S_ & 1;         // this step's staging (t0 is a multiple of kPF)
      constexpr int wbuf = (S_ + 1) & 1;  // the previous step's
      // Ring slots of the positions x, x - 1 and x + 1: the group's absolute
      // position t0 + S_ - 2g mod 4, which runs on across rows (so that a
      // position outside the row, whose slot is zeroed, precedes and follows
      // the row's ends); t0 is a multiple of 4 and -2g mod 4 = gsh, and
      // adding 0 or 2 mod 4 is an xor.
      const int slot = S_ ^ gsh, slot_m = ((S_ + 3) & 3) ^ gsh, slot_p = ((S_ + 1) & 3) ^ gsh;
      if (writer) {
        // outputs of the previous step: lane gg follows group gg, whose
        // position then was (band, x) one step back
        const int gg = (int)threadIdx.x & 63;
        const int y = band * kG + gg;
        const bool act = gg < kG && x >= 0 && x < W && y < H;
        const int64_t row = (int64_t)y * W;
        if (act) {
          Jdl[row + x] = st_dl[wbuf][gg];
          if (x >= dlast)
            Jdr[row + x - dlast] = (uint16_t)(reinterpret_cast<const uint8_t *>(st_dr[wbuf][gg])[dlast]);
        }
        // groups that finished a row: their remaining candidates x_r = W-1-d
        uint64_t ends = __ballot(act && x == W - 1);
        while (ends) {
          const int ge = __builtin_ctzll(ends);
          ends &= ends - 1;
          const int ye = __builtin_amdgcn_readlane(y, ge);
          const int d = gg;
          if (d < dlast && W - 1 - d >= 0)
            Jdr[(int64_t)ye * W + W - 1 - d] = (uint16_t)(reinterpret_cast<const uint8_t *>(st_dr[wbuf][ge])[d]);
        }
        // the band's last group: its path bytes become the carry row
        const int xl = __builtin_amdgcn_readlane(x, kG - 1);
        const int yl = __builtin_amdgcn_readlane(y, kG - 1);
        const int bl = __builtin_amdgcn_readlane(band, kG - 1);
        if (vert && xl >= 0 && xl < W && yl < H && gg < 52)
          *reinterpret_cast<uint32_t *>(Jcarry + (size_t)(bl & 1) * (W + 2) * kSweepCarry +
                                        (size_t)(xl + 1) * kSweepCarry + 4 * gg) = st_carry[wbuf][gg];
      }
      // the writer follows each group one step late: its counters start one
      // step behind (see the set-up below)
      const int y = band * kG + g;
      if (!writer && x >= 0 && x < W && y < H) {
        // Right-view codes move one disparity up per step, lane 0 taking
        // cr(x).  The four slots are renamed instead of moved: at step S_ of
        // an unrolled group, slot k lives in crs[(k - S_) & 3], so the new
        // slot 0 takes the register of the old slot 3 (the same for cand).
        constexpr int R0 = (0 - S_) & 3;
        const uint32_t in = (uint32_t)__builtin_amdgcn_update_dpp((int)ccr, (int)crs[R0], kDppRowShr1, 0xF,
                                                                  0xF, false);
        crs[R0] = in;
        auto CR = [&](int k) -> uint32_t { return crs[(k - S_) & 3]; };
        // matching costs of equation (1), N_b left of the image
        u16x2 C[2];
        uint32_t h[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) h[k] = (uint32_t)__builtin_popcount(ccl ^ CR(k));
        if (__builtin_amdgcn_ballot_w64(x < dbase + 3) == 0) {
          // every active lane is at least 4j + 3 pixels into its row (the
          // common case, taken by the whole wave): no cell is left of the image
#pragma unroll
          for (int q = 0; q < 2; ++q) C[q] = as_pair((h[2 * q] | h[2 * q + 1] << 16) | pad[q]);  // 0xFFFF for d >= D
        } else {
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int d0 = dbase + 2 * q;
            const uint32_t c0 = x >= d0 ? h[2 * q] : nbits;
            const uint32_t c1 = x >= d0 + 1 ? h[2 * q + 1] : nbits;
            C[q] = as_pair((c0 | c1 << 16) | pad[q]);
          }
        }
        u16x2 S[2] = {as_pair(0u), as_pair(0u)};
        if (pL) {
          u16x2 Lc[2];
          path_step(Lh, mh, C, P1, P2, Lc);
          mh = pair_min(Lc);
          Lh[0] = Lc[0];
          Lh[1] = Lc[1];
          S[0] = padd_sat(S[0], Lc[0]);
          S[1] = padd_sat(S[1], Lc[1]);
        }
        if (vert) {
          const bool carry_out = g == kG - 1;
          // path V (0: T2B, 1: TL2BR, 2: TR2BL) with its predecessor at
          // (x, y-1), (x-1, y-1) or (x+1, y-1)
          auto vpath = [&](auto vtag, bool on, int rslot, uint32_t carry_bytes, uint32_t carry_min) {
            constexpr int V = decltype(vtag)::value;
            if (!on) return;
            // the ring of the group above (group 0: the carry row).  Where
            // there is no predecessor (the first row, x - 1 < 0, x + 1 >= W)
            // these read zero path costs with minimum 0, so the path starts
            // as the recurrence's first pixel does (L = C): the carry row of
            // the first band and the carry columns -1 and W are zero, and a
            // group writes zeros into its ring at the positions outside its
            // row.
            const int ga = max(g - 1, 0);
            const uint32_t rb = ring[ga][rslot][V][j], rm = rmin[ga][rslot][V];
            const uint32_t bytes = g > 0 ? rb : carry_bytes, mp = g > 0 ? rm : carry_min;
            u16x2 Lp[2];
            unpack_bytes(bytes, usel, Lp);
            u16x2 Lc[2];
            path_step(Lp, mp, C, P1, P2, Lc);
            const uint32_t mc = pair_min(Lc);
            const uint32_t b = pack_bytes(Lc);
            ring[g][slot][V][j] = b;
            if (j == 0) rmin[g][slot][V] = mc;
            if (carry_out) {
              st_carry[buf][16 * V + j] = b;
              if (j == 0) st_carry[buf][48 + V] = mc;
            }
            S[0] = padd_sat(S[0], Lc[0]);
            S[1] = padd_sat(S[1], Lc[1]);
          };
          vpath(std::integral_constant<int, 0>{}, pT, slot, cv0, cm0);
          vpath(std::integral_constant<int, 1>{}, pTL, slot_m, cv1, cm1);
          vpath(std::integral_constant<int, 2>{}, pTR, slot_p, cv2, cm2);
        }
        // winner-takes-all and the right-view candidates, as (S << 8 | d)
        uint32_t key[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t sv = (k & 1) ? (uint32_t)S[k >> 1].y : (uint32_t)S[k >> 1].x;
          // cells with d >= D: S saturates at 0xFFFF (their path costs are
          // 0xFFFF; valid sums stay <= 4 * 255), so their keys lose to every
          // valid one
          key[k] = sv << 8 | (uint32_t)(dbase + k);
        }
        const uint32_t best = row16_allmin_u32(min(min(key[0], key[1]), min(key[2], key[3])));
        if (j == 0) st_dl[buf][g] = (uint8_t)(best & 0xFF);
        // candidates move one disparity up, the new one (x_r = x) enters at d = 0
        cand[R0] = (uint32_t)__builtin_amdgcn_update_dpp((int)kInf, (int)cand[R0], kDppRowShr1, 0xF, 0xF, false);
#pragma unroll
        for (int k = 0; k < 4; ++k) cand[(k - S_) & 3] = min(cand[(k - S_) & 3], key[k]);
        // the candidate holding d = D-1 is final (x_r = x - D + 1), and at the
        // row end every candidate is (x_r + d' >= W beyond): stage them all
        st_dr[buf][g][j] = (cand[(0 - S_) & 3] & 0xFF) | (cand[(1 - S_) & 3] & 0xFF) << 8 |
                           (cand[(2 - S_) & 3] & 0xFF) << 16 | (cand[(3 - S_) & 3] & 0xFF) << 24;
      } else if (!writer) {
        // outside the row (at least two steps between rows): the next row's
        // L2R path and right-view candidates begin anew, and the ring slot of
        // this position reads as "no predecessor" for the group below
        Lh[0] = as_pair(pad[0]);
        Lh[1] = as_pair(pad[1]);
        mh = 0u;
#pragma unroll
        for (int k = 0; k < 4; ++k) cand[k] = kInf;
        if (vert) {
#pragma unroll
          for (int v = 0; v < 3; ++v) ring[g][slot][v][j] = 0u;
          if (j < 3) rmin[g][slot][j] = 0u;
        }
      }
      // refill the slot for the step kPF ahead once this step is done with
      // it, so that the slot's old and new values can share registers
      prefetch(stag, bandf, xf);
      advance(bandf, xf);
      advance(band, x);
      __syncthreads();
  };
  for (int t0 = 0; t0 < T; t0 += kPF) {
    step(std::integral_constant<int, 0>{});
    step(std::integral_constant<int, 1>{});
    step(std::integral_constant<int, 2>{});
    step(std::integral_constant<int, 3>{});
  }
}

__global__ __launch_bounds__(256) void lr_kernel(JobTable<LRJob> t) {
  const int ji = find_job(t.j, t.n, (int)blockIdx.x);
  const LRJob &J = t.j[ji];
  const int64_t i = (int64_t)((int)blockIdx.x - J.blk0) * 256 + threadIdx.x;
  const int64_t n = (int64_t)J.W * J.H;
  if (i >= n) return;
  const int dl = J.dl[i];
  uint16_t v = (uint16_t)dl;
  if (J.lr_check) {
    const int x = (int)(i % J.W);
    v = (uint16_t)J.invalid;
    if (x - dl >= 0) {
      const int dr = J.dr[i - dl];
      if (abs(dl - dr) <= J.max_diff) v = (uint16_t)dl;
    }
  }
  J.out[i] = v;
}

void launch_sweep(std::vector<SweepJob> jobs, hipStream_t s) {
  for_each_table(
      jobs, [](const SweepJob &j) { return (long)j.count; },
      [&](const JobTable<SweepJob> &t, int blocks) {
        hipLaunchKernelGGL(sweep_kernel, dim3(blocks), dim3(1024), 0, s, t);
      });
}

void launch_lr(std::vector<LRJob> jobs, hipStream_t s) {
  for_each_table(
      jobs, [](const LRJob &j) { return (long)(((int64_t)j.W * j.H + 255) / 256); },
      [&](const JobTable<LRJob> &t, int blocks) {
        hipLaunchKernelGGL(lr_kernel, dim3(blocks), dim3(256), 0, s, t);
      });
}

}  // namespace sgmk
