// Two-pass schedule of the 8-path aggregation with disparity selection fused
// into the second pass (section 3.1.3: the forward paths in one pass over the
// image and the backward paths in a second pass from back to front; equation
// (2) per path, S the sum over paths, WTA and the right-view disparity of
// section 3.1.4).
//
// The four paths whose predecessor lies in the row above or on the same row
// to the left or right (L->R, R->L, TR->BL, BL->TR) run as ordinary
// per-direction waves (agg_kernel) into four uint8 path-cost slots.  The
// vertical and the two remaining diagonal paths run here, a frame split into
// stripes of SW = 4 * WAVES columns, one workgroup per stripe walking the
// rows:
//
//   down pass (T->B, TL->BR), rows top to bottom: writes S_D = L_TB + L_TLBR
//     + the L->R and R->L slots as uint16 [H][W][Dp], each pixel in the
//     chunked layout below;
//   up pass (B->T, BR->TL), rows bottom to top: S = S_D + L_BT + L_BRTL + the
//     TR->BL and BL->TR slots, then the WTA map D_L and each (row, stripe)'s
//     right-view keys, in the layout of the disparity kernel's row segments
//     (segment length SW), so that the LR check and the median read them
//     unchanged.
// Each pass adds two of the slots (the down pass has the memory headroom,
// the up pass moved the most bytes).  A row's slots (and, up, S_D) are
// loaded a row ahead: at the start of a row they are summed into a partial
// sum parked in LDS, and the next row's loads go into the same registers.
//
// Matching costs (equation (1)): read from the uint8 cost volume, or (CODES:
// frames whose horizontal directions run on Census windows, so that their
// code records {left, right} exist) formed from the Census codes, which the
// workgroup stages in LDS a row ahead: the right-view codes of positions
// x0 - Dp + 1 .. x0 + SW - 1 and the left codes of its pixels.
//
// Lane layout: 16 lanes per pixel (a DPP row), lane j owning the K
// disparities jK .. jK+K-1, four pixels per wave, consecutive pixels in
// consecutive rows of a wave.  A pixel's vertical predecessor is its own
// registers; the diagonal predecessor (x -/+ 1 of the previous row) comes
// from a double-buffered LDS row of the stripe's path costs, and at the
// stripe's edge from the neighbouring stripe: the edge pixel's path costs of
// every row are published as 64-bit words {two 16-bit path costs, epoch}
// (in the chunked order) with device-scope relaxed atomic stores; the
// consumer's edge wave (the wave holding the stripe's edge pixel) keeps the
// records of the next rows in flight as device-scope atomic loads (four rows
// ahead in the down pass, one in the up pass, two words per lane), retries a
// row until every word carries the launch's epoch, and hands it to the edge
// pixel through LDS.  The epoch in the word makes a stale record of an
// earlier launch unmistakable, and a 64-bit store is single-copy atomic, so
// neither fences nor flags are needed.  The predecessor is read without a
// branch (a per-lane LDS address and a select) so that the vertical and
// diagonal recurrences share one basic block and their dependent chains
// interleave.
//
// Memory operations go through per-row buffer descriptors (a scalar base and
// a 32-bit lane offset) and stores of pixels outside the image are dropped by
// the descriptor's range check rather than skipped by a branch: both keep the
// compiler's in-order wait counts as loose as the ring allows and the
// registers within the 128 a 1024-thread workgroup has (a spill's reload
// would wait for every load in flight).
//
// Workgroups take their stripe from a ticket counter (one atomic add each):
// a stripe waits only for the stripe before it in ticket order, which took
// its ticket earlier and is therefore running or done, so the waits always
// end whatever the number of workgroups resident at once.  A wait is also
// bounded (after max_polls polls it records an error in the frame's sync
// words, which the host reads when the batch is done, and goes on).
#include "device_util.h"

namespace sgmk {

namespace {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as_pair(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ u16x2 pmin(u16x2 a, u16x2 b) { return __builtin_elementwise_min(a, b); }
__device__ __forceinline__ u16x2 padd_sat(u16x2 a, u16x2 b) { return __builtin_elementwise_add_sat(a, b); }

constexpr uint32_t kInf = 0xFFFFFFFFu;

// One pixel of equation (2) for the lane's K disparities (16 lanes per
// pixel): Lp the predecessor's path costs and C the lane's K matching costs
// (packed pairs).  Pairs with d >= D are forced to 0xFFFF.
template <int K, bool PAD>
__device__ __forceinline__ void recur(const u16x2 (&Lp)[K / 2], const u16x2 (&C)[K / 2], u16x2 P1, u16x2 P2,
                                      const uint32_t (&padmask)[K / 2], u16x2 (&Lc)[K / 2]) {
  constexpr int NP = K / 2;
  const uint32_t prev = (uint32_t)__builtin_amdgcn_update_dpp((int)kInf, (int)as_u32(Lp[NP - 1]), kDppRowShr1,
                                                              0xF, 0xF, false);
  const uint32_t next = (uint32_t)__builtin_amdgcn_update_dpp((int)kInf, (int)as_u32(Lp[0]), kDppRowShl1, 0xF,
                                                              0xF, false);
  // Nb[q] = (L[2q-1], L[2q]): pair q's d-1 values in Nb[q], its d+1 values in Nb[q+1]
  u16x2 Nb[NP + 1];
  Nb[0] = as_pair(__builtin_amdgcn_alignbit(as_u32(Lp[0]), prev, 16));
#pragma unroll
  for (int q = 1; q < NP; ++q) Nb[q] = as_pair(__builtin_amdgcn_alignbit(as_u32(Lp[q]), as_u32(Lp[q - 1]), 16));
  Nb[NP] = as_pair(__builtin_amdgcn_alignbit(next, as_u32(Lp[NP - 1]), 16));
  u16x2 A[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) A[q] = pmin(padd_sat(pmin(Nb[q], Nb[q + 1]), P1), Lp[q]);
  u16x2 lm = Lp[0];
#pragma unroll
  for (int q = 1; q < NP; ++q) lm = pmin(lm, Lp[q]);
  const uint32_t mp = row16_allmin_u32(min((uint32_t)lm.x, (uint32_t)lm.y));
  const u16x2 M = {(unsigned short)mp, (unsigned short)mp};
  const u16x2 MP2 = padd_sat(M, P2);
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    u16x2 v = pmin(A[q], MP2) - M + C[q];
    if (PAD) v = as_pair(as_u32(v) | padmask[q]);
    Lc[q] = v;
  }
}

// Raw buffer stores (row_rsrc: a descriptor over one row of a volume; the
// hardware drops a store whose offset lies beyond the descriptor's size), so
// that pixels outside the image need no branch around their stores: a branch
// that skips memory operations on some path makes the compiler's wait counts
// assume the fewest operations in flight, i.e. wait for older loads and
// stores too soon.
constexpr int kBufNT = 2;              // non-temporal: written once, read by a later kernel
constexpr uint32_t kDropped = 0x80000000u;  // an offset beyond any row

// The chunked pixel layout of 16-bit path-cost sums ([Dp / 2] words per
// pixel), used by the LDS rows of diagonal path costs and by S_D: lane j's NP
// words in chunks of up to four, chunk c of the pixel's 16 lanes side by
// side, so that one 128-bit access of a chunk by a pixel's lanes covers
// consecutive words: no two lanes of an LDS pass on one bank, and whole
// cache lines per store in memory (the disparity order would give each store
// instruction 16-byte pieces at a 32-byte stride, which costs the down pass
// a quarter of its time).
template <int NP>
__host__ __device__ constexpr int chunk_words(int c) {
  return NP - 4 * c < 4 ? NP - 4 * c : 4;
}
template <int NP>
__device__ __forceinline__ int chunk_at(int j, int c) {
  return 64 * c + j * chunk_words<NP>(c);
}

typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));  // 16-byte aligned
typedef uint32_t u32x2v __attribute__((ext_vector_type(2)));

template <int NP, int c>
__device__ __forceinline__ void lds_chunk_read(U32N<NP> &v, const uint32_t *p) {
  if constexpr (NP - 4 * c >= 4) {
    const u32x4v a = *reinterpret_cast<const u32x4v *>(p);
    v.v[4 * c] = a.x, v.v[4 * c + 1] = a.y, v.v[4 * c + 2] = a.z, v.v[4 * c + 3] = a.w;
  } else {
    const u32x2v a = *reinterpret_cast<const u32x2v *>(p);
    v.v[4 * c] = a.x, v.v[4 * c + 1] = a.y;
  }
}
template <int NP, int c>
__device__ __forceinline__ void lds_chunk_write(const U32N<NP> &v, uint32_t *p) {
  if constexpr (NP - 4 * c >= 4)
    *reinterpret_cast<u32x4v *>(p) = u32x4v{v.v[4 * c], v.v[4 * c + 1], v.v[4 * c + 2], v.v[4 * c + 3]};
  else
    *reinterpret_cast<u32x2v *>(p) = u32x2v{v.v[4 * c], v.v[4 * c + 1]};
}

// N words at byte offset off of a row (loads by row descriptor: one 32-bit
// offset per lane instead of a 64-bit address per load)
template <int N, int AUX>
__device__ __forceinline__ U32N<N> load_row(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  U32N<N> v;
  if constexpr (N == 4) {
    const u32x4v a = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, AUX);
    v.v[0] = a.x, v.v[1] = a.y, v.v[2] = a.z, v.v[3] = a.w;
  } else if constexpr (N == 2) {
    const u32x2v a = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX);
    v.v[0] = a.x, v.v[1] = a.y;
  } else if constexpr (N == 1) {
    v.v[0] = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX);
  } else {
    static_assert(N == 3, "row loads of 1 to 4 words");
    const u32x2v a = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX);
    v.v[0] = a.x, v.v[1] = a.y, v.v[2] = __builtin_amdgcn_raw_buffer_load_b32(r, off + 8, 0, AUX);
  }
  return v;
}

// one pixel's sums in the chunked layout to a row of S_D (off: the pixel's
// byte offset in the row, or kDropped)
template <int NP>
__device__ __forceinline__ void store_pixel(const U32N<NP> &v, __amdgpu_buffer_rsrc_t r, uint32_t off, int j) {
  if constexpr (NP >= 4)
    __builtin_amdgcn_raw_buffer_store_b128(u32x4v{v.v[0], v.v[1], v.v[2], v.v[3]}, r, off + 4 * chunk_at<NP>(j, 0),
                                           0, kBufNT);
  else
    __builtin_amdgcn_raw_buffer_store_b64(u32x2v{v.v[0], v.v[1]}, r, off + 4 * chunk_at<NP>(j, 0), 0, kBufNT);
  if constexpr (NP == 8)
    __builtin_amdgcn_raw_buffer_store_b128(u32x4v{v.v[4], v.v[5], v.v[6], v.v[7]}, r, off + 4 * chunk_at<NP>(j, 1),
                                           0, kBufNT);
  else if constexpr (NP == 6)
    __builtin_amdgcn_raw_buffer_store_b64(u32x2v{v.v[4], v.v[5]}, r, off + 4 * chunk_at<NP>(j, 1), 0, kBufNT);
}

// and back (off: the pixel's byte offset in the row)
template <int NP>
__device__ __forceinline__ U32N<NP> load_pixel(__amdgpu_buffer_rsrc_t r, uint32_t off, int j) {
  U32N<NP> v;
  constexpr int c0 = NP >= 4 ? 4 : 2;
  const U32N<c0> a = load_row<c0, kBufNT>(r, off + 4 * chunk_at<NP>(j, 0));
#pragma unroll
  for (int i = 0; i < c0; ++i) v.v[i] = a.v[i];
  if constexpr (NP > 4) {
    const U32N<NP - 4> b = load_row<NP - 4, kBufNT>(r, off + 4 * chunk_at<NP>(j, 1));
#pragma unroll
    for (int i = 0; i < NP - 4; ++i) v.v[4 + i] = b.v[i];
  }
  return v;
}

// LDS slot of staged right-view Census code t (one padding slot per 16: a
// pixel's lanes read codes 16 apart, which then fall on different banks)
__host__ __device__ constexpr int cslot(int t) { return t + (t >> 4); }

// LDS slot of the right-view key of zone position i (two padding slots per K
// positions: the lanes of a pixel update positions K apart, the pixels of a
// wave consecutive positions, and a half wave then hits 32 banks).
template <int K>
__host__ __device__ constexpr int zslot(int i) {
  if constexpr ((K & (K - 1)) == 0) return i + 2 * (i / K);
  else return i + (i >> 3);
}

}  // namespace

template <int K, bool UP, int WAVES, bool PAD, bool CODES>
__global__ __launch_bounds__(WAVES * 64) void stripe_kernel(JobTable<StripeJob> t) {
  constexpr int NP = K / 2, NW = K / 4, SW = 4 * WAVES;
  constexpr int PFR = UP ? 1 : 4, ER = PFR;  // rows of costs and of edge records in flight
  extern __shared__ __align__(16) uint32_t lds[];  // 128-bit row accesses
  __shared__ int s_ticket;
  // ticket counters: word 0 (down pass) and word 2 (up pass) of the table's
  // first job
  if (threadIdx.x == 0) s_ticket = (int)atomicAdd(t.j[0].sync + (UP ? 2 : 0), 1u);
  __syncthreads();
  const int tk = s_ticket;
  // every workgroup of the grid gets one of the grid's tickets; one beyond
  // them (counters not cleared) takes no stripe
  if (tk >= t.j[t.n - 1].blk0 + t.j[t.n - 1].nstripes) return;
  const int ji = find_job(t.j, t.n, tk);
  const StripeJob &J = t.j[ji];
  const int W = J.W, H = J.H, D = J.D, Dp = J.Dp;
  const int ns = J.nstripes;
  const int si = tk - J.blk0;
  const int s = UP ? ns - 1 - si : si;  // up pass: stripes from the right
  const int x0 = s * SW;
  const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
  const int px = wave * 4 + (lane >> 4), j = lane & 15;
  const int x = x0 + px;
  const bool live = x < W;
  const int xc = min(x, W - 1);  // loads of pixels right of the image read the last column
  const int dbase = j * K;
  const int dvalid = PAD ? min(K, max(0, D - dbase)) : K;
  uint32_t padmask[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q)
    padmask[q] = (2 * q < dvalid ? 0u : 0xFFFFu) | (2 * q + 1 < dvalid ? 0u : 0xFFFF0000u);
  const u16x2 P1 = {(unsigned short)J.p1, (unsigned short)J.p1};
  const u16x2 P2 = {(unsigned short)J.p2, (unsigned short)J.p2};
  const uint32_t epoch = J.epoch;

  // LDS: the diagonal path costs of the stripe's pixels for two rows
  // ([2][SW][Dp / 2] words, each pixel in the chunked layout), then the
  // neighbour's edge pixel of the previous row (same layout), then the
  // pixels' partial sums ([SW][Dp / 2] words, same layout), (CODES) two rows
  // of Census codes and (up pass with the LR check) two zone key rows
  uint32_t *dg = lds;
  const int dg_words = SW * Dp / 2;
  const int zn = SW + D - 1;  // zone positions of a segment of SW pixels
  const int zslots = zslot<K>(zn - 1) + 1;
  uint32_t *eslot = lds + 2 * dg_words;
  // each pixel's partial sum of the current row: two slots (up: + S_D)
  uint32_t *pacc = eslot + Dp / 2;
  // (CODES) the Census codes of two rows: right-view codes of positions
  // x0 - Dp + 1 + t, t < span ([2][cr_slots], slot cslot(t)), and the left
  // codes of the stripe's pixels ([2][SW])
  const int span = SW + Dp - 1;
  const int cr_slots = cslot(span - 1) + 1;
  uint64_t *cR = reinterpret_cast<uint64_t *>(pacc + SW * Dp / 2);
  uint64_t *cL = cR + 2 * cr_slots;
  uint32_t *zone = reinterpret_cast<uint32_t *>(CODES ? cL + 2 * SW : cR);
  const int zr = x0 - D + 1;
  if (UP && J.lr_check) {
    for (int i = (int)threadIdx.x; i < 2 * zslots; i += WAVES * 64) zone[i] = kInf;
  }

  // the stripe's edge: the neighbour whose diagonal predecessor we take
  // (down: x0 - 1 from stripe s - 1; up: x0 + SW from stripe s + 1), and
  // the pixel we publish for the stripe on the other side.  The wave that
  // holds the taking pixel (the edge wave) keeps the neighbour's records of
  // the next ER rows in flight, two words per lane, and passes each row's
  // record to the taking pixel through eslot.
  const bool takes_edge = UP ? (px == SW - 1 && s + 1 < ns) : (px == 0 && s > 0);
  const bool gives_edge = UP ? (px == 0 && s > 0) : (px == SW - 1 && s + 1 < ns);
  const bool edge_wave = (UP ? wave == WAVES - 1 : wave == 0) && (UP ? s + 1 < ns : s > 0);
  const int s_in = min(max(UP ? s + 1 : s - 1, 0), ns - 1);  // the neighbour (if any)
  const uint64_t *bnd_in = J.bnd + ((int64_t)s_in * H) * (Dp / 2);
  const int ew = 2 * lane;                  // this lane's first word of a record
  const bool ew_live = ew < Dp / 2;         // Dp / 2 words per record (even)
  bool failed = false;

  const int ystep = UP ? -1 : 1;
  const int y_first = UP ? H - 1 : 0;
  const int64_t row_cells = (int64_t)W * Dp;
  const uint32_t lane_off = (uint32_t)(xc * Dp + dbase);  // the lane's bytes in a uint8 row
  auto load_costs = [&](int pr) {
    return load_row<NW, 0>(row_rsrc(J.cost + (int64_t)(y_first + ystep * pr) * row_cells, (uint32_t)row_cells),
                           lane_off);
  };

  u16x2 Lv[NP];  // vertical path: this pixel's previous row
#pragma unroll
  for (int q = 0; q < NP; ++q) Lv[q] = as_pair(padmask[q]);
  // the edge records of pass rows r .. r + ER - 1 (row r's record is the
  // predecessor of pass row r + 1)
  uint64_t erec[ER][2] = {};
  auto load_rec = [&](int pr, uint64_t (&w)[2]) {
    const uint64_t *q = bnd_in + (int64_t)(y_first + ystep * pr) * (Dp / 2) + ew;
    w[0] = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    w[1] = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  if (edge_wave && ew_live) {
#pragma unroll
    for (int u = 0; u < ER; ++u) load_rec(min(u, H - 1), erec[u]);
  }
  // the costs of the next PFR rows in a register ring (loads are
  // unconditional: past the last row they re-read it)
  U32N<NW> ring[PFR];
  if constexpr (!CODES) {
#pragma unroll
    for (int u = 0; u < PFR; ++u) ring[u] = load_costs(min(u, H - 1));
  }
  // CODES: thread t stages position t's record {left, right} of a row; the
  // records of the row after next are loaded while a row runs (positions
  // right of the image read nothing: the descriptor ends at column W - 1)
  U32N<4> crec;
  const int ct = (int)threadIdx.x;
  auto load_codes = [&](int pr) {
    const int64_t p0 = (int64_t)(y_first + ystep * pr) * W + (x0 - Dp + 1);  // record of t = 0
    const uint32_t n = (uint32_t)min(span, W - x0 + Dp - 1);
    crec = load_row<4, 0>(row_rsrc(J.codes + 2 * p0, n * 16), ct < span ? (uint32_t)ct * 16 : kDropped);
  };
  auto stage_codes = [&](int b) {
    if (ct < span) {
      cR[b * cr_slots + cslot(ct)] = (uint64_t)crec.v[2] | (uint64_t)crec.v[3] << 32;
      if (ct >= Dp - 1) cL[b * SW + ct - (Dp - 1)] = (uint64_t)crec.v[0] | (uint64_t)crec.v[1] << 32;
    }
  };
  if constexpr (CODES) {
    load_codes(0);
    stage_codes(0);
    load_codes(min(1, H - 1));
  }
  const bool left_edge = x0 < Dp - 1;  // some of the stripe's costs reach left of the image
  const uint32_t nbits = (uint32_t)J.nbits;
  // the two path-cost slots this pass adds (down: L->R and R->L, into S_D;
  // up: TR->BL and BL->TR) and, up, S_D, of the next pass row
  constexpr int S0 = UP ? 2 : 0;
  U32N<2 * NW> sl;
  U32N<NP> sd;
  auto load_sums = [&](int pr) {
    const int64_t row0 = (int64_t)(y_first + ystep * pr) * row_cells;
    const int64_t slot = (int64_t)H * row_cells;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const U32N<NW> v =
          load_row<NW, kBufNT>(row_rsrc(J.lr4 + (S0 + p) * slot + row0, (uint32_t)row_cells), lane_off);
#pragma unroll
      for (int i = 0; i < NW; ++i) sl.v[p * NW + i] = v.v[i];
    }
    if constexpr (UP)
      sd = load_pixel<NP>(row_rsrc(J.sd + row0, (uint32_t)(row_cells * 2)), (uint32_t)(xc * Dp * 2), j);
  };
  load_sums(0);
  __syncthreads();  // zone rows cleared

  auto row = [&](int r, U32N<NW> &slot, uint64_t (&prev_rec)[2]) {
    const int y = y_first + r * ystep;
    const int buf = r & 1;
    // the edge wave: validate the neighbour's record of pass row r - 1 (its
    // words carry this launch's epoch once written), hand it to the taking
    // pixel through eslot, and fetch the record of pass row r - 1 + ER
    if (edge_wave && r > 0) {
      bool ok = !ew_live || ((uint32_t)(prev_rec[0] >> 32) == epoch && (uint32_t)(prev_rec[1] >> 32) == epoch);
      for (int n = 0; __builtin_amdgcn_ballot_w64(!ok) != 0 && !failed; ++n) {
        if (n == J.max_polls) {
          failed = true;
          __hip_atomic_store(J.sync + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(2);
        if (ew_live) {
          load_rec(r - 1, prev_rec);
          ok = (uint32_t)(prev_rec[0] >> 32) == epoch && (uint32_t)(prev_rec[1] >> 32) == epoch;
        }
      }
      if (ew_live) {
        int e = ew;
        asm volatile("" : "+v"(e));  // recomputed per row, not held in a register along the row
        eslot[e] = (uint32_t)prev_rec[0];  // records are in the chunked layout
        eslot[e + 1] = (uint32_t)prev_rec[1];
        if (r - 1 + ER < H) load_rec(r - 1 + ER, prev_rec);
      }
    }
    // the lane's K matching costs as pairs: from the cost ring, or formed from
    // the staged Census codes (equation (1): C = popcount(cl ^ cr(x - d)),
    // N_b where x - d < 0), and the next row's codes staged
    u16x2 C[NP];
    if constexpr (!CODES) {
#pragma unroll
      for (int q = 0; q < NP; ++q)  // bytes 2q, 2q+1 of the lane's costs
        C[q] = as_pair(__builtin_amdgcn_perm(0u, slot.v[q >> 1], (q & 1) ? 0x0c030c02u : 0x0c010c00u));
    } else {
      // the lane's codes are positions t0 - k, k < K (K <= 16): consecutive
      // slots except for at most one padding slot, after k = t0 mod 16; the
      // two bases are formed per row (held along the row, each code's
      // address would take a register)
      int t0 = px + Dp - 1 - dbase;  // position of x - dbase
      asm volatile("" : "+v"(t0));
      const uint64_t *crA = cR + buf * cr_slots + cslot(t0);
      const uint64_t *crB = crA - 1;
      const int rk = t0 & 15;
      const uint64_t cl = cL[buf * SW + px];
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        uint32_t c0 = (uint32_t)__popcll(cl ^ (2 * q > rk ? crB : crA)[-2 * q]);
        uint32_t c1 = (uint32_t)__popcll(cl ^ (2 * q + 1 > rk ? crB : crA)[-2 * q - 1]);
        if (left_edge) {
          c0 = x - dbase - 2 * q >= 0 ? c0 : nbits;
          c1 = x - dbase - 2 * q - 1 >= 0 ? c1 : nbits;
        }
        C[q] = as_pair(c0 | c1 << 16);
        // four codes at a time: all of them in flight at once would take 32
        // registers
        if (q % 2 == 1) __builtin_amdgcn_sched_barrier(0);
      }
      stage_codes(buf ^ 1);
      load_codes(min(r + 2, H - 1));
    }
    // this row's two path-cost slots and (up) S_D, loaded a row earlier,
    // summed into the pixel's row of pacc, and the next row's loads issued
    // into the same registers, so that they have a whole row to arrive
    {
      U32N<NP> part;
#pragma unroll
      for (int q = 0; q < NP; ++q) part.v[q] = UP ? sd.v[q] : 0u;
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int i = 0; i < NW; ++i) {
          const uint32_t w = sl.v[p * NW + i];
          part.v[2 * i] += __builtin_amdgcn_perm(0u, w, 0x0c010c00u);
          part.v[2 * i + 1] += __builtin_amdgcn_perm(0u, w, 0x0c030c02u);
        }
      uint32_t *pix = pacc + px * (Dp / 2);
      lds_chunk_write<NP, 0>(part, pix + chunk_at<NP>(j, 0));
      if constexpr (NP > 4) lds_chunk_write<NP, 1>(part, pix + chunk_at<NP>(j, 1));
      load_sums(min(r + 1, H - 1));
    }

    // diagonal path: the predecessor x -/+ 1 of the previous row, read
    // without a branch (the taking pixel from eslot, the others from the
    // previous LDS row; at a path start the values are replaced), so that
    // the vertical and diagonal recurrences below share one basic block and
    // their dependent chains interleave
    const int pp = UP ? px + 1 : px - 1;  // predecessor pixel in the stripe
    const bool start = r == 0 || (UP ? (x + 1 >= W) : (x == 0));
    U32N<NP> pv;
    {
      const uint32_t *pix = takes_edge ? eslot : dg + (buf ^ 1) * dg_words + min(max(pp, 0), SW - 1) * (Dp / 2);
      lds_chunk_read<NP, 0>(pv, pix + chunk_at<NP>(j, 0));  // NP <= 8: at most two chunks
      if constexpr (NP > 4) lds_chunk_read<NP, 1>(pv, pix + chunk_at<NP>(j, 1));
    }
    u16x2 Lp[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) Lp[q] = as_pair(start ? padmask[q] : pv.v[q]);
    // vertical path
    u16x2 Lcv[NP];
    recur<K, PAD>(Lv, C, P1, P2, padmask, Lcv);
    u16x2 Lcd[NP];
    recur<K, PAD>(Lp, C, P1, P2, padmask, Lcd);
    {  // this row's diagonal path costs for the next row's predecessors
      U32N<NP> v;
#pragma unroll
      for (int q = 0; q < NP; ++q) v.v[q] = as_u32(Lcd[q]);
      uint32_t *pix = dg + buf * dg_words + px * (Dp / 2);
      lds_chunk_write<NP, 0>(v, pix + chunk_at<NP>(j, 0));
      if constexpr (NP > 4) lds_chunk_write<NP, 1>(v, pix + chunk_at<NP>(j, 1));
    }
    if (gives_edge && !J.withhold) {
      // (addresses as a row base and a 32-bit lane offset: a 64-bit
      // address per lane would take registers all along the row)
      uint64_t *brow = J.bnd + ((int64_t)s * H + y) * (Dp / 2);
#pragma unroll
      for (int q = 0; q < NP; ++q)
        __hip_atomic_store(brow + (uint32_t)(chunk_at<NP>(j, q / 4) + q % 4),
                           (uint64_t)as_u32(Lcd[q]) | (uint64_t)epoch << 32, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) Lv[q] = Lcv[q];
    // the ring slot's refill once its costs are consumed, into the same
    // registers (a load into fresh ones would need a copy at the loop's back
    // edge, which waits for every memory operation in flight)
    if constexpr (!CODES) slot = load_costs(min(r + PFR, H - 1));

    if constexpr (!UP) {
      // S_D = L_TB + L_TLBR + L_LR + L_RL as packed 16-bit pairs (no carry
      // reaches a valid half, as in the up pass's sum below)
      U32N<NP> o;
      {
        const uint32_t *pix = pacc + px * (Dp / 2);
        lds_chunk_read<NP, 0>(o, pix + chunk_at<NP>(j, 0));
        if constexpr (NP > 4) lds_chunk_read<NP, 1>(o, pix + chunk_at<NP>(j, 1));
      }
#pragma unroll
      for (int q = 0; q < NP; ++q) o.v[q] += as_u32(Lcv[q]) + as_u32(Lcd[q]);
      store_pixel<NP>(o, row_rsrc(J.sd + (int64_t)y * row_cells, (uint32_t)(row_cells * 2)),
                      live ? (uint32_t)(x * Dp * 2) : kDropped, j);
    } else {
      // S over the eight paths as packed 16-bit pairs (no carry reaches a
      // valid half: every valid sum is below 65536, and padding halves lie
      // above the valid ones)
      U32N<NP> part;
      {
        const uint32_t *pix = pacc + px * (Dp / 2);
        lds_chunk_read<NP, 0>(part, pix + chunk_at<NP>(j, 0));
        if constexpr (NP > 4) lds_chunk_read<NP, 1>(part, pix + chunk_at<NP>(j, 1));
      }
      uint32_t acc[NP];
#pragma unroll
      for (int q = 0; q < NP; ++q) acc[q] = part.v[q] + as_u32(Lcv[q]) + as_u32(Lcd[q]);
      uint32_t best = kInf;
      uint32_t *zrow = zone + buf * zslots;
      // the lane's zone positions i0 - k: with K a power of two they cross at
      // most one block of K (two padding slots) after k = i0 mod K, so two
      // bases formed per row address them all (held along the row, each
      // position's address would take a register)
      int i0 = x - dbase - zr;
      asm volatile("" : "+v"(i0));
      uint32_t *zA = zrow + zslot<K>(i0);
      uint32_t *zB = zA - 2;
      const int mk = i0 & (K - 1);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (k < dvalid) {
          const int d = dbase + k;
          const uint32_t Sd = (k & 1) ? acc[k >> 1] >> 16 : acc[k >> 1] & 0xFFFFu;
          const uint32_t key = Sd << 8 | (uint32_t)d;
          best = min(best, key);
          if (J.lr_check && live && x >= d) {
            if constexpr ((K & (K - 1)) == 0) atomicMin((k > mk ? zB : zA) - k, key);
            else atomicMin(&zrow[zslot<K>(x - d - zr)], key);
          }
        }
      }
      best = row16_allmin_u32(best);
      __builtin_amdgcn_raw_buffer_store_b16((unsigned short)(best & 0xFF), row_rsrc(J.dl + (int64_t)y * W, W * 2),
                                            live && j == 0 ? (uint32_t)(x * 2) : kDropped, 0, 0);
    }
    __syncthreads();
    if (UP && J.lr_check) {
      // the row's zone keys out, and the zone row cleared for two rows on
      uint32_t *zrow = zone + buf * zslots;
      const __amdgpu_buffer_rsrc_t prow = row_rsrc(J.part + ((int64_t)y * ns + s) * zn, (uint32_t)zn * 4);
      int i0 = (int)threadIdx.x;
      asm volatile("" : "+v"(i0));  // recomputed per row, not held in a register along the row
      for (int i = i0; i < zn; i += WAVES * 64) {
        __builtin_amdgcn_raw_buffer_store_b32(zrow[zslot<K>(i)], prow, (uint32_t)i * 4, 0, 0);
        zrow[zslot<K>(i)] = kInf;
      }
    }
  };
  // rows in blocks of PFR (= ER): ring slots are compile-time indices
  int r0 = 0;
  for (; r0 + PFR <= H; r0 += PFR) {
#pragma unroll
    for (int u = 0; u < PFR; ++u) row(r0 + u, ring[u], erec[(u + ER - 1) % ER]);
  }
#pragma unroll
  for (int u = 0; u < PFR; ++u)
    if (r0 + u < H) row(r0 + u, ring[u], erec[(u + ER - 1) % ER]);
}

namespace {
__global__ __launch_bounds__(256) void zero_kernel(JobTable<SyncZeroJob> t) {
  const int ji = find_job(t.j, t.n, (int)blockIdx.x);
  const SyncZeroJob &J = t.j[ji];
  const int i = ((int)blockIdx.x - J.blk0) * 256 + (int)threadIdx.x;
  if (i < J.words) J.p[i] = 0;
}
}  // namespace

void launch_zero_sync(std::vector<SyncZeroJob> jobs, hipStream_t s) {
  for_each_table(
      jobs, [](const SyncZeroJob &j) { return (long)((j.words + 255) / 256); },
      [&](const JobTable<SyncZeroJob> &t, int blocks) {
        hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, s, t);
      });
}

size_t stripe_lds(int K, int D, int waves, bool up, bool codes) {
  const int SW = 4 * waves, Dp = 16 * K;
  const int zn = SW + D - 1;
  const int zslots = (K & (K - 1)) == 0 ? zn - 1 + 2 * ((zn - 1) / K) + 1 : zn - 1 + ((zn - 1) >> 3) + 1;
  // diagonal rows, edge pixel, partial sums, (codes) two rows of Census
  // codes, zone rows
  return (size_t)2 * SW * Dp * 2 + (size_t)Dp * 2 + (size_t)SW * Dp * 2 +
         (codes ? (size_t)2 * (cslot(SW + Dp - 2) + 1 + SW) * 8 : 0) + (size_t)2 * zslots * 4;
}

template <int K, bool UP, int WAVES, bool CODES>
static void launch_kw(const JobTable<StripeJob> &t, int blocks, bool pad, size_t lds, hipStream_t s) {
  if (pad)
    hipLaunchKernelGGL((stripe_kernel<K, UP, WAVES, true, CODES>), dim3(blocks), dim3(WAVES * 64), lds, s, t);
  else
    hipLaunchKernelGGL((stripe_kernel<K, UP, WAVES, false, CODES>), dim3(blocks), dim3(WAVES * 64), lds, s, t);
}

template <int K, bool CODES>
static void launch_k(const JobTable<StripeJob> &t, int blocks, bool up, int waves, bool pad, size_t lds,
                     hipStream_t s) {
  if (up && waves == 16) launch_kw<K, true, 16, CODES>(t, blocks, pad, lds, s);
  else if (up) launch_kw<K, true, 8, CODES>(t, blocks, pad, lds, s);
  else if (waves == 16) launch_kw<K, false, 16, CODES>(t, blocks, pad, lds, s);
  else launch_kw<K, false, 8, CODES>(t, blocks, pad, lds, s);
}

void launch_stripes(std::vector<StripeJob> jobs, int K, bool up, int waves, bool codes, hipStream_t s) {
  // one launch per table of jobs; the ticket counter of a table lives in its
  // first job's sync words (the zero kernel cleared it).  Costs from Census
  // code records exist for K = 8 and 16 (the layouts with code records).
  codes = codes && (K == 8 || K == 16);
  bool pad = false;
  int maxd = 1;
  for (auto &j : jobs) {
    pad |= j.D != j.Dp;
    maxd = std::max(maxd, j.D);
    j.nstripes = (j.W + 4 * waves - 1) / (4 * waves);
  }
  const size_t lds = stripe_lds(K, maxd, waves, up, codes);
  for_each_table(
      jobs, [](const StripeJob &j) { return (long)j.nstripes; },
      [&](const JobTable<StripeJob> &t, int blocks) {
        switch (K) {
          case 4: launch_k<4, false>(t, blocks, up, waves, pad, lds, s); break;
          case 8:
            if (codes) launch_k<8, true>(t, blocks, up, waves, pad, lds, s);
            else launch_k<8, false>(t, blocks, up, waves, pad, lds, s);
            break;
          case 12: launch_k<12, false>(t, blocks, up, waves, pad, lds, s); break;
          default:
            if (codes) launch_k<16, true>(t, blocks, up, waves, pad, lds, s);
            else launch_k<16, false>(t, blocks, up, waves, pad, lds, s);
            break;
        }
      });
}

}  // namespace sgmk
