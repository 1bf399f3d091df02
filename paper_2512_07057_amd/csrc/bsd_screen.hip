// Sparse screen of the first two iterations of the initial BP run
// (Appendix A, eqs. (1)-(4) and the stopping rule at t = 1 and t = 2), one
// wavefront per shot.
//
// Iteration 1.  From E(0) = Lambda with every Lambda_j > 0 every sign in
// eq. (1) except (-1)^{s_i} is +1, so at t = 1 detector i sends
// x_i = alpha * (least |Lambda| of its row) to every neighbour but the one
// holding that least, which gets y_i = alpha * (second least); both are
// clamped to the message bound and both carry the sign (-1)^{s_i}.  A column
// none of whose detectors flipped sums positive terms onto a positive prior
// and decides e_j = 0 (eq. (4)).  The columns of flipped detectors are
// summed here in the dense variable phase's order -- Lambda_j, then the
// messages in ascending row order, in single precision -- so every decision
// equals the dense decoder's.
//
// Iteration 2.  E(1) (eq. (2)) can be negative only on the columns of
// flipped detectors.  Eq. (1) at t = 2 sends a negative message only from a
// row that flipped or that receives a negative E(1): the set S2.  Every
// column outside the neighbourhood of S2 receives non-negative messages and
// decides 0.  For a column next to S2 the messages of S2 rows are formed
// exactly (least and second least |E(1)| of the row, sign parity); the
// message of any other row is non-negative and at least alpha * min(least
// zero-syndrome E(1) of the row, least non-negative E(1) on the shot's
// changed columns).  Single-precision addition and multiplication are
// monotone, so the posterior summed in the dense order with those lower
// bounds is at most the exact one: when it is positive the column decides
// 0.  The few columns where it is not (in practice the columns that decide
// 1) get exact messages from full scans of their remaining rows.
//
// When H e-hat equals the syndrome after iteration 1 or 2 the shot is
// finished; otherwise (or when one of the lists below overflows) it is
// appended to the list that the dense persistent decoder takes its shots
// from.
//
// A workgroup keeps the per-row table (x, y, the column of the least
// |Lambda|, the least zero-syndrome E(1)) and the row pointers in LDS for
// the whole launch; each wave holds one shot's bit-vectors, row lists and
// (row, column) pair lists.  Per shot the global reads are its syndrome
// (prefetched during the previous shot) and, per (row, column) pair, the
// column, its prior and its rows.
#include <hip/hip_runtime.h>

#include "bsd_internal.h"

namespace bsd {

namespace {

constexpr int AGENT = __HIP_MEMORY_SCOPE_AGENT;
constexpr int kWaves = kScreenBlock / 64;
constexpr int kSynRegs = 4;  // 8-byte syndrome loads per lane: m <= 2048
#ifndef BSD_SCREEN_UNROLL
#define BSD_SCREEN_UNROLL 4
#endif
#ifndef BSD_SCREEN_MIN_WAVES
#define BSD_SCREEN_MIN_WAVES 4
#endif
constexpr int kUnroll = BSD_SCREEN_UNROLL;   // pairs per lane in flight at t = 1
#ifndef BSD_SCREEN_UNROLL2
#define BSD_SCREEN_UNROLL2 2
#endif
constexpr int kUnroll2 = BSD_SCREEN_UNROLL2; // at t = 2
constexpr int kMaxRows = kScreenMaxFlipped;  // rows of a pair list (flipped rows, S2)
constexpr int kMaxX = 32;                    // rows scanned for exact decisions at t = 2
constexpr int kMaxExact = 32;                // columns decided by exact messages at t = 2
constexpr int kNone = 0xFFFF;                // absent row slot

struct WaveLds {
  uint32_t sbits[64];                  // s by row (m <= 2048)
  uint32_t rbits[64];                  // s + H e-hat
  uint32_t s2bits[64];                 // rows of S2
  uint32_t xbits[64];                  // S2 rows that did not flip; later rows to scan
  int32_t cst[kMaxRows];               // first CSR position of each listed row
  int32_t coff[kMaxRows];              // index of its first (row, column) pair
  uint16_t rows[kMaxRows];             // listed rows, ascending: flipped rows, then S2
  uint16_t xrows[kMaxX];               // S2 rows that did not flip; later rows to scan
  uint16_t fpre[64];                   // flipped rows in earlier words
  uint16_t s2pre[64];                  // S2 rows in earlier words
  uint16_t xpre[64];                   // rows of xbits in earlier words
  uint32_t rm1[kMaxRows + kMaxX];      // per scanned row (S2, then the others): least |E(1)|,
  uint32_t rm2[kMaxRows + kMaxX];      //   second least,
  uint32_t rpar[kMaxRows + kMaxX];     //   s_i xor the parity of negative E(1)
  int32_t xpos[kMaxExact];             // a CSR position of each column decided exactly
  uint8_t cmap[kScreenMaxCand];        // listed row of each (row, column) pair
  int32_t set[kScreenMaxSet];          // columns with e-hat_j = 1
  int32_t nset;
  int32_t nexact;
  int32_t pad[2];
};

__host__ __device__ constexpr size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// Orders this wave's LDS accesses across lanes (the LDS serves a wave's
// instructions in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t bit_of(const uint32_t* bits, int r) {
  return (bits[r >> 5] >> (r & 31)) & 1u;
}

// Place of row r among the rows set in `bits` (`pre`: set bits in earlier words).
__device__ __forceinline__ int rank_of(const uint32_t* bits, const uint16_t* pre, int r) {
  return (int)pre[r >> 5] + __builtin_popcount(bits[r >> 5] & ((1u << (r & 31)) - 1u));
}

__device__ __forceinline__ int row_at(const uint4& rq, int e) {
  const uint32_t w = e < 2 ? rq.x : e < 4 ? rq.y : e < 6 ? rq.z : rq.w;
  return (int)((w >> (16 * (e & 1))) & 0xFFFFu);
}

// Exclusive prefix sum over the wave and the total.
__device__ __forceinline__ int wave_excl_scan(int v, int lane, int* total) {
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  *total = __shfl(x, 63, 64);
  return x - v;
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ void load_syn_regs(const ScreenArgs& a, long long shot, int lane,
                                              uint2 (&v)[kSynRegs]) {
  const uint2* s8 = reinterpret_cast<const uint2*>(a.syn + shot * a.m);
#pragma unroll
  for (int u = 0; u < kSynRegs; ++u) {
    const int d = lane + 64 * u;
    v[u] = d < (a.m >> 3) ? s8[d] : make_uint2(0u, 0u);
  }
}

// Syndrome bits into LDS, from registers (8-byte rows) or byte loads;
// returns nonzero if a byte is neither 0 nor 1.
__device__ __forceinline__ uint32_t syndrome_bits(const ScreenArgs& a, long long shot,
                                                  const uint2 (&v)[kSynRegs], WaveLds& W,
                                                  int lane) {
  uint32_t bad = 0;
  W.sbits[lane] = 0u;
  wave_sync();
  if (a.syn8) {
    uint8_t* sb = reinterpret_cast<uint8_t*>(W.sbits);
#pragma unroll
    for (int u = 0; u < kSynRegs; ++u) {
      const int d = lane + 64 * u;
      if (d < (a.m >> 3)) {
        const uint32_t x = v[u].x, y = v[u].y;
        bad |= (x | y) & 0xFEFEFEFEu;
        const uint32_t lo = (x & 1u) | ((x >> 7) & 2u) | ((x >> 14) & 4u) | ((x >> 21) & 8u);
        const uint32_t hi = (y & 1u) | ((y >> 7) & 2u) | ((y >> 14) & 4u) | ((y >> 21) & 8u);
        sb[d] = (uint8_t)(lo | (hi << 4));
      }
    }
  } else {
    const uint8_t* s = a.syn + shot * a.m;
    for (int r = lane; r < a.m; r += 64) {
      const uint32_t b = s[r];
      bad |= b & 0xFEu;
      if (b & 1u) atomicOr(&W.sbits[r >> 5], 1u << (r & 31));
    }
  }
  wave_sync();
  return bad;
}

// The rows set in a row bit-vector, ascending, into `out` (at most `cap`),
// and each word's count of set rows in earlier words into `pre`; returns
// how many are set.
__device__ __forceinline__ int list_rows(const uint32_t* bits, int words, uint16_t* out, int cap,
                                         uint16_t* pre, int lane) {
  const uint32_t word = lane < words ? bits[lane] : 0u;
  int total;
  const int off = wave_excl_scan(__builtin_popcount(word), lane, &total);
  pre[lane] = (uint16_t)off;
  int q = off;
  for (uint32_t b = word; b; b &= b - 1u, ++q)
    if (q < cap) out[q] = (uint16_t)(lane * 32 + __builtin_ctz(b));
  wave_sync();
  return total;
}

// The (row, column) pairs of the listed rows, numbered row by row: CSR start
// and first pair of each row, and the listed row of each pair.  Returns the
// number of pairs, or -1 when they do not fit.
__device__ __forceinline__ int list_pairs(const int32_t* rptr, const uint16_t* rows, int nrows,
                                          WaveLds& W, int lane) {
  int st = 0, dg = 0;
  if (lane < nrows) {
    const int i = rows[lane];
    st = rptr[i];
    dg = rptr[i + 1] - st;
  }
  int np;
  const int coff = wave_excl_scan(dg, lane, &np);
  if (np > kScreenMaxCand) return -1;
  if (lane < nrows) {
    W.cst[lane] = st;
    W.coff[lane] = coff;
    for (int q = 0; q < dg; ++q) W.cmap[coff + q] = (uint8_t)lane;
  }
  wave_sync();
  return np;
}

// fn(listed row index, row, CSR position, column's rows, (column, Lambda
// bits)) for every pair of the listed rows, U pairs per lane in flight.
template <int U, class Fn>
__device__ __forceinline__ void for_pairs(const ScreenArgs& a, const WaveLds& W,
                                          const uint16_t* rows, int np, int lane, Fn fn) {
  for (int base = 0; base < np; base += 64 * U) {
    uint4 rq[U];
    uint2 jl[U];
    int li[U], pos[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = base + 64 * u + lane;
      li[u] = -1;
      pos[u] = 0;
      if (c < np) {
        li[u] = W.cmap[c];
        pos[u] = W.cst[li[u]] + (c - W.coff[li[u]]);
        rq[u] = a.edge_rows[pos[u]];
        jl[u] = a.edge_col[pos[u]];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (li[u] >= 0) fn(li[u], (int)rows[li[u]], pos[u], rq[u], jl[u]);
  }
}

// Eq. (1) at t = 1 on the edges of column j (rows r[e] ascending, kNone when
// absent): x or y of the row, negative when s_i = 1; 0 on absent slots.
template <int DV>
__device__ __forceinline__ void col_d1(const uint4& rq, int j, const uint4* tab,
                                       const uint32_t* sbits, int (&r)[DV], float (&d)[DV]) {
#pragma unroll
  for (int e = 0; e < DV; ++e) {
    r[e] = row_at(rq, e);
    const bool there = r[e] != kNone;
    const uint4 t = tab[there ? r[e] : 0];
    const uint32_t sb = there ? bit_of(sbits, r[e]) : 0u;
    const float mag = __uint_as_float((int)t.z == j ? t.y : t.x);
    d[e] = there ? (sb ? -mag : mag) : 0.f;
  }
}

// The lowest row of the column's rows that is set in `bits`, or kNone.
template <int DV>
__device__ __forceinline__ int first_in(const uint32_t* bits, const int (&r)[DV]) {
  int first = kNone;
#pragma unroll
  for (int e = DV - 1; e >= 0; --e) first = (r[e] != kNone && bit_of(bits, r[e])) ? r[e] : first;
  return first;
}

// Eq. (2) at t = 1 on edge slot `es` of a column: Lambda_j, then the other
// messages in ascending row order (the prefix before es, then the terms
// after it), clamped to the message bound: the dense variable phase's
// operations (an absent slot adds 0, which changes no sum that starts from a
// positive Lambda_j).
template <int DV>
__device__ __forceinline__ float e1_at(float lam, const float (&d)[DV], int es) {
  float pre = lam;
#pragma unroll
  for (int f = 0; f < DV; ++f) pre = f < es ? pre + d[f] : pre;
  float x = pre;
#pragma unroll
  for (int f = 0; f < DV; ++f) x = f > es ? x + d[f] : x;
  return __builtin_amdgcn_fmed3f(x, -kLlrMax, kLlrMax);
}

template <int DV>
__device__ __forceinline__ void e1_all(float lam, const float (&d)[DV], float (&E)[DV]) {
  float pre = lam;
#pragma unroll
  for (int e = 0; e < DV; ++e) {
    float x = pre;
#pragma unroll
    for (int f = e + 1; f < DV; ++f) x = x + d[f];
    E[e] = __builtin_amdgcn_fmed3f(x, -kLlrMax, kLlrMax);
    pre = pre + d[e];
  }
}

// Eq. (1) at t = 2 on the edge holding v of a scanned row: least (m1) and
// second least (m2) |E(1)| of the row, sign s_i xor the parity of its
// negative E(1) (sp) xor the sign of v; magnitude alpha * m2 on an edge
// holding the least, alpha * m1 elsewhere, clamped -- the dense check
// phase's operations.
__device__ __forceinline__ float d2_exact(float v, uint32_t m1b, uint32_t m2b, uint32_t sp,
                                          float alpha) {
  const float m1 = __uint_as_float(m1b), m2 = __uint_as_float(m2b);
  const float d1 = fminf(alpha * m1, kLlrMax), d2 = fminf(alpha * m2, kLlrMax);
  const float mag = fabsf(v) == m1 ? d2 : d1;
  return ((sp & 1u) ^ (__float_as_uint(v) >> 31)) ? -mag : mag;
}

// Row info of the listed rows, each at `base` + its rank in (ibits, ipre):
// the message bound (the check phase's starting least values) and s_i.
__device__ __forceinline__ void init_row_info(WaveLds& W, const uint16_t* rows, int nrows,
                                              const uint32_t* ibits, const uint16_t* ipre, int base,
                                              int lane) {
  if (lane < nrows) {
    const int r = rows[lane];
    const int q = base + rank_of(ibits, ipre, r);
    W.rm1[q] = W.rm2[q] = __float_as_uint(kLlrMax);
    W.rpar[q] = bit_of(W.sbits, r);
  }
  wave_sync();
}

// One E(1) of a row into its info q.  Each edge of the row takes part once:
// an atomic minimum into rm1 returns the previous least, and the larger of
// the two goes into rm2, so rm2 ends as the least of all values but one copy
// of the row minimum.  Magnitudes compare as unsigned integers.
__device__ __forceinline__ void row_info_add(WaveLds& W, int q, float v) {
  const uint32_t av = __float_as_uint(v) & 0x7FFFFFFFu;
  const uint32_t old = atomicMin(&W.rm1[q], av);
  atomicMin(&W.rm2[q], old > av ? old : av);
  if (__float_as_uint(v) >> 31) atomicXor(&W.rpar[q], 1u);
}

// Least and second least |E(1)| and the sign parity of the listed rows, E(1)
// formed exactly on every edge; info at `base` + rank in (ibits, ipre).
template <int DV>
__device__ __forceinline__ void scan_rows(const ScreenArgs& a, WaveLds& W, const uint4* tab,
                                          const uint16_t* rows, int np, const uint32_t* ibits,
                                          const uint16_t* ipre, int base, int lane) {
  for_pairs<kUnroll2>(a, W, rows, np, lane, [&](int, int i, int, const uint4& rq, const uint2& jl) {
    int r[DV];
    float d[DV];
    col_d1<DV>(rq, (int)jl.x, tab, W.sbits, r, d);
    int es = 0;
#pragma unroll
    for (int e = 0; e < DV; ++e) es = r[e] == i ? e : es;
    row_info_add(W, base + rank_of(ibits, ipre, i), e1_at<DV>(__uint_as_float(jl.y), d, es));
  });
  wave_sync();
}

// Adds column j to e-hat: its detectors join s + H e-hat.
template <int DV>
__device__ __forceinline__ void set_column(WaveLds& W, int j, const int (&r)[DV]) {
  const int q = atomicAdd(&W.nset, 1);
  if (q < kScreenMaxSet) W.set[q] = j;
#pragma unroll
  for (int e = 0; e < DV; ++e)
    if (r[e] != kNone) atomicXor(&W.rbits[r[e] >> 5], 1u << (r[e] & 31));
}

// Eq. (1) at t = 2 on slot e of a column next to S2: exact for S2 rows and
// for scanned rows (rank in `xb` / `xp`, info from index kMaxRows), else the
// lower bound `lb` of the row's message; `exact` is cleared when a bound is used.
template <int DV>
__device__ __forceinline__ float d2_term(const WaveLds& W, const uint4* tab, int r, float v,
                                         float alpha, float gdmin, bool scanned, bool& exact) {
  if (bit_of(W.s2bits, r)) {
    const int q = rank_of(W.s2bits, W.s2pre, r);
    return d2_exact(v, W.rm1[q], W.rm2[q], W.rpar[q], alpha);
  }
  if (scanned) {
    const int q = kMaxRows + rank_of(W.xbits, W.xpre, r);
    return d2_exact(v, W.rm1[q], W.rm2[q], W.rpar[q], alpha);
  }
  exact = false;
  return fminf(alpha * fminf(__uint_as_float(tab[r].w), gdmin), kLlrMax);
}

// Iteration 2 of a shot whose iteration 1 did not converge (W.rows holds its
// `nflip` flipped rows and W.cmap / cst / coff their `ncand` pairs).  Leaves
// e-hat(2) in W.set and s + H e-hat(2) in W.rbits; returns false when a list
// overflowed (the shot then goes to the dense decoder).
template <int DV>
__device__ bool iteration2(const ScreenArgs& a, WaveLds& W, const uint4* tab, const int32_t* rptr,
                           int nflip, int ncand, int lane) {
  const int words = a.words_m;
  const float alpha = a.alpha2;
  // E(1) on every edge of the columns of flipped detectors.  Rows receiving
  // a negative one join S2 (with the flipped rows); the least non-negative
  // one bounds the E(1) that rows outside S2 receive from these columns.
  // These are all the edges of the flipped rows, whose row info is formed
  // here (at their rank among the flipped rows).
  W.s2bits[lane] = W.sbits[lane];
  init_row_info(W, W.rows, nflip, W.sbits, W.fpre, 0, lane);
  float gmin = kLlrMax;
  for_pairs<kUnroll2>(a, W, W.rows, ncand, lane, [&](int, int i, int, const uint4& rq, const uint2& jl) {
    int r[DV];
    float d[DV], E[DV];
    col_d1<DV>(rq, (int)jl.x, tab, W.sbits, r, d);
    if (first_in<DV>(W.sbits, r) != i) return;  // the column's lowest flipped row takes it
    e1_all<DV>(__uint_as_float(jl.y), d, E);
#pragma unroll
    for (int e = 0; e < DV; ++e) {
      if (r[e] == kNone) continue;
      if (__float_as_uint(E[e]) >> 31)
        atomicOr(&W.s2bits[r[e] >> 5], 1u << (r[e] & 31));
      else
        gmin = fminf(gmin, E[e]);
      if (bit_of(W.sbits, r[e])) row_info_add(W, rank_of(W.sbits, W.fpre, r[e]), E[e]);
    }
  });
  wave_sync();
  const float gdmin = wave_min(gmin);
  // S2, ascending; the flipped rows' info moves to their rank in S2.
  int frow = 0;
  uint32_t fm1 = 0u, fm2 = 0u, fpar = 0u;
  if (lane < nflip) {
    frow = W.rows[lane];
    fm1 = W.rm1[lane];
    fm2 = W.rm2[lane];
    fpar = W.rpar[lane];
  }
  wave_sync();
  const int ns2 = list_rows(W.s2bits, words, W.rows, kMaxRows, W.s2pre, lane);
  if (ns2 > kMaxRows) return false;
  if (lane < nflip) {
    const int q = rank_of(W.s2bits, W.s2pre, frow);
    W.rm1[q] = fm1;
    W.rm2[q] = fm2;
    W.rpar[q] = fpar;
  }
  // The S2 rows that did not flip get their info from scans of their edges.
  W.xbits[lane] = W.s2bits[lane] & ~W.sbits[lane];
  wave_sync();
  const int nn = list_rows(W.xbits, words, W.xrows, kMaxX, W.xpre, lane);
  if (nn > kMaxX) return false;
  init_row_info(W, W.xrows, nn, W.s2bits, W.s2pre, 0, lane);
  const int npn = list_pairs(rptr, W.xrows, nn, W, lane);
  if (npn < 0) return false;
  scan_rows<DV>(a, W, tab, W.xrows, npn, W.s2bits, W.s2pre, 0, lane);
  const int np = list_pairs(rptr, W.rows, ns2, W, lane);
  if (np < 0) return false;

  // Posteriors (eq. (3)) of the columns next to S2, each taken by its lowest
  // S2 row.  A column whose bounded posterior is not positive and that used
  // a bound is listed, and its rows outside S2 are marked for a scan.
  W.rbits[lane] = W.sbits[lane];
  W.xbits[lane] = 0u;
  if (lane == 0) {
    W.nset = 0;
    W.nexact = 0;
  }
  wave_sync();
  for_pairs<kUnroll2>(a, W, W.rows, np, lane, [&](int, int i, int pos, const uint4& rq, const uint2& jl) {
    int r[DV];
    float d[DV], E[DV];
    const int j = (int)jl.x;
    col_d1<DV>(rq, j, tab, W.sbits, r, d);
    if (first_in<DV>(W.s2bits, r) != i) return;
    const float lam = __uint_as_float(jl.y);
    e1_all<DV>(lam, d, E);
    float post = lam;
    bool exact = true;
#pragma unroll
    for (int e = 0; e < DV; ++e)
      if (r[e] != kNone) post = post + d2_term<DV>(W, tab, r[e], E[e], alpha, gdmin, false, exact);
    if (!(post <= 0.f)) return;  // e-hat_j = 0 (eq. (4))
    if (exact) {
      set_column<DV>(W, j, r);
      return;
    }
    const int q = atomicAdd(&W.nexact, 1);
    if (q < kMaxExact) W.xpos[q] = pos;
#pragma unroll
    for (int e = 0; e < DV; ++e)
      if (r[e] != kNone && !bit_of(W.s2bits, r[e]))
        atomicOr(&W.xbits[r[e] >> 5], 1u << (r[e] & 31));
  });
  wave_sync();
  const int nexact = W.nexact;
  if (nexact == 0) return true;
  if (nexact > kMaxExact) return false;

  // Exact messages for the listed columns: scan their rows outside S2.
  const int nx = list_rows(W.xbits, words, W.xrows, kMaxX, W.xpre, lane);
  if (nx > kMaxX) return false;
  const int npx = list_pairs(rptr, W.xrows, nx, W, lane);
  if (npx < 0) return false;
  init_row_info(W, W.xrows, nx, W.xbits, W.xpre, kMaxRows, lane);
  scan_rows<DV>(a, W, tab, W.xrows, npx, W.xbits, W.xpre, kMaxRows, lane);
  if (lane < nexact) {
    const int pos = W.xpos[lane];
    const uint4 rq = a.edge_rows[pos];
    const uint2 jl = a.edge_col[pos];
    int r[DV];
    float d[DV], E[DV];
    const int j = (int)jl.x;
    col_d1<DV>(rq, j, tab, W.sbits, r, d);
    const float lam = __uint_as_float(jl.y);
    e1_all<DV>(lam, d, E);
    float post = lam;
    bool exact = true;
#pragma unroll
    for (int e = 0; e < DV; ++e)
      if (r[e] != kNone) post = post + d2_term<DV>(W, tab, r[e], E[e], alpha, gdmin, true, exact);
    if (post <= 0.f) set_column<DV>(W, j, r);
  }
  wave_sync();
  return true;
}

template <int V>
__device__ __forceinline__ void write_corrections(const ScreenArgs& a, uint8_t* row,
                                                  const WaveLds& W, int nset, int lane) {
  const int nchunk = a.n / V;
  for (int c = lane; c < nchunk; c += 64) {
    if constexpr (V == 16) {
      uint32_t w[4] = {0u, 0u, 0u, 0u};
      for (int q = 0; q < nset; ++q) {
        const int j = W.set[q];
        if ((j >> 4) == c) w[(j >> 2) & 3] |= 1u << (8 * (j & 3));
      }
      reinterpret_cast<uint4*>(row)[c] = make_uint4(w[0], w[1], w[2], w[3]);
    } else if constexpr (V == 4) {
      uint32_t w = 0u;
      for (int q = 0; q < nset; ++q) {
        const int j = W.set[q];
        if ((j >> 2) == c) w |= 1u << (8 * (j & 3));
      }
      reinterpret_cast<uint32_t*>(row)[c] = w;
    } else {
      uint32_t b = 0u;
      for (int q = 0; q < nset; ++q) b |= W.set[q] == c ? 1u : 0u;
      row[c] = (uint8_t)b;
    }
  }
}

// V: bytes per correction store; DV: largest column degree rounded up to
// an even number.
template <int V, int DV>
__global__ void __launch_bounds__(kScreenBlock, BSD_SCREEN_MIN_WAVES) k_screen(ScreenArgs a) {
  extern __shared__ __align__(16) char sm[];
  uint4* tab = reinterpret_cast<uint4*>(sm);
  int32_t* rptr = reinterpret_cast<int32_t*>(sm + 16 * (size_t)a.m);
  WaveLds* wl = reinterpret_cast<WaveLds*>(sm + 16 * (size_t)a.m + align16(4 * (size_t)(a.m + 1)));
  for (int i = threadIdx.x; i < a.m; i += kScreenBlock) tab[i] = a.row_tab[i];
  for (int i = threadIdx.x; i <= a.m; i += kScreenBlock) rptr[i] = a.row_ptr[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  WaveLds& W = wl[wv];
  // Shots below `nstatic` go to the waves in turn (wave w takes w, w +
  // nwaves, ...); the rest are claimed one at a time from a counter, so that
  // waves that drew costly shots (iteration 2) take fewer of the rest.  A
  // claim is issued one shot ahead and read one shot later, so no wave waits
  // on it; the syndrome of the next shot is loaded during the current one.
  const long long nwaves = (long long)gridDim.x * kWaves;
  const long long nstatic = (a.shots * 3 / 4) / nwaves * nwaves;
  uint32_t done = 0, done2 = 0, err = 0;
  auto claim = [&]() -> unsigned long long {  // lane 0's result only
    return lane == 0 ? __hip_atomic_fetch_add(&a.st->screen_next, 1ull, __ATOMIC_RELAXED, AGENT)
                     : 0ull;
  };
  auto bcast = [&](unsigned long long v) -> long long {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, 0, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), 0, 64);
    return nstatic + (long long)(((unsigned long long)hi << 32) | lo);
  };
  const long long w0 = (long long)blockIdx.x * kWaves + wv;
  long long shot = w0 < nstatic ? w0 : bcast(claim());
  long long nxt = shot + nwaves < nstatic ? shot + nwaves : bcast(claim());
  uint2 sv[kSynRegs];
  if (a.syn8 && shot < a.shots) load_syn_regs(a, shot, lane, sv);
  for (; shot < a.shots;) {
    const uint32_t t0 = a.lat ? (uint32_t)wall_clock64() : 0u;
    err |= syndrome_bits(a, shot, sv, W, lane);
    if (a.syn8 && nxt < a.shots) load_syn_regs(a, nxt, lane, sv);
    // the shot after nxt: static, or a claim read at the end of this one
    const bool dyn = !(nxt + nwaves < nstatic) && nxt < a.shots;
    const unsigned long long pend = dyn ? claim() : 0ull;
    // Flipped detectors, ascending, and their (row, column) pairs.
    const int nflip = list_rows(W.sbits, a.words_m, W.rows, kMaxRows, W.fpre, lane);
    W.rbits[lane] = W.sbits[lane];
    if (lane == 0) W.nset = 0;
    wave_sync();
    bool ok = nflip <= kMaxRows;
    int ncand = 0;
    if (ok) {
      ncand = list_pairs(rptr, W.rows, nflip, W, lane);
      ok = ncand >= 0;
    }
    if (ok) {
      // Eq. (3) at t = 1: Lambda_j, then the messages of the rows in
      // ascending order (absent slots add nothing).  The column is kept only
      // by its lowest flipped detector, so that it counts once.
      for_pairs<kUnroll>(a, W, W.rows, ncand, lane, [&](int, int i, int, const uint4& rq, const uint2& jl) {
        int r[DV];
        float d[DV];
        const int j = (int)jl.x;
        col_d1<DV>(rq, j, tab, W.sbits, r, d);
        if (first_in<DV>(W.sbits, r) != i) return;
        float post = __uint_as_float(jl.y);
#pragma unroll
        for (int e = 0; e < DV; ++e)
          if (r[e] != kNone) post = post + d[e];
        if (post <= 0.f) set_column<DV>(W, j, r);  // eq. (4): e-hat_j = 1
      });
      wave_sync();
    }
    // Stopping rule: s + H e-hat = 0.
    bool conv = ok && W.nset <= kScreenMaxSet &&
                __ballot(lane < a.words_m && W.rbits[lane] != 0u) == 0ull;
    bool conv2 = false;
    if (ok && !conv && a.t2) {
      conv2 = iteration2<DV>(a, W, tab, rptr, nflip, ncand, lane) && W.nset <= kScreenMaxSet &&
              __ballot(lane < a.words_m && W.rbits[lane] != 0u) == 0ull;
    }
    if (conv || conv2) {
      const int nset = W.nset;
      // (the logical masks are loaded before the stores: a load issued after
      // them would wait for them too)
      const unsigned long long lm = lane < nset ? a.lmask[W.set[lane]] : 0ull;
      write_corrections<V>(a, a.corr + shot * a.n, W, nset, lane);
      uint32_t lo = (uint32_t)lm, hi = (uint32_t)(lm >> 32);
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        lo ^= __shfl_xor(lo, o, 64);
        hi ^= __shfl_xor(hi, o, 64);
      }
      const unsigned long long fl = (unsigned long long)lo | ((unsigned long long)hi << 32);
      if (lane < a.k) a.flips[shot * a.k + lane] = (uint8_t)((fl >> lane) & 1ull);
      if (lane == 0) {
        a.conv[shot] = 1;
        if (conv) ++done;
        else ++done2;
      }
    } else if (lane == 0) {
      const int q = __hip_atomic_fetch_add(&a.st->listed, 1, __ATOMIC_RELAXED, AGENT);
      a.list[q] = (int32_t)shot;
    }
    if (a.lat && lane == 0) a.lat[shot] = (uint32_t)wall_clock64() - t0;
    wave_sync();  // the next shot reuses this wave's LDS
    const long long after = dyn ? bcast(pend) : nxt + nwaves;
    shot = nxt;
    nxt = after;
  }
  if (lane == 0 && (done | done2)) {
    __hip_atomic_fetch_add(&a.st->done, (unsigned long long)(done + done2), __ATOMIC_RELAXED, AGENT);
    __hip_atomic_fetch_add(&a.st->runs, (unsigned long long)(done + done2), __ATOMIC_RELAXED, AGENT);
    __hip_atomic_fetch_add(&a.st->iterations, (unsigned long long)(done + 2 * done2),
                           __ATOMIC_RELAXED, AGENT);
    if (done2) __hip_atomic_fetch_add(&a.st->done2, done2, __ATOMIC_RELAXED, AGENT);
  }
  if (__ballot(err != 0u) && lane == 0) atomicOr(&a.st->error, 1u);
}

}  // namespace

size_t screen_lds_bytes(int m) {
  return 16 * (size_t)m + align16(4 * (size_t)(m + 1)) + kWaves * sizeof(WaveLds);
}

int screen_blocks_per_cu(int m) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_screen<16, 8>, kScreenBlock,
                                                   screen_lds_bytes(m)) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n < 1 ? 1 : n;
}

namespace {
template <int DV>
hipError_t launch_dv(const ScreenArgs& a, int grid, size_t lds, hipStream_t s) {
  switch (a.vec) {
    case 16: hipLaunchKernelGGL((k_screen<16, DV>), dim3(grid), dim3(kScreenBlock), lds, s, a); break;
    case 4: hipLaunchKernelGGL((k_screen<4, DV>), dim3(grid), dim3(kScreenBlock), lds, s, a); break;
    case 1: hipLaunchKernelGGL((k_screen<1, DV>), dim3(grid), dim3(kScreenBlock), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_screen(const ScreenArgs& a, int grid, hipStream_t s) {
  const size_t lds = screen_lds_bytes(a.m);
  switch (a.maxdeg_col) {
    case 1: case 2: return launch_dv<2>(a, grid, lds, s);
    case 3: case 4: return launch_dv<4>(a, grid, lds, s);
    case 5: case 6: return launch_dv<6>(a, grid, lds, s);
    case 7: case 8: return launch_dv<8>(a, grid, lds, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bsd
