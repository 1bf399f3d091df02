// Sparse screen of the first two iterations of the initial BP run
// (Appendix A, eqs. (1)-(4) and the stopping rule at t = 1 and t = 2), one
// wavefront per shot: k_screen12 for both iterations (k_screen1 when only
// iteration 1 is screened).
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
// decides 0.  For a column next to S2 the magnitude of an S2 row's message
// follows from the row's least and second least |E(1)| and the column
// holding the least, and its sign from the parity of the row's negative
// E(1); the message of any other row is non-negative and at least
// alpha * min(least zero-syndrome E(1) of the row, least non-negative E(1)
// on the shot's changed columns).  Single-precision addition and
// multiplication are monotone, so a posterior summed in the dense order with
// lower bounds in place of some terms is at most the exact one: when it is
// positive the column decides 0.  A column is first bounded with every S2
// message taken negative (no E(1) needed), then with the S2 messages exact,
// and the few columns left (in practice the columns that decide 1) get exact
// messages from full scans of their remaining rows.
//
// When H e-hat equals the syndrome after iteration 1 or 2 the shot is
// finished; otherwise (or when one of the lists below overflows) it is
// appended to the list that the dense persistent decoder takes its shots
// from.
//
// A workgroup keeps the row pointers, each row's two iteration-1 message
// magnitudes (x_i, y_i) and for iteration 2 each row's least zero-syndrome
// E(1) in LDS for the whole launch.  Each wave holds one shot's syndrome as
// a byte per row (and for iteration 2 a byte per row naming its entry of
// the row information), bit-vectors for listing rows, row lists and
// (row, column) pair lists.  A column's absent row slots read the entries of
// a row m that are always 0.  Per shot the global reads are its syndrome
// and, per (row, column) pair, two 16-byte records: the column's rows, each
// flagged when the column holds the row's least |Lambda| (it then receives
// y_i), and the column with its prior and logical mask.
#include <hip/hip_runtime.h>

#include "bsd_internal.h"

namespace bsd {

namespace {

constexpr int AGENT = __HIP_MEMORY_SCOPE_AGENT;
constexpr int kWaves1 = kScreenBlock / 64;
constexpr int kWaves2 = kScreen2Block / 64;
constexpr int kSynRegs = 4;  // 8-byte syndrome loads per lane: m <= 2048
#ifndef BSD_SCREEN_UNROLL
#define BSD_SCREEN_UNROLL 4
#endif
#ifndef BSD_SCREEN_UNROLL2
#define BSD_SCREEN_UNROLL2 2
#endif
constexpr int kUnroll = BSD_SCREEN_UNROLL;    // pairs per lane in flight, iteration 1
constexpr int kUnroll2 = BSD_SCREEN_UNROLL2;  // iteration 2
constexpr int kMaxRows = kScreenMaxFlipped;   // rows of a pair list (flipped rows, S2)
constexpr int kMaxX = 32;                     // S2 rows that did not flip; rows scanned for exact decisions
constexpr int kMaxExact = 32;                 // columns decided by exact messages at t = 2
constexpr int kInfo = kMaxRows + kMaxX;       // row info entries: S2 by rank, then scanned rows
constexpr int kMaxHeavy = 64;                 // columns whose t = 2 bound is not positive

// One shot's iteration 1: syndrome and residual bits, the flipped rows and
// their (row, column) pairs, the set decisions.
struct WaveLds1 {
  uint32_t sbits[64];                  // s by row (m <= 2048)
  uint32_t rbits[64];                  // s + H e-hat
  int32_t cst[kMaxRows];               // first CSR position of each listed row
  int32_t coff[kMaxRows];              // index of its first (row, column) pair
  uint16_t rows[kMaxRows];             // listed rows, ascending: flipped rows (then S2)
  uint8_t cmap[kScreenMaxCand];        // listed row of each (row, column) pair
  int32_t set[kScreenMaxSet];          // columns with e-hat_j = 1
  int32_t nset;
  int32_t nexact;
  uint32_t flw[2];                     // A e-hat: logical masks of the set columns, xor-ed
  int32_t hpos[kMaxHeavy];             // queued columns (CSR positions) for a full evaluation
  int32_t nheavy;
};

// Iteration 2 adds S2, the rows to scan and per-row message information.
struct WaveLds2 : WaveLds1 {
  uint32_t s2bits[64];                 // rows of S2
  uint32_t xbits[64];                  // S2 rows that did not flip; later rows to scan
  uint16_t xrows[kMaxX];
  unsigned long long rk1[kInfo];       // per row: least |E(1)| << 32 | its column,
  uint32_t rm2[kInfo];                 //   second least |E(1)|,
  uint32_t rpar[kInfo];                //   s_i xor the parity of negative E(1)
  int32_t xpos[kMaxExact];             // a CSR position of each column decided exactly
};

// A workgroup's shots for iteration 2 (shot + 1; 0 until written).
constexpr int kWgList = 448;
struct WgList {
  int32_t shot[kWgList];
  int32_t count;     // positions reserved by listers
  int32_t taken;     // positions taken by waves
  int32_t finished;  // waves done with iteration 1
  int32_t pad;
};
static_assert(sizeof(WgList) % 16 == 0, "keeps the byte maps 16-byte aligned");

__host__ __device__ constexpr size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// Per-workgroup tables: the row pointers, each row's x and y of eq. (1) at
// t = 1 (0, 0 for row m), and for iteration 2 the least zero-syndrome E(1)
// of each row (0 for row m).
__host__ __device__ constexpr size_t table_bytes(int m, int which) {
  return align16(4 * (size_t)(m + 1)) + align16(8 * (size_t)(m + 1)) +
         (which == 2 ? align16(4 * (size_t)(m + 1)) : 0);
}

// Per-wave byte maps: the syndrome (rows 0..m), and for iteration 2 the
// row information entry + 1 of each row (0: none).
__host__ __device__ constexpr size_t map_bytes(int m) { return align16((size_t)m + 1); }

// Orders this wave's LDS accesses across lanes (the LDS serves a wave's
// instructions in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void set_bit(uint32_t* bits, int r) {
  atomicOr(&bits[r >> 5], 1u << (r & 31));
}

// DPP controls: shift right by n lanes within a row of 16; lane 15 of each
// row to the next row (rows chosen by the row mask); lane 31 to rows 2, 3.
constexpr int kRowShr = 0x110, kRowBcast15 = 0x142, kRowBcast31 = 0x143;

// Exclusive prefix sum over the wave and the total: an inclusive scan within
// each row of 16 lanes by shifts of 1, 2, 4 and 8 (lanes shifted in from
// outside the row add 0), then row 0's total into rows 1 and 3 and rows 0-1's
// total into rows 2 and 3.
__device__ __forceinline__ int wave_excl_scan(int v, int lane, int* total) {
  (void)lane;
  int x = v;
  x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 1, 0xF, 0xF, false);
  x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 2, 0xF, 0xF, false);
  x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 4, 0xF, 0xF, false);
  x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 8, 0xF, 0xF, false);
  x += __builtin_amdgcn_update_dpp(0, x, kRowBcast15, 0xA, 0xF, false);
  x += __builtin_amdgcn_update_dpp(0, x, kRowBcast31, 0xC, 0xF, false);
  *total = __builtin_amdgcn_readlane(x, 63);
  return x - v;
}

// Least value over the wave (lane 63 ends with the least of all lanes; lanes
// shifted in from outside a row, and rows the masks leave out, keep their
// own value).
__device__ __forceinline__ float wave_min(float v) {
  int x = __float_as_int(v);
  x = __float_as_int(fminf(__int_as_float(x), __int_as_float(__builtin_amdgcn_update_dpp(x, x, kRowShr + 1, 0xF, 0xF, false))));
  x = __float_as_int(fminf(__int_as_float(x), __int_as_float(__builtin_amdgcn_update_dpp(x, x, kRowShr + 2, 0xF, 0xF, false))));
  x = __float_as_int(fminf(__int_as_float(x), __int_as_float(__builtin_amdgcn_update_dpp(x, x, kRowShr + 4, 0xF, 0xF, false))));
  x = __float_as_int(fminf(__int_as_float(x), __int_as_float(__builtin_amdgcn_update_dpp(x, x, kRowShr + 8, 0xF, 0xF, false))));
  x = __float_as_int(fminf(__int_as_float(x), __int_as_float(__builtin_amdgcn_update_dpp(x, x, kRowBcast15, 0xA, 0xF, false))));
  x = __float_as_int(fminf(__int_as_float(x), __int_as_float(__builtin_amdgcn_update_dpp(x, x, kRowBcast31, 0xC, 0xF, false))));
  return __int_as_float(__builtin_amdgcn_readlane(x, 63));
}

// A shot's syndrome (m / 8 rows of 8 bytes per lane-slot), read once: non-temporal.
__device__ __forceinline__ void load_syn_regs(const ScreenArgs& a, long long shot, int lane,
                                              uint2 (&v)[kSynRegs]) {
  const uint2* s8 = reinterpret_cast<const uint2*>(a.syn + shot * a.m);
#pragma unroll
  for (int u = 0; u < kSynRegs; ++u) {
    const int d = lane + 64 * u;
    if (d < (a.m >> 3)) {
      const unsigned long long x = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(s8) + d);
      v[u] = make_uint2((uint32_t)x, (uint32_t)(x >> 32));
    } else {
      v[u] = make_uint2(0u, 0u);
    }
  }
}

// The syndrome into LDS: bits (W.sbits) and bytes (smap, rows 0..m-1), from
// registers (8-byte rows) or byte loads; returns nonzero if a byte is
// neither 0 nor 1.
__device__ __forceinline__ uint32_t syndrome_in(const ScreenArgs& a, long long shot,
                                                const uint2 (&v)[kSynRegs], WaveLds1& W,
                                                uint8_t* smap, int lane) {
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
        reinterpret_cast<uint2*>(smap)[d] = make_uint2(x & 0x01010101u, y & 0x01010101u);
      }
    }
  } else {
    const uint8_t* s = a.syn + shot * a.m;
    for (int r = lane; r < a.m; r += 64) {
      const uint32_t b = s[r];
      bad |= b & 0xFEu;
      smap[r] = (uint8_t)(b & 1u);
      if (b & 1u) set_bit(W.sbits, r);
    }
  }
  wave_sync();
  return bad;
}

// The rows set in a row bit-vector, ascending, into `out` (at most `cap`);
// returns how many are set.
__device__ __forceinline__ int list_rows(const uint32_t* bits, int words, uint16_t* out, int cap,
                                         int lane) {
  const uint32_t word = lane < words ? bits[lane] : 0u;
  int total;
  int q = wave_excl_scan(__builtin_popcount(word), lane, &total);
  for (uint32_t b = word; b; b &= b - 1u, ++q)
    if (q < cap) out[q] = (uint16_t)(lane * 32 + __builtin_ctz(b));
  wave_sync();
  return total;
}

// The (row, column) pairs of the listed rows, numbered row by row: CSR start
// and first pair of each row, and the listed row of each pair.  Returns the
// number of pairs, or -1 when they do not fit.
__device__ __forceinline__ int list_pairs(const int32_t* rptr, const uint16_t* rows, int nrows,
                                          WaveLds1& W, int lane) {
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
// bits, logical mask); zeros unless J) for every pair of the listed rows,
// U pairs per lane in flight.
template <int U, bool J = true, class Fn>
__device__ __forceinline__ void for_pairs(const ScreenArgs& a, const WaveLds1& W,
                                          const uint16_t* rows, int np, int lane, Fn fn) {
  for (int base = 0; base < np; base += 64 * U) {
    // Lanes past the last pair read the last pair's data and skip it: every
    // load is unconditional, so that all of them issue together.
    uint4 rq[U];
    uint4 jl[U];
    int li[U], pos[U], c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      c[u] = base + 64 * u + lane;
      li[u] = W.cmap[min(c[u], np - 1)];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) pos[u] = W.cst[li[u]] + (min(c[u], np - 1) - W.coff[li[u]]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      rq[u] = a.edge_rows[pos[u]];
      jl[u] = J ? a.edge_col[pos[u]] : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (c[u] < np) fn(li[u], (int)rows[li[u]], pos[u], rq[u], jl[u]);
  }
}

// The column's rows in slot order (ascending); absent slots give row m.
template <int DV>
__device__ __forceinline__ void col_rows(const uint4& rq, int m, int (&r)[DV]) {
#pragma unroll
  for (int e = 0; e < DV; ++e) {
    const uint32_t w = e < 2 ? rq.x : e < 4 ? rq.y : e < 6 ? rq.z : rq.w;
    r[e] = min((int)((w >> (16 * (e & 1))) & 0xFFFu), m);
  }
}

// A byte per slot from a row map.
template <int DV>
__device__ __forceinline__ void col_map(const uint8_t* map, const int (&r)[DV], uint32_t (&b)[DV]) {
#pragma unroll
  for (int e = 0; e < DV; ++e) b[e] = map[r[e]];
}

// The lowest row of the slots whose flag is set, or -1.
template <int DV>
__device__ __forceinline__ int first_set(const int (&r)[DV], const bool (&f)[DV]) {
  int first = -1;
#pragma unroll
  for (int e = DV - 1; e >= 0; --e) first = f[e] ? r[e] : first;
  return first;
}

// Eq. (1) at t = 1 on the edges of a column: the magnitude of the row's
// message (xy[row].x, or .y when the slot's flag says the column holds the
// row's least |Lambda|; row m gives 0 on absent slots), negative when
// s_i = 1.
template <int DV>
__device__ __forceinline__ void col_d1(const float2* xy, const uint4& rq, const int (&r)[DV],
                                       const uint32_t (&sb)[DV], float (&d)[DV]) {
#pragma unroll
  for (int e = 0; e < DV; ++e) {
    const uint32_t w = e < 2 ? rq.x : e < 4 ? rq.y : e < 6 ? rq.z : rq.w;
    const float2 v = xy[r[e]];
    const float mag = (w >> (16 * (e & 1) + 15)) & 1u ? v.y : v.x;
    d[e] = sb[e] ? -mag : mag;
  }
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

// Adds column j (record jl) to e-hat: its detectors join s + H e-hat and
// its logical mask joins A e-hat.
template <int DV>
__device__ __forceinline__ void set_column(WaveLds1& W, const uint4& jl, const int (&r)[DV], int m) {
  const int q = atomicAdd(&W.nset, 1);
  if (q < kScreenMaxSet) W.set[q] = (int)jl.x;
  atomicXor(&W.flw[0], jl.z);
  atomicXor(&W.flw[1], jl.w);
#pragma unroll
  for (int e = 0; e < DV; ++e)
    if (r[e] < m) atomicXor(&W.rbits[r[e] >> 5], 1u << (r[e] & 31));
}

// Eqs. (3)-(4) at t = 1 for the columns of the flipped rows (W.rows, their
// `ncand` pairs in W.cmap / cst / coff): Lambda_j, then the messages of the
// column's rows in ascending order (absent slots add 0), summed in single
// precision as the dense variable phase does; each column is decided by its
// lowest flipped row only, so that it counts once.  When iteration 1's
// alpha is at most 1 a first pass reads only the columns' rows: a column
// with one flipped row whose record says that one detector cannot decide it
// has a positive posterior, and the others are queued and summed in full,
// one per lane (once kMaxHeavy are queued, the others as they are found).
template <int DV>
__device__ __forceinline__ void iteration1(const ScreenArgs& a, WaveLds1& W, const float2* xy,
                                           const uint8_t* smap, int ncand, int lane) {
  const int m = a.m;
  auto decide = [&](const uint4& rq, const uint4& jl, const int (&r)[DV], const uint32_t (&sb)[DV]) {
    float d[DV];
    col_d1<DV>(xy, rq, r, sb, d);
    float post = __uint_as_float(jl.y);
#pragma unroll
    for (int e = 0; e < DV; ++e) post = post + d[e];
    if (post <= 0.f) set_column<DV>(W, jl, r, m);  // eq. (4): e-hat_j = 1
  };
  if (a.single1) {
    if (lane == 0) W.nheavy = 0;
    wave_sync();
    for_pairs<kUnroll, false>(a, W, W.rows, ncand, lane, [&](int, int i, int pos, const uint4& rq, const uint4&) {
      int r[DV];
      uint32_t sb[DV];
      bool fl[DV];
      col_rows<DV>(rq, m, r);
      col_map<DV>(smap, r, sb);
      int nf = 0;
#pragma unroll
      for (int e = 0; e < DV; ++e) {
        fl[e] = sb[e] != 0u;
        nf += fl[e] ? 1 : 0;
      }
      if (first_set<DV>(r, fl) != i) return;
      if (nf < 2 && !((rq.x >> 14) & 1u)) return;
      const int q = atomicAdd(&W.nheavy, 1);
      if (q < kMaxHeavy)
        W.hpos[q] = pos;
      else
        decide(rq, a.edge_col[pos], r, sb);  // (the queue is full)
    });
    wave_sync();
    if (lane < min(W.nheavy, kMaxHeavy)) {
      const int pos = W.hpos[lane];
      const uint4 rq = a.edge_rows[pos];
      const uint4 jl = a.edge_col[pos];
      int r[DV];
      uint32_t sb[DV];
      col_rows<DV>(rq, m, r);
      col_map<DV>(smap, r, sb);
      decide(rq, jl, r, sb);
    }
    wave_sync();
    return;
  }
  for_pairs<kUnroll>(a, W, W.rows, ncand, lane, [&](int, int i, int, const uint4& rq, const uint4& jl) {
    int r[DV];
    uint32_t sb[DV];
    bool fl[DV];
    col_rows<DV>(rq, m, r);
    col_map<DV>(smap, r, sb);
#pragma unroll
    for (int e = 0; e < DV; ++e) fl[e] = sb[e] != 0u;
    if (first_set<DV>(r, fl) == i) decide(rq, jl, r, sb);
  });
  wave_sync();
}

// Row information entry q: the message bound (the check phase's starting
// least values) and s_i.
__device__ __forceinline__ void init_info(WaveLds2& W, int q, uint32_t s) {
  W.rk1[q] = ((unsigned long long)__float_as_uint(kLlrMax) << 32) | 0xFFFFFFFFull;
  W.rm2[q] = __float_as_uint(kLlrMax);
  W.rpar[q] = s;
}

// One E(1) (held by column j) of a row into its information q.  Each edge
// of the row takes part once: an atomic minimum of (|v|, j) into rk1 returns
// the previous least, and the larger magnitude of the two goes into rm2, so
// rm2 ends as the least of all magnitudes but one copy of the row minimum.
// Magnitudes compare as unsigned integers.
__device__ __forceinline__ void row_info_add(WaveLds2& W, int q, float v, int j) {
  const uint32_t av = __float_as_uint(v) & 0x7FFFFFFFu;
  const unsigned long long old = atomicMin(&W.rk1[q], ((unsigned long long)av << 32) | (uint32_t)j);
  const uint32_t oav = (uint32_t)(old >> 32);
  atomicMin(&W.rm2[q], oav > av ? oav : av);
  if (__float_as_uint(v) >> 31) atomicXor(&W.rpar[q], 1u);
}

// Row information of the listed rows (entry imap[row] - 1), E(1) formed
// exactly on every edge of each row.
template <int DV>
__device__ __forceinline__ void scan_rows(const ScreenArgs& a, WaveLds2& W, const float2* xy,
                                          const uint8_t* smap, const uint8_t* imap,
                                          const uint16_t* rows, int np, int lane) {
  for_pairs<kUnroll2>(a, W, rows, np, lane, [&](int, int i, int, const uint4& rq, const uint4& jl) {
    int r[DV];
    uint32_t sb[DV];
    float d[DV];
    col_rows<DV>(rq, a.m, r);
    col_map<DV>(smap, r, sb);
    col_d1<DV>(xy, rq, r, sb, d);
    int es = 0;
#pragma unroll
    for (int e = 0; e < DV; ++e) es = r[e] == i ? e : es;
    row_info_add(W, (int)imap[i] - 1, e1_at<DV>(__uint_as_float(jl.y), d, es), (int)jl.x);
  });
  wave_sync();
}

// Magnitude of eq. (1) at t = 2 that a row with information q sends to
// column j: alpha * second least |E(1)| to the column holding the least,
// alpha * least to the others, clamped.  (When another column ties for the
// least, both are equal.)
__device__ __forceinline__ float d2_mag(const WaveLds2& W, int q, int j, float alpha) {
  const unsigned long long k1 = W.rk1[q];
  const float mm = (int)(uint32_t)k1 == j ? __uint_as_float(W.rm2[q])
                                          : __uint_as_float((uint32_t)(k1 >> 32));
  return fminf(alpha * mm, kLlrMax);
}

// Per slot of a column: the row's information entry (-1 outside S2 and,
// with `scanned`, the scanned rows).
template <int DV>
__device__ __forceinline__ void d2_rows(const uint8_t* imap, const int (&r)[DV], bool scanned,
                                        int (&q)[DV]) {
#pragma unroll
  for (int e = 0; e < DV; ++e) {
    const int v = (int)imap[r[e]] - 1;
    q[e] = (v >= 0 && (scanned || v < kMaxRows)) ? v : -1;
  }
}

// Per slot of a column next to S2 (entries q from d2_rows): the magnitude of
// its t = 2 message to column j (rows with an entry) or a lower bound of it
// (other rows: 0 on absent slots).
template <int DV>
__device__ __forceinline__ void d2_mags(const WaveLds2& W, const float* e1min, const int (&r)[DV],
                                        const int (&q)[DV], int j, float alpha, float gdmin,
                                        float (&mag)[DV]) {
#pragma unroll
  for (int e = 0; e < DV; ++e) {
    const float lb = fminf(alpha * fminf(e1min[r[e]], gdmin), kLlrMax);
    const float mm = d2_mag(W, q[e] >= 0 ? q[e] : 0, j, alpha);
    mag[e] = q[e] >= 0 ? mm : lb;
  }
}

template <int DV>
__device__ __forceinline__ void d2_slots(const WaveLds2& W, const uint8_t* imap, const float* e1min,
                                         const int (&r)[DV], int j, float alpha, float gdmin,
                                         bool scanned, int (&q)[DV], float (&mag)[DV]) {
  d2_rows<DV>(imap, r, scanned, q);
  d2_mags<DV>(W, e1min, r, q, j, alpha, gdmin, mag);
}

// Iteration 2 of a shot whose iteration 1 did not converge (W.rows holds its
// `nflip` flipped rows and W.cmap / cst / coff their `ncand` pairs; imap is
// all 0).  Leaves e-hat(2) in W.set and s + H e-hat(2) in W.rbits; returns
// false when a list overflowed (the shot then goes to the dense decoder).
template <int DV>
__device__ bool iteration2(const ScreenArgs& a, WaveLds2& W, const float2* xy, const uint8_t* smap,
                           uint8_t* imap, const float* e1min, const int32_t* rptr, int nflip,
                           int ncand, int lane) {
  const int words = a.words_m, m = a.m;
  const float alpha = a.alpha2;
  // E(1) on every edge of the columns of flipped detectors.  Rows receiving
  // a negative one join S2 (with the flipped rows); the least non-negative
  // one bounds the E(1) that rows outside S2 receive from these columns.
  // These are all the edges of the flipped rows, whose row information is
  // formed here (entry: rank among the flipped rows).
  W.s2bits[lane] = W.sbits[lane];
  if (lane < nflip) {
    imap[W.rows[lane]] = (uint8_t)(lane + 1);
    init_info(W, lane, 1u);
  }
  wave_sync();
  float gmin = kLlrMax;
  for_pairs<kUnroll2>(a, W, W.rows, ncand, lane, [&](int, int i, int, const uint4& rq, const uint4& jl) {
    int r[DV];
    uint32_t sb[DV];
    bool fl[DV];
    float d[DV], E[DV];
    const int j = (int)jl.x;
    col_rows<DV>(rq, m, r);
    col_map<DV>(smap, r, sb);
#pragma unroll
    for (int e = 0; e < DV; ++e) fl[e] = sb[e] != 0u;
    if (first_set<DV>(r, fl) != i) return;  // the column's lowest flipped row takes it
    col_d1<DV>(xy, rq, r, sb, d);
    e1_all<DV>(__uint_as_float(jl.y), d, E);
#pragma unroll
    for (int e = 0; e < DV; ++e) {
      if (r[e] >= m) continue;
      if (__float_as_uint(E[e]) >> 31)
        set_bit(W.s2bits, r[e]);
      else
        gmin = fminf(gmin, E[e]);
      if (sb[e]) row_info_add(W, (int)imap[r[e]] - 1, E[e], j);
    }
  });
  wave_sync();
  const float gdmin = wave_min(gmin);
  // S2, ascending; the flipped rows' information moves to their rank in S2.
  int frow = 0;
  unsigned long long fk1 = 0ull;
  uint32_t fm2 = 0u, fpar = 0u;
  if (lane < nflip) {
    frow = W.rows[lane];
    fk1 = W.rk1[lane];
    fm2 = W.rm2[lane];
    fpar = W.rpar[lane];
  }
  wave_sync();
  const int ns2 = list_rows(W.s2bits, words, W.rows, kMaxRows, lane);
  if (ns2 > kMaxRows) return false;
  if (lane < ns2) imap[W.rows[lane]] = (uint8_t)(lane + 1);
  wave_sync();
  if (lane < nflip) {
    const int q = (int)imap[frow] - 1;
    W.rk1[q] = fk1;
    W.rm2[q] = fm2;
    W.rpar[q] = fpar;
  }
  // The S2 rows that did not flip get theirs from scans of their edges.
  W.xbits[lane] = W.s2bits[lane] & ~W.sbits[lane];
  wave_sync();
  const int nn = list_rows(W.xbits, words, W.xrows, kMaxX, lane);
  if (nn > kMaxX) return false;
  if (lane < nn) init_info(W, (int)imap[W.xrows[lane]] - 1, 0u);
  const int npn = list_pairs(rptr, W.xrows, nn, W, lane);
  if (npn < 0) return false;
  scan_rows<DV>(a, W, xy, smap, imap, W.xrows, npn, lane);
  const int np = list_pairs(rptr, W.rows, ns2, W, lane);
  if (np < 0) return false;

  // Posteriors (eq. (3)) of the columns next to S2, each taken by its lowest
  // S2 row: first with every S2 message taken negative; the columns this
  // leaves open are queued and then taken one per lane with the S2 messages
  // exact (so that the pass over all pairs stays short and uniform; once
  // kMaxHeavy are queued the pass takes the others as it finds them).  A
  // column whose bounded posterior is still not positive and that used a
  // bound for a row outside S2 is listed, and those rows are marked for a
  // scan.
  W.rbits[lane] = W.sbits[lane];
  W.xbits[lane] = 0u;
  if (lane == 0) {
    W.nset = 0;
    W.nexact = 0;
    W.nheavy = 0;
    W.flw[0] = W.flw[1] = 0u;
  }
  wave_sync();
  // A column left open by the bound: the S2 messages exact (the sign of each
  // from its row's parity and the sign of E(1) on the edge).
  auto open_column = [&](int pos, const uint4& rq, const uint4& jl, const int (&r)[DV],
                         const int (&q)[DV], const float (&mag)[DV]) {
    uint32_t sb[DV];
    float d[DV], E[DV];
    const float lam = __uint_as_float(jl.y);
    col_map<DV>(smap, r, sb);
    col_d1<DV>(xy, rq, r, sb, d);
    e1_all<DV>(lam, d, E);
    float post = lam;
    bool exact = true;
#pragma unroll
    for (int e = 0; e < DV; ++e) {
      const bool in2 = q[e] >= 0;
      const bool neg = in2 && ((W.rpar[in2 ? q[e] : 0] & 1u) ^ (__float_as_uint(E[e]) >> 31));
      exact = exact && (in2 || r[e] >= m);
      post = post + (neg ? -mag[e] : mag[e]);
    }
    if (!(post <= 0.f)) return;
    if (exact) {
      set_column<DV>(W, jl, r, m);
      return;
    }
    const int qx = atomicAdd(&W.nexact, 1);
    if (qx < kMaxExact) W.xpos[qx] = pos;
#pragma unroll
    for (int e = 0; e < DV; ++e)
      if (r[e] < m && q[e] < 0) set_bit(W.xbits, r[e]);
  };
  for_pairs<kUnroll2>(a, W, W.rows, np, lane, [&](int, int i, int pos, const uint4& rq, const uint4& jl) {
    int r[DV], q[DV];
    bool in2[DV];
    float mag[DV];
    col_rows<DV>(rq, m, r);
    d2_rows<DV>(imap, r, false, q);
#pragma unroll
    for (int e = 0; e < DV; ++e) in2[e] = q[e] >= 0;
    if (first_set<DV>(r, in2) != i) return;
    d2_mags<DV>(W, e1min, r, q, (int)jl.x, alpha, gdmin, mag);
    float lb = __uint_as_float(jl.y);
#pragma unroll
    for (int e = 0; e < DV; ++e) lb = lb + (in2[e] ? -mag[e] : mag[e]);
    if (lb > 0.f) return;  // e-hat_j = 0 (eq. (4))
    const int qh = atomicAdd(&W.nheavy, 1);
    if (qh < kMaxHeavy)
      W.hpos[qh] = pos;
    else
      open_column(pos, rq, jl, r, q, mag);  // (the queue is full)
  });
  wave_sync();
  if (lane < min(W.nheavy, kMaxHeavy)) {
    const int pos = W.hpos[lane];
    const uint4 rq = a.edge_rows[pos];
    const uint4 jl = a.edge_col[pos];
    int r[DV], q[DV];
    float mag[DV];
    col_rows<DV>(rq, m, r);
    d2_slots<DV>(W, imap, e1min, r, (int)jl.x, alpha, gdmin, false, q, mag);
    open_column(pos, rq, jl, r, q, mag);
  }
  wave_sync();
  const int nexact = W.nexact;
  if (nexact == 0) return true;
  if (nexact > kMaxExact) return false;

  // Exact messages for the listed columns: scan their rows outside S2.
  const int nx = list_rows(W.xbits, words, W.xrows, kMaxX, lane);
  if (nx > kMaxX) return false;
  if (lane < nx) {
    imap[W.xrows[lane]] = (uint8_t)(kMaxRows + lane + 1);
    init_info(W, kMaxRows + lane, 0u);
  }
  const int npx = list_pairs(rptr, W.xrows, nx, W, lane);
  if (npx < 0) return false;
  scan_rows<DV>(a, W, xy, smap, imap, W.xrows, npx, lane);
  if (lane < nexact) {
    const int pos = W.xpos[lane];
    const uint4 rq = a.edge_rows[pos];
    const uint4 jl = a.edge_col[pos];
    int r[DV], q[DV];
    uint32_t sb[DV];
    float d[DV], E[DV], mag[DV];
    const int j = (int)jl.x;
    col_rows<DV>(rq, m, r);
    d2_slots<DV>(W, imap, e1min, r, j, alpha, gdmin, true, q, mag);
    col_map<DV>(smap, r, sb);
    col_d1<DV>(xy, rq, r, sb, d);
    const float lam = __uint_as_float(jl.y);
    e1_all<DV>(lam, d, E);
    float post = lam;
#pragma unroll
    for (int e = 0; e < DV; ++e) {  // (every present slot is in S2 or scanned)
      const bool neg = q[e] >= 0 && ((W.rpar[q[e] >= 0 ? q[e] : 0] & 1u) ^ (__float_as_uint(E[e]) >> 31));
      post = post + (neg ? -mag[e] : mag[e]);
    }
    if (post <= 0.f) set_column<DV>(W, jl, r, m);
  }
  wave_sync();
  return true;
}

// e-hat as bytes, V per store: lane c of each pass of 64 stores writes chunk
// c; one ballot finds the set columns whose chunks fall in the pass.  The
// 16-byte stores are non-temporal: the corrections stream past the L2, which
// keeps the per-pair records that every shot gathers.
// `myj`: the lane's entry of the set, or -1.
template <int V>
__device__ __forceinline__ void write_corrections(const ScreenArgs& a, uint8_t* row, int myj,
                                                  int lane) {
  const int nchunk = a.n / V;
  const int mych = myj >= 0 ? myj / V : -1;
  for (int c0 = 0; c0 < nchunk; c0 += 64) {
    const int c = c0 + lane;
    unsigned long long mk = __ballot(mych >= c0 && mych < c0 + 64);
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    while (mk) {
      const int q = __builtin_ctzll(mk);
      mk &= mk - 1ull;
      const int j = __builtin_amdgcn_readlane(myj, q);
      const uint32_t b = j / V == c ? (V == 1 ? 1u : 1u << (8 * (j & 3))) : 0u;
      const int wi = V == 16 ? (j >> 2) & 3 : 0;  // word of the chunk
#pragma unroll
      for (int u = 0; u < 4; ++u) w[u] |= wi == u ? b : 0u;
    }
    if (c < nchunk) {
      if constexpr (V == 16) {
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        const u32x4 v = {w[0], w[1], w[2], w[3]};
        __builtin_nontemporal_store(v, reinterpret_cast<u32x4*>(row) + c);
      } else if constexpr (V == 4) {
        reinterpret_cast<uint32_t*>(row)[c] = w[0];
      } else {
        row[c] = (uint8_t)(w[0] & 1u);
      }
    }
  }
}

// Outputs of a finished shot from W.set and W.flw: corrections, logical
// flips (A e-hat), converged flag.
template <int V>
__device__ __forceinline__ void write_shot(const ScreenArgs& a, const WaveLds1& W, long long shot,
                                           int lane) {
  const int nset = W.nset;
  const int myj = lane < nset ? W.set[lane] : -1;
  const uint32_t fw = W.flw[lane >= 32 ? 1 : 0];
  write_corrections<V>(a, a.corr + shot * a.n, myj, lane);
  if (lane < a.k) a.flips[shot * a.k + lane] = (uint8_t)((fw >> (lane & 31)) & 1u);
  if (lane == 0) a.conv[shot] = 1;
}

// Outputs of a shot whose syndrome is all zero: from E(0) = Lambda > 0 every
// message at t = 1 is positive, e-hat(1) = 0 satisfies s = 0, and the run
// stops there (the same outputs as the full iteration-1 path).
template <int V>
__device__ __forceinline__ void write_zero_shot(const ScreenArgs& a, long long shot, int lane) {
  write_corrections<V>(a, a.corr + shot * a.n, -1, lane);
  if (lane < a.k) a.flips[shot * a.k + lane] = 0;
  if (lane == 0) a.conv[shot] = 1;
}

// True in every lane when the syndrome held in `v` (8-byte rows) is all zero.
__device__ __forceinline__ bool syndrome_zero(const uint2 (&v)[kSynRegs]) {
  uint32_t any = 0u;
#pragma unroll
  for (int u = 0; u < kSynRegs; ++u) any |= v[u].x | v[u].y;
  return __ballot(any != 0u) == 0ull;
}

// Appends a shot to the dense decoder's list (an atomic store: a decoder
// launched beside the screen may take it at once).  When latencies are
// measured the store has release order, so that the decoder sees the shot's
// latency so far; otherwise nothing written before it is needed there, and a
// release (a write-back of this XCD's L2) is not paid.
__device__ __forceinline__ void list_dense(const ScreenArgs& a, long long shot) {
  const int q = __hip_atomic_fetch_add(&a.st->listed, 1, __ATOMIC_RELAXED, AGENT);
  if (a.lat)
    __hip_atomic_store(&a.list[q], (int32_t)shot, __ATOMIC_RELEASE, AGENT);
  else
    __hip_atomic_store(&a.list[q], (int32_t)shot, __ATOMIC_RELAXED, AGENT);
}


// Flipped rows and their pairs; false when the lists overflow.
__device__ __forceinline__ bool flipped_pairs(const ScreenArgs& a, WaveLds1& W, const int32_t* rptr,
                                              int lane, int* nflip, int* ncand) {
  *nflip = list_rows(W.sbits, a.words_m, W.rows, kMaxRows, lane);
  *ncand = 0;
  if (*nflip > kMaxRows) return false;
  *ncand = list_pairs(rptr, W.rows, *nflip, W, lane);
  return *ncand >= 0;
}

// Iteration 1 only.  V: bytes per correction store; DV: largest column
// degree rounded up to an even number.  Wave w takes shots w, w + nwaves,
// ...; the syndrome of its next shot is loaded during the current one.
template <int V, int DV>
__global__ void __launch_bounds__(kScreenBlock, kScreen1MinWaves) k_screen1(ScreenArgs a) {
  extern __shared__ __align__(16) char sm[];
  const int m = a.m;
  int32_t* rptr = reinterpret_cast<int32_t*>(sm);
  float2* xy = reinterpret_cast<float2*>(sm + align16(4 * (size_t)(m + 1)));
  WaveLds1* wl = reinterpret_cast<WaveLds1*>(sm + table_bytes(m, 1));
  for (int i = threadIdx.x; i <= m; i += kScreenBlock) {
    rptr[i] = a.row_ptr[i];
    xy[i] = a.row_xy[i];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  WaveLds1& W = wl[wv];
  uint8_t* smap = reinterpret_cast<uint8_t*>(sm + table_bytes(m, 1) + align16(kWaves1 * sizeof(WaveLds1))) +
                  wv * map_bytes(m);
  if (lane == 0) smap[m] = 0;  // absent row slots
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(&a.st->screen_begun, 1u, __ATOMIC_RELAXED, AGENT);
  const long long nwaves = (long long)gridDim.x * kWaves1;
  uint32_t done = 0, err = 0;
  long long shot = (long long)blockIdx.x * kWaves1 + wv;
  uint2 sv[kSynRegs];
  if (a.syn8 && shot < a.shots) load_syn_regs(a, shot, lane, sv);
  for (; shot < a.shots; shot += nwaves) {
    const uint32_t t0 = a.lat ? (uint32_t)wall_clock64() : 0u;
    if (a.syn8 && syndrome_zero(sv)) {  // (load_syn_regs zeroes the rows past m)
      if (shot + nwaves < a.shots) load_syn_regs(a, shot + nwaves, lane, sv);
      write_zero_shot<V>(a, shot, lane);
      ++done;
      if (a.lat && lane == 0) a.lat[shot] = (uint32_t)wall_clock64() - t0;
      continue;
    }
    err |= syndrome_in(a, shot, sv, W, smap, lane);
    if (a.syn8 && shot + nwaves < a.shots) load_syn_regs(a, shot + nwaves, lane, sv);
    W.rbits[lane] = W.sbits[lane];
    if (lane == 0) {
      W.nset = 0;
      W.flw[0] = W.flw[1] = 0u;
    }
    int nflip, ncand;
    const bool ok = flipped_pairs(a, W, rptr, lane, &nflip, &ncand);
    if (ok) iteration1<DV>(a, W, xy, smap, ncand, lane);
    // Stopping rule: s + H e-hat = 0.
    const bool conv = ok && W.nset <= kScreenMaxSet &&
                      __ballot(lane < a.words_m && W.rbits[lane] != 0u) == 0ull;
    if (conv) {
      write_shot<V>(a, W, shot, lane);
      ++done;
      if (a.lat && lane == 0) a.lat[shot] = (uint32_t)wall_clock64() - t0;
    } else if (lane == 0) {
      if (a.lat) a.lat[shot] = (uint32_t)wall_clock64() - t0;
      list_dense(a, shot);
    }
    wave_sync();  // the next shot reuses this wave's LDS
  }
  if (lane == 0 && done) {
    __hip_atomic_fetch_add(&a.st->done, (unsigned long long)done, __ATOMIC_RELAXED, AGENT);
    __hip_atomic_fetch_add(&a.st->runs, (unsigned long long)done, __ATOMIC_RELAXED, AGENT);
    __hip_atomic_fetch_add(&a.st->iterations, (unsigned long long)done, __ATOMIC_RELAXED, AGENT);
  }
  if (__ballot(err != 0u) && lane == 0) atomicOr(&a.st->error, 1u);
  if (lane == 0) __hip_atomic_fetch_add(&a.st->screen_live, -1, __ATOMIC_RELAXED, AGENT);
}

// Iterations 1 and 2 in one kernel.  Each wave first takes its share of
// the shots for iteration 1 (wave w: shots w, w + nwaves, ...) and lists in
// its workgroup's LDS those that need iteration 2; then the workgroup's
// waves take listed shots one at a time, so that waves that finish early
// take the costly iteration-2 shots of their siblings.  A wave may wait
// only for waves of its own workgroup (all resident together): a taken
// position is served once a sibling lists a shot there, or given up when
// every sibling has finished iteration 1 and the list is shorter.
template <int V, int DV>
__global__ void __launch_bounds__(kScreen2Block, kScreen2MinWaves) k_screen12(ScreenArgs a) {
  extern __shared__ __align__(16) char sm[];
  const int m = a.m;
  int32_t* rptr = reinterpret_cast<int32_t*>(sm);
  float2* xy = reinterpret_cast<float2*>(sm + align16(4 * (size_t)(m + 1)));
  float* e1min = reinterpret_cast<float*>(sm + align16(4 * (size_t)(m + 1)) + align16(8 * (size_t)(m + 1)));
  WaveLds2* wl = reinterpret_cast<WaveLds2*>(sm + table_bytes(m, 2));
  WgList* gl = reinterpret_cast<WgList*>(sm + table_bytes(m, 2) + align16(kWaves2 * sizeof(WaveLds2)));
  for (int i = threadIdx.x; i <= m; i += kScreen2Block) {
    rptr[i] = a.row_ptr[i];
    xy[i] = a.row_xy[i];
    e1min[i] = i < m ? a.row_e1min[i] : 0.f;  // (row m: absent slots, bound 0)
  }
  for (int i = threadIdx.x; i < kWgList; i += kScreen2Block) gl->shot[i] = 0;
  if (threadIdx.x == 0) gl->count = gl->taken = gl->finished = 0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  WaveLds2& W = wl[wv];
  uint8_t* smap = reinterpret_cast<uint8_t*>(gl + 1) + wv * 2 * map_bytes(m);
  uint8_t* imap = smap + map_bytes(m);
  if (lane == 0) smap[m] = 0;  // absent row slots
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(&a.st->screen_begun, 1u, __ATOMIC_RELAXED, AGENT);
  const long long nwaves = (long long)gridDim.x * kWaves2;
  uint32_t done = 0, done2 = 0, err = 0;
  long long shot = (long long)blockIdx.x * kWaves2 + wv;
  uint2 sv[kSynRegs];
  if (a.syn8 && shot < a.shots) load_syn_regs(a, shot, lane, sv);
  for (; shot < a.shots; shot += nwaves) {
    const uint32_t t0 = a.lat ? (uint32_t)wall_clock64() : 0u;
    if (a.syn8 && syndrome_zero(sv)) {  // (load_syn_regs zeroes the rows past m)
      if (shot + nwaves < a.shots) load_syn_regs(a, shot + nwaves, lane, sv);
      write_zero_shot<V>(a, shot, lane);
      ++done;
      if (a.lat && lane == 0) a.lat[shot] = (uint32_t)wall_clock64() - t0;
      continue;
    }
    err |= syndrome_in(a, shot, sv, W, smap, lane);
    if (a.syn8 && shot + nwaves < a.shots) load_syn_regs(a, shot + nwaves, lane, sv);
    W.rbits[lane] = W.sbits[lane];
    if (lane == 0) {
      W.nset = 0;
      W.flw[0] = W.flw[1] = 0u;
    }
    int nflip, ncand;
    const bool ok = flipped_pairs(a, W, rptr, lane, &nflip, &ncand);
    if (ok) iteration1<DV>(a, W, xy, smap, ncand, lane);
    const bool conv = ok && W.nset <= kScreenMaxSet &&
                      __ballot(lane < a.words_m && W.rbits[lane] != 0u) == 0ull;
    if (conv) {
      write_shot<V>(a, W, shot, lane);
      ++done;
      if (a.lat && lane == 0) a.lat[shot] = (uint32_t)wall_clock64() - t0;
    } else if (lane == 0) {
      if (a.lat) a.lat[shot] = (uint32_t)wall_clock64() - t0;
      const int q = ok ? atomicAdd(&gl->count, 1) : kWgList;
      if (q < kWgList)
        __hip_atomic_store(&gl->shot[q], (int32_t)shot + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      else
        list_dense(a, shot);
    }
    wave_sync();  // the next shot reuses this wave's LDS
  }
  if (lane == 0) atomicAdd(&gl->finished, 1);
  // Iteration 2 of the workgroup's listed shots.
  for (;;) {
    int s2 = -1;
    if (lane == 0) {
      const int c = atomicAdd(&gl->taken, 1);
      for (;;) {
        const int v = __hip_atomic_load(&gl->shot[c < kWgList ? c : 0], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_WORKGROUP);
        if (c < kWgList && v != 0) {
          s2 = v - 1;
          break;
        }
        // (count is final once every wave has finished iteration 1)
        const int fin = __hip_atomic_load(&gl->finished, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const int cnt = __hip_atomic_load(&gl->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (c >= kWgList || (fin == kWaves2 && c >= cnt)) break;
        __builtin_amdgcn_s_sleep(4);
      }
    }
    s2 = __builtin_amdgcn_readfirstlane(s2);
    if (s2 < 0) break;
    if (a.syn8) load_syn_regs(a, s2, lane, sv);
    const uint32_t t0 = a.lat ? (uint32_t)wall_clock64() : 0u;
    for (int q = lane; q < (int)map_bytes(m) / 16; q += 64)
      reinterpret_cast<uint4*>(imap)[q] = make_uint4(0u, 0u, 0u, 0u);
    syndrome_in(a, s2, sv, W, smap, lane);
    int nflip, ncand;
    bool ok = flipped_pairs(a, W, rptr, lane, &nflip, &ncand);
    ok = ok && iteration2<DV>(a, W, xy, smap, imap, e1min, rptr, nflip, ncand, lane) &&
         W.nset <= kScreenMaxSet && __ballot(lane < a.words_m && W.rbits[lane] != 0u) == 0ull;
    if (ok) {
      write_shot<V>(a, W, s2, lane);
      ++done2;
      if (a.lat && lane == 0) a.lat[s2] += (uint32_t)wall_clock64() - t0;
    } else if (lane == 0) {
      if (a.lat) a.lat[s2] += (uint32_t)wall_clock64() - t0;
      list_dense(a, s2);
    }
    wave_sync();
  }
  if (lane == 0 && (done | done2)) {
    __hip_atomic_fetch_add(&a.st->done, (unsigned long long)(done + done2), __ATOMIC_RELAXED, AGENT);
    __hip_atomic_fetch_add(&a.st->runs, (unsigned long long)(done + done2), __ATOMIC_RELAXED, AGENT);
    __hip_atomic_fetch_add(&a.st->iterations, (unsigned long long)(done + 2 * done2),
                           __ATOMIC_RELAXED, AGENT);
    if (done2) __hip_atomic_fetch_add(&a.st->done2, (unsigned long long)done2, __ATOMIC_RELAXED, AGENT);
  }
  if (__ballot(err != 0u) && lane == 0) atomicOr(&a.st->error, 1u);
  if (lane == 0) __hip_atomic_fetch_add(&a.st->screen_live, -1, __ATOMIC_RELAXED, AGENT);
}

size_t lds1(int m) { return table_bytes(m, 1) + align16(kWaves1 * sizeof(WaveLds1)) + kWaves1 * map_bytes(m); }
size_t lds2(int m) {
  return table_bytes(m, 2) + align16(kWaves2 * sizeof(WaveLds2)) + sizeof(WgList) +
         kWaves2 * 2 * map_bytes(m);
}

template <int DV>
hipError_t launch_dv(const ScreenArgs& a, int grid1, int grid2, hipStream_t s) {
  if (a.t2) {
    switch (a.vec) {
      case 16: hipLaunchKernelGGL((k_screen12<16, DV>), dim3(grid2), dim3(kScreen2Block), lds2(a.m), s, a); break;
      case 4: hipLaunchKernelGGL((k_screen12<4, DV>), dim3(grid2), dim3(kScreen2Block), lds2(a.m), s, a); break;
      case 1: hipLaunchKernelGGL((k_screen12<1, DV>), dim3(grid2), dim3(kScreen2Block), lds2(a.m), s, a); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (a.vec) {
      case 16: hipLaunchKernelGGL((k_screen1<16, DV>), dim3(grid1), dim3(kScreenBlock), lds1(a.m), s, a); break;
      case 4: hipLaunchKernelGGL((k_screen1<4, DV>), dim3(grid1), dim3(kScreenBlock), lds1(a.m), s, a); break;
      case 1: hipLaunchKernelGGL((k_screen1<1, DV>), dim3(grid1), dim3(kScreenBlock), lds1(a.m), s, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

}  // namespace

int screen_blocks_per_cu(int m, int which) {
  int n = 0;
  const hipError_t e =
      which == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_screen1<16, 8>, kScreenBlock, lds1(m))
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_screen12<16, 8>, kScreen2Block, lds2(m));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n < 1 ? 1 : n;
}

hipError_t launch_screen(const ScreenArgs& a, int grid1, int grid2, hipStream_t s) {
  switch (a.maxdeg_col) {
    case 1: case 2: return launch_dv<2>(a, grid1, grid2, s);
    case 3: case 4: return launch_dv<4>(a, grid1, grid2, s);
    case 5: case 6: return launch_dv<6>(a, grid1, grid2, s);
    case 7: case 8: return launch_dv<8>(a, grid1, grid2, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bsd
