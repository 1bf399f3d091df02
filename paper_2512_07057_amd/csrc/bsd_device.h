// Device code of the beam-search decoder for gfx950 (templates; instantiated
// per column-position word count PW in bsd_kernels_pw*.hip).
//
// One workgroup runs one BP run at a time with the run's edge messages held
// in LDS (fp32, one word per Tanner edge, jagged-diagonal order).  A run is
// the masked min-sum BP of Algorithm 2: eq. (1) in the check phase (one lane
// per detector row), eqs. (2)-(4) in the variable phase (lanes own columns
// c * blockDim + tid), the stopping rule through an LDS residual bit-vector,
// and, when a run fails, the path score and least reliable node of
// Algorithm 3.  The graph data a lane needs (LDS positions of its columns'
// edges, degrees, priors, the rows it checks) is read once per launch into
// registers, so a run touches only LDS apart from its syndrome, its
// warm-start messages and its results.
//
// LDS layout: a fixed 7072-byte area of small arrays at offset 0 (constant
// offsets), then the messages, then one word of 0.0 per lane that a
// column's absent edges load from and store 0.0 back to (variable phase),
// and one shared word of 0.0 for absent row slots (check phase), so the
// inner loops need no branches.
//
// Floating-point order follows the paper's formulas left to right: sums run
// over neighbours in ascending row index, E of eq. (2) is a literal exclusive
// sum (the shared prefix is reused, the skipped term is never added and
// subtracted), sum_LLR accumulates in iteration order, and the path score
// sums |sum_LLR| as an aligned pairwise tree over column index.  Built with
// -ffp-contract=off.
#pragma once

#include "bsd_internal.h"

namespace bsd {
namespace dev {

constexpr int AGENT = __HIP_MEMORY_SCOPE_AGENT;
constexpr uint32_t kInfBits = 0x7F800000u;
constexpr uint32_t kSignBit = 0x80000000u;

// Fixed LDS offsets (bytes).
constexpr int kMaxWordsM = 64;                       // m <= 2048
constexpr int kOffDiag = 0;                          // int32[256] jagged-diagonal starts
constexpr int kOffSprime = kOffDiag + 1024;          // uint32[64] s' by row rank
constexpr int kOffResid = kOffSprime + 256;          // uint32[2][64] s' xor H e-hat
constexpr int kOffPairs = kOffResid + 512;           // int32[64] packed (col << 1) | val
constexpr int kOffMisc = kOffPairs + 256;            // int32[32]
constexpr int kOffFlips = kOffMisc + 128;            // uint32[4] logical-flip accumulator
constexpr int kOffRedf = kOffFlips + 16;             // float[32][16] score partials
constexpr int kOffPart = kOffRedf + 2048;            // float[32]
constexpr int kOffAminv = kOffPart + 128;            // float[16]
constexpr int kOffAminj = kOffAminv + 64;            // int32[16]
constexpr int kOffOrder = kOffAminj + 64;            // int32[128] rank of each child
constexpr int kOffByrank = kOffOrder + 512;          // int32[128] child of each rank
constexpr int kOffMark = kOffByrank + 512;           // int32[196]
constexpr int kOffNewslots = kOffMark + 784;         // int32[192]
constexpr int kOffMsg = kOffNewslots + 768;          // float[nnz_pad + kTrashWords + 4]
static_assert(kOffMsg % 16 == 0, "message area must be 16-byte aligned");

struct Lds {
  char* base;
  __device__ __forceinline__ uint32_t* u32(int off) const { return reinterpret_cast<uint32_t*>(base + off); }
  __device__ __forceinline__ int32_t* i32(int off) const { return reinterpret_cast<int32_t*>(base + off); }
  __device__ __forceinline__ float* f32(int off) const { return reinterpret_cast<float*>(base + off); }
  __device__ __forceinline__ float* msg() const { return f32(kOffMsg); }
  __device__ __forceinline__ uint32_t* msgu() const { return u32(kOffMsg); }
  __device__ __forceinline__ int32_t* misc() const { return i32(kOffMisc); }
  __device__ __forceinline__ int32_t* pairs() const { return i32(kOffPairs); }
  __device__ __forceinline__ uint32_t* sprime() const { return u32(kOffSprime); }
  __device__ __forceinline__ uint32_t* resid(int b) const { return u32(kOffResid + 256 * b); }
};

// After the messages: one word per lane for a column's absent edges, then
// one word for absent row slots; all stay 0.0.
__host__ __device__ inline size_t lds_need(const DevGraph& g) {
  return (size_t)kOffMsg + ((size_t)g.nnz_pad + kTrashWords + 4) * 4;
}

// Barrier for LDS data only: waits for this wave's LDS operations, not for
// its outstanding global stores.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Graph data of one lane, read once per launch.  Lane tid owns columns
// c * B + tid (c < CPT) and detector rows of rank q * B + tid (q < 2).
template <int CPT, int PW>
struct Res {
  float lam[CPT];
  uint32_t pos[CPT][PW];          // LDS positions of the column's edges (16 bits each, CSC
                                  // order); absent edges point at the zero word
  uint32_t deg[(CPT + 7) / 8];    // 4 bits per column
  uint32_t dmx[(CPT + 7) / 8];    // 4 bits per column: largest degree in the wave
  uint32_t row[2];                // original row (bits 0..15) | degree << 16 | 1 << 31; 0 past m
};

// Hide a lane's graph registers from loop-invariant code motion, so that
// values derived from them are recomputed where used instead of being kept
// live (unpacked) across runs.
template <int CPT, int PW>
__device__ __forceinline__ void opaque_res(Res<CPT, PW>& R) {
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
#pragma unroll
    for (int w = 0; w < PW; ++w) asm volatile("" : "+v"(R.pos[c][w]));
    asm volatile("" : "+v"(R.lam[c]));
  }
#pragma unroll
  for (int w = 0; w < (CPT + 7) / 8; ++w)
    asm volatile("" : "+v"(R.deg[w]), "+v"(R.dmx[w]));
  asm volatile("" : "+v"(R.row[0]), "+v"(R.row[1]));
}

// threadIdx.x as a value the compiler cannot treat as loop-invariant:
// addresses derived from it are recomputed inside the persistent loop rather
// than kept live (and spilled) across it.
__device__ __forceinline__ int fresh_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

template <int CPT>
struct RunRegs {
  float sumllr[CPT];
  uint32_t ebits;  // hard decision of unmasked columns at the last iteration
  uint32_t mbits;  // masked columns
  uint32_t vbits;  // values of masked columns
};

// Largest workgroup a kernel instance is compiled for: lanes that own more
// than 9 columns get a 256-register budget (at most 512 threads).
constexpr int max_block_for(int cpt) { return cpt > 9 ? 512 : 1024; }

struct RunRes {
  int iters;
  int conv;
  int cancelled;
};

// Loads a persistent workgroup issues during a shot's initial run for the
// step after it, so that they complete while the run computes instead of on
// the way out: the next shot's syndrome bits (after the prologue), the
// logical mask of each lane's lowest set hard decision and the work queue's
// length (after each variable phase), and the first-iteration table entries
// for the next shot (after each convergence barrier).  Values are consumed
// only on output.
struct EarlyLoads {
  const uint8_t* next_syn;          // next shot's syndrome, or nullptr
  const int32_t* work_count;        // read by thread 0
  const uint64_t* lmask;            // [n] logical masks
  uint32_t sb[2];                   // out: syndrome bytes of the lane's row slots
  int32_t work_hint;                // out, thread 0
  unsigned long long lm;            // out: lmask of the lowest set bit of ebits, else 0
  const FirstIter* fi;              // first-iteration table for the next shot, or nullptr
  uint4 rt[2];                      // out: its entries for the lane's row slots
};

template <int CPT, int PW>
__device__ __forceinline__ int col_deg(const Res<CPT, PW>& R, int c) {
  return (int)((R.deg[c >> 3] >> (4 * (c & 7))) & 15u);
}

template <int CPT, int PW>
__device__ __forceinline__ int col_dmax(const Res<CPT, PW>& R, int c) {
  return __builtin_amdgcn_readfirstlane((int)((R.dmx[c >> 3] >> (4 * (c & 7))) & 15u));
}

template <int CPT, int PW>
__device__ __forceinline__ uint32_t col_pos(const Res<CPT, PW>& R, int c, int e) {
  return (R.pos[c][e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ uint32_t trash_pos(const DevGraph& g) {
  return (uint32_t)g.nnz_pad + (threadIdx.x & 63u);
}

__device__ __forceinline__ uint32_t zero_pos(const DevGraph& g) {
  return (uint32_t)g.nnz_pad + kTrashWords;
}


// Load a lane's graph data (called by every thread, before any run).
template <int CPT, int PW>
__device__ __forceinline__ void load_res(const DevGraph& g, const Lds& L, Res<CPT, PW>& R) {
  const int tid = threadIdx.x, B = blockDim.x;
  for (int i = tid; i < 256; i += B) L.i32(kOffDiag)[i] = i <= g.maxdeg_row ? g.diag_ptr[i] : 0;
  if (tid == 0) L.msg()[zero_pos(g)] = 0.f;
  if (tid < kTrashWords) L.msg()[g.nnz_pad + tid] = 0.f;
  // Absent edges of a column point at the lane's own word after the
  // messages (kept at 0.0: the variable phase writes back what it read).
  const uint32_t tp = trash_pos(g);
#pragma unroll
  for (int w = 0; w < (CPT + 7) / 8; ++w) R.deg[w] = R.dmx[w] = 0u;
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int j = c * B + tid;
    int dg = 0;
    R.lam[c] = 0.f;
    int st = 0;
    if (j < g.n) {
      const uint32_t info = g.colinfo[j];
      st = (int)(info & 0xFFFFFFu);
      dg = (int)(info >> 24);
      R.lam[c] = g.lambda[j];
    }
#pragma unroll
    for (int w = 0; w < PW; ++w) {
      const uint32_t p0 = 2 * w < dg ? (g.cedge[st + 2 * w] & 0xFFFFu) : tp;
      const uint32_t p1 = 2 * w + 1 < dg ? (g.cedge[st + 2 * w + 1] & 0xFFFFu) : tp;
      R.pos[c][w] = p0 | (p1 << 16);
    }
    R.deg[c >> 3] |= (uint32_t)dg << (4 * (c & 7));
    R.dmx[c >> 3] |= (uint32_t)wave_max_i(dg) << (4 * (c & 7));
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int r = q * B + tid;
    R.row[q] = r < g.m ? ((uint32_t)g.row_of_rank[r] | ((uint32_t)g.deg_of_rank[r] << 16) | kSignBit)
                       : 0u;
  }
  __syncthreads();
}

// Running least and second least magnitude: m1 <= m2 and |v| joins them.
// The median of (m1, m2, |v|) is the new second least, the median of
// (m1, |v|, -inf) the new least.  fmed3 takes the absolute value as a free
// source modifier.  `ninf` is -inf passed in a register: with the constant
// visible the compiler turns the second median into an IEEE minimum, which
// costs two extra canonicalising instructions per edge.
__device__ __forceinline__ void min2_step(float& m1, float& m2, uint32_t v, float ninf) {
  const float a = fabsf(__uint_as_float(v));
  m2 = __builtin_amdgcn_fmed3f(m1, m2, a);
  m1 = __builtin_amdgcn_fmed3f(m1, a, ninf);
}

// Output of eq. (1) on one edge holding v: magnitude d2 if |v| is the row
// minimum m1 (the minimum over the other edges), else d1; sign of the row
// product times that of v.  Masked edges (+inf) keep their value.
template <bool MASKED>
__device__ __forceinline__ uint32_t check_out(uint32_t v, uint32_t sgn, float m1, float d1, float d2) {
  const float mag = fabsf(__uint_as_float(v)) == m1 ? d2 : d1;
  const uint32_t d = ((sgn ^ v) & kSignBit) | (__float_as_uint(mag) & ~kSignBit);
  return (MASKED && v == kInfBits) ? v : d;
}

// Eq. (1) for the detector rows of rank q * B + tid, in place: E(t-1) -> D(t)
// on the unmasked edges (masked edges hold +inf and are skipped).  Magnitudes
// of non-negative floats compare as unsigned integers.  An edge whose
// magnitude equals the row minimum receives the second minimum: that is the
// minimum over the other edges whether the minimum is unique or tied.  Ranks
// are sorted by degree, so in a wave every row has at least the last lane's
// degree and at most the first lane's: only that range needs predicates.
template <bool MASKED>
__device__ __forceinline__ void check_rows(const DevGraph& g, const Lds& L, uint32_t rowinfo, int r,
                                           float alpha) {
  uint32_t* msg = L.msgu();
  const int32_t* diag = L.i32(kOffDiag);
  asm volatile("" : "+v"(rowinfo));
  const int dg = (int)((rowinfo >> 16) & 0xFFu);
  const int kmax = __builtin_amdgcn_readfirstlane(dg);
  if (kmax == 0) return;
  const int kmin = __builtin_amdgcn_readlane(dg, 63);
  const uint32_t zp = zero_pos(g);
  uint32_t sgn = dg ? ((L.sprime()[r >> 5] >> (r & 31)) & 1u) << 31 : 0u;
  float m1 = kLlrMax, m2 = kLlrMax;
  float ninf = -__builtin_inff();
  asm volatile("" : "+v"(ninf));
  int k = 0;
  for (; k + 4 <= kmin; k += 4) {
    const int4 dd = *reinterpret_cast<const int4*>(diag + k);
    const uint32_t vv[4] = {msg[dd.x + r], msg[dd.y + r], msg[dd.z + r], msg[dd.w + r]};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      sgn ^= vv[u];
      min2_step(m1, m2, vv[u], ninf);
    }
  }
  for (; k < kmax; ++k) {
    const bool ok = k < dg;
    const uint32_t v = msg[ok ? (uint32_t)(diag[k] + r) : zp];
    sgn ^= v;
    min2_step(m1, m2, ok ? v : kInfBits, ninf);
  }
  const float d1 = fminf(alpha * m1, kLlrMax), d2 = fminf(alpha * m2, kLlrMax);
  k = 0;
  for (; k + 4 <= kmin; k += 4) {
    const int4 dd = *reinterpret_cast<const int4*>(diag + k);
    const int pp[4] = {dd.x + r, dd.y + r, dd.z + r, dd.w + r};
    uint32_t vv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) vv[u] = msg[pp[u]];
#pragma unroll
    for (int u = 0; u < 4; ++u) msg[pp[u]] = check_out<MASKED>(vv[u], sgn, m1, d1, d2);
  }
  for (; k < kmax; ++k) {
    if (k < dg) {
      const uint32_t p = (uint32_t)(diag[k] + r);
      msg[p] = check_out<MASKED>(msg[p], sgn, m1, d1, d2);
    }
  }
}

// Eqs. (2)-(4) for one column with at most D edges (D uniform over the wave).
// Absent edges load from and store to the lane's own zero word; inactive
// lanes (masked nodes, columns past n) store back the values they loaded.
template <int D, int CPT, int PW>
__device__ __forceinline__ void var_col(const DevGraph& g, const Lds& L, const Res<CPT, PW>& R,
                                        int c, bool active, float& sl, uint32_t& eb) {
  float* msg = L.msg();
  uint32_t dw = R.deg[c >> 3];
  asm volatile("" : "+v"(dw));
  const int dg = (int)((dw >> (4 * (c & 7))) & 15u);
  uint32_t p[D];
  float d[D];
  // Unpack the positions here, inside the iteration: kept packed across
  // iterations they cost half the registers.
  uint32_t pk[PW];
#pragma unroll
  for (int w = 0; w < PW; ++w) {
    pk[w] = R.pos[c][w];
    asm volatile("" : "+v"(pk[w]));
  }
#pragma unroll
  for (int e = 0; e < D; ++e) {
    p[e] = (pk[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
    d[e] = msg[p[e]];
  }
  float pre = R.lam[c];
#pragma unroll
  for (int e = 0; e < D; ++e) {  // eq. (2): the prefix before e, then the terms after e
    float x = pre;
#pragma unroll
    for (int f = e + 1; f < D; ++f) x = x + d[f];
    // Absent edges (lane's zero word) and inactive lanes write back what
    // they read: one address per edge for the load and the store.
    msg[p[e]] = (active && e < dg) ? __builtin_amdgcn_fmed3f(x, -kLlrMax, kLlrMax) : d[e];
    pre = pre + d[e];
  }
  const float post = pre;  // eq. (3)
  sl = active ? sl + post : sl;
  eb = (active && post <= 0.f) ? 1u : 0u;  // eq. (4)
}

// The syndrome residual s' + H e-hat: each set hard decision flips the bits
// of its column's detectors.  Done after all columns so that a wave waits
// for one round of rank-table loads.
__device__ __forceinline__ void flip_resid(const DevGraph& g, uint32_t* resid, uint32_t ebits) {
  for (uint32_t mk = ebits; mk; mk &= mk - 1u) {
    const int c = __builtin_ctz(mk);
    const uint4 rq = g.crank[c * (int)blockDim.x + fresh_tid()];
    const uint32_t rw[4] = {rq.x, rq.y, rq.z, rq.w};
#pragma unroll
    for (int e = 0; e < kMaxDv; ++e) {
      const uint32_t rk = (rw[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
      if (rk != 0xFFFFu) atomicXor(&resid[rk >> 5], 1u << (rk & 31));
    }
  }
}

template <int CPT, int PW>
__device__ __forceinline__ void var_phase(const DevGraph& g, const Lds& L, uint32_t* resid,
                                          const Res<CPT, PW>& R, RunRegs<CPT>& rg) {
  const int B = blockDim.x, tid = fresh_tid();
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int j = c * B + tid;
    const bool active = j < g.n && !((rg.mbits >> c) & 1u);
    uint32_t eb = 0;
    const int D = col_dmax(R, c);
    switch (D) {
      case 1: var_col<1>(g, L, R, c, active, rg.sumllr[c], eb); break;
      case 2: var_col<2>(g, L, R, c, active, rg.sumllr[c], eb); break;
      case 3: if constexpr (PW >= 2) var_col<3>(g, L, R, c, active, rg.sumllr[c], eb); break;
      case 4: if constexpr (PW >= 2) var_col<4>(g, L, R, c, active, rg.sumllr[c], eb); break;
      case 5: if constexpr (PW >= 3) var_col<5>(g, L, R, c, active, rg.sumllr[c], eb); break;
      case 6: if constexpr (PW >= 3) var_col<6>(g, L, R, c, active, rg.sumllr[c], eb); break;
      case 7: if constexpr (PW >= 4) var_col<7>(g, L, R, c, active, rg.sumllr[c], eb); break;
      case 8: if constexpr (PW >= 4) var_col<8>(g, L, R, c, active, rg.sumllr[c], eb); break;
      default: break;
    }
    rg.ebits = (rg.ebits & ~(1u << c)) | (eb << c);
  }
  flip_resid(g, resid, rg.ebits);
}

// D(1) on the edges of the lane's rows (ranks q * B + tid) from the
// first-iteration table entries `rt` and the rows' syndrome bits.
template <int CPT, int PW>
__device__ __forceinline__ void write_d1(const DevGraph& g, const Lds& L, const Res<CPT, PW>& R,
                                         const FirstIter* fi, const uint4* rt,
                                         const uint32_t* sbit) {
  const int tid = fresh_tid(), B = blockDim.x;
  // Magnitude y on the edge of the least |Lambda|, x elsewhere; sign
  // (-1)^{s_i} times the parity of the other edges' priors.
  const int32_t* diag = L.i32(kOffDiag);
  uint32_t* mu = L.msgu();
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int r = q * B + tid;
    const int dg = (int)((R.row[q] >> 16) & 0xFFu);
    const uint32_t x = rt[q].x, y = rt[q].y, info = rt[q].z;
    const int argk = (int)(info & 0xFFu);
    const uint32_t sg = (((info >> 8) & 1u) ^ sbit[q]) << 31;
    if ((info >> 9) & 1u) {  // some prior of the row is negative
      for (int k = 0; k < dg; ++k) {
        const int pq = diag[k] + r;
        const uint32_t nb = ((fi->negbits[pq >> 5] >> (pq & 31)) & 1u) << 31;
        mu[pq] = (k == argk ? y : x) | (sg ^ nb);
      }
    } else {
      // Every edge gets x, then the edge of the least |Lambda| gets y: a
      // lane's LDS writes land in program order.
      const uint32_t xs = x | sg;
      int k = 0;
      for (; k + 8 <= dg; k += 8) {
        const int4 d0 = *reinterpret_cast<const int4*>(diag + k);
        const int4 d1 = *reinterpret_cast<const int4*>(diag + k + 4);
        mu[d0.x + r] = xs;
        mu[d0.y + r] = xs;
        mu[d0.z + r] = xs;
        mu[d0.w + r] = xs;
        mu[d1.x + r] = xs;
        mu[d1.y + r] = xs;
        mu[d1.z + r] = xs;
        mu[d1.w + r] = xs;
      }
      for (; k + 4 <= dg; k += 4) {
        const int4 dd = *reinterpret_cast<const int4*>(diag + k);
        mu[dd.x + r] = xs;
        mu[dd.y + r] = xs;
        mu[dd.z + r] = xs;
        mu[dd.w + r] = xs;
      }
      for (; k < dg; ++k) mu[diag[k] + r] = xs;
      if (argk < dg) mu[diag[argk] + r] = y | sg;
    }
  }
}

// One masked BP run (Algorithm 2).  The caller has placed `npairs` packed
// pairs in LDS and synchronised.  Warm start from `parent` (LDS order) or
// `parent_csc` (CSC order), else from the priors.  When `cancel` is given the
// run stops early once *cancel < my_gen (a lower generation converged).
//
// A run from the priors with no masked node and `fi` enabled writes the
// check phase of iteration 1 from the per-row table fi->rows: with E(0) =
// Lambda on every edge, eq. (1) at t = 1 depends on the syndrome only through
// the factor (-1)^{s_i}.  The values are bit for bit those check_rows would
// form.
template <int CPT, int PW>
__device__ __forceinline__ RunRes bp_run(const DevGraph& g, const Lds& L, Res<CPT, PW>& R,
                                         const float* parent, const float* parent_csc, int npairs,
                                         const uint8_t* syn, int T, bool stop, float alpha,
                                         const int32_t* cancel, int my_gen, RunRegs<CPT>& rg,
                                         uint32_t* err, const FirstIter* fi = nullptr,
                                         bool have_pf = false, uint32_t pf = 0u,
                                         const float* asched = nullptr, int nsched = 0,
                                         EarlyLoads* early = nullptr, bool d1_done = false) {
  const int tid = fresh_tid(), B = blockDim.x, lane = tid & 63, wave = tid >> 6;
  float* msg = L.msg();
  const bool table = fi && fi->enabled && !parent && !parent_csc && npairs == 0 && T >= 1;
  rg.mbits = rg.vbits = rg.ebits = 0;
  for (int q = 0; q < npairs; ++q) {
    const int pv = L.pairs()[q];
    const int d = (pv >> 1) - tid;
    if (d >= 0 && d % B == 0 && d / B < CPT) {
      rg.mbits |= 1u << (d / B);
      rg.vbits |= (uint32_t)(pv & 1) << (d / B);
    }
  }
  if (tid < 2) L.u32(kOffFlips)[tid] = 0u;
  // s by row rank, 64 ranks per wave ballot.  A table run also fills the
  // residual of iteration 1 here (s' = s without masked nodes).
  uint32_t sbit[2];
  uint4 rt[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    rt[q] = make_uint4(0u, 0u, 0u, 0u);
    if (table && !d1_done && (R.row[q] >> 31)) rt[q] = fi->rows[q * B + tid];
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    uint32_t bit = 0;
    if (R.row[q] >> 31) {
      const uint32_t b = have_pf ? (pf >> (8 * q)) & 0xFFu : syn[R.row[q] & 0xFFFFu];
      if (b > 1u) atomicOr(err, 1u);
      bit = b & 1u;
    }
    sbit[q] = bit;
    const unsigned long long bal = __ballot(bit);
    if (lane == 0) {
      const int w = (q * B + wave * 64) >> 5;
      if (w < g.words_m) L.sprime()[w] = (uint32_t)bal;
      if (w + 1 < g.words_m) L.sprime()[w + 1] = (uint32_t)(bal >> 32);
      if (table) {
        if (w < g.words_m) L.resid(1)[w] = (uint32_t)bal;
        if (w + 1 < g.words_m) L.resid(1)[w + 1] = (uint32_t)(bal >> 32);
      }
    }
  }
  if (table && !d1_done) write_d1<CPT, PW>(g, L, R, fi, rt, sbit);
  if (parent) {
    const float4* src = reinterpret_cast<const float4*>(parent);
    float4* dst = reinterpret_cast<float4*>(msg);
    for (int i = tid; i < g.nnz_pad / 4; i += B) dst[i] = src[i];
  }
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    rg.sumllr[c] = 0.f;
    const int j = c * B + tid;
    if (!parent && !table && j < g.n) {
      const int dg = col_deg(R, c);
      if (parent_csc) {
        const int st = (int)(g.colinfo[j] & 0xFFFFFFu);
        for (int e = 0; e < dg; ++e) msg[g.cedge[st + e] & 0xFFFFu] = parent_csc[st + e] + 0.f;
      } else {
#pragma unroll
        for (int e = 0; e < 2 * PW; ++e)
          if (e < dg) msg[col_pos(R, c, e)] = R.lam[c];
      }
    }
  }
  lds_barrier();
  // Masked nodes leave every check (+inf) and fold their value into s'.
  if (npairs) {
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      if ((rg.mbits >> c) & 1u) {
        const int j = c * B + tid;
        const int st = (int)(g.colinfo[j] & 0xFFFFFFu), dg = col_deg(R, c);
        for (int e = 0; e < dg; ++e) {
          const uint32_t w = g.cedge[st + e];
          msg[w & 0xFFFFu] = __builtin_inff();
          if ((rg.vbits >> c) & 1u) {
            const uint32_t rk = w >> 16;
            atomicXor(&L.sprime()[rk >> 5], 1u << (rk & 31));
          }
        }
      }
    }
    lds_barrier();
  }
  if (early) {
    if (tid < 2) L.u32(kOffFlips)[2 + tid] = 0u;  // read by everyone before the barrier above
    early->sb[0] = early->sb[1] = 0u;
    if (early->next_syn) {
#pragma unroll
      for (int q = 0; q < 2; ++q)
        if (R.row[q] >> 31) early->sb[q] = early->next_syn[R.row[q] & 0xFFFFu];
    }
  }

  RunRes rr{0, 0, 0};
  for (int t = 1; t <= T; ++t) {
    uint32_t* resid = L.resid(t & 1);
    if (!(table && t == 1)) {
      for (int w = tid; w < g.words_m; w += B) resid[w] = L.sprime()[w];
      const float at = asched ? asched[min(t, nsched) - 1] : alpha;
      if (npairs) {
#pragma unroll
        for (int q = 0; q < 2; ++q) check_rows<true>(g, L, R.row[q], q * B + tid, at);
      } else {
#pragma unroll
        for (int q = 0; q < 2; ++q) check_rows<false>(g, L, R.row[q], q * B + tid, at);
      }
      lds_barrier();
    }
    var_phase<CPT, PW>(g, L, resid, R, rg);
    if (early) {
      const uint32_t eb = rg.ebits & ~rg.mbits;
      early->lm = eb ? early->lmask[__builtin_ctz(eb) * B + tid] : 0ull;
      if (tid == 0) early->work_hint = __hip_atomic_load(early->work_count, __ATOMIC_RELAXED, AGENT);
    }
    if (tid == 0) {
      int cx = 0;
      if (cancel) cx = __hip_atomic_load(cancel, __ATOMIC_RELAXED, AGENT) < my_gen;
      L.misc()[0] = cx;
    }
    lds_barrier();
    if (early && early->fi) {  // loaded here, not across the variable phase: fewer live registers
#pragma unroll
      for (int q = 0; q < 2; ++q)
        if (R.row[q] >> 31) early->rt[q] = early->fi->rows[q * B + tid];
    }
    uint32_t any = 0;
    for (int w = 0; w < g.words_m; w += 2) {
      const uint2 x = *reinterpret_cast<const uint2*>(resid + w);
      any |= x.x | x.y;
    }
    rr.iters = t;
    rr.conv = any ? 0 : 1;
    if (stop && rr.conv) break;
    if (L.misc()[0]) {
      rr.cancelled = 1;
      break;
    }
  }
  return rr;
}

// Path score and next branching node of a finished run (Algorithm 3):
// next_pos = least |sum_LLR| over unmasked nodes (lowest index on ties),
// score = aligned pairwise-tree sum of |sum_LLR| over unmasked nodes / iters.
template <int CPT>
__device__ __forceinline__ void score_next(const DevGraph& g, const Lds& L,
                                           const RunRegs<CPT>& rg, int iters, float* score,
                                           int* next_pos) {
  const int tid = threadIdx.x, B = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = B >> 6;
  float* redf = L.f32(kOffRedf);
  float bv = __builtin_inff();
  int bj = 0x7FFFFFFF;
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int j = c * B + tid;
    const bool ok = j < g.n && !((rg.mbits >> c) & 1u);
    float a = ok ? fabsf(rg.sumllr[c]) : 0.f;
    if (ok && a < bv) {
      bv = a;
      bj = j;
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) a = a + __shfl_xor(a, o, 64);
    if (lane == 0) redf[c * kMaxWaves + wave] = a;
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const float ov = __shfl_xor(bv, o, 64);
    const int oj = __shfl_xor(bj, o, 64);
    if (ov < bv || (ov == bv && oj < bj)) {
      bv = ov;
      bj = oj;
    }
  }
  if (lane == 0) {
    L.f32(kOffAminv)[wave] = bv;
    L.i32(kOffAminj)[wave] = bj;
  }
  __syncthreads();
  if (tid == 0) {
    // Aligned pairwise tree: over the waves of each column block, then over blocks.
    float* part = L.f32(kOffPart);
    for (int c = 0; c < CPT; ++c) {
      float* v = redf + c * kMaxWaves;
      for (int len = nw; len > 1; len >>= 1)
        for (int i = 0; i < len / 2; ++i) v[i] = v[2 * i] + v[2 * i + 1];
      part[c] = v[0];
    }
    int c2 = 1;
    while (c2 < CPT) c2 <<= 1;
    for (int c = CPT; c < c2; ++c) part[c] = 0.f;
    for (int len = c2; len > 1; len >>= 1)
      for (int i = 0; i < len / 2; ++i) part[i] = part[2 * i] + part[2 * i + 1];
    const float sc = iters > 0 ? part[0] / (float)iters : 0.f;
    float mv = __builtin_inff();
    int mj = 0x7FFFFFFF;
    for (int w = 0; w < nw; ++w) {
      const float av = L.f32(kOffAminv)[w];
      const int aj = L.i32(kOffAminj)[w];
      if (av < mv || (av == mv && aj < mj)) {
        mv = av;
        mj = aj;
      }
    }
    L.misc()[4] = __float_as_int(sc);
    L.misc()[5] = (mj == 0x7FFFFFFF) ? -1 : mj;
  }
  __syncthreads();
  *score = __int_as_float(L.misc()[4]);
  *next_pos = L.misc()[5];
}

// Hard-decision bits (one bit per column) to a global bit-vector.
template <int CPT>
__device__ __forceinline__ void store_bits(const DevGraph& g, uint32_t* dst, uint32_t bits) {
  const int tid = threadIdx.x, B = blockDim.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int j = c * B + tid;
    const unsigned long long bal = __ballot(j < g.n && ((bits >> c) & 1u));
    if (lane == 0) {
      const int w = (c * B + wave * 64) >> 5;
      if (w < g.words_n) dst[w] = (uint32_t)bal;
      if (w + 1 < g.words_n) dst[w + 1] = (uint32_t)(bal >> 32);
    }
  }
}

// wt(e-hat) = sum_j e_j log((1-p_j)/p_j) (Appendix B) in double precision,
// summed in ascending column order, and a 64-bit digest of e-hat, by thread
// 0 from an LDS bit-vector.  Every thread calls this; `bits` holds the hard
// decisions of columns c*B + tid.
template <int CPT>
__device__ __forceinline__ void weight_hash(const DevGraph& g, const Lds& L, const double* lam64,
                                            uint32_t bits, double* wt, uint64_t* hash) {
  const int tid = threadIdx.x, B = blockDim.x, lane = tid & 63, wave = tid >> 6;
  uint32_t* bm = L.u32(kOffRedf);  // words_n <= 512
  lds_barrier();
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int j = c * B + tid;
    const unsigned long long bal = __ballot(j < g.n && ((bits >> c) & 1u));
    if (lane == 0) {
      const int w = (c * B + wave * 64) >> 5;
      if (w < g.words_n) bm[w] = (uint32_t)bal;
      if (w + 1 < g.words_n) bm[w + 1] = (uint32_t)(bal >> 32);
    }
  }
  lds_barrier();
  if (tid == 0) {
    double s = 0.0;
    uint64_t h = 0xcbf29ce484222325ull;
    for (int w = 0; w < g.words_n; ++w) {
      uint32_t x = bm[w];
      h = (h ^ x) * 0x100000001b3ull;
      while (x) {
        s += lam64[w * 32 + __builtin_ctz(x)];
        x &= x - 1u;
      }
    }
    *wt = s;
    *hash = h;
  }
  lds_barrier();
}

__device__ __forceinline__ void store_msg(const DevGraph& g, const Lds& L, float* dst) {
  const float4* src = reinterpret_cast<const float4*>(L.msg());
  float4* d = reinterpret_cast<float4*>(dst);
  for (int i = threadIdx.x; i < g.nnz_pad / 4; i += blockDim.x) d[i] = src[i];
}

// Logical flips A e-hat: lanes holding a 1 fold their column's mask into an
// LDS accumulator (zeroed at the start of every run); one barrier, then the
// bytes are written.
__device__ __forceinline__ void flip_fold(const Lds& L, unsigned long long f, int w = 0) {
  if (f) {
    atomicXor(&L.u32(kOffFlips)[w], (uint32_t)f);
    atomicXor(&L.u32(kOffFlips)[w + 1], (uint32_t)(f >> 32));
  }
}

// Batched calls fold an initial run's flips into the second accumulator
// (words 2 and 3) and write them out only after the next scheduling
// barrier, which saves the output step a barrier of its own.  The words are
// cleared by the next initial run after its prologue barrier, once every
// lane has read them.
__device__ __forceinline__ void flip_write_late(const DevGraph& g, const Lds& L, uint8_t* flips) {
  const int tid = fresh_tid();
  if (tid < g.k) {
    const unsigned long long t =
        (unsigned long long)L.u32(kOffFlips)[2] | ((unsigned long long)L.u32(kOffFlips)[3] << 32);
    for (int r = tid; r < g.k; r += blockDim.x) flips[r] = (uint8_t)((t >> r) & 1ull);
  }
}

__device__ __forceinline__ void flip_write(const DevGraph& g, const Lds& L, uint8_t* flips) {
  lds_barrier();
  const unsigned long long t =
      (unsigned long long)L.u32(kOffFlips)[0] | ((unsigned long long)L.u32(kOffFlips)[1] << 32);
  for (int r = fresh_tid(); r < g.k; r += blockDim.x) flips[r] = (uint8_t)((t >> r) & 1ull);
}

// Shot output from register-resident hard decisions (columns c*B + tid),
// with the loads the run issued early (EarlyLoads): the logical masks, the
// next shot's syndrome bits and the work queue's length.  Only a lane with
// more than one set decision loads here.
template <int CPT, int PW>
__device__ __forceinline__ void emit_from_regs(const DevGraph& g, const Lds& L, uint32_t bits,
                                               uint8_t* corr, uint8_t* flips,
                                               const EarlyLoads& el, long long next_shot,
                                               long long& pf_shot, uint32_t& pf, int& work_hint,
                                               bool late_flips) {
  const int B = blockDim.x, tid = fresh_tid();
  unsigned long long f = el.lm;
  for (uint32_t mk = bits & (bits - 1u); mk; mk &= mk - 1u) f ^= g.lmask[__builtin_ctz(mk) * B + tid];
  if (tid == 0) work_hint = el.work_hint;
  if (next_shot >= 0) {
    pf = el.sb[0] | (el.sb[1] << 8);
    pf_shot = next_shot;
  }
  asm volatile("" : "+v"(f)::"memory");  // every load completes before the stores
  flip_fold(L, f, late_flips ? 2 : 0);
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int j = c * B + tid;
    if (j < g.n) corr[j] = (uint8_t)((bits >> c) & 1u);
  }
  if (!late_flips) flip_write(g, L, flips);
}

// Shot output from a global bit-vector.
__device__ __forceinline__ void emit_from_bits(const DevGraph& g, const Lds& L,
                                               const uint32_t* bits, uint8_t* corr, uint8_t* flips) {
  if (threadIdx.x < 2) L.u32(kOffFlips)[threadIdx.x] = 0u;
  lds_barrier();
  unsigned long long f = 0;
  for (int j = threadIdx.x; j < g.n; j += blockDim.x) {
    const uint32_t b = (bits[j >> 5] >> (j & 31)) & 1u;
    corr[j] = (uint8_t)b;
    if (b) f ^= g.lmask[j];
  }
  flip_fold(L, f);
  flip_write(g, L, flips);
}

// ---------------------------------------------------------------------------
// Device queues: multi-producer multi-consumer rings of 32-bit items
// ---------------------------------------------------------------------------

// The count only reserves items; the data an item refers to is published by
// the release of its ring entry (a release store, or a release fence before
// a batch of relaxed stores) and taken by one acquire fence after the entry
// has been seen.
__device__ __forceinline__ bool ring_pop(Ring* r, uint32_t* buf, uint32_t* out) {
  if (__hip_atomic_load(&r->count, __ATOMIC_RELAXED, AGENT) <= 0) return false;
  const int c = __hip_atomic_fetch_add(&r->count, -1, __ATOMIC_RELAXED, AGENT);
  if (c <= 0) {
    __hip_atomic_fetch_add(&r->count, 1, __ATOMIC_RELAXED, AGENT);
    return false;
  }
  const uint32_t h = __hip_atomic_fetch_add(&r->head, 1u, __ATOMIC_RELAXED, AGENT) & (r->cap - 1u);
  uint32_t x;
  while ((x = __hip_atomic_load(&buf[h], __ATOMIC_RELAXED, AGENT)) == 0u) __builtin_amdgcn_s_sleep(2);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __hip_atomic_store(&buf[h], 0u, __ATOMIC_RELAXED, AGENT);
  *out = x - 1u;
  return true;
}

// `fenced`: the caller has issued a release fence since its last writes.
__device__ __forceinline__ void ring_push(Ring* r, uint32_t* buf, uint32_t item, bool fenced = false) {
  const uint32_t t = __hip_atomic_fetch_add(&r->tail, 1u, __ATOMIC_RELAXED, AGENT) & (r->cap - 1u);
  while (__hip_atomic_load(&buf[t], __ATOMIC_RELAXED, AGENT) != 0u) __builtin_amdgcn_s_sleep(2);
  if (fenced)
    __hip_atomic_store(&buf[t], item + 1u, __ATOMIC_RELAXED, AGENT);
  else
    __hip_atomic_store(&buf[t], item + 1u, __ATOMIC_RELEASE, AGENT);
  __hip_atomic_fetch_add(&r->count, 1, __ATOMIC_RELAXED, AGENT);
}

__device__ __forceinline__ char* slot_ptr(const BatchArgs& a, int ctx, int s) {
  return a.slots + ((size_t)ctx * a.slots_per_ctx + s) * a.slot_stride;
}

__device__ __forceinline__ uint32_t dev_clock() { return (uint32_t)wall_clock64(); }

// A shot's latency: with the iteration-1 screen in front, its share was
// written first and this kernel's time is added (one thread).
__device__ __forceinline__ void put_latency(const BatchArgs& a, long long row, uint32_t ticks) {
  a.lat[row] = a.shot_list ? a.lat[row] + ticks : ticks;
}

// Row of a shot's syndrome and outputs (serving: a ring slot).
__device__ __forceinline__ long long io_row(const BatchArgs& a, long long shot) {
  return a.stream ? (long long)((unsigned long long)shot & a.io_mask) : shot;
}

// Serving: make the shot's outputs visible to the host, then raise its flag.
// Called by every thread after it has written its part of the outputs.
__device__ __forceinline__ void publish_done(const BatchArgs& a, long long shot) {
  if (!a.stream) return;
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(&a.done_flag[io_row(a, shot)], (uint32_t)(shot + 1), __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
}

// Write the shot's outputs from a slot's hard-decision bits and retire the context.
__device__ __forceinline__ void finish_deep(const BatchArgs& a, const Lds& L, int ctx,
                                            long long shot, const uint32_t* bits, int converged,
                                            uint32_t t_start) {
  const DevGraph& g = a.g;
  const long long row = io_row(a, shot);
  emit_from_bits(g, L, bits, a.corr + row * g.n, a.flips + row * g.k);
  if (threadIdx.x == 0) {
    a.conv[row] = (uint8_t)converged;
    if (a.lat) put_latency(a, row, dev_clock() - t_start);
  }
  publish_done(a, shot);
  // The barrier orders every lane's writes before thread 0's release in
  // ring_push, which publishes them at device scope.
  __syncthreads();
  if (threadIdx.x == 0) {
    ring_push(&a.st->ctxq, a.ctx_ring, (uint32_t)ctx);
    __hip_atomic_fetch_add(&a.st->done, 1ull, __ATOMIC_RELEASE, AGENT);
  }
}

// Output the lightest result (least wt; the first found among equals).
__device__ __forceinline__ void finish_lightest(const BatchArgs& a, const Lds& L, int ctx,
                                                long long shot, int nres, uint32_t t_start) {
  const Ctx* C = a.ctxs + ctx;
  if (threadIdx.x == 0) {
    int best = 0;
    for (int r = 1; r < nres; ++r)
      if (C->res_wt[r] < C->res_wt[best]) best = r;
    L.misc()[18] = best;
  }
  __syncthreads();
  const int best = L.misc()[18];
  const uint32_t* bits = a.results + ((size_t)ctx * a.num_results + best) * a.g.words_n;
  finish_deep(a, L, ctx, shot, bits, 1, t_start);
}

// Selection at the end of a round (Algorithm 3 with Appendix B), run by the
// workgroup that finished the round's last child.
__device__ __forceinline__ void select_round(const BatchArgs& a, const Lds& L, int ctx) {
  const DevGraph& g = a.g;
  Ctx* C = a.ctxs + ctx;
  const int tid = threadIdx.x;
  const int nset = C->nset, round = C->round, best = C->best_gen;
  const long long shot = C->shot;
  const uint32_t t0 = C->t_start;
  const int nch = 2 * nset;
  int32_t* order = L.i32(kOffOrder);
  int32_t* misc = L.misc();
  if (best != 0x7FFFFFFF) {
    // First converged child in exploration order.
    const int s = C->slots[nset + best];
    finish_deep(a, L, ctx, shot, (const uint32_t*)(slot_ptr(a, ctx, s) + slot_ehat_off(g)), 1, t0);
    return;
  }
  int nres = C->nresults;
  if (a.num_results > 1) {
    // Converged children join the results in exploration order (generation),
    // once each; the search ends when num_results distinct ones are found.
    // Digests of the results so far are mirrored in LDS, so that every
    // thread takes the same branches.
    uint32_t* res0 = a.results + (size_t)ctx * a.num_results * g.words_n;
    uint64_t* rh = reinterpret_cast<uint64_t*>(L.u32(kOffOrder));  // [kMaxResults]
    for (int r = tid; r < nres; r += blockDim.x) rh[r] = C->res_hash[r];
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
      if (C->parent_next_pos[c >> 1] < 0 || C->child_state[c] != 1) continue;
      const uint32_t* cb = (const uint32_t*)(slot_ptr(a, ctx, C->slots[nset + c]) + slot_ehat_off(g));
      const uint64_t h = C->child_hash[c];
      bool dup = false;
      for (int r = 0; r < nres && !dup; ++r) {
        if (rh[r] != h) continue;
        if (tid == 0) misc[17] = 0;
        __syncthreads();
        const uint32_t* rb = res0 + (size_t)r * g.words_n;
        for (int w = tid; w < g.words_n; w += blockDim.x)
          if (cb[w] != rb[w]) misc[17] = 1;
        __syncthreads();
        dup = misc[17] == 0;
        __syncthreads();
      }
      if (dup) continue;
      uint32_t* dst = res0 + (size_t)nres * g.words_n;
      for (int w = tid; w < g.words_n; w += blockDim.x) dst[w] = cb[w];
      if (tid == 0) {
        C->res_wt[nres] = C->child_wt[c];
        C->res_hash[nres] = h;
        rh[nres] = h;
      }
      __syncthreads();
      ++nres;
      if (nres >= a.num_results) break;
    }
    __syncthreads();  // thread 0's later releases publish every lane's result writes
    if (tid == 0) C->nresults = nres;
    if (nres >= a.num_results) {
      finish_lightest(a, L, ctx, shot, nres, t0);
      return;
    }
  }
  // Rank the children by (score desc, generation asc); children of parents
  // that could not branch do not exist.
  for (int i = tid; i < nch; i += blockDim.x) {
    int rank = -1;
    if (C->parent_next_pos[i >> 1] >= 0) {
      const float si = C->child_score[i];
      rank = 0;
      for (int q = 0; q < nch; ++q) {
        if (q == i || C->parent_next_pos[q >> 1] < 0) continue;
        const float sq = C->child_score[q];
        if (sq > si || (sq == si && q < i)) ++rank;
      }
    }
    order[i] = rank;
  }
  __syncthreads();
  if (tid == 0) {
    int cnt = 0;
    int32_t* byrank = L.i32(kOffByrank);
    int32_t* mark = L.i32(kOffMark);
    for (int i = 0; i < nch; ++i)
      if (order[i] >= 0) {
        byrank[order[i]] = i;
        ++cnt;
      }
    const int ns = cnt < a.bw ? cnt : a.bw;
    int action;  // 0: next round, 1: fail with best survivor, 2: fail with the initial decision
    int nbranch = 0;
    if (round >= a.max_rounds) {
      action = ns > 0 ? 1 : 2;
    } else {
      for (int q = 0; q < ns; ++q) nbranch += C->child_next_pos[byrank[q]] >= 0;
      action = nbranch > 0 ? 0 : 2;
    }
    if (action != 0 && nres > 0) action = 3;  // the search ends with results: the lightest
    misc[8] = action;
    misc[9] = ns > 0 ? C->slots[nset + byrank[0]] : 0;
    if (action == 0) {
      const int ntot = 3 * a.bw;
      int32_t* newslots = L.i32(kOffNewslots);
      for (int s = 0; s < ntot; ++s) mark[s] = 0;
      for (int q = 0; q < ns; ++q) {
        const int c = byrank[q];
        newslots[q] = C->slots[nset + c];
        mark[newslots[q]] = 1;
        C->parent_next_pos[q] = C->child_next_pos[c];
      }
      int k = ns;
      for (int q = 0; q < ntot; ++q) {
        const int s = C->slots[q];
        if (!mark[s]) newslots[k++] = s;
      }
      for (int q = 0; q < ntot; ++q) C->slots[q] = newslots[q];
      C->nset = ns;
      C->round = round + 1;
      C->best_gen = 0x7FFFFFFF;
      C->pending = 2 * nbranch;
      __threadfence();  // one release for the whole batch of pushes
      for (int q = 0; q < ns; ++q)
        if (C->parent_next_pos[q] >= 0) {
          ring_push(&a.st->work, a.work_ring, ((uint32_t)ctx << 8) | (uint32_t)(2 * q), true);
          ring_push(&a.st->work, a.work_ring, ((uint32_t)ctx << 8) | (uint32_t)(2 * q + 1), true);
        }
    }
  }
  __syncthreads();
  const int action = misc[8];
  const int s0 = misc[9];
  __syncthreads();
  if (action == 3) {
    finish_lightest(a, L, ctx, shot, nres, t0);
  } else if (action == 1) {
    finish_deep(a, L, ctx, shot, (const uint32_t*)(slot_ptr(a, ctx, s0) + slot_ehat_off(g)), 0, t0);
  } else if (action == 2) {
    finish_deep(a, L, ctx, shot,
                (const uint32_t*)(slot_ptr(a, ctx, 3 * a.bw) + slot_ehat_off(g)), 0, t0);
  }
}

// Initial BP run of a shot.  `ctx` is the workgroup's spare context; the
// return value tells whether the shot went deep and consumed it.
template <int CPT, int PW>
__device__ __forceinline__ bool process_init(const BatchArgs& a, const Lds& L,
                                             Res<CPT, PW>& R, long long shot, int ctx,
                                             unsigned long long& nruns, unsigned long long& niters,
                                             int& work_hint, long long next_shot, long long& pf_shot,
                                             uint32_t& pf, long long& flips_row, long long& d1_shot) {
  const DevGraph& g = a.g;
  // The clock is read only when latencies are asked for, by one wave: the
  // read returns on the same counter as LDS operations.
  const uint32_t t0 = (a.lat && threadIdx.x < 64) ? dev_clock() : 0u;
  RunRegs<CPT> rg;
  const long long row = io_row(a, shot);
  EarlyLoads el;
  el.next_syn = next_shot >= 0 ? a.syn + next_shot * g.m : nullptr;
  el.work_count = &a.st->work.count;
  el.lmask = g.lmask;
  el.work_hint = -1;
  el.lm = 0ull;
  // Batched calls write the next shot's D(1) right after this shot's output,
  // while other waves finish theirs and thread 0 schedules (see below).
  const bool spec = !a.stream && next_shot >= 0 && a.fi.enabled && a.init_iters >= 1;
  el.fi = spec ? &a.fi : nullptr;
  el.rt[0] = el.rt[1] = make_uint4(0u, 0u, 0u, 0u);
  const bool d1_done = d1_shot == shot;
  d1_shot = -1;
  const RunRes rr = bp_run<CPT, PW>(g, L, R, nullptr, nullptr, 0, a.syn + row * g.m,
                                    a.init_iters, true, a.alpha, nullptr, 0, rg, &a.st->error,
                                    &a.fi, pf_shot == shot, pf, a.alpha_sched, a.n_sched, &el,
                                    d1_done);
  pf_shot = -1;
  nruns += 1;
  niters += rr.iters;
  const bool many = a.num_results > 1;
  if ((rr.conv && !many) || a.max_rounds == 0) {
    // The work queue's length was read during the run: the next scheduling
    // step skips the queue when it was empty.
    emit_from_regs<CPT, PW>(g, L, rg.ebits, a.corr + row * g.n, a.flips + row * g.k, el,
                            next_shot, pf_shot, pf, work_hint, !a.stream);
    if (!a.stream) flips_row = row;  // written after the next scheduling barrier
    const uint32_t lat = (a.lat && threadIdx.x == 0) ? dev_clock() - t0 : 0u;
    if (spec && rr.iters >= 1) {
      // The messages of this run are no longer read (the other waves only
      // read the residual and their registers from here on), so the next
      // shot's iteration-1 messages can go in now.
      uint32_t sb[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) sb[q] = (pf >> (8 * q)) & 1u;
      write_d1<CPT, PW>(g, L, R, &a.fi, el.rt, sb);
      d1_shot = next_shot;
    }
    if (threadIdx.x == 0) {
      a.conv[row] = (uint8_t)rr.conv;
      if (a.lat) put_latency(a, row, lat);
      __hip_atomic_fetch_add(&a.st->done, 1ull, __ATOMIC_RELAXED, AGENT);
    }
    publish_done(a, shot);
    return false;
  }
  float score;
  int next_pos;
  score_next<CPT>(g, L, rg, rr.iters, &score, &next_pos);
  Ctx* C = a.ctxs + ctx;
  for (int s = threadIdx.x; s < 3 * a.bw; s += blockDim.x) C->slots[s] = s;
  char* seed = slot_ptr(a, ctx, 0);
  store_msg(g, L, (float*)seed);
  store_bits<CPT>(g, (uint32_t*)(slot_ptr(a, ctx, 3 * a.bw) + slot_ehat_off(g)), rg.ebits);
  if (rr.conv) {  // num_results > 1: the initial solution is the first result
    store_bits<CPT>(g, a.results + (size_t)ctx * a.num_results * g.words_n, rg.ebits);
    weight_hash<CPT>(g, L, a.lam64, rg.ebits, &C->res_wt[0], &C->res_hash[0]);
  }
  if (threadIdx.x == 0) {
    *(int32_t*)(seed + slot_pairs_off(g)) = 0;
    C->shot = (int32_t)shot;
    C->round = 1;
    C->nset = 1;
    C->pending = 2;
    C->best_gen = 0x7FFFFFFF;
    C->nresults = rr.conv ? 1 : 0;
    C->t_start = t0;
    C->parent_next_pos[0] = next_pos;
    __hip_atomic_fetch_add(&a.st->deep, 1ull, __ATOMIC_RELAXED, AGENT);
  }
  __syncthreads();  // then thread 0's release publishes every lane's slot writes
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    ring_push(&a.st->work, a.work_ring, ((uint32_t)ctx << 8) | 0u, true);
    ring_push(&a.st->work, a.work_ring, ((uint32_t)ctx << 8) | 1u, true);
  }
  return true;
}

template <int CPT, int PW>
__device__ __forceinline__ void process_child(const BatchArgs& a, const Lds& L,
                                              Res<CPT, PW>& R, uint32_t item,
                                              unsigned long long& nruns,
                                              unsigned long long& niters) {
  const DevGraph& g = a.g;
  const int ctx = (int)(item >> 8), c = (int)(item & 255u);
  Ctx* C = a.ctxs + ctx;
  const int tid = threadIdx.x;
  int32_t* misc = L.misc();
  if (tid == 0) {  // the pop of `item` acquired what the round's selection released
    misc[10] = C->nset;
    misc[11] = C->slots[c >> 1];
    misc[12] = C->slots[C->nset + c];
    misc[13] = C->parent_next_pos[c >> 1];
    misc[14] = C->shot;
    misc[15] = __hip_atomic_load(&C->best_gen, __ATOMIC_RELAXED, AGENT) < c;
  }
  __syncthreads();  // every lane's reads follow thread 0's acquire
  const int ps = misc[11], ms = misc[12], npos = misc[13], skip = misc[15];
  const long long shot = misc[14];
  char* pslot = slot_ptr(a, ctx, ps);
  char* mslot = slot_ptr(a, ctx, ms);
  int state = 2;
  if (!skip) {
    const int np = *(const int32_t*)(pslot + slot_pairs_off(g));
    const int32_t* pp = (const int32_t*)(pslot + slot_pairs_off(g) + 16);
    int32_t* mp = (int32_t*)(mslot + slot_pairs_off(g) + 16);
    for (int q = tid; q <= np; q += blockDim.x) {
      const int32_t v = q < np ? pp[q] : ((npos << 1) | (c & 1));
      L.pairs()[q] = v;
      mp[q] = v;
    }
    if (tid == 0) *(int32_t*)(mslot + slot_pairs_off(g)) = np + 1;
    __syncthreads();
    RunRegs<CPT> rg;
    const bool many = a.num_results > 1;  // converged children keep branching; no cancellation
    const RunRes rr = bp_run<CPT, PW>(g, L, R, (const float*)pslot, nullptr, np + 1,
                                      a.syn + io_row(a, shot) * g.m, a.round_iters, true, a.alpha,
                                      many ? nullptr : &C->best_gen, c, rg, &a.st->error, nullptr,
                                      false, 0u, a.alpha_sched, a.n_sched);
    nruns += 1;
    niters += rr.iters;
    uint32_t* mbitsv = (uint32_t*)(mslot + slot_ehat_off(g));
    const uint32_t filled = (rg.ebits & ~rg.mbits) | rg.vbits;
    if (rr.cancelled) {
      state = 2;
    } else if (rr.conv && !many) {
      state = 1;
      store_bits<CPT>(g, mbitsv, filled);
      if (tid == 0) __hip_atomic_fetch_min(&C->best_gen, c, __ATOMIC_RELAXED, AGENT);
    } else {
      state = rr.conv ? 1 : 0;
      float score;
      int next_pos;
      score_next<CPT>(g, L, rg, rr.iters, &score, &next_pos);
      store_msg(g, L, (float*)mslot);
      store_bits<CPT>(g, mbitsv, filled);
      if (rr.conv) weight_hash<CPT>(g, L, a.lam64, filled, &C->child_wt[c], &C->child_hash[c]);
      if (tid == 0) {
        C->child_score[c] = score;
        C->child_next_pos[c] = next_pos;
      }
    }
  }
  if (tid == 0) C->child_state[c] = state;
  __syncthreads();  // then thread 0's acquire-release decrement publishes every lane's writes
  if (tid == 0) {
    const int left = __hip_atomic_fetch_add(&C->pending, -1, __ATOMIC_ACQ_REL, AGENT);
    misc[16] = (left == 1);
  }
  __syncthreads();
  const int last = misc[16];
  __syncthreads();
  if (last) select_round(a, L, ctx);  // after thread 0's acquire and two barriers
}

// Persistent batched decoder.  Each workgroup holds one spare context for
// the shot whose initial run fails; it claims shots in chunks and prefers
// queued child runs of shots already in the beam.
template <int CPT, int PW>
__global__ void __launch_bounds__(max_block_for(CPT)) k_batched(BatchArgs a) {
  extern __shared__ __align__(16) char lds_raw[];
  const Lds L{lds_raw};
  const int tid = threadIdx.x;
  if (!a.stream) {
    // Batched: nothing to do once every shot is done (the screen may have
    // finished them all); a launch beside the screen ends at once unless the
    // whole screen launch has begun (it must not keep the screen off the
    // device, since it may wait for the screen's list).
    if (tid == 0) {
      bool quit = __hip_atomic_load(&a.st->done, __ATOMIC_RELAXED, AGENT) >= (unsigned long long)a.shots;
      if (a.helper &&
          __hip_atomic_load(&a.st->screen_begun, __ATOMIC_RELAXED, AGENT) < (uint32_t)a.screen_grid)
        quit = true;
      L.misc()[30] = quit ? 1 : 0;
    }
    __syncthreads();
    if (L.misc()[30]) return;
  }
  Res<CPT, PW> R;
  load_res<CPT, PW>(a.g, L, R);
  unsigned long long nruns = 0, niters = 0;
  if (a.stream) {
    // Serving.  A launch that the host has replaced (it waited behind another
    // persistent kernel on a shared hardware queue) ends before touching
    // any state.
    if (tid == 0)
      L.misc()[31] = __hip_atomic_load(a.gen_host, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) != a.gen;
    __syncthreads();
    if (L.misc()[31]) return;
    if (tid == 0) {
      __hip_atomic_store(a.begun, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      // The last workgroup to begin tells the host that all are resident
      // (the count runs on over relaunches of the same decoder).
      const uint32_t k = __hip_atomic_fetch_add(&a.st->started_wgs, 1u, __ATOMIC_RELAXED, AGENT) + 1u;
      if (k % gridDim.x == 0) __hip_atomic_store(a.started, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
  int spare = -1;                 // thread 0 only
  long long cnext = 0, cend = 0;  // thread 0 only: claimed positions [cnext, cend)
  // Thread 0 only: positions to claim, and the shot at a position (the
  // screen's list, written by the previous kernel, or the identity).
  long long nclaim = a.shots;
  if (a.shot_list && tid == 0) nclaim = __hip_atomic_load(&a.st->listed, __ATOMIC_RELAXED, AGENT);
  // Shots per claim: 8, fewer when there are under 32 per workgroup (a short
  // list from the screen), so that every workgroup gets some.
  // (one at a time beside the screen, whose list is still growing)
  const long long chunk =
      a.helper ? 1 : nclaim >= 32ll * gridDim.x ? 8 : nclaim >= 4ll * gridDim.x ? 2 : 1;
  auto shot_at = [&](long long q) -> long long { return a.shot_list ? (long long)a.shot_list[q] : q; };
  // Beside the screen: an entry below the listed count is written at once by
  // the running screen wave that counted it.  When latencies are measured it
  // is read with acquire order, so that what the screen wrote before it (the
  // shot's latency so far) is seen; the shot itself needs nothing else the
  // screen wrote, and an acquire (an invalidation of this XCD's L2, which
  // the screen's waves there rely on) is not paid otherwise.
  auto listed_at = [&](long long q) -> long long {
    for (;;) {
      const int32_t v = a.lat ? __hip_atomic_load(&a.shot_list[q], __ATOMIC_ACQUIRE, AGENT)
                              : __hip_atomic_load(&a.shot_list[q], __ATOMIC_RELAXED, AGENT);
      if (v >= 0) return (long long)v;
      __builtin_amdgcn_s_sleep(2);
    }
  };
  bool exhausted = false;         // thread 0 only
  int work_hint = -1;             // thread 0 only: queue length read late in the last step, -1 unknown
  bool idling = false;            // thread 0 only, serving: in an idle stretch since idle_since
  int backoff = 1;                // thread 0 only, serving: sleep units of the next idle pass
  uint32_t idle_since = 0;
  long long pf_shot = -1;         // shot whose syndrome bits `pf` holds (uniform)
  uint32_t pf = 0;
  long long flips_row = -1;       // output row whose flips wait in the second accumulator
  long long d1_shot = -1;         // shot whose iteration-1 messages are already in LDS
  int32_t* misc = L.misc();
  for (int it = 0;; ++it) {
    opaque_res<CPT, PW>(R);
    int32_t* box = misc + 20 + 6 * (it & 1);  // alternating slots: one barrier per step
    if (tid == 0) {
      int kind = 0;
      uint32_t item = 0;
      long long shot = -1;
      const bool try_work = work_hint != 0;
      work_hint = -1;
      if (try_work && ring_pop(&a.st->work, a.work_ring, &item)) {
        kind = 1;
      } else if (a.stream) {
        // Serving: take the next published shot, if any, with a spare context.
        if (spare < 0) {
          uint32_t cx;
          if (ring_pop(&a.st->ctxq, a.ctx_ring, &cx)) spare = (int)cx;
        }
        if (spare >= 0) {
          const unsigned long long pub = __hip_atomic_load(&a.st->pub, __ATOMIC_ACQUIRE, AGENT);
          unsigned long long b = __hip_atomic_load(&a.st->next_shot, __ATOMIC_RELAXED, AGENT);
          if (b < pub && __hip_atomic_compare_exchange_strong(&a.st->next_shot, &b, b + 1ull,
                                                              __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                              AGENT)) {
            // The syndrome was written by the host before it published the count.
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
            kind = 2;
            shot = (long long)b;
            item = (uint32_t)spare;
          }
        }
      } else if (!exhausted) {
        if (spare < 0) {
          uint32_t cx;
          if (ring_pop(&a.st->ctxq, a.ctx_ring, &cx)) spare = (int)cx;
        }
        if (spare >= 0 && a.helper) {
          // A claimed position past the listed count is kept until the
          // screen lists a shot there, or ends without doing so.
          if (cnext >= cend) {
            cnext = (long long)__hip_atomic_fetch_add(&a.st->next_shot, 1ull, __ATOMIC_RELAXED, AGENT);
            cend = cnext + 1;
          }
          if (cnext >= nclaim) {
            nclaim = __hip_atomic_load(&a.st->listed, __ATOMIC_RELAXED, AGENT);
            if (cnext >= nclaim && __hip_atomic_load(&a.st->screen_live, __ATOMIC_RELAXED, AGENT) <= 0) {
              nclaim = __hip_atomic_load(&a.st->listed, __ATOMIC_RELAXED, AGENT);  // final
              if (cnext >= nclaim) exhausted = true;
            }
          }
          if (cnext < nclaim) {
            kind = 2;
            shot = listed_at(cnext++);
            item = (uint32_t)spare;
          }
        } else if (spare >= 0) {
          if (cnext >= cend) {
            const unsigned long long b = __hip_atomic_fetch_add(
                &a.st->next_shot, (unsigned long long)chunk, __ATOMIC_RELAXED, AGENT);
            cnext = (long long)b;
            cend = (long long)b + chunk < nclaim ? (long long)b + chunk : nclaim;
            if (cnext >= nclaim) exhausted = true;
          }
          if (cnext < cend) {
            kind = 2;
            shot = shot_at(cnext++);
            item = (uint32_t)spare;
            if (cnext >= cend && !exhausted) {  // claim the next chunk now: its first shot is prefetched
              const unsigned long long b = __hip_atomic_fetch_add(
                  &a.st->next_shot, (unsigned long long)chunk, __ATOMIC_RELAXED, AGENT);
              cnext = (long long)b;
              cend = (long long)b + chunk < nclaim ? (long long)b + chunk : nclaim;
              if (cnext >= nclaim) exhausted = true;
            }
          }
        }
      }
      if (kind == 0) {
        if (a.stream) {
          // One idle workgroup at a time reads the host's counters (over the
          // bus) and mirrors them for the others.
          if (__hip_atomic_load(&a.st->poll_token, __ATOMIC_RELAXED, AGENT) == 0u) {
            uint32_t zero = 0u;
            if (__hip_atomic_compare_exchange_strong(&a.st->poll_token, &zero, 1u, __ATOMIC_ACQUIRE,
                                                     __ATOMIC_RELAXED, AGENT)) {
              const unsigned long long ph =
                  __hip_atomic_load(a.pub_host, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
              const uint32_t sh = __hip_atomic_load(a.stop_host, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
              if (ph > __hip_atomic_load(&a.st->pub, __ATOMIC_RELAXED, AGENT))
                __hip_atomic_store(&a.st->pub, ph, __ATOMIC_RELEASE, AGENT);
              if (sh) __hip_atomic_store(&a.st->stop, 1u, __ATOMIC_RELEASE, AGENT);
              __hip_atomic_store(&a.st->poll_token, 0u, __ATOMIC_RELEASE, AGENT);
            }
          }
          const uint32_t now = dev_clock();
          if (!idling) {
            idling = true;
            idle_since = now;
          }
          if (__hip_atomic_load(&a.st->stop, __ATOMIC_ACQUIRE, AGENT) ||
              now - idle_since > a.idle_limit)
            kind = 3;
          else {
            // Idle workgroups back off (up to about 8K cycles a pass), so
            // that their polling does not crowd the queue counters' cache
            // lines when a decoder has many more workgroups than requests.
            for (int u = 0; u < backoff; ++u) __builtin_amdgcn_s_sleep(16);
            backoff = backoff < 8 ? 2 * backoff : 8;
          }
        } else if (__hip_atomic_load(&a.st->done, __ATOMIC_ACQUIRE, AGENT) >=
                   (unsigned long long)a.shots) {
          kind = 3;
        } else {
          // Waiting for child runs of deep shots: back off too (up to about
          // 4K cycles a pass), as thousands of small workgroups polling the
          // same counters slow down the atomics of the busy ones.
          for (int u = 0; u < backoff; ++u) __builtin_amdgcn_s_sleep(8);
          backoff = backoff < 8 ? 2 * backoff : 8;
        }
      } else {
        idling = false;
        backoff = 1;
      }
      box[0] = kind;
      box[1] = (int)item;
      box[2] = (int)(shot & 0xFFFFFFFF);
      box[3] = (int)(shot >> 32);
      const long long nx = (kind == 2 && cnext < cend && !a.helper) ? shot_at(cnext) : -1;
      box[4] = (int)(nx & 0xFFFFFFFF);
      box[5] = (int)(nx >> 32);
    }
    // LDS only: the previous step's output stores may still be in flight.
    lds_barrier();
    const int kind = box[0];
    const uint32_t item = (uint32_t)box[1];
    const long long shot = (long long)(uint32_t)box[2] | ((long long)box[3] << 32);
    const long long next_shot = (long long)(uint32_t)box[4] | ((long long)box[5] << 32);
    if (flips_row >= 0) {
      flip_write_late(a.g, L, a.flips + flips_row * a.g.k);
      flips_row = -1;
    }
    if (kind != 2) d1_shot = -1;
    if (kind == 3) break;
    if (kind == 2) {
      if (process_init<CPT, PW>(a, L, R, shot, (int)item, nruns, niters, work_hint, next_shot,
                                pf_shot, pf, flips_row, d1_shot) &&
          tid == 0)
        spare = -1;
    } else if (kind == 1) {
      process_child<CPT, PW>(a, L, R, item, nruns, niters);
    }
  }
  if (tid == 0) {
    // Serving: the spare context goes back, since a decoder that ends when
    // idle is started again later and needs every context.  (A batched
    // call's next launch resets the context queue.)
    if (a.stream && spare >= 0) ring_push(&a.st->ctxq, a.ctx_ring, (uint32_t)spare);
    __hip_atomic_fetch_add(&a.st->runs, nruns, __ATOMIC_RELAXED, AGENT);
    __hip_atomic_fetch_add(&a.st->iterations, niters, __ATOMIC_RELAXED, AGENT);
  }
}

// A single BP run launched on its own (grid of one workgroup).
template <int CPT, int PW>
__global__ void __launch_bounds__(max_block_for(CPT)) k_single(SingleArgs a) {
  extern __shared__ __align__(16) char lds_raw[];
  const DevGraph& g = a.g;
  const Lds L{lds_raw};
  Res<CPT, PW> R;
  load_res<CPT, PW>(g, L, R);
  const int tid = threadIdx.x, B = blockDim.x;
  for (int q = tid; q < a.npairs; q += B) L.pairs()[q] = a.pairs[q];
  __syncthreads();
  RunRegs<CPT> rg;
  const RunRes rr = bp_run<CPT, PW>(g, L, R, a.parent, a.parent_csc, a.npairs, a.syn, a.max_iters,
                                    a.stop != 0, a.alpha, nullptr, 0, rg, a.error, nullptr, false, 0u,
                                    a.alpha_sched, a.n_sched);
  float score = 0.f;
  int next_pos = -1;
  if (a.want_score) score_next<CPT>(g, L, rg, rr.iters, &score, &next_pos);
  if (a.out_msg && (!rr.conv || a.keep_msg)) store_msg(g, L, a.out_msg);
  const uint32_t filled = (rg.ebits & ~rg.mbits) | rg.vbits;
  if (a.out_ehat_bits) store_bits<CPT>(g, a.out_ehat_bits, filled);
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int j = c * B + tid;
    if (j >= g.n) continue;
    const bool mk = (rg.mbits >> c) & 1u;
    if (a.out_sumllr) a.out_sumllr[j] = mk ? 0.f : rg.sumllr[c];
    if (a.out_ehat)
      a.out_ehat[j] = (uint8_t)(((rr.conv ? filled : (rg.ebits & ~rg.mbits)) >> c) & 1u);
    if (a.out_csc) {
      const int st = (int)(g.colinfo[j] & 0xFFFFFFu), dg = col_deg(R, c);
      for (int e = 0; e < dg; ++e) a.out_csc[st + e] = L.msg()[g.cedge[st + e] & 0xFFFFu];
    }
  }
  if (tid == 0) {
    a.result[0] = rr.iters;
    a.result[1] = rr.conv;
    a.result[2] = next_pos;
    a.result[3] = __float_as_int(score);
  }
}

}  // namespace dev

// Per-PW entry points (defined in bsd_kernels_pw<PW>.hip).
template <int PW>
hipError_t launch_single_pw(const SingleArgs& a, int block, int cpt, size_t lds, hipStream_t s);
template <int PW>
hipError_t launch_batched_pw(const BatchArgs& a, int grid, int block, int cpt, size_t lds,
                             hipStream_t s);
template <int PW>
hipError_t limits_pw(int cpt, size_t lds);
template <int PW>
hipError_t occupancy_pw(int cpt, int block, size_t lds, int* n);

#define BSD_DECLARE_PW(P)                                                                        \
  template <> hipError_t launch_single_pw<P>(const SingleArgs&, int, int, size_t, hipStream_t);  \
  template <> hipError_t launch_batched_pw<P>(const BatchArgs&, int, int, int, size_t,           \
                                              hipStream_t);                                      \
  template <> hipError_t limits_pw<P>(int, size_t);                                              \
  template <> hipError_t occupancy_pw<P>(int, int, size_t, int*);
BSD_DECLARE_PW(1)
BSD_DECLARE_PW(2)
BSD_DECLARE_PW(3)
BSD_DECLARE_PW(4)
#undef BSD_DECLARE_PW

}  // namespace bsd

// Instantiates the per-PW entry points for CPT = 1..16 (used by bsd_kernels_pw<PW>.hip).
#define BSD_DEFINE_PW(PWV)                                                                       \
  namespace bsd {                                                                                \
  namespace {                                                                                    \
  template <int CPT>                                                                             \
  hipError_t ls_(const SingleArgs& a, int block, size_t lds, hipStream_t s) {                    \
    hipLaunchKernelGGL((dev::k_single<CPT, PWV>), dim3(1), dim3(block), lds, s, a);              \
    return hipGetLastError();                                                                    \
  }                                                                                              \
  template <int CPT>                                                                             \
  hipError_t lb_(const BatchArgs& a, int grid, int block, size_t lds, hipStream_t s) {           \
    hipLaunchKernelGGL((dev::k_batched<CPT, PWV>), dim3(grid), dim3(block), lds, s, a);          \
    return hipGetLastError();                                                                    \
  }                                                                                              \
  template <int CPT>                                                                             \
  hipError_t lim_(size_t lds) {                                                                  \
    hipError_t e = hipFuncSetAttribute((const void*)dev::k_single<CPT, PWV>,                     \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);    \
    if (e != hipSuccess) return e;                                                               \
    return hipFuncSetAttribute((const void*)dev::k_batched<CPT, PWV>,                            \
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);            \
  }                                                                                              \
  template <int CPT>                                                                             \
  hipError_t occ_(int block, size_t lds, int* n) {                                               \
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, dev::k_batched<CPT, PWV>, block, lds); \
  }                                                                                              \
  }                                                                                              \
  template <>                                                                                    \
  hipError_t launch_single_pw<PWV>(const SingleArgs& a, int block, int cpt, size_t lds,          \
                                   hipStream_t s) {                                              \
    BSD_CPT_SWITCH(cpt, ls_, (a, block, lds, s))                                                 \
  }                                                                                              \
  template <>                                                                                    \
  hipError_t launch_batched_pw<PWV>(const BatchArgs& a, int grid, int block, int cpt,            \
                                    size_t lds, hipStream_t s) {                                 \
    BSD_CPT_SWITCH(cpt, lb_, (a, grid, block, lds, s))                                           \
  }                                                                                              \
  template <>                                                                                    \
  hipError_t limits_pw<PWV>(int cpt, size_t lds) { BSD_CPT_SWITCH(cpt, lim_, (lds)) }            \
  template <>                                                                                    \
  hipError_t occupancy_pw<PWV>(int cpt, int block, size_t lds, int* n) {                         \
    BSD_CPT_SWITCH(cpt, occ_, (block, lds, n))                                                   \
  }                                                                                              \
  }

#define BSD_CPT_SWITCH(cpt, F, ARGS)            \
  switch (cpt) {                                \
    case 1: return F<1> ARGS;                   \
    case 2: return F<2> ARGS;                   \
    case 3: return F<3> ARGS;                   \
    case 4: return F<4> ARGS;                   \
    case 5: return F<5> ARGS;                   \
    case 6: return F<6> ARGS;                   \
    case 7: return F<7> ARGS;                   \
    case 8: return F<8> ARGS;                   \
    case 9: return F<9> ARGS;                   \
    case 10: return F<10> ARGS;                 \
    case 11: return F<11> ARGS;                 \
    case 12: return F<12> ARGS;                 \
    case 13: return F<13> ARGS;                 \
    case 14: return F<14> ARGS;                 \
    case 15: return F<15> ARGS;                 \
    case 16: return F<16> ARGS;                 \
    case 17: return F<17> ARGS;                 \
    case 20: return F<20> ARGS;                 \
    case 24: return F<24> ARGS;                 \
    case 32: return F<32> ARGS;                 \
    default: return hipErrorInvalidValue;       \
  }
