// HIP kernels of the beam-search decoder for gfx950.
//
// One workgroup runs one BP run at a time with the run's edge messages held
// in LDS (fp32, one word per Tanner edge, jagged-diagonal order).  A run is
// the masked min-sum BP of Algorithm 2: eq. (1) in the check phase (one lane
// per detector row), eqs. (2)-(4) in the variable phase (lanes own columns
// c * blockDim + tid), the syndrome test through an LDS residual bit-vector,
// and at the end of a failed run the path score and the least reliable node
// of Algorithm 3.  The persistent kernel pulls initial runs (one per shot)
// and masked child runs (one per shot, path and value) from device queues;
// the workgroup that finishes the last child of a round performs the
// selection of Algorithm 3 (first converged child in exploration order, or
// the beam_width best paths) and queues the next round.
//
// Floating-point order matches the natural order of the paper's formulas:
// sums run left to right over neighbours in ascending row index, E of
// eq. (2) is a literal exclusive sum, sum_LLR accumulates in iteration
// order, and the path score sums |sum_LLR| as an aligned pairwise tree over
// column index.  No FMA contraction (built with -ffp-contract=off).

#include "bsd_internal.h"

namespace bsd {

namespace {

constexpr int AGENT = __HIP_MEMORY_SCOPE_AGENT;

struct LdsMap {
  float* msg;
  uint32_t* sprime;  // masked syndrome s' by row rank
  uint32_t* resid;   // s' xor H e-hat
  int32_t* pairs;    // packed (col << 1) | val
  float* redf;       // [kMaxCpt][kMaxWaves] score partials
  float* aminv;      // [kMaxWaves]
  int32_t* aminj;    // [kMaxWaves]
  uint32_t* flw;     // [2 * kMaxWaves] logical flip partials
  int32_t* misc;     // [32]
  int32_t* order;    // [2 * kMaxBw] rank of each child
  int32_t* byrank;   // [2 * kMaxBw] child of each rank
  int32_t* mark;     // [3 * kMaxBw + 1]
  int32_t* newslots; // [3 * kMaxBw]
  float* part;       // [kMaxCpt] score partials per column block
};

__device__ __forceinline__ LdsMap lds_map(const DevGraph& g, char* lds) {
  LdsMap L;
  char* p = lds;
  L.msg = (float*)p;
  p += (size_t)g.nnz_pad * 4;
  L.sprime = (uint32_t*)p;
  p += (size_t)g.words_m * 4;
  L.resid = (uint32_t*)p;
  p += (size_t)g.words_m * 4;
  L.pairs = (int32_t*)p;
  p += kMaxRounds * 4;
  L.redf = (float*)p;
  p += kMaxCpt * kMaxWaves * 4;
  L.aminv = (float*)p;
  p += kMaxWaves * 4;
  L.aminj = (int32_t*)p;
  p += kMaxWaves * 4;
  L.flw = (uint32_t*)p;
  p += 2 * kMaxWaves * 4;
  L.misc = (int32_t*)p;
  p += 32 * 4;
  L.order = (int32_t*)p;
  p += 2 * kMaxBw * 4;
  L.byrank = (int32_t*)p;
  p += 2 * kMaxBw * 4;
  L.mark = (int32_t*)p;
  p += (3 * kMaxBw + 1) * 4;
  L.newslots = (int32_t*)p;
  p += 3 * kMaxBw * 4;
  L.part = (float*)p;
  return L;
}

}  // namespace

size_t lds_bytes_for(const DevGraph& g, int /*block*/, int /*cpt*/) {
  size_t b = (size_t)g.nnz_pad * 4 + (size_t)g.words_m * 8 + kMaxRounds * 4 +
             kMaxCpt * kMaxWaves * 4 + kMaxWaves * 8 + 2 * kMaxWaves * 4 + 32 * 4 +
             4 * kMaxBw * 4 + (3 * kMaxBw + 1) * 4 + 3 * kMaxBw * 4 + kMaxCpt * 4;
  return (b + 15) & ~(size_t)15;
}

namespace {

template <int CPT>
struct Cols {
  float sumllr[CPT];
  uint32_t info[CPT];
  float lam[CPT];
  uint32_t ebits;  // hard decision of unmasked columns at the last iteration
  uint32_t mbits;  // masked columns
  uint32_t vbits;  // values of masked columns
};

struct RunRes {
  int iters;
  int conv;
  int cancelled;
};

__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Eq. (1) for the detector row of rank r, in place: E(t-1) -> D(t) on the
// unmasked edges (masked edges hold +inf and are skipped).
__device__ __forceinline__ void check_row(const DevGraph& g, float* msg, const uint32_t* sprime, int r,
                                 float alpha) {
  const int dg = g.deg_of_rank[r];
  const int kmax = __builtin_amdgcn_readfirstlane(dg);  // ranks are sorted by degree
  bool neg = (sprime[r >> 5] >> (r & 31)) & 1u;
  float m1 = kLlrMax, m2 = kLlrMax;
  int arg = -1;
  for (int k = 0; k < kmax; ++k) {
    if (k < dg) {
      const float v = msg[g.diag_ptr[k] + r];
      const float a = fabsf(v);
      neg ^= (v < 0.f);
      if (a < m1) {
        m2 = m1;
        m1 = a;
        arg = k;
      } else if (a < m2) {
        m2 = a;
      }
    }
  }
  const float d1 = fminf(alpha * m1, kLlrMax);
  const float d2 = fminf(alpha * m2, kLlrMax);
  for (int k = 0; k < kmax; ++k) {
    if (k < dg) {
      const int p = g.diag_ptr[k] + r;
      const float v = msg[p];
      if (v != __builtin_inff()) {
        const float mag = (k == arg) ? d2 : d1;
        msg[p] = (neg ^ (v < 0.f)) ? -mag : mag;
      }
    }
  }
}

// Eqs. (2)-(4) for one column with at most D edges (D uniform over the wave).
template <int D>
__device__ __forceinline__ void var_col(const DevGraph& g, float* msg, uint32_t* resid, uint32_t info,
                               float lam, bool active, float& sl, uint32_t& eb) {
  const int st = (int)(info & 0xFFFFFFu);
  const int dg = (int)(info >> 24);
  uint32_t w[D];
  float d[D];
#pragma unroll
  for (int e = 0; e < D; ++e) {
    if (active && e < dg) {
      w[e] = g.cedge[st + e];
      d[e] = msg[w[e] & 0xFFFFu];
    } else {
      w[e] = 0u;
      d[e] = 0.f;
    }
  }
  if (!active) return;
  float post = lam;  // eq. (3)
#pragma unroll
  for (int e = 0; e < D; ++e) post = post + d[e];
#pragma unroll
  for (int e = 0; e < D; ++e) {
    if (e < dg) {  // eq. (2): exclusive sum in ascending row order
      float x = lam;
#pragma unroll
      for (int f = 0; f < D; ++f)
        if (f != e) x = x + d[f];
      msg[w[e] & 0xFFFFu] = fminf(fmaxf(x, -kLlrMax), kLlrMax);
    }
  }
  sl = sl + post;
  eb = post <= 0.f ? 1u : 0u;  // eq. (4)
  if (eb) {
#pragma unroll
    for (int e = 0; e < D; ++e) {
      if (e < dg) {
        const uint32_t rk = w[e] >> 16;
        atomicXor(&resid[rk >> 5], 1u << (rk & 31));
      }
    }
  }
}

template <int CPT>
__device__ __forceinline__ void var_phase(const DevGraph& g, const LdsMap& L, Cols<CPT>& cs,
                                 const int (&dmax)[CPT]) {
  const int B = blockDim.x;
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int j = c * B + threadIdx.x;
    const bool active = j < g.n && !((cs.mbits >> c) & 1u);
    uint32_t eb = 0;
    switch (dmax[c]) {
      case 0: break;
      case 1: var_col<1>(g, L.msg, L.resid, cs.info[c], cs.lam[c], active, cs.sumllr[c], eb); break;
      case 2: var_col<2>(g, L.msg, L.resid, cs.info[c], cs.lam[c], active, cs.sumllr[c], eb); break;
      case 3: var_col<3>(g, L.msg, L.resid, cs.info[c], cs.lam[c], active, cs.sumllr[c], eb); break;
      case 4: var_col<4>(g, L.msg, L.resid, cs.info[c], cs.lam[c], active, cs.sumllr[c], eb); break;
      case 5: var_col<5>(g, L.msg, L.resid, cs.info[c], cs.lam[c], active, cs.sumllr[c], eb); break;
      case 6: var_col<6>(g, L.msg, L.resid, cs.info[c], cs.lam[c], active, cs.sumllr[c], eb); break;
      case 7: var_col<7>(g, L.msg, L.resid, cs.info[c], cs.lam[c], active, cs.sumllr[c], eb); break;
      default: var_col<8>(g, L.msg, L.resid, cs.info[c], cs.lam[c], active, cs.sumllr[c], eb); break;
    }
    cs.ebits = (cs.ebits & ~(1u << c)) | (eb << c);
  }
}

// One masked BP run (Algorithm 2).  The caller has placed `npairs` packed
// pairs in L.pairs and synchronised.  Warm start from `parent` (LDS order) or
// `parent_csc` (CSC order), else from the priors.  When `cancel` is given the
// run stops early once *cancel < my_gen (a lower generation converged).
template <int CPT>
__device__ __forceinline__ RunRes bp_run(const DevGraph& g, const LdsMap& L, const float* parent,
                         const float* parent_csc, int npairs, const uint8_t* syn, int T,
                         bool stop, float alpha, const int32_t* cancel, int my_gen, Cols<CPT>& cs,
                         uint32_t* err) {
  const int tid = threadIdx.x, B = blockDim.x, lane = tid & 63, wave = tid >> 6;
  cs.mbits = cs.vbits = cs.ebits = 0;
  for (int q = 0; q < npairs; ++q) {
    const int pv = L.pairs[q];
    const int d = (pv >> 1) - tid;
    if (d >= 0 && d % B == 0 && d / B < CPT) {
      cs.mbits |= 1u << (d / B);
      cs.vbits |= (uint32_t)(pv & 1) << (d / B);
    }
  }
  // s by row rank, packed 64 ranks per wave ballot.
  for (int base = 0; base < g.m; base += B) {
    const int r = base + tid;
    uint32_t bit = 0;
    if (r < g.m) {
      const uint32_t b = syn[g.row_of_rank[r]];
      if (b > 1u) atomicOr(err, 1u);
      bit = b & 1u;
    }
    const unsigned long long bal = __ballot(bit);
    if (lane == 0) {
      const int w = (base + wave * 64) >> 5;
      if (w < g.words_m) L.sprime[w] = (uint32_t)bal;
      if (w + 1 < g.words_m) L.sprime[w + 1] = (uint32_t)(bal >> 32);
    }
  }
  if (parent) {
    const float4* src = reinterpret_cast<const float4*>(parent);
    float4* dst = reinterpret_cast<float4*>(L.msg);
    for (int i = tid; i < g.nnz_pad / 4; i += B) dst[i] = src[i];
  }
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int j = c * B + tid;
    cs.sumllr[c] = 0.f;
    cs.info[c] = 0u;
    cs.lam[c] = 0.f;
    if (j < g.n) {
      cs.info[c] = g.colinfo[j];
      cs.lam[c] = g.lambda[j];
      if (!parent) {
        const int st = (int)(cs.info[c] & 0xFFFFFFu), dg = (int)(cs.info[c] >> 24);
        for (int e = 0; e < dg; ++e) {
          const uint32_t w = g.cedge[st + e];
          L.msg[w & 0xFFFFu] = parent_csc ? parent_csc[st + e] : cs.lam[c];
        }
      }
    }
  }
  __syncthreads();
  // Masked nodes leave every check (+inf) and fold their value into s'.
  int dmax[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int st = (int)(cs.info[c] & 0xFFFFFFu), dg = (int)(cs.info[c] >> 24);
    if ((cs.mbits >> c) & 1u) {
      for (int e = 0; e < dg; ++e) {
        const uint32_t w = g.cedge[st + e];
        L.msg[w & 0xFFFFu] = __builtin_inff();
        if ((cs.vbits >> c) & 1u) {
          const uint32_t rk = w >> 16;
          atomicXor(&L.sprime[rk >> 5], 1u << (rk & 31));
        }
      }
    }
    dmax[c] = wave_max_i(((cs.mbits >> c) & 1u) ? 0 : dg);
  }
  __syncthreads();

  RunRes rr{0, 0, 0};
  for (int t = 1; t <= T; ++t) {
    for (int w = tid; w < g.words_m; w += B) L.resid[w] = L.sprime[w];
    for (int r = tid; r < g.m; r += B) check_row(g, L.msg, L.sprime, r, alpha);
    __syncthreads();
    var_phase<CPT>(g, L, cs, dmax);
    __syncthreads();
    int nz = 0;
    for (int w = tid; w < g.words_m; w += B) nz |= (L.resid[w] != 0u);
    if (tid == 0) {
      int c = 0;
      if (cancel) c = __hip_atomic_load(cancel, __ATOMIC_RELAXED, AGENT) < my_gen;
      L.misc[0] = c;
    }
    const int any = __syncthreads_or(nz);
    rr.iters = t;
    rr.conv = any ? 0 : 1;
    if (stop && rr.conv) break;
    if (L.misc[0]) {
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
__device__ __forceinline__ void score_next(const DevGraph& g, const LdsMap& L, const Cols<CPT>& cs, int iters,
                           float* score, int* next_pos) {
  const int tid = threadIdx.x, B = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = B >> 6;
  float bv = __builtin_inff();
  int bj = 0x7FFFFFFF;
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int j = c * B + tid;
    const bool ok = j < g.n && !((cs.mbits >> c) & 1u);
    float a = ok ? fabsf(cs.sumllr[c]) : 0.f;
    if (ok && a < bv) {
      bv = a;
      bj = j;
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) a = a + __shfl_xor(a, o, 64);
    if (lane == 0) L.redf[c * kMaxWaves + wave] = a;
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
    L.aminv[wave] = bv;
    L.aminj[wave] = bj;
  }
  __syncthreads();
  if (tid == 0) {
    // Aligned pairwise tree: over the waves of each column block, then over blocks.
    for (int c = 0; c < CPT; ++c) {
      float* v = L.redf + c * kMaxWaves;
      for (int len = nw; len > 1; len >>= 1)
        for (int i = 0; i < len / 2; ++i) v[i] = v[2 * i] + v[2 * i + 1];
      L.part[c] = v[0];
    }
    int c2 = 1;
    while (c2 < CPT) c2 <<= 1;
    for (int c = CPT; c < c2; ++c) L.part[c] = 0.f;
    for (int len = c2; len > 1; len >>= 1)
      for (int i = 0; i < len / 2; ++i) L.part[i] = L.part[2 * i] + L.part[2 * i + 1];
    const float sc = iters > 0 ? L.part[0] / (float)iters : 0.f;
    float mv = __builtin_inff();
    int mj = 0x7FFFFFFF;
    for (int w = 0; w < nw; ++w) {
      if (L.aminv[w] < mv || (L.aminv[w] == mv && L.aminj[w] < mj)) {
        mv = L.aminv[w];
        mj = L.aminj[w];
      }
    }
    L.misc[4] = __float_as_int(sc);
    L.misc[5] = (mj == 0x7FFFFFFF) ? -1 : mj;
  }
  __syncthreads();
  *score = __int_as_float(L.misc[4]);
  *next_pos = L.misc[5];
  __syncthreads();
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

__device__ __forceinline__ void store_msg(const DevGraph& g, const LdsMap& L, float* dst) {
  const float4* src = reinterpret_cast<const float4*>(L.msg);
  float4* d = reinterpret_cast<float4*>(dst);
  for (int i = threadIdx.x; i < g.nnz_pad / 4; i += blockDim.x) d[i] = src[i];
}

// Reduce per-lane 64-bit logical flip masks over the workgroup; returns the
// total in every thread.
__device__ __forceinline__ unsigned long long block_xor64(const LdsMap& L, unsigned long long f) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  uint32_t lo = (uint32_t)f, hi = (uint32_t)(f >> 32);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    lo ^= __shfl_xor(lo, o, 64);
    hi ^= __shfl_xor(hi, o, 64);
  }
  if (lane == 0) {
    L.flw[2 * wave] = lo;
    L.flw[2 * wave + 1] = hi;
  }
  __syncthreads();
  unsigned long long t = 0;
  for (int w = 0; w < nw; ++w) t ^= (unsigned long long)L.flw[2 * w] | ((unsigned long long)L.flw[2 * w + 1] << 32);
  __syncthreads();
  return t;
}

__device__ __forceinline__ void write_flips(const DevGraph& g, unsigned long long t, uint8_t* flips) {
  for (int r = threadIdx.x; r < g.k; r += blockDim.x) flips[r] = (uint8_t)((t >> r) & 1ull);
}

// Shot output from register-resident hard decisions (columns c*B + tid).
template <int CPT>
__device__ __forceinline__ void emit_from_regs(const DevGraph& g, const LdsMap& L, uint32_t bits, uint8_t* corr,
                               uint8_t* flips) {
  const int B = blockDim.x;
  unsigned long long f = 0;
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int j = c * B + threadIdx.x;
    if (j < g.n) {
      const uint32_t b = (bits >> c) & 1u;
      corr[j] = (uint8_t)b;
      if (b) f ^= g.lmask[j];
    }
  }
  write_flips(g, block_xor64(L, f), flips);
}

// Shot output from a global bit-vector.
__device__ __forceinline__ void emit_from_bits(const DevGraph& g, const LdsMap& L, const uint32_t* bits,
                               uint8_t* corr, uint8_t* flips) {
  unsigned long long f = 0;
  for (int j = threadIdx.x; j < g.n; j += blockDim.x) {
    const uint32_t b = (bits[j >> 5] >> (j & 31)) & 1u;
    corr[j] = (uint8_t)b;
    if (b) f ^= g.lmask[j];
  }
  write_flips(g, block_xor64(L, f), flips);
}

// ---------------------------------------------------------------------------
// Device queues
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool ring_pop(Ring* r, uint32_t* buf, uint32_t* out) {
  if (__hip_atomic_load(&r->count, __ATOMIC_RELAXED, AGENT) <= 0) return false;
  const int c = __hip_atomic_fetch_add(&r->count, -1, __ATOMIC_ACQ_REL, AGENT);
  if (c <= 0) {
    __hip_atomic_fetch_add(&r->count, 1, __ATOMIC_RELAXED, AGENT);
    return false;
  }
  const uint32_t h = __hip_atomic_fetch_add(&r->head, 1u, __ATOMIC_RELAXED, AGENT) & (r->cap - 1u);
  uint32_t x;
  while ((x = __hip_atomic_load(&buf[h], __ATOMIC_ACQUIRE, AGENT)) == 0u) __builtin_amdgcn_s_sleep(2);
  __hip_atomic_store(&buf[h], 0u, __ATOMIC_RELAXED, AGENT);
  *out = x - 1u;
  return true;
}

__device__ __forceinline__ void ring_push(Ring* r, uint32_t* buf, uint32_t item) {
  const uint32_t t = __hip_atomic_fetch_add(&r->tail, 1u, __ATOMIC_RELAXED, AGENT) & (r->cap - 1u);
  while (__hip_atomic_load(&buf[t], __ATOMIC_RELAXED, AGENT) != 0u) __builtin_amdgcn_s_sleep(2);
  __hip_atomic_store(&buf[t], item + 1u, __ATOMIC_RELEASE, AGENT);
  __hip_atomic_fetch_add(&r->count, 1, __ATOMIC_RELEASE, AGENT);
}

__device__ __forceinline__ char* slot_ptr(const BatchArgs& a, int ctx, int s) {
  return a.slots + ((size_t)ctx * a.slots_per_ctx + s) * a.slot_stride;
}

__device__ __forceinline__ uint32_t dev_clock() { return (uint32_t)wall_clock64(); }

// Write the shot's outputs from a slot's hard-decision bits and retire the context.
__device__ __forceinline__ void finish_deep(const BatchArgs& a, const LdsMap& L, int ctx, long long shot,
                            const uint32_t* bits, int converged, uint32_t t_start) {
  const DevGraph& g = a.g;
  emit_from_bits(g, L, bits, a.corr + shot * g.n, a.flips + shot * g.k);
  if (threadIdx.x == 0) {
    a.conv[shot] = (uint8_t)converged;
    if (a.lat) a.lat[shot] = dev_clock() - t_start;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    ring_push(&a.st->ctxq, a.ctx_ring, (uint32_t)ctx);
    __hip_atomic_fetch_add(&a.st->done, 1ull, __ATOMIC_RELEASE, AGENT);
  }
}

// Selection at the end of a round (Algorithm 3 with Appendix B), run by the
// workgroup that finished the round's last child.
__device__ __forceinline__ void select_round(const BatchArgs& a, const LdsMap& L, int ctx) {
  const DevGraph& g = a.g;
  Ctx* C = a.ctxs + ctx;
  const int tid = threadIdx.x;
  const int nset = C->nset, round = C->round, best = C->best_gen;
  const long long shot = C->shot;
  const uint32_t t0 = C->t_start;
  const int nch = 2 * nset;
  if (best != 0x7FFFFFFF) {
    // First converged child in exploration order.
    const int s = C->slots[nset + best];
    finish_deep(a, L, ctx, shot, (const uint32_t*)(slot_ptr(a, ctx, s) + slot_ehat_off(g)), 1, t0);
    return;
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
    L.order[i] = rank;
  }
  __syncthreads();
  if (tid == 0) {
    int cnt = 0;
    int32_t* byrank = L.byrank;
    for (int i = 0; i < nch; ++i)
      if (L.order[i] >= 0) {
        byrank[L.order[i]] = i;
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
    L.misc[8] = action;
    L.misc[9] = ns > 0 ? C->slots[nset + byrank[0]] : 0;
    if (action == 0) {
      const int ntot = 3 * a.bw;
      int32_t* newslots = L.newslots;
      for (int s = 0; s < ntot; ++s) L.mark[s] = 0;
      for (int q = 0; q < ns; ++q) {
        const int c = byrank[q];
        newslots[q] = C->slots[nset + c];
        L.mark[newslots[q]] = 1;
        C->parent_next_pos[q] = C->child_next_pos[c];
      }
      int k = ns;
      for (int q = 0; q < ntot; ++q) {
        const int s = C->slots[q];
        if (!L.mark[s]) newslots[k++] = s;
      }
      for (int q = 0; q < ntot; ++q) C->slots[q] = newslots[q];
      C->nset = ns;
      C->round = round + 1;
      C->best_gen = 0x7FFFFFFF;
      C->pending = 2 * nbranch;
      __threadfence();
      for (int q = 0; q < ns; ++q)
        if (C->parent_next_pos[q] >= 0) {
          ring_push(&a.st->work, a.work_ring, ((uint32_t)ctx << 8) | (uint32_t)(2 * q));
          ring_push(&a.st->work, a.work_ring, ((uint32_t)ctx << 8) | (uint32_t)(2 * q + 1));
        }
    }
  }
  __syncthreads();
  const int action = L.misc[8];
  const int s0 = L.misc[9];
  __syncthreads();
  if (action == 1) {
    finish_deep(a, L, ctx, shot, (const uint32_t*)(slot_ptr(a, ctx, s0) + slot_ehat_off(g)), 0, t0);
  } else if (action == 2) {
    finish_deep(a, L, ctx, shot,
                (const uint32_t*)(slot_ptr(a, ctx, 3 * a.bw) + slot_ehat_off(g)), 0, t0);
  }
}

template <int CPT>
__device__ __forceinline__ void process_init(const BatchArgs& a, const LdsMap& L, long long shot, int ctx,
                             unsigned long long& nruns, unsigned long long& niters) {
  const DevGraph& g = a.g;
  const uint32_t t0 = dev_clock();
  Cols<CPT> cs;
  const RunRes rr = bp_run<CPT>(g, L, nullptr, nullptr, 0, a.syn + shot * g.m, a.init_iters,
                                true, a.alpha, nullptr, 0, cs, &a.st->error);
  nruns += 1;
  niters += rr.iters;
  if (rr.conv || a.max_rounds == 0) {
    emit_from_regs<CPT>(g, L, cs.ebits, a.corr + shot * g.n, a.flips + shot * g.k);
    if (threadIdx.x == 0) {
      a.conv[shot] = (uint8_t)rr.conv;
      if (a.lat) a.lat[shot] = dev_clock() - t0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      ring_push(&a.st->ctxq, a.ctx_ring, (uint32_t)ctx);
      __hip_atomic_fetch_add(&a.st->done, 1ull, __ATOMIC_RELEASE, AGENT);
    }
    return;
  }
  float score;
  int next_pos;
  score_next<CPT>(g, L, cs, rr.iters, &score, &next_pos);
  Ctx* C = a.ctxs + ctx;
  for (int s = threadIdx.x; s < 3 * a.bw; s += blockDim.x) C->slots[s] = s;
  char* seed = slot_ptr(a, ctx, 0);
  store_msg(g, L, (float*)seed);
  store_bits<CPT>(g, (uint32_t*)(slot_ptr(a, ctx, 3 * a.bw) + slot_ehat_off(g)), cs.ebits);
  if (threadIdx.x == 0) {
    *(int32_t*)(seed + slot_pairs_off(g)) = 0;
    C->shot = (int32_t)shot;
    C->round = 1;
    C->nset = 1;
    C->pending = 2;
    C->best_gen = 0x7FFFFFFF;
    C->nresults = 0;
    C->t_start = t0;
    C->parent_next_pos[0] = next_pos;
    __hip_atomic_fetch_add(&a.st->deep, 1ull, __ATOMIC_RELAXED, AGENT);
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    ring_push(&a.st->work, a.work_ring, ((uint32_t)ctx << 8) | 0u);
    ring_push(&a.st->work, a.work_ring, ((uint32_t)ctx << 8) | 1u);
  }
}

template <int CPT>
__device__ __forceinline__ void process_child(const BatchArgs& a, const LdsMap& L, uint32_t item,
                              unsigned long long& nruns, unsigned long long& niters) {
  const DevGraph& g = a.g;
  const int ctx = (int)(item >> 8), c = (int)(item & 255u);
  Ctx* C = a.ctxs + ctx;
  const int tid = threadIdx.x;
  if (tid == 0) {
    __threadfence();
    L.misc[10] = C->nset;
    L.misc[11] = C->slots[c >> 1];
    L.misc[12] = C->slots[C->nset + c];
    L.misc[13] = C->parent_next_pos[c >> 1];
    L.misc[14] = C->shot;
    L.misc[15] = __hip_atomic_load(&C->best_gen, __ATOMIC_RELAXED, AGENT) < c;
  }
  __syncthreads();
  __threadfence();
  const int ps = L.misc[11], ms = L.misc[12], npos = L.misc[13], skip = L.misc[15];
  const long long shot = L.misc[14];
  char* pslot = slot_ptr(a, ctx, ps);
  char* mslot = slot_ptr(a, ctx, ms);
  int state = 2;
  if (!skip) {
    const int np = *(const int32_t*)(pslot + slot_pairs_off(g));
    const int32_t* pp = (const int32_t*)(pslot + slot_pairs_off(g) + 16);
    int32_t* mp = (int32_t*)(mslot + slot_pairs_off(g) + 16);
    for (int q = tid; q <= np; q += blockDim.x) {
      const int32_t v = q < np ? pp[q] : ((npos << 1) | (c & 1));
      L.pairs[q] = v;
      mp[q] = v;
    }
    if (tid == 0) *(int32_t*)(mslot + slot_pairs_off(g)) = np + 1;
    __syncthreads();
    Cols<CPT> cs;
    const RunRes rr = bp_run<CPT>(g, L, (const float*)pslot, nullptr, np + 1, a.syn + shot * g.m,
                                  a.round_iters, true, a.alpha, &C->best_gen, c, cs,
                                  &a.st->error);
    nruns += 1;
    niters += rr.iters;
    uint32_t* mbitsv = (uint32_t*)(mslot + slot_ehat_off(g));
    if (rr.cancelled) {
      state = 2;
    } else if (rr.conv) {
      state = 1;
      store_bits<CPT>(g, mbitsv, (cs.ebits & ~cs.mbits) | cs.vbits);
      if (tid == 0) __hip_atomic_fetch_min(&C->best_gen, c, __ATOMIC_RELAXED, AGENT);
    } else {
      state = 0;
      float score;
      int next_pos;
      score_next<CPT>(g, L, cs, rr.iters, &score, &next_pos);
      store_msg(g, L, (float*)mslot);
      store_bits<CPT>(g, mbitsv, (cs.ebits & ~cs.mbits) | cs.vbits);
      if (tid == 0) {
        C->child_score[c] = score;
        C->child_next_pos[c] = next_pos;
      }
    }
  }
  if (tid == 0) C->child_state[c] = state;
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    const int left = __hip_atomic_fetch_add(&C->pending, -1, __ATOMIC_ACQ_REL, AGENT);
    L.misc[16] = (left == 1);
  }
  __syncthreads();
  const int last = L.misc[16];
  __syncthreads();
  if (last) {
    __threadfence();
    select_round(a, L, ctx);
  }
}

template <int CPT>
__global__ void __launch_bounds__(1024) k_batched(BatchArgs a) {
  extern __shared__ __align__(16) char lds_raw[];
  const LdsMap L = lds_map(a.g, lds_raw);
  unsigned long long nruns = 0, niters = 0;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) {
      int kind = 0;
      uint32_t item = 0;
      long long shot = -1;
      if (ring_pop(&a.st->work, a.work_ring, &item)) {
        kind = 1;
      } else if (__hip_atomic_load(&a.st->next_shot, __ATOMIC_RELAXED, AGENT) <
                 (unsigned long long)a.shots) {
        uint32_t ctx;
        if (ring_pop(&a.st->ctxq, a.ctx_ring, &ctx)) {
          const unsigned long long s =
              __hip_atomic_fetch_add(&a.st->next_shot, 1ull, __ATOMIC_RELAXED, AGENT);
          if (s < (unsigned long long)a.shots) {
            kind = 2;
            item = ctx;
            shot = (long long)s;
          } else {
            ring_push(&a.st->ctxq, a.ctx_ring, ctx);
          }
        }
      }
      if (kind == 0) {
        if (__hip_atomic_load(&a.st->done, __ATOMIC_ACQUIRE, AGENT) >= (unsigned long long)a.shots)
          kind = 3;
        else
          __builtin_amdgcn_s_sleep(8);
      }
      L.misc[20] = kind;
      L.misc[21] = (int)item;
      L.misc[22] = (int)(shot & 0xFFFFFFFF);
      L.misc[23] = (int)(shot >> 32);
    }
    __syncthreads();
    const int kind = L.misc[20];
    const uint32_t item = (uint32_t)L.misc[21];
    const long long shot = (long long)(uint32_t)L.misc[22] | ((long long)L.misc[23] << 32);
    __syncthreads();
    if (kind == 3) break;
    if (kind == 2) process_init<CPT>(a, L, shot, (int)item, nruns, niters);
    else if (kind == 1) process_child<CPT>(a, L, item, nruns, niters);
  }
  if (tid == 0) {
    __hip_atomic_fetch_add(&a.st->runs, nruns, __ATOMIC_RELAXED, AGENT);
    __hip_atomic_fetch_add(&a.st->iterations, niters, __ATOMIC_RELAXED, AGENT);
  }
}

__global__ void k_batch_reset(BatchArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = gridDim.x * blockDim.x;
  for (uint32_t q = i; q < a.work_cap; q += n) a.work_ring[q] = 0u;
  for (uint32_t q = i; q < a.ctx_cap; q += n) a.ctx_ring[q] = q < (uint32_t)a.nctx ? q + 1u : 0u;
  if (i == 0) {
    a.st->work.cap = a.work_cap;
    a.st->ctxq.cap = a.ctx_cap;
    a.st->next_shot = 0;
    a.st->done = 0;
    a.st->runs = 0;
    a.st->iterations = 0;
    a.st->deep = 0;
    a.st->error = 0;
    a.st->work.head = 0;
    a.st->work.tail = 0;
    a.st->work.count = 0;
    a.st->ctxq.head = 0;
    a.st->ctxq.tail = (uint32_t)a.nctx;
    a.st->ctxq.count = a.nctx;
  }
}

// A single BP run launched on its own (grid of one workgroup).
template <int CPT>
__global__ void __launch_bounds__(1024) k_single(SingleArgs a) {
  extern __shared__ __align__(16) char lds_raw[];
  const DevGraph& g = a.g;
  const LdsMap L = lds_map(g, lds_raw);
  const int tid = threadIdx.x, B = blockDim.x;
  for (int q = tid; q < a.npairs; q += B) L.pairs[q] = a.pairs[q];
  __syncthreads();
  Cols<CPT> cs;
  const RunRes rr = bp_run<CPT>(g, L, a.parent, a.parent_csc, a.npairs, a.syn, a.max_iters,
                                a.stop != 0, a.alpha, nullptr, 0, cs, a.error);
  float score = 0.f;
  int next_pos = -1;
  if (a.want_score) score_next<CPT>(g, L, cs, rr.iters, &score, &next_pos);
  if (a.out_msg && !rr.conv) store_msg(g, L, a.out_msg);
  const uint32_t filled = (cs.ebits & ~cs.mbits) | cs.vbits;
  if (a.out_ehat_bits) store_bits<CPT>(g, a.out_ehat_bits, filled);
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int j = c * B + tid;
    if (j >= g.n) continue;
    const bool mk = (cs.mbits >> c) & 1u;
    if (a.out_sumllr) a.out_sumllr[j] = mk ? 0.f : cs.sumllr[c];
    if (a.out_ehat) a.out_ehat[j] = (uint8_t)(((rr.conv ? filled : (cs.ebits & ~cs.mbits)) >> c) & 1u);
    if (a.out_csc) {
      const int st = (int)(cs.info[c] & 0xFFFFFFu), dg = (int)(cs.info[c] >> 24);
      for (int e = 0; e < dg; ++e) a.out_csc[st + e] = L.msg[g.cedge[st + e] & 0xFFFFu];
    }
  }
  if (tid == 0) {
    a.result[0] = rr.iters;
    a.result[1] = rr.conv;
    a.result[2] = next_pos;
    a.result[3] = __float_as_int(score);
  }
}

__global__ void k_emit(EmitArgs a) {
  __shared__ uint32_t flw[2 * kMaxWaves];
  const DevGraph& g = a.g;
  unsigned long long f = 0;
  for (int j = threadIdx.x; j < g.n; j += blockDim.x) {
    uint32_t b = (a.ehat_bits[j >> 5] >> (j & 31)) & 1u;
    for (int q = 0; q < a.nfill; ++q)
      if ((a.fill_pairs[q] >> 1) == j) b = (uint32_t)(a.fill_pairs[q] & 1);
    a.corr[j] = (uint8_t)b;
    if (b) f ^= g.lmask[j];
  }
  uint32_t lo = (uint32_t)f, hi = (uint32_t)(f >> 32);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    lo ^= __shfl_xor(lo, o, 64);
    hi ^= __shfl_xor(hi, o, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) {
    flw[2 * wave] = lo;
    flw[2 * wave + 1] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < nw; ++w) t ^= (unsigned long long)flw[2 * w] | ((unsigned long long)flw[2 * w + 1] << 32);
    for (int r = 0; r < g.k; ++r) a.flips[r] = (uint8_t)((t >> r) & 1ull);
    a.conv[0] = (uint8_t)a.converged;
  }
}

template <int CPT>
hipError_t launch_single_t(const SingleArgs& a, int block, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_single<CPT>, dim3(1), dim3(block), lds, s, a);
  return hipGetLastError();
}

template <int CPT>
hipError_t launch_batched_t(const BatchArgs& a, int grid, int block, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_batched<CPT>, dim3(grid), dim3(block), lds, s, a);
  return hipGetLastError();
}

template <int CPT>
hipError_t limits_t(size_t lds) {
  hipError_t e = hipFuncSetAttribute((const void*)k_single<CPT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_batched<CPT>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int CPT>
hipError_t occ_t(int block, size_t lds, int* n) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_batched<CPT>, block, lds);
}

}  // namespace

#define BSD_CPT_SWITCH(cpt, CALL)        \
  switch (cpt) {                         \
    case 1: return CALL(1);              \
    case 2: return CALL(2);              \
    case 3: return CALL(3);              \
    case 4: return CALL(4);              \
    case 5: return CALL(5);              \
    case 6: return CALL(6);              \
    case 7: return CALL(7);              \
    case 8: return CALL(8);              \
    case 9: return CALL(9);              \
    case 10: return CALL(10);            \
    case 11: return CALL(11);            \
    case 12: return CALL(12);            \
    case 13: return CALL(13);            \
    case 14: return CALL(14);            \
    case 15: return CALL(15);            \
    case 16: return CALL(16);            \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_single(const SingleArgs& a, int block, int cpt, size_t lds, hipStream_t s) {
#define C_(N) launch_single_t<N>(a, block, lds, s)
  BSD_CPT_SWITCH(cpt, C_)
#undef C_
}

hipError_t launch_batched(const BatchArgs& a, int grid, int block, int cpt, size_t lds,
                          hipStream_t s) {
#define C_(N) launch_batched_t<N>(a, grid, block, lds, s)
  BSD_CPT_SWITCH(cpt, C_)
#undef C_
}

hipError_t set_kernel_limits(int cpt, size_t lds) {
#define C_(N) limits_t<N>(lds)
  BSD_CPT_SWITCH(cpt, C_)
#undef C_
}

hipError_t batched_occupancy(int cpt, int block, size_t lds, int* blocks_per_cu) {
#define C_(N) occ_t<N>(block, lds, blocks_per_cu)
  BSD_CPT_SWITCH(cpt, C_)
#undef C_
}

hipError_t launch_batch_reset(const BatchArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(64), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_emit(const EmitArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_emit, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace bsd
