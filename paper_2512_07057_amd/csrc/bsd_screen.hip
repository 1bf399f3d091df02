// Sparse screen of iteration 1 of the initial BP run (Appendix A, eqs. (1),
// (3), (4) and the stopping rule at t = 1), one wavefront per shot.
//
// From E(0) = Lambda with every Lambda_j > 0 every sign in eq. (1) except
// (-1)^{s_i} is +1, so at t = 1 detector i sends x_i = alpha * (least
// |Lambda| of its row) to every neighbour but the one holding that least,
// which gets y_i = alpha * (second least); both are clamped to the message
// bound and both carry the sign (-1)^{s_i}.  A column none of whose
// detectors flipped sums positive terms onto a positive prior and decides
// e_j = 0 (eq. (4)).  The columns of flipped detectors are summed here in
// the dense variable phase's order -- Lambda_j, then the messages in
// ascending row order, in single precision -- so every decision equals the
// dense decoder's.  When H e-hat equals the syndrome the shot is finished
// (iteration 1 of the initial run converged); otherwise it is appended to
// the list that the dense persistent decoder takes its shots from.
//
// A workgroup keeps the per-row table (x, y and the column of the least
// |Lambda|) and the row pointers in LDS for the whole launch; each wave
// holds one shot's syndrome bits, residual and candidate lists.  Per shot
// the only global reads are its syndrome (prefetched during the previous
// shot) and one entry per (flipped detector, column) pair: the column, its
// prior and its rows.
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
#define BSD_SCREEN_MIN_WAVES 1
#endif
constexpr int kUnroll = BSD_SCREEN_UNROLL;  // candidates per lane in flight

struct WaveLds {
  uint32_t sbits[64];                    // s by row (m <= 2048)
  uint32_t rbits[64];                    // s + H e-hat
  int32_t cst[kScreenMaxFlipped];        // first CSR position of each flipped row
  int32_t coff[kScreenMaxFlipped];       // index of its first (row, column) pair
  uint16_t flipped[kScreenMaxFlipped];   // rows with s_i = 1, ascending
  uint8_t cmap[kScreenMaxCand];          // flipped row of each (row, column) pair
  int32_t set[kScreenMaxSet];            // columns with e-hat_j = 1
  int32_t nset;
  int32_t pad[3];
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
  const long long nwaves = (long long)gridDim.x * kWaves;
  uint32_t done = 0, err = 0;
  long long shot = (long long)blockIdx.x * kWaves + wv;
  uint2 sv[kSynRegs];
  if (a.syn8 && shot < a.shots) load_syn_regs(a, shot, lane, sv);
  for (; shot < a.shots; shot += nwaves) {
    const uint32_t t0 = a.lat ? (uint32_t)wall_clock64() : 0u;
    err |= syndrome_bits(a, shot, sv, W, lane);
    if (a.syn8 && shot + nwaves < a.shots) load_syn_regs(a, shot + nwaves, lane, sv);
    // Flipped detectors, ascending; their (row, column) pairs, numbered.
    const uint32_t word = lane < a.words_m ? W.sbits[lane] : 0u;
    int nflip;
    const int off = wave_excl_scan(__builtin_popcount(word), lane, &nflip);
    {
      int q = off;
      for (uint32_t b = word; b; b &= b - 1u, ++q)
        if (q < kScreenMaxFlipped) W.flipped[q] = (uint16_t)(lane * 32 + __builtin_ctz(b));
    }
    W.rbits[lane] = word;
    if (lane == 0) W.nset = 0;
    wave_sync();
    bool ok = nflip <= kScreenMaxFlipped;
    int ncand = 0;
    if (ok) {
      int st = 0, dg = 0;
      if (lane < nflip) {
        const int i = W.flipped[lane];
        st = rptr[i];
        dg = rptr[i + 1] - st;
      }
      const int coff = wave_excl_scan(dg, lane, &ncand);
      ok = ncand <= kScreenMaxCand;
      if (ok && lane < nflip) {
        W.cst[lane] = st;
        W.coff[lane] = coff;
        for (int q = 0; q < dg; ++q) W.cmap[coff + q] = (uint8_t)lane;
      }
      wave_sync();
    }
    if (ok) {
      for (int base = 0; base < ncand; base += 64 * kUnroll) {
        uint4 rq[kUnroll];
        uint2 jl[kUnroll];
        int fi[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int c = base + 64 * u + lane;
          fi[u] = -1;
          if (c < ncand) {
            fi[u] = W.cmap[c];
            const int pos = W.cst[fi[u]] + (c - W.coff[fi[u]]);
            rq[u] = a.edge_rows[pos];
            jl[u] = a.edge_col[pos];
          }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          if (fi[u] < 0) continue;
          const int i = W.flipped[fi[u]], j = (int)jl[u].x;
          // Eq. (3): Lambda_j, then the messages of the rows in ascending
          // order (absent slots add nothing).  The column is kept only by
          // its lowest flipped detector, so that it counts once.
          float post = __uint_as_float(jl[u].y);
          int first = 0xFFFF;
#pragma unroll
          for (int e = 0; e < DV; ++e) {
            const int r = row_at(rq[u], e);
            const bool there = r != 0xFFFF;
            const uint4 t = tab[there ? r : 0];
            const uint32_t sb = there ? bit_of(W.sbits, r) : 0u;
            first = (sb && first == 0xFFFF) ? r : first;
            const float mag = __uint_as_float((int)t.z == j ? t.y : t.x);
            if (there) post = post + (sb ? -mag : mag);
          }
          if (first == i && post <= 0.f) {  // eq. (4): e-hat_j = 1; its detectors join s + H e-hat
            const int q = atomicAdd(&W.nset, 1);
            if (q < kScreenMaxSet) W.set[q] = j;
#pragma unroll
            for (int e = 0; e < DV; ++e) {
              const int r = row_at(rq[u], e);
              if (r != 0xFFFF) atomicXor(&W.rbits[r >> 5], 1u << (r & 31));
            }
          }
        }
      }
      wave_sync();
    }
    const int nset = W.nset;
    // Stopping rule: s + H e-hat = 0.
    ok = ok && nset <= kScreenMaxSet &&
         __ballot(lane < a.words_m && W.rbits[lane] != 0u) == 0ull;
    if (ok) {
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
        ++done;
      }
    } else if (lane == 0) {
      const int q = __hip_atomic_fetch_add(&a.st->listed, 1, __ATOMIC_RELAXED, AGENT);
      a.list[q] = (int32_t)shot;
    }
    if (a.lat && lane == 0) a.lat[shot] = (uint32_t)wall_clock64() - t0;
    wave_sync();  // the next shot reuses this wave's LDS
  }
  if (lane == 0 && done) {
    __hip_atomic_fetch_add(&a.st->done, (unsigned long long)done, __ATOMIC_RELAXED, AGENT);
    __hip_atomic_fetch_add(&a.st->runs, (unsigned long long)done, __ATOMIC_RELAXED, AGENT);
    __hip_atomic_fetch_add(&a.st->iterations, (unsigned long long)done, __ATOMIC_RELAXED, AGENT);
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
