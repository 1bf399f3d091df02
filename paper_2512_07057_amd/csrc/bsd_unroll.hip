// Differentiable unrolled min-sum: forward pass and its hand-written adjoint.
//
// Forward (Appendix A, eqs. (1)-(3)): T flooding iterations from E(0) =
// Lambda on every edge, the detector-to-error messages of eq. (1) scaled by
// alpha_t at iteration t, no early stop; the output is post(T).  Every D and
// E is saturated to +-llr_max as in the decoder.  E(t) is saved every K
// iterations (t = 0, K, 2K, ...).
//
// Adjoint: given dL/dpost(T), the gradients with respect to Lambda and
// alpha.  Segment by segment from the last, E(t) is recomputed from the
// segment's checkpoint and the gradient is carried back through
//   variable phase:  E_e(t) = Lambda_j + sum_{f in N(j), f != e} D_f(t),
//                    post_j(T) = Lambda_j + sum_{f in N(j)} D_f(T);
//   check phase:     D_e(t) = alpha_t * sigma_e * m_e, with sigma_e the sign
//                    factor (-1)^{s_i} prod_{f != e} sgn(E_f(t-1)) (locally
//                    constant) and m_e = min_{f != e} |E_f(t-1)|, whose
//                    derivative reaches the argmin of the row for every other
//                    edge and the second minimum for the argmin's own edge;
//   E(0) = Lambda.
// The map is differentiable wherever no row has a tie between its two
// smallest |E| and no E is 0; there the derivative is exact.  The
// saturation never acts on the workloads here; the adjoint treats it as
// inactive.
//
// One wave per shot; all state of the shot in LDS.
#include <hip/hip_runtime.h>

#include <mutex>

#include "bsd_internal.h"

namespace bsd {

namespace {

// Per-shot partial gradients of bsd_unroll_backward_noalloc, in memory the
// library never allocates: every device the library runs on holds this
// array until the process ends.  Calls on one device share it, so calls
// that overlap on one device race; nothing in it needs clearing between
// calls (the backward kernel writes every partial before the sum reads it).
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

template <typename F>
__device__ __forceinline__ F clampv(F x, F lim) {
  return x < -lim ? -lim : (x > lim ? lim : x);
}

template <typename F>
struct RowMin {
  F m1, m2;   // least and second least |E| of the row
  int a1, a2; // their positions in the row (a2 = -1 if the row has one edge)
  int par;    // parity of the number of negative E
};

// Least and second least magnitude of a row's messages (first position on ties).
template <typename F>
__device__ __forceinline__ RowMin<F> row_min(const UnrollArgs& a, const F* E, int i, F lim) {
  RowMin<F> r{lim, lim, -1, -1, 0};
  const int b = a.rowptr[i], d = a.rowptr[i + 1] - b;
  for (int k = 0; k < d; ++k) {
    const F v = E[a.rowedge[b + k]];
    const F x = v < F(0) ? -v : v;
    r.par ^= v < F(0) ? 1 : 0;
    if (x < r.m1) {
      r.m2 = r.m1;
      r.a2 = r.a1;
      r.m1 = x;
      r.a1 = k;
    } else if (x < r.m2) {
      r.m2 = x;
      r.a2 = k;
    }
  }
  return r;
}

// Eq. (1) times alpha_t for every edge, from E (read) into D (written).
template <typename F>
__device__ __forceinline__ void check_step(const UnrollArgs& a, const uint8_t* syn, const F* E, F* D,
                                           F alpha_t, F lim) {
  for (int i = threadIdx.x; i < a.m; i += blockDim.x) {
    const RowMin<F> r = row_min<F>(a, E, i, lim);
    const int b = a.rowptr[i], d = a.rowptr[i + 1] - b;
    const int s = syn[i] & 1;
    for (int k = 0; k < d; ++k) {
      const int e = a.rowedge[b + k];
      const int neg = s ^ r.par ^ (E[e] < F(0) ? 1 : 0);  // sign of the other edges times (-1)^s
      const F mag = alpha_t * (k == r.a1 ? r.m2 : r.m1);
      D[e] = clampv<F>(neg ? -mag : mag, lim);
    }
  }
}

// Eqs. (3) and (2) in ascending row order: posteriors (when post != null)
// and the new E.
template <typename F>
__device__ __forceinline__ void var_step(const UnrollArgs& a, const F* lam, const F* D, F* E, F* post,
                                         F lim) {
  for (int j = threadIdx.x; j < a.n; j += blockDim.x) {
    const int b = a.colptr[j], d = a.colptr[j + 1] - b;
    F p = lam[j];
    for (int k = 0; k < d; ++k) p = p + D[b + k];
    if (post) post[j] = p;
    for (int k = 0; k < d; ++k) {
      F x = lam[j];
      for (int f = 0; f < d; ++f)
        if (f != k) x = x + D[b + f];
      E[b + k] = clampv<F>(x, lim);
    }
  }
}

template <typename F>
__global__ void k_unroll_fwd(UnrollArgs a) {
  extern __shared__ __align__(16) char sm[];
  F* E = reinterpret_cast<F*>(sm);
  F* D = E + a.nnz;
  const long long shot = blockIdx.x;
  const uint8_t* syn = a.syn + shot * a.m;
  const F* lam = static_cast<const F*>(a.lam);
  const F* alpha = static_cast<const F*>(a.alpha);
  const F lim = (F)a.llr_max;
  F* ck = static_cast<F*>(a.ckpt) + shot * (long long)a.nseg * a.nnz;
  for (int j = threadIdx.x; j < a.n; j += blockDim.x)
    for (int e = a.colptr[j]; e < a.colptr[j + 1]; ++e) E[e] = lam[j];
  __syncthreads();
  F* out = static_cast<F*>(a.post) + shot * a.n;
  if (a.T == 0)
    for (int j = threadIdx.x; j < a.n; j += blockDim.x) out[j] = lam[j];
  for (int t = 1; t <= a.T; ++t) {
    if ((t - 1) % a.K == 0)  // E(t-1) starts a segment
      for (int e = threadIdx.x; e < a.nnz; e += blockDim.x) ck[((t - 1) / a.K) * a.nnz + e] = E[e];
    check_step<F>(a, syn, E, D, alpha[t - 1], lim);
    __syncthreads();
    var_step<F>(a, lam, D, E, t == a.T ? out : nullptr, lim);
    __syncthreads();
  }
}

template <typename F>
__global__ void k_unroll_bwd(UnrollArgs a) {
  extern __shared__ __align__(16) char sm[];
  const int nnz = a.nnz;
  F* Es = reinterpret_cast<F*>(sm);  // [K][nnz]: E(t0) .. E(t0 + K - 1)
  F* D = Es + (size_t)a.K * nnz;     // scratch of the recomputation
  F* gE = D + nnz;                   // dL/dE(t)
  F* gD = gE + nnz;                  // dL/dD(t)
  F* gL = gD + nnz;                  // [n] dL/dLambda (this shot)
  F* red = gL + a.n;                 // [blockDim.x / 64] wave partials
  const long long shot = blockIdx.x;
  const uint8_t* syn = a.syn + shot * a.m;
  const F* lam = static_cast<const F*>(a.lam);
  const F* alpha = static_cast<const F*>(a.alpha);
  const F* gpost = static_cast<const F*>(a.gpost) + shot * a.n;
  const F* ck = static_cast<const F*>(a.ckpt) + shot * (long long)a.nseg * nnz;
  F* ga = static_cast<F*>(a.ga_part) + shot * a.T;
  const F lim = (F)a.llr_max;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int e = threadIdx.x; e < nnz; e += blockDim.x) gE[e] = F(0);  // E(T) does not reach the loss
  // With no iteration post(0) = Lambda, so dL/dLambda starts at dL/dpost;
  // otherwise post(T) reaches Lambda through the variable phase of t = T.
  for (int j = threadIdx.x; j < a.n; j += blockDim.x) gL[j] = a.T == 0 ? gpost[j] : F(0);
  __syncthreads();
  for (int seg = a.nseg - 1; seg >= 0; --seg) {
    const int t0 = seg * a.K, t1 = min(t0 + a.K, a.T);
    for (int e = threadIdx.x; e < nnz; e += blockDim.x) Es[e] = ck[(size_t)seg * nnz + e];
    __syncthreads();
    for (int t = t0 + 1; t < t1; ++t) {  // E(t0+1) .. E(t1-1)
      check_step<F>(a, syn, Es + (size_t)(t - 1 - t0) * nnz, D, alpha[t - 1], lim);
      __syncthreads();
      var_step<F>(a, lam, D, Es + (size_t)(t - t0) * nnz, nullptr, lim);
      __syncthreads();
    }
    for (int t = t1; t > t0; --t) {
      const F* Ep = Es + (size_t)(t - 1 - t0) * nnz;  // E(t-1)
      // Variable phase: dL/dD(t) and the Lambda terms of E(t) and post(T).
      for (int j = threadIdx.x; j < a.n; j += blockDim.x) {
        const int b = a.colptr[j], d = a.colptr[j + 1] - b;
        F ge = F(0);
        for (int k = 0; k < d; ++k) ge = ge + gE[b + k];
        const F gp = t == a.T ? gpost[j] : F(0);
        for (int k = 0; k < d; ++k) gD[b + k] = (ge - gE[b + k]) + gp;
        gL[j] = gL[j] + (ge + gp);
      }
      __syncthreads();
      // Check phase: dL/dalpha_t and dL/dE(t-1).
      const F at = alpha[t - 1];
      F gat = F(0);
      for (int i = threadIdx.x; i < a.m; i += blockDim.x) {
        const RowMin<F> r = row_min<F>(a, Ep, i, lim);
        const int b = a.rowptr[i], d = a.rowptr[i + 1] - b;
        const int s = syn[i] & 1;
        F to_a1 = F(0), to_a2 = F(0);
        for (int k = 0; k < d; ++k) {
          const int e = a.rowedge[b + k];
          const F sig = (s ^ r.par ^ (Ep[e] < F(0) ? 1 : 0)) ? F(-1) : F(1);
          const F me = k == r.a1 ? r.m2 : r.m1;
          gat = gat + gD[e] * sig * me;
          if (k == r.a1)
            to_a2 = to_a2 + gD[e] * at * sig;
          else
            to_a1 = to_a1 + gD[e] * at * sig;
        }
        for (int k = 0; k < d; ++k) {
          const int e = a.rowedge[b + k];
          const F sg = Ep[e] < F(0) ? F(-1) : F(1);
          F g = F(0);
          if (k == r.a1) g = to_a1 * sg;
          if (k == r.a2) g = to_a2 * sg;  // a2 >= 0 only with two or more edges
          gE[e] = g;
        }
      }
      for (int o = 32; o >= 1; o >>= 1) gat = gat + __shfl_xor(gat, o, 64);
      if (lane == 0) red[wave] = gat;
      __syncthreads();
      if (threadIdx.x == 0) {
        F s_ = F(0);
        for (int w = 0; w < nw; ++w) s_ = s_ + red[w];
        ga[t - 1] = s_;
      }
    }
  }
  // E(0) = Lambda.
  for (int j = threadIdx.x; j < a.n; j += blockDim.x) {
    F ge = F(0);
    for (int e = a.colptr[j]; e < a.colptr[j + 1]; ++e) ge = ge + gE[e];
    gL[j] = gL[j] + ge;
  }
  __syncthreads();
  F* gl = static_cast<F*>(a.gl_part) + shot * a.n;
  for (int j = threadIdx.x; j < a.n; j += blockDim.x) gl[j] = gL[j];
}

// Sum the per-shot partials over shots in shot order (deterministic).
template <typename F>
__global__ void k_unroll_reduce(UnrollArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.n) {
    const F* p = static_cast<const F*>(a.gl_part);
    F s = F(0);
    for (long long b = 0; b < a.shots; ++b) s = s + p[b * a.n + i];
    static_cast<F*>(a.grad_lam)[i] = s;
  } else if (i < a.n + a.T) {
    const int t = i - a.n;
    const F* p = static_cast<const F*>(a.ga_part);
    F s = F(0);
    for (long long b = 0; b < a.shots; ++b) s = s + p[b * a.T + t];
    static_cast<F*>(a.grad_alpha)[t] = s;
  }
}

template <typename F>
hipError_t launch_fwd(const UnrollArgs& a, hipStream_t s) {
  const size_t lds = 2 * (size_t)a.nnz * sizeof(F);
  hipError_t e = hipFuncSetAttribute((const void*)k_unroll_fwd<F>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_unroll_fwd<F>, dim3((unsigned)a.shots), dim3(kUnrollBlock), lds, s, a);
  return hipGetLastError();
}

template <typename F>
hipError_t launch_bwd(const UnrollArgs& a, hipStream_t s) {
  const size_t lds = ((size_t)(a.K + 3) * a.nnz + a.n + kUnrollBlock / 64) * sizeof(F);
  hipError_t e = hipFuncSetAttribute((const void*)k_unroll_bwd<F>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (a.shots > 0) {  // with no shots the reduction writes zeros
    hipLaunchKernelGGL(k_unroll_bwd<F>, dim3((unsigned)a.shots), dim3(kUnrollBlock), lds, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int tot = a.n + a.T;
  hipLaunchKernelGGL(k_unroll_reduce<F>, dim3((tot + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t noalloc_scratch(int device, void** ptr) {
  // The array's name is a host-side stand-in; its device address is looked
  // up once per device, with that device current (the caller's job).
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

size_t unroll_bwd_lds(const UnrollArgs& a, int elem) {
  return ((size_t)(a.K + 3) * a.nnz + a.n + kUnrollBlock / 64) * elem;
}

hipError_t launch_unroll_forward(const UnrollArgs& a, int elem, hipStream_t s) {
  return elem == 8 ? launch_fwd<double>(a, s) : launch_fwd<float>(a, s);
}

hipError_t launch_unroll_backward(const UnrollArgs& a, int elem, hipStream_t s) {
  return elem == 8 ? launch_bwd<double>(a, s) : launch_bwd<float>(a, s);
}

}  // namespace bsd
