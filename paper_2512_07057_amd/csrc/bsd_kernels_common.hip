// Launch dispatch and the small auxiliary kernels of the decoder.
#include "bsd_device.h"

namespace bsd {

namespace {

__global__ void k_batch_reset(BatchArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = gridDim.x * blockDim.x;
  for (uint32_t q = i; q < a.work_cap; q += n) a.work_ring[q] = 0u;
  for (uint32_t q = i; q < a.ctx_cap; q += n) a.ctx_ring[q] = q < (uint32_t)a.nctx ? q + 1u : 0u;
  if (a.shot_list) {  // the screen's list for the dense decoder: entries -1 until written
    int32_t* list = const_cast<int32_t*>(a.shot_list);
    for (long long q = i; q < a.shots; q += n) list[q] = -1;
  }
  if (i == 0) {
    a.st->next_shot = 0;
    a.st->done = 0;
    a.st->runs = 0;
    a.st->iterations = 0;
    a.st->deep = 0;
    a.st->sticky |= a.st->error;
    a.st->error = 0;
    a.st->started_wgs = 0;
    a.st->work.head = 0;
    a.st->work.tail = 0;
    a.st->work.count = 0;
    a.st->work.cap = a.work_cap;
    a.st->ctxq.head = 0;
    a.st->ctxq.tail = (uint32_t)a.nctx;
    a.st->ctxq.count = a.nctx;
    a.st->ctxq.cap = a.ctx_cap;
    a.st->pub = 0;
    a.st->stop = 0;
    a.st->poll_token = 0;
    a.st->listed = 0;
    a.st->done2 = 0;
    a.st->screen_begun = 0;
    a.st->screen_live = a.screen_waves;
  }
}


// Final output of one shot from a hard-decision bit-vector (plain form).
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
    for (int w = 0; w < nw; ++w)
      t ^= (unsigned long long)flw[2 * w] | ((unsigned long long)flw[2 * w + 1] << 32);
    for (int r = 0; r < g.k; ++r) a.flips[r] = (uint8_t)((t >> r) & 1ull);
    a.conv[0] = (uint8_t)a.converged;
  }
}

}  // namespace

size_t lds_bytes_for(const DevGraph& g) { return (dev::lds_need(g) + 15) & ~(size_t)15; }

#define BSD_PW_SWITCH(pw, CALL)                  \
  switch (pw) {                                  \
    case 1: return CALL(1);                      \
    case 2: return CALL(2);                      \
    case 3: return CALL(3);                      \
    case 4: return CALL(4);                      \
    default: return hipErrorInvalidValue;        \
  }

hipError_t launch_single(const SingleArgs& a, int block, int cpt, int pw, size_t lds,
                         hipStream_t s) {
#define C_(P) launch_single_pw<P>(a, block, cpt, lds, s)
  BSD_PW_SWITCH(pw, C_)
#undef C_
}

hipError_t launch_batched(const BatchArgs& a, int grid, int block, int cpt, int pw, size_t lds,
                          hipStream_t s) {
#define C_(P) launch_batched_pw<P>(a, grid, block, cpt, lds, s)
  BSD_PW_SWITCH(pw, C_)
#undef C_
}

hipError_t set_kernel_limits(int cpt, int pw, size_t lds) {
#define C_(P) limits_pw<P>(cpt, lds)
  BSD_PW_SWITCH(pw, C_)
#undef C_
}

hipError_t batched_occupancy(int cpt, int pw, int block, size_t lds, int* blocks_per_cu) {
#define C_(P) occupancy_pw<P>(cpt, block, lds, blocks_per_cu)
  BSD_PW_SWITCH(pw, C_)
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
