// Internal layout shared by the decoder's kernels and its host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bsd {

constexpr int kMaxDv = 8;          // largest column degree handled
constexpr int kMaxDc = 255;        // largest row degree handled
constexpr int kMaxBw = 64;         // largest beam width
constexpr int kMaxRounds = 64;     // largest number of fixed nodes on a path
constexpr int kMaxResults = 64;    // largest num_results
constexpr int kMaxWaves = 16;      // 1024 threads per workgroup at most
constexpr int kMaxCpt = 32;        // columns per thread at most
constexpr float kLlrMax = 1e30f;   // saturation of every message
constexpr int kLdsBytes = 160 * 1024;
constexpr int kTrashWords = 64;  // LDS trash words after the messages, one per lane

// Device-resident Tanner graph.  Rows are renumbered by "rank" (descending
// degree); the LDS message of the edge (row of rank r, k-th neighbour in
// ascending column order) lives at position diag_ptr[k] + r (jagged
// diagonals), so that lanes holding consecutive ranks touch consecutive
// words in the check phase.
struct DevGraph {
  int32_t m, n, nnz, k;
  int32_t nnz_pad;      // nnz rounded up to a multiple of 4 (16-byte vector copies)
  int32_t words_m;      // 32-bit words of a row bit-vector, rounded up to a multiple of 2
  int32_t words_n;      // 32-bit words of a column bit-vector, rounded up to a multiple of 2
  int32_t maxdeg_row;
  const int32_t* diag_ptr;     // [maxdeg_row + 1]
  const uint16_t* row_of_rank; // [m] original row of each rank
  const uint8_t* deg_of_rank;  // [m]
  const uint32_t* colinfo;     // [n] first CSC edge (bits 0..23) | degree << 24
  const uint32_t* cedge;       // [nnz] CSC order: LDS position (bits 0..15) | row rank << 16
  const uint4* crank;          // [n] row ranks of column j's edges, 16 bits each (8 slots, 0xFFFF unused)
  const float* lambda;         // [n] prior LLRs
  const uint64_t* lmask;       // [n] logical rows flipped by each column
};

// One device-resident path (a beam "slot"): its edge messages in LDS order,
// the hard decision of its last iteration, and its fixed nodes.
//   float    msg[nnz_pad]
//   uint32_t ehat[words_n]
//   int32_t  npairs, pad[3]
//   int32_t  pairs[kMaxRounds]   packed (column << 1) | value
inline __host__ __device__ size_t slot_ehat_off(const DevGraph& g) { return (size_t)g.nnz_pad * 4; }
inline __host__ __device__ size_t slot_pairs_off(const DevGraph& g) {
  return slot_ehat_off(g) + (size_t)g.words_n * 4;
}
inline __host__ __device__ size_t slot_bytes(const DevGraph& g) {
  size_t b = slot_pairs_off(g) + 16 + 4 * kMaxRounds;
  return (b + 255) & ~(size_t)255;
}

// A shot whose initial BP run failed: the beam of Algorithm 3 in flight.
struct Ctx {
  int32_t shot;
  int32_t round;          // round whose children are running (1-based)
  int32_t nset;           // paths in the current set (parents of this round)
  int32_t pending;        // children of this round not yet finished
  int32_t best_gen;       // smallest converged child generation this round
  int32_t nresults;
  uint32_t t_start;       // device clock at the start of the initial run
  int32_t pad0;
  int32_t slots[3 * kMaxBw];          // first nset: parents in rank order; rest free
  int32_t parent_next_pos[kMaxBw];
  float child_score[2 * kMaxBw];
  int32_t child_next_pos[2 * kMaxBw];
  int32_t child_state[2 * kMaxBw];    // 0 ran, 1 converged, 2 cancelled
  double child_wt[2 * kMaxBw];        // converged children (num_results > 1): wt(e-hat)
  uint64_t child_hash[2 * kMaxBw];    //   and a digest of e-hat
  double res_wt[kMaxResults];         // results found so far, in the order found
  uint64_t res_hash[kMaxResults];
  uint32_t init_ehat_off;             // unused padding kept for alignment
  int32_t pad1[3];
};

// Multi-producer multi-consumer ring of 32-bit items (item + 1 stored; 0 = empty).
struct Ring {
  uint32_t head;
  uint32_t tail;
  int32_t count;
  uint32_t cap;
};

struct BatchState {
  unsigned long long next_shot;
  unsigned long long done;
  unsigned long long runs;
  unsigned long long iterations;
  unsigned long long deep;
  uint32_t error;
  uint32_t started_wgs;  // serving: workgroups of the launch that have begun
  Ring work;
  Ring ctxq;
  // Serving: mirrors of the host's published count and stop flag, refreshed
  // by whichever idle workgroup holds the poll token.
  unsigned long long pub;  // shots published
  uint32_t stop;           // nonzero: end the kernel
  uint32_t poll_token;     // 1 while a workgroup is reading the host counters
  int32_t listed;          // shots the screen handed to the dense decoder
  uint32_t screen_begun;   // workgroups of the screen launch that have begun
  int32_t screen_live;     // waves of the screen launch that have not finished
  unsigned long long done2;  // shots the screen finished at iteration 2
  uint32_t sticky;         // errors of earlier calls on this workspace, until reported
};

// The check phase of iteration 1 in a run from the priors with no masked
// node depends on the syndrome only through the signs (-1)^{s_i} of eq. (1),
// since E(0) = Lambda for every shot.  Per detector rank the table holds what
// eq. (1) needs for s = 0, formed with the kernels' single-precision
// operations: x = alpha * least |Lambda| of the row and y = alpha * second
// least (both clamped to the message bound), the diagonal index of the edge
// holding the least (it receives y, every other edge x), and the parity of
// the row's negative priors.
struct FirstIter {
  const uint4* rows;        // [m] per rank: x bits, y bits, argk | parity << 8 | anyneg << 9, 0
  const uint32_t* negbits;  // [nnz_pad / 32 + 1] LDS order: sign bit of Lambda of the edge's column
  int32_t enabled;
};

// Device workspace of one batched decoder instance: queue state, rings,
// per-shot contexts and their path slots.
struct BatchWs {
  int bw = 0, nctx = 0;
  BatchState* st = nullptr;
  BatchState* st_host = nullptr;  // pinned copy for read-back
  uint32_t* work_ring = nullptr;
  uint32_t work_cap = 0;
  uint32_t* ctx_ring = nullptr;
  uint32_t ctx_cap = 0;
  Ctx* ctxs = nullptr;
  char* slots = nullptr;
  uint32_t* results = nullptr;  // num_results > 1
  size_t results_words = 0;
};

struct BatchArgs {
  DevGraph g;
  FirstIter fi;
  const double* lam64;    // [n] wt(e) contributions log((1-p_j)/p_j) in double precision
  uint32_t* results;      // num_results > 1: [nctx][num_results][words_n] e-hat bits
  // Serving (stream != 0): shots arrive over time through a ring of
  // io_mask + 1 rows in host memory; `shots` is unused.
  int32_t stream;
  unsigned long long io_mask;  // row of a shot's input and outputs = shot & io_mask
  const unsigned long long* pub_host;  // host memory: shots published
  const uint32_t* stop_host;           // host memory: nonzero ends the kernel
  uint32_t* done_flag;         // per row: low 32 bits of shot + 1 once its outputs are written
  uint32_t* started;           // host memory: set to 1 once every workgroup of the launch runs
  uint32_t* begun;             // host memory: set to 1 when the launch's first workgroup runs
  const uint32_t* gen_host;    // host memory: the decoder's current launch generation
  uint32_t gen;                // this launch's generation (a replaced launch ends at once)
  uint32_t idle_limit;         // also end after this many 100 MHz ticks with nothing to do
  long long shots;
  const uint8_t* syn;
  uint8_t* corr;
  uint8_t* flips;
  uint8_t* conv;
  uint32_t* lat;
  int32_t max_rounds, bw, init_iters, round_iters, num_results;
  float alpha;
  const float* alpha_sched;  // or NULL: iteration t scales eq. (1) by alpha_sched[min(t, n_sched) - 1]
  int32_t n_sched;
  BatchState* st;
  // With the iteration-1 screen: the shots left to this kernel, in claim
  // order (st->listed of them); without it every shot 0..shots-1.  The
  // screen has already written the outputs of the others and counted them
  // as done, and its share of each listed shot's latency.
  const int32_t* shot_list;
  // A launch beside the screen (helper = 1) starts on the workgroups the
  // screen leaves and takes listed shots while the screen still lists them
  // (entries -1 until written); it ends at once unless every one of the
  // screen's screen_grid workgroups had begun, so that it never holds the
  // device from a screen that has not started.  The launch after the screen
  // finishes whatever is left.
  int32_t helper;
  int32_t screen_grid;
  int32_t screen_waves;   // reset: the screen launch's waves (0: no screen)
  uint32_t* work_ring;
  uint32_t work_cap;      // power of two
  uint32_t* ctx_ring;
  uint32_t ctx_cap;       // power of two
  Ctx* ctxs;
  int32_t nctx;
  char* slots;            // nctx * slots_per_ctx slots
  size_t slot_stride;
  int32_t slots_per_ctx;  // 3 * bw + 1 (the last one keeps the initial run's hard decision)
};

// Sparse check of iterations 1 and 2 of the initial run, one wavefront per
// shot.  From E(0) = Lambda with every Lambda_j > 0, eq. (1) at t = 1 sends
// each column a message of magnitude x_i (the row's least alpha |Lambda|) or
// y_i (the second least, to the edge holding the least) with the sign
// (-1)^{s_i}.  A column with no flipped detector therefore has a positive
// posterior and decides 0, so the hard decision of iteration 1 is found by
// summing the posteriors of the columns of flipped detectors only, in the
// same single-precision order as the dense variable phase.  Iteration 2 is
// found in the same way from the rows that can send a negative message and
// lower bounds of the others' messages.  Shots whose decision satisfies the
// syndrome are finished here (one run; one or two iterations); the others
// are appended to `list` for the dense decoder.
struct ScreenArgs {
  int32_t m, n, k;
  int32_t words_m;
  int32_t vec;                 // bytes per correction store: 16, 4 or 1 (divides n; aligned)
  int32_t syn8;                // 1: m % 8 == 0 and the syndromes are 8-byte aligned
  int32_t maxdeg_col;          // largest column degree (1..8)
  int32_t t2;                  // 1: also screen iteration 2 (initial_iters >= 2)
  int32_t single1;             // 1: iteration 1's alpha <= 1, so bit 14 of edge_rows holds
  float alpha2;                // scaling of eq. (1) at iteration 2
  const int32_t* row_ptr;      // [m + 1] rows (original numbering) in CSR form
  const uint4* edge_rows;      // [nnz] CSR order: rows of the edge's column, 16 bits each,
                               //   ascending: row in bits 0-11, bit 15 set when the column
                               //   holds the row's least |Lambda| (0xFFFF unused); bit 14 of
                               //   the first slot set when one detector alone may decide the
                               //   column (for alpha <= 1)
  const uint4* edge_col;       // [nnz] CSR order: the edge's column, its Lambda bits, its
                               //   logical mask (low, high 32 bits)
  const float2* row_xy;        // [m + 1] per row, the magnitudes of eq. (1) at t = 1: x_i to
                               //   every column but the holder of the least |Lambda|, y_i to
                               //   that one (row m: 0, 0)
  const float* row_e1min;      // [m] least E(1) the row receives for s = 0 (a lower bound)
  long long shots;
  const uint8_t* syn;
  uint8_t* corr;
  uint8_t* flips;
  uint8_t* conv;
  uint32_t* lat;               // or NULL
  BatchState* st;              // error, done, done2, runs, iterations, listed
  int32_t* list;               // [shots] shots for the dense decoder (-1 until written)
};
constexpr int kScreenBlock = 512;        // iteration 1: eight shots in flight per workgroup
constexpr int kScreen1MinWaves = 4;      // iteration 1: waves per SIMD the registers must allow
constexpr int kScreen2Block = 512;       // iteration 2
constexpr int kScreen2MinWaves = 4;      // iteration 2: waves per SIMD the registers must allow
constexpr int kScreenMaxFlipped = 64;    // more flipped detectors: dense decoder
constexpr int kScreenMaxCand = 2048;     // more (detector, column) pairs: dense decoder
constexpr int kScreenMaxSet = 64;        // more set decisions: dense decoder
// Resident workgroups per CU of the iteration-1 (which = 1) or iteration-2
// (which = 2) screen kernel for m detectors.
int screen_blocks_per_cu(int m, int which);

// Arguments of a single BP run launched on its own (plain form, bsd_bp_run).
struct SingleArgs {
  DevGraph g;
  const float* parent;      // warm start in LDS order, or NULL
  const float* parent_csc;  // warm start in CSC order, or NULL
  const int32_t* pairs;     // device, packed (col << 1) | val
  int32_t npairs;
  const uint8_t* syn;       // [m]
  int32_t max_iters;
  int32_t stop;
  float alpha;
  const float* alpha_sched;  // as in BatchArgs
  int32_t n_sched;
  int32_t want_score;
  float* out_msg;           // LDS order, written when not converged or keep_msg (or NULL)
  int32_t keep_msg;
  float* out_csc;           // CSC order (or NULL)
  float* out_sumllr;        // [n] (or NULL)
  uint8_t* out_ehat;        // [n] bytes (or NULL)
  uint32_t* out_ehat_bits;  // [words_n] (or NULL)
  int32_t* out_pairs;       // [1 + kMaxRounds]: npairs, pairs (or NULL)
  int32_t* result;          // [4]: iters, converged, next_pos, score bits
  uint32_t* error;
};

// Final output of a shot from a hard-decision bit-vector (plain form).
struct EmitArgs {
  DevGraph g;
  const uint32_t* ehat_bits;
  const int32_t* fill_pairs; // packed pairs to fill in, or NULL
  int32_t nfill;
  uint8_t* corr;             // [n]
  uint8_t* flips;            // [k]
  uint8_t* conv;             // [1]
  int32_t converged;
};

// Host-side launchers (bsd_kernels_common.hip).  pw = words of 16-bit edge
// positions per column kept in registers = ceil(largest column degree / 2).
hipError_t launch_single(const SingleArgs& a, int block, int cpt, int pw, size_t lds,
                         hipStream_t s);
hipError_t launch_batched(const BatchArgs& a, int grid, int block, int cpt, int pw, size_t lds,
                          hipStream_t s);
hipError_t launch_batch_reset(const BatchArgs& a, hipStream_t s);
// Both screen kernels (the second when a.t2), in stream order.
hipError_t launch_screen(const ScreenArgs& a, int grid1, int grid2, hipStream_t s);

constexpr int kMaxServe = 8;  // codes one server can hold

// Differentiable unrolled min-sum (bsd_unroll.hip).  Graph in CSC order
// (edge = CSC position) with each row's edges in ascending column order.
constexpr int kUnrollBlock = 64;  // one wave per shot
struct UnrollArgs {
  int32_t m, n, nnz, T, K, nseg;  // nseg = ceil(T / K) checkpoints per shot
  const int32_t* colptr;          // [n + 1]
  const int32_t* rowptr;          // [m + 1]
  const int32_t* rowedge;         // [nnz]
  long long shots;
  const uint8_t* syn;             // [shots][m]
  const void* lam;                // [n]
  const void* alpha;              // [T]
  void* post;                     // forward output [shots][n]
  void* ckpt;                     // [shots][nseg][nnz]: E(0), E(K), E(2K), ...
  const void* gpost;              // backward input [shots][n]
  void* gl_part;                  // [shots][n] per-shot dL/dLambda
  void* ga_part;                  // [shots][T] per-shot dL/dalpha
  void* grad_lam;                 // [n]
  void* grad_alpha;               // [T]
  double llr_max;
};
// bsd_unroll_backward_noalloc: the partial gradients live in a device array
// of the library (bsd_unroll.hip); noalloc_scratch gives its address on
// `device`, which must be current.
constexpr size_t kNoAllocScratchBytes = (size_t)8 << 20;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(int device, void** ptr);
hipError_t launch_unroll_forward(const UnrollArgs& a, int elem, hipStream_t s);
hipError_t launch_unroll_backward(const UnrollArgs& a, int elem, hipStream_t s);
size_t unroll_bwd_lds(const UnrollArgs& a, int elem);
hipError_t launch_emit(const EmitArgs& a, hipStream_t s);
hipError_t set_kernel_limits(int cpt, int pw, size_t lds);
hipError_t batched_occupancy(int cpt, int pw, int block, size_t lds, int* blocks_per_cu);

size_t lds_bytes_for(const DevGraph& g);

// Columns-per-lane values that have compiled kernels: the smallest one >= c.
inline int supported_cpt(int c) {
  if (c <= 16) return c < 1 ? 1 : c;
  if (c <= 17) return 17;
  if (c <= 20) return 20;
  if (c <= 24) return 24;
  if (c <= 32) return 32;
  return -1;
}
inline int max_block_for_cpt(int cpt) { return cpt > 9 ? 512 : 1024; }

}  // namespace bsd
