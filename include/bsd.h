/*
 * bsd.h -- C ABI of the MI355X beam-search decoder for quantum LDPC codes.
 *
 * The decoder is the BP-guided beam search of "Beam search decoder for
 * quantum LDPC codes" (Ye, Wecker, Delfosse): min-sum belief propagation on
 * the Tanner graph of a check matrix H (Appendix A, eqs. (1)-(4)), masked BP
 * runs that fix the least reliable error node to 0 and to 1 (Algorithm 2),
 * and a beam of paths scored by their summed posterior LLRs and pruned to
 * beam_width (Algorithm 3, Appendix B).  All decoding runs on the GPU in
 * hand-written HIP kernels for gfx950.
 *
 * Conventions
 *  - Matrices are given in compressed sparse column form (CSC): colptr has
 *    n+1 entries starting at 0, rowidx lists the rows of column j in
 *    colptr[j]..colptr[j+1]-1 in strictly ascending order.
 *  - Edge messages exchanged through bsd_bp_run are indexed by the position
 *    of the edge in the CSC of H.
 *  - All functions return a bsd_status; on failure bsd_last_error() returns
 *    a message for the calling thread.  Outputs are unspecified on failure.
 *  - A syndrome that no correction satisfies is not an error: the shot is
 *    reported with converged = 0.
 */
#ifndef BSD_H
#define BSD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BSD_OK = 0,
  BSD_EINVAL = -1,  /* invalid argument (message says which) */
  BSD_ENOMEM = -2,  /* device or host allocation failed */
  BSD_EDEVICE = -3, /* HIP runtime error (message includes hipGetErrorString) */
  BSD_EBUSY = -4    /* code handle still in use */
} bsd_status;

typedef enum {
  BSD_MODE_BATCHED = 0, /* one persistent kernel decodes every shot of the call */
  BSD_MODE_PLAIN = 1    /* one kernel launch per BP run; beam bookkeeping on the host */
} bsd_mode;

/* Opaque handle: the device-resident Tanner graph of H, the prior LLRs and
 * the logical matrix A. */
typedef struct bsd_code_s* bsd_code;

/* Decoder parameters: the five parameters of Algorithm 3 (Table I names
 * configurations by them) plus the min-sum scaling and the execution mode.
 *   max_rounds       rounds of branching after the initial BP run (>= 0)
 *   beam_width       paths kept after each round (1..64)
 *   initial_iters    iterations of the initial BP run (>= 0)
 *   iters_per_round  iterations of each masked BP run (>= 0)
 *   num_results      solutions to collect before returning (1..64); with
 *                    more than one, the lightest by wt(e) = sum_j e_j
 *                    log((1-p_j)/p_j) is returned (Appendix B)
 *   alpha            scaling of the detector-to-error messages of eq. (1);
 *                    1.0 is eq. (1) as printed (> 0, finite)
 *   mode             a bsd_mode value
 *   flags            bsd_flag bits */
typedef struct {
  int32_t max_rounds;
  int32_t beam_width;
  int32_t initial_iters;
  int32_t iters_per_round;
  int32_t num_results;
  float alpha;
  int32_t mode;
  int32_t flags; /* bitwise OR of bsd_flag values (0 = defaults) */
} bsd_params;

typedef enum {
  /* Batched mode: record the call's kernels in a HIP graph and replay it
   * when a later call repeats the same buffers, shot count and parameters. */
  BSD_FLAG_GRAPH = 1,
  /* Compute the check phase of iteration 1 of every initial BP run with
   * eq. (1).  By default it is taken from a table formed once per (code,
   * alpha): from the priors, eq. (1) depends on the syndrome only through
   * the factor (-1)^{s_i}, and the table holds the s = 0 values formed with
   * the kernels' own single-precision operations.  Results are identical
   * either way; this flag exists to check that. */
  BSD_FLAG_DENSE_FIRST = 2,
  /* Scale eq. (1) at iteration t of every BP run (initial and masked) by the
   * code's schedule entry min(t, n) (bsd_code_set_alpha_schedule) instead of
   * alpha: the per-iteration factors the unrolled decoder learns. */
  BSD_FLAG_ALPHA_SCHEDULE = 4,
  /* Batched mode: skip the sparse screen of iteration 1.  By default, when
   * every prior LLR is positive, initial_iters >= 1 and num_results = 1, a
   * first kernel computes iteration 1 of each shot's initial run only for
   * the columns of its flipped detectors (every other column decides 0 at
   * t = 1) and finishes the shots that converge there; the persistent
   * decoder takes the rest.  Results are identical either way. */
  BSD_FLAG_NO_SCREEN = 8,
  /* Batched mode: screen iteration 1 only.  By default the screen also
   * computes iteration 2 of shots that iteration 1 leaves unconverged (when
   * initial_iters >= 2): only rows that flipped or receive a negative E(1)
   * can send a negative message at t = 2, every other row's message is
   * bounded from below, and the columns whose bounded posterior is not
   * positive get exact messages.  Results are identical either way. */
  BSD_FLAG_NO_SCREEN2 = 16,
  /* Batched mode with the screen: also launch the persistent decoder on a
   * second stream beside the screen, where it takes the shots the screen
   * hands on while the screen still runs, as compute units free up.  It is
   * launched only while the stream's last synchronous call handed on under
   * 2 % of its shots (beside a screen that hands on many it slows both), and
   * not with BSD_FLAG_GRAPH.  The dense work then hides under the screen's
   * last waves but slows them as much; calls pipelined on two streams fill
   * that tail anyway.  Results are identical either way. */
  BSD_FLAG_BESIDE = 32
} bsd_flag;

/* Work counters of one bsd_decode_ex call. */
typedef struct {
  int64_t runs;           /* BP runs executed (initial and masked) */
  int64_t iterations;     /* BP iterations summed over runs */
  int64_t edge_updates;   /* iterations x Tanner edges, summed over runs */
  int64_t deep_shots;     /* shots whose initial BP run did not converge */
  double kernel_ms;       /* device time of the decoding kernels (HIP events) */
  int64_t screened_shots; /* batched mode: shots finished by the screen (iteration 1 or 2) */
  double screen_ms;       /* batched mode: device time of the screen (part of kernel_ms) */
  int64_t screened2_shots; /* batched mode: of those, shots finished at iteration 2 */
} bsd_stats;

/* Build a code handle on the current HIP device (Appendix A: the decoding
 * problem (H, A, p)).
 *   m, n, k      detectors (rows of H), fault columns, logical rows of A
 *   h_colptr     host, n+1 int32: CSC column pointers of H
 *   h_rowidx     host, nnz int32: CSC row indices of H (ascending per column)
 *   p            host, n doubles: fault probabilities, 0 < p_j < 1; the
 *                prior LLRs log((1-p_j)/p_j) are formed in double precision
 *                and rounded once to float
 *   l_colptr     host, n+1 int32: CSC column pointers of A (may be NULL if k = 0)
 *   l_rowidx     host, int32: CSC row indices of A
 *   out          receives the handle
 * The caller keeps ownership of every array; they may be freed on return.
 * Limits: m <= 2048, n <= 16384, k <= 64, column degree <= 8, row degree
 * <= 252, and the fp32 edge messages of one BP run (4 * nnz bytes plus
 * about 7 KB of per-run state) must fit in the 160 KB LDS of one compute
 * unit (nnz <= 39150).
 * Errors: BSD_EINVAL for malformed CSC, p outside (0,1) or limits exceeded;
 * BSD_ENOMEM, BSD_EDEVICE. */
bsd_status bsd_code_create(int32_t m, int32_t n, int32_t k, const int32_t* h_colptr,
                           const int32_t* h_rowidx, const double* p, const int32_t* l_colptr,
                           const int32_t* l_rowidx, bsd_code* out);

/* Release a code handle and every device buffer it owns, after the work
 * that asynchronous calls enqueued has finished.  BSD_EBUSY if a call on it
 * is still in progress in another thread, or a server holds it. */
bsd_status bsd_code_destroy(bsd_code code);

/* Decode `shots` syndromes with the beam search of Algorithm 3.
 *   syndromes      uint8 [shots x m], values 0/1 (s = H e)
 *   corrections    uint8 [shots x n]: the returned e-hat (0/1)
 *   logical_flips  uint8 [shots x k]: A e-hat mod 2 (compare with A e)
 *   converged      uint8 [shots]: 1 iff H e-hat = s was reached
 *   stream         hipStream_t to run on (NULL: the default stream)
 * Buffers may be device memory (decoded in place) or host memory (told apart
 * with hipPointerGetAttributes; then staged through device buffers the code
 * handle keeps, bus transfers included).  They are owned by the caller and
 * must not overlap.
 * Batched mode with every buffer in device memory is asynchronous: the call
 * returns once the work is enqueued on `stream`, and the outputs are ready
 * when that work completes.  Syndrome bytes outside {0,1} are then found on
 * the device and reported by bsd_code_sync.  A handle may be used from
 * several streams at once (and from several host threads): each stream gets
 * a workspace of its own, allocated on its first batched call, for at most 8
 * streams per handle (BSD_EBUSY beyond).  Batches enqueued in turn on
 * several streams overlap on the device: a call made while other streams'
 * calls are still running gives the persistent decoder a share of its grid
 * (results are identical).  Host buffers and the plain mode are
 * synchronous.
 * Errors: BSD_EINVAL for bad parameters (and, when synchronous, syndrome
 * bytes outside {0,1}); BSD_ENOMEM when the workspace cannot be allocated;
 * BSD_EDEVICE. */
bsd_status bsd_decode(bsd_code code, const bsd_params* prm, int64_t shots,
                      const uint8_t* syndromes, uint8_t* corrections, uint8_t* logical_flips,
                      uint8_t* converged, void* stream);

/* Wait for the work that calls on `stream` enqueued on this code, and
 * report what an asynchronous call found since the last check: BSD_EINVAL
 * if syndrome bytes outside {0,1} were seen (reported once), BSD_EDEVICE if
 * the last call finished fewer shots than it was given.  BSD_OK when the
 * handle has no work on that stream. */
bsd_status bsd_code_sync(bsd_code code, void* stream);

/* As bsd_decode, synchronous, also filling `stats` (host, may be NULL) and,
 * when `latency_ticks` (uint32 [shots], may be NULL) is given, the
 * per-shot decode time in 10 ns ticks: batched mode, the 100 MHz device
 * clock from the start of the shot's initial BP run to the write of its
 * result; plain mode, the host's time for the shot (all its launches and
 * transfers). */
bsd_status bsd_decode_ex(bsd_code code, const bsd_params* prm, int64_t shots,
                         const uint8_t* syndromes, uint8_t* corrections, uint8_t* logical_flips,
                         uint8_t* converged, void* stream, bsd_stats* stats,
                         uint32_t* latency_ticks);

/* One run of masked BP (Algorithm 2) on the GPU, for checking messages.
 *   e_start    device, float [nnz] in CSC edge order: E(0); NULL = priors
 *   pairs      host, int32 [2 * npairs]: (column, value) of the masked nodes
 *   syndrome   device, uint8 [m]
 *   max_iters  iterations to run (>= 0); stop_on_converge != 0 stops at the
 *              first iteration whose hard decision satisfies H e = s'
 *   alpha      scaling of eq. (1)
 * Outputs (device, may be NULL): e_out float [nnz] (E at the last iteration,
 * CSC order), sum_llr float [n] (posteriors summed over the iterations run;
 * 0 on masked nodes), ehat uint8 [n] (last hard decision; masked nodes hold
 * their value if the run converged, else 0), and on the host: iters,
 * converged, next_pos (least reliable unmasked node, -1 if none) and score
 * (sum of |sum_llr| over unmasked nodes divided by iters).
 * Synchronous.  Errors: BSD_EINVAL, BSD_EDEVICE. */
bsd_status bsd_bp_run(bsd_code code, const float* e_start, const int32_t* pairs, int32_t npairs,
                      const uint8_t* syndrome, int32_t max_iters, float alpha,
                      int32_t stop_on_converge, float* e_out, float* sum_llr, uint8_t* ehat,
                      int32_t* iters, int32_t* converged, int32_t* next_pos, float* score,
                      void* stream);

/* Choose the batched kernel's workgroup size and number of resident
 * workgroups for this code and parameters by timing each admissible choice
 * on the given syndromes (device, uint8 [shots x m]), and keep the fastest
 * for later calls.  When the environment variable BSD_TUNE_CACHE names a
 * file, choices are read from and appended to it, keyed by a digest of
 * (H, p, parameters, device).  Outputs (host, may be NULL): the chosen
 * block size, grid size and the best time of one call in milliseconds.
 * Errors: as bsd_decode. */
bsd_status bsd_code_autotune(bsd_code code, const bsd_params* prm, int64_t shots,
                             const uint8_t* syndromes, int32_t* block_threads,
                             int32_t* grid_blocks, float* best_ms, void* stream);

/* Set (n > 0, host floats, each positive and finite; copied) or clear
 * (n = 0) the per-iteration scaling schedule that BSD_FLAG_ALPHA_SCHEDULE
 * selects.  BSD_EBUSY while a decode on the code is running. */
bsd_status bsd_code_set_alpha_schedule(bsd_code code, int32_t n, const float* alphas);

/* Geometry of a code handle: nnz of H and the threads per workgroup and
 * workgroups the batched kernel will use.  Any pointer may be NULL. */
bsd_status bsd_code_info(bsd_code code, int64_t* nnz, int32_t* block_threads, int32_t* grid_blocks,
                         int32_t* lds_bytes);

/* ------------------------------------------------------------------------
 * Serving: requests that arrive over time are decoded continuously.
 *
 * A server keeps one persistent decoder per code running on the GPU, each on
 * its own stream with its own workgroups.  By default a code whose BP run
 * fills a compute unit's LDS gets one workgroup on each of 1/32 of the units,
 * and any other code beam_width workgroups (at least 16): sizes for a few
 * thousand requests per second per code, since idle workgroups poll.
 * Heavier loads pass larger grid_blocks.  Requests pass through a ring per
 * code in pinned host memory.  The host writes the syndrome and publishes it,
 * and the decoder claims it as soon as one of its workgroups is free.  This
 * is the decoder's own work queue, so several requests of a code and the
 * child runs of deep ones share the workgroups (continuous batching).  The
 * decoder writes the outputs back into the ring row and raises that row's
 * done flag.  Admission is by memory: a code's ring has a fixed number of
 * rows, sized from a byte budget, and a request is admitted only when its
 * row is free.
 * Idle workgroups take turns (one at a time per decoder) reading the host's
 * published count over the bus and mirroring it in device memory.
 * The decoders must all run at once: each needs a hardware queue of its own
 * (HIP's GPU_MAX_HW_QUEUES bounds them per process) and its compute units.
 * Creation launches them one at a time, largest LDS first, and waits until
 * every workgroup of one is resident before launching the next; a decoder
 * that does not get there within 5 s makes creation fail with BSD_EDEVICE.
 * A server holds its codes (bsd_code_destroy returns BSD_EBUSY meanwhile).
 * Its kernels end when it is destroyed.  A decoder also ends on its own
 * after a stretch without work (20 s by default, bsd_server_opts.idle_ms),
 * giving its compute units back; the next submit or poll on that code
 * starts it again, with every earlier request and context intact. */
typedef struct bsd_server_s* bsd_server;

/* Options of bsd_server_create_ex (zero-initialised = defaults). */
typedef struct {
  int64_t ring_bytes; /* pinned host memory for the request rings (0 = 64 MiB) */
  int64_t idle_ms;    /* a decoder ends after this long without work, 1..40000
                         (0 = 20 s); a later request starts it again */
} bsd_server_opts;

/* Create a server for ncodes (1..8) distinct codes of the current device.
 *   params       host, [ncodes]: decoder of each code (batched mode)
 *   grid_blocks  host, [ncodes] or NULL: workgroups per decoder (0 = automatic)
 *   ring_bytes   pinned host memory for the request rings (0 = 64 MiB), split
 *                evenly; each code gets a power of two in [64, 4096] rows
 * Errors: BSD_EINVAL, BSD_ENOMEM, BSD_EDEVICE. */
bsd_status bsd_server_create(int32_t ncodes, const bsd_code* codes, const bsd_params* params,
                             const int32_t* grid_blocks, int64_t ring_bytes, bsd_server* out);

/* As bsd_server_create, with options (may be NULL).  Also BSD_EINVAL when
 * ncodes exceeds the hardware queues HIP gives the process
 * (GPU_MAX_HW_QUEUES, default 4), since every decoder needs one. */
bsd_status bsd_server_create_ex(int32_t ncodes, const bsd_code* codes, const bsd_params* params,
                                const int32_t* grid_blocks, const bsd_server_opts* opts,
                                bsd_server* out);

/* State of one code's decoder: whether its kernel is running now, and how
 * many times it has been launched (1 + relaunches after idle exits).  Either
 * pointer may be NULL. */
bsd_status bsd_server_info(bsd_server s, int32_t code, int32_t* running, int64_t* launches);

/* Submit one syndrome (host, uint8 [m], copied) for code `code`; `ticket`
 * receives the request's number within that code.  BSD_EBUSY when the ring
 * row it needs is still held by an earlier request (poll that one first).
 * Starts the code's decoder again if it has ended after its idle limit
 * (BSD_EDEVICE if it cannot get every workgroup running within 5 s; the
 * request stays published and a later poll tries again). */
bsd_status bsd_server_submit(bsd_server s, int32_t code, const uint8_t* syndrome, int64_t* ticket);

/* If request `ticket` of `code` has finished, copy its outputs (host, may be
 * NULL: corrections [n], logical_flips [k], converged [1], device_ticks: the
 * decode time on the device in 100 MHz ticks) and release its ring row;
 * BSD_EBUSY (no message) when it has not finished yet. */
bsd_status bsd_server_poll(bsd_server s, int32_t code, int64_t ticket, uint8_t* corrections,
                           uint8_t* logical_flips, uint8_t* converged, uint32_t* device_ticks);

/* Stop the server's kernels and release it. */
bsd_status bsd_server_destroy(bsd_server s);

/* Latency summary of bsd_serve_poisson (microseconds, arrival to result as
 * seen by the host; percentiles by nearest rank). */
typedef struct {
  int64_t requests;
  double seconds;        /* first arrival to last result */
  double offered_per_s;  /* requests / span of the arrival times */
  double served_per_s;   /* requests / seconds */
  double p50_us, p99_us, p999_us, max_us;
  int64_t code_requests[8];
  double code_p50_us[8], code_p99_us[8], code_p999_us[8];
  int64_t admission_waits; /* requests that found their ring row busy and waited */
} bsd_serve_report;

/* Drive a server with `requests` Poisson arrivals at `rate` per second.
 * Each arrival picks code i with probability mix[i] / sum(mix) (seeded, a
 * counter-based generator) and takes the next syndrome of that code from
 * syndromes[i] (host, uint8 [n_syndromes[i] x m_i], used in order,
 * cyclically).  Outputs, all host and optional: corrections[i] [n_syndromes[i]
 * x n_i], logical_flips[i], converged[i] by syndrome index; latency_us and
 * code_of [requests]; report.  Runs in the calling thread until every request
 * has been answered (errors: BSD_EDEVICE after a generous timeout). */
bsd_status bsd_serve_poisson(bsd_server s, double rate, const double* mix, int64_t requests,
                             const uint8_t* const* syndromes, const int64_t* n_syndromes,
                             uint64_t seed, uint8_t* const* corrections,
                             uint8_t* const* logical_flips, uint8_t* const* converged,
                             double* latency_us, int32_t* code_of, bsd_serve_report* report);

/* ------------------------------------------------------------------------
 * Differentiable unrolled min-sum (training the decoder's factors).
 *
 * Forward: T flooding iterations of min-sum (Appendix A, eqs. (1)-(3)) from
 * E(0) = Lambda, with the messages of eq. (1) scaled by alpha_t at
 * iteration t, no early stop; output post(T), the final posterior LLRs (the
 * final marginal is P(e_j = 1) = 1 / (1 + exp(post_j))).  Messages are
 * saturated to +-1e30 as in the decoder.  The adjoint gives dL/dLambda and
 * dL/dalpha from dL/dpost(T), recomputing every K iterations from
 * checkpoints E(0), E(K), E(2K), ... written by the forward pass.  It is
 * exact wherever no check has a tie between its two smallest |E| and no
 * message is 0 (there the map is not differentiable), and treats the
 * saturation as inactive.  One wavefront per shot with the shot's messages
 * in LDS: (K + 3) * nnz + n elements must fit in 160 KB.
 *
 * Arrays are device memory of element size elem_bytes (4: float, 8: double)
 * and belong to the caller:
 *   syndromes    uint8 [shots x m] (0/1)
 *   lambda       [n] prior LLRs;   alpha [T] scalings
 *   post         [shots x n] output of the forward pass
 *   checkpoints  [shots x ceil(T/K) x nnz] (bsd_unroll_sizes), written by the
 *                forward pass and read by the backward pass (E in CSC order)
 *   grad_post    [shots x n] dL/dpost(T)
 *   grad_lambda  [n], grad_alpha [T] outputs, summed over shots in shot order
 *   workspace    [shots x (n + T)] scratch of the backward pass
 * Both calls are asynchronous on `stream`.  Errors: BSD_EINVAL, BSD_ENOMEM,
 * BSD_EDEVICE. */
bsd_status bsd_unroll_sizes(bsd_code code, int32_t T, int32_t K, int64_t shots,
                            int64_t* checkpoint_elems, int64_t* workspace_elems);
bsd_status bsd_unroll_forward(bsd_code code, int32_t elem_bytes, int32_t T, int32_t K, int64_t shots,
                              const uint8_t* syndromes, const void* lambda, const void* alpha,
                              void* post, void* checkpoints, void* stream);
bsd_status bsd_unroll_backward(bsd_code code, int32_t elem_bytes, int32_t T, int32_t K, int64_t shots,
                               const uint8_t* syndromes, const void* lambda, const void* alpha,
                               const void* checkpoints, const void* grad_post, void* grad_lambda,
                               void* grad_alpha, void* workspace, void* stream);

/* As bsd_unroll_backward, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): no workspace argument, and no allocation.  The per-shot
 * partial gradients go to an 8 MiB array the library holds on each device
 * it runs on, until the process ends: shots * (n + T) * elem_bytes must not
 * exceed 8 MiB (BSD_EINVAL with the limit otherwise; 6,200 shots of the
 * [[144,12,12]] graph at T = 25 in double precision).  Calls on one device
 * share the array: calls that overlap on one device race.  Results equal
 * bsd_unroll_backward's bit for bit.  Asynchronous on `stream`. */
bsd_status bsd_unroll_backward_noalloc(bsd_code code, int32_t elem_bytes, int32_t T, int32_t K,
                                       int64_t shots, const uint8_t* syndromes, const void* lambda,
                                       const void* alpha, const void* checkpoints,
                                       const void* grad_post, void* grad_lambda, void* grad_alpha,
                                       void* stream);

/* Thread-local message describing the last failure in this thread. */
const char* bsd_last_error(void);

/* Library version string. */
const char* bsd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BSD_H */
