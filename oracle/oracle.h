/*
 * CPU oracle of the BP-guided beam-search decoder (test infrastructure).
 *
 * This header belongs to the oracle only.  The oracle is a plain, slow,
 * step-by-step implementation of the paper's Appendix A (min-sum BP,
 * eqs. (1)-(4)), Algorithm 2 (masked BP) and Algorithm 3 with Appendix B
 * (beam search).  It exists to check the GPU library; nothing in the
 * product path may call it.  Every routine is instantiated twice: in double
 * precision (the correctness reference) and in single precision with the
 * same, natural order of operations (every sum left to right in ascending
 * neighbour index; the path score as an aligned pairwise tree over column
 * index).
 *
 * Arrays are host memory owned by the caller.  Edge messages are indexed by
 * the position of the edge in the CSC of H (columns in order, rows ascending
 * within a column).
 */
#ifndef BSD_ORACLE_H
#define BSD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oracle_problem_s* oracle_problem;

typedef struct {
  int32_t col; /* masked error node j */
  int32_t val; /* its fixed value v in {0,1} */
} oracle_pair;

typedef struct {
  int32_t max_rounds, beam_width, initial_iters, iters_per_round, num_results;
  double alpha;   /* min-sum scaling applied to eq. (1); 1.0 is eq. (1) as printed */
  double llr_max; /* saturation of every D and E message (and of an empty min) */
  /* Optional per-iteration scaling: iteration t of every BP run (initial and
   * masked) scales eq. (1) by alpha_sched[min(t, n_alpha) - 1] instead of
   * alpha.  NULL / 0: alpha throughout. */
  const double* alpha_sched;
  int32_t n_alpha;
} oracle_params;

typedef struct {
  double min_abs_post;      /* smallest |posterior LLR| computed in any iteration of any run */
  double min_nextpos_gap;   /* smallest gap between the two least |sum_LLR| of any run (inf if none) */
  double min_score_gap_rel; /* smallest relative gap between adjacent ranked child scores */
  int64_t runs;             /* BP runs executed */
  int64_t iterations;       /* sum of iterations over runs */
  int64_t clamp_events;     /* messages saturated at +-llr_max */
  int32_t rounds;           /* beam rounds entered */
  int32_t winner_round;     /* round of the returned solution (0 = initial BP), -1 if none */
  int32_t winner_gen;       /* generation index of the winner within its round */
  int32_t n_results;        /* valid solutions collected (num_results > 1) */
} oracle_shot_diag;

/* Build from the CSC of H (m x n), priors p (0 < p_j < 1) and the CSC of the
 * logical matrix A (k x n).  Returns NULL on malformed input. */
oracle_problem oracle_problem_create(int32_t m, int32_t n, int32_t k,
                                     const int32_t* h_colptr, const int32_t* h_rowidx,
                                     const double* p,
                                     const int32_t* l_colptr, const int32_t* l_rowidx);
void oracle_problem_destroy(oracle_problem pr);

/* One run of masked BP (Algorithm 2) from E(0) = e_start (NULL: the priors
 * on every edge).  Runs up to max_iters iterations, stopping at the first
 * iteration whose hard decision satisfies the (masked) syndrome when
 * stop_on_converge != 0.  Outputs: e_out (nnz) = E at the last iteration,
 * sum_llr (n) = sum of posteriors over the iterations run (masked nodes 0),
 * ehat (n) = last hard decision (masked nodes = 0, or their value v if the
 * run converged), post_last (n, may be NULL) = last posteriors, iters,
 * converged.  Returns 0, or -1 on bad arguments. */
int oracle_bp_run_f64(oracle_problem pr, const double* e_start, const oracle_pair* pairs,
                      int32_t npairs, const uint8_t* s, int32_t max_iters, double alpha,
                      double llr_max, int32_t stop_on_converge, double* e_out, double* sum_llr,
                      uint8_t* ehat, double* post_last, int32_t* iters, int32_t* converged);
int oracle_bp_run_f32(oracle_problem pr, const float* e_start, const oracle_pair* pairs,
                      int32_t npairs, const uint8_t* s, int32_t max_iters, float alpha,
                      float llr_max, int32_t stop_on_converge, float* e_out, float* sum_llr,
                      uint8_t* ehat, float* post_last, int32_t* iters, int32_t* converged);

/* Path score and next branching node of a finished run (Algorithm 3):
 * next_pos = argmin over unmasked j of |sum_llr[j]| (lowest j on ties, -1 if
 * every node is masked); score = sum over unmasked j of |sum_llr[j]| / iters
 * (0 when iters == 0). */
int oracle_score_f64(oracle_problem pr, const double* sum_llr, const oracle_pair* pairs,
                     int32_t npairs, int32_t iters, int32_t* next_pos, double* score);
int oracle_score_f32(oracle_problem pr, const float* sum_llr, const oracle_pair* pairs,
                     int32_t npairs, int32_t iters, int32_t* next_pos, float* score);

/* Beam-search decoding (Algorithm 3) of `shots` syndromes (uint8 shots x m).
 * Outputs corrections (shots x n), logical flips A*ehat mod 2 (shots x k),
 * converged (shots), and per-shot diagnostics (may be NULL).  Shots are
 * spread over `threads` host threads (0 = all cores).  Returns 0 or -1. */
int oracle_decode_f64(oracle_problem pr, const oracle_params* prm, int64_t shots,
                      const uint8_t* syndromes, uint8_t* corrections, uint8_t* flips,
                      uint8_t* converged, oracle_shot_diag* diag, int32_t threads);
int oracle_decode_f32(oracle_problem pr, const oracle_params* prm, int64_t shots,
                      const uint8_t* syndromes, uint8_t* corrections, uint8_t* flips,
                      uint8_t* converged, oracle_shot_diag* diag, int32_t threads);

#ifdef __cplusplus
}
#endif
#endif
