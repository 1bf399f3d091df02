// CPU oracle of the BP-guided beam-search decoder -- TEST INFRASTRUCTURE.
//
// Only the tests, the smoke check and the bench's CPU-baseline leg may load
// this library.  It is written from the paper alone and shares no code with
// the GPU library: min-sum BP (Appendix A, eqs. (1)-(4) and the stopping
// rule), masked BP (Algorithm 2) and the beam search (Algorithm 3, with the
// ordering and on-the-fly pruning of Appendix B).  It favours being
// obviously correct over being fast: eq. (1) is evaluated literally, as a
// product and a minimum over N(d_i) minus {e_j}, for every edge.
//
// Readings where the paper is silent (they bind the GPU library too):
//  * eq. (1) is scaled by alpha (alpha = 1 is eq. (1) as printed);
//  * sgn(x) = -1 iff x < 0; eq. (4) uses "<= 0", so both zeros decide 1;
//  * a minimum over an empty set is llr_max, and every D and E message is
//    saturated to [-llr_max, llr_max];
//  * sums run left to right in ascending neighbour index; E is the literal
//    exclusive sum of eq. (2), not posterior minus D;
//  * sum_LLR sums the posteriors of iterations 1..iters of the current run;
//  * the path score sums |sum_LLR| over unmasked nodes as an aligned pairwise
//    tree over column index (zeros for masked nodes and padding), then
//    divides by iters (score 0 when iters = 0);
//  * next_pos ties go to the lowest column; a path with no unmasked node
//    cannot branch and is dropped;
//  * paths are explored by (score desc, generation asc), child generation
//    2k+v for the k-th explored parent and value v; pruning keeps the first
//    beam_width children in that order, which is what on-the-fly insertion
//    with strict ">" and ejection of the latest-generated minimum keeps;
//  * when no solution is found the output is the last hard decision (masked
//    values filled in) of the best path of the final set, converged = 0;
//  * num_results > 1: results is a set of distinct solutions; converged
//    children keep branching; ties in weight go to the first found; if the
//    rounds run out with fewer results than asked, the lightest found is
//    returned.

#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <memory>
#include <thread>
#include <vector>

namespace {

struct Problem {
  int m = 0, n = 0, k = 0;
  std::vector<int> colptr, rowidx;            // CSC of H: edge e = position in CSC
  std::vector<std::vector<int>> row_edges;    // N(d_i) as CSC edge ids, ascending column
  std::vector<int> edge_col;                  // column of each edge
  std::vector<double> lambda64;               // Lambda_j = log((1 - p_j) / p_j)
  std::vector<float> lambda32;
  std::vector<double> weight;                 // wt contribution of e_j (same as Lambda_j)
  std::vector<std::vector<int>> l_rows;       // logical rows flipped by column j
};

template <class T> const std::vector<T>& lambda_of(const Problem& p);
template <> const std::vector<double>& lambda_of<double>(const Problem& p) { return p.lambda64; }
template <> const std::vector<float>& lambda_of<float>(const Problem& p) { return p.lambda32; }

template <class T>
struct RunOut {
  std::vector<T> e;        // E at the last iteration (CSC edge order)
  std::vector<T> sum_llr;  // per column
  std::vector<uint8_t> ehat;
  std::vector<T> post;     // last posteriors
  int iters = 0;
  bool converged = false;
  double min_abs_post = std::numeric_limits<double>::infinity();
  int64_t clamps = 0;
};

template <class T>
inline T saturate(T x, T lim, int64_t& clamps) {
  if (x > lim) { ++clamps; return lim; }
  if (x < -lim) { ++clamps; return -lim; }
  return x;
}

// Algorithm 2 (masked_BP), built on the min-sum updates of Appendix A.
// Scaling of eq. (1) at iteration t (1-based): the schedule's entry, the last
// one past its end, or the single alpha.
template <class T>
T alpha_at(T alpha, const std::vector<T>& sched, int t) {
  if (sched.empty()) return alpha;
  return sched[std::min<size_t>((size_t)t, sched.size()) - 1];
}

template <class T>
void masked_bp(const Problem& P, const T* e_start, const std::vector<oracle_pair>& pairs,
               const uint8_t* s, int max_iters, T alpha, T llr_max, bool stop, RunOut<T>& out,
               const std::vector<T>& sched = {}) {
  const int m = P.m, n = P.n;
  const int nnz = P.colptr[n];
  const std::vector<T>& lam = lambda_of<T>(P);

  // Masked nodes, and the syndrome with the columns of the nodes fixed to 1 flipped.
  std::vector<uint8_t> masked(n, 0);
  std::vector<uint8_t> sp(s, s + m);
  for (const oracle_pair& pv : pairs) {
    masked[pv.col] = 1;
    if (pv.val == 1)
      for (int e = P.colptr[pv.col]; e < P.colptr[pv.col + 1]; ++e) sp[P.rowidx[e]] ^= 1;
  }

  // E(0): the warm-start messages, or the priors on every edge.
  std::vector<T> E(nnz), D(nnz, T(0));
  for (int e = 0; e < nnz; ++e) E[e] = e_start ? e_start[e] : lam[P.edge_col[e]];

  out.sum_llr.assign(n, T(0));
  out.ehat.assign(n, 0);
  out.post.assign(n, T(0));
  out.converged = false;
  out.iters = 0;

  for (int t = 1; t <= max_iters; ++t) {
    const T at = alpha_at<T>(alpha, sched, t);
    // Eq. (1): detector-to-error messages from E(t-1), unmasked neighbours only.
    for (int i = 0; i < m; ++i) {
      const std::vector<int>& nb = P.row_edges[i];
      for (int a : nb) {
        if (masked[P.edge_col[a]]) continue;
        bool negative = sp[i] != 0;        // (-1)^{s_i}
        T mag = llr_max;                   // min over an empty set
        for (int b : nb) {
          if (b == a || masked[P.edge_col[b]]) continue;
          if (E[b] < T(0)) negative = !negative;
          T ab = std::fabs(E[b]);
          if (ab < mag) mag = ab;
        }
        T d = saturate<T>(at * mag, llr_max, out.clamps);
        D[a] = negative ? -d : d;
      }
    }
    // Eqs. (2)-(4) for the unmasked error nodes.
    for (int j = 0; j < n; ++j) {
      if (masked[j]) { out.ehat[j] = 0; continue; }
      const int e0 = P.colptr[j], e1 = P.colptr[j + 1];
      T post = lam[j];                              // eq. (3)
      for (int e = e0; e < e1; ++e) post = post + D[e];
      for (int e = e0; e < e1; ++e) {               // eq. (2), exclusive sum
        T x = lam[j];
        for (int f = e0; f < e1; ++f)
          if (f != e) x = x + D[f];
        E[e] = saturate<T>(x, llr_max, out.clamps);
      }
      out.sum_llr[j] = out.sum_llr[j] + post;
      out.post[j] = post;
      out.ehat[j] = post <= T(0) ? 1 : 0;           // eq. (4)
      double ap = std::fabs((double)post);
      if (ap < out.min_abs_post) out.min_abs_post = ap;
    }
    out.iters = t;
    // Stopping rule: H ehat(t) = s', with the masked positions at 0.
    bool ok = true;
    for (int i = 0; i < m && ok; ++i) {
      int parity = 0;
      for (int a : P.row_edges[i]) parity ^= out.ehat[P.edge_col[a]];
      if (parity != sp[i]) ok = false;
    }
    if (ok) {
      out.converged = true;
      for (const oracle_pair& pv : pairs) out.ehat[pv.col] = (uint8_t)pv.val;
      if (stop) break;
      for (const oracle_pair& pv : pairs) out.ehat[pv.col] = 0;
      out.converged = false;  // not stopping: only the final iteration counts
    }
  }
  if (!stop && out.iters > 0) {
    // With stop disabled, report whether the last iteration satisfied the syndrome.
    bool ok = true;
    for (int i = 0; i < m && ok; ++i) {
      int parity = 0;
      for (int a : P.row_edges[i]) parity ^= out.ehat[P.edge_col[a]];
      if (parity != sp[i]) ok = false;
    }
    out.converged = ok;
    if (ok)
      for (const oracle_pair& pv : pairs) out.ehat[pv.col] = (uint8_t)pv.val;
  }
  out.e.assign(E.begin(), E.end());
}

// Aligned pairwise sum over x[lo, lo+len), zeros beyond n.
template <class T>
T tree_sum(const std::vector<T>& x, size_t lo, size_t len) {
  if (len == 1) return lo < x.size() ? x[lo] : T(0);
  size_t h = len / 2;
  return tree_sum(x, lo, h) + tree_sum(x, lo + h, h);
}

// next_pos and score of a finished run (Algorithm 3, Appendix B).
template <class T>
void score_run(const Problem& P, const std::vector<T>& sum_llr, const std::vector<uint8_t>& masked,
               int iters, int& next_pos, T& score, double& gap) {
  const int n = P.n;
  std::vector<T> a(n, T(0));
  next_pos = -1;
  T best = T(0), second = std::numeric_limits<T>::infinity();
  for (int j = 0; j < n; ++j) {
    if (masked[j]) continue;
    a[j] = std::fabs(sum_llr[j]);
    if (next_pos < 0 || a[j] < best) {
      if (next_pos >= 0) second = best;
      best = a[j];
      next_pos = j;
    } else if (a[j] < second) {
      second = a[j];
    }
  }
  gap = next_pos >= 0 ? (double)second - (double)best : std::numeric_limits<double>::infinity();
  size_t len = 1;
  while (len < (size_t)n) len <<= 1;
  T total = tree_sum(a, 0, len);
  score = iters > 0 ? total / (T)iters : T(0);
}

template <class T>
struct Path {
  std::vector<T> e;                 // edge_msgs
  std::vector<oracle_pair> pairs;   // pos_val_pairs
  std::vector<uint8_t> ehat;        // last hard decision, masked values filled in
  int next_pos = -1;
  T score = T(0);
  int gen = 0;
};

// Algorithm 3 for one syndrome.
template <class T>
void decode_one(const Problem& P, const oracle_params& prm, const uint8_t* s, uint8_t* corr,
                uint8_t* flips, uint8_t* conv, oracle_shot_diag& dg) {
  const int n = P.n;
  const T alpha = (T)prm.alpha, lmax = (T)prm.llr_max;
  std::vector<T> sched;
  for (int i = 0; i < prm.n_alpha; ++i) sched.push_back((T)prm.alpha_sched[i]);
  const int want = prm.num_results;
  dg.min_abs_post = std::numeric_limits<double>::infinity();
  dg.min_nextpos_gap = std::numeric_limits<double>::infinity();
  dg.min_score_gap_rel = std::numeric_limits<double>::infinity();
  dg.runs = dg.iterations = dg.clamp_events = 0;
  dg.rounds = 0;
  dg.winner_round = -1;
  dg.winner_gen = -1;
  dg.n_results = 0;

  std::vector<std::vector<uint8_t>> results;
  std::vector<double> result_wt;
  std::vector<std::pair<int, int>> result_origin;
  auto add_result = [&](const std::vector<uint8_t>& eh, int round, int gen) {
    for (const auto& r : results)
      if (r == eh) return;
    double w = 0.0;
    for (int j = 0; j < n; ++j)
      if (eh[j]) w += P.weight[j];
    results.push_back(eh);
    result_wt.push_back(w);
    result_origin.emplace_back(round, gen);
  };
  auto finish = [&](const std::vector<uint8_t>& eh, bool ok) {
    for (int j = 0; j < n; ++j) corr[j] = eh[j];
    for (int r = 0; r < P.k; ++r) flips[r] = 0;
    for (int j = 0; j < n; ++j)
      if (eh[j])
        for (int r : P.l_rows[j]) flips[r] ^= 1;
    *conv = ok ? 1 : 0;
  };
  auto finish_results = [&]() {
    size_t best = 0;
    for (size_t r = 1; r < results.size(); ++r)
      if (result_wt[r] < result_wt[best]) best = r;
    dg.winner_round = result_origin[best].first;
    dg.winner_gen = result_origin[best].second;
    dg.n_results = (int)results.size();
    finish(results[best], true);
  };
  auto account = [&](const RunOut<T>& r) {
    dg.runs += 1;
    dg.iterations += r.iters;
    dg.clamp_events += r.clamps;
    if (r.min_abs_post < dg.min_abs_post) dg.min_abs_post = r.min_abs_post;
  };

  // Initial standard BP run from the priors.
  RunOut<T> r0;
  std::vector<oracle_pair> none;
  masked_bp<T>(P, nullptr, none, s, prm.initial_iters, alpha, lmax, true, r0, sched);
  account(r0);
  if (r0.converged) {
    add_result(r0.ehat, 0, 0);
    if ((int)results.size() >= want) { finish_results(); return; }
  }
  std::vector<uint8_t> nomask(n, 0);
  Path<T> seed;
  seed.e = r0.e;
  seed.ehat = r0.ehat;
  double gap;
  T unused;
  score_run<T>(P, r0.sum_llr, nomask, r0.iters, seed.next_pos, unused, gap);
  if (gap < dg.min_nextpos_gap) dg.min_nextpos_gap = gap;
  seed.score = T(0);
  seed.gen = 0;

  std::vector<Path<T>> set;
  set.push_back(std::move(seed));
  const size_t bw = (size_t)prm.beam_width;

  for (int r = 1; r <= prm.max_rounds && !set.empty(); ++r) {
    dg.rounds = r;
    // Explore paths in descending score; equal scores by generation.
    std::stable_sort(set.begin(), set.end(), [](const Path<T>& a, const Path<T>& b) {
      if (a.score != b.score) return a.score > b.score;
      return a.gen < b.gen;
    });
    std::vector<Path<T>> next;   // next_set, bounded on the fly
    std::vector<T> all_scores;
    for (size_t kk = 0; kk < set.size(); ++kk) {
      const Path<T>& par = set[kk];
      if (par.next_pos < 0) continue;
      for (int v = 0; v <= 1; ++v) {
        Path<T> ch;
        ch.pairs = par.pairs;
        ch.pairs.push_back(oracle_pair{par.next_pos, v});
        ch.gen = (int)(2 * kk + v);
        RunOut<T> rr;
        masked_bp<T>(P, par.e.data(), ch.pairs, s, prm.iters_per_round, alpha, lmax, true, rr,
                     sched);
        account(rr);
        if (rr.converged) {
          add_result(rr.ehat, r, ch.gen);
          if ((int)results.size() >= want) { finish_results(); return; }
        }
        std::vector<uint8_t> msk(n, 0);
        for (const oracle_pair& pv : ch.pairs) msk[pv.col] = 1;
        score_run<T>(P, rr.sum_llr, msk, rr.iters, ch.next_pos, ch.score, gap);
        if (gap < dg.min_nextpos_gap) dg.min_nextpos_gap = gap;
        all_scores.push_back(ch.score);
        ch.e = std::move(rr.e);
        ch.ehat = rr.ehat;
        for (const oracle_pair& pv : ch.pairs) ch.ehat[pv.col] = (uint8_t)pv.val;
        // On-the-fly bounded insertion (Appendix B).
        if (next.size() < bw) {
          next.push_back(std::move(ch));
        } else {
          size_t worst = 0;  // minimum score; among equal minima the latest generated
          for (size_t q = 1; q < next.size(); ++q) {
            if (next[q].score < next[worst].score ||
                (next[q].score == next[worst].score && next[q].gen > next[worst].gen))
              worst = q;
          }
          if (ch.score > next[worst].score) next[worst] = std::move(ch);
        }
      }
    }
    std::sort(all_scores.begin(), all_scores.end());
    for (size_t q = 1; q < all_scores.size(); ++q) {
      double a = (double)all_scores[q - 1], b = (double)all_scores[q];
      double den = std::max(std::fabs(a), std::fabs(b));
      double rel = den > 0 ? (b - a) / den : 0.0;
      if (rel < dg.min_score_gap_rel) dg.min_score_gap_rel = rel;
    }
    set = std::move(next);
  }
  if (!results.empty()) { finish_results(); return; }
  // No solution: best path of the final set (or the initial run).
  if (!set.empty() && prm.max_rounds > 0) {
    size_t best = 0;
    for (size_t q = 1; q < set.size(); ++q)
      if (set[q].score > set[best].score ||
          (set[q].score == set[best].score && set[q].gen < set[best].gen))
        best = q;
    finish(set[best].ehat, false);
  } else {
    finish(r0.ehat, false);
  }
}

template <class T>
int bp_run_impl(oracle_problem h, const T* e_start, const oracle_pair* pairs, int npairs,
                const uint8_t* s, int max_iters, T alpha, T llr_max, int stop, T* e_out,
                T* sum_llr, uint8_t* ehat, T* post_last, int32_t* iters, int32_t* converged) {
  const Problem* P = reinterpret_cast<const Problem*>(h);
  if (!P || !s || max_iters < 0 || npairs < 0 || (npairs && !pairs)) return -1;
  std::vector<oracle_pair> pv(pairs, pairs + npairs);
  for (const oracle_pair& q : pv)
    if (q.col < 0 || q.col >= P->n || (q.val != 0 && q.val != 1)) return -1;
  RunOut<T> out;
  masked_bp<T>(*P, e_start, pv, s, max_iters, alpha, llr_max, stop != 0, out);
  const int nnz = P->colptr[P->n];
  if (e_out) std::memcpy(e_out, out.e.data(), sizeof(T) * nnz);
  if (sum_llr) std::memcpy(sum_llr, out.sum_llr.data(), sizeof(T) * P->n);
  if (ehat) std::memcpy(ehat, out.ehat.data(), P->n);
  if (post_last) std::memcpy(post_last, out.post.data(), sizeof(T) * P->n);
  if (iters) *iters = out.iters;
  if (converged) *converged = out.converged ? 1 : 0;
  return 0;
}

template <class T>
int score_impl(oracle_problem h, const T* sum_llr, const oracle_pair* pairs, int npairs, int iters,
               int32_t* next_pos, T* score) {
  const Problem* P = reinterpret_cast<const Problem*>(h);
  if (!P || !sum_llr || npairs < 0) return -1;
  std::vector<T> sl(sum_llr, sum_llr + P->n);
  std::vector<uint8_t> msk(P->n, 0);
  for (int q = 0; q < npairs; ++q) {
    if (pairs[q].col < 0 || pairs[q].col >= P->n) return -1;
    msk[pairs[q].col] = 1;
  }
  int np;
  T sc;
  double gap;
  score_run<T>(*P, sl, msk, iters, np, sc, gap);
  if (next_pos) *next_pos = np;
  if (score) *score = sc;
  return 0;
}

template <class T>
int decode_impl(oracle_problem h, const oracle_params* prm, int64_t shots, const uint8_t* syn,
                uint8_t* corr, uint8_t* flips, uint8_t* conv, oracle_shot_diag* diag, int threads) {
  const Problem* P = reinterpret_cast<const Problem*>(h);
  if (!P || !prm || shots < 0 || (shots && (!syn || !corr || !flips || !conv))) return -1;
  if (prm->beam_width < 1 || prm->max_rounds < 0 || prm->initial_iters < 0 ||
      prm->iters_per_round < 0 || prm->num_results < 1 || !(prm->alpha > 0) ||
      prm->n_alpha < 0 || (prm->n_alpha > 0 && !prm->alpha_sched) ||
      !(prm->llr_max > 0))
    return -1;
  int nt = threads > 0 ? threads : (int)std::thread::hardware_concurrency();
  if (nt < 1) nt = 1;
  if ((int64_t)nt > shots) nt = (int)std::max<int64_t>(shots, 1);
  auto work = [&](int tid) {
    for (int64_t q = tid; q < shots; q += nt) {
      oracle_shot_diag d{};
      decode_one<T>(*P, *prm, syn + q * P->m, corr + q * P->n, flips + q * P->k, conv + q, d);
      if (diag) diag[q] = d;
    }
  };
  if (nt == 1) {
    work(0);
  } else {
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t) pool.emplace_back(work, t);
    for (auto& th : pool) th.join();
  }
  return 0;
}

}  // namespace

extern "C" {

oracle_problem oracle_problem_create(int32_t m, int32_t n, int32_t k, const int32_t* h_colptr,
                                     const int32_t* h_rowidx, const double* p,
                                     const int32_t* l_colptr, const int32_t* l_rowidx) {
  if (m <= 0 || n <= 0 || k < 0 || !h_colptr || !h_rowidx || !p) return nullptr;
  if (h_colptr[0] != 0) return nullptr;
  for (int j = 0; j < n; ++j) {
    if (h_colptr[j + 1] < h_colptr[j]) return nullptr;
    for (int e = h_colptr[j]; e < h_colptr[j + 1]; ++e) {
      if (h_rowidx[e] < 0 || h_rowidx[e] >= m) return nullptr;
      if (e > h_colptr[j] && h_rowidx[e] <= h_rowidx[e - 1]) return nullptr;
    }
    if (!(p[j] > 0.0 && p[j] < 1.0)) return nullptr;
  }
  if (k > 0 && (!l_colptr || !l_rowidx)) return nullptr;
  auto P = std::make_unique<Problem>();
  P->m = m;
  P->n = n;
  P->k = k;
  P->colptr.assign(h_colptr, h_colptr + n + 1);
  const int nnz = P->colptr[n];
  P->rowidx.assign(h_rowidx, h_rowidx + nnz);
  P->edge_col.resize(nnz);
  P->row_edges.assign(m, {});
  for (int j = 0; j < n; ++j)
    for (int e = P->colptr[j]; e < P->colptr[j + 1]; ++e) {
      P->edge_col[e] = j;
      P->row_edges[P->rowidx[e]].push_back(e);  // ascending column order
    }
  P->lambda64.resize(n);
  P->lambda32.resize(n);
  P->weight.resize(n);
  for (int j = 0; j < n; ++j) {
    double lam = std::log((1.0 - p[j]) / p[j]);  // prior LLR, Appendix A
    P->lambda64[j] = lam;
    P->lambda32[j] = (float)lam;
    P->weight[j] = lam;  // wt(e) = sum_j e_j log((1-p_j)/p_j), Appendix B
  }
  P->l_rows.assign(n, {});
  for (int j = 0; j < n && k > 0; ++j)
    for (int e = l_colptr[j]; e < l_colptr[j + 1]; ++e) {
      if (l_rowidx[e] < 0 || l_rowidx[e] >= k) return nullptr;
      P->l_rows[j].push_back(l_rowidx[e]);
    }
  return reinterpret_cast<oracle_problem>(P.release());
}

void oracle_problem_destroy(oracle_problem pr) { delete reinterpret_cast<Problem*>(pr); }

int oracle_bp_run_f64(oracle_problem pr, const double* e_start, const oracle_pair* pairs,
                      int32_t npairs, const uint8_t* s, int32_t max_iters, double alpha,
                      double llr_max, int32_t stop, double* e_out, double* sum_llr,
                      uint8_t* ehat, double* post_last, int32_t* iters, int32_t* converged) {
  return bp_run_impl<double>(pr, e_start, pairs, npairs, s, max_iters, alpha, llr_max, stop, e_out,
                             sum_llr, ehat, post_last, iters, converged);
}

int oracle_bp_run_f32(oracle_problem pr, const float* e_start, const oracle_pair* pairs,
                      int32_t npairs, const uint8_t* s, int32_t max_iters, float alpha,
                      float llr_max, int32_t stop, float* e_out, float* sum_llr, uint8_t* ehat,
                      float* post_last, int32_t* iters, int32_t* converged) {
  return bp_run_impl<float>(pr, e_start, pairs, npairs, s, max_iters, alpha, llr_max, stop, e_out,
                            sum_llr, ehat, post_last, iters, converged);
}

int oracle_score_f64(oracle_problem pr, const double* sum_llr, const oracle_pair* pairs,
                     int32_t npairs, int32_t iters, int32_t* next_pos, double* score) {
  return score_impl<double>(pr, sum_llr, pairs, npairs, iters, next_pos, score);
}

int oracle_score_f32(oracle_problem pr, const float* sum_llr, const oracle_pair* pairs,
                     int32_t npairs, int32_t iters, int32_t* next_pos, float* score) {
  return score_impl<float>(pr, sum_llr, pairs, npairs, iters, next_pos, score);
}

int oracle_decode_f64(oracle_problem pr, const oracle_params* prm, int64_t shots,
                      const uint8_t* syndromes, uint8_t* corrections, uint8_t* flips,
                      uint8_t* converged, oracle_shot_diag* diag, int32_t threads) {
  return decode_impl<double>(pr, prm, shots, syndromes, corrections, flips, converged, diag,
                             threads);
}

int oracle_decode_f32(oracle_problem pr, const oracle_params* prm, int64_t shots,
                      const uint8_t* syndromes, uint8_t* corrections, uint8_t* flips,
                      uint8_t* converged, oracle_shot_diag* diag, int32_t threads) {
  return decode_impl<float>(pr, prm, shots, syndromes, corrections, flips, converged, diag,
                            threads);
}

}  // extern "C"
