// Host runtime of the beam-search decoder: the C ABI declared in bsd.h.
//
// bsd_code_create renumbers the detector rows by descending degree, lays the
// edge messages out as jagged diagonals (the order they have in LDS and in
// every device slot), forms the prior LLRs in double precision, and uploads
// the graph once.  bsd_decode runs either the persistent batched kernel
// (every shot of the call in one launch, beams advanced on the device) or
// the plain form (one launch per BP run, beam bookkeeping on the host).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bsd.h"
#include "bsd_internal.h"

using namespace bsd;

namespace {

thread_local std::string g_err;

bsd_status fail(bsd_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_OR_FAIL(expr)                                                                     \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(BSD_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));                \
  } while (0)

template <class T>
hipError_t dev_upload(T** dst, const std::vector<T>& v) {
  size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
  hipError_t e = hipMalloc((void**)dst, bytes);
  if (e != hipSuccess) return e;
  if (!v.empty()) e = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

uint32_t pow2_at_least(uint64_t x) {
  uint32_t c = 1;
  while (c < x) c <<= 1;
  return c;
}

}  // namespace

// What batched calls on one stream use: the workspace (queues, contexts,
// slots), the screen's shot list, events, and the HIP graph of the last call
// (BSD_FLAG_GRAPH).  Calls on one stream run in stream order, so they share
// it; calls on different streams have their own and may run concurrently.
// With BSD_FLAG_BESIDE, the decoder beside the screen runs while the screen
// hands on less than this share of a call's shots; below the same share the
// decoder after the screen takes a share of the grid while other streams'
// calls run.
constexpr double kBesideMaxListed = 0.02;
constexpr double kShareMaxListed = 0.02;

struct Lane {
  hipStream_t stream = nullptr;
  std::mutex mu;                   // held while a call enqueues its work
  BatchWs ws;
  int32_t* d_list = nullptr;
  int64_t list_cap = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, evs = nullptr;  // evs: end of the screen
  hipEvent_t done = nullptr;       // recorded after each call's last kernel
  bool pending = false;            // `done` has been recorded
  int64_t last_shots = 0;          // shots of the last call (checked by bsd_code_sync)
  hipStream_t cap_stream = nullptr;
  hipStream_t side = nullptr;      // the dense decoder launched beside the screen
  hipEvent_t ev_side = nullptr;    // end of that launch
  double listed_frac = 0.0;        // share of shots the screen handed on in the last
                                   //   synchronous call (decides the launch beside it)
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<char> gkey;
};

// Tables of iteration 1 for one scaling (see FirstIter): by rank for the
// persistent decoder, by original row for the screen.
struct FiTab {
  float alpha = 0.f;
  uint4* d_rows = nullptr;
  uint32_t* d_negbits = nullptr;
  float* d_e1min = nullptr;    // screen: least zero-syndrome E(1) per row (lowered 1 %)
  float* d_rowxy = nullptr;    // screen: per row (and row m), x and y of eq. (1) at t = 1
  FirstIter fi{};
};

struct bsd_code_s {
  int device = 0;
  DevGraph g{};
  int block = 64, cpt = 1, pw = 1, grid = 1;
  size_t lds = 0;
  std::vector<void*> owned;  // device buffers of the graph
  std::vector<int32_t> colptr, rowidx;
  std::vector<float> lam_host;        // prior LLRs as uploaded
  std::vector<double> lam64_host;     // the same in double precision: wt(e) terms (Appendix B)
  double* d_lam64 = nullptr;
  uint32_t* d_resbits = nullptr;      // plain form: the chosen result's bits
  uint8_t* d_stage = nullptr;         // staging of host buffers passed to bsd_decode
  size_t stage_bytes = 0;
  int32_t *u_colptr = nullptr, *u_rowptr = nullptr, *u_rowedge = nullptr;  // unrolled decoder
  std::vector<float> asched;          // per-iteration scaling (BSD_FLAG_ALPHA_SCHEDULE)
  float* d_asched = nullptr;
  std::vector<uint32_t> cedge_host;   // LDS position | rank << 16, CSC order
  // First-iteration tables, one per scaling used so far.
  std::vector<FiTab*> fi_tabs;
  // Shared by calls that enqueue work; exclusive for changes to what
  // kernels in flight read (tables, schedule, launch geometry).
  std::shared_mutex cfg_mu;
  // Iteration-1 screen: rows in CSR form and per edge in that order its
  // column's rows, column and prior.
  bool all_pos = false;  // every prior LLR > 0 in single precision
  int32_t* s_rowptr = nullptr;
  uint4* s_edgerows = nullptr;
  uint4* s_edgecol = nullptr;
  int screen_per_cu = 1, screen2_per_cu = 1;
  int maxdeg_col = 1;
  // Batched decoding: one lane per stream the handle has been used on.
  std::vector<Lane*> lanes;
  std::mutex lanes_mu;
  std::mutex stage_mu;                // the staging buffer of host-memory calls
  size_t slot_stride = 0;
  // Plain-form and single-run workspace.
  char* pslots = nullptr;
  int p_bw = 0;
  int32_t* d_pairs = nullptr;
  int32_t* d_result = nullptr;
  uint32_t* d_error = nullptr;
  int32_t* h_pinned = nullptr;  // pairs staging [kMaxRounds] + result [4] + error [1]
  std::mutex mu;
  std::atomic<int> busy{0};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // plain form's timing
  int grid_frac_half = 0;  // autotuner: use half the resident workgroups
  int ncu = 1;             // compute units of the device
};

namespace {

void ws_free(BatchWs& w) {
  hipFree(w.st);
  hipHostFree(w.st_host);
  hipFree(w.work_ring);
  hipFree(w.ctx_ring);
  hipFree(w.ctxs);
  hipFree(w.slots);
  hipFree(w.results);
  w = BatchWs{};
}

void drop_graph(Lane* l) {
  if (l->gexec) hipGraphExecDestroy(l->gexec);
  if (l->graph) hipGraphDestroy(l->graph);
  l->gexec = nullptr;
  l->graph = nullptr;
  l->gkey.clear();
}

// How many other streams' batched calls on this handle may still be running
// (their lanes' end events not yet reached).  Skips the check (0) rather
// than wait when another thread holds the lane list.
int other_lanes_busy(bsd_code c, const Lane* self) {
  std::unique_lock<std::mutex> lock(c->lanes_mu, std::try_to_lock);
  if (!lock.owns_lock()) return 0;
  int busy = 0;
  for (const Lane* o : c->lanes)
    if (o != self && o->done && hipEventQuery(o->done) == hipErrorNotReady) ++busy;
  (void)hipGetLastError();  // (a query that is not ready is no error)
  return busy;
}

// Wait until the lane's enqueued work has finished.
void lane_wait(Lane* l) {
  if (l->pending) (void)hipEventSynchronize(l->done);
  l->pending = false;
}

void lane_free(Lane* l) {
  lane_wait(l);
  drop_graph(l);
  if (l->cap_stream) hipStreamDestroy(l->cap_stream);
  if (l->side) hipStreamDestroy(l->side);
  if (l->ev_side) hipEventDestroy(l->ev_side);
  ws_free(l->ws);
  hipFree(l->d_list);
  for (hipEvent_t e : {l->ev0, l->ev1, l->evs, l->done})
    if (e) hipEventDestroy(e);
  delete l;
}

// The lane of `stream`, created on first use (nullptr on failure).
Lane* get_lane(bsd_code c, hipStream_t stream, bool create = true);

// Every lane idle, and no graph kept: before shared tables or the launch
// geometry change under work in flight.
void quiesce(bsd_code c);

// Allocate (or grow) a batched workspace for beam width bw, nctx contexts and
// num_results results per context.
bsd_status ws_ensure(const DevGraph& g, BatchWs& w, int bw, int nctx, int num_results) {
  if (!(w.bw >= bw && w.st && w.nctx >= nctx)) {
    ws_free(w);
    const int per = 3 * bw + 1;
    const size_t slot_total = (size_t)nctx * per * slot_bytes(g);
    w.work_cap = pow2_at_least((uint64_t)nctx * 2 * bw + 1);
    w.ctx_cap = pow2_at_least((uint64_t)nctx + 1);
    if (hipMalloc((void**)&w.st, sizeof(BatchState)) != hipSuccess ||
        hipHostMalloc((void**)&w.st_host, sizeof(BatchState), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&w.work_ring, (size_t)w.work_cap * 4) != hipSuccess ||
        hipMalloc((void**)&w.ctx_ring, (size_t)w.ctx_cap * 4) != hipSuccess ||
        hipMalloc((void**)&w.ctxs, (size_t)nctx * sizeof(Ctx)) != hipSuccess ||
        hipMalloc((void**)&w.slots, slot_total) != hipSuccess) {
      ws_free(w);
      (void)hipGetLastError();
      return fail(BSD_ENOMEM, "cannot allocate the batched workspace (%zu bytes of slots)", slot_total);
    }
    if (hipMemset(w.st, 0, sizeof(BatchState)) != hipSuccess) {  // the latched error starts clear
      ws_free(w);
      (void)hipGetLastError();
      return fail(BSD_EDEVICE, "cannot clear the batched workspace");
    }
    w.nctx = nctx;
    w.bw = bw;
  }
  const size_t need = (size_t)w.nctx * num_results * g.words_n;
  if (num_results > 1 && w.results_words < need) {
    hipFree(w.results);
    w.results = nullptr;
    w.results_words = 0;
    if (hipMalloc((void**)&w.results, need * 4) != hipSuccess) {
      (void)hipGetLastError();
      return fail(BSD_ENOMEM, "cannot allocate %zu bytes for num_results = %d", need * 4, num_results);
    }
    w.results_words = need;
  }
  return BSD_OK;
}

bsd_status ensure_batched(bsd_code c, Lane* l, int bw, int num_results) {
  const BatchWs before = l->ws;
  const bool grow = !(before.bw >= bw && before.st && before.nctx >= c->grid + 64) ||
                    (num_results > 1 &&
                     before.results_words < (size_t)before.nctx * num_results * c->g.words_n);
  if (grow) lane_wait(l);  // the lane's earlier kernels may still use the old buffers
  bsd_status st = ws_ensure(c->g, l->ws, bw, c->grid + 64, num_results);
  if (l->ws.st != before.st || l->ws.results != before.results) drop_graph(l);
  return st;
}

void fitab_free(FiTab* t) {
  hipFree(t->d_rows);
  hipFree(t->d_negbits);
  hipFree(t->d_e1min);
  hipFree(t->d_rowxy);
  delete t;
}

constexpr size_t kMaxLanes = 8;  // streams one handle decodes on

Lane* get_lane(bsd_code c, hipStream_t stream, bool create) {
  std::lock_guard<std::mutex> lock(c->lanes_mu);
  for (Lane* l : c->lanes)
    if (l->stream == stream) return l;
  if (!create || c->lanes.size() >= kMaxLanes) return nullptr;
  Lane* l = new (std::nothrow) Lane;
  if (!l) return nullptr;
  l->stream = stream;
  if (hipEventCreate(&l->ev0) != hipSuccess || hipEventCreate(&l->ev1) != hipSuccess ||
      hipEventCreate(&l->evs) != hipSuccess ||
      hipEventCreateWithFlags(&l->done, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    lane_free(l);
    return nullptr;
  }
  c->lanes.push_back(l);
  return l;
}

void quiesce(bsd_code c) {
  std::lock_guard<std::mutex> lock(c->lanes_mu);
  for (Lane* l : c->lanes) {
    lane_wait(l);
    drop_graph(l);
  }
}

bsd_status ensure_plain(bsd_code c, int bw) {
  if (!c->d_pairs) {
    if (hipMalloc((void**)&c->d_pairs, kMaxRounds * 4) != hipSuccess ||
        hipMalloc((void**)&c->d_result, 16) != hipSuccess ||
        hipMalloc((void**)&c->d_error, 4) != hipSuccess ||
        hipMalloc((void**)&c->d_resbits, (size_t)c->g.words_n * 4) != hipSuccess ||
        hipHostMalloc((void**)&c->h_pinned, (kMaxRounds + 8) * 4, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return fail(BSD_ENOMEM, "cannot allocate the single-run workspace");
    }
  }
  if (bw > 0 && c->p_bw < bw) {
    hipFree(c->pslots);
    c->pslots = nullptr;
    c->slot_stride = slot_bytes(c->g);
    if (hipMalloc((void**)&c->pslots, (size_t)(3 * bw + 1) * c->slot_stride) != hipSuccess) {
      (void)hipGetLastError();
      c->p_bw = 0;
      return fail(BSD_ENOMEM, "cannot allocate plain-form slots");
    }
    c->p_bw = bw;
  }
  return BSD_OK;
}

bsd_status check_params(const bsd_code c, const bsd_params* p) {
  if (!p) return fail(BSD_EINVAL, "params is NULL");
  if (p->max_rounds < 0 || p->max_rounds > kMaxRounds)
    return fail(BSD_EINVAL, "max_rounds must be in [0, %d]", kMaxRounds);
  if (p->beam_width < 1 || p->beam_width > kMaxBw)
    return fail(BSD_EINVAL, "beam_width must be in [1, %d]", kMaxBw);
  if (p->initial_iters < 0 || p->iters_per_round < 0)
    return fail(BSD_EINVAL, "iteration counts must be >= 0");
  if (p->num_results < 1 || p->num_results > kMaxResults)
    return fail(BSD_EINVAL, "num_results must be in [1, %d]", kMaxResults);
  if (!(p->alpha > 0.f) || !std::isfinite(p->alpha))
    return fail(BSD_EINVAL, "alpha must be positive and finite");
  if (p->mode != BSD_MODE_BATCHED && p->mode != BSD_MODE_PLAIN)
    return fail(BSD_EINVAL, "unknown mode %d", p->mode);
  if ((p->flags & BSD_FLAG_ALPHA_SCHEDULE) && c->asched.empty())
    return fail(BSD_EINVAL, "BSD_FLAG_ALPHA_SCHEDULE without a schedule (bsd_code_set_alpha_schedule)");
  return BSD_OK;
}

struct RunOut {
  int iters, conv, next_pos;
  float score;
};

// One BP run of the plain form: pairs up, launch, result down (synchronous).
bsd_status plain_run(bsd_code c, hipStream_t s, const float* parent, const std::vector<int32_t>& pairs,
                     const uint8_t* syn, int T, float alpha, float* out_msg, uint32_t* out_bits,
                     RunOut* r, bool keep_msg = false, bool sched = false) {
  SingleArgs a{};
  a.g = c->g;
  if (sched) {
    a.alpha_sched = c->d_asched;
    a.n_sched = (int32_t)c->asched.size();
  }
  a.parent = parent;
  a.npairs = (int)pairs.size();
  if (!pairs.empty()) {
    std::memcpy(c->h_pinned, pairs.data(), pairs.size() * 4);
    HIP_OR_FAIL(hipMemcpyAsync(c->d_pairs, c->h_pinned, pairs.size() * 4, hipMemcpyHostToDevice, s));
  }
  a.pairs = c->d_pairs;
  a.syn = syn;
  a.max_iters = T;
  a.stop = 1;
  a.alpha = alpha;
  a.want_score = 1;
  a.out_msg = out_msg;
  a.keep_msg = keep_msg ? 1 : 0;
  a.out_ehat_bits = out_bits;
  a.result = c->d_result;
  a.error = c->d_error;
  HIP_OR_FAIL(launch_single(a, c->block, c->cpt, c->pw, c->lds, s));
  int32_t* res = c->h_pinned + kMaxRounds;
  HIP_OR_FAIL(hipMemcpyAsync(res, c->d_result, 16, hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(hipStreamSynchronize(s));
  r->iters = res[0];
  r->conv = res[1];
  r->next_pos = res[2];
  std::memcpy(&r->score, &res[3], 4);
  return BSD_OK;
}

struct HostPath {
  int slot;
  std::vector<int32_t> pairs;
  int next_pos;
  float score;
  int gen;
};

bsd_status decode_plain(bsd_code c, const bsd_params* p, int64_t shots, const uint8_t* syn,
                        uint8_t* corr, uint8_t* flips, uint8_t* conv, hipStream_t s,
                        bsd_stats* stats, uint32_t* lat) {
  const DevGraph& g = c->g;
  bsd_status st = ensure_plain(c, p->beam_width);
  if (st != BSD_OK) return st;
  HIP_OR_FAIL(hipMemsetAsync(c->d_error, 0, 4, s));
  const int bw = p->beam_width;
  const int want = p->num_results;
  const bool many = want > 1;  // converged runs keep their messages and keep branching
  const bool sched = (p->flags & BSD_FLAG_ALPHA_SCHEDULE) != 0;
  auto slot = [&](int i) { return c->pslots + (size_t)i * c->slot_stride; };
  auto msg_of = [&](int i) { return (float*)slot(i); };
  auto bits_of = [&](int i) { return (uint32_t*)(slot(i) + slot_ehat_off(g)); };
  const int keeper = 3 * bw;
  int64_t runs = 0, iters = 0, deep = 0;
  std::vector<std::vector<uint32_t>> res;  // num_results > 1: distinct solutions, in the order found
  std::vector<double> res_wt;
  std::vector<uint32_t> hb((size_t)g.words_n);
  // Adds the solution in `slot` unless already found; true once `want` are found.
  auto add_result = [&](int sl, bool* full) -> bsd_status {
    HIP_OR_FAIL(hipMemcpyAsync(hb.data(), bits_of(sl), hb.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    *full = false;
    for (const auto& r : res)
      if (r == hb) return BSD_OK;
    double w = 0.0;
    for (int j = 0; j < g.n; ++j)
      if ((hb[j >> 5] >> (j & 31)) & 1u) w += c->lam64_host[j];
    res.push_back(hb);
    res_wt.push_back(w);
    *full = (int)res.size() >= want;
    return BSD_OK;
  };
  // Per-shot host time (10 ns units, the unit of the batched form's device clock).
  std::vector<uint32_t> lat_h(lat ? (size_t)shots : 0);
  HIP_OR_FAIL(hipEventRecord(c->ev0, s));
  for (int64_t q = 0; q < shots; ++q) {
    const auto t_shot = std::chrono::steady_clock::now();
    const uint8_t* sq = syn + q * g.m;
    EmitArgs e{};
    e.g = g;
    e.corr = corr + q * g.n;
    e.flips = flips + q * g.k;
    e.conv = conv + q;
    res.clear();
    res_wt.clear();
    RunOut r0;
    st = plain_run(c, s, nullptr, {}, sq, p->initial_iters, p->alpha, msg_of(0), bits_of(keeper), &r0,
                   many, sched);
    if (st != BSD_OK) return st;
    ++runs;
    iters += r0.iters;
    int emit_slot = keeper, emit_conv = r0.conv;
    bool emit_lightest = false;
    if ((!r0.conv || many) && p->max_rounds > 0) {
      ++deep;
      bool done = false;
      if (r0.conv) {
        st = add_result(keeper, &done);
        if (st != BSD_OK) return st;
      }
      std::vector<HostPath> set{{0, {}, r0.next_pos, 0.f, 0}};
      std::vector<int> free_slots;
      for (int i = 3 * bw - 1; i >= 1; --i) free_slots.push_back(i);
      for (int rd = 1; rd <= p->max_rounds && !done; ++rd) {
        std::stable_sort(set.begin(), set.end(), [](const HostPath& a, const HostPath& b) {
          if (a.score != b.score) return a.score > b.score;
          return a.gen < b.gen;
        });
        std::vector<HostPath> kids;
        for (size_t k = 0; k < set.size() && !done; ++k) {
          if (set[k].next_pos < 0) continue;
          for (int v = 0; v <= 1 && !done; ++v) {
            HostPath ch;
            ch.pairs = set[k].pairs;
            ch.pairs.push_back((set[k].next_pos << 1) | v);
            ch.gen = (int)(2 * k + v);
            ch.slot = free_slots.back();
            free_slots.pop_back();
            RunOut rr;
            st = plain_run(c, s, msg_of(set[k].slot), ch.pairs, sq, p->iters_per_round, p->alpha,
                           msg_of(ch.slot), bits_of(ch.slot), &rr, many, sched);
            if (st != BSD_OK) return st;
            ++runs;
            iters += rr.iters;
            if (rr.conv && !many) {
              emit_slot = ch.slot;
              emit_conv = 1;
              done = true;
              break;
            }
            if (rr.conv) {
              bool full = false;
              st = add_result(ch.slot, &full);
              if (st != BSD_OK) return st;
              if (full) {
                emit_lightest = true;
                done = true;
                break;
              }
            }
            ch.next_pos = rr.next_pos;
            ch.score = rr.score;
            kids.push_back(ch);
          }
        }
        if (done) break;
        std::stable_sort(kids.begin(), kids.end(), [](const HostPath& a, const HostPath& b) {
          if (a.score != b.score) return a.score > b.score;
          return a.gen < b.gen;
        });
        for (const HostPath& par : set) free_slots.push_back(par.slot);
        for (size_t k = (size_t)bw; k < kids.size(); ++k) free_slots.push_back(kids[k].slot);
        if (kids.size() > (size_t)bw) kids.resize(bw);
        set = std::move(kids);
        bool last = rd == p->max_rounds;
        if (!last) {
          bool any = false;
          for (const HostPath& h : set) any |= h.next_pos >= 0;
          if (!any) {  // nothing can branch: the search ends with the initial decision
            emit_slot = keeper;
            emit_conv = 0;
            last = true;
          }
        } else {
          emit_slot = set.empty() ? keeper : set[0].slot;
          emit_conv = 0;
        }
        if (last) {
          emit_lightest = !res.empty();
          break;
        }
      }
    }
    if (emit_lightest) {
      size_t best = 0;
      for (size_t r = 1; r < res.size(); ++r)
        if (res_wt[r] < res_wt[best]) best = r;
      HIP_OR_FAIL(hipMemcpyAsync(c->d_resbits, res[best].data(), res[best].size() * 4,
                                 hipMemcpyHostToDevice, s));
      e.ehat_bits = c->d_resbits;
      e.converged = 1;
    } else {
      e.ehat_bits = bits_of(emit_slot);
      e.converged = emit_conv;
    }
    HIP_OR_FAIL(launch_emit(e, s));
    if (emit_lightest || lat) HIP_OR_FAIL(hipStreamSynchronize(s));  // res[best] is pageable
    if (lat)
      lat_h[q] = (uint32_t)std::min<double>(
          4e9, std::chrono::duration<double, std::nano>(std::chrono::steady_clock::now() - t_shot)
                       .count() / 10.0);
  }
  if (lat && shots > 0)
    HIP_OR_FAIL(hipMemcpyAsync(lat, lat_h.data(), lat_h.size() * 4, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(hipEventRecord(c->ev1, s));
  uint32_t err = 0;
  HIP_OR_FAIL(hipMemcpyAsync(c->h_pinned + kMaxRounds + 4, c->d_error, 4, hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(hipStreamSynchronize(s));
  std::memcpy(&err, c->h_pinned + kMaxRounds + 4, 4);
  if (err) return fail(BSD_EINVAL, "syndrome bytes must be 0 or 1");
  if (stats) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, c->ev0, c->ev1);
    stats->runs = runs;
    stats->iterations = iters;
    stats->edge_updates = iters * (int64_t)g.nnz;
    stats->deep_shots = deep;
    stats->kernel_ms = ms;
  }
  return BSD_OK;
}

// Check phase of iteration 1 from the priors for a zero syndrome (eq. (1)
// with E(0) = Lambda), per detector row, in the kernels' single-precision
// operations: least and second least magnitude of the row, alpha times each,
// clamped to the message bound; the diagonal index of the least (the first
// in column order: on a tie both values are equal) and its column; the
// parity of the row's negative priors.  Built once per alpha, under the
// exclusive configuration lock, and kept until the handle is destroyed, so
// that kernels in flight never see a table change.
bsd_status build_first(bsd_code c, float alpha, const FiTab** out) {
  for (const FiTab* t : c->fi_tabs)
    if (t->alpha == alpha) {
      *out = t;
      return BSD_OK;
    }
  const DevGraph& g = c->g;
  const int n = g.n, m = g.m, nnz = g.nnz;
  const std::vector<int32_t>& cp = c->colptr;
  const std::vector<int32_t>& ri = c->rowidx;
  const std::vector<float>& lam = c->lam_host;
  std::vector<int> ecol(nnz);
  for (int j = 0; j < n; ++j)
    for (int e = cp[j]; e < cp[j + 1]; ++e) ecol[e] = j;
  std::vector<std::vector<int>> rows(m);
  for (int e = 0; e < nnz; ++e) rows[ri[e]].push_back(e);  // ascending column = diagonal order
  std::vector<uint4> rt((size_t)m), rtab((size_t)m, make_uint4(0u, 0u, 0xFFFFFFFFu, 0u));
  std::vector<float> t_e1min, t_rowxy((size_t)2 * (m + 1), 0.f);
  std::vector<uint32_t> neg((size_t)g.nnz_pad / 32 + 1, 0u);
  for (int i = 0; i < m; ++i) {
    float m1 = kLlrMax, m2 = kLlrMax;
    bool par = false, anyneg = false;
    int argk = 0, kk = 0;
    for (int e : rows[i]) {
      const float v = lam[ecol[e]], a = std::fabs(v);
      par ^= std::signbit(v);
      anyneg |= std::signbit(v);
      if (std::signbit(v)) {
        const uint32_t pos = c->cedge_host[e] & 0xFFFFu;
        neg[pos >> 5] |= 1u << (pos & 31);
      }
      if (a < m1) argk = kk;
      m2 = std::max(m1, std::min(m2, a));
      m1 = std::min(m1, a);
      ++kk;
    }
    const float x = std::fmin(alpha * m1, kLlrMax), y = std::fmin(alpha * m2, kLlrMax);
    const uint32_t rank = rows[i].empty() ? 0u : (c->cedge_host[rows[i][0]] >> 16);
    if (rows[i].empty()) continue;
    uint32_t xb, yb;
    std::memcpy(&xb, &x, 4);
    std::memcpy(&yb, &y, 4);
    rt[rank] = make_uint4(xb, yb, (uint32_t)argk | ((uint32_t)par << 8) | ((uint32_t)anyneg << 9), 0u);
    rtab[i] = make_uint4(xb, yb, (uint32_t)ecol[rows[i][argk]], 0u);
    t_rowxy[2 * (size_t)i] = x;
    t_rowxy[2 * (size_t)i + 1] = y;
  }
  // Per row, the least E(1) it receives for s = 0 (eq. (2) at t = 1 from the
  // table's x and y, in the variable phase's single-precision order): the
  // screen's iteration 2 bounds messages from below with it.  Every prior
  // LLR is positive wherever the screen runs, so these are positive too.
  {
    std::vector<float> e1min((size_t)m, kLlrMax);
    float d[kMaxDv];
    for (int j = 0; j < n; ++j) {
      const int dg = cp[j + 1] - cp[j];
      for (int e = 0; e < dg; ++e) {
        const uint4& t = rtab[ri[cp[j] + e]];
        std::memcpy(&d[e], (int)t.z == j ? &t.y : &t.x, 4);
      }
      float pre = lam[j];
      for (int e = 0; e < dg; ++e) {
        float x = pre;
        for (int f = e + 1; f < dg; ++f) x = x + d[f];
        x = std::fmin(std::fmax(x, -kLlrMax), kLlrMax);
        float& mn = e1min[ri[cp[j] + e]];
        mn = std::fmin(mn, x);
        pre = pre + d[e];
      }
    }
    // (kept 1 % low: a bound stays valid under any difference in the last
    // bits between this host arithmetic and the device's)
    for (int i = 0; i < m; ++i) e1min[i] = 0.99f * e1min[i];
    t_e1min.swap(e1min);
  }
  FiTab* t = new (std::nothrow) FiTab;
  if (!t) return fail(BSD_ENOMEM, "host allocation failed");
  t->alpha = alpha;
  if (dev_upload(&t->d_rows, rt) != hipSuccess || dev_upload(&t->d_e1min, t_e1min) != hipSuccess ||
      dev_upload(&t->d_rowxy, t_rowxy) != hipSuccess ||
      dev_upload(&t->d_negbits, neg) != hipSuccess) {
    (void)hipGetLastError();
    fitab_free(t);
    return fail(BSD_ENOMEM, "cannot allocate the first-iteration table");
  }
  t->fi.rows = t->d_rows;
  t->fi.negbits = t->d_negbits;
  t->fi.enabled = 1;
  c->fi_tabs.push_back(t);
  *out = t;
  return BSD_OK;
}

bool needs_first(const bsd_params* p) {
  return !(p->flags & BSD_FLAG_DENSE_FIRST) && p->initial_iters >= 1;
}

// Iteration 1's scaling (configuration lock held).
float first_alpha(const bsd_code c, const bsd_params* p) {
  return (p->flags & BSD_FLAG_ALPHA_SCHEDULE) && !c->asched.empty() ? c->asched[0] : p->alpha;
}

// The table a call needs, or nullptr (configuration lock held, shared or exclusive).
const FiTab* find_first(const bsd_code c, const bsd_params* p) {
  if (!needs_first(p)) return nullptr;
  const float a1 = first_alpha(c, p);
  for (const FiTab* t : c->fi_tabs)
    if (t->alpha == a1) return t;
  return nullptr;
}

// Runs fn(table) with the configuration lock shared and the iteration-1
// table the call needs (built first, under the exclusive lock, if missing).
template <class F>
bsd_status with_tables(bsd_code c, const bsd_params* p, F fn) {
  for (int attempt = 0; attempt < 2; ++attempt) {
    {
      std::shared_lock<std::shared_mutex> cfg(c->cfg_mu);
      const FiTab* ft = find_first(c, p);
      if (ft || !needs_first(p)) return fn(ft);
    }
    std::unique_lock<std::shared_mutex> cfg(c->cfg_mu);
    const FiTab* t = nullptr;
    bsd_status st = build_first(c, first_alpha(c, p), &t);
    if (st != BSD_OK) return st;
  }
  return fail(BSD_EBUSY, "the scaling schedule changed during the call");
}

// Kernel arguments common to every batched launch on workspace w.
BatchArgs batch_args(bsd_code c, const BatchWs& w, const bsd_params* p, const FiTab* ft) {
  BatchArgs a{};
  a.g = c->g;
  if (ft) a.fi = ft->fi;
  if (p->flags & BSD_FLAG_ALPHA_SCHEDULE) {
    a.alpha_sched = c->d_asched;
    a.n_sched = (int32_t)c->asched.size();
  }
  a.max_rounds = p->max_rounds;
  a.bw = p->beam_width;
  a.init_iters = p->initial_iters;
  a.round_iters = p->iters_per_round;
  a.num_results = p->num_results;
  a.alpha = p->alpha;
  a.lam64 = c->d_lam64;
  a.results = w.results;
  a.st = w.st;
  a.work_ring = w.work_ring;
  a.work_cap = w.work_cap;
  a.ctx_ring = w.ctx_ring;
  a.ctx_cap = w.ctx_cap;
  a.ctxs = w.ctxs;
  a.nctx = w.nctx;
  a.slots = w.slots;
  a.slot_stride = slot_bytes(c->g);
  a.slots_per_ctx = 3 * w.bw + 1;
  return a;
}

// Whether a batched call starts with the sparse screen of iteration 1: the
// initial run from the priors has an iteration 1 whose check phase comes
// from the table (every prior LLR positive), and a shot that converges there
// is finished (one result wanted).
bool use_screen(const bsd_code c, const bsd_params* p, const BatchArgs& a) {
  return !(p->flags & (BSD_FLAG_DENSE_FIRST | BSD_FLAG_NO_SCREEN)) && p->initial_iters >= 1 &&
         p->num_results == 1 && c->all_pos && a.fi.enabled;
}

ScreenArgs screen_args(const bsd_code c, const bsd_params* p, const BatchArgs& a, const FiTab* ft) {
  const DevGraph& g = c->g;
  ScreenArgs sa{};
  // Iteration 2 as well when the initial run has one; its scaling is the
  // schedule's second entry (the last, if shorter) or alpha.
  sa.t2 = (p->initial_iters >= 2 && !(p->flags & BSD_FLAG_NO_SCREEN2)) ? 1 : 0;
  sa.single1 = first_alpha(c, p) <= 1.0f ? 1 : 0;
  sa.alpha2 = (a.alpha_sched && !c->asched.empty())
                  ? c->asched[std::min<size_t>(2, c->asched.size()) - 1]
                  : a.alpha;
  sa.m = g.m;
  sa.n = g.n;
  sa.k = g.k;
  sa.words_m = (g.m + 31) / 32;
  const uintptr_t cp = (uintptr_t)a.corr;
  sa.vec = (g.n % 16 == 0 && cp % 16 == 0) ? 16 : (g.n % 4 == 0 && cp % 4 == 0) ? 4 : 1;
  sa.syn8 = (g.m % 8 == 0 && (uintptr_t)a.syn % 8 == 0) ? 1 : 0;
  sa.maxdeg_col = c->maxdeg_col;
  sa.row_ptr = c->s_rowptr;
  sa.edge_rows = c->s_edgerows;
  sa.edge_col = c->s_edgecol;
  sa.row_xy = ft ? reinterpret_cast<const float2*>(ft->d_rowxy) : nullptr;
  sa.row_e1min = ft ? ft->d_e1min : nullptr;
  sa.shots = a.shots;
  sa.syn = a.syn;
  sa.corr = a.corr;
  sa.flips = a.flips;
  sa.conv = a.conv;
  sa.lat = a.lat;
  sa.st = a.st;
  sa.list = const_cast<int32_t*>(a.shot_list);
  return sa;
}

// Screen grids: the workgroups of each kernel that fit on the device at
// once (each holds the row tables in LDS), fewer for small batches; each
// wave takes shots until none are left.
int screen_grid(const bsd_code c, int64_t shots, int which) {
  const int waves = (which == 1 ? kScreenBlock : kScreen2Block) / 64;
  const int64_t want = (shots + waves - 1) / waves;
  const int per_cu = which == 1 ? c->screen_per_cu : c->screen2_per_cu;
  return (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)per_cu * c->ncu));
}

// One batched call on lane l (its mutex and the configuration lock held).
// With `async` it returns once the work is enqueued on the lane's stream.
bsd_status decode_batched(bsd_code c, Lane* l, const bsd_params* p, const FiTab* ft,
                          int64_t shots, const uint8_t* syn, uint8_t* corr, uint8_t* flips,
                          uint8_t* conv, bool async, bsd_stats* stats, uint32_t* lat) {
  const hipStream_t s = l->stream;
  bsd_status st = ensure_batched(c, l, p->beam_width, p->num_results);
  if (st != BSD_OK) return st;
  BatchArgs a = batch_args(c, l->ws, p, ft);
  a.shots = shots;
  a.syn = syn;
  a.corr = corr;
  a.flips = flips;
  a.conv = conv;
  a.lat = lat;
  const bool screen = use_screen(c, p, a);
  if (screen) {
    if (l->list_cap < shots) {
      lane_wait(l);
      hipFree(l->d_list);
      l->d_list = nullptr;
      l->list_cap = 0;
      // the shots the screen hands to the dense decoder
      if (hipMalloc((void**)&l->d_list, (size_t)shots * 4) != hipSuccess) {
        (void)hipGetLastError();
        return fail(BSD_ENOMEM, "cannot allocate the screen's shot list (%lld shots)", (long long)shots);
      }
      l->list_cap = shots;
      drop_graph(l);
    }
    a.shot_list = l->d_list;
  }
  const ScreenArgs sa = screen_args(c, p, a, ft);
  const int sgrid = screen_grid(c, shots, 1);
  const int sgrid2 = screen_grid(c, shots, 2);
  if (screen) {  // (the screen's progress, for the dense decoder beside it)
    a.screen_grid = sa.t2 ? sgrid2 : sgrid;
    a.screen_waves = a.screen_grid * ((sa.t2 ? kScreen2Block : kScreenBlock) / 64);
  }
  if (p->flags & BSD_FLAG_GRAPH) {
    // Replay the recorded reset + decode kernels when the arguments repeat.
    std::vector<char> key(sizeof a + 3 * sizeof(int));
    std::memcpy(key.data(), &a, sizeof a);
    const int geo[3] = {c->grid, c->block, c->cpt};
    std::memcpy(key.data() + sizeof a, geo, sizeof geo);
    if (!l->gexec || key != l->gkey) {
      drop_graph(l);
      if (!l->cap_stream) HIP_OR_FAIL(hipStreamCreateWithFlags(&l->cap_stream, hipStreamNonBlocking));
      HIP_OR_FAIL(hipStreamBeginCapture(l->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t e1 = launch_batch_reset(a, l->cap_stream);
      if (e1 == hipSuccess && screen) e1 = launch_screen(sa, sgrid, sgrid2, l->cap_stream);
      hipError_t e2 = launch_batched(a, c->grid, c->block, c->cpt, c->pw, c->lds, l->cap_stream);
      hipGraph_t gr = nullptr;
      hipError_t e3 = hipStreamEndCapture(l->cap_stream, &gr);
      if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        if (gr) hipGraphDestroy(gr);
        return fail(BSD_EDEVICE, "graph capture failed: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2 != hipSuccess ? e2 : e3));
      }
      l->graph = gr;
      HIP_OR_FAIL(hipGraphInstantiate(&l->gexec, l->graph, nullptr, nullptr, 0));
      l->gkey = key;
    }
    HIP_OR_FAIL(hipEventRecord(l->ev0, s));
    HIP_OR_FAIL(hipGraphLaunch(l->gexec, s));
    HIP_OR_FAIL(hipEventRecord(l->ev1, s));
  } else {
    HIP_OR_FAIL(launch_batch_reset(a, s));
    HIP_OR_FAIL(hipEventRecord(l->ev0, s));
    if (screen) HIP_OR_FAIL(launch_screen(sa, sgrid, sgrid2, s));
    // On request, a dense decoder beside the screen, on a second stream: its
    // workgroups start as the screen's leave the device and take the listed
    // shots while the screen still runs.  The launch after the screen takes
    // whatever it leaves (and ends at once when it left nothing).  Only
    // when the screen hands on few shots (the dense work then hides under
    // the screen's last waves); with more, running beside the screen slows
    // both, so the share of the lane's last synchronous call decides.
    const bool beside =
        screen && (p->flags & BSD_FLAG_BESIDE) && l->listed_frac < kBesideMaxListed;
    if (beside) {
      if (!l->side) {
        HIP_OR_FAIL(hipStreamCreateWithFlags(&l->side, hipStreamNonBlocking));
        HIP_OR_FAIL(hipEventCreateWithFlags(&l->ev_side, hipEventDisableTiming));
      }
      BatchArgs h = a;
      h.helper = 1;
      HIP_OR_FAIL(hipStreamWaitEvent(l->side, l->ev0, 0));
      HIP_OR_FAIL(launch_batched(h, c->grid, c->block, c->cpt, c->pw, c->lds, l->side));
      HIP_OR_FAIL(hipEventRecord(l->ev_side, l->side));
    }
    HIP_OR_FAIL(hipEventRecord(l->evs, s));
    // While other streams' calls run (calls pipelined on several streams)
    // and the screen hands on few shots, the decoder after the screen takes
    // an equal share of the grid: each workgroup holds a whole compute unit,
    // mostly waiting on its few shots' iterations, and the other streams'
    // screens get the rest.  On one stream the whole grid finishes those
    // shots sooner.
    const int others = screen && !beside && l->listed_frac < kShareMaxListed
                           ? other_lanes_busy(c, l) : 0;
    const int dgrid = std::max(1, c->grid / (1 + others));
    HIP_OR_FAIL(launch_batched(a, dgrid, c->block, c->cpt, c->pw, c->lds, s));
    if (beside) HIP_OR_FAIL(hipStreamWaitEvent(s, l->ev_side, 0));
    HIP_OR_FAIL(hipEventRecord(l->ev1, s));
  }
  HIP_OR_FAIL(hipEventRecord(l->done, s));
  l->pending = true;
  l->last_shots = shots;
  if (async) return BSD_OK;
  HIP_OR_FAIL(hipMemcpyAsync(l->ws.st_host, l->ws.st, sizeof(BatchState), hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(hipStreamSynchronize(s));
  l->pending = false;
  BatchState& h = *l->ws.st_host;
  if (h.error) {  // reported here, so not again by bsd_code_sync
    h.error = 0;
    HIP_OR_FAIL(hipMemcpyAsync(l->ws.st, l->ws.st_host, sizeof(BatchState), hipMemcpyHostToDevice, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    return fail(BSD_EINVAL, "syndrome bytes must be 0 or 1");
  }
  if (h.done != (unsigned long long)shots)
    return fail(BSD_EDEVICE, "batched decoder finished %llu of %lld shots", h.done, (long long)shots);
  if (screen) l->listed_frac = (double)h.listed / (double)shots;
  if (stats) {
    float ms = 0.f, sms = 0.f;
    (void)hipEventElapsedTime(&ms, l->ev0, l->ev1);
    stats->runs = (int64_t)h.runs;
    stats->iterations = (int64_t)h.iterations;
    stats->edge_updates = (int64_t)h.iterations * c->g.nnz;
    stats->deep_shots = (int64_t)h.deep;
    stats->kernel_ms = ms;
    if (screen) {
      // (a graph replay is timed as a whole: screen_ms stays 0)
      if (!(p->flags & BSD_FLAG_GRAPH)) (void)hipEventElapsedTime(&sms, l->ev0, l->evs);
      stats->screened_shots = shots - (int64_t)h.listed;
      stats->screened2_shots = (int64_t)h.done2;
      stats->screen_ms = sms;
    }
  }
  return BSD_OK;
}

// Workgroup size `block` and resident workgroups (all that fit, or half).
bsd_status set_geometry(bsd_code c, int block, int half) {
  const DevGraph& g = c->g;
  const int cpt = supported_cpt((g.n + block - 1) / block);
  if (block < 64 || block > 1024 || cpt < 0 || g.m > 2 * block || block > max_block_for_cpt(cpt))
    return fail(BSD_EINVAL, "no kernel for %d threads with n = %d, m = %d", block, g.n, g.m);
  hipError_t he = set_kernel_limits(cpt, c->pw, c->lds);
  if (he != hipSuccess) return fail(BSD_EDEVICE, "hipFuncSetAttribute: %s", hipGetErrorString(he));
  int per_cu = 0, ncu = 0;
  he = batched_occupancy(cpt, c->pw, block, c->lds, &per_cu);
  if (he == hipSuccess) he = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
  if (he != hipSuccess || per_cu < 1)
    return fail(BSD_EDEVICE, "occupancy query failed: %s (blocks per CU %d)", hipGetErrorString(he), per_cu);
  const int grid = half && per_cu > 1 ? (per_cu / 2) * ncu : per_cu * ncu;
  if (grid != c->grid || block != c->block) quiesce(c);
  c->ncu = ncu;
  c->block = block;
  c->cpt = cpt;
  c->grid = grid;
  c->grid_frac_half = half && per_cu > 1;
  return BSD_OK;
}

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

}  // namespace

extern "C" {

const char* bsd_last_error(void) { return g_err.c_str(); }

const char* bsd_version(void) { return "bsd-mi355x 0.1 (gfx950)"; }

bsd_status bsd_code_create(int32_t m, int32_t n, int32_t k, const int32_t* h_colptr,
                           const int32_t* h_rowidx, const double* p, const int32_t* l_colptr,
                           const int32_t* l_rowidx, bsd_code* out) {
  if (!out) return fail(BSD_EINVAL, "out is NULL");
  *out = nullptr;
  if (m <= 0 || n <= 0 || k < 0) return fail(BSD_EINVAL, "m, n must be > 0 and k >= 0");
  if (m > 2048) return fail(BSD_EINVAL, "m must be <= 2048");
  if (k > 64) return fail(BSD_EINVAL, "k must be <= 64");
  if (!h_colptr || !h_rowidx || !p) return fail(BSD_EINVAL, "H and p are required");
  if (k > 0 && (!l_colptr || !l_rowidx)) return fail(BSD_EINVAL, "A is required when k > 0");
  if (h_colptr[0] != 0) return fail(BSD_EINVAL, "h_colptr[0] must be 0");
  for (int j = 0; j < n; ++j) {
    const int d = h_colptr[j + 1] - h_colptr[j];
    if (d < 0) return fail(BSD_EINVAL, "h_colptr is not non-decreasing at column %d", j);
    if (d > kMaxDv) return fail(BSD_EINVAL, "column %d has degree %d > %d", j, d, kMaxDv);
    for (int e = h_colptr[j]; e < h_colptr[j + 1]; ++e) {
      if (h_rowidx[e] < 0 || h_rowidx[e] >= m)
        return fail(BSD_EINVAL, "row index out of range in column %d", j);
      if (e > h_colptr[j] && h_rowidx[e] <= h_rowidx[e - 1])
        return fail(BSD_EINVAL, "rows of column %d are not strictly ascending", j);
    }
    if (!(p[j] > 0.0 && p[j] < 1.0)) return fail(BSD_EINVAL, "p[%d] is not in (0,1)", j);
  }
  const int nnz = h_colptr[n];
  if (nnz <= 0) return fail(BSD_EINVAL, "H has no edges");
  if (k > 0) {
    if (l_colptr[0] != 0) return fail(BSD_EINVAL, "l_colptr[0] must be 0");
    for (int j = 0; j < n; ++j) {
      if (l_colptr[j + 1] < l_colptr[j]) return fail(BSD_EINVAL, "l_colptr decreasing at %d", j);
      for (int e = l_colptr[j]; e < l_colptr[j + 1]; ++e)
        if (l_rowidx[e] < 0 || l_rowidx[e] >= k)
          return fail(BSD_EINVAL, "logical row index out of range in column %d", j);
    }
  }
  // Rows by descending degree (ties: ascending row), jagged diagonals.
  std::vector<int> rdeg(m, 0);
  for (int e = 0; e < nnz; ++e) rdeg[h_rowidx[e]]++;
  std::vector<int> order(m);
  for (int i = 0; i < m; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return rdeg[a] > rdeg[b]; });
  const int maxdeg = rdeg[order[0]];
  if (maxdeg > kMaxDc) return fail(BSD_EINVAL, "a row has degree %d > %d", maxdeg, kMaxDc);
  std::vector<int> rank_of_row(m);
  std::vector<uint16_t> row_of_rank(m);
  std::vector<uint8_t> deg_of_rank(m);
  for (int r = 0; r < m; ++r) {
    rank_of_row[order[r]] = r;
    row_of_rank[r] = (uint16_t)order[r];
    deg_of_rank[r] = (uint8_t)rdeg[order[r]];
  }
  std::vector<int32_t> diag_ptr(maxdeg + 1, 0);
  for (int kk = 0; kk < maxdeg; ++kk) {
    int cnt = 0;
    while (cnt < m && rdeg[order[cnt]] > kk) ++cnt;
    diag_ptr[kk + 1] = diag_ptr[kk] + cnt;
  }
  if (diag_ptr[maxdeg] != nnz) return fail(BSD_EINVAL, "internal: diagonal layout mismatch");
  std::vector<int> seen(m, 0);
  std::vector<uint32_t> cedge(nnz), colinfo(n);
  for (int j = 0; j < n; ++j) {
    colinfo[j] = (uint32_t)h_colptr[j] | ((uint32_t)(h_colptr[j + 1] - h_colptr[j]) << 24);
    for (int e = h_colptr[j]; e < h_colptr[j + 1]; ++e) {
      const int i = h_rowidx[e];
      const int pos = diag_ptr[seen[i]++] + rank_of_row[i];
      cedge[e] = (uint32_t)pos | ((uint32_t)rank_of_row[i] << 16);
    }
  }
  std::vector<uint16_t> crank((size_t)n * 8, 0xFFFFu);  // 0xFFFF: no edge
  for (int j = 0; j < n; ++j)
    for (int e = h_colptr[j]; e < h_colptr[j + 1]; ++e)
      crank[(size_t)j * 8 + (e - h_colptr[j])] = (uint16_t)(cedge[e] >> 16);
  std::vector<float> lam(n);
  std::vector<double> lam64(n);
  for (int j = 0; j < n; ++j) lam64[j] = std::log((1.0 - p[j]) / p[j]);
  for (int j = 0; j < n; ++j) lam[j] = (float)lam64[j];
  std::vector<uint64_t> lmask(n, 0);
  for (int j = 0; j < n && k > 0; ++j)
    for (int e = l_colptr[j]; e < l_colptr[j + 1]; ++e) lmask[j] ^= 1ull << l_rowidx[e];

  bsd_code c = new (std::nothrow) bsd_code_s;
  if (!c) return fail(BSD_ENOMEM, "host allocation failed");
  HIP_OR_FAIL(hipGetDevice(&c->device));
  DevGraph& g = c->g;
  g.m = m;
  g.n = n;
  g.nnz = nnz;
  g.k = k;
  g.nnz_pad = (nnz + 3) & ~3;
  g.words_m = (((m + 31) / 32) + 1) & ~1;
  g.words_n = (((n + 31) / 32) + 1) & ~1;
  g.maxdeg_row = maxdeg;
  c->colptr.assign(h_colptr, h_colptr + n + 1);
  c->rowidx.assign(h_rowidx, h_rowidx + nnz);
  c->lam_host = lam;
  c->lam64_host = lam64;
  c->cedge_host = cedge;
  int32_t* d_diag;
  uint16_t* d_ror;
  uint8_t* d_dor;
  uint32_t *d_ci, *d_ce;
  uint16_t* d_cr;
  double* d_l64;
  float* d_lam;
  uint64_t* d_lm;
  if (dev_upload(&d_diag, diag_ptr) != hipSuccess || dev_upload(&d_ror, row_of_rank) != hipSuccess ||
      dev_upload(&d_dor, deg_of_rank) != hipSuccess || dev_upload(&d_ci, colinfo) != hipSuccess ||
      dev_upload(&d_ce, cedge) != hipSuccess || dev_upload(&d_cr, crank) != hipSuccess ||
      dev_upload(&d_lam, lam) != hipSuccess || dev_upload(&d_lm, lmask) != hipSuccess ||
      dev_upload(&d_l64, lam64) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return fail(BSD_ENOMEM, "cannot upload the graph");
  }
  // Screen: rows in CSR form (ascending columns); per edge in that order,
  // its column's rows (original numbering, ascending), each flagged when the
  // column holds that row's least |Lambda| (the first column in ascending
  // order with the least, as in the first-iteration table), and its column
  // with the column's prior LLR and logical mask.
  std::vector<int32_t> srp(m + 1, 0);
  std::vector<uint16_t> ser((size_t)nnz * 8, 0xFFFFu);
  std::vector<uint32_t> sec((size_t)nnz * 4);
  for (int e = 0; e < nnz; ++e) srp[h_rowidx[e] + 1]++;
  for (int i = 0; i < m; ++i) srp[i + 1] += srp[i];
  {
    std::vector<int32_t> hold((size_t)m, -1);
    std::vector<float> least((size_t)m, kLlrMax), second((size_t)m, kLlrMax);
    for (int j = 0; j < n; ++j)
      for (int e = h_colptr[j]; e < h_colptr[j + 1]; ++e) {
        const int i = h_rowidx[e];
        const float a = std::fabs(lam[j]);
        if (hold[i] < 0) hold[i] = j;
        second[i] = std::max(least[i], std::min(second[i], a));
        if (a < least[i]) {
          least[i] = a;
          hold[i] = j;
        }
      }
    // Whether one flipped detector alone can make column j decide 1 at t = 1
    // for some alpha <= 1: with row f flipped the posterior is Lambda_j +
    // alpha (b - a), a the magnitude base f sends (its least |Lambda|, or
    // its second least to the holder) and b the sum of the others', so it
    // stays at least Lambda_j + min(0, b - a).  A margin far above the
    // rounding of the single-precision sum keeps the answer on the safe side.
    std::vector<uint8_t> single((size_t)n, 0);
    for (int j = 0; j < n; ++j) {
      double tot = 0.0;
      for (int e = h_colptr[j]; e < h_colptr[j + 1]; ++e) {
        const int i = h_rowidx[e];
        tot += hold[i] == j ? second[i] : least[i];
      }
      for (int e = h_colptr[j]; e < h_colptr[j + 1]; ++e) {
        const int i = h_rowidx[e];
        const double a = hold[i] == j ? second[i] : least[i];
        const double lo = (double)lam[j] + std::min(0.0, (tot - a) - a);
        if (lo <= 1e-3 * ((double)std::fabs(lam[j]) + tot)) single[j] = 1;
      }
    }
    std::vector<int32_t> fill(srp.begin(), srp.end() - 1);
    for (int j = 0; j < n; ++j)
      for (int e = h_colptr[j]; e < h_colptr[j + 1]; ++e) {
        const int q = fill[h_rowidx[e]]++;
        for (int f = h_colptr[j]; f < h_colptr[j + 1]; ++f) {
          const int i = h_rowidx[f];
          ser[(size_t)q * 8 + (f - h_colptr[j])] =
              (uint16_t)(i | (hold[i] == j ? 0x8000 : 0) | (f == h_colptr[j] && single[j] ? 0x4000 : 0));
        }
        uint32_t lb;
        std::memcpy(&lb, &lam[j], 4);
        sec[(size_t)q * 4] = (uint32_t)j;
        sec[(size_t)q * 4 + 1] = lb;
        sec[(size_t)q * 4 + 2] = (uint32_t)lmask[j];
        sec[(size_t)q * 4 + 3] = (uint32_t)(lmask[j] >> 32);
      }
  }
  c->owned = {d_diag, d_ror, d_dor, d_ci, d_ce, d_cr, d_lam, d_lm, d_l64};
  c->all_pos = true;
  for (int j = 0; j < n; ++j) c->all_pos = c->all_pos && lam[j] > 0.f;
  uint16_t* d_ser = nullptr;
  uint32_t* d_sec = nullptr;
  if (dev_upload(&c->s_rowptr, srp) != hipSuccess || dev_upload(&d_ser, ser) != hipSuccess ||
      dev_upload(&d_sec, sec) != hipSuccess) {
    (void)hipGetLastError();
    hipFree(d_ser);
    hipFree(d_sec);
    bsd_code_destroy(c);
    return fail(BSD_ENOMEM, "cannot upload the graph");
  }
  c->s_edgerows = reinterpret_cast<uint4*>(d_ser);
  c->s_edgecol = reinterpret_cast<uint4*>(d_sec);
  // Unrolled decoder: the CSC pointers, and each row's edges (CSC positions)
  // in ascending column order.
  {
    std::vector<int32_t> re((size_t)nnz);
    std::vector<int32_t> fill(srp.begin(), srp.end() - 1);
    for (int j = 0; j < n; ++j)
      for (int e = h_colptr[j]; e < h_colptr[j + 1]; ++e) re[fill[h_rowidx[e]]++] = e;
    if (dev_upload(&c->u_colptr, c->colptr) != hipSuccess || dev_upload(&c->u_rowptr, srp) != hipSuccess ||
        dev_upload(&c->u_rowedge, re) != hipSuccess) {
      (void)hipGetLastError();
      bsd_code_destroy(c);
      return fail(BSD_ENOMEM, "cannot upload the unrolled decoder's tables");
    }
  }
  c->screen_per_cu = screen_blocks_per_cu(m, 1);
  c->screen2_per_cu = screen_blocks_per_cu(m, 2);
  c->d_lam64 = d_l64;
  g.diag_ptr = d_diag;
  g.row_of_rank = d_ror;
  g.deg_of_rank = d_dor;
  g.colinfo = d_ci;
  g.cedge = d_ce;
  g.crank = reinterpret_cast<const uint4*>(d_cr);
  g.lambda = d_lam;
  g.lmask = d_lm;

  // Launch geometry: one BP run per workgroup; columns c * block + tid,
  // detector rows of rank q * block + tid (q < 2).
  c->lds = lds_bytes_for(g);
  if (c->lds > (size_t)kLdsBytes || g.nnz_pad + kTrashWords + 1 > 65535 || maxdeg > 252) {
    bsd_code_destroy(c);
    return fail(BSD_EINVAL, "graph too large: %d edges need %zu bytes of LDS (limit %d)", nnz,
                c->lds, kLdsBytes);
  }
  int maxdeg_col = 1;
  for (int j = 0; j < n; ++j) maxdeg_col = std::max(maxdeg_col, h_colptr[j + 1] - h_colptr[j]);
  c->pw = (maxdeg_col + 1) / 2;
  c->maxdeg_col = maxdeg_col;
  // A workgroup of 1024 lanes holds up to 9 columns per lane in registers;
  // beyond that 512 lanes get twice the registers.  Small graphs get 512-lane
  // workgroups, one per CU: with thousands of single-wave workgroups, the
  // idle ones' polling of the queue counters slowed the busy ones' atomics
  // (W0, W1 and the XYZ workload ran 1.3 to 4.7 times slower), and two per
  // CU ran 7 to 30 % slower than one (fewer than one per CU, slower still).
  // BSD_BLOCK overrides the choice; bsd_code_autotune measures.
  int block;
  if (c->lds > 64 * 1024) {
    block = supported_cpt((n + 1023) / 1024) <= 9 ? 1024 : 512;
  } else {
    block = 512;
    while (supported_cpt((n + block - 1) / block) > 16 || m > 2 * block) block *= 2;
  }
  if (const char* eb = getenv("BSD_BLOCK")) {
    const int b = atoi(eb);
    if (b >= 64 && b <= 1024 && (b & (b - 1)) == 0) block = b;
  }
  {
    bsd_status gs = set_geometry(c, block, c->lds > 64 * 1024 ? 0 : 1);
    if (gs != BSD_OK) {
      std::string msg = g_err;
      bsd_code_destroy(c);
      return fail(gs, "%s", msg.c_str());
    }
  }
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    bsd_code_destroy(c);
    return fail(BSD_EDEVICE, "hipEventCreate failed");
  }
  *out = c;
  return BSD_OK;
}

bsd_status bsd_code_destroy(bsd_code c) {
  if (!c) return BSD_OK;
  {
    std::unique_lock<std::shared_mutex> cfg(c->cfg_mu);
    if (c->busy.load() != 0) return fail(BSD_EBUSY, "code handle is in use");
  }
  // Work enqueued by asynchronous calls finishes before its memory goes.
  for (Lane* l : c->lanes) lane_free(l);
  c->lanes.clear();
  for (FiTab* t : c->fi_tabs) fitab_free(t);
  c->fi_tabs.clear();
  hipFree(c->d_stage);
  hipFree(c->d_resbits);
  hipFree(c->d_asched);
  hipFree(c->u_colptr);
  hipFree(c->u_rowptr);
  hipFree(c->u_rowedge);
  hipFree(c->s_rowptr);
  hipFree(c->s_edgerows);
  hipFree(c->s_edgecol);
  for (void* p : c->owned) hipFree(p);
  hipFree(c->pslots);
  hipFree(c->d_pairs);
  hipFree(c->d_result);
  hipFree(c->d_error);
  hipHostFree(c->h_pinned);
  if (c->ev0) hipEventDestroy(c->ev0);
  if (c->ev1) hipEventDestroy(c->ev1);
  delete c;
  return BSD_OK;
}

bsd_status bsd_code_set_alpha_schedule(bsd_code c, int32_t n, const float* alphas) {
  if (!c) return fail(BSD_EINVAL, "code is NULL");
  if (n < 0 || n > 4096 || (n > 0 && !alphas)) return fail(BSD_EINVAL, "need 0 <= n <= 4096 scalings");
  for (int i = 0; i < n; ++i)
    if (!(alphas[i] > 0.f) || !std::isfinite(alphas[i]))
      return fail(BSD_EINVAL, "scaling %d must be positive and finite", i);
  std::unique_lock<std::shared_mutex> cfg(c->cfg_mu);
  if (c->busy.load() != 0) return fail(BSD_EBUSY, "code handle is in use");
  quiesce(c);  // asynchronous calls may still read the old schedule
  hipFree(c->d_asched);
  c->d_asched = nullptr;
  c->asched.assign(alphas, alphas + n);
  if (n > 0 && dev_upload(&c->d_asched, c->asched) != hipSuccess) {
    (void)hipGetLastError();
    c->asched.clear();
    return fail(BSD_ENOMEM, "cannot upload the schedule");
  }
  return BSD_OK;
}

bsd_status bsd_code_info(bsd_code c, int64_t* nnz, int32_t* block, int32_t* grid, int32_t* lds) {
  if (!c) return fail(BSD_EINVAL, "code is NULL");
  if (nnz) *nnz = c->g.nnz;
  if (block) *block = c->block;
  if (grid) *grid = c->grid;
  if (lds) *lds = (int32_t)c->lds;
  return BSD_OK;
}

}  // extern "C"

namespace {

// True for memory the device can address directly (device memory, or host
// memory allocated or registered with HIP).
bool is_device_ptr(const void* ptr) {
  hipPointerAttribute_t at{};
  if (hipPointerGetAttributes(&at, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged ||
         at.devicePointer != nullptr;
}

// Host buffers: copy the syndromes in and the outputs back through device
// buffers of the code handle (grown on demand); synchronous.
// Configuration lock shared and c->stage_mu held; the lane's mutex (batched)
// or c->mu (plain) is taken here.
bsd_status decode_staged(bsd_code c, Lane* l, const FiTab* ft, const bsd_params* p, int64_t shots,
                         const uint8_t* syn, uint8_t* corr, uint8_t* flips, uint8_t* conv,
                         hipStream_t s, bsd_stats* stats, uint32_t* lat) {
  const DevGraph& g = c->g;
  const size_t need = (size_t)shots * (g.m + g.n + std::max(g.k, 1) + 1 + 4) + 64;
  if (c->stage_bytes < need) {
    hipFree(c->d_stage);
    c->d_stage = nullptr;
    c->stage_bytes = 0;
    if (hipMalloc((void**)&c->d_stage, need) != hipSuccess) {
      (void)hipGetLastError();
      return fail(BSD_ENOMEM, "cannot allocate %zu bytes to stage host buffers", need);
    }
    c->stage_bytes = need;
  }
  uint8_t* ds = c->d_stage;
  uint8_t* dc = ds + (size_t)shots * g.m;
  uint8_t* df = dc + (size_t)shots * g.n;
  uint8_t* dv = df + (size_t)shots * std::max(g.k, 1);
  uint32_t* dl = reinterpret_cast<uint32_t*>(((uintptr_t)(dv + shots) + 15) & ~(uintptr_t)15);
  const bool dev_syn = is_device_ptr(syn);
  HIP_OR_FAIL(hipMemcpyAsync(ds, syn, (size_t)shots * g.m,
                             dev_syn ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  bsd_status st;
  if (p->mode == BSD_MODE_PLAIN) {
    std::lock_guard<std::mutex> lock(c->mu);
    st = decode_plain(c, p, shots, ds, dc, df, dv, s, stats, lat ? dl : nullptr);
  } else {
    std::lock_guard<std::mutex> lock(l->mu);
    st = decode_batched(c, l, p, ft, shots, ds, dc, df, dv, false, stats, lat ? dl : nullptr);
  }
  if (st != BSD_OK) return st;
  HIP_OR_FAIL(hipMemcpyAsync(corr, dc, (size_t)shots * g.n, hipMemcpyDefault, s));
  if (g.k > 0) HIP_OR_FAIL(hipMemcpyAsync(flips, df, (size_t)shots * g.k, hipMemcpyDefault, s));
  HIP_OR_FAIL(hipMemcpyAsync(conv, dv, (size_t)shots, hipMemcpyDefault, s));
  if (lat) HIP_OR_FAIL(hipMemcpyAsync(lat, dl, (size_t)shots * 4, hipMemcpyDefault, s));
  HIP_OR_FAIL(hipStreamSynchronize(s));
  return BSD_OK;
}

}  // namespace

extern "C" {

bsd_status bsd_decode_ex(bsd_code c, const bsd_params* p, int64_t shots, const uint8_t* syn,
                         uint8_t* corr, uint8_t* flips, uint8_t* conv, void* stream,
                         bsd_stats* stats, uint32_t* lat) {
  if (!c) return fail(BSD_EINVAL, "code is NULL");
  bsd_status st = check_params(c, p);
  if (st != BSD_OK) return st;
  if (shots < 0) return fail(BSD_EINVAL, "shots must be >= 0");
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (shots == 0) return BSD_OK;
  if (shots > (int64_t)0x7FFFFFFF) return fail(BSD_EINVAL, "at most 2^31-1 shots per call");
  if (!syn || !corr || !conv || (c->g.k > 0 && !flips))
    return fail(BSD_EINVAL, "syndromes, corrections, logical_flips and converged are required");
  c->busy++;
  int dev_prev = 0;
  (void)hipGetDevice(&dev_prev);
  (void)hipSetDevice(c->device);
  hipStream_t s = (hipStream_t)stream;
  const bool staged = !is_device_ptr(syn) || !is_device_ptr(corr) || !is_device_ptr(conv) ||
                      (c->g.k > 0 && !is_device_ptr(flips)) || (lat && !is_device_ptr(lat));
  // Device buffers in batched mode with neither stats nor latencies asked
  // for: return once the work is enqueued (errors: bsd_code_sync).
  const bool async = !staged && !stats && !lat && p->mode == BSD_MODE_BATCHED;
  Lane* l = p->mode == BSD_MODE_BATCHED ? get_lane(c, s) : nullptr;
  if (p->mode == BSD_MODE_BATCHED && !l) {
    st = fail(BSD_EBUSY, "no workspace for another stream (at most %zu streams per code)", kMaxLanes);
  } else {
    std::unique_lock<std::mutex> stage;
    if (staged) stage = std::unique_lock<std::mutex>(c->stage_mu);
    st = with_tables(c, p, [&](const FiTab* ft) -> bsd_status {
      if (staged) return decode_staged(c, l, ft, p, shots, syn, corr, flips, conv, s, stats, lat);
      if (p->mode == BSD_MODE_PLAIN) {
        std::lock_guard<std::mutex> lock(c->mu);
        return decode_plain(c, p, shots, syn, corr, flips, conv, s, stats, lat);
      }
      std::lock_guard<std::mutex> lock(l->mu);
      return decode_batched(c, l, p, ft, shots, syn, corr, flips, conv, async, stats, lat);
    });
  }
  (void)hipSetDevice(dev_prev);
  c->busy--;
  return st;
}

bsd_status bsd_code_sync(bsd_code c, void* stream) {
  if (!c) return fail(BSD_EINVAL, "code is NULL");
  hipStream_t s = (hipStream_t)stream;
  Lane* l = get_lane(c, s, false);
  if (!l) return BSD_OK;
  std::shared_lock<std::shared_mutex> cfg(c->cfg_mu);
  std::lock_guard<std::mutex> lock(l->mu);
  if (!l->ws.st) return BSD_OK;
  HIP_OR_FAIL(hipMemcpyAsync(l->ws.st_host, l->ws.st, sizeof(BatchState), hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(hipStreamSynchronize(s));
  l->pending = false;
  BatchState& h = *l->ws.st_host;
  const bool bad = h.error || h.sticky;
  const unsigned long long done = h.done;
  if (bad) {  // report once
    h.error = 0;
    h.sticky = 0;
    HIP_OR_FAIL(hipMemcpyAsync(l->ws.st, l->ws.st_host, sizeof(BatchState), hipMemcpyHostToDevice, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    return fail(BSD_EINVAL, "syndrome bytes must be 0 or 1 (a call on this stream since the last check)");
  }
  if (l->last_shots && done != (unsigned long long)l->last_shots)
    return fail(BSD_EDEVICE, "batched decoder finished %llu of %lld shots", done, (long long)l->last_shots);
  return BSD_OK;
}

bsd_status bsd_decode(bsd_code c, const bsd_params* p, int64_t shots, const uint8_t* syn,
                      uint8_t* corr, uint8_t* flips, uint8_t* conv, void* stream) {
  return bsd_decode_ex(c, p, shots, syn, corr, flips, conv, stream, nullptr, nullptr);
}

bsd_status bsd_bp_run(bsd_code c, const float* e_start, const int32_t* pairs, int32_t npairs,
                      const uint8_t* syndrome, int32_t max_iters, float alpha,
                      int32_t stop_on_converge, float* e_out, float* sum_llr, uint8_t* ehat,
                      int32_t* iters, int32_t* converged, int32_t* next_pos, float* score,
                      void* stream) {
  if (!c) return fail(BSD_EINVAL, "code is NULL");
  if (!syndrome) return fail(BSD_EINVAL, "syndrome is NULL");
  if (max_iters < 0) return fail(BSD_EINVAL, "max_iters must be >= 0");
  if (npairs < 0 || npairs > kMaxRounds) return fail(BSD_EINVAL, "npairs must be in [0, %d]", kMaxRounds);
  if (npairs > 0 && !pairs) return fail(BSD_EINVAL, "pairs is NULL");
  if (!(alpha > 0.f) || !std::isfinite(alpha)) return fail(BSD_EINVAL, "alpha must be positive and finite");
  std::vector<int32_t> packed(npairs);
  for (int q = 0; q < npairs; ++q) {
    const int col = pairs[2 * q], val = pairs[2 * q + 1];
    if (col < 0 || col >= c->g.n || (val != 0 && val != 1))
      return fail(BSD_EINVAL, "pair %d = (%d, %d) is invalid", q, col, val);
    for (int r = 0; r < q; ++r)
      if ((packed[r] >> 1) == col) return fail(BSD_EINVAL, "column %d is masked twice", col);
    packed[q] = (col << 1) | val;
  }
  std::lock_guard<std::mutex> lock(c->mu);
  bsd_status st = ensure_plain(c, 0);
  if (st != BSD_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  HIP_OR_FAIL(hipMemsetAsync(c->d_error, 0, 4, s));
  if (npairs) {
    std::memcpy(c->h_pinned, packed.data(), npairs * 4);
    HIP_OR_FAIL(hipMemcpyAsync(c->d_pairs, c->h_pinned, npairs * 4, hipMemcpyHostToDevice, s));
  }
  SingleArgs a{};
  a.g = c->g;
  a.parent_csc = e_start;
  a.pairs = c->d_pairs;
  a.npairs = npairs;
  a.syn = syndrome;
  a.max_iters = max_iters;
  a.stop = stop_on_converge ? 1 : 0;
  a.alpha = alpha;
  a.want_score = 1;
  a.out_csc = e_out;
  a.out_sumllr = sum_llr;
  a.out_ehat = ehat;
  a.result = c->d_result;
  a.error = c->d_error;
  HIP_OR_FAIL(launch_single(a, c->block, c->cpt, c->pw, c->lds, s));
  int32_t* res = c->h_pinned + kMaxRounds;
  HIP_OR_FAIL(hipMemcpyAsync(res, c->d_result, 16, hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(hipMemcpyAsync(res + 4, c->d_error, 4, hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(hipStreamSynchronize(s));
  if (res[4]) return fail(BSD_EINVAL, "syndrome bytes must be 0 or 1");
  if (iters) *iters = res[0];
  if (converged) *converged = res[1];
  if (next_pos) *next_pos = res[2];
  if (score) std::memcpy(score, &res[3], 4);
  return BSD_OK;
}

bsd_status bsd_code_autotune(bsd_code c, const bsd_params* p, int64_t shots, const uint8_t* syn,
                             int32_t* out_block, int32_t* out_grid, float* out_ms, void* stream) {
  if (!c) return fail(BSD_EINVAL, "code is NULL");
  bsd_status st = check_params(c, p);
  if (st != BSD_OK) return st;
  if (shots <= 0 || !syn) return fail(BSD_EINVAL, "autotune needs a non-empty batch of syndromes");
  hipDeviceProp_t prop;
  HIP_OR_FAIL(hipGetDeviceProperties(&prop, c->device));
  uint64_t h = 1469598103934665603ull;
  h = fnv1a(h, &c->g.m, sizeof c->g.m);
  h = fnv1a(h, &c->g.n, sizeof c->g.n);
  h = fnv1a(h, c->colptr.data(), c->colptr.size() * 4);
  h = fnv1a(h, c->rowidx.data(), c->rowidx.size() * 4);
  const int32_t pk[5] = {p->max_rounds, p->beam_width, p->initial_iters, p->iters_per_round,
                         p->num_results};
  h = fnv1a(h, pk, sizeof pk);
  h = fnv1a(h, prop.gcnArchName, strlen(prop.gcnArchName));
  const char* cache = getenv("BSD_TUNE_CACHE");
  if (cache) {
    if (FILE* f = fopen(cache, "r")) {
      unsigned long long key;
      int b, half;
      float ms;
      bool hit = false;
      while (fscanf(f, "%llx %d %d %f", &key, &b, &half, &ms) == 4) {
        if (key == h) {
          std::unique_lock<std::shared_mutex> cfg(c->cfg_mu);
          if (set_geometry(c, b, half) == BSD_OK) {
            hit = true;
            if (out_ms) *out_ms = ms;
          }
        }
      }
      fclose(f);
      if (hit) {
        if (out_block) *out_block = c->block;
        if (out_grid) *out_grid = c->grid;
        return BSD_OK;
      }
    }
  }
  uint8_t *corr = nullptr, *flips = nullptr, *conv = nullptr;
  if (hipMalloc((void**)&corr, (size_t)shots * c->g.n) != hipSuccess ||
      hipMalloc((void**)&flips, (size_t)shots * std::max(c->g.k, 1)) != hipSuccess ||
      hipMalloc((void**)&conv, (size_t)shots) != hipSuccess) {
    hipFree(corr);
    hipFree(flips);
    (void)hipGetLastError();
    return fail(BSD_ENOMEM, "autotune scratch allocation failed");
  }
  const int b0 = c->block, h0 = c->grid_frac_half;
  int best_b = b0, best_h = h0;
  float best_ms = 3.0e38f;
  bsd_params q = *p;
  q.mode = BSD_MODE_BATCHED;
  q.flags = 0;
  for (int b = 64; b <= 1024 && st == BSD_OK; b *= 2) {
    for (int half = 0; half <= 1; ++half) {
      {
        std::unique_lock<std::shared_mutex> cfg(c->cfg_mu);
        if (set_geometry(c, b, half) != BSD_OK) break;
        if (half && !c->grid_frac_half) break;
      }
      float ms_min = 3.0e38f;
      for (int rep = 0; rep < 3 && st == BSD_OK; ++rep) {
        bsd_stats sts;
        st = bsd_decode_ex(c, &q, shots, syn, corr, flips, conv, stream, &sts, nullptr);
        if (st == BSD_OK && rep > 0) ms_min = std::min(ms_min, (float)sts.kernel_ms);
      }
      if (st == BSD_OK && ms_min < best_ms) {
        best_ms = ms_min;
        best_b = b;
        best_h = half;
      }
    }
  }
  hipFree(corr);
  hipFree(flips);
  hipFree(conv);
  {
    std::unique_lock<std::shared_mutex> cfg(c->cfg_mu);
    bsd_status s2 = set_geometry(c, best_b, best_h);
    if (st == BSD_OK) st = s2;
  }
  if (st != BSD_OK) return st;
  if (cache) {
    if (FILE* f = fopen(cache, "a")) {
      fprintf(f, "%llx %d %d %.6f\n", (unsigned long long)h, best_b, best_h, best_ms);
      fclose(f);
    }
  }
  if (out_block) *out_block = c->block;
  if (out_grid) *out_grid = c->grid;
  if (out_ms) *out_ms = best_ms;
  return BSD_OK;
}

// ---------------------------------------------------------------------------
// Serving: persistent decoders fed through rings in host memory
// ---------------------------------------------------------------------------

}  // extern "C"

namespace {

constexpr uint32_t kDecoderIdleTicks = 2000000000u;  // default idle limit: 20 s at 100 MHz

struct ServeQ {
  bsd_code code = nullptr;
  bsd_params prm{};
  hipStream_t stream = nullptr;
  BatchWs ws;
  int grid = 0;
  uint32_t rows = 0;  // ring rows, a power of two
  // Pinned host memory (device views in d_*): syndromes, outputs, flags.
  uint8_t *syn = nullptr, *corr = nullptr, *flips = nullptr, *conv = nullptr;
  uint32_t *lat = nullptr, *done = nullptr, *started = nullptr, *begun = nullptr, *gen = nullptr;
  unsigned long long* pub = nullptr;
  uint8_t *d_syn = nullptr, *d_corr = nullptr, *d_flips = nullptr, *d_conv = nullptr;
  uint32_t *d_lat = nullptr, *d_done = nullptr, *d_started = nullptr, *d_begun = nullptr,
           *d_gen = nullptr;
  std::vector<hipStream_t> old_streams;  // streams of replaced launches (destroyed with the server)
  unsigned long long* d_pub = nullptr;
  uint64_t next = 0;                   // tickets issued
  std::vector<int64_t> row_ticket;     // ticket holding each row, -1 if free
  BatchArgs args{};                    // of the decoder's launches
  int64_t launches = 0;                // the first and every relaunch after an idle exit
};

template <class T>
hipError_t pinned(T** host, T** dev, size_t count) {
  hipError_t e = hipHostMalloc((void**)host, count * sizeof(T), hipHostMallocMapped | hipHostMallocCoherent);
  if (e != hipSuccess) return e;
  std::memset(*host, 0, count * sizeof(T));
  return hipHostGetDevicePointer((void**)dev, *host, 0);
}

double now_us() {
  return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

struct bsd_server_s {
  int n = 0;
  int device = 0;
  ServeQ q[kMaxServe];
  uint32_t* stop = nullptr;
  uint32_t* d_stop = nullptr;
  bool launched = false;
};

namespace {

void server_free(bsd_server s) {
  for (int i = 0; i < s->n; ++i) {
    ServeQ& q = s->q[i];
    ws_free(q.ws);
    hipHostFree(q.syn);
    hipHostFree(q.corr);
    hipHostFree(q.flips);
    hipHostFree(q.conv);
    hipHostFree(q.lat);
    hipHostFree(q.done);
    hipHostFree(q.started);
    hipHostFree(q.begun);
    hipHostFree(q.gen);
    hipHostFree(q.pub);
    if (q.stream) hipStreamDestroy(q.stream);
    for (hipStream_t os : q.old_streams) hipStreamDestroy(os);
    if (q.code) q.code->busy--;
  }
  hipHostFree(s->stop);
  delete s;
}

// Ask every kernel of the server to end and wait (bounded) until they have.
bsd_status server_stop(bsd_server s) {
  if (!s->launched) return BSD_OK;
  __atomic_store_n(s->stop, 1u, __ATOMIC_RELEASE);
  const double t0 = now_us();
  for (;;) {
    bool all = true;
    for (int i = 0; i < s->n; ++i) {
      all = all && hipStreamQuery(s->q[i].stream) != hipErrorNotReady;
      for (hipStream_t os : s->q[i].old_streams) all = all && hipStreamQuery(os) != hipErrorNotReady;
    }
    if (all) break;
    if (now_us() - t0 > 60e6) return fail(BSD_EDEVICE, "serving kernels did not stop within 60 s");
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
  s->launched = false;
  return BSD_OK;
}

bool decoder_running(const ServeQ& q) { return hipStreamQuery(q.stream) == hipErrorNotReady; }

// Launch (or relaunch) one decoder and wait until every workgroup runs.
// HIP maps streams to a limited set of hardware queues; two decoders whose
// streams share one run in turn, and a persistent decoder behind another
// never starts.  A launch none of whose workgroups has begun after a short
// wait is therefore replaced: the generation moves on (the old launch ends
// at once whenever it starts) and the decoder is launched on a new stream.
bsd_status launch_decoder(ServeQ& q, int index) {
  constexpr int kAttempts = 6;
  for (int attempt = 0; attempt < kAttempts; ++attempt) {
    const uint32_t g = __atomic_load_n(q.gen, __ATOMIC_RELAXED) + 1u;
    __atomic_store_n(q.begun, 0u, __ATOMIC_RELAXED);
    __atomic_store_n(q.started, 0u, __ATOMIC_RELAXED);
    __atomic_store_n(q.gen, g, __ATOMIC_RELEASE);
    q.args.gen = g;
    hipError_t he = launch_batched(q.args, q.grid, q.code->block, q.code->cpt, q.code->pw,
                                   q.code->lds, q.stream);
    if (he != hipSuccess) return fail(BSD_EDEVICE, "serving launch: %s", hipGetErrorString(he));
    const double t0 = now_us();
    bool begun = false;
    while (!(begun = __atomic_load_n(q.begun, __ATOMIC_ACQUIRE)) && now_us() - t0 < 250e3)
      std::this_thread::sleep_for(std::chrono::microseconds(100));
    if (!begun) {  // queued behind another kernel: a new stream for the next attempt
      hipStream_t ns = nullptr;
      he = hipStreamCreateWithFlags(&ns, hipStreamNonBlocking);
      if (he != hipSuccess) return fail(BSD_EDEVICE, "serving stream: %s", hipGetErrorString(he));
      q.old_streams.push_back(q.stream);
      q.stream = ns;
      continue;
    }
    ++q.launches;  // (a replaced launch is not counted)
    while (!__atomic_load_n(q.started, __ATOMIC_ACQUIRE)) {
      if (now_us() - t0 > 5e6)
        return fail(BSD_EDEVICE, "serving decoder %d (%d workgroups) did not have every "
                    "workgroup running within 5 s; fewer workgroups may be needed", index, q.grid);
      std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    return BSD_OK;
  }
  // (the generation moves on once more, so that no queued launch runs later)
  __atomic_store_n(q.gen, __atomic_load_n(q.gen, __ATOMIC_RELAXED) + 1u, __ATOMIC_RELEASE);
  return fail(BSD_EDEVICE, "serving decoder %d did not start on any of %d streams: every "
              "hardware queue tried was busy with another persistent kernel", index, kAttempts);
}

// A decoder that ended after its idle limit is started again: requests
// published since are claimed by the new launch (its state, rings and
// contexts carry over; every context was returned when the workgroups ended).
bsd_status ensure_decoder(bsd_server s, int code) {
  if (!s->launched) return fail(BSD_EDEVICE, "serving kernels have stopped");
  ServeQ& q = s->q[code];
  if (decoder_running(q)) return BSD_OK;
  return launch_decoder(q, code);
}

// Hardware queues HIP gives this process (GPU_MAX_HW_QUEUES, default 4).
int hw_queues() {
  const char* e = getenv("GPU_MAX_HW_QUEUES");
  const int v = e ? atoi(e) : 0;
  return v > 0 ? v : 4;
}

}  // namespace

extern "C" {

bsd_status bsd_server_create(int32_t ncodes, const bsd_code* codes, const bsd_params* params,
                             const int32_t* grid_blocks, int64_t ring_bytes, bsd_server* out) {
  bsd_server_opts o{};
  o.ring_bytes = ring_bytes;
  return bsd_server_create_ex(ncodes, codes, params, grid_blocks, &o, out);
}

bsd_status bsd_server_create_ex(int32_t ncodes, const bsd_code* codes, const bsd_params* params,
                                const int32_t* grid_blocks, const bsd_server_opts* opts,
                                bsd_server* out) {
  if (!out) return fail(BSD_EINVAL, "out is NULL");
  *out = nullptr;
  if (ncodes < 1 || ncodes > kMaxServe || !codes || !params)
    return fail(BSD_EINVAL, "need 1..%d codes and their params", kMaxServe);
  const int64_t ring_bytes = opts ? opts->ring_bytes : 0;
  const int64_t idle_ms = opts ? opts->idle_ms : 0;
  if (ring_bytes < 0) return fail(BSD_EINVAL, "ring_bytes must be >= 0");
  if (idle_ms < 0 || idle_ms > 40000) return fail(BSD_EINVAL, "idle_ms must be in [0, 40000]");
  // Each decoder is a persistent kernel on a stream of its own; they must all
  // run at once, which needs a hardware queue each.
  if (ncodes > hw_queues())
    return fail(BSD_EINVAL, "serving %d codes needs %d hardware queues, and this process has %d "
                "(set GPU_MAX_HW_QUEUES before HIP initialises)", ncodes, ncodes, hw_queues());
  const uint32_t idle_ticks = idle_ms > 0 ? (uint32_t)(idle_ms * 100000) : kDecoderIdleTicks;
  int dev = 0;
  HIP_OR_FAIL(hipGetDevice(&dev));
  for (int i = 0; i < ncodes; ++i) {
    if (!codes[i]) return fail(BSD_EINVAL, "code %d is NULL", i);
    if (codes[i]->device != dev) return fail(BSD_EINVAL, "code %d lives on another device", i);
    bsd_status st = check_params(codes[i], &params[i]);
    if (st != BSD_OK) return st;
    if (params[i].mode != BSD_MODE_BATCHED) return fail(BSD_EINVAL, "serving needs the batched mode");
    for (int j = 0; j < i; ++j)
      if (codes[j] == codes[i]) return fail(BSD_EINVAL, "code %d is listed twice", i);
  }
  int ncu = 0;
  HIP_OR_FAIL(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  bsd_server s = new (std::nothrow) bsd_server_s;
  if (!s) return fail(BSD_ENOMEM, "host allocation failed");
  s->device = dev;
  // Automatic sizes.  Idle workgroups poll the queue counters, and on a
  // mixed load of a few thousand requests per second per code fewer
  // workgroups gave lower latency at every percentile: a code whose run
  // fills a compute unit's LDS gets ncu/32 workgroups (one per unit), any
  // other code one per beam path (at least 16), half the children of one
  // round of a deep shot.
  const int64_t budget = ring_bytes > 0 ? ring_bytes : (int64_t)64 << 20;
  for (int i = 0; i < ncodes; ++i) {
    ServeQ& q = s->q[i];
    bsd_code c = codes[i];
    q.code = c;
    c->busy++;
    s->n = i + 1;
    q.prm = params[i];
    const bool big = c->lds > 64 * 1024;
    q.grid = grid_blocks && grid_blocks[i] > 0 ? grid_blocks[i]
             : big ? std::max(1, ncu / 32)
                   : std::min(c->grid, std::max(16, q.prm.beam_width));
    const DevGraph& g = c->g;
    const size_t per = (size_t)g.m + g.n + std::max(g.k, 1) + 1 + 8;
    uint64_t rows = 64;
    while (rows * 2 <= 4096 && (int64_t)(rows * 2 * per) <= budget / ncodes) rows *= 2;
    q.rows = (uint32_t)rows;
    q.row_ticket.assign(rows, -1);
    bsd_status st = ws_ensure(g, q.ws, q.prm.beam_width, q.grid + 64, q.prm.num_results);
    hipError_t e = hipSuccess;
    if (st == BSD_OK) {
      if ((e = pinned(&q.syn, &q.d_syn, rows * g.m)) != hipSuccess ||
          (e = pinned(&q.corr, &q.d_corr, rows * g.n)) != hipSuccess ||
          (e = pinned(&q.flips, &q.d_flips, rows * std::max(g.k, 1))) != hipSuccess ||
          (e = pinned(&q.conv, &q.d_conv, rows)) != hipSuccess ||
          (e = pinned(&q.lat, &q.d_lat, rows)) != hipSuccess ||
          (e = pinned(&q.done, &q.d_done, rows)) != hipSuccess ||
          (e = pinned(&q.started, &q.d_started, 1)) != hipSuccess ||
          (e = pinned(&q.begun, &q.d_begun, 1)) != hipSuccess ||
          (e = pinned(&q.gen, &q.d_gen, 1)) != hipSuccess ||
          (e = pinned(&q.pub, &q.d_pub, 1)) != hipSuccess ||
          (e = hipStreamCreateWithFlags(&q.stream, hipStreamNonBlocking)) != hipSuccess)
        st = fail(BSD_ENOMEM, "serving buffers for code %d: %s", i, hipGetErrorString(e));
    }
    if (st != BSD_OK) {
      server_free(s);
      return st;
    }
  }
  hipError_t e = pinned(&s->stop, &s->d_stop, 1);
  if (e != hipSuccess) {
    server_free(s);
    return fail(BSD_ENOMEM, "serving control: %s", hipGetErrorString(e));
  }
  // Arguments; reset every workspace before any persistent kernel starts.
  std::vector<BatchArgs> args(ncodes);
  for (int i = 0; i < ncodes; ++i) {
    ServeQ& q = s->q[i];
    const FiTab* ft = nullptr;
    bsd_status st = BSD_OK;
    if (needs_first(&q.prm)) {  // kept until the code is destroyed, which the server prevents
      std::unique_lock<std::shared_mutex> cfg(q.code->cfg_mu);
      st = build_first(q.code, first_alpha(q.code, &q.prm), &ft);
    }
    if (st == BSD_OK) args[i] = batch_args(q.code, q.ws, &q.prm, ft);
    hipError_t he = st == BSD_OK ? set_kernel_limits(q.code->cpt, q.code->pw, q.code->lds) : hipSuccess;
    if (st == BSD_OK && he != hipSuccess) st = fail(BSD_EDEVICE, "hipFuncSetAttribute: %s", hipGetErrorString(he));
    if (st != BSD_OK) {
      server_free(s);
      return st;
    }
    BatchArgs& a = args[i];
    a.stream = 1;
    a.io_mask = q.rows - 1;
    a.syn = q.d_syn;
    a.corr = q.d_corr;
    a.flips = q.d_flips;
    a.conv = q.d_conv;
    a.lat = q.d_lat;
    a.done_flag = q.d_done;
    a.pub_host = q.d_pub;
    a.stop_host = s->d_stop;
    a.started = q.d_started;
    a.begun = q.d_begun;
    a.gen_host = q.d_gen;
    a.idle_limit = idle_ticks;
    a.shots = 0;
    he = launch_batch_reset(a, q.stream);
    if (he == hipSuccess) he = hipStreamSynchronize(q.stream);
    if (he != hipSuccess) {
      server_free(s);
      return fail(BSD_EDEVICE, "serving reset: %s", hipGetErrorString(he));
    }
  }
  // Largest LDS first, so that the compute units they need are still free.
  std::vector<int> order(ncodes);
  for (int i = 0; i < ncodes; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return s->q[x].code->lds > s->q[y].code->lds; });
  // One at a time: each kernel must have every workgroup resident before
  // the next is launched, so that the units a large-LDS decoder needs are
  // not taken by the small decoders' workgroups first, and no kernel waits
  // behind another on a shared hardware queue.
  s->launched = true;
  for (int i : order) {
    ServeQ& q = s->q[i];
    q.args = args[i];
    const bsd_status st = launch_decoder(q, i);
    if (st != BSD_OK) {
      const std::string msg = g_err;
      if (server_stop(s) == BSD_OK) server_free(s);
      return fail(st, "%s", msg.c_str());
    }
  }
  *out = s;
  return BSD_OK;
}

bsd_status bsd_server_submit(bsd_server s, int32_t code, const uint8_t* syndrome, int64_t* ticket) {
  if (!s || code < 0 || code >= s->n || !syndrome) return fail(BSD_EINVAL, "bad server, code or syndrome");
  ServeQ& q = s->q[code];
  const DevGraph& g = q.code->g;
  const uint64_t t = q.next;
  const uint32_t row = (uint32_t)(t & (q.rows - 1));
  if (q.row_ticket[row] >= 0) return fail(BSD_EBUSY, "ring of code %d is full", code);
  if (!s->launched) return fail(BSD_EDEVICE, "serving kernels have stopped");
  for (int i = 0; i < g.m; ++i)
    if (syndrome[i] > 1) return fail(BSD_EINVAL, "syndrome bytes must be 0 or 1");
  std::memcpy(q.syn + (size_t)row * g.m, syndrome, g.m);
  q.row_ticket[row] = (int64_t)t;
  q.next = t + 1;
  __atomic_store_n(q.pub, (unsigned long long)(t + 1), __ATOMIC_RELEASE);
  if (ticket) *ticket = (int64_t)t;
  // Published first, then checked: a decoder that ends after this check
  // is started again by the poll that finds the request unanswered.
  return ensure_decoder(s, code);
}

bsd_status bsd_server_poll(bsd_server s, int32_t code, int64_t ticket, uint8_t* corrections,
                           uint8_t* logical_flips, uint8_t* converged, uint32_t* device_ticks) {
  if (!s || code < 0 || code >= s->n || ticket < 0) return fail(BSD_EINVAL, "bad server, code or ticket");
  ServeQ& q = s->q[code];
  const DevGraph& g = q.code->g;
  const uint32_t row = (uint32_t)((uint64_t)ticket & (q.rows - 1));
  if (q.row_ticket[row] != ticket) return fail(BSD_EINVAL, "ticket %lld is not in flight", (long long)ticket);
  if (__atomic_load_n(&q.done[row], __ATOMIC_ACQUIRE) != (uint32_t)(ticket + 1)) {
    const bsd_status st = ensure_decoder(s, code);
    if (st != BSD_OK) return st;
    return BSD_EBUSY;  // not finished yet (no error message)
  }
  if (corrections) std::memcpy(corrections, q.corr + (size_t)row * g.n, g.n);
  if (logical_flips) std::memcpy(logical_flips, q.flips + (size_t)row * std::max(g.k, 1), g.k);
  if (converged) *converged = q.conv[row];
  if (device_ticks) *device_ticks = q.lat[row];
  q.row_ticket[row] = -1;
  return BSD_OK;
}

bsd_status bsd_server_info(bsd_server s, int32_t code, int32_t* running, int64_t* launches) {
  if (!s || code < 0 || code >= s->n) return fail(BSD_EINVAL, "bad server or code");
  if (running) *running = s->launched && decoder_running(s->q[code]) ? 1 : 0;
  if (launches) *launches = s->q[code].launches;
  return BSD_OK;
}

bsd_status bsd_server_destroy(bsd_server s) {
  if (!s) return BSD_OK;
  bsd_status st = server_stop(s);
  if (st != BSD_OK) return st;  // kernels still running: keep their memory
  server_free(s);
  return BSD_OK;
}

bsd_status bsd_serve_poisson(bsd_server s, double rate, const double* mix, int64_t requests,
                             const uint8_t* const* syndromes, const int64_t* n_syndromes,
                             uint64_t seed, uint8_t* const* corrections,
                             uint8_t* const* logical_flips, uint8_t* const* converged,
                             double* latency_us, int32_t* code_of, bsd_serve_report* report) {
  if (!s || !(rate > 0) || !mix || requests < 0 || !syndromes || !n_syndromes)
    return fail(BSD_EINVAL, "bad serving arguments");
  const int n = s->n;
  double cum[kMaxServe], tot = 0;
  for (int i = 0; i < n; ++i) {
    if (!(mix[i] >= 0) || n_syndromes[i] < 1 || !syndromes[i]) return fail(BSD_EINVAL, "bad mix or inputs for code %d", i);
    tot += mix[i];
    cum[i] = tot;
  }
  if (!(tot > 0)) return fail(BSD_EINVAL, "mix sums to zero");
  // Arrival times (exponential gaps) and codes from a counter-based generator.
  struct Req {
    double t;
    int code;
    int64_t idx, ticket;
  };
  std::vector<Req> req((size_t)requests);
  std::vector<int64_t> used(n, 0);
  uint64_t x = seed;
  auto next_u = [&]() {
    x += 0x9e3779b97f4a7c15ull;
    uint64_t z = x;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return ((z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  };
  double t = 0;
  for (int64_t k = 0; k < requests; ++k) {
    t += -std::log(next_u()) / rate * 1e6;
    const double u = next_u() * tot;
    int c = 0;
    while (c < n - 1 && u >= cum[c]) ++c;
    req[k] = {t, c, used[c]++ % n_syndromes[c], -1};
  }
  std::vector<double> lat((size_t)requests, 0.0);
  std::vector<std::deque<int64_t>> waiting(n), inflight(n);
  int64_t next_arrival = 0, completed = 0, waits = 0;
  std::vector<uint8_t> waited((size_t)requests, 0);
  const double span = requests ? req[requests - 1].t : 0.0;
  const double start = now_us();
  const double deadline = start + std::max(30e6, 20.0 * span);
  double last_done = start;
  while (completed < requests) {
    const double now = now_us();
    if (now > deadline) return fail(BSD_EDEVICE, "serving loop timed out with %lld of %lld done",
                                    (long long)completed, (long long)requests);
    while (next_arrival < requests && req[next_arrival].t <= now - start)
      waiting[req[next_arrival].code].push_back(next_arrival), ++next_arrival;
    for (int c = 0; c < n; ++c) {
      while (!waiting[c].empty()) {
        Req& r = req[waiting[c].front()];
        const int64_t k = waiting[c].front();
        const bsd_status st = bsd_server_submit(s, c, syndromes[c] + r.idx * s->q[c].code->g.m, &r.ticket);
        if (st == BSD_EBUSY) {
          if (!waited[k]) ++waits;
          waited[k] = 1;
          break;
        }
        if (st != BSD_OK) return st;
        waiting[c].pop_front();
        inflight[c].push_back(k);
      }
    }
    for (int c = 0; c < n; ++c) {
      const DevGraph& g = s->q[c].code->g;
      for (auto it = inflight[c].begin(); it != inflight[c].end();) {
        Req& r = req[*it];
        uint8_t* co = corrections && corrections[c] ? corrections[c] + r.idx * g.n : nullptr;
        uint8_t* fl = logical_flips && logical_flips[c] ? logical_flips[c] + r.idx * g.k : nullptr;
        uint8_t* cv = converged && converged[c] ? converged[c] + r.idx : nullptr;
        const bsd_status st = bsd_server_poll(s, c, r.ticket, co, fl, cv, nullptr);
        if (st == BSD_EBUSY) {
          ++it;
          continue;
        }
        if (st != BSD_OK) return st;
        const double tn = now_us();
        lat[*it] = tn - start - r.t;
        last_done = tn;
        ++completed;
        it = inflight[c].erase(it);
      }
    }
  }
  if (latency_us) std::memcpy(latency_us, lat.data(), lat.size() * sizeof(double));
  if (code_of)
    for (int64_t k = 0; k < requests; ++k) code_of[k] = req[k].code;
  if (report) {
    bsd_serve_report r{};
    r.requests = requests;
    r.seconds = (last_done - start) * 1e-6;
    r.offered_per_s = span > 0 ? requests / (span * 1e-6) : 0.0;
    r.served_per_s = r.seconds > 0 ? requests / r.seconds : 0.0;
    r.admission_waits = waits;
    auto pct = [](std::vector<double> v, double q) {  // nearest rank
      if (v.empty()) return 0.0;
      std::sort(v.begin(), v.end());
      const double rank = std::max(0.0, std::ceil(q * (double)v.size()) - 1.0);
      return v[std::min(v.size() - 1, (size_t)rank)];
    };
    r.p50_us = pct(lat, 0.50);
    r.p99_us = pct(lat, 0.99);
    r.p999_us = pct(lat, 0.999);
    r.max_us = pct(lat, 1.0);
    for (int c = 0; c < n; ++c) {
      std::vector<double> v;
      for (int64_t k = 0; k < requests; ++k)
        if (req[k].code == c) v.push_back(lat[k]);
      r.code_requests[c] = (int64_t)v.size();
      r.code_p50_us[c] = pct(v, 0.50);
      r.code_p99_us[c] = pct(v, 0.99);
      r.code_p999_us[c] = pct(v, 0.999);
    }
    *report = r;
  }
  return BSD_OK;
}


// ---------------------------------------------------------------------------
// Differentiable unrolled min-sum
// ---------------------------------------------------------------------------

}  // extern "C"

namespace {

bsd_status unroll_prepare(bsd_code c, int32_t elem, int32_t T, int32_t K, int64_t shots,
                          UnrollArgs* a) {
  if (!c) return fail(BSD_EINVAL, "code is NULL");
  if (elem != 4 && elem != 8) return fail(BSD_EINVAL, "element size must be 4 (float) or 8 (double)");
  if (T < 0 || T > 4096 || K < 1 || shots < 0 || shots > (int64_t)1 << 31)
    return fail(BSD_EINVAL, "need 0 <= T <= 4096, K >= 1, 0 <= shots < 2^31");
  const DevGraph& g = c->g;
  UnrollArgs u{};
  u.m = g.m;
  u.n = g.n;
  u.nnz = g.nnz;
  u.T = T;
  u.K = K;
  u.nseg = (T + K - 1) / K;
  u.colptr = c->u_colptr;
  u.rowptr = c->u_rowptr;
  u.rowedge = c->u_rowedge;
  u.shots = shots;
  u.llr_max = kLlrMax;
  if (unroll_bwd_lds(u, elem) > (size_t)kLdsBytes)
    return fail(BSD_EINVAL, "graph too large for the unrolled decoder: %zu bytes of LDS with K = %d",
                unroll_bwd_lds(u, elem), K);
  *a = u;
  return BSD_OK;
}

}  // namespace

extern "C" {

bsd_status bsd_unroll_sizes(bsd_code code, int32_t T, int32_t K, int64_t shots,
                            int64_t* checkpoint_elems, int64_t* workspace_elems) {
  UnrollArgs a{};
  bsd_status st = unroll_prepare(code, 8, T, K, shots, &a);
  if (st != BSD_OK) return st;
  if (checkpoint_elems) *checkpoint_elems = shots * (int64_t)a.nseg * a.nnz;
  if (workspace_elems) *workspace_elems = shots * (int64_t)(a.n + a.T);
  return BSD_OK;
}

bsd_status bsd_unroll_forward(bsd_code code, int32_t elem_bytes, int32_t T, int32_t K, int64_t shots,
                              const uint8_t* syndromes, const void* lambda, const void* alpha,
                              void* post, void* checkpoints, void* stream) {
  UnrollArgs a{};
  bsd_status st = unroll_prepare(code, elem_bytes, T, K, shots, &a);
  if (st != BSD_OK) return st;
  if (shots == 0) return BSD_OK;
  if (!syndromes || !lambda || (T > 0 && !alpha) || !post || (T > 0 && !checkpoints))
    return fail(BSD_EINVAL, "NULL buffer");
  a.syn = syndromes;
  a.lam = lambda;
  a.alpha = alpha;
  a.post = post;
  a.ckpt = checkpoints;
  int dev_prev = 0;
  HIP_OR_FAIL(hipGetDevice(&dev_prev));
  HIP_OR_FAIL(hipSetDevice(code->device));
  const hipError_t e = launch_unroll_forward(a, elem_bytes, (hipStream_t)stream);
  (void)hipSetDevice(dev_prev);
  if (e != hipSuccess) return fail(BSD_EDEVICE, "unrolled forward: %s", hipGetErrorString(e));
  return BSD_OK;
}

bsd_status bsd_unroll_backward(bsd_code code, int32_t elem_bytes, int32_t T, int32_t K, int64_t shots,
                               const uint8_t* syndromes, const void* lambda, const void* alpha,
                               const void* checkpoints, const void* grad_post, void* grad_lambda,
                               void* grad_alpha, void* workspace, void* stream) {
  UnrollArgs a{};
  bsd_status st = unroll_prepare(code, elem_bytes, T, K, shots, &a);
  if (st != BSD_OK) return st;
  if (!grad_lambda || (T > 0 && !grad_alpha)) return fail(BSD_EINVAL, "NULL gradient buffer");
  if (shots > 0 && (!syndromes || !lambda || (T > 0 && !alpha) || (T > 0 && !checkpoints) ||
                    !grad_post || !workspace))
    return fail(BSD_EINVAL, "NULL buffer");
  a.syn = syndromes;
  a.lam = lambda;
  a.alpha = alpha;
  a.ckpt = const_cast<void*>(checkpoints);  // read only by the backward kernels
  a.gpost = grad_post;
  a.gl_part = workspace;
  a.ga_part = static_cast<char*>(workspace) + (size_t)shots * a.n * elem_bytes;
  a.grad_lam = grad_lambda;
  a.grad_alpha = grad_alpha;
  int dev_prev = 0;
  HIP_OR_FAIL(hipGetDevice(&dev_prev));
  HIP_OR_FAIL(hipSetDevice(code->device));
  const hipError_t e = launch_unroll_backward(a, elem_bytes, (hipStream_t)stream);
  (void)hipSetDevice(dev_prev);
  if (e != hipSuccess) return fail(BSD_EDEVICE, "unrolled backward: %s", hipGetErrorString(e));
  return BSD_OK;
}

bsd_status bsd_unroll_backward_noalloc(bsd_code code, int32_t elem_bytes, int32_t T, int32_t K,
                                       int64_t shots, const uint8_t* syndromes, const void* lambda,
                                       const void* alpha, const void* checkpoints,
                                       const void* grad_post, void* grad_lambda, void* grad_alpha,
                                       void* stream) {
  UnrollArgs a{};
  bsd_status st = unroll_prepare(code, elem_bytes, T, K, shots, &a);
  if (st != BSD_OK) return st;
  const size_t need = (size_t)shots * ((size_t)a.n + (size_t)a.T) * (size_t)elem_bytes;
  if (need > kNoAllocScratchBytes)
    return fail(BSD_EINVAL, "needs %zu bytes of scratch for %lld shots; the limit is %zu bytes "
                "(%lld shots of this graph and T)", need, (long long)shots, kNoAllocScratchBytes,
                (long long)(kNoAllocScratchBytes / (((size_t)a.n + a.T) * elem_bytes)));
  if (!grad_lambda || (T > 0 && !grad_alpha)) return fail(BSD_EINVAL, "NULL gradient buffer");
  if (shots > 0 && (!syndromes || !lambda || (T > 0 && !alpha) || (T > 0 && !checkpoints) ||
                    !grad_post))
    return fail(BSD_EINVAL, "NULL buffer");
  int dev_prev = 0;
  HIP_OR_FAIL(hipGetDevice(&dev_prev));
  HIP_OR_FAIL(hipSetDevice(code->device));
  void* ws = nullptr;
  hipError_t e = noalloc_scratch(code->device, &ws);
  if (e == hipSuccess) {
    a.syn = syndromes;
    a.lam = lambda;
    a.alpha = alpha;
    a.ckpt = const_cast<void*>(checkpoints);  // read only by the backward kernels
    a.gpost = grad_post;
    a.gl_part = ws;
    a.ga_part = static_cast<char*>(ws) + (size_t)shots * a.n * elem_bytes;
    a.grad_lam = grad_lambda;
    a.grad_alpha = grad_alpha;
    e = launch_unroll_backward(a, elem_bytes, (hipStream_t)stream);
  }
  (void)hipSetDevice(dev_prev);
  if (e != hipSuccess) return fail(BSD_EDEVICE, "unrolled backward: %s", hipGetErrorString(e));
  return BSD_OK;
}

}  // extern "C"
