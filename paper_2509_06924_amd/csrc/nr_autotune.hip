// Autotuner of the plan schedule (nr_autotune): times nr_loglik_grad on the
// caller's data under candidate nr_plan_options and keeps the fastest.  Host
// code on the public C ABI only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <set>
#include <vector>

#include "nr.h"

namespace {

constexpr double kMinGain = 0.03;     // a candidate must be this much faster
constexpr double kWarmupSeconds = 0.3;
constexpr int kConfirmRounds = 3;
constexpr int kXcdRuns[] = {1, 4, 8, 16, 32};
constexpr int kNodeGroups[] = {2, 4, 8, 17};

struct Buffers {
  void* ws = nullptr;
  size_t ws_bytes = 0;
  double* logL = nullptr;
  double* g_rows = nullptr;
  double* g_inst = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  ~Buffers() {
    if (ws) (void)hipFree(ws);
    if (logL) (void)hipFree(logL);
    if (g_rows) (void)hipFree(g_rows);
    if (g_inst) (void)hipFree(g_inst);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }
};

// A plan for the options with a workspace large enough for it.
struct Candidate {
  nr_plan* plan = nullptr;
  ~Candidate() { nr_plan_destroy(plan); }
};

nr_status make_candidate(const nr_batch_desc* d, const nr_plan_options& o, Buffers& b,
                         Candidate& c) {
  nr_status s = nr_plan_create_ex(d, &o, &c.plan);
  if (s != NR_OK) return s;
  size_t need = 0;
  s = nr_workspace_size(c.plan, NR_OP_LOGLIK_GRAD, &need);
  if (s != NR_OK) return s;
  if (need > b.ws_bytes) {
    if (b.ws) (void)hipFree(b.ws);
    b.ws = nullptr;
    b.ws_bytes = 0;
    if (hipMalloc(&b.ws, need) != hipSuccess) return NR_ENOMEM;
    b.ws_bytes = need;
  }
  return NR_OK;
}

nr_status call(const Candidate& c, const nr_values* v, Buffers& b, hipStream_t s) {
  return nr_loglik_grad(c.plan, v, b.logL, b.g_rows, b.g_inst, b.ws, b.ws_bytes, s);
}

// Median of reps timed calls (events on the stream) after one untimed call.
nr_status time_calls(const Candidate& c, const nr_values* v, Buffers& b, int reps, hipStream_t s,
                     double* ms) {
  nr_status st = call(c, v, b, s);
  if (st != NR_OK) return st;
  std::vector<float> t;
  for (int r = 0; r < reps; ++r) {
    if (hipEventRecord(b.ev0, s) != hipSuccess) return NR_EHIP;
    st = call(c, v, b, s);
    if (st != NR_OK) return st;
    if (hipEventRecord(b.ev1, s) != hipSuccess) return NR_EHIP;
    if (hipEventSynchronize(b.ev1) != hipSuccess) return NR_EHIP;
    float x = 0.0f;
    if (hipEventElapsedTime(&x, b.ev0, b.ev1) != hipSuccess) return NR_EHIP;
    t.push_back(x);
  }
  std::sort(t.begin(), t.end());
  *ms = t[t.size() / 2];
  return NR_OK;
}

nr_status time_options(const nr_batch_desc* d, const nr_values* v, const nr_plan_options& o,
                       Buffers& b, int reps, hipStream_t s, double* ms) {
  Candidate c;
  nr_status st = make_candidate(d, o, b, c);
  if (st != NR_OK) return st;
  return time_calls(c, v, b, reps, s, ms);
}

bool same(const nr_plan_options& x, const nr_plan_options& y) {
  for (int k = 0; k < NR_NUM_BUCKETS; ++k)
    if (x.grad_variant[k] != y.grad_variant[k]) return false;
  return x.xcd_run == y.xcd_run && x.pack_tails == y.pack_tails &&
         x.split_tails == y.split_tails && x.side_stream == y.side_stream &&
         x.node_groups == y.node_groups;
}

}  // namespace

extern "C" nr_status nr_autotune(const nr_batch_desc* d, const nr_values* v, int32_t reps,
                                 nr_plan_options* best_out, double* ms_out, void* stream) {
  if (!d || !v || !best_out || reps < 1) return NR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  nr_plan_options def;
  nr_plan_options_default(&def);
  *best_out = def;
  if (d->n_items <= 0) return NR_OK;
  Buffers b;
  int64_t rows = d->row_off[d->n_items];
  if (hipMalloc(reinterpret_cast<void**>(&b.logL), sizeof(double) * d->n_items) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&b.g_rows), sizeof(double) * 4 * rows) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&b.g_inst), sizeof(double) * 2 * d->n_items) !=
          hipSuccess)
    return NR_ENOMEM;
  if (hipEventCreate(&b.ev0) != hipSuccess || hipEventCreate(&b.ev1) != hipSuccess)
    return NR_EHIP;

  // warm the device up (clocks, caches) for a fixed time on the default plan
  {
    Candidate c;
    nr_status st = make_candidate(d, def, b, c);
    if (st != NR_OK) return st;
    const auto t_end =
        std::chrono::steady_clock::now() + std::chrono::duration<double>(kWarmupSeconds);
    do {
      st = call(c, v, b, s);
      if (st != NR_OK) return st;
      if (hipStreamSynchronize(s) != hipSuccess) return NR_EHIP;
    } while (std::chrono::steady_clock::now() < t_end);
  }

  // any smeared dataset in use (the node-group tilings apply to them)
  bool smeared = false;
  for (int i = 0; i < d->n_items; ++i) smeared |= d->dq_over_q[d->dataset_of_item[i]] > 0.0;
  // the buckets present that have both forms
  std::set<int> used;
  const int smax = nr_store_max_layers(d->precision);
  for (int i = 0; i < d->n_items; ++i) {
    const int L = (int)(d->row_off[i + 1] - d->row_off[i]) - 2;
    for (int k = 0; k < NR_NUM_BUCKETS; ++k)
      if (L <= nr_bucket_lmax(k)) {
        if (nr_bucket_lmax(k) <= smax) used.insert(k);
        break;
      }
  }

  nr_plan_options best = def;
  double best_ms = 0.0, def_ms = 0.0;
  nr_status st = time_options(d, v, best, b, reps, s, &best_ms);
  if (st != NR_OK) return st;
  def_ms = best_ms;
  auto consider = [&](const nr_plan_options& o) -> nr_status {
    double t = 0.0;
    nr_status r = time_options(d, v, o, b, reps, s, &t);
    if (r != NR_OK) return r;
    // ties (within run-to-run noise) keep the current schedule
    if (t < best_ms * (1.0 - kMinGain)) {
      best = o;
      best_ms = t;
    }
    return NR_OK;
  };
  for (int k : used)
    for (int var : {NR_VARIANT_STORE, NR_VARIANT_RECOMPUTE}) {
      nr_plan_options o = best;
      o.grad_variant[k] = var;
      if ((st = consider(o)) != NR_OK) return st;
    }
  for (int run : kXcdRuns)
    if (run != best.xcd_run) {
      nr_plan_options o = best;
      o.xcd_run = run;
      if ((st = consider(o)) != NR_OK) return st;
    }
  {
    nr_plan_options o = best;
    o.pack_tails = 1 - o.pack_tails;
    if ((st = consider(o)) != NR_OK) return st;
  }
  for (int bit : {NR_TAILS_LONE, NR_TAILS_SPLIT, NR_SPLIT_SMALL}) {
    nr_plan_options o = best;
    o.split_tails ^= bit;
    if ((st = consider(o)) != NR_OK) return st;
  }
  {
    nr_plan_options o = best;
    o.side_stream = 1 - o.side_stream;
    if ((st = consider(o)) != NR_OK) return st;
  }
  // the (sample, Q) tiling: node groups per point (64 / G points per wave)
  if (smeared)
    for (int g : kNodeGroups)
      if (g != best.node_groups) {
        nr_plan_options o = best;
        o.node_groups = g;
        if ((st = consider(o)) != NR_OK) return st;
      }

  // confirm against the defaults, interleaved so that drift cancels
  if (!same(best, def)) {
    Candidate cd, cb;
    if ((st = make_candidate(d, def, b, cd)) != NR_OK) return st;
    if ((st = make_candidate(d, best, b, cb)) != NR_OK) return st;
    std::vector<double> td, tb;
    for (int r = 0; r < kConfirmRounds; ++r) {
      double x = 0.0;
      if ((st = time_calls(cd, v, b, reps, s, &x)) != NR_OK) return st;
      td.push_back(x);
      if ((st = time_calls(cb, v, b, reps, s, &x)) != NR_OK) return st;
      tb.push_back(x);
    }
    std::sort(td.begin(), td.end());
    std::sort(tb.begin(), tb.end());
    def_ms = td[td.size() / 2];
    if (tb[tb.size() / 2] >= def_ms * (1.0 - kMinGain)) {
      best = def;
      best_ms = def_ms;
    } else {
      best_ms = tb[tb.size() / 2];
    }
  }
  *best_out = best;
  if (ms_out) {
    ms_out[0] = best_ms;
    ms_out[1] = def_ms;
  }
  return NR_OK;
}
