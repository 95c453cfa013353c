// C ABI of the reflectivity log-likelihood library: argument validation, plan
// construction (work list, record offsets, quadrature rule) and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "nr.h"
#include "nr_internal.hpp"

using namespace nr;

namespace {

thread_local std::string g_last_hip_error;

nr_status hip_fail(hipError_t e, const char* what) {
  g_last_hip_error = std::string(what) + ": " + hipGetErrorString(e);
  return NR_EHIP;
}

// 17-point Gauss-Legendre rule on [-1, 1]: Newton iteration on P_17 from
// Tricomi's asymptotic initial guesses, in long double, weights
// 2 / ((1 - x^2) P'_17(x)^2).  Nodes ascending; the centre node is exactly 0.
void legendre_rule(int n, double* x_out, double* u_out) {
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 1; k <= n; ++k) {
    const long double th = pi * (4.0L * k - 1.0L) / (4.0L * n + 2.0L);
    long double x = (1.0L - (n - 1.0L) / (8.0L * n * n * n)) * std::cos(th);
    long double dp = 0.0L;
    for (int it = 0; it < 60; ++it) {
      long double pm1 = 1.0L, p = x;
      for (int m = 2; m <= n; ++m) {
        const long double pn = ((2.0L * m - 1.0L) * x * p - (m - 1.0L) * pm1) / m;
        pm1 = p;
        p = pn;
      }
      dp = n * (pm1 - x * p) / (1.0L - x * x);
      const long double step = p / dp;
      x -= step;
      if (std::fabs(step) <= 1e-32L) break;
    }
    {
      long double pm1 = 1.0L, p = x;
      for (int m = 2; m <= n; ++m) {
        const long double pn = ((2.0L * m - 1.0L) * x * p - (m - 1.0L) * pm1) / m;
        pm1 = p;
        p = pn;
      }
      dp = n * (pm1 - x * p) / (1.0L - x * x);
    }
    // k = 1 is the largest root
    x_out[n - k] = (double)x;
    u_out[n - k] = (double)(2.0L / ((1.0L - x * x) * dp * dp));
  }
  if (n % 2) x_out[n / 2] = 0.0;
}

// Normalised Gaussian smearing weights over nodes 3.5 x_k (units of sigma_Q).
void smearing_rule(double* t, double* w) {
  double x[kSmearNodes], u[kSmearNodes];
  legendre_rule(kSmearNodes, x, u);
  long double g[kSmearNodes], total = 0.0L;
  for (int k = 0; k < kSmearNodes; ++k) {
    t[k] = 3.5 * x[k];
    const long double tk = t[k];
    g[k] = (long double)u[k] * std::exp(-tk * tk / 2.0L);
    total += g[k];
  }
  for (int k = 0; k < kSmearNodes; ++k) w[k] = (double)(g[k] / total);
}

// Tables for the device exp and sincos, correctly rounded from long double:
// (sin, cos)(k pi/32) for k = 0..63, interleaved, then 2^(j/64) for j = 0..63.
void append_math_tables(std::vector<double>& v) {
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 0; k < 64; ++k) {
    v.push_back((double)std::sin(pi * k / 32.0L));
    v.push_back((double)std::cos(pi * k / 32.0L));
  }
  for (int j = 0; j < 64; ++j) v.push_back((double)std::exp2((long double)j / 64.0L));
}

struct Launch {
  int bucket = 0;
  int n_wu = 0;
  int32_t* item = nullptr;
  int32_t* p0 = nullptr;
  int64_t* rec_grad = nullptr;
  int64_t* rec_ll = nullptr;
};

template <class T>
hipError_t upload(T** dst, const std::vector<T>& src) {
  *dst = nullptr;
  if (src.empty()) return hipSuccess;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), src.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

}  // namespace

struct nr_plan {
  int device = 0;
  int32_t n_datasets = 0, n_items = 0, precision = NR_F64;
  std::vector<int64_t> q_off, row_off, out_off;
  std::vector<int32_t> dataset_of_item;
  std::vector<double> dqq;
  int64_t n_wu_total = 0, rec_grad_total = 0;
  // device copies
  int32_t* d_dataset_of_item = nullptr;
  int64_t* d_q_off = nullptr;
  int64_t* d_row_off = nullptr;
  double* d_dqq = nullptr;
  int64_t* d_out_off = nullptr;
  int64_t* d_item_wu_first = nullptr;
  int32_t* d_item_wu_count = nullptr;
  int64_t* d_rec_of_wu_grad = nullptr;
  int64_t* d_rec_of_wu_ll = nullptr;
  double* d_rule = nullptr;
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
  std::vector<Launch> launches;
  double node_t[kSmearNodes], node_w[kSmearNodes];
  std::vector<void*> owned;
};

namespace {

void plan_free(nr_plan* p) {
  for (void* ptr : p->owned)
    if (ptr) (void)hipFree(ptr);
  p->owned.clear();
}

nr_status validate_desc(const nr_batch_desc* d) {
  if (!d) return NR_EINVAL;
  if (d->n_datasets < 0 || d->n_items < 0) return NR_EINVAL;
  if (d->precision != NR_F64 && d->precision != NR_F32) return NR_EINVAL;
  if (!d->q_off || !d->row_off) return NR_EINVAL;
  if (d->n_datasets > 0 && !d->dq_over_q) return NR_EINVAL;
  if (d->n_items > 0 && !d->dataset_of_item) return NR_EINVAL;
  if (d->q_off[0] != 0 || d->row_off[0] != 0) return NR_EINVAL;
  for (int s = 0; s < d->n_datasets; ++s) {
    if (d->q_off[s + 1] < d->q_off[s]) return NR_EINVAL;
    if (d->q_off[s + 1] - d->q_off[s] > (int64_t)INT32_MAX) return NR_EINVAL;
    const double r = d->dq_over_q[s];
    if (!(r >= 0.0) || !std::isfinite(r)) return NR_EINVAL;
  }
  for (int b = 0; b < d->n_items; ++b) {
    const int64_t rows = d->row_off[b + 1] - d->row_off[b];
    if (rows < 2 || rows > NR_MAX_LAYERS + 2) return NR_EINVAL;
    const int32_t s = d->dataset_of_item[b];
    if (s < 0 || s >= d->n_datasets) return NR_EINVAL;
  }
  return NR_OK;
}

nr_status check_call(const nr_plan* p, const nr_values* v, bool need_data) {
  if (!p || !v) return NR_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device) return NR_EINVAL;
  if (p->n_items == 0) return NR_OK;
  if (!v->layers || !v->scale || !v->bkg) return NR_EINVAL;
  if (p->q_off.back() > 0) {
    if (!v->q) return NR_EINVAL;
    if (need_data && (!v->r_obs || !v->r_err)) return NR_EINVAL;
  }
  return NR_OK;
}

KernelArgs base_args(const nr_plan* p, const nr_values* v) {
  KernelArgs a;
  std::memset(&a, 0, sizeof(a));
  a.dataset_of_item = p->d_dataset_of_item;
  a.q_off = p->d_q_off;
  a.row_off = p->d_row_off;
  a.dq_over_q = p->d_dqq;
  a.out_off = p->d_out_off;
  a.q = v->q;
  a.r_obs = v->r_obs;
  a.r_err = v->r_err;
  a.layers = v->layers;
  a.scale = v->scale;
  a.bkg = v->bkg;
  a.item_status = v->item_status;
  a.rule = p->d_rule;
  return a;
}

nr_status run_launches(const nr_plan* p, int op, KernelArgs a, hipStream_t st) {
  if (p->ev_start) {
    hipError_t e = hipEventRecord(p->ev_start, st);
    if (e != hipSuccess) return hip_fail(e, "timing event");
  }
  for (const Launch& L : p->launches) {
    a.wu_item = L.item;
    a.wu_p0 = L.p0;
    a.wu_rec = (op == kOpLoglikGrad) ? L.rec_grad : L.rec_ll;
    hipError_t e = (op == kOpLoglikGrad) ? launch_grad(L.bucket, a, L.n_wu, st)
                                         : launch_forward(op, a, L.n_wu, st);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
  }
  if (p->ev_stop) {
    hipError_t e = hipEventRecord(p->ev_stop, st);
    if (e != hipSuccess) return hip_fail(e, "timing event");
  }
  return NR_OK;
}

}  // namespace

extern "C" {

int32_t nr_version(void) { return NR_VERSION; }

const char* nr_status_string(nr_status s) {
  switch (s) {
    case NR_OK:
      return "ok";
    case NR_EINVAL:
      return "invalid argument";
    case NR_EWORKSPACE:
      return "workspace missing or too small";
    case NR_EHIP:
      return g_last_hip_error.empty() ? "HIP error" : g_last_hip_error.c_str();
    case NR_ENOMEM:
      return "device allocation failed";
    default:
      return "unknown status";
  }
}

nr_status nr_plan_create(const nr_batch_desc* d, nr_plan** out) {
  if (!out) return NR_EINVAL;
  *out = nullptr;
  nr_status st = validate_desc(d);
  if (st != NR_OK) return st;
  nr_plan* p = new nr_plan();
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return NR_EHIP;
  }
  p->n_datasets = d->n_datasets;
  p->n_items = d->n_items;
  p->precision = d->precision;
  p->q_off.assign(d->q_off, d->q_off + d->n_datasets + 1);
  p->row_off.assign(d->row_off, d->row_off + d->n_items + 1);
  p->dataset_of_item.assign(d->dataset_of_item, d->dataset_of_item + d->n_items);
  p->dqq.assign(d->dq_over_q, d->dq_over_q + d->n_datasets);
  smearing_rule(p->node_t, p->node_w);

  // work units, item-major numbering
  const int nI = d->n_items;
  std::vector<int64_t> item_wu_first(nI), rec_of_wu_grad, rec_of_wu_ll;
  std::vector<int32_t> item_wu_count(nI);
  p->out_off.assign(nI + 1, 0);
  struct Wu {
    int32_t item, p0;
    int64_t g;
    double cost;
  };
  std::vector<std::vector<Wu>> per_bucket(kNumBuckets);
  int64_t g = 0, rec = 0;
  for (int b = 0; b < nI; ++b) {
    const int s = p->dataset_of_item[b];
    const int64_t nq = p->q_off[s + 1] - p->q_off[s];
    const int N = (int)(p->row_off[b + 1] - p->row_off[b]) - 2;
    const int K = p->dqq[s] > 0.0 ? kSmearNodes : 1;
    const int nwu = (int)((nq + kWuPoints - 1) / kWuPoints);
    const int bk = bucket_of(N);
    item_wu_first[b] = g;
    item_wu_count[b] = nwu;
    p->out_off[b + 1] = p->out_off[b] + nq;
    for (int k = 0; k < nwu; ++k) {
      const int p0 = k * kWuPoints;
      const double pts = (double)std::min<int64_t>(kWuPoints, nq - p0);
      per_bucket[bk].push_back({b, p0, g, pts * K * (N + 1)});
      rec_of_wu_grad.push_back(rec);
      rec_of_wu_ll.push_back(g);
      rec += 3 + 4 * (N + 2);
      ++g;
    }
  }
  p->n_wu_total = g;
  p->rec_grad_total = rec;

  hipError_t e = hipSuccess;
  auto keep = [&](void* ptr) { p->owned.push_back(ptr); };
  e = upload(&p->d_dataset_of_item, p->dataset_of_item);
  keep(p->d_dataset_of_item);
  if (e == hipSuccess) { e = upload(&p->d_q_off, p->q_off); keep(p->d_q_off); }
  if (e == hipSuccess) { e = upload(&p->d_row_off, p->row_off); keep(p->d_row_off); }
  if (e == hipSuccess) { e = upload(&p->d_dqq, p->dqq); keep(p->d_dqq); }
  if (e == hipSuccess) { e = upload(&p->d_out_off, p->out_off); keep(p->d_out_off); }
  if (e == hipSuccess) { e = upload(&p->d_item_wu_first, item_wu_first); keep(p->d_item_wu_first); }
  if (e == hipSuccess) { e = upload(&p->d_item_wu_count, item_wu_count); keep(p->d_item_wu_count); }
  if (e == hipSuccess) { e = upload(&p->d_rec_of_wu_grad, rec_of_wu_grad); keep(p->d_rec_of_wu_grad); }
  if (e == hipSuccess) { e = upload(&p->d_rec_of_wu_ll, rec_of_wu_ll); keep(p->d_rec_of_wu_ll); }
  if (e == hipSuccess) {
    std::vector<double> rule(p->node_t, p->node_t + kSmearNodes);
    rule.insert(rule.end(), p->node_w, p->node_w + kSmearNodes);
    append_math_tables(rule);
    e = upload(&p->d_rule, rule);
    keep(p->d_rule);
  }

  // one launch per non-empty bucket, heaviest buckets first, LPT order inside
  std::vector<int> order;
  for (int bk = 0; bk < kNumBuckets; ++bk)
    if (!per_bucket[bk].empty()) order.push_back(bk);
  std::sort(order.begin(), order.end(), [](int x, int y) { return x > y; });
  for (int bk : order) {
    if (e != hipSuccess) break;
    auto& v = per_bucket[bk];
    std::stable_sort(v.begin(), v.end(), [](const Wu& x, const Wu& y) { return x.cost > y.cost; });
    std::vector<int32_t> it(v.size()), p0(v.size());
    std::vector<int64_t> rg(v.size()), rl(v.size());
    for (size_t k = 0; k < v.size(); ++k) {
      it[k] = v[k].item;
      p0[k] = v[k].p0;
      rg[k] = rec_of_wu_grad[v[k].g];
      rl[k] = rec_of_wu_ll[v[k].g];
    }
    Launch L;
    L.bucket = bk;
    L.n_wu = (int)v.size();
    e = upload(&L.item, it);
    keep(L.item);
    if (e == hipSuccess) { e = upload(&L.p0, p0); keep(L.p0); }
    if (e == hipSuccess) { e = upload(&L.rec_grad, rg); keep(L.rec_grad); }
    if (e == hipSuccess) { e = upload(&L.rec_ll, rl); keep(L.rec_ll); }
    p->launches.push_back(L);
  }
  if (e != hipSuccess) {
    plan_free(p);
    delete p;
    g_last_hip_error = std::string("plan upload: ") + hipGetErrorString(e);
    return (e == hipErrorOutOfMemory) ? NR_ENOMEM : NR_EHIP;
  }
  *out = p;
  return NR_OK;
}

nr_status nr_plan_set_timing_events(nr_plan* p, void* start, void* stop) {
  if (!p || ((start == nullptr) != (stop == nullptr))) return NR_EINVAL;
  p->ev_start = static_cast<hipEvent_t>(start);
  p->ev_stop = static_cast<hipEvent_t>(stop);
  return NR_OK;
}

nr_status nr_plan_destroy(nr_plan* p) {
  if (!p) return NR_OK;
  plan_free(p);
  delete p;
  return NR_OK;
}

nr_status nr_workspace_size(const nr_plan* p, int32_t op, size_t* bytes) {
  if (!p || !bytes) return NR_EINVAL;
  switch (op) {
    case NR_OP_REFLECTIVITY:
      *bytes = 0;
      return NR_OK;
    case NR_OP_LOGLIK:
      *bytes = sizeof(double) * (size_t)p->n_wu_total;
      return NR_OK;
    case NR_OP_LOGLIK_GRAD:
      *bytes = sizeof(double) * (size_t)p->rec_grad_total;
      return NR_OK;
    default:
      return NR_EINVAL;
  }
}

nr_status nr_output_offsets(const nr_plan* p, int64_t* out_off) {
  if (!p || !out_off) return NR_EINVAL;
  std::memcpy(out_off, p->out_off.data(), sizeof(int64_t) * p->out_off.size());
  return NR_OK;
}

nr_status nr_reflectivity(const nr_plan* p, const nr_values* v, double* r_hat, void* ws,
                          size_t ws_bytes, void* stream) {
  (void)ws;
  (void)ws_bytes;
  nr_status st = check_call(p, v, false);
  if (st != NR_OK) return st;
  if (p->n_items == 0 || p->out_off.back() == 0) return NR_OK;
  if (!r_hat) return NR_EINVAL;
  KernelArgs a = base_args(p, v);
  a.out = r_hat;
  return run_launches(p, kOpReflectivity, a, (hipStream_t)stream);
}

nr_status nr_loglik(const nr_plan* p, const nr_values* v, double* logL, void* ws,
                    size_t ws_bytes, void* stream) {
  nr_status st = check_call(p, v, true);
  if (st != NR_OK) return st;
  if (p->n_items == 0) return NR_OK;
  if (!logL) return NR_EINVAL;
  const size_t need = sizeof(double) * (size_t)p->n_wu_total;
  if (need > 0 && (!ws || ws_bytes < need)) return NR_EWORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  KernelArgs a = base_args(p, v);
  a.rec = static_cast<double*>(ws);
  st = run_launches(p, kOpLoglik, a, s);
  if (st != NR_OK) return st;
  ReduceArgs r;
  std::memset(&r, 0, sizeof(r));
  r.n_items = p->n_items;
  r.item_wu_first = p->d_item_wu_first;
  r.item_wu_count = p->d_item_wu_count;
  r.rec_of_wu = p->d_rec_of_wu_ll;
  r.rec = static_cast<double*>(ws);
  r.logL = logL;
  hipError_t e = launch_reduce(kOpLoglik, r, s);
  return e == hipSuccess ? NR_OK : hip_fail(e, "reduce launch");
}

nr_status nr_loglik_grad(const nr_plan* p, const nr_values* v, double* logL, double* g_rows,
                         double* g_inst, void* ws, size_t ws_bytes, void* stream) {
  nr_status st = check_call(p, v, true);
  if (st != NR_OK) return st;
  if (p->n_items == 0) return NR_OK;
  if (!logL || !g_rows || !g_inst) return NR_EINVAL;
  const size_t need = sizeof(double) * (size_t)p->rec_grad_total;
  if (need > 0 && (!ws || ws_bytes < need)) return NR_EWORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  KernelArgs a = base_args(p, v);
  a.rec = static_cast<double*>(ws);
  st = run_launches(p, kOpLoglikGrad, a, s);
  if (st != NR_OK) return st;
  ReduceArgs r;
  std::memset(&r, 0, sizeof(r));
  r.n_items = p->n_items;
  r.item_wu_first = p->d_item_wu_first;
  r.item_wu_count = p->d_item_wu_count;
  r.rec_of_wu = p->d_rec_of_wu_grad;
  r.rec = static_cast<double*>(ws);
  r.row_off = p->d_row_off;
  r.layers = v->layers;
  r.logL = logL;
  r.g_rows = g_rows;
  r.g_inst = g_inst;
  hipError_t e = launch_reduce(kOpLoglikGrad, r, s);
  return e == hipSuccess ? NR_OK : hip_fail(e, "reduce launch");
}

}  // extern "C"
