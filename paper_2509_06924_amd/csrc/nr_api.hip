// C ABI of the reflectivity log-likelihood library: argument validation, plan
// construction (work list, record offsets, quadrature rule) and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
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

// Workspace of nr_loglik_grad_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends.  Host code must not pass the array's
// name to a kernel or a copy (on the host it is only a stand-in symbol): the
// device address of each GPU's copy is looked up once, with that GPU
// current, and kept in scratch_addr.  Every call on one GPU shares its copy.
__device__ __align__(256) unsigned char scratch[NR_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// The device address of `dev`'s scratch copy (dev must be current).
nr_status scratch_addr(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return NR_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "scratch symbol address");
    g_scratch_addr[dev] = ptr;
  }
  *out = g_scratch_addr[dev];
  return NR_OK;
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
// (sin, cos)(k pi/64) for k = 0..127, interleaved, then 2^(j/64) for j = 0..63.
void append_math_tables(std::vector<double>& v) {
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 0; k < 128; ++k) {
    v.push_back((double)std::sin(pi * k / 64.0L));
    v.push_back((double)std::cos(pi * k / 64.0L));
  }
  for (int j = 0; j < 64; ++j) v.push_back((double)std::exp2((long double)j / 64.0L));
}

// One kernel launch: a work list for one layer-count bucket.  Full units
// cover 64 consecutive points of one item; tail units pack the trailing
// partial groups of several items of equal depth, lane by lane.
struct Launch {
  int bucket = 0;
  bool store = false;  // gradient: store variant (else recompute)
  bool tail = false;
  bool split = false;  // split tail units (one item's partial group, lanes over node groups)
  int scan_ch = 0;     // deep lists: the largest levels-per-lane of its items at 64 lanes
  bool side = false;   // runs on the plan's side stream
  int n_wu = 0;
  int32_t* item = nullptr;      // [n_wu]: the unit's item (first item for tails)
  int32_t* split_code = nullptr;  // [n_wu] split units: points | node groups << 16
  int32_t* p0 = nullptr;        // [n_wu]: first point (full units)
  int64_t* rec = nullptr;       // [n_wu]: record offset (full units)
  int32_t* lane_item = nullptr; // [n_wu * 64] (tail units)
  int32_t* lane_pt = nullptr;   // [n_wu * 64]
  int64_t* lane_rec = nullptr;  // [n_wu * 64], -1 for idle lanes
};

// Per-item lists of record offsets summed by the reduction kernels.
struct RecordLists {
  int64_t* first = nullptr;
  int32_t* count = nullptr;
  int64_t* offs = nullptr;
};

// Workgroups are dispatched to the 8 XCDs round-robin (block b -> XCD b % 8)
// and each XCD has its own L2.  Block b takes entry xcd_order(b, n, run) of
// the cost-sorted unit list: within each chunk of 8 x run blocks, one XCD
// gets a run of `run` consecutive entries (the units of one item are
// consecutive), so an item's layer records are fetched into one L2, while
// the chunks keep the longest-first order.  The last partial chunk maps to
// itself.
constexpr int kXcds = 8;
// deepest bucket whose partial point groups may get a wave of their own
constexpr int kSplitTailMaxLayers = 10;
size_t xcd_order(size_t b, size_t n, size_t run) {
  const size_t chunk = kXcds * run;
  const size_t c0 = (b / chunk) * chunk;
  if (c0 + chunk > n) return b;
  const size_t r = b - c0;
  return c0 + (r % kXcds) * run + r / kXcds;
}

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
  nr_plan_options opts;
  bool bucket_store[kNumBuckets];
  std::vector<int64_t> q_off, row_off, out_off;
  std::vector<int32_t> dataset_of_item;
  std::vector<double> dqq;
  int64_t rec_ll_total = 0, rec_grad_total = 0;
  // device copies
  int32_t* d_dataset_of_item = nullptr;
  int64_t* d_q_off = nullptr;
  int64_t* d_row_off = nullptr;
  double* d_dqq = nullptr;
  int64_t* d_out_off = nullptr;
  RecordLists lists_ll, lists_grad;
  double* d_rule = nullptr;
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
  std::vector<Launch> launches_fwd, launches_grad;
  uint8_t* d_row_kind = nullptr;  // 0 fronting, 1 layer, 2 backing, per row
  int uniform_rows = 0;           // rows per item if all items agree, else 0
  int max_rows = 2;               // rows of the deepest item
  double node_t[kSmearNodes], node_w[kSmearNodes];
  std::vector<void*> owned;
  // second stream for the gradient's tail and split launches (side_stream)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;          // eager calls
  hipEvent_t ev_fork_cap = nullptr, ev_join_cap = nullptr;  // calls under graph capture
  mutable std::mutex side_mu;  // one fork ... join sequence at a time
};

namespace {

void plan_free(nr_plan* p) {
  for (void* ptr : p->owned)
    if (ptr) (void)hipFree(ptr);
  p->owned.clear();
  for (hipEvent_t ev : {p->ev_fork, p->ev_join, p->ev_fork_cap, p->ev_join_cap})
    if (ev) (void)hipEventDestroy(ev);
  if (p->side) (void)hipStreamDestroy(p->side);
  p->ev_fork = p->ev_join = p->ev_fork_cap = p->ev_join_cap = nullptr;
  p->side = nullptr;
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
    if (rows < 2 || rows > NR_MAX_DEEP_LAYERS + 2) return NR_EINVAL;
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
  a.dq = v->dq;
  a.dqq_item = v->dqq_item;
  a.rule = p->d_rule;
  return a;
}

// Workspace layout: per-row layer records (6 doubles per row of every item),
// their float copies (8 floats per row), then the per-work-unit partial
// records of the operation.
size_t consts_doubles(const nr_plan* p) {
  return (size_t)p->row_off.back() * (kRecDoubles + kRecFloats / 2);
}
const float* consts_floats(const nr_plan* p, const double* ws) {
  return reinterpret_cast<const float*>(ws + (size_t)p->row_off.back() * kRecDoubles);
}

size_t op_doubles(const nr_plan* p, int op) {
  size_t n = consts_doubles(p);
  if (op == NR_OP_LOGLIK) n += (size_t)p->rec_ll_total;
  if (op == NR_OP_LOGLIK_GRAD) n += (size_t)p->rec_grad_total;
  return n;
}

nr_status run_launches(const nr_plan* p, int op, KernelArgs a, hipStream_t st,
                       bool events = true, bool res = false);

// res: gradient launches take the form that also yields the derivative with
// respect to the relative resolution.
nr_status run_launches(const nr_plan* p, int op, KernelArgs a, hipStream_t st, bool events,
                       bool res) {
  {
    hipError_t e = launch_item_consts(p->d_row_off, a.layers, const_cast<double*>(a.consts),
                                      const_cast<float*>(a.constsf), p->n_items, st);
    if (e != hipSuccess) return hip_fail(e, "constants launch");
  }
  if (events && p->ev_start) {
    hipError_t e = hipEventRecord(p->ev_start, st);
    if (e != hipSuccess) return hip_fail(e, "timing event");
  }
  const bool grad = (op == kOpLoglikGrad);
  // fork: the side stream waits for the constants (and everything before
  // them on st); join: st waits for the side stream's launches
  const bool fork = grad && p->side != nullptr;
  std::unique_lock<std::mutex> lock;
  // A call being captured into a graph uses an event pair of its own, so that
  // no event object is shared between captured and eager fork/joins.
  hipEvent_t ev_fork = p->ev_fork, ev_join = p->ev_join;
  if (fork) {
    lock = std::unique_lock<std::mutex>(p->side_mu);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(st, &cs);
    if (e == hipSuccess && cs != hipStreamCaptureStatusNone) {
      ev_fork = p->ev_fork_cap;
      ev_join = p->ev_join_cap;
    }
    if (e == hipSuccess) e = hipEventRecord(ev_fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->side, ev_fork, 0);
    if (e != hipSuccess) return hip_fail(e, "side stream fork");
  }
  hipError_t launch_err = hipSuccess;
  for (const Launch& L : grad ? p->launches_grad : p->launches_fwd) {
    a.wu_item = L.item;
    a.wu_p0 = L.p0;
    a.wu_rec = L.rec;
    a.wu_split = L.split_code;
    a.tail_item = L.lane_item;
    a.tail_pt = L.lane_pt;
    a.tail_rec = L.lane_rec;
    const int form = res ? kFormRecomputeRes : L.store ? kFormStore : kFormRecompute;
    const int mode = L.tail ? kModeTail : L.split ? kModeSplit : kModeFull;
    const hipStream_t ls = (fork && L.side) ? p->side : st;
    if (!grad)
      launch_err = launch_forward(p->precision, op, L.split, a, L.n_wu, ls);
    else if (L.bucket == kDeepBucket)
      launch_err = launch_grad_scan(res, L.scan_ch, a, L.n_wu, ls);
    else
      launch_err = launch_grad(p->precision, L.bucket, form, mode, a, L.n_wu, ls);
    if (launch_err != hipSuccess) break;
  }
  if (fork) {
    // joined even after a failed launch, so that a capture stays well formed
    hipError_t e = hipEventRecord(ev_join, p->side);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ev_join, 0);
    if (e != hipSuccess && launch_err == hipSuccess) return hip_fail(e, "side stream join");
  }
  if (launch_err != hipSuccess) return hip_fail(launch_err, "kernel launch");
  if (events && p->ev_stop) {
    hipError_t e = hipEventRecord(p->ev_stop, st);
    if (e != hipSuccess) return hip_fail(e, "timing event");
  }
  return NR_OK;
}

// Enqueues the whole logL + gradient evaluation (validated arguments); with
// seed set, the vector-Jacobian product of R_hat instead.
nr_status enqueue_grad(const nr_plan* p, const nr_values* v, double* logL, double* g_rows,
                       double* g_inst, void* ws, hipStream_t s, bool events,
                       const double* seed = nullptr, double* g_res = nullptr) {
  KernelArgs a = base_args(p, v);
  a.seed = seed;
  a.consts = static_cast<double*>(ws);
  a.constsf = consts_floats(p, a.consts);
  a.rec = static_cast<double*>(ws) + consts_doubles(p);
  nr_status st = run_launches(p, kOpLoglikGrad, a, s, events, g_res != nullptr);
  if (st != NR_OK) return st;
  ReduceArgs r;
  std::memset(&r, 0, sizeof(r));
  r.n_items = p->n_items;
  r.item_wu_first = p->lists_grad.first;
  r.item_wu_count = p->lists_grad.count;
  r.rec_of_wu = p->lists_grad.offs;
  r.rec = a.rec;
  r.row_off = p->d_row_off;
  r.layers = v->layers;
  r.logL = logL;
  r.g_rows = g_rows;
  r.g_inst = g_inst;
  r.g_res = g_res;
  r.max_rows = p->max_rows;
  hipError_t e = launch_reduce(kOpLoglikGrad, r, s);
  return e == hipSuccess ? NR_OK : hip_fail(e, "reduce launch");
}

nr_status check_hmc(const nr_plan* p, const nr_values* data, const nr_hmc_state* st, double dt,
                    int32_t n_steps, void* ws, size_t ws_bytes) {
  if (!p || !data || !st || n_steps < 0 || !std::isfinite(dt)) return NR_EINVAL;
  nr_values v = *data;
  v.layers = st->layers;
  v.scale = st->scale;
  v.bkg = st->bkg;
  nr_status s = check_call(p, &v, true);
  if (s != NR_OK) return s;
  if (p->n_items == 0) return NR_OK;
  if (!st->mom_rows || !st->mom_inst || !st->logL || !st->g_rows || !st->g_inst)
    return NR_EINVAL;
  const size_t need = sizeof(double) * op_doubles(p, NR_OP_LOGLIK_GRAD);
  if (need > 0 && (!ws || ws_bytes < need)) return NR_EWORKSPACE;
  return NR_OK;
}

nr_status enqueue_leapfrog(const nr_plan* p, const nr_values* data, const nr_hmc_state* st,
                           double dt, int32_t n_steps, void* ws, hipStream_t s, bool events) {
  if (p->n_items == 0) return NR_OK;
  nr_values v = *data;
  v.layers = st->layers;
  v.scale = st->scale;
  v.bkg = st->bkg;
  const int64_t nre = p->row_off.back() * 4;
  const int64_t ni = p->n_items;
  for (int32_t k = 0; k < n_steps; ++k) {
    hipError_t e = launch_kick(nre, 2 * ni, st->mom_rows, st->g_rows, st->mom_inst, st->g_inst,
                               0.5 * dt, s);
    if (e != hipSuccess) return hip_fail(e, "kick launch");
    e = launch_drift(nre, ni, p->d_row_kind, st->layers, st->scale, st->bkg, st->mom_rows,
                     st->mom_inst, st->inv_mass_rows, st->inv_mass_inst, dt, s);
    if (e != hipSuccess) return hip_fail(e, "drift launch");
    nr_status r = enqueue_grad(p, &v, st->logL, st->g_rows, st->g_inst, ws, s, events);
    if (r != NR_OK) return r;
    e = launch_kick(nre, 2 * ni, st->mom_rows, st->g_rows, st->mom_inst, st->g_inst, 0.5 * dt, s);
    if (e != hipSuccess) return hip_fail(e, "kick launch");
  }
  return NR_OK;
}

}  // namespace

struct nr_graph {
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct nr_hmc {
  const nr_plan* plan = nullptr;
  nr_hmc_config cfg;
  int64_t n_entries = 0;  // 4 x rows + 2 x items
  double* buf = nullptr;  // r, z0, g0, wmean, wm2 (n_entries each), then the chain scalars
  uint64_t* iter = nullptr;
};

namespace {

bool chains_complete(const nr_hmc_chains* ch) {
  const void* need[] = {ch->z_rows, ch->z_inst, ch->kind_rows, ch->kind_inst, ch->a_rows,
                        ch->b_rows, ch->a_inst, ch->b_inst, ch->inv_mass_rows,
                        ch->inv_mass_inst, ch->step, ch->layers, ch->scale, ch->bkg,
                        ch->logL, ch->g_rows, ch->g_inst, ch->potential, ch->accept_prob,
                        ch->energy_error, ch->n_accept, ch->n_divergent};
  for (const void* q : need)
    if (!q) return false;
  return true;
}

nr_status check_chains(const nr_hmc* h, const nr_values* data, const nr_hmc_chains* ch, void* ws,
                       size_t ws_bytes) {
  if (!h || !data || !ch) return NR_EINVAL;
  nr_values v = *data;
  v.layers = ch->layers;
  v.scale = ch->scale;
  v.bkg = ch->bkg;
  nr_status s = check_call(h->plan, &v, true);
  if (s != NR_OK) return s;
  if (h->plan->n_items == 0) return NR_OK;
  if (!chains_complete(ch)) return NR_EINVAL;
  const size_t bytes = sizeof(double) * op_doubles(h->plan, NR_OP_LOGLIK_GRAD);
  if (bytes > 0 && (!ws || ws_bytes < bytes)) return NR_EWORKSPACE;
  return NR_OK;
}

HmcArgs hmc_args(const nr_hmc* h, const nr_hmc_chains* ch) {
  const nr_plan* p = h->plan;
  HmcArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n_items = p->n_items;
  a.n_row_entries = p->row_off.back() * 4;
  a.row_off = p->d_row_off;
  a.row_kind = p->d_row_kind;
  a.z_rows = ch->z_rows;
  a.z_inst = ch->z_inst;
  a.kind_rows = ch->kind_rows;
  a.kind_inst = ch->kind_inst;
  a.a_rows = ch->a_rows;
  a.b_rows = ch->b_rows;
  a.a_inst = ch->a_inst;
  a.b_inst = ch->b_inst;
  a.im_rows = ch->inv_mass_rows;
  a.im_inst = ch->inv_mass_inst;
  a.step = ch->step;
  a.layers = ch->layers;
  a.scale = ch->scale;
  a.bkg = ch->bkg;
  a.logL = ch->logL;
  a.g_rows = ch->g_rows;
  a.g_inst = ch->g_inst;
  a.U = ch->potential;
  a.accept_prob = ch->accept_prob;
  a.energy_error = ch->energy_error;
  a.n_accept = ch->n_accept;
  a.n_divergent = ch->n_divergent;
  const int64_t n = h->n_entries;
  a.r = h->buf;
  a.z0 = h->buf + n;
  a.g0 = h->buf + 2 * n;
  a.wmean = h->buf + 3 * n;
  a.wm2 = h->buf + 4 * n;
  a.cs = h->buf + 5 * n;
  a.iter = h->iter;
  a.seed = h->cfg.seed;
  a.max_energy_error = h->cfg.max_energy_error;
  a.target_accept = h->cfg.target_accept;
  return a;
}

}  // namespace

struct nr_vi_mvn {
  const nr_plan* plan = nullptr;
  nr_vi_mvn_config cfg;
  int32_t P = 0, rows = 0;
  double* buf = nullptr;  // eps, z, h, f, layers, scale, bkg, logL, g_rows, g_inst, adam m, v
  uint64_t* iter = nullptr;
  MvnArgs args;           // driver-owned pointers and configuration
};

namespace {

nr_status check_mvn(const nr_vi_mvn* m, const nr_values* data, const nr_vi_mvn_params* prm,
                    void* ws, size_t ws_bytes) {
  if (!m || !data || !prm) return NR_EINVAL;
  const void* need[] = {prm->kind, prm->a, prm->b, prm->theta_fixed, prm->mu, prm->omega,
                        prm->lam, prm->elbo, prm->grad_mu, prm->grad_omega, prm->grad_lam};
  for (const void* q : need)
    if (!q) return NR_EINVAL;
  nr_values v = *data;
  v.layers = m->args.layers;
  v.scale = m->args.scale;
  v.bkg = m->args.bkg;
  nr_status s = check_call(m->plan, &v, true);
  if (s != NR_OK) return s;
  const size_t bytes = sizeof(double) * op_doubles(m->plan, NR_OP_LOGLIK_GRAD);
  if (bytes > 0 && (!ws || ws_bytes < bytes)) return NR_EWORKSPACE;
  return NR_OK;
}

MvnArgs mvn_args(const nr_vi_mvn* m, const nr_vi_mvn_params* prm) {
  MvnArgs a = m->args;
  a.kind = prm->kind;
  a.a = prm->a;
  a.b = prm->b;
  a.theta_fixed = prm->theta_fixed;
  a.mu = prm->mu;
  a.omega = prm->omega;
  a.lam = prm->lam;
  a.grad_mu = prm->grad_mu;
  a.grad_omega = prm->grad_omega;
  a.grad_lam = prm->grad_lam;
  a.elbo = prm->elbo;
  return a;
}

// One step: draws, logL + gradient of every draw, the z-gradients, the
// per-restart ELBO and gradient, Adam (optional), the iteration tick.
nr_status enqueue_mvn_step(const nr_vi_mvn* m, const nr_values* data,
                           const nr_vi_mvn_params* prm, bool adam, void* ws, hipStream_t s,
                           bool events) {
  const MvnArgs a = mvn_args(m, prm);
  nr_values v = *data;
  v.layers = a.layers;
  v.scale = a.scale;
  v.bkg = a.bkg;
  hipError_t e = launch_mvn(kMvnSample, a, s);
  if (e != hipSuccess) return hip_fail(e, "mvn sample");
  nr_status r = enqueue_grad(m->plan, &v, a.logL, a.g_rows, a.g_inst, ws, s, events);
  if (r != NR_OK) return r;
  e = launch_mvn(kMvnChain, a, s);
  if (e == hipSuccess) e = launch_mvn(kMvnReduce, a, s);
  if (e == hipSuccess && adam) e = launch_mvn(kMvnAdam, a, s);
  if (e == hipSuccess) e = launch_mvn(kMvnTick, a, s);
  return e == hipSuccess ? NR_OK : hip_fail(e, "mvn launch");
}

nr_values chain_values(const nr_values* data, const nr_hmc_chains* ch) {
  nr_values v = *data;
  v.layers = ch->layers;
  v.scale = ch->scale;
  v.bkg = ch->bkg;
  return v;
}

// One transition (Sec. 2.3): begin (momentum, first half kick), then per
// leapfrog step drift, logL + gradient, kick (a full kick where two half
// kicks meet), then the accept.
nr_status enqueue_transition(const nr_hmc* h, const nr_values* data, const nr_hmc_chains* ch,
                             int32_t adapt, void* ws, hipStream_t s, bool events) {
  const nr_plan* p = h->plan;
  if (p->n_items == 0) return NR_OK;
  const HmcArgs a = hmc_args(h, ch);
  const nr_values v = chain_values(data, ch);
  hipError_t e = launch_hmc(kHmcBegin, a, 0, 0.0, s);
  if (e != hipSuccess) return hip_fail(e, "hmc begin");
  const int L = h->cfg.n_leapfrog;
  for (int k = 0; k < L; ++k) {
    e = launch_hmc(kHmcDrift, a, 0, 0.0, s);
    if (e != hipSuccess) return hip_fail(e, "hmc drift");
    nr_status r = enqueue_grad(p, &v, ch->logL, ch->g_rows, ch->g_inst, ws, s, events);
    if (r != NR_OK) return r;
    e = launch_hmc(kHmcKick, a, 0, (k + 1 < L) ? 1.0 : 0.5, s);
    if (e != hipSuccess) return hip_fail(e, "hmc kick");
  }
  e = launch_hmc(kHmcEnd, a, adapt, 0.0, s);
  return e == hipSuccess ? NR_OK : hip_fail(e, "hmc end");
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
    case NR_ESCRATCH:
      return "the plan's workspace exceeds the fixed scratch of nr_loglik_grad_noalloc "
             "(NR_NOALLOC_SCRATCH_BYTES); use nr_loglik_grad with a workspace";
    default:
      return "unknown status";
  }
}

nr_status nr_smearing_rule(double* t, double* w) {
  if (!t || !w) return NR_EINVAL;
  smearing_rule(t, w);
  return NR_OK;
}

nr_status nr_plan_options_default(nr_plan_options* o) {
  if (!o) return NR_EINVAL;
  for (int k = 0; k < NR_NUM_BUCKETS; ++k) o->grad_variant[k] = NR_VARIANT_AUTO;
  o->xcd_run = 8;
  o->pack_tails = 1;
  o->split_tails = NR_TAILS_LONE | NR_TAILS_SPLIT | NR_SPLIT_SMALL;
  o->side_stream = 1;
  o->node_groups = 0;
  return NR_OK;
}

int32_t nr_bucket_lmax(int32_t k) { return (k < 0 || k >= kNumBuckets) ? -1 : kBucketLmax[k]; }

int32_t nr_store_max_layers(int32_t precision) {
  if (precision != NR_F64 && precision != NR_F32) return -1;
  return store_max_layers(precision);
}

nr_status nr_plan_create(const nr_batch_desc* d, nr_plan** out) {
  return nr_plan_create_ex(d, nullptr, out);
}

nr_status nr_plan_create_ex(const nr_batch_desc* d, const nr_plan_options* opts, nr_plan** out) {
  if (!out) return NR_EINVAL;
  *out = nullptr;
  nr_status st = validate_desc(d);
  if (st != NR_OK) return st;
  nr_plan_options o;
  nr_plan_options_default(&o);
  if (opts) o = *opts;
  if (o.xcd_run < 1 || o.xcd_run > 64 || (o.pack_tails != 0 && o.pack_tails != 1) ||
      (o.split_tails & ~(NR_TAILS_LONE | NR_TAILS_SPLIT | NR_SPLIT_SMALL)) ||
      (o.side_stream != 0 && o.side_stream != 1) ||
      !(o.node_groups == 0 || (o.node_groups >= 2 && o.node_groups <= kSmearNodes)))
    return NR_EINVAL;
  bool bucket_store[kNumBuckets];
  for (int k = 0; k < kNumBuckets; ++k) {
    const int v = o.grad_variant[k];
    const bool can_store = kBucketLmax[k] <= store_max_layers(d->precision);
    if (v == NR_VARIANT_AUTO) {
      bucket_store[k] = kBucketLmax[k] <= default_store_layers(d->precision);
    } else if (v == NR_VARIANT_STORE) {
      if (!can_store) return NR_EINVAL;
      bucket_store[k] = true;
    } else if (v == NR_VARIANT_RECOMPUTE) {
      bucket_store[k] = false;
    } else {
      return NR_EINVAL;
    }
  }
  nr_plan* p = new nr_plan();
  p->opts = o;
  for (int k = 0; k < kNumBuckets; ++k) p->bucket_store[k] = bucket_store[k];
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

  // ---- work lists -------------------------------------------------------
  // Forward ops: one unit per item x 64 points (the last may be partial),
  // one record (a logL partial) per unit.  Gradient op: full units as above
  // plus tail units that pack the trailing partial groups of items with the
  // same depth and node count; a full unit writes one record, and so does
  // each item's group of lanes in a tail unit.  Every item's records are
  // listed contiguously.
  const int nI = d->n_items;
  p->out_off.assign(nI + 1, 0);
  struct Wu {
    int32_t item, p0;
    int64_t rec;
    double cost;
    int32_t split = 0;  // split tail units: points | node groups << 16
  };
  struct Tail {
    int32_t item, p0, count;
    int64_t rec0;  // record of its first point
  };
  // one list per bucket, then the deep lists: forward one (kDeepBucket),
  // gradient three (kDeepBucket + c), by the levels per lane an item needs at
  // 64 lanes (c = 0: up to 8, 1: up to 16, 2: more), which set the waves per
  // data point of the scan kernel (1, 2, 4), so that shallower deep items do
  // not run with the idle lanes of the deepest one
  constexpr int kDeepClasses = 3;
  std::vector<std::vector<Wu>> fwd_units(kNumBuckets + 1);
  std::vector<std::vector<Wu>> grad_units(kNumBuckets + kDeepClasses);
  std::vector<std::vector<Wu>> split_units(kNumBuckets), fwd_split_units(kNumBuckets);
  int scan_ch[kDeepClasses] = {0, 0, 0};
  std::map<std::pair<int, int>, std::vector<Tail>> tails;  // (depth, nodes)
  std::vector<int64_t> ll_first(nI), ll_offs, gr_first(nI), gr_offs;
  std::vector<int32_t> ll_count(nI), gr_count(nI);
  int64_t rec_ll = 0, rec_gr = 0;
  // Small problems (NR_SPLIT_SMALL): fewer full units than one round of the
  // device leave most of it idle for the whole call, each wave running all 17
  // nodes of its points; splitting the nodes of every point group over G
  // lanes gives G times the waves, each running 17 / G nodes.
  // The value kernels (nr_loglik, nr_reflectivity) take the same split, with
  // their own unit count (deep items included: they have no scan form).
  int small_G = 1, small_G_fwd = 1;
  if (p->opts.split_tails & NR_SPLIT_SMALL) {
    int64_t units = 0, units_fwd = 0;
    for (int b = 0; b < nI; ++b) {
      const int s = p->dataset_of_item[b];
      const int N = (int)(p->row_off[b + 1] - p->row_off[b]) - 2;
      const int64_t u = (p->q_off[s + 1] - p->q_off[s] + kWuPoints - 1) / kWuPoints;
      units_fwd += u;
      if (bucket_of(N) != kDeepBucket) units += u;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) !=
        hipSuccess)
      cus = 0;
    const int64_t round = 2 * 4 * (int64_t)cus;
    if (units > 0 && units < round)
      small_G = (int)std::min<int64_t>(kSmearNodes, round / units);
    if (units_fwd > 0 && units_fwd < round)
      small_G_fwd = (int)std::min<int64_t>(kSmearNodes, round / units_fwd);
  }
  // a tiling given by the caller: every point group split over node_groups
  if (p->opts.node_groups >= 2) small_G = p->opts.node_groups;
  for (int b = 0; b < nI; ++b) {
    const int s = p->dataset_of_item[b];
    const int64_t nq = p->q_off[s + 1] - p->q_off[s];
    const int N = (int)(p->row_off[b + 1] - p->row_off[b]) - 2;
    const int K = p->dqq[s] > 0.0 ? kSmearNodes : 1;
    const int bk = bucket_of(N);
    const int64_t rsz = 4 + 4 * (N + 2);
    p->out_off[b + 1] = p->out_off[b] + nq;
    ll_first[b] = (int64_t)ll_offs.size();
    if (K > 1 && small_G_fwd >= 2) {
      // value units split like the gradient's (lane = g npts + p)
      const int npts = kWuPoints / small_G_fwd;
      int32_t cnt = 0;
      for (int64_t p0 = 0; p0 < nq; p0 += npts) {
        const int np = (int)std::min<int64_t>(npts, nq - p0);
        Wu u{b, (int32_t)p0, rec_ll, (double)np * K * (N + 1)};
        u.split = np | (small_G_fwd << 16);
        fwd_split_units[std::min(bk, kNumBuckets - 1)].push_back(u);
        ll_offs.push_back(rec_ll++);
        ++cnt;
      }
      ll_count[b] = cnt;
    } else {
      const int nwu = (int)((nq + kWuPoints - 1) / kWuPoints);
      ll_count[b] = nwu;
      for (int k = 0; k < nwu; ++k) {
        const int p0 = k * kWuPoints;
        const double pts = (double)std::min<int64_t>(kWuPoints, nq - p0);
        fwd_units[bk].push_back({b, p0, rec_ll, pts * K * (N + 1)});
        ll_offs.push_back(rec_ll++);
      }
    }
    p->max_rows = std::max(p->max_rows, N + 2);
    if (bk == kDeepBucket) {
      // one unit per data point; its lanes split the layers
      gr_first[b] = (int64_t)gr_offs.size();
      gr_count[b] = (int32_t)nq;
      const int ch64 = (N + 1 + 63) / 64;
      const int cls = ch64 <= 8 ? 0 : ch64 <= 16 ? 1 : 2;
      scan_ch[cls] = std::max(scan_ch[cls], ch64);
      for (int64_t k = 0; k < nq; ++k) {
        grad_units[kDeepBucket + cls].push_back({b, (int32_t)k, rec_gr, (double)K * (N + 1) * 64});
        gr_offs.push_back(rec_gr);
        rec_gr += rsz;
      }
      continue;
    }
    if (K > 1 && small_G >= 2) {
      // every point group split over small_G node groups (lane = g npts + p)
      const int npts = kWuPoints / small_G;
      gr_first[b] = (int64_t)gr_offs.size();
      int32_t cnt = 0;
      for (int64_t p0 = 0; p0 < nq; p0 += npts) {
        const int np = (int)std::min<int64_t>(npts, nq - p0);
        Wu u{b, (int32_t)p0, rec_gr, (double)np * K * (N + 1)};
        u.split = np | (small_G << 16);
        split_units[bk].push_back(u);
        gr_offs.push_back(rec_gr);
        rec_gr += rsz;
        ++cnt;
      }
      gr_count[b] = cnt;
      continue;
    }
    const int nfull = (int)(nq / kWuPoints);
    const int ntail = (int)(nq % kWuPoints);
    gr_first[b] = (int64_t)gr_offs.size();
    gr_count[b] = nfull + (ntail > 0 ? 1 : 0);
    for (int k = 0; k < nfull; ++k) {
      grad_units[bk].push_back({b, k * kWuPoints, rec_gr, (double)kWuPoints * K * (N + 1)});
      gr_offs.push_back(rec_gr);
      rec_gr += rsz;
    }
    if (ntail > 0) {
      // a smeared tail that fills most of a wave with node groups x points
      // gets a wave of its own (uniform item); else the tail's lanes join a
      // packed unit and sum into one record of the item
      const int G = std::min(kWuPoints / ntail, K);
      // measured on MI355X: a wave of its own pays off up to 10 layers (the
      // 4096-draw batch: 3 % faster); deeper kernels, at one wave per SIMD,
      // lose more to the idle lanes and the split kernel's registers than
      // they gain from scalar record loads (16384-item ragged batch: 8 %
      // slower), so their tails stay packed
      const bool own_wave = kBucketLmax[bk] <= kSplitTailMaxLayers;
      if (own_wave && (p->opts.split_tails & NR_TAILS_LONE) && ntail >= 48) {
        // most of a wave: a full unit with idle lanes (uniform item)
        grad_units[bk].push_back({b, nfull * kWuPoints, rec_gr, (double)ntail * K * (N + 1)});
      } else if (own_wave && (p->opts.split_tails & NR_TAILS_SPLIT) && K > 1 && G >= 2 &&
                 G <= 4 && ntail * G >= 48) {
        // at least four nodes per lane, so that the wave's epilogue (one
        // reduction of every record field) stays small beside its work
        Wu u{b, nfull * kWuPoints, rec_gr, (double)ntail * K * (N + 1)};
        u.split = ntail | (G << 16);
        split_units[bk].push_back(u);
      } else {
        tails[{N, K}].push_back({b, nfull * kWuPoints, ntail, rec_gr});
      }
      gr_offs.push_back(rec_gr);
      rec_gr += rsz;
    }
  }
  p->rec_ll_total = rec_ll;
  p->rec_grad_total = rec_gr;

  hipError_t e = hipSuccess;
  auto keep = [&](void* ptr) { p->owned.push_back(ptr); };
  e = upload(&p->d_dataset_of_item, p->dataset_of_item);
  keep(p->d_dataset_of_item);
  if (e == hipSuccess) { e = upload(&p->d_q_off, p->q_off); keep(p->d_q_off); }
  if (e == hipSuccess) { e = upload(&p->d_row_off, p->row_off); keep(p->d_row_off); }
  if (e == hipSuccess) { e = upload(&p->d_dqq, p->dqq); keep(p->d_dqq); }
  if (e == hipSuccess) { e = upload(&p->d_out_off, p->out_off); keep(p->d_out_off); }
  auto upload_lists = [&](RecordLists& L, const std::vector<int64_t>& first,
                          const std::vector<int32_t>& count, const std::vector<int64_t>& offs) {
    if (e == hipSuccess) { e = upload(&L.first, first); keep(L.first); }
    if (e == hipSuccess) { e = upload(&L.count, count); keep(L.count); }
    if (e == hipSuccess) { e = upload(&L.offs, offs); keep(L.offs); }
  };
  {
    std::vector<uint8_t> kind((size_t)p->row_off.back(), 1);
    p->uniform_rows = nI > 0 ? (int)(p->row_off[1] - p->row_off[0]) : 0;
    for (int b = 0; b < nI; ++b) {
      kind[(size_t)p->row_off[b]] = 0;
      kind[(size_t)p->row_off[b + 1] - 1] = 2;
      if (p->row_off[b + 1] - p->row_off[b] != p->uniform_rows) p->uniform_rows = 0;
    }
    if (e == hipSuccess) { e = upload(&p->d_row_kind, kind); keep(p->d_row_kind); }
  }
  upload_lists(p->lists_ll, ll_first, ll_count, ll_offs);
  upload_lists(p->lists_grad, gr_first, gr_count, gr_offs);
  if (e == hipSuccess) {
    std::vector<double> rule(p->node_t, p->node_t + kSmearNodes);
    rule.insert(rule.end(), p->node_w, p->node_w + kSmearNodes);
    append_math_tables(rule);
    e = upload(&p->d_rule, rule);
    keep(p->d_rule);
  }

  std::vector<Launch> tail_launches;  // after the full units
  // tail launches: per (depth, nodes) group, largest tails first, first fit
  // into 64-lane units; then one launch per bucket over all its groups (the
  // units holding a single item join the full units below)
  {
    std::vector<std::vector<int32_t>> b_item(kNumBuckets), b_litem(kNumBuckets), b_lpt(kNumBuckets);
    std::vector<std::vector<int64_t>> b_lrec(kNumBuckets);
    for (auto& kv : tails) {
      const int bk = bucket_of(kv.first.first);
      auto& v = kv.second;
      std::stable_sort(v.begin(), v.end(),
                       [](const Tail& x, const Tail& y) { return x.count > y.count; });
      std::vector<int> fill;                   // lanes used per unit of this group
      std::vector<std::vector<size_t>> units;  // the tails of each unit
      for (size_t t = 0; t < v.size(); ++t) {
        size_t u = p->opts.pack_tails ? 0 : fill.size();
        while (u < fill.size() && fill[u] + v[t].count > kWuPoints) ++u;
        if (u == fill.size()) {
          fill.push_back(0);
          units.emplace_back();
        }
        units[u].push_back(t);
        fill[u] += v[t].count;
      }
      for (const auto& un : units) {
        if (un.size() == 1) {
          // a unit of one item is a full unit with idle lanes (its layer
          // records stay scalar loads)
          const Tail& t = v[un[0]];
          grad_units[bk].push_back(
              {t.item, t.p0, t.rec0, (double)t.count * kv.first.second * (kv.first.first + 1)});
          continue;
        }
        const size_t base = b_item[bk].size() * kWuPoints;
        b_item[bk].push_back(v[un[0]].item);
        b_litem[bk].insert(b_litem[bk].end(), kWuPoints, -1);
        b_lpt[bk].insert(b_lpt[bk].end(), kWuPoints, 0);
        b_lrec[bk].insert(b_lrec[bk].end(), kWuPoints, -1);
        int f = 0;
        for (size_t ti : un) {
          const Tail& t = v[ti];
          for (int l = 0; l < t.count; ++l) {
            b_litem[bk][base + f + l] = t.item;
            b_lpt[bk][base + f + l] = t.p0 + l;
            b_lrec[bk][base + f + l] = t.rec0;
          }
          f += t.count;
        }
      }
    }
    for (int bk = kNumBuckets - 1; bk >= 0; --bk) {
      if (b_item[bk].empty() || e != hipSuccess) continue;
      // idle lanes repeat lane 0 of their unit (a valid point, result unused)
      for (size_t u = 0; u < b_item[bk].size(); ++u)
        for (int l = 0; l < kWuPoints; ++l)
          if (b_litem[bk][u * kWuPoints + l] < 0) {
            b_litem[bk][u * kWuPoints + l] = b_litem[bk][u * kWuPoints];
            b_lpt[bk][u * kWuPoints + l] = b_lpt[bk][u * kWuPoints];
          }
      Launch L;
      L.bucket = bk;
      L.store = p->bucket_store[bk];
      L.tail = true;
      L.n_wu = (int)b_item[bk].size();
      e = upload(&L.item, b_item[bk]);
      keep(L.item);
      if (e == hipSuccess) { e = upload(&L.lane_item, b_litem[bk]); keep(L.lane_item); }
      if (e == hipSuccess) { e = upload(&L.lane_pt, b_lpt[bk]); keep(L.lane_pt); }
      if (e == hipSuccess) { e = upload(&L.lane_rec, b_lrec[bk]); keep(L.lane_rec); }
      tail_launches.push_back(L);
    }
  }

  // full-unit launches: one per non-empty bucket, deepest first, LPT order
  auto make_full = [&](std::vector<std::vector<Wu>>& units, std::vector<Launch>& out_list,
                       bool split) {
    for (int bk = (int)units.size() - 1; bk >= 0; --bk) {
      auto& v = units[bk];
      if (v.empty() || e != hipSuccess) continue;
      std::stable_sort(v.begin(), v.end(), [](const Wu& x, const Wu& y) { return x.cost > y.cost; });
      std::vector<int32_t> it(v.size()), p0(v.size()), sc(v.size());
      std::vector<int64_t> rc(v.size());
      for (size_t k = 0; k < v.size(); ++k) {
        const size_t src = xcd_order(k, v.size(), (size_t)p->opts.xcd_run);
        it[k] = v[src].item;
        p0[k] = v[src].p0;
        rc[k] = v[src].rec;
        sc[k] = v[src].split;
      }
      Launch L;
      L.bucket = std::min(bk, kDeepBucket);
      L.store = bk < kNumBuckets && p->bucket_store[bk];
      L.scan_ch = bk >= kDeepBucket ? std::max(scan_ch[bk - kDeepBucket], 1) : 0;
      L.split = split;
      L.n_wu = (int)v.size();
      e = upload(&L.item, it);
      keep(L.item);
      if (e == hipSuccess) { e = upload(&L.p0, p0); keep(L.p0); }
      if (e == hipSuccess) { e = upload(&L.rec, rc); keep(L.rec); }
      if (e == hipSuccess && split) { e = upload(&L.split_code, sc); keep(L.split_code); }
      out_list.push_back(L);
    }
  };
  make_full(fwd_units, p->launches_fwd, false);
  make_full(fwd_split_units, p->launches_fwd, true);
  make_full(grad_units, p->launches_grad, false);
  const size_t n_main = p->launches_grad.size();
  make_full(split_units, p->launches_grad, true);
  p->launches_grad.insert(p->launches_grad.end(), tail_launches.begin(), tail_launches.end());
  // Tail and split launches of at most one round of the chip (two waves per
  // SIMD) leave most of it idle when they run after the full units; on the
  // side stream they run beside them.  Larger ones gain nothing there and
  // only interfere (the 4096-draw batch's 4096 split units: 2 % slower).
  // Every second full-unit launch (one per layer-count bucket, deepest first)
  // goes there too, so that one bucket's last waves overlap the next bucket's
  // first (16384-item ragged batch: 1.8 % faster in FP64).
  if (e == hipSuccess && p->opts.side_stream && n_main > 0) {
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
    const int round = 2 * 4 * std::max(cus, 1);
    bool any = false;
    for (size_t k = 1; k < n_main; k += 2) any = p->launches_grad[k].side = true;
    for (size_t k = n_main; k < p->launches_grad.size() && e == hipSuccess; ++k)
      if (p->launches_grad[k].n_wu <= round) any = p->launches_grad[k].side = true;
    if (any && e == hipSuccess) e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
    if (any && e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
    if (any && e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming);
    if (any && e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_fork_cap, hipEventDisableTiming);
    if (any && e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_join_cap, hipEventDisableTiming);
  }
  for (int c = 0; c < kDeepClasses && e == hipSuccess; ++c)
    if (scan_ch[c] > 0) e = prepare_grad_scan(scan_ch[c]);
  if (e == hipSuccess) e = prepare_reduce(p->max_rows);

  if (e != hipSuccess) {
    plan_free(p);
    delete p;
    g_last_hip_error = std::string("plan upload: ") + hipGetErrorString(e);
    return (e == hipErrorOutOfMemory) ? NR_ENOMEM : NR_EHIP;
  }
  *out = p;
  return NR_OK;
}

nr_status nr_leapfrog(const nr_plan* p, const nr_values* data, const nr_hmc_state* st, double dt,
                      int32_t n_steps, void* ws, size_t ws_bytes, void* stream) {
  nr_status s = check_hmc(p, data, st, dt, n_steps, ws, ws_bytes);
  if (s != NR_OK) return s;
  return enqueue_leapfrog(p, data, st, dt, n_steps, ws, (hipStream_t)stream, true);
}

nr_status nr_leapfrog_graph_create(const nr_plan* p, const nr_values* data, const nr_hmc_state* st,
                                   double dt, int32_t n_steps, void* ws, size_t ws_bytes,
                                   nr_graph** out) {
  if (!out) return NR_EINVAL;
  *out = nullptr;
  nr_status s = check_hmc(p, data, st, dt, n_steps, ws, ws_bytes);
  if (s != NR_OK) return s;
  nr_graph* g = new nr_graph();
  hipError_t e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(e, "graph stream");
  }
  e = hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    s = enqueue_leapfrog(p, data, st, dt, n_steps, ws, g->stream, false);
    hipError_t e2 = hipStreamEndCapture(g->stream, &g->graph);
    if (s == NR_OK && e2 != hipSuccess) s = hip_fail(e2, "end capture");
  } else {
    s = hip_fail(e, "begin capture");
  }
  if (s == NR_OK) {
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) s = hip_fail(e, "graph instantiate");
  }
  if (s != NR_OK) {
    nr_graph_destroy(g);
    return s;
  }
  *out = g;
  return NR_OK;
}

nr_status nr_hmc_create(const nr_plan* p, const nr_hmc_config* cfg, nr_hmc** out) {
  if (!out) return NR_EINVAL;
  *out = nullptr;
  if (!p || !cfg || cfg->n_leapfrog < 1 || !(cfg->max_energy_error > 0.0) ||
      !(cfg->target_accept > 0.0 && cfg->target_accept < 1.0))
    return NR_EINVAL;
  nr_hmc* h = new nr_hmc();
  h->plan = p;
  h->cfg = *cfg;
  h->n_entries = p->row_off.back() * 4 + 2 * (int64_t)p->n_items;
  const size_t nd = (size_t)(5 * h->n_entries + (int64_t)kChainScalars * p->n_items);
  hipError_t e = hipSuccess;
  if (nd > 0) {
    e = hipMalloc(reinterpret_cast<void**>(&h->buf), nd * sizeof(double));
    if (e == hipSuccess) e = hipMemset(h->buf, 0, nd * sizeof(double));
  }
  if (e == hipSuccess && p->n_items > 0) {
    e = hipMalloc(reinterpret_cast<void**>(&h->iter), p->n_items * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMemset(h->iter, 0, p->n_items * sizeof(uint64_t));
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    nr_hmc_destroy(h);
    (void)hip_fail(e, "hmc state");
    return (e == hipErrorOutOfMemory) ? NR_ENOMEM : NR_EHIP;
  }
  *out = h;
  return NR_OK;
}

nr_status nr_hmc_destroy(nr_hmc* h) {
  if (!h) return NR_OK;
  if (h->buf) (void)hipFree(h->buf);
  if (h->iter) (void)hipFree(h->iter);
  delete h;
  return NR_OK;
}

nr_status nr_hmc_init(nr_hmc* h, const nr_values* data, const nr_hmc_chains* ch,
                      int32_t from_theta, void* ws, size_t ws_bytes, void* stream) {
  nr_status s = check_chains(h, data, ch, ws, ws_bytes);
  if (s != NR_OK) return s;
  if (h->plan->n_items == 0) return NR_OK;
  hipStream_t st = (hipStream_t)stream;
  const HmcArgs a = hmc_args(h, ch);
  hipError_t e = launch_hmc(kHmcTheta, a, from_theta ? 1 : 0, 0.0, st);
  if (e != hipSuccess) return hip_fail(e, "hmc theta");
  const nr_values v = chain_values(data, ch);
  s = enqueue_grad(h->plan, &v, ch->logL, ch->g_rows, ch->g_inst, ws, st, true);
  if (s != NR_OK) return s;
  e = launch_hmc(kHmcPotential, a, 0, 0.0, st);
  return e == hipSuccess ? NR_OK : hip_fail(e, "hmc potential");
}

nr_status nr_hmc_transition(nr_hmc* h, const nr_values* data, const nr_hmc_chains* ch,
                            int32_t adapt, void* ws, size_t ws_bytes, void* stream) {
  nr_status s = check_chains(h, data, ch, ws, ws_bytes);
  if (s != NR_OK) return s;
  if (adapt & ~(NR_HMC_ADAPT_MASS | NR_HMC_ADAPT_STEP)) return NR_EINVAL;
  return enqueue_transition(h, data, ch, adapt, ws, (hipStream_t)stream, true);
}

nr_status nr_hmc_graph_create(nr_hmc* h, const nr_values* data, const nr_hmc_chains* ch,
                              int32_t adapt, int32_t n_transitions, void* ws, size_t ws_bytes,
                              nr_graph** out) {
  if (!out) return NR_EINVAL;
  *out = nullptr;
  nr_status s = check_chains(h, data, ch, ws, ws_bytes);
  if (s != NR_OK) return s;
  if (n_transitions < 0 || (adapt & ~(NR_HMC_ADAPT_MASS | NR_HMC_ADAPT_STEP))) return NR_EINVAL;
  nr_graph* g = new nr_graph();
  hipError_t e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(e, "graph stream");
  }
  e = hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    for (int32_t t = 0; t < n_transitions && s == NR_OK; ++t)
      s = enqueue_transition(h, data, ch, adapt, ws, g->stream, false);
    hipError_t e2 = hipStreamEndCapture(g->stream, &g->graph);
    if (s == NR_OK && e2 != hipSuccess) s = hip_fail(e2, "end capture");
  } else {
    s = hip_fail(e, "begin capture");
  }
  if (s == NR_OK) {
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) s = hip_fail(e, "graph instantiate");
  }
  if (s != NR_OK) {
    nr_graph_destroy(g);
    return s;
  }
  *out = g;
  return NR_OK;
}

nr_status nr_hmc_adapt(nr_hmc* h, const nr_hmc_chains* ch, int32_t actions, void* stream) {
  if (!h || !ch) return NR_EINVAL;
  if (actions & ~(NR_HMC_MASS_WINDOW_END | NR_HMC_STEP_RESTART | NR_HMC_STEP_FINAL))
    return NR_EINVAL;
  if (h->plan->n_items == 0 || actions == 0) return NR_OK;
  if (!chains_complete(ch)) return NR_EINVAL;
  hipError_t e = launch_hmc(kHmcAdapt, hmc_args(h, ch), actions, 0.0, (hipStream_t)stream);
  return e == hipSuccess ? NR_OK : hip_fail(e, "hmc adapt");
}

nr_status nr_vi_mvn_create(const nr_plan* p, const nr_vi_mvn_config* cfg, nr_vi_mvn** out) {
  if (!out) return NR_EINVAL;
  *out = nullptr;
  if (!p || !cfg || cfg->n_restarts < 1 || cfg->n_draws < 1 ||
      (int64_t)cfg->n_restarts * cfg->n_draws != p->n_items || p->uniform_rows < 2 ||
      p->uniform_rows > kMaxLayers + 2 ||
      !(cfg->lr > 0.0) || !(cfg->beta1 >= 0.0 && cfg->beta1 < 1.0) ||
      !(cfg->beta2 >= 0.0 && cfg->beta2 < 1.0) || !(cfg->adam_eps > 0.0))
    return NR_EINVAL;
  nr_vi_mvn* m = new nr_vi_mvn();
  m->plan = p;
  m->cfg = *cfg;
  m->rows = p->uniform_rows;
  m->P = 4 * m->rows + 2;
  const int64_t items = p->n_items, P = m->P, R = cfg->n_restarts;
  const int64_t n_adam = R * (2 * P + P * P);
  const int64_t sizes[] = {items * P, items * P, items * P, items, items * 4 * m->rows,
                           items, items, items, items * 4 * m->rows, items * 2, n_adam, n_adam};
  int64_t total = 0;
  for (int64_t v : sizes) total += v;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&m->buf), (size_t)total * sizeof(double));
  if (e == hipSuccess) e = hipMemset(m->buf, 0, (size_t)total * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&m->iter), sizeof(uint64_t));
  if (e == hipSuccess) e = hipMemset(m->iter, 0, sizeof(uint64_t));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    nr_vi_mvn_destroy(m);
    (void)hip_fail(e, "mvn state");
    return (e == hipErrorOutOfMemory) ? NR_ENOMEM : NR_EHIP;
  }
  double* ptrs[12];
  double* q = m->buf;
  for (int k = 0; k < 12; ++k) {
    ptrs[k] = q;
    q += sizes[k];
  }
  MvnArgs& a = m->args;
  std::memset(&a, 0, sizeof(a));
  a.R = cfg->n_restarts;
  a.S = cfg->n_draws;
  a.P = m->P;
  a.rows = m->rows;
  a.eps = ptrs[0];
  a.z = ptrs[1];
  a.h = ptrs[2];
  a.f = ptrs[3];
  a.layers = ptrs[4];
  a.scale = ptrs[5];
  a.bkg = ptrs[6];
  a.logL = ptrs[7];
  a.g_rows = ptrs[8];
  a.g_inst = ptrs[9];
  a.adam_m = ptrs[10];
  a.adam_v = ptrs[11];
  a.iter = m->iter;
  a.seed = cfg->seed;
  a.lr = cfg->lr;
  a.beta1 = cfg->beta1;
  a.beta2 = cfg->beta2;
  a.adam_eps = cfg->adam_eps;
  *out = m;
  return NR_OK;
}

nr_status nr_vi_mvn_destroy(nr_vi_mvn* m) {
  if (!m) return NR_OK;
  if (m->buf) (void)hipFree(m->buf);
  if (m->iter) (void)hipFree(m->iter);
  delete m;
  return NR_OK;
}

nr_status nr_vi_mvn_step(nr_vi_mvn* m, const nr_values* data, const nr_vi_mvn_params* prm,
                         int32_t adam, void* ws, size_t ws_bytes, void* stream) {
  nr_status s = check_mvn(m, data, prm, ws, ws_bytes);
  if (s != NR_OK) return s;
  return enqueue_mvn_step(m, data, prm, adam != 0, ws, (hipStream_t)stream, true);
}

nr_status nr_vi_mvn_graph_create(nr_vi_mvn* m, const nr_values* data, const nr_vi_mvn_params* prm,
                                 int32_t n_steps, void* ws, size_t ws_bytes, nr_graph** out) {
  if (!out) return NR_EINVAL;
  *out = nullptr;
  nr_status s = check_mvn(m, data, prm, ws, ws_bytes);
  if (s != NR_OK) return s;
  if (n_steps < 0) return NR_EINVAL;
  nr_graph* g = new nr_graph();
  hipError_t e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(e, "graph stream");
  }
  e = hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    for (int32_t t = 0; t < n_steps && s == NR_OK; ++t)
      s = enqueue_mvn_step(m, data, prm, true, ws, g->stream, false);
    hipError_t e2 = hipStreamEndCapture(g->stream, &g->graph);
    if (s == NR_OK && e2 != hipSuccess) s = hip_fail(e2, "end capture");
  } else {
    s = hip_fail(e, "begin capture");
  }
  if (s == NR_OK) {
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) s = hip_fail(e, "graph instantiate");
  }
  if (s != NR_OK) {
    nr_graph_destroy(g);
    return s;
  }
  *out = g;
  return NR_OK;
}

nr_status nr_graph_launch(nr_graph* g, void* stream) {
  if (!g || !g->exec) return NR_EINVAL;
  hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  return e == hipSuccess ? NR_OK : hip_fail(e, "graph launch");
}

nr_status nr_graph_destroy(nr_graph* g) {
  if (!g) return NR_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->stream) (void)hipStreamDestroy(g->stream);
  delete g;
  return NR_OK;
}

nr_status nr_vi_elbo_grad(const nr_plan* p, const nr_values* data, const nr_vi_args* vi,
                          void* ws, size_t ws_bytes, void* stream) {
  if (!p || !data || !vi) return NR_EINVAL;
  if (p->n_items == 0) return NR_EINVAL;
  const int rows = p->uniform_rows;
  if (rows < 2) return NR_EINVAL;
  if (!vi->mu || !vi->omega || !vi->mask || !vi->eps || !vi->layers || !vi->scale ||
      !vi->bkg || !vi->logL || !vi->g_rows || !vi->g_inst || !vi->grad_mu ||
      !vi->grad_omega || !vi->elbo)
    return NR_EINVAL;
  nr_values v = *data;
  v.layers = vi->layers;
  v.scale = vi->scale;
  v.bkg = vi->bkg;
  nr_status s = check_call(p, &v, true);
  if (s != NR_OK) return s;
  const size_t need = sizeof(double) * op_doubles(p, NR_OP_LOGLIK_GRAD);
  if (need > 0 && (!ws || ws_bytes < need)) return NR_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  const int P = rows * 4 + 2;
  hipError_t e = launch_vi_sample(p->n_items, P, rows, vi->mu, vi->omega, vi->mask, vi->eps,
                                  vi->layers, vi->scale, vi->bkg, st);
  if (e != hipSuccess) return hip_fail(e, "sampler launch");
  s = enqueue_grad(p, &v, vi->logL, vi->g_rows, vi->g_inst, ws, st, true);
  if (s != NR_OK) return s;
  e = launch_vi_reduce(p->n_items, P, rows, vi->omega, vi->mask, vi->eps, vi->logL, vi->g_rows,
                       vi->g_inst, vi->grad_mu, vi->grad_omega, vi->elbo, st);
  return e == hipSuccess ? NR_OK : hip_fail(e, "reduction launch");
}

nr_status nr_tie_sum(int64_t n_out, const int64_t* first, const int64_t* src, const double* in,
                     double* out, void* stream) {
  if (n_out < 0) return NR_EINVAL;
  if (n_out == 0) return NR_OK;
  if (!first || !src || !in || !out) return NR_EINVAL;
  hipError_t e = launch_tie_sum(n_out, first, src, in, out, (hipStream_t)stream);
  return e == hipSuccess ? NR_OK : hip_fail(e, "tie-sum launch");
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
  if (op != NR_OP_REFLECTIVITY && op != NR_OP_LOGLIK && op != NR_OP_LOGLIK_GRAD) return NR_EINVAL;
  *bytes = sizeof(double) * op_doubles(p, op);
  return NR_OK;
}

nr_status nr_output_offsets(const nr_plan* p, int64_t* out_off) {
  if (!p || !out_off) return NR_EINVAL;
  std::memcpy(out_off, p->out_off.data(), sizeof(int64_t) * p->out_off.size());
  return NR_OK;
}

nr_status nr_reflectivity(const nr_plan* p, const nr_values* v, double* r_hat, void* ws,
                          size_t ws_bytes, void* stream) {
  nr_status st = check_call(p, v, false);
  if (st != NR_OK) return st;
  if (p->n_items == 0 || p->out_off.back() == 0) return NR_OK;
  if (!r_hat) return NR_EINVAL;
  if (!ws || ws_bytes < sizeof(double) * op_doubles(p, NR_OP_REFLECTIVITY)) return NR_EWORKSPACE;
  KernelArgs a = base_args(p, v);
  a.out = r_hat;
  a.consts = static_cast<double*>(ws);
  a.constsf = consts_floats(p, a.consts);
  return run_launches(p, kOpReflectivity, a, (hipStream_t)stream);
}

nr_status nr_loglik(const nr_plan* p, const nr_values* v, double* logL, void* ws,
                    size_t ws_bytes, void* stream) {
  nr_status st = check_call(p, v, true);
  if (st != NR_OK) return st;
  if (p->n_items == 0) return NR_OK;
  if (!logL) return NR_EINVAL;
  const size_t need = sizeof(double) * op_doubles(p, NR_OP_LOGLIK);
  if (need > 0 && (!ws || ws_bytes < need)) return NR_EWORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  KernelArgs a = base_args(p, v);
  a.consts = static_cast<double*>(ws);
  a.constsf = consts_floats(p, a.consts);
  a.rec = static_cast<double*>(ws) + consts_doubles(p);
  st = run_launches(p, kOpLoglik, a, s);
  if (st != NR_OK) return st;
  ReduceArgs r;
  std::memset(&r, 0, sizeof(r));
  r.n_items = p->n_items;
  r.item_wu_first = p->lists_ll.first;
  r.item_wu_count = p->lists_ll.count;
  r.rec_of_wu = p->lists_ll.offs;
  r.rec = a.rec;
  r.logL = logL;
  hipError_t e = launch_reduce(kOpLoglik, r, s);
  return e == hipSuccess ? NR_OK : hip_fail(e, "reduce launch");
}

nr_status nr_reflectivity_vjp(const nr_plan* p, const nr_values* v, const double* seed,
                              double* dot, double* g_rows, double* g_inst, void* ws,
                              size_t ws_bytes, void* stream) {
  nr_status st = check_call(p, v, false);
  if (st != NR_OK) return st;
  if (p->n_items == 0) return NR_OK;
  if (!dot || !g_rows || !g_inst) return NR_EINVAL;
  if (p->out_off.back() > 0 && !seed) return NR_EINVAL;
  const size_t need = sizeof(double) * op_doubles(p, NR_OP_LOGLIK_GRAD);
  if (need > 0 && (!ws || ws_bytes < need)) return NR_EWORKSPACE;
  return enqueue_grad(p, v, dot, g_rows, g_inst, ws, (hipStream_t)stream, true, seed);
}

nr_status nr_loglik_grad_res(const nr_plan* p, const nr_values* v, double* logL, double* g_rows,
                             double* g_inst, double* g_res, void* ws, size_t ws_bytes,
                             void* stream) {
  nr_status st = check_call(p, v, true);
  if (st != NR_OK) return st;
  if (p->n_items == 0) return NR_OK;
  if (!logL || !g_rows || !g_inst || !g_res) return NR_EINVAL;
  const size_t need = sizeof(double) * op_doubles(p, NR_OP_LOGLIK_GRAD);
  if (need > 0 && (!ws || ws_bytes < need)) return NR_EWORKSPACE;
  return enqueue_grad(p, v, logL, g_rows, g_inst, ws, (hipStream_t)stream, true, nullptr, g_res);
}

nr_status nr_loglik_grad(const nr_plan* p, const nr_values* v, double* logL, double* g_rows,
                         double* g_inst, void* ws, size_t ws_bytes, void* stream) {
  nr_status st = check_call(p, v, true);
  if (st != NR_OK) return st;
  if (p->n_items == 0) return NR_OK;
  if (!logL || !g_rows || !g_inst) return NR_EINVAL;
  const size_t need = sizeof(double) * op_doubles(p, NR_OP_LOGLIK_GRAD);
  if (need > 0 && (!ws || ws_bytes < need)) return NR_EWORKSPACE;
  return enqueue_grad(p, v, logL, g_rows, g_inst, ws, (hipStream_t)stream, true);
}

nr_status nr_loglik_grad_noalloc(const nr_plan* p, const nr_values* v, double* logL,
                                 double* g_rows, double* g_inst, void* stream) {
  nr_status st = check_call(p, v, true);
  if (st != NR_OK) return st;
  if (p->n_items == 0) return NR_OK;
  if (!logL || !g_rows || !g_inst) return NR_EINVAL;
  const size_t need = sizeof(double) * op_doubles(p, NR_OP_LOGLIK_GRAD);
  if (need > (size_t)NR_NOALLOC_SCRATCH_BYTES) return NR_ESCRATCH;
  void* ws = nullptr;
  st = scratch_addr(p->device, &ws);
  if (st != NR_OK) return st;
  return enqueue_grad(p, v, logL, g_rows, g_inst, ws, (hipStream_t)stream, true);
}

}  // extern "C"
