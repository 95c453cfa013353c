// Driver for the address / undefined-behaviour sanitizer build of the CPU
// oracle (tests/test_oracle_sanitizers.py compiles it together with
// oracle/nr_oracle.cpp).  It calls every exported oracle function on small
// stacks of 0..40 layers, a 300-layer stack (value functions), empty and
// one-point grids, smeared and unsmeared, and the batched entry point with a
// ragged batch on one and two threads.  Every result must be finite; the
// sanitizers report any out-of-bounds access, use after free, leak, signed
// overflow or other undefined behaviour and make the process fail.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
int orc_version(void);
int orc_gauss_legendre17(double* x, double* u);
int orc_smear_rule(double dq_over_q, double* t, double* w);
int orc_smear_nodes(int nq, const double* Q, double dq_over_q, double* q_nodes);
int orc_kz(double x, double y, double* out);
int orc_reflectivity(int L, const double* rows, int nq, const double* q, double* R);
int orc_reflectivity_parratt(int L, const double* rows, int nq, const double* q, double* R);
int orc_reflectivity_linsys(int L, const double* rows, int nq, const double* q, double* R);
int orc_model_curve(int L, const double* rows, double scale, double bkg, int nq, const double* Q,
                    double dq_over_q, double* Rhat);
int orc_smeared(int L, const double* rows, int nq, const double* Q, double dq_over_q,
                double* Rsm);
double orc_loglik(int L, const double* rows, double scale, double bkg, int nq, const double* Q,
                  const double* Robs, const double* Rerr, double dq_over_q);
int orc_loglik_grad_cs(int L, const double* rows, double scale, double bkg, int nq,
                       const double* Q, const double* Robs, const double* Rerr,
                       double dq_over_q, double* logL, double* g_rows, double* g_inst);
int orc_loglik_grad_fd(int L, const double* rows, double scale, double bkg, int nq,
                       const double* Q, const double* Robs, const double* Rerr,
                       double dq_over_q, double rel_step, double* g_rows, double* g_inst);
int orc_model_vjp_cs(int L, const double* rows, double scale, double bkg, int nq,
                     const double* Q, double dq_over_q, const double* seed, double* g_rows,
                     double* g_inst);
int orc_reflectivity_jac_cs(int L, const double* rows, int nq, const double* q, double* dR);
int orc_loglik_grad_batch(int n_datasets, const int64_t* q_off, const double* Q,
                          const double* Robs, const double* Rerr, const double* dq_over_q,
                          int n_items, const int32_t* dataset_of_item, const int64_t* row_off,
                          const double* layers, const double* scale, const double* bkg,
                          int want_grad, int nthreads, double* logL, double* g_rows,
                          double* g_inst);
int orc_reflectivity_dq_cs(int L, const double* rows, int nq, const double* q, double* dRdq);
int orc_model_curve_res(int L, const double* rows, double scale, double bkg, int nq,
                        const double* Q, double dq_over_q, const double* dQ, double* Rhat);
int orc_loglik_grad_res_cs(int L, const double* rows, double scale, double bkg, int nq,
                           const double* Q, const double* Robs, const double* Rerr,
                           double dq_over_q, const double* dQ, double* logL, double* g_rows,
                           double* g_inst, double* g_res);
int orc_loglik_res_fd(int L, const double* rows, double scale, double bkg, int nq,
                      const double* Q, const double* Robs, const double* Rerr, double dq_over_q,
                      double rel_step, double* g_res);
int orc_max_threads(void);
}

namespace {

int g_fail = 0;

void expect(bool ok, const char* what, int L, int nq) {
  if (!ok) {
    std::fprintf(stderr, "FAIL %s (L=%d, nq=%d)\n", what, L, nq);
    g_fail = 1;
  }
}

bool finite(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

std::vector<double> stack(std::mt19937_64& g, int L) {
  std::uniform_real_distribution<double> d(10.0, 300.0), rho(-0.5e-6, 6.5e-6), im(1e-9, 1e-8),
      sg(1.0, 15.0);
  std::vector<double> r((L + 2) * 4, 0.0);
  for (int j = 1; j <= L; ++j) {
    r[4 * j] = d(g);
    r[4 * j + 1] = rho(g);
    r[4 * j + 2] = im(g);
  }
  r[4 * (L + 1) + 1] = 2.07e-6;
  r[4 * (L + 1) + 2] = 1e-9;
  for (int j = 1; j <= L + 1; ++j) r[4 * j + 3] = sg(g);
  return r;
}

std::vector<double> grid(int n) {
  std::vector<double> q(n);
  for (int i = 0; i < n; ++i)
    q[i] = n == 1 ? 0.05 : 0.006 * std::pow(0.3 / 0.006, (double)i / (n - 1));
  return q;
}

void one_stack(std::mt19937_64& g, int L, int nq, double dqq, bool grads) {
  const std::vector<double> rows = stack(g, L);
  const std::vector<double> Q = grid(nq);
  const int K = dqq > 0.0 ? 17 : 1;
  std::vector<double> R(nq), Rp(nq), Rhat(nq), Rsm(nq), nodes((size_t)nq * 17);
  expect(orc_reflectivity(L, rows.data(), nq, Q.data(), R.data()) == 0 && finite(R), "R", L, nq);
  expect(orc_reflectivity_parratt(L, rows.data(), nq, Q.data(), Rp.data()) == 0 && finite(Rp),
         "parratt", L, nq);
  expect(orc_smear_nodes(nq, Q.data(), dqq, nodes.data()) == K, "nodes", L, nq);
  expect(orc_model_curve(L, rows.data(), 1.01, 1e-7, nq, Q.data(), dqq, Rhat.data()) == 0 &&
             finite(Rhat),
         "model", L, nq);
  expect(orc_smeared(L, rows.data(), nq, Q.data(), dqq, Rsm.data()) == 0 && finite(Rsm),
         "smeared", L, nq);
  std::vector<double> Robs(nq), Rerr(nq), seed(nq);
  for (int i = 0; i < nq; ++i) {
    Rerr[i] = 0.03 * Rhat[i];
    Robs[i] = 1.02 * Rhat[i];
    seed[i] = 1.0 / (1.0 + i);
  }
  const double ll = orc_loglik(L, rows.data(), 1.0, 1e-7, nq, Q.data(), Robs.data(), Rerr.data(),
                               dqq);
  expect(std::isfinite(ll), "loglik", L, nq);
  std::vector<double> dq(nq);
  for (int i = 0; i < nq; ++i) dq[i] = 0.05 * Q[i];
  expect(orc_model_curve_res(L, rows.data(), 1.0, 1e-7, nq, Q.data(), dqq, dq.data(),
                             Rhat.data()) == 0 &&
             finite(Rhat),
         "model_res", L, nq);
  if (!grads) return;
  if (L <= 8) {
    std::vector<double> Rl(nq);
    expect(orc_reflectivity_linsys(L, rows.data(), nq, Q.data(), Rl.data()) == 0 && finite(Rl),
           "linsys", L, nq);
  }
  const int np = (L + 2) * 4;
  std::vector<double> gr(np), gi(2), gf(np), gif(2), jac((size_t)nq * np), dRdq(nq);
  double lg = 0.0, gres = 0.0;
  expect(orc_loglik_grad_cs(L, rows.data(), 1.0, 1e-7, nq, Q.data(), Robs.data(), Rerr.data(),
                            dqq, &lg, gr.data(), gi.data()) == 0 &&
             finite(gr) && finite(gi),
         "grad_cs", L, nq);
  expect(orc_loglik_grad_fd(L, rows.data(), 1.0, 1e-7, nq, Q.data(), Robs.data(), Rerr.data(),
                            dqq, 1e-4, gf.data(), gif.data()) == 0 &&
             finite(gf),
         "grad_fd", L, nq);
  expect(orc_model_vjp_cs(L, rows.data(), 1.0, 1e-7, nq, Q.data(), dqq, seed.data(), gr.data(),
                          gi.data()) == 0 &&
             finite(gr),
         "vjp", L, nq);
  expect(orc_reflectivity_jac_cs(L, rows.data(), nq, Q.data(), jac.data()) == 0 && finite(jac),
         "jac", L, nq);
  expect(orc_reflectivity_dq_cs(L, rows.data(), nq, Q.data(), dRdq.data()) == 0 && finite(dRdq),
         "dRdq", L, nq);
  expect(orc_loglik_grad_res_cs(L, rows.data(), 1.0, 1e-7, nq, Q.data(), Robs.data(),
                                Rerr.data(), dqq, nullptr, &lg, gr.data(), gi.data(),
                                &gres) == 0 &&
             std::isfinite(gres),
         "grad_res", L, nq);
  expect(orc_loglik_grad_res_cs(L, rows.data(), 1.0, 1e-7, nq, Q.data(), Robs.data(),
                                Rerr.data(), dqq, dq.data(), &lg, gr.data(), gi.data(),
                                &gres) == 0,
         "grad_res_pointwise", L, nq);
  if (dqq > 0.0)
    expect(orc_loglik_res_fd(L, rows.data(), 1.0, 1e-7, nq, Q.data(), Robs.data(), Rerr.data(),
                             dqq, 1e-3, &gres) == 0 &&
               std::isfinite(gres),
           "res_fd", L, nq);
}

void batch(std::mt19937_64& g, int nthreads) {
  const int nds = 3, ni = 7;
  const int nqs[nds] = {9, 0, 5};
  const double dqqs[nds] = {0.05, 0.0, 0.02};
  std::vector<int64_t> q_off{0};
  std::vector<double> Q;
  for (int s = 0; s < nds; ++s) {
    const std::vector<double> q = grid(nqs[s]);
    Q.insert(Q.end(), q.begin(), q.end());
    q_off.push_back((int64_t)Q.size());
  }
  std::vector<double> Robs(Q.size()), Rerr(Q.size());
  for (size_t i = 0; i < Q.size(); ++i) {
    Robs[i] = 1e-3 / (1.0 + i);
    Rerr[i] = 0.03 * Robs[i];
  }
  const int Ls[ni] = {0, 3, 1, 6, 2, 0, 4};
  std::vector<int64_t> row_off{0};
  std::vector<double> layers;
  std::vector<int32_t> dsi;
  for (int b = 0; b < ni; ++b) {
    const std::vector<double> r = stack(g, Ls[b]);
    layers.insert(layers.end(), r.begin(), r.end());
    row_off.push_back(row_off.back() + Ls[b] + 2);
    dsi.push_back(b % nds);
  }
  std::vector<double> sc(ni, 1.0), bk(ni, 1e-7), ll(ni), gr(layers.size()), gi(2 * ni);
  for (int want = 0; want < 2; ++want)
    expect(orc_loglik_grad_batch(nds, q_off.data(), Q.data(), Robs.data(), Rerr.data(), dqqs,
                                 ni, dsi.data(), row_off.data(), layers.data(), sc.data(),
                                 bk.data(), want, nthreads, ll.data(), gr.data(),
                                 gi.data()) == 0 &&
               finite(ll),
           "batch", -1, (int)Q.size());
  dsi[2] = 5;  // an invalid dataset index is reported, not followed
  expect(orc_loglik_grad_batch(nds, q_off.data(), Q.data(), Robs.data(), Rerr.data(), dqqs, ni,
                               dsi.data(), row_off.data(), layers.data(), sc.data(), bk.data(), 1,
                               nthreads, ll.data(), gr.data(), gi.data()) == -1,
         "batch_bad_dataset", -1, 0);
}

}  // namespace

int main() {
  std::mt19937_64 g(2509069240ULL);
  double x[17], u[17], t[17], w[17], k[2];
  expect(orc_version() == 1, "version", 0, 0);
  expect(orc_gauss_legendre17(x, u) == 0, "gl17", 0, 0);
  expect(orc_smear_rule(0.05, t, w) == 17 && orc_smear_rule(0.0, t, w) == 1, "rule", 0, 0);
  expect(orc_smear_rule(-1.0, t, w) == -1, "rule_reject", 0, 0);
  expect(orc_kz(-4e-6, -0.0, k) == 0 && k[0] == 0.0, "kz_cut", 0, 0);
  expect(orc_kz(0.0, 0.0, k) == 0 && k[0] == 0.0 && k[1] == 0.0, "kz_zero", 0, 0);
  for (int L : {0, 1, 4, 12})
    for (int nq : {0, 1, 6})
      for (double dqq : {0.0, 0.05}) one_stack(g, L, nq, dqq, true);
  one_stack(g, 40, 3, 0.05, true);
  one_stack(g, 300, 4, 0.05, false);
  batch(g, 1);
  batch(g, 2);
  expect(orc_max_threads() >= 1, "threads", 0, 0);
  std::printf(g_fail ? "oracle sanitizer driver: FAILED\n" : "oracle sanitizer driver: ok\n");
  return g_fail;
}
