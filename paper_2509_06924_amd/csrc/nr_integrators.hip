// Element-wise kernels around the likelihood gradient: the leapfrog kick and
// drift of Hamiltonian Monte Carlo (Sec. 2.3, leapfrog equations), the
// reparameterised sampler and sample reduction of the variational ELBO
// gradient (Sec. 2.4, Monte-Carlo estimate of the loss and its gradient), and
// the gather-sum that ties co-fitted parameters (Sec. 4.2 shared parameters).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "nr_device.hpp"
#include "nr_internal.hpp"

namespace nr {

// Whether the model reads field f of a row of kind k (0 fronting: rho_re only;
// 1 finite layer: all four; 2 backing: no thickness).
__device__ __forceinline__ bool entry_read(uint8_t kind, int f) {
  return kind == 1 || (kind == 0 && f == 1) || (kind == 2 && f != 0);
}

// r <- r + h g over the packed rows and the instrument pairs.
__global__ __launch_bounds__(256) void k_kick(int64_t n_row_entries, int64_t n_inst,
                                              double* mom_rows, const double* g_rows,
                                              double* mom_inst, const double* g_inst, double h) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_row_entries) {
    mom_rows[i] = fma(h, g_rows[i], mom_rows[i]);
  } else if (i < n_row_entries + n_inst) {
    const int64_t j = i - n_row_entries;
    mom_inst[j] = fma(h, g_inst[j], mom_inst[j]);
  }
}

// theta <- theta + dt M^-1 r on every entry the model reads (M diagonal;
// identity when the inverse-mass arrays are null).
__global__ __launch_bounds__(256) void k_drift(int64_t n_row_entries, int64_t n_items,
                                               const uint8_t* row_kind, double* layers,
                                               double* scale, double* bkg,
                                               const double* mom_rows, const double* mom_inst,
                                               const double* im_rows, const double* im_inst,
                                               double dt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_row_entries) {
    if (!entry_read(row_kind[i >> 2], (int)(i & 3))) return;
    const double im = im_rows ? im_rows[i] : 1.0;
    layers[i] = fma(dt * im, mom_rows[i], layers[i]);
  } else if (i < n_row_entries + 2 * n_items) {
    const int64_t j = i - n_row_entries;
    const double im = im_inst ? im_inst[j] : 1.0;
    double* x = (j & 1) ? &bkg[j >> 1] : &scale[j >> 1];
    *x = fma(dt * im, mom_inst[j], *x);
  }
}

// softplus and its derivative, written to stay finite for large |w|.
__device__ __forceinline__ double softplus(double w) {
  return (w > 0.0) ? w + log1p(exp(-w)) : log1p(exp(w));
}
__device__ __forceinline__ double sigmoid(double w) {
  return (w >= 0.0) ? 1.0 / (1.0 + exp(-w)) : exp(w) / (1.0 + exp(w));
}

// theta_i = mu + softplus(omega) eps_i on variational entries (mask != 0),
// mu elsewhere, for every sample i.  P = entries per sample = rows*4 + 2.
__global__ __launch_bounds__(256) void k_vi_sample(int64_t n_samples, int P, int rows,
                                                   const double* mu, const double* omega,
                                                   const uint8_t* mask, const double* eps,
                                                   double* layers, double* scale, double* bkg) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_samples * P) return;
  const int64_t i = t / P;
  const int p = (int)(t - i * P);
  double v = mu[p];
  if (mask[p]) v = fma(softplus(omega[p]), eps[t], v);
  if (p < rows * 4)
    layers[i * rows * 4 + p] = v;
  else if (p == rows * 4)
    scale[i] = v;
  else
    bkg[i] = v;
}

// One thread per variational entry p: sums over samples in order.
//   dELBO/dmu_p    = mean_i g_ip
//   dELBO/domega_p = mean_i g_ip eps_ip s'(omega_p) + s'(omega_p)/s(omega_p)
// (the last term is the gradient of the entropy sum_p ln s(omega_p)); zero for
// entries outside the mask.  Thread P also forms the ELBO estimate
// mean_i logL_i + sum_p ln s(omega_p) (the Gaussian entropy up to its
// constant).
__global__ __launch_bounds__(256) void k_vi_reduce(int64_t n_samples, int P, int rows,
                                                   const double* omega, const uint8_t* mask,
                                                   const double* eps, const double* logL,
                                                   const double* g_rows, const double* g_inst,
                                                   double* grad_mu, double* grad_omega,
                                                   double* elbo) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) {
    if (!mask[p]) {
      grad_mu[p] = 0.0;
      grad_omega[p] = 0.0;
      return;
    }
    double gm = 0.0, ge = 0.0;
    for (int64_t i = 0; i < n_samples; ++i) {
      const double g = (p < rows * 4) ? g_rows[i * rows * 4 + p] : g_inst[i * 2 + (p - rows * 4)];
      gm += g;
      ge = fma(g, eps[i * P + p], ge);
    }
    const double inv = 1.0 / (double)n_samples;
    const double sp = sigmoid(omega[p]);
    const double s = softplus(omega[p]);
    grad_mu[p] = gm * inv;
    grad_omega[p] = ge * inv * sp + sp / s;
  } else if (p == P) {
    double ll = 0.0;
    for (int64_t i = 0; i < n_samples; ++i) ll += logL[i];
    double h = 0.0;
    for (int q = 0; q < P; ++q)
      if (mask[q]) h += log(softplus(omega[q]));
    *elbo = ll / (double)n_samples + h;
  }
}

// out[k] = sum over t in [first[k], first[k+1]) of in[src[t]], in order.
__global__ __launch_bounds__(256) void k_tie_sum(int64_t n_out, const int64_t* first,
                                                 const int64_t* src, const double* in,
                                                 double* out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_out) return;
  double s = 0.0;
  for (int64_t t = first[k]; t < first[k + 1]; ++t) s += in[src[t]];
  out[k] = s;
}

static dim3 grid_for(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_kick(int64_t n_row_entries, int64_t n_inst, double* mom_rows,
                       const double* g_rows, double* mom_inst, const double* g_inst, double h,
                       hipStream_t st) {
  const int64_t n = n_row_entries + n_inst;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kick, grid_for(n), dim3(256), 0, st, n_row_entries, n_inst, mom_rows,
                     g_rows, mom_inst, g_inst, h);
  return hipGetLastError();
}

hipError_t launch_drift(int64_t n_row_entries, int64_t n_items, const uint8_t* row_kind,
                        double* layers, double* scale, double* bkg, const double* mom_rows,
                        const double* mom_inst, const double* im_rows, const double* im_inst,
                        double dt, hipStream_t st) {
  const int64_t n = n_row_entries + 2 * n_items;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_drift, grid_for(n), dim3(256), 0, st, n_row_entries, n_items, row_kind,
                     layers, scale, bkg, mom_rows, mom_inst, im_rows, im_inst, dt);
  return hipGetLastError();
}

hipError_t launch_vi_sample(int64_t n_samples, int P, int rows, const double* mu,
                            const double* omega, const uint8_t* mask, const double* eps,
                            double* layers, double* scale, double* bkg, hipStream_t st) {
  const int64_t n = n_samples * P;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_vi_sample, grid_for(n), dim3(256), 0, st, n_samples, P, rows, mu, omega,
                     mask, eps, layers, scale, bkg);
  return hipGetLastError();
}

hipError_t launch_vi_reduce(int64_t n_samples, int P, int rows, const double* omega,
                            const uint8_t* mask, const double* eps, const double* logL,
                            const double* g_rows, const double* g_inst, double* grad_mu,
                            double* grad_omega, double* elbo, hipStream_t st) {
  hipLaunchKernelGGL(k_vi_reduce, grid_for((int64_t)P + 1), dim3(256), 0, st, n_samples, P, rows,
                     omega, mask, eps, logL, g_rows, g_inst, grad_mu, grad_omega, elbo);
  return hipGetLastError();
}

hipError_t launch_tie_sum(int64_t n_out, const int64_t* first, const int64_t* src,
                          const double* in, double* out, hipStream_t st) {
  if (n_out <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tie_sum, grid_for(n_out), dim3(256), 0, st, n_out, first, src, in, out);
  return hipGetLastError();
}

}  // namespace nr
