// Kernels of the full-rank Gaussian VI fit (Sec. 2.4 VI; Sec. 4.2: a
// multivariate normal surrogate in unconstrained space, Adam, independent
// restarts).  The plan's items are R restarts x S draws (item = r S + s), all
// with the same rows; entry p of a draw is row entry p (4 per row), then
// scale, bkg.  Per restart the surrogate is z = mu + L eps with L lower
// triangular, L_ii = softplus(omega_i), L_ij = lambda_ij (i > j); only the
// moving entries (transform other than FIXED, read by the model) take part.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "nr_device.hpp"
#include "nr_internal.hpp"
#include "nr_rng.hpp"

namespace nr {

namespace {

__device__ __forceinline__ bool mvn_moving(const MvnArgs& v, int p) {
  if (v.kind[p] == NR_TF_FIXED) return false;
  if (p >= 4 * v.rows) return true;
  const int row = p >> 2, f = p & 3;
  if (row == 0) return f == 1;              // fronting: rho_re only
  if (row == v.rows - 1) return f != 0;     // backing: no thickness
  return true;
}

// theta of entry p of item `item` (its slot in the sample arrays)
__device__ __forceinline__ double* mvn_theta(const MvnArgs& v, int64_t item, int p) {
  if (p < 4 * v.rows) return v.layers + item * 4 * v.rows + p;
  return (p == 4 * v.rows) ? v.scale + item : v.bkg + item;
}

}  // namespace

// Draws and positions: eps (Philox, purpose 2), z = mu + L eps, theta = T(z)
// on moving entries, the fixed values elsewhere.  One workgroup per item.
__global__ __launch_bounds__(256) void k_mvn_sample(MvnArgs v) {
  __shared__ double eps_s[kMvnMaxEntries];
  const int64_t item = blockIdx.x;
  const int r = (int)(item / v.S);
  const int P = v.P;
  const uint64_t it = *v.iter;
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    const double e = mvn_moving(v, p) ? rng_normal(v.seed, it, (uint64_t)item, p, kPurposeVi)
                                      : 0.0;
    eps_s[p] = e;
    v.eps[item * P + p] = e;
  }
  __syncthreads();
  const double* mu = v.mu + (int64_t)r * P;
  const double* om = v.omega + (int64_t)r * P;
  const double* lam = v.lam + (int64_t)r * P * P;
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    double* th = mvn_theta(v, item, p);
    if (!mvn_moving(v, p)) {
      *th = v.theta_fixed[p];
      v.z[item * P + p] = 0.0;
      continue;
    }
    // row p of L times eps (eps of FIXED entries is 0)
    double z = mu[p];
    const double* lrow = lam + (int64_t)p * P;
    for (int j = 0; j < p; ++j) z = fma(lrow[j], eps_s[j], z);
    z = fma(softplus_d(om[p]), eps_s[p], z);
    v.z[item * P + p] = z;
    *th = transform_z(v.kind[p], v.a[p], v.b[p], z).theta;
  }
}

// After logL + gradient of every item: h = the z-gradient of the log target
// (dlogL/dtheta dtheta/dz + d ln|dtheta/dz|/dz) and f = logL + sum ln|dtheta/dz|.
__global__ __launch_bounds__(64) void k_mvn_chain(MvnArgs v) {
  const int64_t item = blockIdx.x;
  const int P = v.P;
  double lj = 0.0;
  for (int p = threadIdx.x; p < P; p += 64) {
    double hp = 0.0;
    if (mvn_moving(v, p)) {
      const Tf t = transform_z(v.kind[p], v.a[p], v.b[p], v.z[item * P + p]);
      const double g = (p < 4 * v.rows) ? v.g_rows[item * 4 * v.rows + p]
                                        : v.g_inst[2 * item + (p - 4 * v.rows)];
      hp = g * t.dtdz + t.dlogj;
      lj += t.logj;
    }
    v.h[item * P + p] = hp;
  }
  lj = wave_sum(lj);
  if (threadIdx.x == 0) v.f[item] = v.logL[item] + lj;
}

// Per restart r and coordinate i (one workgroup, lanes over j): the sums over
// the restart's S draws in order,
//   G_ij = (1/S) sum_s h_si eps_sj  ->  dELBO/dlambda_ij (j < i),
//   dELBO/dmu_i = mean_s h_si, dELBO/domega_i = (G_ii + 1/L_ii) sigmoid(omega_i);
// workgroup (r, 0) also forms the ELBO estimate
//   mean_s f_s + sum_i ln L_ii + (n/2) ln(2 pi e)   (n moving coordinates).
__global__ __launch_bounds__(64) void k_mvn_reduce(MvnArgs v) {
  const int r = blockIdx.x;
  const int i = blockIdx.y;
  const int P = v.P, S = v.S;
  const int64_t base = (int64_t)r * S;
  const double invS = 1.0 / (double)S;
  const bool mi = mvn_moving(v, i);
  double* glam = v.grad_lam + ((int64_t)r * P + i) * P;
  for (int j = threadIdx.x; j < P; j += 64) {
    if (j >= i) {
      if (j > i) glam[j] = 0.0;
      continue;
    }
    double acc = 0.0;
    if (mi && mvn_moving(v, j))
      for (int s = 0; s < S; ++s)
        acc = fma(v.h[(base + s) * P + i], v.eps[(base + s) * P + j], acc);
    glam[j] = acc * invS;
  }
  if (threadIdx.x == 0) {
    glam[i] = 0.0;
    double gm = 0.0, gd = 0.0;
    if (mi)
      for (int s = 0; s < S; ++s) {
        const double hv = v.h[(base + s) * P + i];
        gm += hv;
        gd = fma(hv, v.eps[(base + s) * P + i], gd);
      }
    const double w = v.omega[(int64_t)r * P + i];
    v.grad_mu[(int64_t)r * P + i] = mi ? gm * invS : 0.0;
    v.grad_omega[(int64_t)r * P + i] = mi ? (gd * invS + 1.0 / softplus_d(w)) * sigmoid_d(w) : 0.0;
  }
  if (i == 0 && threadIdx.x == 0) {
    double fs = 0.0;
    for (int s = 0; s < S; ++s) fs += v.f[base + s];
    double ld = 0.0;
    int n = 0;
    for (int p = 0; p < P; ++p)
      if (mvn_moving(v, p)) {
        ld += log(softplus_d(v.omega[(int64_t)r * P + p]));
        ++n;
      }
    v.elbo[r] = fs * invS + ld + 0.5 * n * log(2.0 * M_PI * M_E);
  }
}

// Adam ascent (Kingma and Ba 2015, Algorithm 1) of every restart's mu, omega
// and lambda below the diagonal, on moving coordinates; t = iteration + 1.
__global__ __launch_bounds__(256) void k_mvn_adam(MvnArgs v) {
  const int P = v.P;
  const int64_t per = 2 * (int64_t)P + (int64_t)P * P;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)v.R * per) return;
  const int64_t r = k / per;
  const int64_t o = k - r * per;
  double* x;
  const double* g;
  bool live;
  if (o < P) {
    x = v.mu + r * P + o;
    g = v.grad_mu + r * P + o;
    live = mvn_moving(v, (int)o);
  } else if (o < 2 * P) {
    x = v.omega + r * P + (o - P);
    g = v.grad_omega + r * P + (o - P);
    live = mvn_moving(v, (int)(o - P));
  } else {
    const int64_t q = o - 2 * P;
    const int i = (int)(q / P), j = (int)(q - (int64_t)i * P);
    x = v.lam + r * P * P + q;
    g = v.grad_lam + r * P * P + q;
    live = j < i && mvn_moving(v, i) && mvn_moving(v, j);
  }
  if (!live) return;
  const double t = (double)(*v.iter + 1);
  const double gv = *g;
  const double m = v.beta1 * v.adam_m[k] + (1.0 - v.beta1) * gv;
  const double s = v.beta2 * v.adam_v[k] + (1.0 - v.beta2) * gv * gv;
  v.adam_m[k] = m;
  v.adam_v[k] = s;
  const double mh = m / (1.0 - pow(v.beta1, t));
  const double vh = s / (1.0 - pow(v.beta2, t));
  *x += v.lr * mh / (sqrt(vh) + v.adam_eps);
}

__global__ void k_mvn_tick(uint64_t* iter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *iter += 1;
}

hipError_t launch_mvn(int which, const MvnArgs& v, hipStream_t st) {
  const int64_t items = (int64_t)v.R * v.S;
  if (items <= 0) return hipSuccess;
  switch (which) {
    case kMvnSample:
      hipLaunchKernelGGL(k_mvn_sample, dim3((unsigned)items), dim3(256), 0, st, v);
      break;
    case kMvnChain:
      hipLaunchKernelGGL(k_mvn_chain, dim3((unsigned)items), dim3(64), 0, st, v);
      break;
    case kMvnReduce:
      hipLaunchKernelGGL(k_mvn_reduce, dim3((unsigned)v.R, (unsigned)v.P), dim3(64), 0, st, v);
      break;
    case kMvnAdam: {
      const int64_t n = (int64_t)v.R * (2 * (int64_t)v.P + (int64_t)v.P * v.P);
      hipLaunchKernelGGL(k_mvn_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, v);
      break;
    }
    case kMvnTick:
      hipLaunchKernelGGL(k_mvn_tick, dim3(1), dim3(64), 0, st, v.iter);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nr
