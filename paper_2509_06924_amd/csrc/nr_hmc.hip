// Per-chain kernels of the HMC driver (Sec. 2.3): momentum draws from the
// counter-based generator of nr_rng.hpp, the leapfrog kick and drift in the sampler's
// unconstrained coordinates, the Metropolis-Hastings accept, and the warm-up
// adaptation (Welford window of positions for the diagonal inverse mass, dual
// averaging of the step size).  One 64-lane workgroup per chain (= plan item);
// lanes stride over the chain's entries (4 per row, then scale and bkg), so
// per-chain sums are one wave reduction.  The likelihood gradient between
// drift and kick is the library's own nr_loglik_grad path.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "nr_device.hpp"
#include "nr_internal.hpp"
#include "nr_rng.hpp"

namespace nr {

namespace {

// One entry of a chain: where its coordinate, parameter, gradient and inverse
// mass live, and whether the sampler moves it (a transform other than FIXED,
// on an entry the model reads).
struct Ent {
  bool moving;
  int64_t k;  // index into the driver's entry arrays (rows, then instrument)
  double* z;
  double* th;
  double* g;
  double* im;
  uint8_t kind;
  double a, b;
};

__device__ Ent entry(const HmcArgs& h, int c, int64_t r0, int nrows, int e) {
  Ent t;
  if (e < 4 * nrows) {
    const int64_t i = 4 * r0 + e;
    t.kind = h.kind_rows[i];
    t.moving = t.kind != NR_TF_FIXED && row_entry_read(h.row_kind[r0 + (e >> 2)], e & 3);
    t.k = i;
    t.z = h.z_rows + i;
    t.th = h.layers + i;
    t.g = h.g_rows + i;
    t.im = h.im_rows + i;
    t.a = h.a_rows[i];
    t.b = h.b_rows[i];
  } else {
    const int j = e - 4 * nrows;
    const int64_t i = 2 * (int64_t)c + j;
    t.kind = h.kind_inst[i];
    t.moving = t.kind != NR_TF_FIXED;
    t.k = h.n_row_entries + i;
    t.z = h.z_inst + i;
    t.th = j ? h.bkg + c : h.scale + c;
    t.g = h.g_inst + i;
    t.im = h.im_inst + i;
    t.a = h.a_inst[i];
    t.b = h.b_inst[i];
  }
  return t;
}

// dU/dz = -(dlogL/dtheta dtheta/dz + d ln|dtheta/dz| / dz)
__device__ __forceinline__ double grad_U(const Ent& t, const Tf& f) {
  return -(*t.g * f.dtdz + f.dlogj);
}

struct ChainView {
  int c;
  int64_t r0;
  int nrows, n;
};

__device__ __forceinline__ ChainView chain_view(const HmcArgs& h) {
  ChainView v;
  v.c = blockIdx.x;
  v.r0 = h.row_off[v.c];
  v.nrows = (int)(h.row_off[v.c + 1] - v.r0);
  v.n = 4 * v.nrows + 2;
  return v;
}

// per-chain scalars of the driver (HmcArgs::cs, kChainScalars per chain)
enum { kH0 = 0, kU0, kLogL0, kWn, kDaMu, kDaLogBar, kDaHBar, kDaT };

}  // namespace

// theta <- T(z) (or z <- T^-1(theta) first) on moving entries.
__global__ __launch_bounds__(64) void k_hmc_theta(HmcArgs h, int from_theta) {
  const ChainView v = chain_view(h);
  for (int e = threadIdx.x; e < v.n; e += 64) {
    const Ent t = entry(h, v.c, v.r0, v.nrows, e);
    if (!t.moving) continue;
    if (from_theta) *t.z = inverse_transform_z(t.kind, t.a, t.b, *t.th);
    *t.th = transform_z(t.kind, t.a, t.b, *t.z).theta;
  }
}

// U = -logL - sum ln|dtheta/dz| at the current position.
__global__ __launch_bounds__(64) void k_hmc_potential(HmcArgs h) {
  const ChainView v = chain_view(h);
  double lj = 0.0;
  for (int e = threadIdx.x; e < v.n; e += 64) {
    const Ent t = entry(h, v.c, v.r0, v.nrows, e);
    if (t.moving) lj += transform_z(t.kind, t.a, t.b, *t.z).logj;
  }
  lj = wave_sum(lj);
  if (threadIdx.x == 0) h.U[v.c] = -h.logL[v.c] - lj;
}

// Start of a transition: draw r ~ N(0, M), keep the state for a rejection,
// H0 = U + r^T M^-1 r / 2, then the first half kick.
__global__ __launch_bounds__(64) void k_hmc_begin(HmcArgs h) {
  const ChainView v = chain_view(h);
  const uint64_t it = h.iter[v.c];
  const double dt = h.step[v.c];
  double kin = 0.0;
  for (int e = threadIdx.x; e < v.n; e += 64) {
    const Ent t = entry(h, v.c, v.r0, v.nrows, e);
    const double xi = rng_normal(h.seed, it, (uint64_t)v.c, e, kPurposeMomentum);
    const double im = *t.im;
    const bool live = t.moving && im > 0.0;
    double r = live ? xi * sqrt(1.0 / im) : 0.0;
    if (live) kin += im * (r * r);
    h.z0[t.k] = *t.z;
    h.g0[t.k] = *t.g;
    if (live) r -= (0.5 * dt) * grad_U(t, transform_z(t.kind, t.a, t.b, *t.z));
    h.r[t.k] = r;
  }
  kin = wave_sum(kin);
  if (threadIdx.x == 0) {
    double* cs = h.cs + (int64_t)kChainScalars * v.c;
    cs[kH0] = h.U[v.c] + 0.5 * kin;
    cs[kU0] = h.U[v.c];
    cs[kLogL0] = h.logL[v.c];
  }
}

// z <- z + dt M^-1 r; theta <- T(z).
__global__ __launch_bounds__(64) void k_hmc_drift(HmcArgs h) {
  const ChainView v = chain_view(h);
  const double dt = h.step[v.c];
  for (int e = threadIdx.x; e < v.n; e += 64) {
    const Ent t = entry(h, v.c, v.r0, v.nrows, e);
    const double im = *t.im;
    if (!(t.moving && im > 0.0)) continue;
    const double z = *t.z + (dt * im) * h.r[t.k];
    *t.z = z;
    *t.th = transform_z(t.kind, t.a, t.b, z).theta;
  }
}

// r <- r - frac dt dU/dz at the new position (frac 1/2 for the last kick of a
// transition, 1 where two half kicks meet).
__global__ __launch_bounds__(64) void k_hmc_kick(HmcArgs h, double frac) {
  const ChainView v = chain_view(h);
  const double hdt = frac * h.step[v.c];
  for (int e = threadIdx.x; e < v.n; e += 64) {
    const Ent t = entry(h, v.c, v.r0, v.nrows, e);
    if (!(t.moving && *t.im > 0.0)) continue;
    h.r[t.k] -= hdt * grad_U(t, transform_z(t.kind, t.a, t.b, *t.z));
  }
}

// End of a transition: energy error, divergence, Metropolis-Hastings accept
// (restore on rejection), statistics, and the adaptation updates.
__global__ __launch_bounds__(64) void k_hmc_end(HmcArgs h, int adapt) {
  const ChainView v = chain_view(h);
  const int lane = threadIdx.x;
  double* cs = h.cs + (int64_t)kChainScalars * v.c;
  double lj = 0.0, kin = 0.0;
  for (int e = lane; e < v.n; e += 64) {
    const Ent t = entry(h, v.c, v.r0, v.nrows, e);
    if (!t.moving) continue;
    lj += transform_z(t.kind, t.a, t.b, *t.z).logj;
    const double im = *t.im;
    const double r = h.r[t.k];
    if (im > 0.0) kin += im * (r * r);
  }
  lj = wave_sum(lj);
  kin = wave_sum(kin);
  const double U1 = -h.logL[v.c] - lj;
  const double delta = (U1 + 0.5 * kin) - cs[kH0];
  const bool divergent = !(delta <= h.max_energy_error);
  const double alpha = divergent ? 0.0 : fmin(1.0, exp(-delta));
  const uint64_t it = h.iter[v.c];
  const bool accept = rng_uniform(h.seed, it, (uint64_t)v.c, kPurposeAccept) < alpha;
  if (!accept) {
    for (int e = lane; e < v.n; e += 64) {
      const Ent t = entry(h, v.c, v.r0, v.nrows, e);
      *t.g = h.g0[t.k];
      if (!t.moving) continue;
      const double z = h.z0[t.k];
      *t.z = z;
      *t.th = transform_z(t.kind, t.a, t.b, z).theta;
    }
  }
  if (adapt & NR_HMC_ADAPT_MASS) {
    const double n = cs[kWn] + 1.0;
    for (int e = lane; e < v.n; e += 64) {
      const Ent t = entry(h, v.c, v.r0, v.nrows, e);
      if (!t.moving) continue;
      const double z = *t.z;
      const double d = z - h.wmean[t.k];
      const double m = h.wmean[t.k] + d / n;
      h.wmean[t.k] = m;
      h.wm2[t.k] += d * (z - m);
    }
  }
  if (lane == 0) {
    if (!accept) h.logL[v.c] = cs[kLogL0];
    h.U[v.c] = accept ? U1 : cs[kU0];
    h.accept_prob[v.c] = alpha;
    h.energy_error[v.c] = delta;
    h.n_accept[v.c] += accept ? 1 : 0;
    h.n_divergent[v.c] += divergent ? 1 : 0;
    h.iter[v.c] = it + 1;
    if (adapt & NR_HMC_ADAPT_MASS) cs[kWn] += 1.0;
    if (adapt & NR_HMC_ADAPT_STEP) {
      // dual averaging (Hoffman and Gelman 2014): gamma 0.05, t0 10, kappa 0.75
      const double t = cs[kDaT] + 1.0;
      const double w = 1.0 / (t + 10.0);
      const double hbar = (1.0 - w) * cs[kDaHBar] + w * (h.target_accept - alpha);
      const double log_eps = cs[kDaMu] - sqrt(t) / 0.05 * hbar;
      const double eta = pow(t, -0.75);
      cs[kDaLogBar] = eta * log_eps + (1.0 - eta) * cs[kDaLogBar];
      cs[kDaHBar] = hbar;
      cs[kDaT] = t;
      h.step[v.c] = exp(log_eps);
    }
  }
}

// Warm-up controls between transitions.
__global__ __launch_bounds__(64) void k_hmc_adapt(HmcArgs h, int actions) {
  const ChainView v = chain_view(h);
  double* cs = h.cs + (int64_t)kChainScalars * v.c;
  if (actions & NR_HMC_MASS_WINDOW_END) {
    const double n = cs[kWn];
    for (int e = threadIdx.x; e < v.n; e += 64) {
      const Ent t = entry(h, v.c, v.r0, v.nrows, e);
      if (t.moving && n >= 2.0) {
        const double var = h.wm2[t.k] / (n - 1.0);
        *t.im = (n / (n + 5.0)) * var + 1e-3 * (5.0 / (n + 5.0));
      }
      h.wmean[t.k] = 0.0;
      h.wm2[t.k] = 0.0;
    }
  }
  // the lane-0 updates read cs[kWn] above: all lanes are one wave, and the
  // loop's read precedes this write in every lane's program order
  if (threadIdx.x == 0) {
    if (actions & NR_HMC_MASS_WINDOW_END) cs[kWn] = 0.0;
    if (actions & NR_HMC_STEP_FINAL) h.step[v.c] = exp(cs[kDaLogBar]);
    if (actions & NR_HMC_STEP_RESTART) {
      cs[kDaMu] = log(10.0 * h.step[v.c]);
      cs[kDaLogBar] = 0.0;
      cs[kDaHBar] = 0.0;
      cs[kDaT] = 0.0;
    }
  }
}

hipError_t launch_hmc(int which, const HmcArgs& h, int arg, double frac, hipStream_t st) {
  if (h.n_items <= 0) return hipSuccess;
  const dim3 grid(h.n_items), block(64);
  switch (which) {
    case kHmcTheta:
      hipLaunchKernelGGL(k_hmc_theta, grid, block, 0, st, h, arg);
      break;
    case kHmcPotential:
      hipLaunchKernelGGL(k_hmc_potential, grid, block, 0, st, h);
      break;
    case kHmcBegin:
      hipLaunchKernelGGL(k_hmc_begin, grid, block, 0, st, h);
      break;
    case kHmcDrift:
      hipLaunchKernelGGL(k_hmc_drift, grid, block, 0, st, h);
      break;
    case kHmcKick:
      hipLaunchKernelGGL(k_hmc_kick, grid, block, 0, st, h, frac);
      break;
    case kHmcEnd:
      hipLaunchKernelGGL(k_hmc_end, grid, block, 0, st, h, arg);
      break;
    case kHmcAdapt:
      hipLaunchKernelGGL(k_hmc_adapt, grid, block, 0, st, h, arg);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nr
