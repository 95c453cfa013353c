// HIP kernels for gfx950: Abeles reflectivity with Nevot-Croce roughness,
// Gaussian resolution smearing, instrument scale/background, Gaussian
// log-likelihood, and the hand-written adjoint of the whole chain.
//
// Work decomposition: one work unit (WU) = one item x up to 64 consecutive data
// points of its dataset, one wave (64 lanes) per WU, lane = data point.  The
// item is wave-uniform, so its per-layer constants (precomputed per item by a
// small prologue kernel) are read with scalar loads into scalar registers.  A lane walks all quadrature nodes of its point; for
// each node it runs the layer product bottom-up (substrate -> surface), then
// the adjoint top down, and accumulates w_k dR(q_k)/d(theta) in registers;
// the point's likelihood seed multiplies the accumulators once at the end.
//
// The layer product is written in a scaled form: the Abeles column
// v_j = C_j v_{j+1} is divided by E_j at every layer, which leaves r = v1/v0
// unchanged and turns the phase factor into e_j = E_j^-2 = exp(-2 i kz_j d_j),
// whose modulus is <= 1 on the chosen branch (Im kz <= 0):
//   P <- P + r'_j Qv,   Qv <- e_j (r'_j P + Qv),   starting from (1, 0).
//
// Two gradient variants (one source, selected by template):
//   store     - the forward sweep keeps each level's state (P, Qv) and phase
//               e_j in LDS and each medium's kz_j, 1/|kz_j|^2 and interface
//               coefficients in registers; the adjoint recomputes nothing.
//   recompute - for deep stacks: the state tape stays in registers and the
//               adjoint recomputes every layer's wavevector and phase.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "nr_device.hpp"
#include "nr_internal.hpp"

namespace nr {

// ---------------------------------------------------------------------------
// Per-item layer records, written by k_item_consts into the workspace (six
// doubles per medium m = 0..N+1, indexed like the item's rows) and read by the
// main kernels with scalar loads, since every lane of a wave uses the same
// item:
//   A  = 4 pi (rho_re,m - rho_re,0)        (0 for the fronting medium)
//   B  = 4 pi |rho_im,m|                   (0 for the fronting: lossless)
//   Nr + i Ni = w_m - w_{m+1} = (A_{m+1} - A_m) + i (B_{m+1} - B_m), the
//        Q-independent numerator of r_m = (w_m - w_{m+1}) / (kz_m + kz_{m+1})^2
//   C  = -2 sigma_{m+1}^2                  (Nevot-Croce exponent factor)
//   D  = 2 d_m                             (layers 1..N)
// Interface fields of the backing record are 0.
// ---------------------------------------------------------------------------
constexpr int kRec = 6;

struct Layers {
  const double* rec;  // the item's records
  int z;              // an opaque zero (see opaque_zero)
  __device__ __forceinline__ double at(int m, int f) const { return rec[(m + z) * kRec + f]; }
  __device__ __forceinline__ double A(int m) const { return at(m, 0); }
  __device__ __forceinline__ double B(int m) const { return at(m, 1); }
  __device__ __forceinline__ double Nr(int m) const { return at(m, 2); }
  __device__ __forceinline__ double Ni(int m) const { return at(m, 3); }
  __device__ __forceinline__ double C(int m) const { return at(m, 4); }
  __device__ __forceinline__ double D(int m) const { return at(m, 5); }
};

// Layer records are indexed with (m + z) where z = k & KernelArgs::zero_mask
// (the mask is 0): z is 0 at run time but varies with the node counter k as
// far as the compiler can tell, so the records are re-read (with scalar
// loads) inside the node loop instead of being hoisted out of it, which would
// need far more scalar registers than exist.

// One block of 64 per item, one lane per medium.
__global__ __launch_bounds__(64) void k_item_consts(const int64_t* row_off, const double* layers,
                                                    double* rec, int n_items) {
  const int b = blockIdx.x;
  const int m = threadIdx.x;
  if (b >= n_items) return;
  const int64_t r0 = row_off[b];
  const int NR = (int)(row_off[b + 1] - r0);
  if (m >= NR) return;
  const double* rows = layers + 4 * r0;
  const double rho0 = rows[1];
  auto Af = [&](int j) { return (j == 0) ? 0.0 : kFourPi * (rows[4 * j + 1] - rho0); };
  auto Bf = [&](int j) { return (j == 0) ? 0.0 : kFourPi * fabs(rows[4 * j + 2]); };
  double* out = rec + (r0 + m) * kRec;
  const double A = Af(m), B = Bf(m);
  out[0] = A;
  out[1] = B;
  if (m + 1 < NR) {
    const double sg = rows[4 * (m + 1) + 3];
    out[2] = Af(m + 1) - A;
    out[3] = Bf(m + 1) - B;
    out[4] = -2.0 * (sg * sg);
  } else {
    out[2] = 0.0;
    out[3] = 0.0;
    out[4] = 0.0;
  }
  out[5] = 2.0 * rows[4 * m];
}

// The quadrature rule and the exp/sincos tables, staged per block in LDS.
struct Shared {
  double t[kSmearNodes], w[kSmearNodes];
  MathTables tab;
};

// Reads of staged LDS values that every lane shares are volatile so that the
// compiler re-reads them at each use instead of holding them in registers.
typedef __attribute__((address_space(3))) const volatile double lds_cv_double;
__device__ __forceinline__ double ld(const double& x) { return *(lds_cv_double*)(&x); }

__device__ __forceinline__ void stage_shared(Shared& s, int lane, const double* rule) {
  if (lane < kSmearNodes) {
    s.t[lane] = rule[lane];
    s.w[lane] = rule[kSmearNodes + lane];
  }
  // tables follow the rule in the same device buffer
  const double* tb = rule + 2 * kSmearNodes;
  s.tab.sc[lane][0] = tb[2 * lane];
  s.tab.sc[lane][1] = tb[2 * lane + 1];
  s.tab.e2[lane] = tb[128 + lane];
  __syncthreads();
}

// Interface quantities shared by the forward and adjoint sweeps.
struct Iface {
  cd s;   // 1/(kz_j + kz_{j+1})
  cd r;   // Fresnel coefficient
  cd f;   // Nevot-Croce factor
  cd rp;  // r f
  cd kk;  // kz_j kz_{j+1}
};

__device__ __forceinline__ Iface interface_coeffs(const MathTables& T, cd kzc, cd kzn, double Nr,
                                                  double Ni, double C) {
  Iface o;
  o.s = crecip(kzc + kzn);
  const cd s2 = o.s * o.s;
  // identical media: r = 0 exactly (also avoids 0 * inf when both kz vanish)
  o.r = (Nr == 0.0 && Ni == 0.0) ? mk(0.0, 0.0) : mk(Nr, Ni) * s2;
  o.kk = kzc * kzn;
  o.f = cexp_tab(T, C * o.kk);
  o.rp = o.r * o.f;
  return o;
}

// e_j = exp(-2 i kz_j d_j) = exp(D Im kz) cis(-D Re kz), D = 2 d_j.
__device__ __forceinline__ cd layer_phase(const MathTables& T, cd kz, double D) {
  return cexp_tab(T, mk(D * kz.im, -D * kz.re));
}

__device__ __forceinline__ Root medium_root(const Layers& L, double kz0sq, int m) {
  return kz_root(kz_real_part(kz0sq, L.A(m)), -L.B(m));
}

// ---------------------------------------------------------------------------
// Forward-only reflectivity of one node (no state kept; runtime layer loop).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double node_reflectivity(const MathTables& T, const Layers& L, int N,
                                                    double q) {
  const double kz0sq = kz0_squared(q);
  cd kzn = medium_root(L, kz0sq, N + 1).kz;
  cd P = mk(1.0, 0.0), Qv = mk(0.0, 0.0);
  for (int jj = N; jj >= 1; --jj) {
    const cd kzc = medium_root(L, kz0sq, jj).kz;
    const Iface it = interface_coeffs(T, kzc, kzn, L.Nr(jj), L.Ni(jj), L.C(jj));
    const cd Pn = P + it.rp * Qv;
    const cd t = it.rp * P + Qv;
    Qv = layer_phase(T, kzc, L.D(jj)) * t;
    P = Pn;
    kzn = kzc;
  }
  {
    const Iface it = interface_coeffs(T, mk(0.5 * q, 0.0), kzn, L.Nr(0), L.Ni(0), L.C(0));
    const cd Pn = P + it.rp * Qv;
    Qv = it.rp * P + Qv;
    P = Pn;
  }
  return cabs2(Qv * crecip(P));
}

// Shared WU prologue.
struct WuInfo {
  int item, ds, N, nq, i;
  int64_t qoff, roff;
  bool active;
  double Q, dqq;
};

__device__ __forceinline__ WuInfo wu_setup(const KernelArgs& a, int w, int lane) {
  WuInfo u;
  u.item = a.wu_item[w];
  const int p0 = a.wu_p0[w];
  u.ds = a.dataset_of_item[u.item];
  u.qoff = a.q_off[u.ds];
  u.nq = (int)(a.q_off[u.ds + 1] - u.qoff);
  u.roff = a.row_off[u.item];
  u.N = (int)(a.row_off[u.item + 1] - u.roff) - 2;
  u.i = p0 + lane;
  u.active = u.i < u.nq;
  // idle lanes evaluate the WU's first point and discard the result
  u.Q = a.q[u.qoff + (u.active ? u.i : p0)];
  u.dqq = a.dq_over_q[u.ds];
  return u;
}

// Tail work units pack the last partial group of points of several items of
// equal depth into one wave: lane l evaluates point tail_pt[l] of item
// tail_item[l]; the lanes of one item are contiguous and share its tail
// record offset tail_rec[l] (idle lanes have tail_rec = -1 and repeat lane
// 0's point).  The depth is wave-uniform and taken from wu_item[w].
__device__ __forceinline__ WuInfo tail_setup(const KernelArgs& a, int w, int lane) {
  WuInfo u;
  const int first = a.wu_item[w];
  u.N = (int)(a.row_off[first + 1] - a.row_off[first]) - 2;
  const int64_t slot = (int64_t)w * 64 + lane;
  u.active = a.tail_rec[slot] >= 0;
  u.item = a.tail_item[slot];
  u.i = a.tail_pt[slot];
  u.ds = a.dataset_of_item[u.item];
  u.qoff = a.q_off[u.ds];
  u.nq = (int)(a.q_off[u.ds + 1] - u.qoff);
  u.roff = a.row_off[u.item];
  u.Q = a.q[u.qoff + u.i];
  u.dqq = a.dq_over_q[u.ds];
  return u;
}

__device__ __forceinline__ void flag(int32_t* status, int item, uint32_t bits) {
  if (status != nullptr && bits != 0u)
    atomicOr(reinterpret_cast<unsigned int*>(status + item), bits);
}

// ---------------------------------------------------------------------------
// R_hat per point (nr_reflectivity).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_reflectivity(KernelArgs a) {
  __shared__ Shared s;
  const int lane = threadIdx.x;
  const int w = blockIdx.x;
  const WuInfo u = wu_setup(a, w, lane);
  stage_shared(s, lane, a.rule);
  const double* lrec = a.consts + u.roff * kRec;
  const int K = (u.dqq > 0.0) ? kSmearNodes : 1;
  double Rsm = 0.0;
  bool badq = !(u.Q > 0.0);
  for (int k = 0; k < K; ++k) {
    const double q = (K == 1) ? u.Q : smear_node(u.Q, u.dqq, ld(s.t[k]));
    badq |= !(q > 0.0);
    const double wk = (K == 1) ? 1.0 : ld(s.w[k]);
    const Layers L{lrec, k & a.zero_mask};
    Rsm += wk * node_reflectivity(s.tab, L, u.N, q);
  }
  if (u.active) {
    double Rhat = a.scale[u.item] * Rsm + a.bkg[u.item];
    uint32_t bits = 0;
    if (badq) {
      Rhat = __builtin_nan("");
      bits |= kItemBadQ;
    }
    if (!isfinite(Rhat)) bits |= kItemNonfinite;
    flag(a.item_status, u.item, bits);
    a.out[a.out_off[u.item] + u.i] = Rhat;
  }
}

// Log-likelihood term of one point; sets status bits.
__device__ __forceinline__ double point_loglik(double Rhat, double Robs, double e, bool badq,
                                               uint32_t& bits) {
  const double z = (Rhat - Robs) / e;
  double ll = -0.5 * (z * z) - log(e) - kHalfLn2Pi;
  if (!(e > 0.0) || !isfinite(e)) bits |= kItemBadErr;
  if (badq) bits |= kItemBadQ;
  if (bits) ll = __builtin_nan("");
  if (!isfinite(ll)) bits |= kItemNonfinite;
  return ll;
}

// ---------------------------------------------------------------------------
// logL partial per WU (nr_loglik): record = 1 double.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_loglik(KernelArgs a) {
  __shared__ Shared s;
  const int lane = threadIdx.x;
  const int w = blockIdx.x;
  const WuInfo u = wu_setup(a, w, lane);
  stage_shared(s, lane, a.rule);
  const double* lrec = a.consts + u.roff * kRec;
  const int K = (u.dqq > 0.0) ? kSmearNodes : 1;
  double Rsm = 0.0;
  bool badq = !(u.Q > 0.0);
  for (int k = 0; k < K; ++k) {
    const double q = (K == 1) ? u.Q : smear_node(u.Q, u.dqq, ld(s.t[k]));
    badq |= !(q > 0.0);
    const double wk = (K == 1) ? 1.0 : ld(s.w[k]);
    const Layers L{lrec, k & a.zero_mask};
    Rsm += wk * node_reflectivity(s.tab, L, u.N, q);
  }
  double ll = 0.0;
  uint32_t bits = 0;
  if (u.active) {
    const double Rhat = a.scale[u.item] * Rsm + a.bkg[u.item];
    ll = point_loglik(Rhat, a.r_obs[u.qoff + u.i], a.r_err[u.qoff + u.i], badq, bits);
  }
  flag(a.item_status, u.item, bits);
  ll = wave_sum(ll);
  if (lane == 0) a.rec[a.wu_rec[w]] = ll;
}

// ---------------------------------------------------------------------------
// Adjoint of one interface/layer step (shared by both gradient variants).
// In: state (Ps, Qs) entering level j (= state of level j+1), cotangents
// (Pb, Qb) of the state leaving level j, kz_j, kz_{j+1}, the interface
// coefficients, the phase e_j (j >= 1).  Out: cotangents of the state entering
// the level, kzbar contributions, and the d / sigma accumulators.
// ---------------------------------------------------------------------------
struct AdjStep {
  cd Pb, Qb;   // cotangents of the state entering level j
  cd kzb_c;    // contribution to kzbar_j
  cd kzb_n;    // contribution to kzbar_{j+1}
  double dd;   // dl/dd_j
  double ss;   // Re(conj(ubar) kz_j kz_{j+1})  (times -4 sigma_{j+1} later)
};

__device__ __forceinline__ AdjStep adjoint_step(cd Ps, cd Qs, cd Pb, cd Qb, cd kzc, cd kzn,
                                                const Iface& it, double C, bool has_phase, cd e,
                                                double D) {
  AdjStep o;
  const cd t = it.rp * Ps + Qs;
  cd tb, eb = mk(0.0, 0.0);
  if (has_phase) {
    eb = cmulc(t, Qb);
    tb = cmulc(e, Qb);
  } else {
    tb = Qb;
  }
  // P_new = P + r' Qv ; t = r' P + Qv
  const cd rpb = cmulc(Qs, Pb) + cmulc(Ps, tb);
  o.Pb = Pb + cmulc(it.rp, tb);
  o.Qb = cmulc(it.rp, Pb) + tb;
  // r' = r f, f = exp(C kz_j kz_{j+1})
  const cd rb = cmulc(it.f, rpb);
  const cd ub = cmulc(it.rp, rpb);
  o.ss = ub.re * it.kk.re + ub.im * it.kk.im;
  // r = (kz_j - kz_{j+1}) s: dr/dkz_j = 2 kz_{j+1} s^2, dr/dkz_{j+1} = -2 kz_j s^2
  const cd s2 = it.s * it.s;
  o.kzb_c = cmulc(C * kzn, ub) + cmulc(2.0 * (kzn * s2), rb);
  o.kzb_n = cmulc(C * kzc, ub) + cmulc(-2.0 * (kzc * s2), rb);
  o.dd = 0.0;
  if (has_phase) {
    // e = exp(-2 i kz d): de/dkz = -i D e, de/dd = -2 i kz e
    o.kzb_c += cmulc(mk(D * e.im, -D * e.re), eb);
    const cd ze = kzc * e;
    o.dd = eb.re * (2.0 * ze.im) + eb.im * (-2.0 * ze.re);
  }
  return o;
}

// wbar = conj(dkz/dw) kzbar = conj(1/(2 kz)) kzbar = kz kzbar / (2 |kz|^2)
__device__ __forceinline__ cd wbar_of(cd kz, double inv_abs2, cd kzb) {
  return (0.5 * inv_abs2) * (kz * kzb);
}

// Per-lane gradient accumulators for one point: sum_k w_k dR(q_k)/d(.)
template <int LMAX>
struct Accum {
  cd Hw[LMAX + 2];
  double Hd[LMAX + 2], Hs[LMAX + 2];
};

template <int LMAX>
struct GradTape {
  // per-lane state entering each level and the layer phase, lane-minor
  double2 P[LMAX + 1][64], Qv[LMAX + 1][64], E[LMAX + 1][64];
};

__device__ __forceinline__ double2 to_d2(cd z) { return make_double2(z.re, z.im); }
__device__ __forceinline__ cd from_d2(double2 v) { return mk(v.x, v.y); }

// ---------------------------------------------------------------------------
// One node, store variant: forward with the tape in LDS and kz in registers,
// then the adjoint.  Returns R(q) and adds w_k dR/d(.) to the accumulators.
// ---------------------------------------------------------------------------
template <int LMAX>
__device__ __forceinline__ double node_grad_store(const MathTables& T, const Layers& L,
                                                  GradTape<LMAX>& tp, Accum<LMAX>& acc, int N,
                                                  int lane, double q, double wk) {
  const double kz0sq = kz0_squared(q);
  cd kz[LMAX + 2];
  double ia[LMAX + 2];
  Iface ifc[LMAX + 1];
  cd P = mk(1.0, 0.0), Qv = mk(0.0, 0.0);
#pragma unroll
  for (int jj = LMAX + 1; jj >= 0; --jj) {
    if (jj == N + 1) {
      const Root rt = medium_root(L, kz0sq, jj);
      kz[jj] = rt.kz;
      ia[jj] = rt.inv_abs2;
    } else if (jj <= N) {
      if (jj == 0) {
        kz[0] = mk(0.5 * q, 0.0);
        ia[0] = 0.0;
      } else {
        const Root rt = medium_root(L, kz0sq, jj);
        kz[jj] = rt.kz;
        ia[jj] = rt.inv_abs2;
      }
      const Iface it =
          interface_coeffs(T, kz[jj], kz[jj + 1], L.Nr(jj), L.Ni(jj), L.C(jj));
      ifc[jj] = it;
      tp.P[jj][lane] = to_d2(P);
      tp.Qv[jj][lane] = to_d2(Qv);
      const cd Pn = P + it.rp * Qv;
      const cd t = it.rp * P + Qv;
      if (jj >= 1) {
        const cd e = layer_phase(T, kz[jj], L.D(jj));
        tp.E[jj][lane] = to_d2(e);
        Qv = e * t;
      } else {
        Qv = t;
      }
      P = Pn;
    }
  }
  const cd iP = crecip(P);
  const cd r = Qv * iP;
  const cd rbar = (2.0 * wk) * r;
  cd Pb = cmulc(-(r * iP), rbar);  // conj(dr/dP) rbar, dr/dP = -r/P
  cd Qb = cmulc(iP, rbar);         // conj(dr/dQv) rbar, dr/dQv = 1/P
  cd kzbc = mk(0.0, 0.0);
#pragma unroll
  for (int jj = 0; jj <= LMAX; ++jj) {
    if (jj <= N) {
      const double C = L.C(jj);
      const Iface& it = ifc[jj];
      const cd Ps = from_d2(tp.P[jj][lane]);
      const cd Qs = from_d2(tp.Qv[jj][lane]);
      const bool ph = jj >= 1;
      const cd e = ph ? from_d2(tp.E[jj][lane]) : mk(1.0, 0.0);
      const AdjStep st =
          adjoint_step(Ps, Qs, Pb, Qb, kz[jj], kz[jj + 1], it, C, ph, e, ph ? L.D(jj) : 0.0);
      kzbc += st.kzb_c;
      acc.Hs[jj + 1] += st.ss;
      if (ph) {
        acc.Hd[jj] += st.dd;
        acc.Hw[jj] += wbar_of(kz[jj], ia[jj], kzbc);
      }
      if (jj == N) acc.Hw[jj + 1] += wbar_of(kz[jj + 1], ia[jj + 1], st.kzb_n);
      Pb = st.Pb;
      Qb = st.Qb;
      kzbc = st.kzb_n;
    }
  }
  return cabs2(r);
}

// ---------------------------------------------------------------------------
// One node, recompute variant: the state tape stays in registers; the adjoint
// recomputes each medium's wavevector and each layer's phase.
// ---------------------------------------------------------------------------
template <int LMAX>
__device__ __forceinline__ double node_grad_recompute(const MathTables& T, const Layers& L,
                                                      Accum<LMAX>& acc, int N, double q,
                                                      double wk) {
  const double kz0sq = kz0_squared(q);
  const cd kz0 = mk(0.5 * q, 0.0);
  cd tapeP[LMAX + 1], tapeQ[LMAX + 1];
  cd kzn = medium_root(L, kz0sq, N + 1).kz;
  cd P = mk(1.0, 0.0), Qv = mk(0.0, 0.0);
#pragma unroll
  for (int jj = LMAX; jj >= 0; --jj) {
    if (jj <= N) {
      const cd kzc = (jj == 0) ? kz0 : medium_root(L, kz0sq, jj).kz;
      tapeP[jj] = P;
      tapeQ[jj] = Qv;
      const Iface it = interface_coeffs(T, kzc, kzn, L.Nr(jj), L.Ni(jj), L.C(jj));
      const cd Pn = P + it.rp * Qv;
      const cd t = it.rp * P + Qv;
      Qv = (jj >= 1) ? layer_phase(T, kzc, L.D(jj)) * t : t;
      P = Pn;
      kzn = kzc;
    }
    __builtin_amdgcn_sched_barrier(0x0100);  // only LDS reads may move across
  }
  const cd iP = crecip(P);
  const cd r = Qv * iP;
  const cd rbar = (2.0 * wk) * r;
  cd Pb = cmulc(-(r * iP), rbar);
  cd Qb = cmulc(iP, rbar);
  cd kzc = kz0;
  double iac = 0.0;
  cd kzbc = mk(0.0, 0.0);
#pragma unroll
  for (int jj = 0; jj <= LMAX; ++jj) {
    if (jj <= N) {
      const Root rn = medium_root(L, kz0sq, jj + 1);
      const double C = L.C(jj);
      const Iface it = interface_coeffs(T, kzc, rn.kz, L.Nr(jj), L.Ni(jj), C);
      const bool ph = jj >= 1;
      const double D = ph ? L.D(jj) : 0.0;
      const cd e = ph ? layer_phase(T, kzc, D) : mk(1.0, 0.0);
      const AdjStep st = adjoint_step(tapeP[jj], tapeQ[jj], Pb, Qb, kzc, rn.kz, it, C, ph, e, D);
      kzbc += st.kzb_c;
      acc.Hs[jj + 1] += st.ss;
      if (ph) {
        acc.Hd[jj] += st.dd;
        acc.Hw[jj] += wbar_of(kzc, iac, kzbc);
      }
      if (jj == N) acc.Hw[jj + 1] += wbar_of(rn.kz, rn.inv_abs2, st.kzb_n);
      Pb = st.Pb;
      Qb = st.Qb;
      kzc = rn.kz;
      iac = rn.inv_abs2;
      kzbc = st.kzb_n;
    }
    __builtin_amdgcn_sched_barrier(0x0100);  // only LDS reads may move across
  }
  return cabs2(r);
}

// ---------------------------------------------------------------------------
// logL + gradient partials per WU (nr_loglik_grad).
// Record layout (NR = N + 2 media):
//   [0] logL, [1] d/dscale, [2] d/dbkg,
//   [3 + m]        sum Re wbar_m     (wbar_m = cotangent of w_m = kz_m^2)
//   [3 + NR + m]   sum Im wbar_m
//   [3 + 2NR + m]  sum dl/dd_m
//   [3 + 3NR + m]  sum Re(conj(ubar) kz_{m-1} kz_m)   (sigma_m factor applied later)
// ---------------------------------------------------------------------------
template <int LMAX, bool STORE, bool TAIL>
__global__ __launch_bounds__(64) void k_loglik_grad(KernelArgs a) {
  __shared__ Shared s;
  using Tape = typename std::conditional<STORE, GradTape<LMAX>, char>::type;
  __shared__ Tape tape;
  const int lane = threadIdx.x;
  const int w = blockIdx.x;
  const WuInfo u = TAIL ? tail_setup(a, w, lane) : wu_setup(a, w, lane);
  stage_shared(s, lane, a.rule);
  const double* lrec = a.consts + u.roff * kRec;
  const int N = u.N;
  const int K = (u.dqq > 0.0) ? kSmearNodes : 1;

  Accum<LMAX> acc;
#pragma unroll
  for (int m = 0; m < LMAX + 2; ++m) {
    acc.Hw[m] = mk(0.0, 0.0);
    acc.Hd[m] = 0.0;
    acc.Hs[m] = 0.0;
  }

  double Rsm = 0.0;
  bool badq = !(u.Q > 0.0);
  for (int k = 0; k < K; ++k) {
    const double q = (K == 1) ? u.Q : smear_node(u.Q, u.dqq, ld(s.t[k]));
    badq |= !(q > 0.0);
    const double wk = (K == 1) ? 1.0 : ld(s.w[k]);
    const Layers L{lrec, k & a.zero_mask};
    double R;
    if constexpr (STORE)
      R = node_grad_store<LMAX>(s.tab, L, tape, acc, N, lane, q, wk);
    else
      R = node_grad_recompute<LMAX>(s.tab, L, acc, N, q, wk);
    Rsm += wk * R;
  }

  // ---- instrument, likelihood, seeds ----
  double ll = 0.0, gsc = 0.0, gbk = 0.0, fac = 0.0;
  uint32_t bits = 0;
  if (u.active) {
    const double sc = a.scale[u.item];
    const double Rhat = sc * Rsm + a.bkg[u.item];
    const double e = a.r_err[u.qoff + u.i];
    ll = point_loglik(Rhat, a.r_obs[u.qoff + u.i], e, badq, bits);
    const double ghat = -(Rhat - a.r_obs[u.qoff + u.i]) / (e * e);
    gsc = ghat * Rsm;
    gbk = ghat;
    fac = ghat * sc;
  }
  flag(a.item_status, u.item, bits);

  const int NR = N + 2;
  const int nf = 3 + 4 * NR;
  if constexpr (TAIL) {
    // Lanes of one item are contiguous; idle lanes (key -1) follow the last
    // item.  A segmented inclusive scan over the lanes leaves each item's
    // sums in its last lane, which writes the item's tail record.
    const int key = u.active ? u.item : -1;
    bool take[6];
#pragma unroll
    for (int s6 = 0; s6 < 6; ++s6) {
      const int off = 1 << s6;
      // every lane takes part in the shuffle (it must not sit behind the
      // lane test, which would leave its source lanes inactive)
      const int kp = __shfl_up(key, off, 64);
      take[s6] = (lane >= off) && (kp == key);
    }
    const int key_next = __shfl_down(key, 1, 64);
    const bool writer = u.active && (lane == 63 || key_next != key);
    double* rec = a.rec + a.tail_rec[(int64_t)w * 64 + lane];
    auto seg_put = [&](int f, double v) {
#pragma unroll
      for (int s6 = 0; s6 < 6; ++s6) {
        const double o = __shfl_up(v, 1 << s6, 64);
        if (take[s6]) v += o;
      }
      if (writer) rec[f] = v;
    };
    seg_put(0, ll);
    seg_put(1, gsc);
    seg_put(2, gbk);
#pragma unroll
    for (int m = 0; m < LMAX + 2; ++m) {
      if (m < NR) {
        seg_put(3 + m, fac * acc.Hw[m].re);
        seg_put(3 + NR + m, fac * acc.Hw[m].im);
        seg_put(3 + 2 * NR + m, fac * acc.Hd[m]);
        seg_put(3 + 3 * NR + m, fac * acc.Hs[m]);
      }
    }
    return;
  }
  // ---- wave reduction; the sums go through LDS into one coalesced store ----
  __shared__ double stage[3 + 4 * (LMAX + 2)];
  ll = wave_sum(ll);
  gsc = wave_sum(gsc);
  gbk = wave_sum(gbk);
  if (lane == 0) {
    stage[0] = ll;
    stage[1] = gsc;
    stage[2] = gbk;
  }
#pragma unroll
  for (int m = 0; m < LMAX + 2; ++m) {
    if (m < NR) {
      const double wr = wave_sum(fac * acc.Hw[m].re);
      const double wi = wave_sum(fac * acc.Hw[m].im);
      const double dd = wave_sum(fac * acc.Hd[m]);
      const double ss = wave_sum(fac * acc.Hs[m]);
      if (lane == 0) {
        stage[3 + m] = wr;
        stage[3 + NR + m] = wi;
        stage[3 + 2 * NR + m] = dd;
        stage[3 + 3 * NR + m] = ss;
      }
    }
  }
  __syncthreads();
  double* rec = a.rec + a.wu_rec[w];
  for (int f = lane; f < nf; f += 64) rec[f] = stage[f];
}

// ---------------------------------------------------------------------------
// Deterministic per-item reductions of the WU records.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce_loglik(ReduceArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.n_items) return;
  const int64_t first = a.item_wu_first[b];
  const int cnt = a.item_wu_count[b];
  double s = 0.0;
  for (int k = 0; k < cnt; ++k) s += a.rec[a.rec_of_wu[first + k]];
  a.logL[b] = s;
}

// One wave per item: lanes sum record fields over the item's WUs, then turn
// the sums into gradients of the row entries.
__global__ __launch_bounds__(64) void k_reduce_grad(ReduceArgs a) {
  extern __shared__ double fsum[];
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t first = a.item_wu_first[b];
  const int cnt = a.item_wu_count[b];
  const int64_t roff = a.row_off[b];
  const int NR = (int)(a.row_off[b + 1] - roff);
  const int nf = 3 + 4 * NR;
  for (int f = lane; f < nf; f += 64) {
    double v = 0.0;
    for (int k = 0; k < cnt; ++k) v += a.rec[a.rec_of_wu[first + k] + f];
    fsum[f] = v;
  }
  __syncthreads();
  const double* rows = a.layers + 4 * roff;
  double* g = a.g_rows + 4 * roff;
  for (int m = lane; m < NR; m += 64) {
    const double wr = fsum[3 + m], wi = fsum[3 + NR + m];
    const double dd = fsum[3 + 2 * NR + m], ss = fsum[3 + 3 * NR + m];
    double gd = 0.0, gre = 0.0, gim = 0.0, gsig = 0.0;
    if (m >= 1) {
      gre = -kFourPi * wr;
      const double sgn = (rows[4 * m + 2] < 0.0) ? -1.0 : 1.0;
      gim = -kFourPi * sgn * wi;
      gsig = -4.0 * rows[4 * m + 3] * ss;
      if (m <= NR - 2) gd = dd;
    }
    g[4 * m + 0] = gd;
    g[4 * m + 1] = gre;
    g[4 * m + 2] = gim;
    g[4 * m + 3] = gsig;
  }
  // fronting rho_re: the model depends on rho_re,m - rho_re,0 only
  double part = 0.0;
  for (int m = 1 + lane; m < NR; m += 64) part += fsum[3 + m];
  part = wave_sum(part);
  if (lane == 0) {
    g[1] = kFourPi * part;
    a.logL[b] = fsum[0];
    a.g_inst[2 * b + 0] = fsum[1];
    a.g_inst[2 * b + 1] = fsum[2];
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_item_consts(const int64_t* row_off, const double* layers, double* rec,
                              int n_items, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_item_consts, dim3(n_items), dim3(64), 0, st, row_off, layers, rec, n_items);
  return hipGetLastError();
}

hipError_t launch_forward(int op, const KernelArgs& a, int n_wu, hipStream_t st) {
  if (n_wu <= 0) return hipSuccess;
  if (op == kOpReflectivity)
    hipLaunchKernelGGL(k_reflectivity, dim3(n_wu), dim3(64), 0, st, a);
  else
    hipLaunchKernelGGL(k_loglik, dim3(n_wu), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_grad(int bucket, bool tail, const KernelArgs& a, int n_wu, hipStream_t st) {
  if (n_wu <= 0) return hipSuccess;
  switch (kBucketLmax[bucket]) {
#define NR_CASE(LM)                                                                           \
  case LM:                                                                                    \
    if (tail)                                                                                 \
      hipLaunchKernelGGL((k_loglik_grad<LM, (LM <= kStoreMaxLayers), true>), dim3(n_wu),      \
                         dim3(64), 0, st, a);                                                 \
    else                                                                                      \
      hipLaunchKernelGGL((k_loglik_grad<LM, (LM <= kStoreMaxLayers), false>), dim3(n_wu),     \
                         dim3(64), 0, st, a);                                                 \
    return hipGetLastError();
    NR_BUCKETS(NR_CASE)
#undef NR_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_reduce(int op, const ReduceArgs& a, hipStream_t st) {
  if (a.n_items <= 0) return hipSuccess;
  if (op == kOpLoglik) {
    hipLaunchKernelGGL(k_reduce_loglik, dim3((a.n_items + 255) / 256), dim3(256), 0, st, a);
  } else {
    const size_t shmem = sizeof(double) * (3 + 4 * (kMaxLayers + 2));
    hipLaunchKernelGGL(k_reduce_grad, dim3(a.n_items), dim3(64), shmem, st, a);
  }
  return hipGetLastError();
}

}  // namespace nr
