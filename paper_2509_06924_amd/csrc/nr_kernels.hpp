// HIP kernels for gfx950: Abeles reflectivity with Nevot-Croce roughness,
// Gaussian resolution smearing, instrument scale/background, Gaussian
// log-likelihood, and the hand-written adjoint of the whole chain.  One
// source for both precisions: a policy P (F64 or F32) sets the type of the
// layer product; the quadrature nodes, kz0^2 - 4 pi drho, the smearing sums,
// chi^2, the seeds and the per-point gradient accumulators are FP64 in both.
//
// Work decomposition: one work unit (WU) = one item x up to 64 consecutive data
// points of its dataset, one wave (64 lanes) per WU, lane = data point.  The
// item is wave-uniform, so its per-layer constants (precomputed per item by a
// small prologue kernel) are read with scalar loads into scalar registers.  A
// lane walks all quadrature nodes of its point; for each node it runs the
// layer product bottom-up (substrate -> surface), then the adjoint top down,
// and accumulates w_k dR(q_k)/d(theta) in registers; the point's likelihood
// seed multiplies the accumulators once at the end.
//
// The layer product is written in a scaled form: the Abeles column
// v_j = C_j v_{j+1} is divided by E_j at every layer, which leaves r = v1/v0
// unchanged and turns the phase factor into e_j = E_j^-2 = exp(-2 i kz_j d_j),
// whose modulus is <= 1 on the chosen branch (Im kz <= 0):
//   P <- P + r'_j Qv,   Qv <- e_j (r'_j P + Qv),   starting from (1, 0).
// The state therefore stays bounded (|P| <= prod (1 + |r'_j|)) and needs no
// rescaling in FP32 either.
//
// Two gradient variants (one source, selected by template):
//   store     - the forward sweep keeps each level's state (P, Qv) and phase
//               e_j in LDS and each medium's kz_j, 1/|kz_j|^2 and interface
//               coefficients in registers; the adjoint recomputes nothing.
//   recompute - for deep stacks: the state tape stays in registers and the
//               adjoint recomputes every layer's wavevector, interface
//               coefficients and phase.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "nr_device.hpp"
#include "nr_internal.hpp"

namespace nr {

// Precision policies of the layer product.
// kSlimMax: the deepest bucket whose store variant keeps only g = s^2 f per
// interface in registers and re-forms r' and kz_j kz_{j+1} in the adjoint
// (8 more FMAs per level, 8 fewer registers).  Measured on MI355X: in FP64 it
// lifts LMAX = 6 to two waves per SIMD (0.43 -> 0.45 of peak) but slows
// LMAX = 10 (3.49 -> 3.53 ms on the 4096-draw batch); FP32 has registers to
// spare and only loses.
//
// min_waves(LMAX): the waves per SIMD the gradient kernel is compiled for (its
// register budget is 512 / min_waves per lane).
struct F64 {
  using real = double;
  static constexpr int kStoreMax = kStoreMaxLayers;
  static constexpr int kSlimMax = 6;
  // (packed = a tail or split unit, whose extra bookkeeping the 4-layer store
  // kernel does not fit into two waves' registers)
  static constexpr int min_waves(int lmax, bool store, bool packed = false) {
    return ((!store && lmax <= 14) || (store && lmax <= 4 && !packed)) ? 2 : 1;
  }
  // recompute variant: levels whose phase e and g = s^2 f are kept in LDS
  // (2 KB per level per wave), and below them e_levels levels whose phase
  // alone is kept (1 KB each).  A wave may use 20 KB at two waves per SIMD
  // (up to 14 layers): 8 + 1 levels; 40 KB at one wave: 18 + 1 levels.
  // With the rule, the tables (2.8 KB) and the record staging sharing the
  // cache, that fills both budgets to within 240 B.
  static constexpr int ef_levels(int lmax) {
    return lmax <= 14 ? (lmax + 1 < 8 ? lmax + 1 : 8) : (lmax + 1 < 18 ? lmax + 1 : 18);
  }
  static constexpr int e_levels(int lmax) {
    return lmax + 1 > ef_levels(lmax) ? 1 : 0;
  }
  // recompute variant: keep the state of every second level only (the
  // register tape of the deepest buckets otherwise spills to scratch)
  static constexpr bool checkpoint(int lmax) { return lmax == 12 || lmax == 14 || lmax >= 28; }
  // the node's scheduling regions span several levels: at one wave per SIMD
  static constexpr bool grouped_regions(int lmax) { return min_waves(lmax, false) == 1; }
  // one wave per SIMD leaves the latency of the table and record reads
  // exposed: the recompute variant then issues each level's reads one level
  // ahead of their use.  The full units of 6 to 10 layers do so too, at two
  // waves: 6 and 8 layers 5 and 4 % faster, the 4096-draw batch 1.3 %.  Their
  // packed, split and resolution forms would spill 50-200 B per lane, so
  // they keep per-level regions.
  static constexpr bool pipelined(int lmax, bool packed_or_res = false) {
    return min_waves(lmax, false) == 1 || (!packed_or_res && lmax >= 6 && lmax <= 10);
  }
};
struct F32 {
  using real = float;
  static constexpr int kStoreMax = kStoreMaxLayersF32;
  static constexpr int kSlimMax = 0;
  // two waves per SIMD up to 28 layers, except 16, where one wave with
  // multi-level scheduling regions measured 3 % faster.  The FP64 gradient
  // accumulators dominate the registers; from 18 layers the checkpointed
  // tape keeps the spill small (none at 18, 204 B per lane at 24, 364 B at
  // 28), and two waves ran 23, 22 and 4 % faster than one at 20, 24 and 28
  // layers; at 32-40 layers (516-836 B) they lost 6-27 %.
  static constexpr int min_waves(int lmax, bool, bool = false) {
    return (lmax <= 28 && lmax != 16) ? 2 : 1;
  }
  // 1 KB per level; up to 28 layers the LDS of a kernel that may share the
  // SIMD with a second wave stays within 20 KB (17 levels, the record
  // staging sharing the cache); beyond, 37 levels within 40 KB; up to 10
  // layers the kernel fits three waves per SIMD in registers, and 9 levels
  // keep its LDS within 160 KB / 12 waves (10 levels fit too but measured
  // 2.5 % slower; at 11 levels only 11 waves fit a CU: 3-5 % slower)
  static constexpr int ef_levels(int lmax) {
    return lmax <= 10   ? (lmax + 1 < 9 ? lmax + 1 : 9)
           : lmax <= 28 ? (lmax + 1 < 17 ? lmax + 1 : 17)
                        : (lmax + 1 < 37 ? lmax + 1 : 37);
  }
  static constexpr int e_levels(int) { return 0; }
  static constexpr bool checkpoint(int lmax) { return lmax == 18 || lmax == 20 || lmax >= 24; }
  // from 12 layers, at one or two waves per SIMD (12 layers 5 % faster, 14-28
  // equal or faster); not at 32-40 layers (3-5 % slower)
  static constexpr bool grouped_regions(int lmax) { return lmax >= 12 && lmax < 32; }
  // from 12 layers the kernels read their records and LDS cache a level
  // ahead, as the one-wave FP64 kernels do (the exponentials are the
  // hardware functions, so there are no table reads to issue early): the
  // one-wave kernels (16, 32-40 layers) 7-22 % faster, the two-wave ones of
  // 12-28 layers 4-7 %; ragged FP32 batch 29.6 -> 25.4 ms.  At 10 layers it
  // would cost the third wave per SIMD.
  static constexpr bool pipelined(int lmax, bool = false) { return lmax >= 12; }
};

// ---------------------------------------------------------------------------
// Per-item layer records, written by k_item_consts into the workspace and
// read by the main kernels with scalar loads, since every lane of a wave uses
// the same item.  Per medium m = 0..N+1 (indexed like the item's rows), six
// doubles:
//   A  = 4 pi (rho_re,m - rho_re,0)        (0 for the fronting medium)
//   B  = 4 pi |rho_im,m|                   (0 for the fronting: lossless)
//   Nr + i Ni = w_m - w_{m+1} = (A_{m+1} - A_m) + i (B_{m+1} - B_m), the
//        Q-independent numerator of r_m = (w_m - w_{m+1}) / (kz_m + kz_{m+1})^2
//   C  = -2 sigma_{m+1}^2                  (Nevot-Croce exponent factor)
//   D  = 2 d_m                             (layers 1..N; 0 for the fronting
//                                           and the backing)
// and eight floats: B, Nr, Ni, C, D rounded to float, then padding (the FP32
// variant reads A from the doubles: kz0^2 - A is formed in FP64).
// Interface fields of the backing record are 0.
// ---------------------------------------------------------------------------
constexpr int kRec = kRecDoubles;
constexpr int kRecF = kRecFloats;

// Layer records are indexed with (m + z) where z = k & KernelArgs::zero_mask
// (the mask is 0): z is 0 at run time but varies with the node counter k as
// far as the compiler can tell, so the records are re-read (with scalar
// loads) inside the node loop instead of being hoisted out of it, which would
// need far more scalar registers than exist.
//
// Media below the backing (m > N + 1, used when an item is evaluated at its
// bucket's depth LMAX > N) read the backing's record: the same wavevector,
// a zero interface numerator, sigma 0 and thickness 0 (k_item_consts stores
// D = 0 for the backing).  Such a medium is an exact copy of the backing
// joined by r' = 0, so the state below the backing stays (1, 0) and the
// forward product is unchanged; in the adjoint the copies are the backing's
// own parameters, and their w-cotangents are added to the backing's.
template <class P>
struct Layers {
  using Re = typename P::real;
  static constexpr bool kF64 = std::is_same<Re, double>::value;
  const double* rec;   // the item's double records
  const float* recf;   // the item's float records
  int z;               // an opaque zero
  int nb;              // the backing medium, N + 1
  __device__ __forceinline__ int med(int m) const { return (m < nb ? m : nb) + z; }
  __device__ __forceinline__ double at(int m, int f) const { return rec[med(m) * kRec + f]; }
  __device__ __forceinline__ Re get(int m, int fd, int ff) const {
    if constexpr (kF64)
      return at(m, fd);
    else
      return recf[med(m) * kRecF + ff];
  }
  // the whole record of medium m (loaded a level ahead by the pipelined sweeps)
  struct Rec {
    double A;
    Re B, Nr, Ni, C, D;
  };
  __device__ __forceinline__ Rec rec_of(int m) const {
    Rec r;
    r.A = A(m);
    r.B = B(m);
    r.Nr = Nr(m);
    r.Ni = Ni(m);
    r.C = C(m);
    r.D = D(m);
    return r;
  }
  __device__ __forceinline__ double A(int m) const { return at(m, 0); }
  __device__ __forceinline__ Re B(int m) const { return get(m, 1, 0); }
  __device__ __forceinline__ Re Nr(int m) const { return get(m, 2, 1); }
  __device__ __forceinline__ Re Ni(int m) const { return get(m, 3, 2); }
  __device__ __forceinline__ Re C(int m) const { return get(m, 4, 3); }
  __device__ __forceinline__ Re D(int m) const { return get(m, 5, 4); }
};

// The quadrature rule and the exp/sincos tables, staged per block in LDS.
struct Shared {
  double t[kSmearNodes], w[kSmearNodes];
  MathTables tab;
};

// Reads of staged LDS values that every lane shares are volatile so that the
// compiler re-reads them at each use instead of holding them in registers.
typedef __attribute__((address_space(3))) const volatile double lds_cv_double;
__device__ __forceinline__ double ld(const double& x) { return *(lds_cv_double*)(&x); }

// (write: the lanes of one wave fill the tables; every thread of the block
// reaches the barrier)
__device__ __forceinline__ void stage_shared(Shared& s, int lane, const double* rule,
                                             bool write = true) {
  if (write) {
    if (lane < kSmearNodes) {
      s.t[lane] = rule[lane];
      s.w[lane] = rule[kSmearNodes + lane];
    }
    // tables follow the rule in the same device buffer
    const double* tb = rule + 2 * kSmearNodes;
    s.tab.sc[lane][0] = tb[2 * lane];
    s.tab.sc[lane][1] = tb[2 * lane + 1];
    s.tab.sc[lane + 64][0] = tb[2 * lane + 128];
    s.tab.sc[lane + 64][1] = tb[2 * lane + 129];
    s.tab.e2[lane] = tb[256 + lane];
  }
  __syncthreads();
}

// Interface quantities shared by the forward and adjoint sweeps.
// r' = r f = N s^2 f with N = w_j - w_{j+1} and s = 1/(kz_j + kz_{j+1}).  The
// adjoint needs s^2 and f only through their product g = s^2 f: the
// cotangent of r is conj(f) r'bar, and it reaches the wavevectors times
// conj(s^2).
template <class Re>
struct Iface {
  cx<Re> g;   // s^2 f
  cx<Re> rp;  // r' = N g
  cx<Re> kk;  // kz_j kz_{j+1}
};

// r = (w_j - w_{j+1}) / (kz_j + kz_{j+1})^2 = N s^2.  For identical media
// N = 0 and r' = 0 exactly: g stays finite because |kz| >= 1e-75 (the root's
// guard), so no separate test is needed.
template <class Re>
__device__ __forceinline__ Iface<Re> interface_coeffs(const MathTables& T, cx<Re> kzc, cx<Re> kzn,
                                                      Re Nr, Re Ni, Re C) {
  Iface<Re> o;
  const cx<Re> s = crecip(kzc + kzn);
  o.kk = kzc * kzn;
  o.g = (s * s) * cexp_tab(T, C * o.kk);
  o.rp = mk(Nr, Ni) * o.g;
  return o;
}

// e_j = exp(-2 i kz_j d_j) = exp(D Im kz) cis(-D Re kz), D = 2 d_j.
template <class Re>
__device__ __forceinline__ cx<Re> layer_phase(const MathTables& T, cx<Re> kz, Re D) {
  return cexp_tab(T, mk(D * kz.im, -D * kz.re));
}

// kz of medium m: w = kz0^2 - A_m - i B_m, with kz0^2 - A_m formed in FP64.
template <class P>
__device__ __forceinline__ RootT<typename P::real> medium_root(const Layers<P>& L, double kz0sq,
                                                               int m) {
  using Re = typename P::real;
  return kz_root(static_cast<Re>(kz_real_part(kz0sq, L.A(m))), -L.B(m));
}

// The same, recording whether w_m = 0 exactly (x = 0 and no absorption): the
// root's derivative 1/(2 kz) is infinite there.
template <class P>
__device__ __forceinline__ RootT<typename P::real> medium_root(const Layers<P>& L, double kz0sq,
                                                               int m, bool& edge) {
  using Re = typename P::real;
  const double x = kz_real_part(kz0sq, L.A(m));
  const Re b = L.B(m);
  edge |= (x == 0.0) & (b == Re(0));
  return kz_root(static_cast<Re>(x), -b);
}

template <class P>
__device__ __forceinline__ cx<typename P::real> fronting_kz(double q) {
  using Re = typename P::real;
  return mk(static_cast<Re>(0.5 * q), Re(0));
}

// ---------------------------------------------------------------------------
// Forward-only reflectivity of one node (no state kept; runtime layer loop).
// ---------------------------------------------------------------------------
template <class P>
__device__ __forceinline__ double node_reflectivity(const MathTables& T, const Layers<P>& L, int N,
                                                    double q) {
  using Re = typename P::real;
  using Cx = cx<Re>;
  const double kz0sq = kz0_squared(q);
  Cx kzn = medium_root(L, kz0sq, N + 1).kz;
  Cx Pv = mk(Re(1), Re(0)), Qv = mk(Re(0), Re(0));
  for (int jj = N; jj >= 1; --jj) {
    const Cx kzc = medium_root(L, kz0sq, jj).kz;
    const Iface<Re> it = interface_coeffs(T, kzc, kzn, L.Nr(jj), L.Ni(jj), L.C(jj));
    const Cx Pn = cmul_add(it.rp, Qv, Pv);
    const Cx t = cmul_add(it.rp, Pv, Qv);
    Qv = layer_phase(T, kzc, L.D(jj)) * t;
    Pv = Pn;
    kzn = kzc;
  }
  {
    const Iface<Re> it = interface_coeffs(T, fronting_kz<P>(q), kzn, L.Nr(0), L.Ni(0), L.C(0));
    const Cx Pn = cmul_add(it.rp, Qv, Pv);
    Qv = cmul_add(it.rp, Pv, Qv);
    Pv = Pn;
  }
  return (double)cabs2(Qv * crecip(Pv));
}

// Shared WU prologue.
struct WuInfo {
  int item, ds, N, nq, i;
  int64_t qoff, roff;
  bool active;
  double Q, dqq;
  double sig;      // sigma_Q of the point
  bool smeared;    // the dataset is smeared (17 nodes)
  bool pointwise;  // widths given per point (no width derivative)
};

__device__ __forceinline__ void resolution_setup(const KernelArgs& a, WuInfo& u, int64_t ip) {
  u.smeared = a.dq_over_q[u.ds] > 0.0;
  u.dqq = a.dqq_item ? a.dqq_item[u.item] : a.dq_over_q[u.ds];
  u.pointwise = a.dq != nullptr;
  u.sig = u.pointwise ? smear_sigma_abs(a.dq[ip]) : smear_sigma_rel(u.Q, u.dqq);
}

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
  resolution_setup(a, u, u.qoff + (u.active ? u.i : p0));
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
  resolution_setup(a, u, u.qoff + u.i);
  return u;
}

// Split tail units hold the last partial group of points (npts < 64) of one
// smeared item: lane l = g npts + p evaluates point p0 + p on the smearing
// nodes k = g, g + G, g + 2G, ... (G node groups, G npts <= 64 lanes busy).
// The item is wave-uniform, so its layer records are scalar loads as in a
// full unit.  Idle lanes repeat point p0 + (l mod npts) and evaluate no node.
struct SplitInfo {
  int g, G, npts;
};
__device__ __forceinline__ WuInfo split_setup(const KernelArgs& a, int w, int lane,
                                              SplitInfo& sp) {
  const int32_t code = a.wu_split[w];
  sp.npts = code & 0xffff;
  sp.G = code >> 16;
  sp.g = lane / sp.npts;
  WuInfo u;
  u.item = a.wu_item[w];
  const int p0 = a.wu_p0[w];
  u.ds = a.dataset_of_item[u.item];
  u.qoff = a.q_off[u.ds];
  u.nq = (int)(a.q_off[u.ds + 1] - u.qoff);
  u.roff = a.row_off[u.item];
  u.N = (int)(a.row_off[u.item + 1] - u.roff) - 2;
  u.i = p0 + lane % sp.npts;
  u.active = sp.g < sp.G;
  u.Q = a.q[u.qoff + u.i];
  resolution_setup(a, u, u.qoff + u.i);
  return u;
}

template <class P>
__device__ __forceinline__ Layers<P> item_layers(const KernelArgs& a, int64_t roff, int N, int k) {
  Layers<P> L;
  L.rec = a.consts + roff * kRec;
  L.recf = a.constsf + roff * kRecF;
  L.z = k & a.zero_mask;
  L.nb = N + 1;
  return L;
}

__device__ __forceinline__ void flag(int32_t* status, int item, uint32_t bits) {
  if (status != nullptr && bits != 0u)
    atomicOr(reinterpret_cast<unsigned int*>(status + item), bits);
}

// ---------------------------------------------------------------------------
// Smeared R of a forward unit's point.  SPLIT: the unit holds npts points of
// one item and lane g npts + p evaluates point p on the nodes g, g + G, ...;
// the point's G lanes then add their partial sums, so that every one of them
// holds the point's smeared R (split_setup).
// ---------------------------------------------------------------------------
template <class P, bool SPLIT>
__device__ __forceinline__ double forward_point(const KernelArgs& a, const Shared& s,
                                                const WuInfo& u, const SplitInfo& sp, int lane,
                                                bool& badq) {
  const int K = u.smeared ? kSmearNodes : 1;
  const int k0 = SPLIT ? (u.active ? sp.g : K) : 0;
  const int kstep = SPLIT ? sp.G : 1;
  double Rsm = 0.0;
  badq = !(u.Q > 0.0);
  for (int k = k0; k < K; k += kstep) {
    const double q = (K == 1) ? u.Q : smear_at(u.Q, u.sig, ld(s.t[k]));
    badq |= !(q > 0.0);
    const double wk = (K == 1) ? 1.0 : ld(s.w[k]);
    Rsm += wk * node_reflectivity(s.tab, item_layers<P>(a, u.roff, u.N, k), u.N, q);
  }
  if constexpr (SPLIT) {
    double tot = 0.0;
    int bq = 0;
    for (int gg = 0; gg < sp.G; ++gg) {
      const int src = gg * sp.npts + lane % sp.npts;
      tot += __shfl(Rsm, src, 64);
      bq |= __shfl(badq ? 1 : 0, src, 64);
    }
    Rsm = tot;
    badq = bq != 0;
  }
  return Rsm;
}

// ---------------------------------------------------------------------------
// R_hat per point (nr_reflectivity).
// ---------------------------------------------------------------------------
template <class P, bool SPLIT = false>
__global__ __launch_bounds__(64) void k_reflectivity(KernelArgs a) {
  __shared__ Shared s;
  const int lane = threadIdx.x;
  const int w = blockIdx.x;
  SplitInfo sp{0, 1, 64};
  const WuInfo u = SPLIT ? split_setup(a, w, lane, sp) : wu_setup(a, w, lane);
  stage_shared(s, lane, a.rule);
  bool badq = false;
  const double Rsm = forward_point<P, SPLIT>(a, s, u, sp, lane, badq);
  if (u.active && sp.g == 0) {
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
template <class P, bool SPLIT = false>
__global__ __launch_bounds__(64) void k_loglik(KernelArgs a) {
  __shared__ Shared s;
  const int lane = threadIdx.x;
  const int w = blockIdx.x;
  SplitInfo sp{0, 1, 64};
  const WuInfo u = SPLIT ? split_setup(a, w, lane, sp) : wu_setup(a, w, lane);
  stage_shared(s, lane, a.rule);
  bool badq = false;
  const double Rsm = forward_point<P, SPLIT>(a, s, u, sp, lane, badq);
  double ll = 0.0;
  uint32_t bits = 0;
  if (u.active && sp.g == 0) {
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
// coefficients, the phase e_j (j >= 1) and the running kzbar_j (the
// contribution of level j - 1).  Out: cotangents of the state entering the
// level, kzbar_j complete and kzbar_{j+1}'s first part, and the terms of the
// d and sigma accumulators.
// ---------------------------------------------------------------------------
template <class Re>
struct AdjStep {
  cx<Re> Pb, Qb;   // cotangents of the state entering level j
  cx<Re> kzb_c;    // kzbar_j: the running sum passed in plus this level's part
  cx<Re> kzb_n;    // contribution to kzbar_{j+1}
  cx<Re> ub;       // cotangent of the Nevot-Croce exponent
  cx<Re> w;        // conj(e) ebar (phase levels)
};


// Per level (cotangent convention zbar = dl/dRe z + i dl/dIm z):
//   t = r' P + Qv;  ebar = conj(t) Qbar;  tbar = conj(e) Qbar
//   r'bar = conj(Qv) Pbar + conj(P) tbar;  Pbar_in = Pbar + conj(r') tbar;
//   Qbar_in = conj(r') Pbar + tbar
//   rbar = conj(f) r'bar;  ubar = conj(r') r'bar   (u = C kz_j kz_{j+1}, f = e^u)
//   r = (kz_j - kz_{j+1}) s: dr/dkz_j = 2 kz_{j+1} s^2, dr/dkz_{j+1} = -2 kz_j s^2
//   kzbar_j     += conj(kz_{j+1}) (C ubar + 2 Y)
//   kzbar_{j+1} += conj(kz_j)     (C ubar - 2 Y),   Y = conj(s^2) rbar = conj(g) r'bar
//   e = exp(-2 i kz d): with w = conj(e) ebar = conj(t) tbar,
//   kzbar_j += i D w  (D = 2d),   dl/dd = 2 Im(kz_j conj(w))
template <class Re>
__device__ __forceinline__ AdjStep<Re> adjoint_step(cx<Re> Ps, cx<Re> Qs, cx<Re> Pb, cx<Re> Qb,
                                                    cx<Re> kzc, cx<Re> kzn, const Iface<Re>& it,
                                                    Re C, bool has_phase, cx<Re> e, Re D,
                                                    cx<Re> kzbc) {
  using Cx = cx<Re>;
  AdjStep<Re> o;
  Cx tb;
  o.w = mk(Re(0), Re(0));
  if (has_phase) {
    const Cx t = cmul_add(it.rp, Ps, Qs);
    tb = cmulc(e, Qb);
    o.w = cmulc(t, tb);
  } else {
    tb = Qb;
  }
  const Cx rpb = cmulc_add(Ps, tb, cmulc(Qs, Pb));
  o.Pb = cmulc_add(it.rp, tb, Pb);
  o.Qb = cmulc_add(it.rp, Pb, tb);
  o.ub = cmulc(it.rp, rpb);
  const Cx X = C * o.ub;
  const Cx Y = cmulc(it.g, rpb);
  const Cx Zc = mk(fma(Re(2), Y.re, X.re), fma(Re(2), Y.im, X.im));
  const Cx Zn = mk(fma(Re(-2), Y.re, X.re), fma(Re(-2), Y.im, X.im));
  o.kzb_c = cmulc_add(kzn, Zc, kzbc);
  o.kzb_n = cmulc(kzc, Zn);
  if (has_phase) {
    o.kzb_c.re = fma(-D, o.w.im, o.kzb_c.re);
    o.kzb_c.im = fma(D, o.w.re, o.kzb_c.im);
  }
  return o;
}

// acc += Re(conj(a) b), accumulated in FP64 (the sigma sums: a = ubar,
// b = kz_j kz_{j+1}).
__device__ __forceinline__ void acc_re_dot(double& acc, cd a, cd b) {
  acc = fma(a.re, b.re, fma(a.im, b.im, acc));
}
__device__ __forceinline__ void acc_re_dot(double& acc, cf a, cf b) {
  acc += (double)(a.re * b.re + a.im * b.im);
}
// The accumulators hold fixed multiples of the sums they stand for; the
// factors are applied once, when the record is written (kHdScale, kHwScale).
//
// acc += Im(kz conj(w)): half the thickness derivative 2 Im(kz conj(w)), in FP64.
constexpr double kHdScale = 2.0;
__device__ __forceinline__ void acc_dd(double& acc, cd kz, cd w) {
  acc = fma(kz.im, w.re, fma(-kz.re, w.im, acc));
}
__device__ __forceinline__ void acc_dd(double& acc, cf kz, cf w) {
  acc += (double)(kz.im * w.re - kz.re * w.im);
}
// acc += 2 wbar, wbar = conj(dkz/dw) kzbar = conj(1/(2 kz)) kzbar = kz kzbar / (2 |kz|^2),
// and with RES also sw += 2 Re(wbar) (the node's sum over media, for dR/dq:
// every w_j moves with kz0^2, dw_j/dq = kz0).  Doubling is exact, so the
// halved record equals the sum of the wbar terms bit for bit.
constexpr double kHwScale = 0.5;
template <bool RES>
__device__ __forceinline__ void acc_wbar(cd& acc, double& sw, cd kz, double inv_abs2, cd kzb) {
  const cd p = kz * kzb;
  acc.re = fma(inv_abs2, p.re, acc.re);
  acc.im = fma(inv_abs2, p.im, acc.im);
  if constexpr (RES) sw = fma(inv_abs2, p.re, sw);
}
template <bool RES>
__device__ __forceinline__ void acc_wbar(cd& acc, double& sw, cf kz, float inv_abs2, cf kzb) {
  const cd v = widen(inv_abs2 * (kz * kzb));
  acc += v;
  if constexpr (RES) sw += v.re;
}
template <class Cx, class Re>
__device__ __forceinline__ void acc_wbar(cd& acc, Cx kz, Re inv_abs2, Cx kzb) {
  double unused = 0.0;
  acc_wbar<false>(acc, unused, kz, inv_abs2, kzb);
}

// Per-lane gradient accumulators for one point, FP64 in both precisions:
// sum_k w_k dR(q_k)/d(.)
template <int LMAX>
struct Accum {
  cd Hw[LMAX + 2];
  double Hd[LMAX + 2], Hs[LMAX + 2];
};

// LDS tape of the store variant: per-lane state entering each level and the
// layer phase, as separate real and imaginary planes, lane-minor (a level's
// two planes are 64 elements apart, one ds_write2/ds_read2 per value).
template <class Re, int LMAX>
struct alignas(16) GradTape {
  Re P[LMAX + 1][2][64], Qv[LMAX + 1][2][64], E[LMAX + 1][2][64];
};

template <class Re>
__device__ __forceinline__ void tape_put(Re (&slot)[2][64], int lane, cx<Re> z) {
  slot[0][lane] = z.re;
  slot[1][lane] = z.im;
}
template <class Re>
__device__ __forceinline__ cx<Re> tape_get(const Re (&slot)[2][64], int lane) {
  return mk(slot[0][lane], slot[1][lane]);
}

// ---------------------------------------------------------------------------
// One node, store variant: forward with the tape in LDS and kz in registers,
// then the adjoint.  Returns R(q) and adds w_k dR/d(.) to the accumulators.
// ---------------------------------------------------------------------------
template <class P, int LMAX>
__device__ __forceinline__ double node_grad_store(const MathTables& T, const Layers<P>& L,
                                                  GradTape<typename P::real, LMAX>& tp,
                                                  Accum<LMAX>& acc, int lane, double q,
                                                  double wk, bool& edge) {
  using Re = typename P::real;
  using Cx = cx<Re>;
  const double kz0sq = kz0_squared(q);
  Cx kz[LMAX + 2];
  Re ia[LMAX + 2];
  // per interface, kept for the adjoint: g = s^2 f, and unless the bucket is
  // slim, r' and kz_j kz_{j+1} too
  constexpr bool kSlim = LMAX <= P::kSlimMax;
  Cx kg[LMAX + 1];
  Cx krp[kSlim ? 1 : LMAX + 1], kkk[kSlim ? 1 : LMAX + 1];
  Cx Pv = mk(Re(1), Re(0)), Qv = mk(Re(0), Re(0));
  {
    const RootT<Re> rt = medium_root(L, kz0sq, LMAX + 1, edge);
    kz[LMAX + 1] = rt.kz;
    ia[LMAX + 1] = rt.inv_abs2;
  }
  // every level is evaluated (the depth is the bucket's), so the whole node
  // is straight-line code the scheduler can interleave across levels
#pragma unroll
  for (int jj = LMAX; jj >= 0; --jj) {
    if (jj == 0) {
      kz[0] = fronting_kz<P>(q);
      ia[0] = Re(0);
    } else {
      const RootT<Re> rt = medium_root(L, kz0sq, jj, edge);
      kz[jj] = rt.kz;
      ia[jj] = rt.inv_abs2;
    }
    const Iface<Re> it = interface_coeffs(T, kz[jj], kz[jj + 1], L.Nr(jj), L.Ni(jj), L.C(jj));
    kg[jj] = it.g;
    if constexpr (!kSlim) {
      krp[jj] = it.rp;
      kkk[jj] = it.kk;
    }
    tape_put(tp.P[jj], lane, Pv);
    tape_put(tp.Qv[jj], lane, Qv);
    const Cx Pn = cmul_add(it.rp, Qv, Pv);
    const Cx t = cmul_add(it.rp, Pv, Qv);
    if (jj >= 1) {
      const Cx e = layer_phase(T, kz[jj], L.D(jj));
      tape_put(tp.E[jj], lane, e);
      Qv = e * t;
    } else {
      Qv = t;
    }
    Pv = Pn;
  }
  const Cx iP = crecip(Pv);
  const Cx r = Qv * iP;
  const Cx rbar = static_cast<Re>(2.0 * wk) * r;
  Cx Pb = cmulc(-(r * iP), rbar);  // conj(dr/dP) rbar, dr/dP = -r/P
  Cx Qb = cmulc(iP, rbar);         // conj(dr/dQv) rbar, dr/dQv = 1/P
  Cx kzbc = mk(Re(0), Re(0));
#pragma unroll
  for (int jj = 0; jj <= LMAX; ++jj) {
    const Re C = L.C(jj);
    Iface<Re> it;
    it.g = kg[jj];
    if constexpr (kSlim) {
      it.rp = mk(L.Nr(jj), L.Ni(jj)) * it.g;
      it.kk = kz[jj] * kz[jj + 1];
    } else {
      it.rp = krp[jj];
      it.kk = kkk[jj];
    }
    const Cx Ps = tape_get(tp.P[jj], lane);
    const Cx Qs = tape_get(tp.Qv[jj], lane);
    const bool ph = jj >= 1;
    const Cx e = ph ? tape_get(tp.E[jj], lane) : mk(Re(1), Re(0));
    const AdjStep<Re> st = adjoint_step(Ps, Qs, Pb, Qb, kz[jj], kz[jj + 1], it, C, ph, e,
                                        ph ? L.D(jj) : Re(0), kzbc);
    kzbc = st.kzb_c;
    acc_re_dot(acc.Hs[jj + 1], st.ub, it.kk);
    if (ph) {
      acc_dd(acc.Hd[jj], kz[jj], st.w);
      acc_wbar(acc.Hw[jj], kz[jj], ia[jj], kzbc);
    }
    if (jj == LMAX) acc_wbar(acc.Hw[jj + 1], kz[jj + 1], ia[jj + 1], st.kzb_n);
    Pb = st.Pb;
    Qb = st.Qb;
    kzbc = st.kzb_n;
  }
  return (double)cabs2(r);
}

// LDS cache of the recompute variant: for levels 0..KS-1, the layer phase e
// and g = s^2 f, the Nevot-Croce factor times the squared interface
// reciprocal (planes e.re, e.im, g.re, g.im, lane-minor); for levels
// KS..KS+KE-1 the phase alone.
template <class Re, int KS, int KE>
struct alignas(16) EfCache {
  Re v[KS][4][64];
  Re ve[KE][2][64];
  __device__ __forceinline__ cx<Re> e_extra(int jj, int lane) const {
    return mk(ve[jj - KS][0][lane], ve[jj - KS][1][lane]);
  }
  __device__ __forceinline__ void put_e_extra(int jj, int lane, cx<Re> e) {
    ve[jj - KS][0][lane] = e.re;
    ve[jj - KS][1][lane] = e.im;
  }
};
template <class Re, int KS>
struct alignas(16) EfCache<Re, KS, 0> {
  Re v[KS][4][64];
  __device__ __forceinline__ cx<Re> e_extra(int, int) const { return mk(Re(0), Re(0)); }
  __device__ __forceinline__ void put_e_extra(int, int, cx<Re>) {}
};

// ---------------------------------------------------------------------------
// One node, recompute variant: the state tape stays in registers; the adjoint
// recomputes each medium's wavevector; below the KS cached levels also the
// interface reciprocal and the Nevot-Croce factor, and below the KE levels
// after them, whose phase alone is cached, the phase.
// ---------------------------------------------------------------------------
template <class P, int LMAX, int KS, int KE, bool CK, bool RES, bool PIPE>
__device__ __forceinline__ double node_grad_recompute(const MathTables& T, const Layers<P>& L,
                                                      EfCache<typename P::real, KS, KE>& ef,
                                                      Accum<LMAX>& acc, int lane, double q,
                                                      double wk, bool& edge, double& Hq,
                                                      double c) {
  using Re = typename P::real;
  using Cx = cx<Re>;
  static_assert(!CK || LMAX % 2 == 0, "checkpointed tape needs an even depth");
  const double kz0sq = kz0_squared(q);
  const Cx kz0 = fronting_kz<P>(q);
  // state tape: every level, or (CK) every second one; level j (odd) is then
  // re-formed in the adjoint by applying level j + 1 to the state at j + 1
  constexpr int NT = CK ? LMAX / 2 + 1 : LMAX + 1;
  Cx tapeP[NT], tapeQ[NT];
  // Scheduling regions.  By default every level is a region of its own,
  // which keeps the registers of a two-wave kernel in check.  The latency of
  // the scalar record loads and LDS table lookups can then only be hidden by
  // another wave.  Where the precision policy's grouped_regions says so (all
  // one-wave FP64 kernels, FP32 from 12 layers), the forward sweep is one
  // region and the adjoint is cut every kAdjGroup levels.  The kz, interface
  // and phase of one level do not depend on the state, so the scheduler
  // overlaps neighbouring levels' chains.
  //
  // Where PIPE (the policy's pipelined) says so (the one-wave kernels, and the
  // plain full units of 6 to 10 layers in FP64), both sweeps are
  // software-pipelined instead: the region of one level also
  // forms the next level's wavevector and interface and issues its LDS table
  // (or cache) reads, and loads the layer record the region after it needs.
  // Each read then has a whole level of work to arrive in; left to the
  // compiler, a read was used about 10 instructions after its issue, and the
  // one wave stalled on it.
  constexpr bool kGrouped = P::grouped_regions(LMAX);
  constexpr int kAdjGroup = kGrouped ? 8 : 1;
  constexpr bool kPipe = PIPE;
  Cx kzn = medium_root(L, kz0sq, LMAX + 1, edge).kz;
  Cx Pv = mk(Re(1), Re(0)), Qv = mk(Re(0), Re(0));
  // Pipelined forward sweep: the region of level jj also forms level jj-1's
  // wavevector and interface and issues its table reads, which level jj-1
  // uses a region later; it loads the record of level jj-2.
  struct FwdPre {
    Cx kz;  // medium jj (jj = 0: the fronting medium)
    Cx s2;  // 1/(kz_jj + kz_jj+1)^2
    CexpPart<Re> f, e;
  };
  using Rec = typename Layers<P>::Rec;
  auto fwd_pre = [&](int jj, Cx kzb, const Rec& rj) {
    FwdPre o;
    if (jj == 0) {
      o.kz = kz0;
    } else {
      const double x = kz_real_part(kz0sq, rj.A);
      edge |= (x == 0.0) & (rj.B == Re(0));
      o.kz = kz_root(static_cast<Re>(x), -rj.B).kz;
    }
    const Cx s = crecip(o.kz + kzb);
    o.s2 = s * s;
    o.f = cexp_issue(T, rj.C * (o.kz * kzb));
    if (jj >= 1) o.e = cexp_issue(T, mk(rj.D * o.kz.im, -rj.D * o.kz.re));
    return o;
  };
  if constexpr (kPipe) {
    Rec R[LMAX + 1];
    R[LMAX] = L.rec_of(LMAX);
    if (LMAX >= 1) R[LMAX - 1] = L.rec_of(LMAX - 1);
    FwdPre cur = fwd_pre(LMAX, kzn, R[LMAX]);
#pragma unroll
    for (int jj = LMAX; jj >= 0; --jj) {
      if (jj >= 2) R[jj - 2] = L.rec_of(jj - 2);
      FwdPre nxt;
      if (jj >= 1) nxt = fwd_pre(jj - 1, cur.kz, R[jj - 1]);
      if (!CK || jj % 2 == 0) {
        tapeP[CK ? jj / 2 : jj] = Pv;
        tapeQ[CK ? jj / 2 : jj] = Qv;
      }
      const Cx g = cur.s2 * cexp_finish(cur.f);
      const Cx rp = mk(R[jj].Nr, R[jj].Ni) * g;
      const Cx Pn = cmul_add(rp, Qv, Pv);
      const Cx t = cmul_add(rp, Pv, Qv);
      const Cx e = (jj >= 1) ? cexp_finish(cur.e) : mk(Re(1), Re(0));
      if (jj < KS) {
        ef.v[jj][0][lane] = e.re;
        ef.v[jj][1][lane] = e.im;
        ef.v[jj][2][lane] = g.re;
        ef.v[jj][3][lane] = g.im;
      } else if (jj < KS + KE) {
        ef.put_e_extra(jj, lane, e);
      }
      Qv = (jj >= 1) ? e * t : t;
      Pv = Pn;
      if (jj >= 1) cur = nxt;
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
#pragma unroll
    for (int jj = LMAX; jj >= 0; --jj) {
      const Cx kzc = (jj == 0) ? kz0 : medium_root(L, kz0sq, jj, edge).kz;
      if (!CK || jj % 2 == 0) {
        tapeP[CK ? jj / 2 : jj] = Pv;
        tapeQ[CK ? jj / 2 : jj] = Qv;
      }
      const Iface<Re> it = interface_coeffs(T, kzc, kzn, L.Nr(jj), L.Ni(jj), L.C(jj));
      const Cx Pn = cmul_add(it.rp, Qv, Pv);
      const Cx t = cmul_add(it.rp, Pv, Qv);
      const Cx e = (jj >= 1) ? layer_phase(T, kzc, L.D(jj)) : mk(Re(1), Re(0));
      if (jj < KS) {
        ef.v[jj][0][lane] = e.re;
        ef.v[jj][1][lane] = e.im;
        ef.v[jj][2][lane] = it.g.re;
        ef.v[jj][3][lane] = it.g.im;
      } else if (jj < KS + KE) {
        ef.put_e_extra(jj, lane, e);
      }
      Qv = (jj >= 1) ? e * t : t;
      Pv = Pn;
      kzn = kzc;
      if (!kGrouped || jj == 0)
        __builtin_amdgcn_sched_barrier(0x0100);  // only LDS reads may move across
    }
  }
  const Cx iP = crecip(Pv);
  const Cx r = Qv * iP;
  const Cx rbar = static_cast<Re>(2.0 * wk) * r;
  Cx Pb = cmulc(-(r * iP), rbar);
  Cx Qb = cmulc(iP, rbar);
  Cx kzbc = mk(Re(0), Re(0));
  double sw = 0.0;

  // the coefficients of level jj (kz_jj = kzc known), recomputed or from the
  // LDS cache
  struct Lev {
    RootT<Re> rn;  // medium jj + 1
    Iface<Re> it;
    Cx e;
    Re C, D;
  };
  auto level = [&](int jj, Cx kzc) {
    Lev o;
    o.rn = medium_root(L, kz0sq, jj + 1);
    o.C = L.C(jj);
    const bool ph = jj >= 1;
    o.D = ph ? L.D(jj) : Re(0);
    if (jj < KS) {
      o.it.g = mk(ef.v[jj][2][lane], ef.v[jj][3][lane]);
      o.it.rp = mk(L.Nr(jj), L.Ni(jj)) * o.it.g;
      o.it.kk = kzc * o.rn.kz;
      o.e = ph ? mk(ef.v[jj][0][lane], ef.v[jj][1][lane]) : mk(Re(1), Re(0));
    } else {
      o.it = interface_coeffs(T, kzc, o.rn.kz, L.Nr(jj), L.Ni(jj), o.C);
      o.e = !ph ? mk(Re(1), Re(0))
                : (jj < KS + KE) ? ef.e_extra(jj, lane) : layer_phase(T, kzc, o.D);
    }
    return o;
  };
  // the adjoint of level jj from the state (Ps, Qs) entering it
  auto step = [&](int jj, const Lev& lv, Cx Ps, Cx Qs, Cx kzc, Re iac) {
    const bool ph = jj >= 1;
    const AdjStep<Re> st =
        adjoint_step(Ps, Qs, Pb, Qb, kzc, lv.rn.kz, lv.it, lv.C, ph, lv.e, lv.D, kzbc);
    kzbc = st.kzb_c;
    if constexpr (RES)
      if (jj == 0) Hq = fma(0.5 * c, (double)kzbc.re, Hq);
    acc_re_dot(acc.Hs[jj + 1], st.ub, lv.it.kk);
    if (ph) {
      acc_dd(acc.Hd[jj], kzc, st.w);
      acc_wbar<RES>(acc.Hw[jj], sw, kzc, iac, kzbc);
    }
    if (jj == LMAX) acc_wbar<RES>(acc.Hw[jj + 1], sw, lv.rn.kz, lv.rn.inv_abs2, st.kzb_n);
    Pb = st.Pb;
    Qb = st.Qb;
    kzbc = st.kzb_n;
  };

  Cx kzc = kz0;
  Re iac = Re(0);
  // Pipelined adjoint: the region of level jj also forms level jj+1's
  // wavevector and interface and issues its table (or cache) reads.
  struct AdjPre {
    RootT<Re> rn;  // medium jj + 1
    Cx s2, kk;     // s^2 (below the cache), kz_jj kz_jj+1
    Cx gv, ev;     // g (jj < KS) and e (jj < KS + KE) from the LDS cache
    CexpPart<Re> f, e;
    Re C, D, Nr, Ni;
  };
  // (ri: the record of level jj, rn: that of medium jj + 1)
  auto adj_pre = [&](int jj, Cx kzb, const Rec& ri, const Rec& rn) {
    AdjPre o;
    o.rn = kz_root(static_cast<Re>(kz_real_part(kz0sq, rn.A)), -rn.B);
    o.C = ri.C;
    o.Nr = ri.Nr;
    o.Ni = ri.Ni;
    const bool ph = jj >= 1;
    o.D = ph ? ri.D : Re(0);
    o.kk = kzb * o.rn.kz;
    if (jj < KS) {
      o.gv = mk(ef.v[jj][2][lane], ef.v[jj][3][lane]);
      o.ev = ph ? mk(ef.v[jj][0][lane], ef.v[jj][1][lane]) : mk(Re(1), Re(0));
    } else {
      const Cx s = crecip(kzb + o.rn.kz);
      o.s2 = s * s;
      o.f = cexp_issue(T, o.C * o.kk);
      if (ph) {
        if (jj < KS + KE)
          o.ev = ef.e_extra(jj, lane);
        else
          o.e = cexp_issue(T, mk(o.D * kzb.im, -o.D * kzb.re));
      }
    }
    return o;
  };
  auto adj_level = [&](int jj, const AdjPre& p) {
    Lev o;
    o.rn = p.rn;
    o.C = p.C;
    o.D = p.D;
    o.it.kk = p.kk;
    o.it.g = (jj < KS) ? p.gv : p.s2 * cexp_finish(p.f);
    o.it.rp = mk(p.Nr, p.Ni) * o.it.g;
    o.e = (jj < 1) ? mk(Re(1), Re(0)) : (jj < KS + KE) ? p.ev : cexp_finish(p.e);
    return o;
  };
  // records of media 0 .. LMAX + 1, each loaded a region before its use
  Rec RA[kPipe ? LMAX + 2 : 1];
  auto load_rec = [&](int m) {
    if (m <= LMAX + 1) RA[m] = L.rec_of(m);
  };
  if constexpr (kPipe && CK) {
    // pairs of levels (jj, jj + 1), jj odd, after level 0: the region that
    // finishes level jj issues level jj + 1's reads; the next one finishes
    // level jj + 1, re-forms the state entering level jj, takes both adjoint
    // steps and issues level jj + 2's reads
    load_rec(0);
    load_rec(1);
    load_rec(2);
    AdjPre cur = adj_pre(0, kzc, RA[0], RA[1]);
    {
      load_rec(3);
      const AdjPre nxt = adj_pre(1, cur.rn.kz, RA[1], RA[2]);
      const Lev l0 = adj_level(0, cur);
      step(0, l0, tapeP[0], tapeQ[0], kzc, iac);
      kzc = l0.rn.kz;
      iac = l0.rn.inv_abs2;
      cur = nxt;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int jj = 1; jj <= LMAX; jj += 2) {
      load_rec(jj + 3);
      const AdjPre pb = adj_pre(jj + 1, cur.rn.kz, RA[jj + 1], RA[jj + 2]);
      const Lev la = adj_level(jj, cur);
      __builtin_amdgcn_sched_barrier(0);
      load_rec(jj + 4);
      AdjPre nxt;
      if (jj + 1 < LMAX) nxt = adj_pre(jj + 2, pb.rn.kz, RA[jj + 2], RA[jj + 3]);
      const Lev lb = adj_level(jj + 1, pb);
      const Cx P1 = tapeP[(jj + 1) / 2], Q1 = tapeQ[(jj + 1) / 2];
      const Cx P0 = cmul_add(lb.it.rp, Q1, P1);
      const Cx Q0 = lb.e * cmul_add(lb.it.rp, P1, Q1);
      step(jj, la, P0, Q0, kzc, iac);
      step(jj + 1, lb, P1, Q1, la.rn.kz, la.rn.inv_abs2);
      kzc = lb.rn.kz;
      iac = lb.rn.inv_abs2;
      if (jj + 1 < LMAX) cur = nxt;
      __builtin_amdgcn_sched_barrier(0);
    }
  } else if constexpr (kPipe) {
    load_rec(0);
    load_rec(1);
    load_rec(2);
    AdjPre cur = adj_pre(0, kzc, RA[0], RA[1]);
#pragma unroll
    for (int jj = 0; jj <= LMAX; ++jj) {
      load_rec(jj + 3);
      AdjPre nxt;
      if (jj < LMAX) nxt = adj_pre(jj + 1, cur.rn.kz, RA[jj + 1], RA[jj + 2]);
      const Lev lv = adj_level(jj, cur);
      step(jj, lv, tapeP[jj], tapeQ[jj], kzc, iac);
      kzc = lv.rn.kz;
      iac = lv.rn.inv_abs2;
      if (jj < LMAX) cur = nxt;
      __builtin_amdgcn_sched_barrier(0);
    }
  } else if constexpr (!CK) {
#pragma unroll
    for (int jj = 0; jj <= LMAX; ++jj) {
      const Lev lv = level(jj, kzc);
      step(jj, lv, tapeP[jj], tapeQ[jj], kzc, iac);
      kzc = lv.rn.kz;
      iac = lv.rn.inv_abs2;
      if ((jj + 1) % kAdjGroup == 0)
        __builtin_amdgcn_sched_barrier(0x0100);  // only LDS reads may move across
    }
  } else {
    {
      const Lev l0 = level(0, kzc);
      step(0, l0, tapeP[0], tapeQ[0], kzc, iac);
      kzc = l0.rn.kz;
      iac = l0.rn.inv_abs2;
    }
    __builtin_amdgcn_sched_barrier(0x0100);
#pragma unroll
    for (int jj = 1; jj <= LMAX; jj += 2) {
      const Lev la = level(jj, kzc);
      const Lev lb = level(jj + 1, la.rn.kz);
      const Cx P1 = tapeP[(jj + 1) / 2], Q1 = tapeQ[(jj + 1) / 2];
      const Cx P0 = cmul_add(lb.it.rp, Q1, P1);
      const Cx Q0 = lb.e * cmul_add(lb.it.rp, P1, Q1);
      step(jj, la, P0, Q0, kzc, iac);
      step(jj + 1, lb, P1, Q1, la.rn.kz, la.rn.inv_abs2);
      kzc = lb.rn.kz;
      iac = lb.rn.inv_abs2;
      if ((jj + 1) % kAdjGroup == 0)
        __builtin_amdgcn_sched_barrier(0x0100);  // only LDS reads may move across
    }
  }
  // Hq += c dR/dq (seeded): dkz0/dq = 1/2 (added at level 0), dw_j/dq = kz0
  if constexpr (RES) Hq = fma(0.25 * q * c, sw, Hq);  // sw holds 2 sum Re(wbar)
  return (double)cabs2(r);
}

// ---------------------------------------------------------------------------
// logL + gradient partials per WU (nr_loglik_grad).
// Record layout (NR = N + 2 media):
//   [0] logL, [1] d/dscale, [2] d/dbkg,
//   [3 + m]        sum Re wbar_m     (wbar_m = cotangent of w_m = kz_m^2)
//   [3 + NR + m]   sum Im wbar_m
//   [3 + 2NR + m]  sum dl/dd_m
//   [3 + 3NR + m]  sum Re(conj(ubar) kz_{m-1} kz_m)   (sigma_m factor applied later)
//   [3 + 4NR]      d/d(dQ/Q) (relative resolution)
// ---------------------------------------------------------------------------
template <class P, int LMAX, bool STORE, bool TAIL, bool RES, bool SPLIT = false>
__global__ __launch_bounds__(64, P::min_waves(LMAX, STORE, TAIL || SPLIT)) void k_loglik_grad(
    KernelArgs a) {
  static_assert(!(STORE && RES), "the resolution derivative has the recompute form only");
  static_assert(!(TAIL && SPLIT), "a unit is packed or split, not both");
  using Re = typename P::real;
  __shared__ Shared s;
  using Tape = typename std::conditional<STORE, GradTape<Re, LMAX>, char>::type;
  __shared__ Tape tape;
  constexpr int KS = STORE ? 1 : P::ef_levels(LMAX);
  constexpr int KE = STORE ? 0 : P::e_levels(LMAX);
  using Ef = typename std::conditional<STORE, char, EfCache<Re, KS, KE>>::type;
  __shared__ Ef efc;
  const int lane = threadIdx.x;
  const int w = blockIdx.x;
  SplitInfo sp{0, 1, 64};
  const WuInfo u = TAIL ? tail_setup(a, w, lane)
                        : SPLIT ? split_setup(a, w, lane, sp) : wu_setup(a, w, lane);
  stage_shared(s, lane, a.rule);
  const int N = u.N;
  const int K = u.smeared ? kSmearNodes : 1;

  Accum<LMAX> acc;
#pragma unroll
  for (int m = 0; m < LMAX + 2; ++m) {
    acc.Hw[m] = mk(0.0, 0.0);
    acc.Hd[m] = 0.0;
    acc.Hs[m] = 0.0;
  }

  double Rsm = 0.0;
  double Hq = 0.0;  // sum_k w_k dR(q_k)/dq_k dq_k/d(dQ/Q)
  bool badq = !(u.Q > 0.0);
  bool edge = false;
  // dq_k/d(dQ/Q) = Q t_k / (2 sqrt(2 ln 2)) for a relative width
  const double dq_dres = (u.smeared && !u.pointwise) ? u.Q / kFwhmPerSigma : 0.0;
  // a split unit's lane takes every G-th node from its group's first
  const int k0 = SPLIT ? (u.active ? sp.g : K) : 0;
  const int kstep = SPLIT ? sp.G : 1;
  for (int k = k0; k < K; k += kstep) {
    const double tk = ld(s.t[k]);
    const double q = (K == 1) ? u.Q : smear_at(u.Q, u.sig, tk);
    badq |= !(q > 0.0);
    const double wk = (K == 1) ? 1.0 : ld(s.w[k]);
    const Layers<P> L = item_layers<P>(a, u.roff, N, k);
    double R;
    if constexpr (STORE)
      R = node_grad_store<P, LMAX>(s.tab, L, tape, acc, lane, q, wk, edge);
    else
      R = node_grad_recompute<P, LMAX, KS, KE, P::checkpoint(LMAX), RES,
                              P::pipelined(LMAX, TAIL || SPLIT || RES)>(
          s.tab, L, efc, acc, lane, q, wk, edge, Hq, RES ? dq_dres * tk : 0.0);
    Rsm += wk * R;
  }
  // the item was evaluated at depth LMAX: the copies of the backing below it
  // (media N + 2 .. LMAX + 1) are the backing's parameters
  {
    cd back = mk(0.0, 0.0);
#pragma unroll
    for (int m = 1; m < LMAX + 2; ++m)
      if (m >= N + 1) back += acc.Hw[m];
#pragma unroll
    for (int m = 1; m < LMAX + 2; ++m)
      if (m == N + 1) acc.Hw[m] = back;
  }

  if constexpr (SPLIT) {
    // the point's smeared R and its q test over its node groups' lanes
    double tot = 0.0;
    int bq = 0;
    for (int gg = 0; gg < sp.G; ++gg) {
      const int src = gg * sp.npts + lane % sp.npts;
      tot += __shfl(Rsm, src, 64);
      bq |= __shfl(badq ? 1 : 0, src, 64);
    }
    Rsm = tot;
    badq = bq != 0;
  }

  // ---- instrument, likelihood, seeds ----
  double ll = 0.0, gsc = 0.0, gbk = 0.0, fac = 0.0;
  uint32_t bits = 0;
  if (u.active) {
    const double sc = a.scale[u.item];
    const double Rhat = sc * Rsm + a.bkg[u.item];
    double ghat;
    if (a.seed != nullptr) {
      // vector-Jacobian product of R_hat: the seed replaces dlogL/dR_hat
      ghat = a.seed[a.out_off[u.item] + u.i];
      ll = badq ? __builtin_nan("") : ghat * Rhat;
      if (badq) bits |= kItemBadQ;
      if (!isfinite(ll)) bits |= kItemNonfinite;
    } else {
      const double e = a.r_err[u.qoff + u.i];
      ll = point_loglik(Rhat, a.r_obs[u.qoff + u.i], e, badq, bits);
      ghat = -(Rhat - a.r_obs[u.qoff + u.i]) / (e * e);
    }
    gsc = ghat * Rsm;
    gbk = ghat;
    fac = ghat * sc;
    if (edge) bits |= kItemEdgeSingular;
    if (SPLIT && sp.g != 0) {
      // the point's value terms once, from its first node group's lane
      ll = 0.0;
      gsc = 0.0;
      gbk = 0.0;
    }
  }
  flag(a.item_status, u.item, bits);

  const int NR = N + 2;
  const double fw = kHwScale * fac, fd = kHdScale * fac;
  // record of 4 + 4 NR doubles; the last field is the resolution sum (0
  // outside the RES form, written all the same so that the records of
  // consecutive units form one contiguous store)
  const int nf = 4 + 4 * NR;
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
        seg_put(3 + m, fw * acc.Hw[m].re);
        seg_put(3 + NR + m, fw * acc.Hw[m].im);
        seg_put(3 + 2 * NR + m, fd * acc.Hd[m]);
        seg_put(3 + 3 * NR + m, fac * acc.Hs[m]);
      }
    }
    if constexpr (RES)
      seg_put(3 + 4 * NR, fac * Hq);
    else if (writer)
      rec[3 + 4 * NR] = 0.0;
    return;
  }
  // ---- wave reduction; the sums go through LDS into one coalesced store ----
  // (staged in the unit's tape or cache, which the sweeps no longer read; a
  // block is one wave, so its LDS accesses stay in program order)
  using Sweep = typename std::conditional<STORE, Tape, Ef>::type;
  static_assert(sizeof(Sweep) >= sizeof(double) * (4 + 4 * (LMAX + 2)),
                "the record staging must fit in the sweep's LDS");
  double* stage = STORE ? reinterpret_cast<double*>(&tape) : reinterpret_cast<double*>(&efc);
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
      const double wr = wave_sum(fw * acc.Hw[m].re);
      const double wi = wave_sum(fw * acc.Hw[m].im);
      const double dd = wave_sum(fd * acc.Hd[m]);
      const double ss = wave_sum(fac * acc.Hs[m]);
      if (lane == 0) {
        stage[3 + m] = wr;
        stage[3 + NR + m] = wi;
        stage[3 + 2 * NR + m] = dd;
        stage[3 + 3 * NR + m] = ss;
      }
    }
  }
  if constexpr (RES) {
    const double hq = wave_sum(fac * Hq);
    if (lane == 0) stage[3 + 4 * NR] = hq;
  } else {
    if (lane == 0) stage[3 + 4 * NR] = 0.0;
  }
  __syncthreads();
  double* rec = a.rec + a.wu_rec[w];
  for (int f = lane; f < nf; f += 64) rec[f] = stage[f];
}

// ---------------------------------------------------------------------------
// Launchers of one precision (instantiated in nr_kernels_f64.hip and
// nr_kernels_f32.hip).
// ---------------------------------------------------------------------------
template <class P>
hipError_t launch_forward_p(int op, bool split, const KernelArgs& a, int n_wu, hipStream_t st) {
  if (n_wu <= 0) return hipSuccess;
  if (op == kOpReflectivity) {
    if (split)
      hipLaunchKernelGGL((k_reflectivity<P, true>), dim3(n_wu), dim3(64), 0, st, a);
    else
      hipLaunchKernelGGL((k_reflectivity<P, false>), dim3(n_wu), dim3(64), 0, st, a);
  } else {
    if (split)
      hipLaunchKernelGGL((k_loglik<P, true>), dim3(n_wu), dim3(64), 0, st, a);
    else
      hipLaunchKernelGGL((k_loglik<P, false>), dim3(n_wu), dim3(64), 0, st, a);
  }
  return hipGetLastError();
}

// Launch of one gradient bucket; BUCKETS is the list macro of the buckets
// this translation unit compiles.
#define NR_LAUNCH(LM, S, RES)                                                                 \
  if (mode == kModeTail)                                                                      \
    hipLaunchKernelGGL((k_loglik_grad<P, LM, S, true, RES>), dim3(n_wu), dim3(64), 0, st, a);  \
  else if (mode == kModeSplit)                                                                \
    hipLaunchKernelGGL((k_loglik_grad<P, LM, S, false, RES, true>), dim3(n_wu), dim3(64), 0,  \
                       st, a);                                                                \
  else                                                                                        \
    hipLaunchKernelGGL((k_loglik_grad<P, LM, S, false, RES>), dim3(n_wu), dim3(64), 0, st, a);
// the kernel form (GradForm) of bucket LM
#define NR_FORMS(LM)                                                                          \
  if (form == kFormRecomputeRes) {                                                            \
    NR_LAUNCH(LM, false, true)                                                                \
  } else if (form == kFormStore) {                                                            \
    if constexpr (LM <= P::kStoreMax) {                                                       \
      NR_LAUNCH(LM, true, false)                                                              \
    } else {                                                                                  \
      return hipErrorInvalidValue;                                                            \
    }                                                                                         \
  } else {                                                                                    \
    NR_LAUNCH(LM, false, false)                                                               \
  }
#define NR_CASE(LM)                                                                           \
  case LM:                                                                                    \
    NR_FORMS(LM)                                                                              \
    return hipGetLastError();
#define NR_DEFINE_GRAD_LAUNCHER(NAME, BUCKETS)                                                \
  template <class P>                                                                          \
  hipError_t NAME(int bucket, int form, int mode, const KernelArgs& a, int n_wu,            \
                  hipStream_t st) {                                                           \
    if (n_wu <= 0) return hipSuccess;                                                         \
    switch (kBucketLmax[bucket]) {                                                            \
      BUCKETS(NR_CASE)                                                                        \
      default:                                                                                \
        return hipErrorInvalidValue;                                                          \
    }                                                                                         \
  }

}  // namespace nr
