// Gradient kernel for deep stacks (more than NR_MAX_LAYERS layers, e.g.
// microsliced SLD profiles): the layer product is split across the 64 lanes
// of a wave and combined by an associative scan of 2x2 transfer matrices; the
// adjoint runs as the reverse scan.  One wave per (item, data point); the
// point's smearing nodes are processed in turn.
//
// In the scaled form the state entering level j maps to the state leaving it
// by T_j = [[1, r'_j], [e_j r'_j, e_j]] (e_0 = 1), so the top state is
// T_0 T_1 ... T_N (1, 0)^T and r = Qv / P.  Lane l owns the levels
// [l CH, (l + 1) CH) (CH = ceil((N + 1) / 64)) and the media of those levels:
//   1. its chunk product M_l = T_{l CH} ... T_{(l+1) CH - 1} (two columns);
//   2. an inclusive suffix scan U_l = M_l ... M_63 gives the state entering
//      each chunk from below (column 0 of U_{l+1}) and the top state (U_0);
//      an inclusive prefix scan W_l = M_0 ... M_l gives, with V_l = W_{l-1},
//      the cotangent of the state leaving the chunk at its top, V_l^H c_0
//      (the cotangent of a linear map's input is its conjugate transpose
//      applied to the output's cotangent);
//   3. the lane's own forward sweep from its entering state (the state tape
//      in LDS) and the level-by-level adjoint of the shallow kernels.
// A medium at a chunk boundary receives cotangent contributions from two
// lanes; the lower lane's part is kept in an extra slot and added to the
// upper lane's slot before the record is written.  Every level's arithmetic
// is that of the shallow kernels (same helpers), in FP64.
#include "nr_kernels.hpp"

namespace nr {

namespace {

struct M2 {
  cd a, b, c, d;  // [[a, b], [c, d]]
};

__device__ __forceinline__ M2 m2_mul(const M2& x, const M2& y) {
  M2 z;
  z.a = x.a * y.a + x.b * y.c;
  z.b = x.a * y.b + x.b * y.d;
  z.c = x.c * y.a + x.d * y.c;
  z.d = x.c * y.b + x.d * y.d;
  return z;
}

__device__ __forceinline__ M2 m2_identity() {
  M2 z;
  z.a = mk(1.0, 0.0);
  z.b = mk(0.0, 0.0);
  z.c = mk(0.0, 0.0);
  z.d = mk(1.0, 0.0);
  return z;
}

__device__ __forceinline__ cd shfl_cd(cd v, int src) {
  return mk(__shfl(v.re, src, 64), __shfl(v.im, src, 64));
}

__device__ __forceinline__ M2 shfl_m2(const M2& m, int src) {
  M2 z;
  z.a = shfl_cd(m.a, src);
  z.b = shfl_cd(m.b, src);
  z.c = shfl_cd(m.c, src);
  z.d = shfl_cd(m.d, src);
  return z;
}

// Level jj's coefficients from kz_jj (kzc) and medium jj + 1's root.
struct Lvl {
  Iface<double> it;
  cd e;
  double C, D;
};

__device__ __forceinline__ Lvl level_coeffs(const MathTables& T, const Layers<F64>& L, int jj,
                                            cd kzc, cd kzn) {
  Lvl o;
  o.C = L.C(jj);
  o.D = (jj >= 1) ? L.D(jj) : 0.0;
  o.it = interface_coeffs(T, kzc, kzn, L.Nr(jj), L.Ni(jj), o.C);
  o.e = (jj >= 1) ? layer_phase(T, kzc, o.D) : mk(1.0, 0.0);
  return o;
}

}  // namespace

// Dynamic LDS: the state tape [ch_max][4][64] (P re, P im, Qv re, Qv im of
// the state entering each of the lane's levels), then the accumulators
// [ch_max + 1][4][64] (Hw re, Hw im, Hd, Hs per medium slot; slot t is medium
// lo + t, the last used slot is the lane's lower boundary medium).
template <bool RES>
__global__ __launch_bounds__(64) void k_loglik_grad_scan(KernelArgs a, int ch_max) {
  __shared__ Shared s;
  extern __shared__ double dyn[];
  const int lane = threadIdx.x;
  const int w = blockIdx.x;
  const int item = a.wu_item[w];
  const int ds = a.dataset_of_item[item];
  const int64_t qoff = a.q_off[ds];
  const int i = a.wu_p0[w];
  const int64_t roff = a.row_off[item];
  const int N = (int)(a.row_off[item + 1] - roff) - 2;
  const int NL = N + 1;  // levels 0..N
  const int CH = (NL + 63) / 64;
  const int lo = min(lane * CH, NL), hi = min(lo + CH, NL);
  const bool own = lo < hi;
  stage_shared(s, lane, a.rule);
  double* tape = dyn;
  double* acc = dyn + (size_t)ch_max * 4 * 64;
  auto TP = [&](int t, int f) -> double& { return tape[(t * 4 + f) * 64 + lane]; };
  auto AC = [&](int t, int f) -> double& { return acc[(t * 4 + f) * 64 + lane]; };
  for (int t = 0; t <= CH; ++t)
    for (int f = 0; f < 4; ++f) AC(t, f) = 0.0;

  const double Q = a.q[qoff + i];
  const bool smeared = a.dq_over_q[ds] > 0.0;
  const double dqq = a.dqq_item ? a.dqq_item[item] : a.dq_over_q[ds];
  const bool pointwise = a.dq != nullptr;
  const double sig = pointwise ? smear_sigma_abs(a.dq[qoff + i]) : smear_sigma_rel(Q, dqq);
  const double dq_dres = (smeared && !pointwise) ? Q / kFwhmPerSigma : 0.0;
  const int K = smeared ? kSmearNodes : 1;
  const Layers<F64> L = item_layers<F64>(a, roff, N, 0);

  double Rsm = 0.0, Hq = 0.0;
  bool badq = !(Q > 0.0);
  bool edge = false;
  for (int k = 0; k < K; ++k) {
    const double tk = ld(s.t[k]);
    const double q = (K == 1) ? Q : smear_at(Q, sig, tk);
    badq |= !(q > 0.0);
    const double wk = (K == 1) ? 1.0 : ld(s.w[k]);
    const double kz0sq = kz0_squared(q);
    const cd kz0 = fronting_kz<F64>(q);

    // 1. the chunk product, applied to both columns bottom-up
    M2 X = m2_identity();
    if (own) {
      cd kzn = medium_root(L, kz0sq, hi).kz;
      for (int jj = hi - 1; jj >= lo; --jj) {
        const cd kzc = (jj == 0) ? kz0 : medium_root(L, kz0sq, jj).kz;
        const Lvl lv = level_coeffs(s.tab, L, jj, kzc, kzn);
        const cd a0 = X.a + lv.it.rp * X.c, b0 = X.b + lv.it.rp * X.d;
        X.c = lv.e * (lv.it.rp * X.a + X.c);
        X.d = lv.e * (lv.it.rp * X.b + X.d);
        X.a = a0;
        X.b = b0;
        kzn = kzc;
      }
    }
    // 2. suffix and prefix scans across the lanes
    M2 U = X, W = X;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const M2 Yu = shfl_m2(U, lane + off < 64 ? lane + off : 63);
      const M2 Yw = shfl_m2(W, lane >= off ? lane - off : 0);
      if (lane + off < 64) U = m2_mul(U, Yu);
      if (lane >= off) W = m2_mul(Yw, W);
    }
    const M2 Ub = shfl_m2(U, lane < 63 ? lane + 1 : 63);
    const M2 V = shfl_m2(W, lane > 0 ? lane - 1 : 0);
    const cd P0 = shfl_cd(U.a, 0), Q0 = shfl_cd(U.c, 0);
    const cd iP = crecip(P0);
    const cd r = Q0 * iP;
    Rsm += wk * cabs2(r);
    const cd rbar = (2.0 * wk) * r;
    const cd Pb0 = cmulc(-(r * iP), rbar);
    const cd Qb0 = cmulc(iP, rbar);
    cd Pb = Pb0, Qb = Qb0;
    if (lane > 0) {
      Pb = cmulc(V.a, Pb0) + cmulc(V.c, Qb0);
      Qb = cmulc(V.b, Pb0) + cmulc(V.d, Qb0);
    }
    cd Ps = mk(1.0, 0.0), Qs = mk(0.0, 0.0);
    if (lane < 63) {
      Ps = Ub.a;
      Qs = Ub.c;
    }
    if (!own) continue;

    // 3. the lane's forward sweep (state tape) and adjoint
    {
      cd Pv = Ps, Qv = Qs;
      cd kzn = medium_root(L, kz0sq, hi, edge).kz;
      for (int jj = hi - 1; jj >= lo; --jj) {
        TP(jj - lo, 0) = Pv.re;
        TP(jj - lo, 1) = Pv.im;
        TP(jj - lo, 2) = Qv.re;
        TP(jj - lo, 3) = Qv.im;
        const cd kzc = (jj == 0) ? kz0 : medium_root(L, kz0sq, jj, edge).kz;
        const Lvl lv = level_coeffs(s.tab, L, jj, kzc, kzn);
        const cd Pn = Pv + lv.it.rp * Qv;
        const cd t = lv.it.rp * Pv + Qv;
        Qv = (jj >= 1) ? lv.e * t : t;
        Pv = Pn;
        kzn = kzc;
      }
    }
    double sw = 0.0;
    RootT<double> rc;
    if (lo == 0) {
      rc.kz = kz0;
      rc.inv_abs2 = 0.0;
    } else {
      rc = medium_root(L, kz0sq, lo);
    }
    cd kzbc = mk(0.0, 0.0);
    for (int jj = lo; jj < hi; ++jj) {
      const RootT<double> rn = medium_root(L, kz0sq, jj + 1);
      const Lvl lv = level_coeffs(s.tab, L, jj, rc.kz, rn.kz);
      const cd Pt = mk(TP(jj - lo, 0), TP(jj - lo, 1));
      const cd Qt = mk(TP(jj - lo, 2), TP(jj - lo, 3));
      const bool ph = jj >= 1;
      const AdjStep<double> st =
          adjoint_step(Pt, Qt, Pb, Qb, rc.kz, rn.kz, lv.it, lv.C, ph, lv.e, lv.D);
      kzbc += st.kzb_c;
      if constexpr (RES)
        if (jj == 0) Hq = fma(0.5 * dq_dres * tk, kzbc.re, Hq);
      {
        double hs = AC(jj + 1 - lo, 3);
        acc_re_dot(hs, st.ub, lv.it.kk);
        AC(jj + 1 - lo, 3) = hs;
      }
      if (ph) {
        double hd = AC(jj - lo, 2);
        acc_dd(hd, rc.kz, st.w);
        AC(jj - lo, 2) = hd;
        cd hw = mk(AC(jj - lo, 0), AC(jj - lo, 1));
        acc_wbar<RES>(hw, sw, rc.kz, rc.inv_abs2, kzbc);
        AC(jj - lo, 0) = hw.re;
        AC(jj - lo, 1) = hw.im;
      }
      Pb = st.Pb;
      Qb = st.Qb;
      kzbc = st.kzb_n;
      rc = rn;
    }
    {
      // this lane's part of the lower boundary medium (hi), from level hi - 1
      cd hw = mk(AC(hi - lo, 0), AC(hi - lo, 1));
      acc_wbar<RES>(hw, sw, rc.kz, rc.inv_abs2, kzbc);
      AC(hi - lo, 0) = hw.re;
      AC(hi - lo, 1) = hw.im;
    }
    if constexpr (RES) Hq = fma(0.5 * q * dq_dres * tk, sw, Hq);
  }

  // ---- the point's likelihood and seed (lane-uniform) ----
  const int NR = N + 2;
  const double sc = a.scale[item];
  const double Rhat = sc * Rsm + a.bkg[item];
  uint32_t bits = 0;
  double ll, ghat;
  if (a.seed != nullptr) {
    ghat = a.seed[a.out_off[item] + i];
    ll = badq ? __builtin_nan("") : ghat * Rhat;
    if (badq) bits |= kItemBadQ;
    if (!isfinite(ll)) bits |= kItemNonfinite;
  } else {
    const double e = a.r_err[qoff + i];
    ll = point_loglik(Rhat, a.r_obs[qoff + i], e, badq, bits);
    ghat = -(Rhat - a.r_obs[qoff + i]) / (e * e);
  }
  const double fac = ghat * sc;
  if (__ballot(edge) != 0) bits |= kItemEdgeSingular;
  if (lane == 0) flag(a.item_status, item, bits);

  // ---- the record: boundary slots join the next lane's first medium ----
  double* rec = a.rec + a.wu_rec[w];
  const int bslot = own ? hi - lo : 0;
  double from_above[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const double v = own ? AC(bslot, f) : 0.0;
    from_above[f] = __shfl(v, lane > 0 ? lane - 1 : 0, 64);
  }
  if (own && lane > 0)
    for (int f = 0; f < 4; ++f) AC(0, f) += from_above[f];
  if (own) {
    for (int t = 0; t < hi - lo; ++t) {
      const int m = lo + t;
      rec[3 + m] = fac * AC(t, 0);
      rec[3 + NR + m] = fac * AC(t, 1);
      rec[3 + 2 * NR + m] = fac * AC(t, 2);
      rec[3 + 3 * NR + m] = fac * AC(t, 3);
    }
    if (hi == NL) {  // the backing medium N + 1
      rec[3 + NL] = fac * AC(bslot, 0);
      rec[3 + NR + NL] = fac * AC(bslot, 1);
      rec[3 + 2 * NR + NL] = fac * AC(bslot, 2);
      rec[3 + 3 * NR + NL] = fac * AC(bslot, 3);
    }
  }
  const double hq = RES ? wave_sum(Hq) : 0.0;
  if (lane == 0) {
    rec[0] = ll;
    rec[1] = ghat * Rsm;
    rec[2] = ghat;
    if (RES) rec[3 + 4 * NR] = fac * hq;
  }
}

size_t scan_lds_bytes(int ch_max) {
  return sizeof(double) * ((size_t)ch_max * 4 * 64 + (size_t)(ch_max + 1) * 4 * 64);
}

hipError_t prepare_grad_scan(int ch_max) {
  const int bytes = (int)scan_lds_bytes(ch_max);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_loglik_grad_scan<false>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_loglik_grad_scan<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  return e;
}

hipError_t launch_grad_scan(bool res, int ch_max, const KernelArgs& a, int n_wu, hipStream_t st) {
  if (n_wu <= 0) return hipSuccess;
  const size_t lds = scan_lds_bytes(ch_max);
  if (res)
    hipLaunchKernelGGL(k_loglik_grad_scan<true>, dim3(n_wu), dim3(64), lds, st, a, ch_max);
  else
    hipLaunchKernelGGL(k_loglik_grad_scan<false>, dim3(n_wu), dim3(64), lds, st, a, ch_max);
  return hipGetLastError();
}

}  // namespace nr
