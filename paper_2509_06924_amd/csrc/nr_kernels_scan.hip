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
//   3. the lane's own forward sweep from its entering state (the state tape,
//      in registers or LDS) and the level-by-level adjoint of the shallow
//      kernels.
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

// Per-lane storage of the state tape (the state entering each of the lane's
// levels) and of the accumulators (Hw re, Hw im, Hd, Hs per medium slot; slot
// t is medium lo + t, slot n = hi - lo the lane's lower boundary medium):
// registers where they fit, else LDS in lane-interleaved planes.
template <int CHT, bool IN_LDS>
struct LaneTape {
  double r[IN_LDS ? 1 : CHT][4];
  __device__ __forceinline__ double& at(double* lds, int lane, int t, int f) {
    if constexpr (IN_LDS)
      return lds[(t * 4 + f) * 64 + lane];
    else
      return r[t][f];
  }
};

// CHT: the largest levels-per-lane the launch's items need (1 .. 32).
template <int CHT, bool RES>
__global__ __launch_bounds__(64) void k_loglik_grad_scan(KernelArgs a) {
  constexpr bool kTapeLds = CHT >= 8;
  constexpr bool kAccLds = CHT >= 32;
  __shared__ Shared s;
  __shared__ double tape_lds[kTapeLds ? CHT * 4 * 64 : 1];
  __shared__ double acc_lds[kAccLds ? (CHT + 1) * 4 * 64 : 1];
  LaneTape<CHT, kTapeLds> tape;
  LaneTape<CHT + 1, kAccLds> accs;
  const int lane = threadIdx.x;
  auto TP = [&](int t, int f) -> double& { return tape.at(tape_lds, lane, t, f); };
  auto AC = [&](int t, int f) -> double& { return accs.at(acc_lds, lane, t, f); };

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
  const int n = hi - lo;  // levels of this lane (0 .. CH <= CHT)
  const bool own = n > 0;
  stage_shared(s, lane, a.rule);
#pragma unroll
  for (int t = 0; t <= CHT; ++t)
#pragma unroll
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

    // 1. the chunk product, applied to both columns bottom-up; each level's
    //    r' and e are kept in its tape slot for the re-run in step 3
    M2 X = m2_identity();
    if (own) {
      cd kzn = medium_root(L, kz0sq, hi, edge).kz;
#pragma unroll
      for (int t = CHT - 1; t >= 0; --t) {
        if (t < n) {
          const int jj = lo + t;
          const cd kzc = (jj == 0) ? kz0 : medium_root(L, kz0sq, jj, edge).kz;
          const Lvl lv = level_coeffs(s.tab, L, jj, kzc, kzn);
          TP(t, 0) = lv.it.rp.re;
          TP(t, 1) = lv.it.rp.im;
          TP(t, 2) = lv.e.re;
          TP(t, 3) = lv.e.im;
          const cd a0 = X.a + lv.it.rp * X.c, b0 = X.b + lv.it.rp * X.d;
          X.c = lv.e * (lv.it.rp * X.a + X.c);
          X.d = lv.e * (lv.it.rp * X.b + X.d);
          X.a = a0;
          X.b = b0;
          kzn = kzc;
        }
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

    // 3. the lane's forward sweep from its entering state with the r' and e
    //    of step 1; each slot then holds the state entering its level
    {
      cd Pv = Ps, Qv = Qs;
#pragma unroll
      for (int t = CHT - 1; t >= 0; --t) {
        if (t < n) {
          const cd rp = mk(TP(t, 0), TP(t, 1));
          const cd e = mk(TP(t, 2), TP(t, 3));
          TP(t, 0) = Pv.re;
          TP(t, 1) = Pv.im;
          TP(t, 2) = Qv.re;
          TP(t, 3) = Qv.im;
          const cd Pn = Pv + rp * Qv;
          Qv = e * (rp * Pv + Qv);  // e = 1 at level 0
          Pv = Pn;
        }
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
#pragma unroll
    for (int t = 0; t < CHT; ++t) {
      if (t < n) {
        const int jj = lo + t;
        const RootT<double> rn = medium_root(L, kz0sq, jj + 1);
        const Lvl lv = level_coeffs(s.tab, L, jj, rc.kz, rn.kz);
        const cd Pt = mk(TP(t, 0), TP(t, 1));
        const cd Qt = mk(TP(t, 2), TP(t, 3));
        const bool ph = jj >= 1;
        const AdjStep<double> st =
            adjoint_step(Pt, Qt, Pb, Qb, rc.kz, rn.kz, lv.it, lv.C, ph, lv.e, lv.D);
        kzbc += st.kzb_c;
        if constexpr (RES)
          if (jj == 0) Hq = fma(0.5 * dq_dres * tk, kzbc.re, Hq);
        {
          double hs = AC(t + 1, 3);
          acc_re_dot(hs, st.ub, lv.it.kk);
          AC(t + 1, 3) = hs;
        }
        if (ph) {
          double hd = AC(t, 2);
          acc_dd(hd, rc.kz, st.w);
          AC(t, 2) = hd;
          cd hw = mk(AC(t, 0), AC(t, 1));
          acc_wbar<RES>(hw, sw, rc.kz, rc.inv_abs2, kzbc);
          AC(t, 0) = hw.re;
          AC(t, 1) = hw.im;
        }
        Pb = st.Pb;
        Qb = st.Qb;
        kzbc = st.kzb_n;
        rc = rn;
        if (t == n - 1) {
          // this lane's part of its lower boundary medium (hi), from level hi - 1
          cd hw = mk(AC(t + 1, 0), AC(t + 1, 1));
          acc_wbar<RES>(hw, sw, rc.kz, rc.inv_abs2, kzbc);
          AC(t + 1, 0) = hw.re;
          AC(t + 1, 1) = hw.im;
        }
      }
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
  double bnd[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 1; t <= CHT; ++t)
    if (t == n)
#pragma unroll
      for (int f = 0; f < 4; ++f) bnd[f] = AC(t, f);
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const double from_above = __shfl(bnd[f], lane > 0 ? lane - 1 : 0, 64);
    if (own && lane > 0) AC(0, f) += from_above;
  }
  if (own) {
#pragma unroll
    for (int t = 0; t < CHT; ++t) {
      if (t < n) {
        const int m = lo + t;
        rec[3 + m] = fac * AC(t, 0);
        rec[3 + NR + m] = fac * AC(t, 1);
        rec[3 + 2 * NR + m] = fac * AC(t, 2);
        rec[3 + 3 * NR + m] = fac * AC(t, 3);
      }
    }
    if (hi == NL) {  // the backing medium N + 1
      rec[3 + NL] = fac * bnd[0];
      rec[3 + NR + NL] = fac * bnd[1];
      rec[3 + 2 * NR + NL] = fac * bnd[2];
      rec[3 + 3 * NR + NL] = fac * bnd[3];
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

// The kernel instance for a launch: levels-per-lane rounded up to a power of
// two (register tape up to 4, register accumulators up to 16).
static int scan_cht(int ch_max) {
  int c = 1;
  while (c < ch_max) c <<= 1;
  return c;
}

size_t scan_lds_bytes(int ch_max) {
  const int c = scan_cht(ch_max);
  size_t b = sizeof(Shared);
  if (c >= 8) b += sizeof(double) * (size_t)c * 4 * 64;
  if (c >= 32) b += sizeof(double) * (size_t)(c + 1) * 4 * 64;
  return b;
}

hipError_t prepare_grad_scan(int ch_max) {
  // static LDS only; the instances exist up to 32 levels per lane
  return (ch_max >= 1 && scan_cht(ch_max) <= kScanMaxChunk) ? hipSuccess : hipErrorInvalidValue;
}

template <int CHT>
static void launch_scan_cht(bool res, const KernelArgs& a, int n_wu, hipStream_t st) {
  if (res)
    hipLaunchKernelGGL((k_loglik_grad_scan<CHT, true>), dim3(n_wu), dim3(64), 0, st, a);
  else
    hipLaunchKernelGGL((k_loglik_grad_scan<CHT, false>), dim3(n_wu), dim3(64), 0, st, a);
}

hipError_t launch_grad_scan(bool res, int ch_max, const KernelArgs& a, int n_wu, hipStream_t st) {
  if (n_wu <= 0) return hipSuccess;
  switch (scan_cht(ch_max)) {
    case 1: launch_scan_cht<1>(res, a, n_wu, st); break;
    case 2: launch_scan_cht<2>(res, a, n_wu, st); break;
    case 4: launch_scan_cht<4>(res, a, n_wu, st); break;
    case 8: launch_scan_cht<8>(res, a, n_wu, st); break;
    case 16: launch_scan_cht<16>(res, a, n_wu, st); break;
    case 32: launch_scan_cht<32>(res, a, n_wu, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nr
