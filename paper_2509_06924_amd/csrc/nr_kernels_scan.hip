// Gradient kernel for deep stacks (more than NR_MAX_LAYERS layers, e.g.
// microsliced SLD profiles): the layer product is split across the 64 lanes
// of a wave and combined by an associative scan of 2x2 transfer matrices; the
// adjoint runs as the reverse scan.  One workgroup of NW waves per (item,
// data point), NT = 64 NW lanes; the point's smearing nodes are processed in
// turn.
//
// In the scaled form the state entering level j maps to the state leaving it
// by T_j = [[1, r'_j], [e_j r'_j, e_j]] (e_0 = 1), so the top state is
// T_0 T_1 ... T_N (1, 0)^T and r = Qv / P.  Lane l owns the levels
// [l CH, (l + 1) CH) (CH = ceil((N + 1) / NT)) and the media of those levels:
//   1. its chunk product M_l = T_{l CH} ... T_{(l+1) CH - 1} (two columns);
//   2. an inclusive suffix scan U_l = M_l ... M_{NT-1} gives the state
//      entering each chunk from below (column 0 of U_{l+1}) and the top
//      state (U_0);
//      an inclusive prefix scan W_l = M_0 ... M_l gives, with V_l = W_{l-1},
//      the cotangent of the state leaving the chunk at its top, V_l^H c_0
//      (the cotangent of a linear map's input is its conjugate transpose
//      applied to the output's cotangent).  Each wave scans its own lanes
//      with shuffles; across waves the scans are completed with the waves'
//      chunk-product totals, exchanged through LDS;
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

// (r: the record of level jj, loaded ahead by the caller)
__device__ __forceinline__ Lvl level_coeffs(const MathTables& T, const Layers<F64>::Rec& r, int jj,
                                            cd kzc, cd kzn) {
  Lvl o;
  o.C = r.C;
  o.D = (jj >= 1) ? r.D : 0.0;
  o.it = interface_coeffs(T, kzc, kzn, r.Nr, r.Ni, o.C);
  o.e = (jj >= 1) ? layer_phase(T, kzc, o.D) : mk(1.0, 0.0);
  return o;
}

// kz of a medium from its record, recording an exact zero of w (the edge).
__device__ __forceinline__ RootT<double> rec_root(const Layers<F64>::Rec& r, double kz0sq,
                                                  bool& edge) {
  const double x = kz_real_part(kz0sq, r.A);
  edge |= (x == 0.0) & (r.B == 0.0);
  return kz_root(x, -r.B);
}
__device__ __forceinline__ RootT<double> rec_root(const Layers<F64>::Rec& r, double kz0sq) {
  return kz_root(kz_real_part(kz0sq, r.A), -r.B);
}

}  // namespace

// Per-lane storage of the state tape (the state entering each of the lane's
// levels; between steps 1 and 3, the level's r' and e) and of the
// accumulators (Hw re, Hw im, Hd, Hs per medium slot; slot t is medium lo + t,
// slot n = hi - lo the lane's lower boundary medium): registers, or LDS in
// planes interleaved over the NT lanes of a data point.
template <int CHT, bool IN_LDS, int NT>
struct LaneTape {
  double r[IN_LDS ? 1 : CHT][4];
  __device__ __forceinline__ double& at(double* lds, int gl, int t, int f) {
    if constexpr (IN_LDS)
      return lds[(t * 4 + f) * NT + gl];
    else
      return r[t][f];
  }
};

__device__ __forceinline__ M2 load_m2(const cd* x) {
  M2 z;
  z.a = x[0];
  z.b = x[1];
  z.c = x[2];
  z.d = x[3];
  return z;
}

// CHT: the largest levels-per-lane the launch's items need (1, 2, 4 or 8);
// NW: waves per data point (1, 2 or 4).
template <int CHT, int NW, bool RES>
__global__ __launch_bounds__(64 * NW, 2) void k_loglik_grad_scan(KernelArgs a) {
  constexpr int NT = 64 * NW;
  constexpr bool kTapeLds = CHT >= 8;
  __shared__ Shared s;
  __shared__ double tape_lds[kTapeLds ? CHT * 4 * NT : 1];
  // per wave: the product of its lanes' chunks, its last lane's boundary
  // slot and its part of the resolution derivative
  __shared__ cd xt[NW][4];
  __shared__ double xb[NW][5];
  LaneTape<CHT, kTapeLds, NT> tape;
  LaneTape<CHT + 1, false, NT> accs;
  const int gl = threadIdx.x;  // lane of the data point
  const int lane = gl & 63;    // lane of the wave
  const int wv = gl >> 6;      // wave of the data point
  auto TP = [&](int t, int f) -> double& { return tape.at(tape_lds, gl, t, f); };
  auto AC = [&](int t, int f) -> double& { return accs.at(nullptr, gl, t, f); };

  const int w = blockIdx.x;
  const int item = a.wu_item[w];
  const int ds = a.dataset_of_item[item];
  const int64_t qoff = a.q_off[ds];
  const int i = a.wu_p0[w];
  const int64_t roff = a.row_off[item];
  const int N = (int)(a.row_off[item + 1] - roff) - 2;
  const int NL = N + 1;  // levels 0..N
  const int CH = (NL + NT - 1) / NT;
  const int lo = min(gl * CH, NL), hi = min(lo + CH, NL);
  const int n = hi - lo;  // levels of this lane (0 .. CH <= CHT)
  const bool own = n > 0;
  stage_shared(s, lane, a.rule, wv == 0);
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
      // each level's record (per-lane vector loads) is loaded a level ahead
      cd kzn = rec_root(L.rec_of(hi), kz0sq, edge).kz;
      Layers<F64>::Rec rnx = L.rec_of(hi - 1);
#pragma unroll
      for (int t = CHT - 1; t >= 0; --t) {
        if (t < n) {
          const int jj = lo + t;
          const Layers<F64>::Rec rc = rnx;
          if (t >= 1) rnx = L.rec_of(jj - 1);
          const cd kzc = (jj == 0) ? kz0 : rec_root(rc, kz0sq, edge).kz;
          const Lvl lv = level_coeffs(s.tab, rc, jj, kzc, kzn);
          TP(t, 0) = lv.it.rp.re;
          TP(t, 1) = lv.it.rp.im;
          TP(t, 2) = lv.e.re;
          TP(t, 3) = lv.e.im;
          const cd a0 = cmul_add(lv.it.rp, X.c, X.a), b0 = cmul_add(lv.it.rp, X.d, X.b);
          X.c = lv.e * cmul_add(lv.it.rp, X.a, X.c);
          X.d = lv.e * cmul_add(lv.it.rp, X.b, X.d);
          X.a = a0;
          X.b = b0;
          kzn = kzc;
        }
      }
    }
    // 2. suffix and prefix scans across the wave's lanes ...
    M2 U = X, W = X;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const M2 Yu = shfl_m2(U, lane + off < 64 ? lane + off : 63);
      const M2 Yw = shfl_m2(W, lane >= off ? lane - off : 0);
      if (lane + off < 64) U = m2_mul(U, Yu);
      if (lane >= off) W = m2_mul(Yw, W);
    }
    // ... and across the waves: with T_v the product of wave v's chunks,
    // U_l = U_l(wave) T_{wv+1} ... T_{NW-1}, W_l = T_0 ... T_{wv-1} W_l(wave)
    M2 Ub, V;
    cd P0, Q0;
    if constexpr (NW == 1) {
      Ub = shfl_m2(U, lane < 63 ? lane + 1 : 63);
      V = shfl_m2(W, lane > 0 ? lane - 1 : 0);
      P0 = shfl_cd(U.a, 0);
      Q0 = shfl_cd(U.c, 0);
    } else {
      if (lane == 0) {
        xt[wv][0] = U.a;
        xt[wv][1] = U.b;
        xt[wv][2] = U.c;
        xt[wv][3] = U.d;
      }
      __syncthreads();
      M2 S = m2_identity(), Pp = m2_identity(), F = load_m2(xt[0]);
#pragma unroll
      for (int v = NW - 1; v >= 1; --v)
        if (v > wv) S = m2_mul(load_m2(xt[v]), S);
#pragma unroll
      for (int v = 0; v < NW - 1; ++v)
        if (v < wv) Pp = m2_mul(Pp, load_m2(xt[v]));
      // the top state, formed in the same order by every lane
#pragma unroll
      for (int v = 1; v < NW; ++v) F = m2_mul(F, load_m2(xt[v]));
      __syncthreads();  // xt is written again at the next node
      U = m2_mul(U, S);
      W = m2_mul(Pp, W);
      Ub = shfl_m2(U, lane < 63 ? lane + 1 : 63);
      V = shfl_m2(W, lane > 0 ? lane - 1 : 0);
      if (lane == 63) Ub = S;  // the next wave's first lane
      if (lane == 0) V = Pp;   // the previous wave's last lane
      P0 = F.a;
      Q0 = F.c;
    }
    const cd iP = crecip(P0);
    const cd r = Q0 * iP;
    Rsm += wk * cabs2(r);
    const cd rbar = (2.0 * wk) * r;
    const cd Pb0 = cmulc(-(r * iP), rbar);
    const cd Qb0 = cmulc(iP, rbar);
    cd Pb = Pb0, Qb = Qb0;
    if (gl > 0) {
      Pb = cmulc(V.a, Pb0) + cmulc(V.c, Qb0);
      Qb = cmulc(V.b, Pb0) + cmulc(V.d, Qb0);
    }
    cd Ps = mk(1.0, 0.0), Qs = mk(0.0, 0.0);
    if (gl < NT - 1) {
      Ps = Ub.a;
      Qs = Ub.c;
    }
    if (!own) continue;

    // 3. the lane's forward sweep from its entering state with the r' and e
    //    of step 1; each slot then holds the state entering its level
    {
      cd Pv = Ps, Qv = Qs;
      // (each slot's r' and e are read a level ahead of their use)
      // (slot n - 1 found by a compile-time loop: the register tape takes
      // no runtime index)
      cd rpn = mk(0.0, 0.0), en = mk(0.0, 0.0);
#pragma unroll
      for (int t = 0; t < CHT; ++t) {
        if (t == n - 1) {
          rpn = mk(TP(t, 0), TP(t, 1));
          en = mk(TP(t, 2), TP(t, 3));
        }
      }
#pragma unroll
      for (int t = CHT - 1; t >= 0; --t) {
        if (t < n) {
          const cd rp = rpn;
          const cd e = en;
          if (t >= 1) {
            rpn = mk(TP(t - 1, 0), TP(t - 1, 1));
            en = mk(TP(t - 1, 2), TP(t - 1, 3));
          }
          TP(t, 0) = Pv.re;
          TP(t, 1) = Pv.im;
          TP(t, 2) = Qv.re;
          TP(t, 3) = Qv.im;
          const cd Pn = cmul_add(rp, Qv, Pv);
          Qv = e * cmul_add(rp, Pv, Qv);  // e = 1 at level 0
          Pv = Pn;
        }
      }
    }
    double sw = 0.0;
    // records a level ahead: ri of level jj, rm of medium jj + 1
    Layers<F64>::Rec ri = L.rec_of(lo), rm = L.rec_of(lo + 1);
    RootT<double> rc;
    if (lo == 0) {
      rc.kz = kz0;
      rc.inv_abs2 = 0.0;
    } else {
      rc = rec_root(ri, kz0sq);
    }
    cd kzbc = mk(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < CHT; ++t) {
      if (t < n) {
        const int jj = lo + t;
        const Layers<F64>::Rec rnext = L.rec_of(jj + 2);
        const RootT<double> rn = rec_root(rm, kz0sq);
        const Lvl lv = level_coeffs(s.tab, ri, jj, rc.kz, rn.kz);
        ri = rm;
        rm = rnext;
        const cd Pt = mk(TP(t, 0), TP(t, 1));
        const cd Qt = mk(TP(t, 2), TP(t, 3));
        const bool ph = jj >= 1;
        const AdjStep<double> st =
            adjoint_step(Pt, Qt, Pb, Qb, rc.kz, rn.kz, lv.it, lv.C, ph, lv.e, lv.D, kzbc);
        kzbc = st.kzb_c;
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
    if constexpr (RES) Hq = fma(0.25 * q * dq_dres * tk, sw, Hq);  // sw: 2 sum Re(wbar)
  }

  // ---- the point's likelihood and seed (uniform over the lanes) ----
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
  const double fw = kHwScale * fac, fd = kHdScale * fac;
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
  double from_above[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) from_above[f] = __shfl(bnd[f], lane > 0 ? lane - 1 : 0, 64);
  double hq = RES ? wave_sum(Hq) : 0.0;
  if constexpr (NW > 1) {
    if (lane == 63)
#pragma unroll
      for (int f = 0; f < 4; ++f) xb[wv][f] = bnd[f];
    if (lane == 0) xb[wv][4] = hq;
    __syncthreads();
    if (lane == 0 && wv > 0)
#pragma unroll
      for (int f = 0; f < 4; ++f) from_above[f] = xb[wv - 1][f];
    if constexpr (RES) {
      hq = 0.0;
#pragma unroll
      for (int v = 0; v < NW; ++v) hq += xb[v][4];
    }
  }
#pragma unroll
  for (int f = 0; f < 4; ++f)
    if (own && gl > 0) AC(0, f) += from_above[f];
  if (own) {
#pragma unroll
    for (int t = 0; t < CHT; ++t) {
      if (t < n) {
        const int m = lo + t;
        rec[3 + m] = fw * AC(t, 0);
        rec[3 + NR + m] = fw * AC(t, 1);
        rec[3 + 2 * NR + m] = fd * AC(t, 2);
        rec[3 + 3 * NR + m] = fac * AC(t, 3);
      }
    }
    if (hi == NL) {  // the backing medium N + 1
      rec[3 + NL] = fw * bnd[0];
      rec[3 + NR + NL] = fw * bnd[1];
      rec[3 + 2 * NR + NL] = fd * bnd[2];
      rec[3 + 3 * NR + NL] = fac * bnd[3];
    }
  }
  if (gl == 0) {
    rec[0] = ll;
    rec[1] = ghat * Rsm;
    rec[2] = ghat;
    if (RES) rec[3 + 4 * NR] = fac * hq;
  }
}

// The configuration of a launch whose deepest item needs ch64 levels per
// lane at 64 lanes: one wave per data point up to 8 levels per lane, else two
// or four waves, so that no lane holds more than 8 levels (the tape then fits
// 2 KB of LDS per level and wave, and the kernel two waves per SIMD); the
// levels per lane round up to a power of two.
static int scan_nw(int ch64) { return ch64 <= 8 ? 1 : ch64 <= 16 ? 2 : 4; }

static int scan_cht(int ch64) {
  const int nw = scan_nw(ch64);
  const int ch = (ch64 + nw - 1) / nw;
  int c = 1;
  while (c < ch) c <<= 1;
  return c;
}

size_t scan_lds_bytes(int ch_max) {
  const int c = scan_cht(ch_max), nt = 64 * scan_nw(ch_max);
  size_t b = sizeof(Shared) + (sizeof(cd) * 4 + sizeof(double) * 5) * (nt / 64);
  if (c >= 8) b += sizeof(double) * (size_t)c * 4 * nt;
  return b;
}

hipError_t prepare_grad_scan(int ch_max) {
  // static LDS only; every depth up to kMaxDeepLayers has an instance
  return (ch_max >= 1 && ch_max <= kScanMaxChunk) ? hipSuccess : hipErrorInvalidValue;
}

template <int CHT, int NW>
static void launch_scan_cht(bool res, const KernelArgs& a, int n_wu, hipStream_t st) {
  if (res)
    hipLaunchKernelGGL((k_loglik_grad_scan<CHT, NW, true>), dim3(n_wu), dim3(64 * NW), 0, st, a);
  else
    hipLaunchKernelGGL((k_loglik_grad_scan<CHT, NW, false>), dim3(n_wu), dim3(64 * NW), 0, st,
                       a);
}

hipError_t launch_grad_scan(bool res, int ch_max, const KernelArgs& a, int n_wu, hipStream_t st) {
  if (n_wu <= 0) return hipSuccess;
  if (ch_max < 1 || ch_max > kScanMaxChunk) return hipErrorInvalidValue;
  switch (scan_nw(ch_max) * 100 + scan_cht(ch_max)) {
    case 101: launch_scan_cht<1, 1>(res, a, n_wu, st); break;
    case 102: launch_scan_cht<2, 1>(res, a, n_wu, st); break;
    case 104: launch_scan_cht<4, 1>(res, a, n_wu, st); break;
    case 108: launch_scan_cht<8, 1>(res, a, n_wu, st); break;
    case 208: launch_scan_cht<8, 2>(res, a, n_wu, st); break;
    case 408: launch_scan_cht<8, 4>(res, a, n_wu, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nr
