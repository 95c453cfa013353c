// ===========================================================================
//  Plain FP64 CPU oracle for the specular neutron-reflectivity log-likelihood
//  and its gradient (arXiv 2509.06924).
//
//  TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
//  call this file: only the test suite, the smoke check and the benchmark's
//  CPU-baseline leg use it.  It shares no code, header, table or constant
//  generator with the HIP library.
//
//  What it computes, and where the paper defines it:
//   * Forward model R(Q, theta) by the Abeles transfer-matrix formalism with
//     slab parameters theta_slab = {thickness, SLD, roughness} and instrument
//     parameters theta_NR = {scale, background}       (Sec. 2.1; Sec. 3 API).
//   * Gaussian interfacial roughness applied per interface, read as the
//     Nevot-Croce factor                    (Sec. 3 dict "rough"; SI Sec. S2).
//   * Constant dQ/Q Gaussian resolution smearing    (Sec. 3 smearing kernels;
//     Sec. 4.1 FWHM smearing), read as a 17-point Gauss-Legendre rule over
//     +-3.5 sigma_Q with normalised Gaussian weights.
//   * R_hat = scale * R_smeared + bkg      (Sec. 2.1 theta_NR; Tables 1-3).
//   * Gaussian log-likelihood with the measured per-point errors
//     (Sec. 2.1 Gaussian approximation of p(R|theta); Sec. 4.1 chi^2 eq.).
//   * Its exact gradient (Sec. 2.1 AD figure; Sec. 3 jax.grad listing) by
//     complex step in a second imaginary unit (bicomplex numbers), with a
//     4th-order Richardson central difference as an independent cross-check.
//   * Two independent re-derivations used only to pin the Abeles product:
//     the Parratt recursion in the physical (Im k >= 0) frame, and for
//     sigma = 0 the direct boundary-matching linear system.
//
//  Conventions (readings where the paper is silent; each one is listed with
//  its reason in the design notes):
//   - kz0 = Q/2 in the fronting medium; kz_j^2 = kz0^2 - 4 pi (rho_j - rho_0)
//     with absorption entering as -i 4 pi |rho_im,j|; the fronting medium's
//     imaginary SLD is ignored (kz0 real).
//   - kz_j is the square root with Re >= 0 and Im <= 0; the layer phase is
//     E_j = exp(i kz_j d_j).  This is the complex conjugate of the physical
//     Im >= 0 frame and gives the same R.
//   - r_j = (kz_j - kz_{j+1}) / (kz_j + kz_{j+1}), r_j = 0 when the two
//     wavevectors are equal (identical media, avoids 0/0 at kz = 0).
//   - Nevot-Croce: r'_j = r_j exp(-2 kz_j kz_{j+1} sigma_{j+1}^2), with
//     sigma taken from the row of the medium BELOW the interface.
//   - M = C_0 C_1 ... C_N, C_j = [[E_j, r'_j E_j], [r'_j/E_j, 1/E_j]],
//     E_0 = 1; r = M10 / M00; R = |r|^2.
//   - Smear, then scale, then add background.
//   - logL = sum_i [ -1/2 ((R_hat_i - R_i)/e_i)^2 - ln e_i - 1/2 ln 2 pi ].
//
//  Row layout for a stack of L finite layers: rows 0..L+1, four doubles each,
//  [d, rho_re, rho_im, sigma]; row 0 = fronting (only rho_re used), rows 1..L
//  = layers, row L+1 = backing (d unused).  sigma of row j is the roughness of
//  the interface above medium j.  Units: Angstrom, Angstrom^-2 (absolute).
//
//  Pins (tests that run this oracle against facts other than itself):
//   Abeles forward ......... single-interface Fresnel/NC closed form; R = 1
//                            below the backing edge; thick-absorber limit
//                            (branch); Parratt (independent recursion, other
//                            frame); sigma = 0 boundary-matching solve; split
//                            layer and zero-thickness insert invariances;
//                            thickness periodicity and Kiessig period;
//                            reciprocity; 50-digit Parratt (mpmath).
//   smearing rule .......... Gauss-Legendre exactness to degree 33, nodes vs
//                            numpy's leggauss, symmetric moments, sum w = 1,
//                            dQ/Q -> 0 limit.
//   instrument / logL ...... perfect-fit closed form; d/dbkg, d/dscale closed
//                            forms; chi^2 relation.
//   gradient ............... Richardson FD; single-interface closed forms;
//                            translation invariance in rho_re; split-layer
//                            identities; periodicity in d.
//   VJP of R_hat ........... the likelihood seed reproduces the logL
//                            gradient; a one-hot seed equals Richardson
//                            differences of the model curve and the
//                            weighted node Jacobian; linear in the seed.
//   batched entry .......... equal, bitwise, to the per-item calls.
//  Every function below is pinned; none is "parity unpinned".
//
//  Build: g++ -O2 -std=c++17 -ffp-contract=off -fopenmp -shared -fPIC
// ===========================================================================

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace orc {

using cplx = std::complex<double>;

// Nearest doubles to 4*pi, ln(2*pi)/2 and the FWHM-to-sigma factor 2 sqrt(2 ln 2).
static const double FOURPI = 12.566370614359172;
static const double HALF_LN_2PI = 0.91893853320467274;
static const double FWHM_PER_SIGMA = 2.3548200450309493;
// Half-width of the smearing window, in units of sigma_Q.
static const double SMEAR_HALF_WIDTH = 3.5;
static const int NGL = 17;

// ---------------------------------------------------------------------------
// Bicomplex numbers z = a + b*J with a, b complex in the ordinary unit I and a
// second, commuting imaginary unit J (J^2 = -1, IJ = JI).  A real parameter p
// is perturbed as p + h*J; for any function built from the operations below
// the J-part of the result divided by h is dF/dp (complex-step derivative).
// Every operation is the exact bicomplex algebra, so no subtraction of nearly
// equal numbers happens and h can be 1e-20.
// ---------------------------------------------------------------------------
struct BC {
  cplx a, b;
  BC() : a(0.0), b(0.0) {}
  BC(double x) : a(x), b(0.0) {}
  BC(cplx x) : a(x), b(0.0) {}
  BC(cplx x, cplx y) : a(x), b(y) {}
};
static inline BC operator+(BC x, BC y) { return BC(x.a + y.a, x.b + y.b); }
static inline BC operator-(BC x, BC y) { return BC(x.a - y.a, x.b - y.b); }
static inline BC operator-(BC x) { return BC(-x.a, -x.b); }
static inline BC operator*(BC x, BC y) {
  return BC(x.a * y.a - x.b * y.b, x.a * y.b + x.b * y.a);
}
static inline BC operator*(double s, BC x) { return BC(s * x.a, s * x.b); }
static inline BC operator*(BC x, double s) { return BC(s * x.a, s * x.b); }
static inline BC operator/(BC x, BC y) {
  // (a + bJ)/(c + dJ) = (a + bJ)(c - dJ)/(c^2 + d^2)
  cplx den = y.a * y.a + y.b * y.b;
  return BC((x.a * y.a + x.b * y.b) / den, (x.b * y.a - x.a * y.b) / den);
}
static inline BC operator/(BC x, double s) { return BC(x.a / s, x.b / s); }
static inline bool operator==(BC x, BC y) { return x.a == y.a && x.b == y.b; }

// Multiplication by the ordinary imaginary unit I.
static inline cplx mul_i(cplx z) { return cplx(-z.imag(), z.real()); }
static inline BC mul_i(BC z) { return BC(mul_i(z.a), mul_i(z.b)); }

// x + I*y from two I-real values, built component-wise so that a zero y keeps
// its sign (w = x - 0i must stay below the branch cut).
static inline cplx make_xy(cplx x, cplx y) { return cplx(x.real(), y.real()); }
static inline BC make_xy(BC x, BC y) {
  return BC(cplx(x.a.real(), y.a.real()), cplx(x.b.real(), y.b.real()));
}

// Complex conjugation in I only (J-linear, so allowed inside complex step).
static inline cplx conj_i(cplx z) { return std::conj(z); }
static inline BC conj_i(BC z) { return BC(std::conj(z.a), std::conj(z.b)); }

// exp: exp(a + bJ) = exp(a) (cos b + J sin b).
static inline cplx exp_z(cplx z) { return std::exp(z); }
static inline BC exp_z(BC z) {
  cplx ea = std::exp(z.a);
  return BC(ea * std::cos(z.b), ea * std::sin(z.b));
}

// The wavevector root: the square root of w with Re >= 0 and Im <= 0.
// Callers build w with Im w <= 0 (a signed zero -0.0 when there is no
// absorption), and for such w the principal branch of the library square
// root is exactly this root (C99 csqrt keeps the sign of a zero imaginary
// part, so sqrt(x - 0i) = -i sqrt(|x|) for x < 0).
static inline cplx kz_root(cplx w) { return std::sqrt(w); }
// Bicomplex square root on the same branch: (c + dJ)^2 = a + bJ with
// c^2 = a (1 + sqrt(1 + (b/a)^2)) / 2 and d = b / (2c).
static inline BC kz_root(BC w) {
  if (w.a == cplx(0.0, 0.0)) return BC(cplx(0.0, 0.0), std::sqrt(w.b));
  cplx ratio = w.b / w.a;
  cplx c2 = w.a * (1.0 + std::sqrt(1.0 + ratio * ratio)) * 0.5;
  // keep c2's imaginary part on the same side of the cut as w.a
  if (c2.imag() == 0.0) c2 = cplx(c2.real(), std::copysign(0.0, w.a.imag()));
  cplx c = std::sqrt(c2);
  return BC(c, w.b / (2.0 * c));
}

// |x| for a lifted real parameter x (sign taken from its real part; the
// derivative at x = 0 is the one-sided +1).
static inline cplx abs_real(cplx x) { return x.real() < 0.0 ? -x : x; }
static inline BC abs_real(BC x) { return x.a.real() < 0.0 ? -x : x; }

static inline double real_part(cplx x) { return x.real(); }
static inline double real_part(BC x) { return x.a.real(); }

// ---------------------------------------------------------------------------
// Smearing rule: 17-point Gauss-Legendre on [-1, 1] (Newton's method on
// P_17 in long double, then rounded), mapped to +-3.5 sigma_Q, with weights
// u_k exp(-(3.5 x_k)^2 / 2) normalised to sum 1.
// ---------------------------------------------------------------------------
static void legendre_and_derivative(int n, long double x, long double* p,
                                    long double* dp) {
  long double p0 = 1.0L, p1 = x;
  for (int k = 2; k <= n; ++k) {
    long double pk = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  *p = p1;
  *dp = n * (x * p1 - p0) / (x * x - 1.0L);
}

static void gauss_legendre(int n, double* x, double* u) {
  const long double PI_L = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    // i-th root from the top, then stored in ascending order
    long double xi = std::cos(PI_L * (i + 0.75L) / (n + 0.5L));
    long double p, dp;
    for (int it = 0; it < 100; ++it) {
      legendre_and_derivative(n, xi, &p, &dp);
      long double dx = p / dp;
      xi -= dx;
      if (std::fabs(dx) < 1e-30L) break;
    }
    legendre_and_derivative(n, xi, &p, &dp);
    long double wi = 2.0L / ((1.0L - xi * xi) * dp * dp);
    x[n - 1 - i] = (double)xi;
    u[n - 1 - i] = (double)wi;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;  // the middle root is exactly zero
}

struct SmearRule {
  int K;
  double t[NGL];  // node offsets in units of sigma_Q: 3.5 x_k
  double w[NGL];  // normalised weights
};

static SmearRule make_rule(double dq_over_q) {
  SmearRule s;
  if (dq_over_q == 0.0) {
    s.K = 1;
    s.t[0] = 0.0;
    s.w[0] = 1.0;
    return s;
  }
  double x[NGL], u[NGL];
  gauss_legendre(NGL, x, u);
  long double g[NGL], sum = 0.0L;
  for (int k = 0; k < NGL; ++k) {
    s.t[k] = SMEAR_HALF_WIDTH * x[k];
    long double tk = s.t[k];
    g[k] = (long double)u[k] * std::exp(-0.5L * tk * tk);
    sum += g[k];
  }
  for (int k = 0; k < NGL; ++k) s.w[k] = (double)(g[k] / sum);
  s.K = NGL;
  return s;
}

// Node k of point Q: q = Q + (dQ/Q * Q / (2 sqrt(2 ln 2))) * t_k, evaluated in
// exactly this order with no contraction.
static inline double node_q(double Q, double dq_over_q, double t) {
  double s = dq_over_q * Q;
  s = s / FWHM_PER_SIGMA;
  return Q + s * t;
}

// ---------------------------------------------------------------------------
// Abeles reflection amplitude at one momentum transfer q.  Z is cplx for the
// value, BC for complex-step derivatives; rows are lifted to Z.
// ---------------------------------------------------------------------------
// The product depends on q only through kz0^2 = q^2/4 (in every w_j) and the
// fronting wavevector kz0 = q/2; abeles_amplitude_k takes both (as Z, so that
// q itself can carry a complex-step perturbation).
template <class Z>
static Z abeles_amplitude_k(int L, const Z* rows, Z kz0sq, Z kz0) {
  const int N = L;
  std::vector<Z> kz(N + 2);
  kz[0] = kz0;
  const Z rho0 = rows[0 * 4 + 1];
  for (int j = 1; j <= N + 1; ++j) {
    const Z rho_re = rows[j * 4 + 1];
    const Z rho_im = abs_real(rows[j * 4 + 2]);
    // w = 0.25 q q - 4 pi (rho_re_j - rho_re_0) - i 4 pi |rho_im_j|
    Z re_part = kz0sq - FOURPI * (rho_re - rho0);
    Z im_part = -(FOURPI * rho_im);  // -0.0 when rho_im = 0
    kz[j] = kz_root(make_xy(re_part, im_part));
  }
  // 2x2 matrix product M = C_0 C_1 ... C_N, left to right.
  Z m00(1.0), m01(0.0), m10(0.0), m11(1.0);
  for (int j = 0; j <= N; ++j) {
    Z r;
    if (kz[j] == kz[j + 1])
      r = Z(0.0);
    else
      r = (kz[j] - kz[j + 1]) / (kz[j] + kz[j + 1]);
    const Z sig = rows[(j + 1) * 4 + 3];
    Z f = exp_z(-2.0 * (kz[j] * kz[j + 1] * (sig * sig)));
    Z rp = r * f;
    Z E(1.0), Einv(1.0);
    if (j >= 1) {
      const Z d = rows[j * 4 + 0];
      E = exp_z(mul_i(kz[j] * d));
      Einv = Z(1.0) / E;
    }
    Z c00 = E, c01 = rp * E, c10 = rp * Einv, c11 = Einv;
    Z n00 = m00 * c00 + m01 * c10;
    Z n01 = m00 * c01 + m01 * c11;
    Z n10 = m10 * c00 + m11 * c10;
    Z n11 = m10 * c01 + m11 * c11;
    m00 = n00;
    m01 = n01;
    m10 = n10;
    m11 = n11;
  }
  return m10 / m00;
}

template <class Z>
static Z abeles_amplitude(int L, const Z* rows, double q) {
  const double kz0sq = 0.25 * q * q;
  return abeles_amplitude_k(L, rows, Z(kz0sq), Z(cplx(0.5 * q, 0.0)));
}

template <class Z>
static Z reflectivity(int L, const Z* rows, double q) {
  Z r = abeles_amplitude(L, rows, q);
  return r * conj_i(r);
}

// R at a lifted momentum transfer (its J-part differentiates through q).
static BC reflectivity_bcq(int L, const BC* rows, BC q) {
  const BC kz0sq = (0.25 * q) * q;
  BC r = abeles_amplitude_k(L, rows, kz0sq, 0.5 * q);
  return r * conj_i(r);
}

// R_hat_i = scale * sum_k w_k R(q_ik) + bkg for every point of one dataset.
template <class Z>
static void model_curve(int L, const Z* rows, Z scale, Z bkg, int nq,
                        const double* Q, double dq_over_q, Z* Rhat) {
  SmearRule rule = make_rule(dq_over_q);
  for (int i = 0; i < nq; ++i) {
    Z Rsm(0.0);
    for (int k = 0; k < rule.K; ++k) {
      double q = node_q(Q[i], dq_over_q, rule.t[k]);
      Rsm = Rsm + rule.w[k] * reflectivity(L, rows, q);
    }
    Rhat[i] = scale * Rsm + bkg;
  }
}

// Resolution given per point (Sec. 3 pointwise Gaussian smearing, Sec. 4.1
// FWHM estimates per point) or as a free relative width (Sec. 4.2: the
// smearing size is an unknown).  For a smeared dataset (dq_over_q > 0) the
// nodes of point i are Q_i + s_i t_k with s_i = dQ_i / (2 sqrt(2 ln 2)) when
// per-point FWHMs dQ are given, else s_i = (dq_over_q Q_i) / (2 sqrt(2 ln 2));
// the weights w_k are the same normalised Gaussian weights either way.
// dqq_j: dq_over_q carrying a J-perturbation (complex step on the width).
static void model_curve_res(int L, const BC* rows, BC scale, BC bkg, int nq, const double* Q,
                            double dq_over_q, const double* dQ, BC dqq_j, BC* Rhat) {
  SmearRule rule = make_rule(dq_over_q);
  for (int i = 0; i < nq; ++i) {
    BC Rsm(0.0);
    for (int k = 0; k < rule.K; ++k) {
      BC q;
      if (rule.K == 1) {
        q = BC(Q[i]);
      } else if (dQ) {
        const double s = dQ[i] / FWHM_PER_SIGMA;
        q = BC(Q[i] + s * rule.t[k]);
      } else {
        BC s = dqq_j * Q[i];
        s = s / FWHM_PER_SIGMA;
        q = BC(Q[i]) + s * rule.t[k];
      }
      Rsm = Rsm + rule.w[k] * reflectivity_bcq(L, rows, q);
    }
    Rhat[i] = scale * Rsm + bkg;
  }
}

static BC loglik_res(int L, const BC* rows, BC scale, BC bkg, int nq, const double* Q,
                     const double* Robs, const double* Rerr, double dq_over_q, const double* dQ,
                     BC dqq_j) {
  std::vector<BC> Rhat(nq);
  model_curve_res(L, rows, scale, bkg, nq, Q, dq_over_q, dQ, dqq_j, Rhat.data());
  BC s(0.0);
  for (int i = 0; i < nq; ++i) {
    BC z = (Rhat[i] - BC(Robs[i])) / Rerr[i];
    s = s + (-0.5) * (z * z) - BC(std::log(Rerr[i]) + HALF_LN_2PI);
  }
  return s;
}

template <class Z>
static Z loglik(int L, const Z* rows, Z scale, Z bkg, int nq, const double* Q,
                const double* Robs, const double* Rerr, double dq_over_q) {
  std::vector<Z> Rhat(nq);
  model_curve(L, rows, scale, bkg, nq, Q, dq_over_q, Rhat.data());
  Z s(0.0);
  for (int i = 0; i < nq; ++i) {
    Z z = (Rhat[i] - Z(Robs[i])) / Rerr[i];
    s = s + (-0.5) * (z * z) - Z(std::log(Rerr[i]) + HALF_LN_2PI);
  }
  return s;
}

// Which row entries the model reads (the rest have gradient exactly 0).
static inline bool entry_used(int L, int row, int field) {
  if (row == 0) return field == 1;               // fronting: rho_re only
  if (row == L + 1) return field != 0;           // backing: no thickness
  return true;                                   // finite layers: all four
}

// Natural unit of each field, used for step sizes.
static inline double natural_unit(int field) {
  switch (field) {
    case 0: return 1.0;     // d, Angstrom
    case 1: return 1e-6;    // rho_re, Angstrom^-2
    case 2: return 1e-6;    // rho_im
    default: return 1.0;    // sigma, Angstrom
  }
}

// Complex-step gradient of F(rows, scale, bkg) with respect to every used row
// entry and the two instrument parameters.  F maps lifted parameters to a BC
// scalar whose J-part carries the derivative.
template <class F>
static void complex_step_grad(int L, const double* rows, double scale,
                              double bkg, F eval, double* g_rows,
                              double* g_inst) {
  const int nr = (L + 2) * 4;
  std::vector<BC> zr(nr);
  for (int p = 0; p < nr; ++p) zr[p] = BC(rows[p]);
  for (int p = 0; p < nr; ++p) {
    g_rows[p] = 0.0;
    if (!entry_used(L, p / 4, p % 4)) continue;
    double h = 1e-20 * std::fmax(natural_unit(p % 4), std::fabs(rows[p]));
    zr[p].b = cplx(h, 0.0);
    BC v = eval(zr.data(), BC(scale), BC(bkg));
    g_rows[p] = v.b.real() / h;
    zr[p].b = cplx(0.0, 0.0);
  }
  {
    double h = 1e-20 * std::fmax(1.0, std::fabs(scale));
    BC v = eval(zr.data(), BC(cplx(scale), cplx(h)), BC(bkg));
    g_inst[0] = v.b.real() / h;
  }
  {
    double h = 1e-20 * std::fmax(1e-7, std::fabs(bkg));
    BC v = eval(zr.data(), BC(scale), BC(cplx(bkg), cplx(h)));
    g_inst[1] = v.b.real() / h;
  }
}

// 4th-order central difference f'(p) ~ [8(f(p+h)-f(p-h)) - (f(p+2h)-f(p-2h))]/(12h).
template <class F>
static void richardson_grad(int L, const double* rows, double scale,
                            double bkg, F eval, double rel_step,
                            double* g_rows, double* g_inst) {
  const int nr = (L + 2) * 4;
  std::vector<double> p(rows, rows + nr);
  auto diff = [&](double* slot, double h, auto call) {
    double x0 = *slot;
    *slot = x0 + h;       double fp1 = call();
    *slot = x0 - h;       double fm1 = call();
    *slot = x0 + 2.0 * h; double fp2 = call();
    *slot = x0 - 2.0 * h; double fm2 = call();
    *slot = x0;
    return (8.0 * (fp1 - fm1) - (fp2 - fm2)) / (12.0 * h);
  };
  double sc = scale, bk = bkg;
  auto call = [&]() { return eval(p.data(), sc, bk); };
  for (int q = 0; q < nr; ++q) {
    g_rows[q] = 0.0;
    if (!entry_used(L, q / 4, q % 4)) continue;
    double h = rel_step * natural_unit(q % 4);
    g_rows[q] = diff(&p[q], h, call);
  }
  g_inst[0] = diff(&sc, rel_step, call);
  g_inst[1] = diff(&bk, rel_step * 1e-7, call);
}

// ---------------------------------------------------------------------------
// Independent Parratt recursion in the physical frame: k_j is the principal
// square root of conj(w_j) (Im k >= 0), amplitude ratios are propagated from
// the bottom interface upward with the phase exp(2 i k d) of the layer between
// two interfaces.  Used only as a pin for the Abeles product.
// ---------------------------------------------------------------------------
static double parratt_R(int L, const double* rows, double q) {
  const int N = L;
  std::vector<cplx> k(N + 2);
  k[0] = cplx(0.5 * q, 0.0);
  for (int j = 1; j <= N + 1; ++j) {
    double x = 0.25 * q * q - FOURPI * (rows[j * 4 + 1] - rows[1]);
    double y = FOURPI * std::fabs(rows[j * 4 + 2]);  // +0.0 when no absorption
    k[j] = std::sqrt(cplx(x, y));
  }
  auto interface_coeff = [&](int j) {
    cplx rf = (k[j] == k[j + 1]) ? cplx(0.0)
                                 : (k[j] - k[j + 1]) / (k[j] + k[j + 1]);
    double s = rows[(j + 1) * 4 + 3];
    return rf * std::exp(-2.0 * k[j] * k[j + 1] * s * s);
  };
  cplx X = interface_coeff(N);
  for (int j = N - 1; j >= 0; --j) {
    cplx ph = std::exp(cplx(0.0, 2.0) * k[j + 1] * rows[(j + 1) * 4 + 0]);
    cplx Y = X * ph;
    cplx rr = interface_coeff(j);
    X = (rr + Y) / (1.0 + rr * Y);
  }
  return std::norm(X);
}

// ---------------------------------------------------------------------------
// sigma = 0 brute force: psi_j(z) = A_j e^{i k_j (z - z_j)} + B_j e^{-i k_j (z - z_j)}
// in each medium (z_j = top of medium j, z_0 = 0 for the fronting), A_0 = 1
// incident, B_{N+1} = 0 (nothing returns from the backing); continuity of psi
// and psi' at every interface; solved by Gaussian elimination with partial
// pivoting.  r = B_0.  Physical frame (principal root, Im k >= 0).
// ---------------------------------------------------------------------------
static double linsys_R(int L, const double* rows, double q) {
  const int N = L;
  std::vector<cplx> k(N + 2);
  k[0] = cplx(0.5 * q, 0.0);
  for (int j = 1; j <= N + 1; ++j) {
    double x = 0.25 * q * q - FOURPI * (rows[j * 4 + 1] - rows[1]);
    double y = FOURPI * std::fabs(rows[j * 4 + 2]);
    k[j] = std::sqrt(cplx(x, y));
  }
  // unknowns: u0 = B_0, then (A_j, B_j) for j = 1..N, then A_{N+1}
  const int n = 2 * N + 2;
  auto idxA = [&](int j) { return (j == N + 1) ? n - 1 : 2 * j - 1; };
  auto idxB = [&](int j) { return (j == 0) ? 0 : 2 * j; };
  std::vector<cplx> M(n * n, cplx(0.0)), rhs(n, cplx(0.0));
  const cplx I(0.0, 1.0);
  for (int j = 0; j <= N; ++j) {
    // interface between medium j (above) and j+1 (below)
    int e0 = 2 * j, e1 = 2 * j + 1;
    // medium j evaluated at its bottom: phase offset = d_j (0 for fronting, z=0)
    cplx pA = 1.0, pB = 1.0;
    if (j >= 1) {
      double d = rows[j * 4 + 0];
      pA = std::exp(I * k[j] * d);
      pB = std::exp(-I * k[j] * d);
    }
    // psi continuity: A_j pA + B_j pB - A_{j+1} - B_{j+1} = 0
    // psi' continuity: k_j (A_j pA - B_j pB) - k_{j+1} (A_{j+1} - B_{j+1}) = 0
    if (j == 0) {
      rhs[e0] -= pA;            // A_0 = 1 moved to the right-hand side
      rhs[e1] -= k[0] * pA;
    } else {
      M[e0 * n + idxA(j)] += pA;
      M[e1 * n + idxA(j)] += k[j] * pA;
    }
    M[e0 * n + idxB(j)] += pB;
    M[e1 * n + idxB(j)] += -k[j] * pB;
    M[e0 * n + idxA(j + 1)] += -1.0;
    M[e1 * n + idxA(j + 1)] += -k[j + 1];
    if (j + 1 <= N) {
      M[e0 * n + idxB(j + 1)] += -1.0;
      M[e1 * n + idxB(j + 1)] += k[j + 1];
    }
  }
  // Gaussian elimination with partial pivoting
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::abs(M[r * n + c]) > std::abs(M[piv * n + c])) piv = r;
    if (piv != c) {
      for (int t = 0; t < n; ++t) std::swap(M[c * n + t], M[piv * n + t]);
      std::swap(rhs[c], rhs[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      cplx f = M[r * n + c] / M[c * n + c];
      if (f == cplx(0.0)) continue;
      for (int t = c; t < n; ++t) M[r * n + t] -= f * M[c * n + t];
      rhs[r] -= f * rhs[c];
    }
  }
  std::vector<cplx> x(n);
  for (int r = n - 1; r >= 0; --r) {
    cplx s = rhs[r];
    for (int t = r + 1; t < n; ++t) s -= M[r * n + t] * x[t];
    x[r] = s / M[r * n + r];
  }
  return std::norm(x[0]);
}

}  // namespace orc

// ===========================================================================
// C entry points (called from Python through ctypes by the tests).
// Return 0 on success, -1 on invalid arguments.
// ===========================================================================
using namespace orc;

extern "C" {

int orc_version(void) { return 1; }

// 17-point Gauss-Legendre nodes x[17] and weights u[17] on [-1, 1].
int orc_gauss_legendre17(double* x, double* u) {
  gauss_legendre(NGL, x, u);
  return 0;
}

// Smearing rule for a given dQ/Q: returns K (1 or 17), fills t[K] (offsets in
// sigma_Q units) and w[K] (normalised weights).
int orc_smear_rule(double dq_over_q, double* t, double* w) {
  if (!(dq_over_q >= 0.0)) return -1;
  SmearRule s = make_rule(dq_over_q);
  for (int k = 0; k < s.K; ++k) {
    t[k] = s.t[k];
    w[k] = s.w[k];
  }
  return s.K;
}

// Node positions for every point: q_nodes[i*K + k].
int orc_smear_nodes(int nq, const double* Q, double dq_over_q, double* q_nodes) {
  if (nq < 0 || !(dq_over_q >= 0.0)) return -1;
  SmearRule s = make_rule(dq_over_q);
  for (int i = 0; i < nq; ++i)
    for (int k = 0; k < s.K; ++k) q_nodes[i * s.K + k] = node_q(Q[i], dq_over_q, s.t[k]);
  return s.K;
}

// Wavevector root for w = x + i y (y <= 0): out = [Re kz, Im kz].
int orc_kz(double x, double y, double* out) {
  cplx k = kz_root(cplx(x, y));
  out[0] = k.real();
  out[1] = k.imag();
  return 0;
}

// Unsmeared Abeles R at nq momentum transfers.
int orc_reflectivity(int L, const double* rows, int nq, const double* q, double* R) {
  if (L < 0 || nq < 0) return -1;
  std::vector<cplx> zr(rows, rows + (L + 2) * 4);
  for (int i = 0; i < nq; ++i) R[i] = reflectivity(L, zr.data(), q[i]).real();
  return 0;
}

int orc_reflectivity_parratt(int L, const double* rows, int nq, const double* q, double* R) {
  if (L < 0 || nq < 0) return -1;
  for (int i = 0; i < nq; ++i) R[i] = parratt_R(L, rows, q[i]);
  return 0;
}

int orc_reflectivity_linsys(int L, const double* rows, int nq, const double* q, double* R) {
  if (L < 0 || nq < 0) return -1;
  for (int i = 0; i < nq; ++i) R[i] = linsys_R(L, rows, q[i]);
  return 0;
}

// R_hat (smeared, scaled, background added) at the nq data points.
int orc_model_curve(int L, const double* rows, double scale, double bkg, int nq,
                    const double* Q, double dq_over_q, double* Rhat) {
  if (L < 0 || nq < 0 || !(dq_over_q >= 0.0)) return -1;
  std::vector<cplx> zr(rows, rows + (L + 2) * 4), out(nq);
  model_curve(L, zr.data(), cplx(scale), cplx(bkg), nq, Q, dq_over_q, out.data());
  for (int i = 0; i < nq; ++i) Rhat[i] = out[i].real();
  return 0;
}

// Smeared R before the instrument (R_sm), for tests of the instrument step.
int orc_smeared(int L, const double* rows, int nq, const double* Q,
                double dq_over_q, double* Rsm) {
  return orc_model_curve(L, rows, 1.0, 0.0, nq, Q, dq_over_q, Rsm);
}

double orc_loglik(int L, const double* rows, double scale, double bkg, int nq,
                  const double* Q, const double* Robs, const double* Rerr,
                  double dq_over_q) {
  std::vector<cplx> zr(rows, rows + (L + 2) * 4);
  return loglik(L, zr.data(), cplx(scale), cplx(bkg), nq, Q, Robs, Rerr, dq_over_q).real();
}

// logL and its complex-step gradient: g_rows[(L+2)*4] (unused entries 0),
// g_inst[2] = {d/dscale, d/dbkg}.
int orc_loglik_grad_cs(int L, const double* rows, double scale, double bkg, int nq,
                       const double* Q, const double* Robs, const double* Rerr,
                       double dq_over_q, double* logL, double* g_rows, double* g_inst) {
  if (L < 0 || nq < 0 || !(dq_over_q >= 0.0)) return -1;
  *logL = orc_loglik(L, rows, scale, bkg, nq, Q, Robs, Rerr, dq_over_q);
  auto eval = [&](const BC* zr, BC sc, BC bk) {
    return loglik(L, zr, sc, bk, nq, Q, Robs, Rerr, dq_over_q);
  };
  complex_step_grad(L, rows, scale, bkg, eval, g_rows, g_inst);
  return 0;
}

// Richardson finite-difference gradient of logL (rel_step in natural units).
int orc_loglik_grad_fd(int L, const double* rows, double scale, double bkg, int nq,
                       const double* Q, const double* Robs, const double* Rerr,
                       double dq_over_q, double rel_step, double* g_rows,
                       double* g_inst) {
  if (L < 0 || nq < 0 || !(dq_over_q >= 0.0)) return -1;
  auto eval = [&](const double* p, double sc, double bk) {
    return orc_loglik(L, p, sc, bk, nq, Q, Robs, Rerr, dq_over_q);
  };
  richardson_grad(L, rows, scale, bkg, eval, rel_step, g_rows, g_inst);
  return 0;
}

// Vector-Jacobian product of R_hat: the gradient of sum_i seed_i R_hat_i.
int orc_model_vjp_cs(int L, const double* rows, double scale, double bkg, int nq,
                     const double* Q, double dq_over_q, const double* seed,
                     double* g_rows, double* g_inst) {
  if (L < 0 || nq < 0 || !(dq_over_q >= 0.0)) return -1;
  auto eval = [&](const BC* zr, BC sc, BC bk) {
    std::vector<BC> out(nq);
    model_curve(L, zr, sc, bk, nq, Q, dq_over_q, out.data());
    BC s(0.0);
    for (int i = 0; i < nq; ++i) s = s + seed[i] * out[i];
    return s;
  };
  complex_step_grad(L, rows, scale, bkg, eval, g_rows, g_inst);
  return 0;
}

// Complex-step derivative of the unsmeared R(q) at every point with respect
// to every used row entry: dR[i * (L+2)*4 + p].
int orc_reflectivity_jac_cs(int L, const double* rows, int nq, const double* q,
                            double* dR) {
  if (L < 0 || nq < 0) return -1;
  const int np = (L + 2) * 4;
  for (int i = 0; i < nq; ++i) {
    double gi[2];
    double qi = q[i];
    auto eval = [&](const BC* zr, BC, BC) { return reflectivity(L, zr, qi); };
    complex_step_grad(L, rows, 1.0, 0.0, eval, dR + (size_t)i * np, gi);
  }
  return 0;
}

// Batched logL and gradient over items that each name their dataset; used by
// the CPU baseline and by parity tests.  Items are independent; nthreads > 1
// runs them concurrently with OpenMP (one item per thread).
//   q_off[n_datasets+1], Q/Robs/Rerr packed per dataset, dq_over_q[n_datasets]
//   row_off[n_items+1] (in rows), layers[row_off[n]*4], scale/bkg[n_items]
int orc_loglik_grad_batch(int n_datasets, const int64_t* q_off, const double* Q,
                          const double* Robs, const double* Rerr,
                          const double* dq_over_q, int n_items,
                          const int32_t* dataset_of_item, const int64_t* row_off,
                          const double* layers, const double* scale,
                          const double* bkg, int want_grad, int nthreads,
                          double* logL, double* g_rows, double* g_inst) {
  if (n_datasets < 0 || n_items < 0) return -1;
  int bad = 0;
#ifdef _OPENMP
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(| : bad)
#endif
  for (int b = 0; b < n_items; ++b) {
    int ds = dataset_of_item[b];
    if (ds < 0 || ds >= n_datasets) { bad |= 1; continue; }
    int L = (int)(row_off[b + 1] - row_off[b]) - 2;
    if (L < 0) { bad |= 1; continue; }
    const double* rows = layers + row_off[b] * 4;
    int64_t q0 = q_off[ds];
    int nq = (int)(q_off[ds + 1] - q0);
    if (want_grad)
      orc_loglik_grad_cs(L, rows, scale[b], bkg[b], nq, Q + q0, Robs + q0, Rerr + q0,
                         dq_over_q[ds], &logL[b], g_rows + row_off[b] * 4, g_inst + 2 * b);
    else
      logL[b] = orc_loglik(L, rows, scale[b], bkg[b], nq, Q + q0, Robs + q0, Rerr + q0,
                           dq_over_q[ds]);
  }
  return bad ? -1 : 0;
}

// --- resolution: pointwise widths and the derivative w.r.t. dQ/Q ---------

// dR/dq (complex step through q) of the unsmeared R at nq momentum transfers.
int orc_reflectivity_dq_cs(int L, const double* rows, int nq, const double* q, double* dRdq) {
  if (L < 0 || nq < 0) return -1;
  std::vector<BC> zr(rows, rows + (L + 2) * 4);
  for (int i = 0; i < nq; ++i) {
    const double h = 1e-20 * std::fmax(1.0, std::fabs(q[i]));
    BC v = reflectivity_bcq(L, zr.data(), BC(cplx(q[i]), cplx(h)));
    dRdq[i] = v.b.real() / h;
  }
  return 0;
}

// R_hat with per-point FWHMs dQ (NULL: dq_over_q * Q) on a smeared dataset.
int orc_model_curve_res(int L, const double* rows, double scale, double bkg, int nq,
                        const double* Q, double dq_over_q, const double* dQ, double* Rhat) {
  if (L < 0 || nq < 0 || !(dq_over_q >= 0.0)) return -1;
  std::vector<BC> zr(rows, rows + (L + 2) * 4), out(nq);
  model_curve_res(L, zr.data(), BC(scale), BC(bkg), nq, Q, dq_over_q, dQ, BC(dq_over_q),
                  out.data());
  for (int i = 0; i < nq; ++i) Rhat[i] = out[i].a.real();
  return 0;
}

// logL and its complex-step gradient with the resolution as data (dQ) or as a
// parameter: g_res = dlogL/d(dQ/Q) (0 when dQ is given or the dataset is
// unsmeared).
int orc_loglik_grad_res_cs(int L, const double* rows, double scale, double bkg, int nq,
                           const double* Q, const double* Robs, const double* Rerr,
                           double dq_over_q, const double* dQ, double* logL, double* g_rows,
                           double* g_inst, double* g_res) {
  if (L < 0 || nq < 0 || !(dq_over_q >= 0.0)) return -1;
  std::vector<BC> zr0(rows, rows + (L + 2) * 4);
  *logL = loglik_res(L, zr0.data(), BC(scale), BC(bkg), nq, Q, Robs, Rerr, dq_over_q, dQ,
                     BC(dq_over_q)).a.real();
  auto eval = [&](const BC* zr, BC sc, BC bk) {
    return loglik_res(L, zr, sc, bk, nq, Q, Robs, Rerr, dq_over_q, dQ, BC(dq_over_q));
  };
  complex_step_grad(L, rows, scale, bkg, eval, g_rows, g_inst);
  *g_res = 0.0;
  if (dq_over_q > 0.0 && !dQ) {
    const double h = 1e-20 * std::fmax(1e-2, dq_over_q);
    BC v = loglik_res(L, zr0.data(), BC(scale), BC(bkg), nq, Q, Robs, Rerr, dq_over_q, nullptr,
                      BC(cplx(dq_over_q), cplx(h)));
    *g_res = v.b.real() / h;
  }
  return 0;
}

// Richardson difference of logL in dQ/Q (step rel_step * dQ/Q).
int orc_loglik_res_fd(int L, const double* rows, double scale, double bkg, int nq,
                      const double* Q, const double* Robs, const double* Rerr,
                      double dq_over_q, double rel_step, double* g_res) {
  if (L < 0 || nq < 0 || !(dq_over_q > 0.0)) return -1;
  std::vector<BC> zr(rows, rows + (L + 2) * 4);
  auto f = [&](double d) {
    return loglik_res(L, zr.data(), BC(scale), BC(bkg), nq, Q, Robs, Rerr, d, nullptr, BC(d))
        .a.real();
  };
  const double h = rel_step * dq_over_q;
  *g_res = (8.0 * (f(dq_over_q + h) - f(dq_over_q - h)) -
            (f(dq_over_q + 2.0 * h) - f(dq_over_q - 2.0 * h))) / (12.0 * h);
  return 0;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
