// Device-side complex arithmetic and the special functions of the layer
// product, for gfx950: the FP64 path and the FP32 variant.
#pragma once

#include <hip/hip_runtime.h>

namespace nr {

// 4 pi, ln(2 pi)/2 and 2 sqrt(2 ln 2) (FWHM of a unit Gaussian), as doubles.
constexpr double kFourPi = 12.566370614359172;
constexpr double kHalfLn2Pi = 0.91893853320467274;
constexpr double kFwhmPerSigma = 2.3548200450309493;

// Complex numbers of either precision (the FP64 path uses cd, the FP32
// variant's layer product cf).  Mixed-precision expressions do not compile,
// so a float computation cannot silently widen to double.
template <class T>
struct cx {
  T re, im;
};
using cd = cx<double>;
using cf = cx<float>;

template <class T>
__device__ __forceinline__ cx<T> mk(T a, T b) {
  cx<T> z;
  z.re = a;
  z.im = b;
  return z;
}
template <class T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <class T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <class T>
__device__ __forceinline__ cx<T> operator-(cx<T> a) { return mk(-a.re, -a.im); }
template <class T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return mk(s * a.re, s * a.im); }
template <class T>
__device__ __forceinline__ cx<T>& operator+=(cx<T>& a, cx<T> b) {
  a.re += b.re;
  a.im += b.im;
  return a;
}
template <class T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return mk(a.re, -a.im); }
// conj(a) * b
template <class T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
// conj(a) b + c and a b + c as four FMAs each.
template <class T>
__device__ __forceinline__ cx<T> cmulc_add(cx<T> a, cx<T> b, cx<T> c) {
  return mk(fma(a.re, b.re, fma(a.im, b.im, c.re)), fma(a.re, b.im, fma(-a.im, b.re, c.im)));
}
template <class T>
__device__ __forceinline__ cx<T> cmul_add(cx<T> a, cx<T> b, cx<T> c) {
  return mk(fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im)));
}
template <class T>
__device__ __forceinline__ T cabs2(cx<T> a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ cd widen(cd a) { return a; }
__device__ __forceinline__ cd widen(cf a) { return mk((double)a.re, (double)a.im); }

// 1/x from the hardware estimate v_rcp_f64 (relative error about 2^-24,
// measured on gfx950) refined by one Newton step r <- r + r (1 - x r), which
// squares the error: about 2^-48 relative.
__device__ __forceinline__ double rcp(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ cd crecip(cd z) {
  const double inv = rcp(z.re * z.re + z.im * z.im);
  return mk(z.re * inv, -z.im * inv);
}

// 1/sqrt(a) from the hardware estimate v_rsq_f64 (about 2^-24 relative)
// refined by one Newton step y <- y + y/2 (1 - a y^2): about 2^-47 relative.
__device__ __forceinline__ double rsq(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  const double e = fma(-(a * y), y, 1.0);
  return fma(0.5 * y, e, y);
}

// ---------------------------------------------------------------------------
// Table-driven exp and sincos.  The tables live in LDS, filled per block from
// plan-owned device memory computed on the host in long double:
//   sc[k] = (sin(k pi/64), cos(k pi/64)), k = 0..127
//   e2[j] = 2^(j/64),                     j = 0..63
// ---------------------------------------------------------------------------
struct MathTables {
  double sc[128][2];
  double e2[64];
};
constexpr int kTableDoubles = 128 * 2 + 64;

typedef __attribute__((address_space(3))) const double lds_double;

// Round-to-nearest integer of a double by the 1.5 * 2^52 shift: for
// |v| < 2^51, t = v + kShift holds round(v) in its low mantissa bits, so
// t - kShift is round(v) as a double and the low word of t is round(v)
// modulo 2^32 (two's complement).
constexpr double kShift = 6755399441055744.0;
__device__ __forceinline__ int low_word(double t) {
  return (int)(unsigned int)__double_as_longlong(t);
}

// sin and cos of x: x = k pi/64 + r with pi/64 split in two doubles (FMA
// Cody-Waite; the dropped third part, 4.7e-35, times k is far below the
// rounding of r for |x| < 1e12), |r| <= pi/128; Taylor polynomials of sin r
// to r^7 and cos r to r^6 (truncation below 1e-20 and 3.3e-18 on
// |r| <= pi/128), then the angle-addition formulas with the tabulated sin and
// cos of (k mod 128) pi/64.
// The table-driven functions come in two halves so that a caller can issue
// the LDS reads of one level well before it needs the values: *_issue forms
// the reduced argument, its polynomial and the table reads, *_finish combines
// them.  sincos_tab, exp_tab and cexp_tab are the two halves back to back.
struct SinCosPart {
  double sr, cr;  // sin r, cos r
  double sa, ca;  // tabulated sin, cos of (k mod 128) pi/64
};
__device__ __forceinline__ SinCosPart sincos_issue(const MathTables& T, double x) {
  constexpr double k64OverPi = 20.371832715762604;
  constexpr double kP1 = 0.04908738521234052;
  constexpr double kP2 = 1.9135106236677394e-18;
  const double t = fma(x, k64OverPi, kShift);
  const double k = t - kShift;
  double r = fma(-k, kP1, x);
  r = fma(-k, kP2, r);
  const int idx = low_word(t) & 127;
  const lds_double* row = (const lds_double*)(&T.sc[idx][0]);
  SinCosPart o;
  o.sa = row[0];
  o.ca = row[1];
  const double r2 = r * r;
  double ps = -0.0001984126984126984;          // -1/7!
  ps = fma(ps, r2, 0.008333333333333333);      //  1/5!
  ps = fma(ps, r2, -0.16666666666666666);      // -1/3!
  o.sr = fma(r * r2, ps, r);
  double pc = -0.001388888888888889;           // -1/6!
  pc = fma(pc, r2, 0.041666666666666664);      //  1/4!
  pc = fma(pc, r2, -0.5);                      // -1/2
  o.cr = fma(r2, pc, 1.0);
  return o;
}
__device__ __forceinline__ void sincos_finish(const SinCosPart& p, double* sn, double* cs) {
  *sn = fma(p.sa, p.cr, p.ca * p.sr);
  *cs = fma(p.ca, p.cr, -(p.sa * p.sr));
}
__device__ __forceinline__ void sincos_tab(const MathTables& T, double x, double* sn,
                                           double* cs) {
  sincos_finish(sincos_issue(T, x), sn, cs);
}

// e^x: x = (64 m + j) ln2/64 + r with ln2/64 split in two doubles,
// |r| <= ln2/128, Taylor polynomial of e^r to r^5 (truncation below 3.5e-17
// relative), times the tabulated 2^(j/64), scaled by 2^m.  The argument is
// clamped to [-746, 710] first: +inf above ~709.8, 0 below ~-745.
struct ExpPart {
  double p;   // e^r
  double tj;  // tabulated 2^(j/64)
  int m;
};
__device__ __forceinline__ ExpPart exp_issue(const MathTables& T, double x) {
  constexpr double k64OverLn2 = 92.33248261689366;
  constexpr double kL1 = 0.010830424696249145;
  constexpr double kL2 = 3.623510646634843e-19;
  x = fmin(fmax(x, -746.0), 710.0);
  const double t = fma(x, k64OverLn2, kShift);
  const double n = t - kShift;
  double r = fma(-n, kL1, x);
  r = fma(-n, kL2, r);
  const int ni = low_word(t);
  const int j = ni & 63;
  ExpPart o;
  o.m = ni >> 6;  // floor(n / 64)
  o.tj = ((const lds_double*)(&T.e2[0]))[j];
  double p = 0.008333333333333333;   // 1/5!
  p = fma(p, r, 0.041666666666666664);
  p = fma(p, r, 0.16666666666666666);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  o.p = fma(p, r, 1.0);
  return o;
}
__device__ __forceinline__ double exp_finish(const ExpPart& e) { return ldexp(e.tj * e.p, e.m); }
__device__ __forceinline__ double exp_tab(const MathTables& T, double x) {
  return exp_finish(exp_issue(T, x));
}

template <class Re>
struct CexpPart;
template <>
struct CexpPart<double> {
  SinCosPart sc;
  ExpPart ex;
};
__device__ __forceinline__ CexpPart<double> cexp_issue(const MathTables& T, cd z) {
  CexpPart<double> o;
  o.sc = sincos_issue(T, z.im);
  o.ex = exp_issue(T, z.re);
  return o;
}
__device__ __forceinline__ cd cexp_finish(const CexpPart<double>& p) {
  double s, c;
  sincos_finish(p.sc, &s, &c);
  const double e = exp_finish(p.ex);
  return mk(e * c, e * s);
}
__device__ __forceinline__ cd cexp_tab(const MathTables& T, cd z) {
  return cexp_finish(cexp_issue(T, z));
}

// Square of the fronting wavevector, kz0^2 = (Q/2)^2, formed as (0.25 q) q
// and then x = kz0^2 - A with no contraction into an FMA, so that the
// critical-edge difference is rounded once, in a fixed order.
__device__ __forceinline__ double kz_real_part(double kz0sq, double A) {
#pragma clang fp contract(off)
  return kz0sq - A;
}
__device__ __forceinline__ double kz0_squared(double q) {
#pragma clang fp contract(off)
  double h = 0.25 * q;
  return h * q;
}

// Root of w = x + i y (y <= 0) with Re >= 0, Im <= 0, and 1/|w| = 1/|kz|^2:
//   t = sqrt((|w| + |x|)/2), p = -y/(2t) (>= 0);  x >= 0 -> (t, -p), x < 0 -> (p, -t).
// Since t^2 - p^2 = |x|, t >= p, so with ts = t carrying the sign of x the
// branch is Re = max(ts, p), Im = min(-p, ts): three instructions (the sign
// is put on (|w| + |x|)/2 before its product with the reciprocal root, so
// the maximum and minimum take arithmetic results) instead of a compare and
// four selects.  Near x = 0, where t and p agree to rounding, either may be
// taken.  The 1e-300 guard keeps t and p NaN together or finite together, so
// the maximum and minimum, which drop a single NaN operand, never hide one.
// A zero y with x < 0 gives (0, -sqrt|x|) whatever the sign of that zero.
// |w|^2 gets 1e-300 added, which changes nothing unless w = 0 exactly, where
// it yields kz of order 1e-75 instead of 0 (and keeps every value finite).
template <class T>
struct RootT {
  cx<T> kz;
  T inv_abs2;
};
using Root = RootT<double>;
__device__ __forceinline__ Root kz_root(double x, double y) {
  const double a = fma(x, x, fma(y, y, 1e-300));
  const double ra = rsq(a);
  const double m = a * ra;
  const double h = 0.5 * (m + fabs(x));
  const double rh = rsq(h);
  const double ts = __builtin_copysign(h, x) * rh;
  const double p = -0.5 * (y * rh);
  Root out;
  out.kz.re = __builtin_fmax(ts, p);
  out.kz.im = __builtin_fmin(-p, ts);
  out.inv_abs2 = ra;
  return out;
}

// ---------------------------------------------------------------------------
// FP32 variant.  The hardware transcendentals of gfx950 are used directly:
// v_rcp_f32, v_rsq_f32 (about 1 ulp), v_exp_f32 (2^x), v_sin_f32 and
// v_cos_f32 (of 2 pi x, for |x| <= 256; the argument is reduced to
// [-1/2, 1/2] revolutions first).
// ---------------------------------------------------------------------------
__device__ __forceinline__ cf crecip(cf z) {
  const float inv = __builtin_amdgcn_rcpf(z.re * z.re + z.im * z.im);
  return mk(z.re * inv, -z.im * inv);
}

__device__ __forceinline__ float exp_f32(float x) {
  constexpr float kLog2e = 1.44269504088896341f;
  return __builtin_amdgcn_exp2f(x * kLog2e);
}

__device__ __forceinline__ void sincos_f32(float x, float* sn, float* cs) {
  constexpr float kInv2Pi = 0.159154943091895336f;
  float u = x * kInv2Pi;
  u = u - __builtin_rintf(u);
  *sn = __builtin_amdgcn_sinf(u);
  *cs = __builtin_amdgcn_cosf(u);
}

// Complex exponential in FP32 (the LDS tables are not used; the issue half
// only holds the argument).
__device__ __forceinline__ cf cexp_f32(cf z) {
  float s, c;
  sincos_f32(z.im, &s, &c);
  const float e = exp_f32(z.re);
  return mk(e * c, e * s);
}
__device__ __forceinline__ cf cexp_tab(const MathTables&, cf z) { return cexp_f32(z); }
template <>
struct CexpPart<float> {
  cf z;
};
__device__ __forceinline__ CexpPart<float> cexp_issue(const MathTables&, cf z) { return {z}; }
__device__ __forceinline__ cf cexp_finish(const CexpPart<float>& p) { return cexp_f32(p.z); }

// The FP32 root of w = x + i y, same branch as kz_root(double, double), with
// selects (o = -p): the select-free form gives the same bits in FP32 but
// measured 2 % slower on the 4096-draw batch; x is the FP64 difference kz0^2 - A rounded once to float, so the
// cancellation near a critical edge happens in FP64.  |w|^2 gets 1e-36 added
// (a floor of 1e-18 on |w|), which keeps w = 0 finite.
__device__ __forceinline__ RootT<float> kz_root(float x, float y) {
  const float a = fmaf(x, x, fmaf(y, y, 1e-36f));
  const float ra = __builtin_amdgcn_rsqf(a);
  const float m = a * ra;
  const float h = 0.5f * (m + fabsf(x));
  const float rh = __builtin_amdgcn_rsqf(h);
  const float t = h * rh;
  const float o = 0.5f * (y * rh);
  RootT<float> out;
  out.kz.re = (x >= 0.0f) ? t : -o;
  out.kz.im = (x >= 0.0f) ? o : -t;
  out.inv_abs2 = ra;
  return out;
}

// Width of the smearing Gaussian of one point: sigma_Q = (dQ/Q) Q /
// (2 sqrt(2 ln 2)), or dQ / (2 sqrt(2 ln 2)) for a given per-point FWHM; and
// the node q = Q + sigma_Q t.  In this order, no FMA.
__device__ __forceinline__ double smear_sigma_rel(double Q, double dqq) {
#pragma clang fp contract(off)
  double s = dqq * Q;
  return s / kFwhmPerSigma;
}
__device__ __forceinline__ double smear_sigma_abs(double dq) {
#pragma clang fp contract(off)
  return dq / kFwhmPerSigma;
}
__device__ __forceinline__ double smear_at(double Q, double sig, double t) {
#pragma clang fp contract(off)
  return Q + sig * t;
}

// Wave-wide sum of a double (all 64 lanes end with the total), fixed order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace nr
