// Device-side complex arithmetic and the special functions of the layer
// product, for gfx950.  Everything here is FP64.
#pragma once

#include <hip/hip_runtime.h>

namespace nr {

// 4 pi, ln(2 pi)/2 and 2 sqrt(2 ln 2) (FWHM of a unit Gaussian), as doubles.
constexpr double kFourPi = 12.566370614359172;
constexpr double kHalfLn2Pi = 0.91893853320467274;
constexpr double kFwhmPerSigma = 2.3548200450309493;

struct cd {
  double re, im;
};

__device__ __forceinline__ cd mk(double a, double b) {
  cd z;
  z.re = a;
  z.im = b;
  return z;
}
__device__ __forceinline__ cd operator+(cd a, cd b) { return mk(a.re + b.re, a.im + b.im); }
__device__ __forceinline__ cd operator-(cd a, cd b) { return mk(a.re - b.re, a.im - b.im); }
__device__ __forceinline__ cd operator-(cd a) { return mk(-a.re, -a.im); }
__device__ __forceinline__ cd operator*(cd a, cd b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
__device__ __forceinline__ cd operator*(double s, cd a) { return mk(s * a.re, s * a.im); }
__device__ __forceinline__ cd& operator+=(cd& a, cd b) {
  a.re += b.re;
  a.im += b.im;
  return a;
}
__device__ __forceinline__ cd cconj(cd a) { return mk(a.re, -a.im); }
// conj(a) * b
__device__ __forceinline__ cd cmulc(cd a, cd b) {
  return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
__device__ __forceinline__ double cabs2(cd a) { return a.re * a.re + a.im * a.im; }
// 1/x from the hardware estimate v_rcp_f64 refined by two Newton steps
// r <- r + r (1 - x r); each step squares the relative error.
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ cd crecip(cd z) {
  const double inv = rcp(z.re * z.re + z.im * z.im);
  return mk(z.re * inv, -z.im * inv);
}

// sin and cos of x: FMA-based Cody-Waite reduction r = x - n pi/2 with pi/2
// split into three doubles (|r| <= pi/4, accurate to a few ulp for
// |x| < 2^40), Taylor series of sin to r^17 and of cos to r^18 (truncation
// below 1e-19 on |r| <= pi/4), then the quadrant n mod 4.
__device__ __forceinline__ void sincos_cw(double x, double* sn, double* cs) {
  constexpr double kTwoOverPi = 0.6366197723675814;
  constexpr double kP1 = 1.5707963267948966;
  constexpr double kP2 = 6.123233995736766e-17;
  constexpr double kP3 = -1.4973849048591698e-33;
  const double n = rint(x * kTwoOverPi);
  double r = fma(-n, kP1, x);
  r = fma(-n, kP2, r);
  r = fma(-n, kP3, r);
  const double r2 = r * r;
  // sin r = r + r^3 ps,  ps = -1/3! + r^2/5! - ... + r^14/17!
  double ps = 2.8114572543455206e-15;
  ps = fma(ps, r2, -7.647163731819816e-13);
  ps = fma(ps, r2, 1.6059043836821613e-10);
  ps = fma(ps, r2, -2.505210838544172e-08);
  ps = fma(ps, r2, 2.7557319223985893e-06);
  ps = fma(ps, r2, -0.0001984126984126984);
  ps = fma(ps, r2, 0.008333333333333333);
  ps = fma(ps, r2, -0.16666666666666666);
  const double s_r = fma(r * r2, ps, r);
  // cos r = 1 - (r^2/2 - r^4 pc),  pc = 1/4! - r^2/6! + ... - r^14/18!
  double pc = -1.5619206968586225e-16;
  pc = fma(pc, r2, 4.779477332387385e-14);
  pc = fma(pc, r2, -1.1470745597729725e-11);
  pc = fma(pc, r2, 2.08767569878681e-09);
  pc = fma(pc, r2, -2.755731922398589e-07);
  pc = fma(pc, r2, 2.48015873015873e-05);
  pc = fma(pc, r2, -0.001388888888888889);
  pc = fma(pc, r2, 0.041666666666666664);
  const double c_r = 1.0 - fma(-(r2 * r2), pc, 0.5 * r2);
  // quadrant q = n mod 4 (exact for |n| < 2^53)
  const int q = (int)(n - 4.0 * floor(0.25 * n));
  const double s_sw = (q & 1) ? c_r : s_r;
  const double c_sw = (q & 1) ? s_r : c_r;
  *sn = (q & 2) ? -s_sw : s_sw;
  *cs = ((q + 1) & 2) ? -c_sw : c_sw;
}

// e^x: reduction x = n ln2 + r, |r| <= ln2/2 (ln2 split into two doubles),
// Taylor series of e^r to r^13 (truncation < 5e-18), scaling by 2^n.
// Saturates to +inf above ~709.8 and to 0 below ~-745.
__device__ __forceinline__ double exp_cw(double x) {
  constexpr double kLog2e = 1.4426950408889634;
  constexpr double kLn2Hi = 0.6931471805599453;
  constexpr double kLn2Lo = 2.3190468138462996e-17;
  double n = rint(x * kLog2e);
  n = fmin(fmax(n, -1100.0), 1100.0);
  double r = fma(-n, kLn2Hi, x);
  r = fma(-n, kLn2Lo, r);
  double p = 1.6059043836821613e-10;  // 1/13!
  p = fma(p, r, 2.08767569878681e-09);
  p = fma(p, r, 2.505210838544172e-08);
  p = fma(p, r, 2.755731922398589e-07);
  p = fma(p, r, 2.7557319223985893e-06);
  p = fma(p, r, 2.48015873015873e-05);
  p = fma(p, r, 0.0001984126984126984);
  p = fma(p, r, 0.001388888888888889);
  p = fma(p, r, 0.008333333333333333);
  p = fma(p, r, 0.041666666666666664);
  p = fma(p, r, 0.16666666666666666);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)n);
}

// exp(z) = e^{Re z} (cos Im z + i sin Im z)
__device__ __forceinline__ cd cexp(cd z) {
  double s, c;
  sincos_cw(z.im, &s, &c);
  const double e = exp_cw(z.re);
  return mk(e * c, e * s);
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

// Root of w = x + i y (y <= 0) with Re >= 0, Im <= 0:
//   t = sqrt((|w| + |x|)/2), o = y/(2t) (<= 0);  x >= 0 -> (t, o), x < 0 -> (-o, -t).
// A zero y with x < 0 gives (0, -sqrt|x|) whatever the sign of that zero.
__device__ __forceinline__ cd kz_root(double x, double y) {
  double m = sqrt(x * x + y * y);
  double t = sqrt(0.5 * (m + fabs(x)));
  double o = (t > 0.0) ? 0.5 * (y / t) : 0.0;
  cd pos = mk(t, o);
  cd neg = mk(-o, -t);
  return (x >= 0.0) ? pos : neg;
}

// Smearing node q = Q + ((dQ/Q) Q / (2 sqrt(2 ln 2))) t, in this order, no FMA.
__device__ __forceinline__ double smear_node(double Q, double dqq, double t) {
#pragma clang fp contract(off)
  double s = dqq * Q;
  s = s / kFwhmPerSigma;
  return Q + s * t;
}

// Wave-wide sum of a double (all 64 lanes end with the total), fixed order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace nr
