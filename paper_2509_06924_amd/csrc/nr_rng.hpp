// Device random numbers and parameter transforms shared by the sampling and
// variational drivers.
//
// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two
// 64 x 64 -> 128-bit products on words 0 and 2; the high halves are XOR-ed
// with the other words and the round key, which is bumped by the Weyl
// increments after every round.  Key (seed, 0); counter (iteration, stream,
// block, purpose).  Normal number e of a stream is Box-Muller normal e mod 4
// of block e / 4 (pairs of uniforms (0, 1) and (2, 3)).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "nr.h"

namespace nr {

struct U4 {
  uint64_t v[4];
};

__device__ __forceinline__ U4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                            uint64_t k0, uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo0 = kM0 * c0, hi0 = __umul64hi(kM0, c0);
    const uint64_t lo1 = kM1 * c2, hi1 = __umul64hi(kM1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += kW0;
    k1 += kW1;
  }
  return U4{{c0, c1, c2, c3}};
}

// The top 53 bits, centred in their interval: an exact double in (0, 1).
__device__ __forceinline__ double open_uniform(uint64_t x) {
  return ((double)(x >> 11) + 0.5) * 0x1.0p-53;
}

constexpr uint64_t kPurposeMomentum = 0, kPurposeAccept = 1, kPurposeVi = 2;

__device__ inline double rng_normal(uint64_t seed, uint64_t iter, uint64_t stream, int e,
                                    uint64_t purpose) {
  const U4 x = philox4x64_10(iter, stream, (uint64_t)(e >> 2), purpose, seed, 0);
  const int j = e & 3;
  const double u0 = open_uniform(x.v[2 * (j >> 1)]);
  const double u1 = open_uniform(x.v[2 * (j >> 1) + 1]);
  const double rad = sqrt(-2.0 * log(u0));
  const double ang = 2.0 * M_PI * u1;
  return rad * ((j & 1) ? sin(ang) : cos(ang));
}

// Output 0 of block 0 of a stream as a uniform.
__device__ __forceinline__ double rng_uniform(uint64_t seed, uint64_t iter, uint64_t stream,
                                              uint64_t purpose) {
  return open_uniform(philox4x64_10(iter, stream, 0, purpose, seed, 0).v[0]);
}

// ---------------------------------------------------------------------------
// Transforms between an unconstrained coordinate z and a parameter theta
// (Sec. 2.3: pre-scaling, log space, hard constraints): theta, dtheta/dz,
// ln|dtheta/dz| and its z-derivative.
// ---------------------------------------------------------------------------
struct Tf {
  double theta, dtdz, logj, dlogj;
};

__device__ __forceinline__ double sigmoid_d(double z) {
  return (z >= 0.0) ? 1.0 / (1.0 + exp(-z)) : exp(z) / (1.0 + exp(z));
}
__device__ __forceinline__ double softplus_d(double z) {
  return (z > 0.0) ? z + log1p(exp(-z)) : log1p(exp(z));
}

__device__ inline Tf transform_z(uint8_t kind, double a, double b, double z) {
  Tf t;
  if (kind == NR_TF_AFFINE) {
    t.theta = a + b * z;
    t.dtdz = b;
    t.logj = log(fabs(b));
    t.dlogj = 0.0;
  } else if (kind == NR_TF_LOG) {
    const double ez = exp(z);
    t.theta = a + b * ez;
    t.dtdz = b * ez;
    t.logj = log(b) + z;
    t.dlogj = 1.0;
  } else {  // NR_TF_LOGIT
    const double s = sigmoid_d(z);
    const double w = b - a;
    t.theta = a + w * s;
    t.dtdz = w * s * (1.0 - s);
    t.logj = log(w) - softplus_d(-z) - softplus_d(z);
    t.dlogj = 1.0 - 2.0 * s;
  }
  return t;
}

__device__ inline double inverse_transform_z(uint8_t kind, double a, double b, double theta) {
  if (kind == NR_TF_AFFINE) return (theta - a) / b;
  if (kind == NR_TF_LOG) return log((theta - a) / b);
  const double f = (theta - a) / (b - a);
  return log(f) - log1p(-f);
}

// Whether the model reads field f of a row of kind k (0 fronting: rho_re only;
// 1 finite layer: all four; 2 backing: no thickness).
__device__ __forceinline__ bool row_entry_read(uint8_t row_kind, int f) {
  return row_kind == 1 || (row_kind == 0 && f == 1) || (row_kind == 2 && f != 0);
}

}  // namespace nr
