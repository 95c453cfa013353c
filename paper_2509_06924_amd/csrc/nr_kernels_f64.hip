// FP64 instantiation of the kernels (shallow buckets; the deeper ones are
// compiled from nr_kernels_bucket.hip), the per-item constant prologue, the per-item
// reductions, and the launch entry points of both precisions.
#include <algorithm>

#include "nr_kernels.hpp"

namespace nr {

NR_DEFINE_GRAD_LAUNCHER(launch_grad_shallow, NR_BUCKETS_SHALLOW)

// One block of 64 per item, lanes over the media: the item's layer records
// (doubles and their float copies for the FP32 variant).
__global__ __launch_bounds__(64) void k_item_consts(const int64_t* row_off, const double* layers,
                                                    double* rec, float* recf, int n_items) {
  const int b = blockIdx.x;
  if (b >= n_items) return;
  const int64_t r0 = row_off[b];
  const int NR = (int)(row_off[b + 1] - r0);
  const double* rows = layers + 4 * r0;
  for (int m = threadIdx.x; m < NR; m += 64) {
  const double rho0 = rows[1];
  auto Af = [&](int j) { return (j == 0) ? 0.0 : kFourPi * (rows[4 * j + 1] - rho0); };
  auto Bf = [&](int j) { return (j == 0) ? 0.0 : kFourPi * fabs(rows[4 * j + 2]); };
  double v[kRecDoubles];
  const double A = Af(m), B = Bf(m);
  v[0] = A;
  v[1] = B;
  if (m + 1 < NR) {
    const double sg = rows[4 * (m + 1) + 3];
    v[2] = Af(m + 1) - A;
    v[3] = Bf(m + 1) - B;
    v[4] = -2.0 * (sg * sg);
  } else {
    v[2] = 0.0;
    v[3] = 0.0;
    v[4] = 0.0;
  }
  // the fronting and backing have no thickness (their rows' d is ignored)
  v[5] = (m == 0 || m + 1 == NR) ? 0.0 : 2.0 * rows[4 * m];
  double* out = rec + (r0 + m) * kRecDoubles;
  for (int f = 0; f < kRecDoubles; ++f) out[f] = v[f];
  float* outf = recf + (r0 + m) * kRecFloats;
  for (int f = 0; f < 5; ++f) outf[f] = (float)v[f + 1];
  for (int f = 5; f < kRecFloats; ++f) outf[f] = 0.0f;
  }
}

// ---------------------------------------------------------------------------
// Deterministic per-item reductions of the WU records.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce_loglik(ReduceArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.n_items) return;
  const int64_t first = a.item_wu_first[b];
  const int cnt = a.item_wu_count[b];
  // eight offsets, then their eight records, per round: independent loads
  // instead of a chain of dependent ones; the sum runs over the units in order
  double s = 0.0;
  for (int k0 = 0; k0 < cnt; k0 += 8) {
    int64_t o[8];
    double r[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = (k0 + j < cnt) ? a.rec_of_wu[first + k0 + j] : 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) r[j] = (k0 + j < cnt) ? a.rec[o[j]] : 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (k0 + j < cnt) s += r[j];
  }
  a.logL[b] = s;
}

// One block per item of 64 x W threads (W from the plan's deepest item, so
// that the thousands of fields of a deep item's records are spread over
// many waves): threads sum record fields over the item's WUs, then turn the
// sums into gradients of the row entries.  With gridDim.y = 4 (plans with
// deep items) an item has four blocks, one per plane of the record (sum
// Re wbar, sum Im wbar, the d sums, the sigma sums): each row-gradient
// column comes from one plane, so the blocks need nothing from each other,
// and a deep item's reduction spreads over four compute units.  Block 0
// also takes the leading fields and the resolution field.
__global__ __launch_bounds__(1024) void k_reduce_grad(ReduceArgs a) {
  extern __shared__ double fsum[];
  __shared__ int64_t offs[64];
  __shared__ double wpart[16];
  const int b = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int64_t first = a.item_wu_first[b];
  const int cnt = a.item_wu_count[b];
  const int64_t roff = a.row_off[b];
  const int NR = (int)(a.row_off[b + 1] - roff);
  // records hold 4 + 4 NR doubles; the last is written by the resolution
  // form only
  const int nf = (a.g_res ? 4 : 3) + 4 * NR;
  const bool by_plane = gridDim.y == 4;
  const int plane = blockIdx.y;
  const bool lead = !by_plane || plane == 0;  // this block's fields include 0, 1, 2
  // the fields this block sums: all nf, or plane `plane` (NR fields) and, for
  // plane 0, the leading ones; field of the block's i-th: fld(i)
  const int nmine = by_plane ? NR + (plane == 0 ? nf - 4 * NR : 0) : nf;
  auto fld = [&](int i) {
    if (!by_plane) return i;
    if (i < NR) return 3 + plane * NR + i;
    return (i - NR < 3) ? i - NR : 3 + 4 * NR;
  };
  // The units' record offsets are staged 64 at a time (one load per
  // thread), so the record loads of a chunk are independent of each other
  // instead of each waiting for its offset; the sum runs over the units in
  // order.  A thread issues 32 record loads before it adds them (in order):
  // an item with few units but thousands of fields (a deep stack) has few
  // blocks, so its time is the latency of these loads.
  constexpr int kAhead = 32;
  for (int k0 = 0; k0 < cnt; k0 += 64) {
    const int kc = min(64, cnt - k0);
    __syncthreads();  // the previous chunk's offsets are no longer read
    if (tid < kc) offs[tid] = a.rec_of_wu[first + k0 + tid];
    __syncthreads();
    for (int i = tid; i < nmine; i += nt) {
      const int f = fld(i);
      double v = (k0 == 0) ? 0.0 : fsum[f];
      int k = 0;
      for (; k + kAhead <= kc; k += kAhead) {
        double r[kAhead];
#pragma unroll
        for (int j = 0; j < kAhead; ++j) r[j] = a.rec[offs[k + j] + f];
#pragma unroll
        for (int j = 0; j < kAhead; ++j) v += r[j];
      }
#pragma unroll 8
      for (; k < kc; ++k) v += a.rec[offs[k] + f];
      fsum[f] = v;
    }
  }
  if (cnt <= 0)
    for (int i = tid; i < nmine; i += nt) fsum[fld(i)] = 0.0;
  __syncthreads();
  const double* rows = a.layers + 4 * roff;
  double* g = a.g_rows + 4 * roff;
  for (int m = tid; m < NR; m += nt) {
    // column c of row m comes from plane (c + 2) % 4 of the record
    if (!by_plane || plane == 2) g[4 * m + 0] = (m >= 1 && m <= NR - 2) ? fsum[3 + 2 * NR + m] : 0.0;
    if (!by_plane || plane == 0) g[4 * m + 1] = (m >= 1) ? -kFourPi * fsum[3 + m] : 0.0;
    if (!by_plane || plane == 1) {
      const double sgn = (rows[4 * m + 2] < 0.0) ? -1.0 : 1.0;
      g[4 * m + 2] = (m >= 1) ? -kFourPi * sgn * fsum[3 + NR + m] : 0.0;
    }
    if (!by_plane || plane == 3)
      g[4 * m + 3] = (m >= 1) ? -4.0 * rows[4 * m + 3] * fsum[3 + 3 * NR + m] : 0.0;
  }
  if (!lead) return;
  // fronting rho_re: the model depends on rho_re,m - rho_re,0 only; the
  // waves' partial sums are added in wave order
  double part = 0.0;
  for (int m = 1 + tid; m < NR; m += nt) part += fsum[3 + m];
  part = wave_sum(part);
  if (lane == 0) wpart[wv] = part;
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int v = 0; v < nt / 64; ++v) tot += wpart[v];
    g[1] = kFourPi * tot;
    a.logL[b] = fsum[0];
    a.g_inst[2 * b + 0] = fsum[1];
    a.g_inst[2 * b + 1] = fsum[2];
    if (a.g_res) a.g_res[b] = fsum[3 + 4 * NR];
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_item_consts(const int64_t* row_off, const double* layers, double* rec,
                              float* recf, int n_items, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_item_consts, dim3(n_items), dim3(64), 0, st, row_off, layers, rec, recf,
                     n_items);
  return hipGetLastError();
}

hipError_t launch_forward(int precision, int op, bool split, const KernelArgs& a, int n_wu,
                          hipStream_t st) {
  return precision == NR_F32 ? launch_forward_f32(op, split, a, n_wu, st)
                             : launch_forward_p<F64>(op, split, a, n_wu, st);
}

hipError_t launch_grad(int precision, int bucket, int form, int mode, const KernelArgs& a,
                       int n_wu, hipStream_t st) {
  if (bucket == kDeepBucket) return hipErrorInvalidValue;  // launch_grad_scan
  if (bucket >= kFirstDeepBucket) {
    switch (kBucketLmax[bucket]) {
#define NR_DEEP_CASE(LM)                                                             \
  case LM:                                                                           \
    return precision == NR_F32 ? NR_DEEP_LAUNCHER(F32, LM)(form, mode, a, n_wu, st) \
                               : NR_DEEP_LAUNCHER(F64, LM)(form, mode, a, n_wu, st);
      NR_BUCKETS_DEEP(NR_DEEP_CASE)
#undef NR_DEEP_CASE
      default:
        return hipErrorInvalidValue;
    }
  }
  return precision == NR_F32 ? launch_grad_f32(bucket, form, mode, a, n_wu, st)
                             : launch_grad_shallow<F64>(bucket, form, mode, a, n_wu, st);
}

hipError_t prepare_reduce(int max_rows) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_reduce_grad),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(sizeof(double) * (4 + 4 * (size_t)max_rows)));
}

hipError_t launch_reduce(int op, const ReduceArgs& a, hipStream_t st) {
  if (a.n_items <= 0) return hipSuccess;
  if (op == kOpLoglik) {
    hipLaunchKernelGGL(k_reduce_loglik, dim3((a.n_items + 255) / 256), dim3(256), 0, st, a);
  } else {
    const size_t shmem = sizeof(double) * (4 + 4 * (size_t)a.max_rows);
    // one wave per 64 rows of the deepest item, at most 16; beyond 64 rows,
    // one block per record plane and item
    const int waves = std::min(16, std::max(1, (a.max_rows + 63) / 64));
    const int planes = a.max_rows > 64 ? 4 : 1;
    hipLaunchKernelGGL(k_reduce_grad, dim3(a.n_items, planes), dim3(64 * waves), shmem, st, a);
  }
  return hipGetLastError();
}

}  // namespace nr
