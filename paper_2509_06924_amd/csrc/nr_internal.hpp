// Internal interface between the C ABI (nr_api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "nr.h"

namespace nr {

constexpr int kSmearNodes = NR_SMEAR_NODES;
constexpr int kMaxLayers = NR_MAX_LAYERS;
constexpr int kWuPoints = 64;  // data points per work unit (one per lane)
// Deepest stack whose gradient kernel keeps the per-level state and phases
// in LDS (3 x 16 B x 64 lanes per level in FP64, 3 x 8 B in FP32); deeper
// stacks recompute them.
constexpr int kStoreMaxLayers = 10;
constexpr int kStoreMaxLayersF32 = 10;
// Per-row layer records in the workspace: 6 doubles, then (in a second
// array) 8 floats.
constexpr int kRecDoubles = 6;
constexpr int kRecFloats = 8;

constexpr uint32_t kItemNonfinite = NR_ITEM_NONFINITE;
constexpr uint32_t kItemBadQ = NR_ITEM_BAD_Q;
constexpr uint32_t kItemBadErr = NR_ITEM_BAD_ERR;
constexpr uint32_t kItemEdgeSingular = NR_ITEM_EDGE_SINGULAR;

constexpr int kOpReflectivity = NR_OP_REFLECTIVITY;
constexpr int kOpLoglik = NR_OP_LOGLIK;
constexpr int kOpLoglikGrad = NR_OP_LOGLIK_GRAD;

// Layer-count buckets: a kernel instantiated for LMAX serves items with
// N <= LMAX finite layers (its layer loops are unrolled to LMAX and skip the
// levels beyond N).
// (shallow and deep buckets are compiled in separate translation units)
#define NR_BUCKETS_SHALLOW(X) X(1) X(2) X(4) X(6) X(8) X(10) X(12)
#define NR_BUCKETS_DEEP(X) X(14) X(16) X(18) X(20) X(24) X(28) X(32) X(36) X(40)
#define NR_BUCKETS(X) NR_BUCKETS_SHALLOW(X) NR_BUCKETS_DEEP(X)
constexpr int kFirstDeepBucket = 7;
constexpr int kBucketLmax[] = {1, 2, 4, 6, 8, 10, 12, 14, 16, 18, 20, 24, 28, 32, 36, 40};
constexpr int kNumBuckets = sizeof(kBucketLmax) / sizeof(int);
static_assert(kNumBuckets == NR_NUM_BUCKETS, "bucket table and ABI disagree");

// Items deeper than the unrolled buckets form one more work list, served by
// the parallel-in-layers scan kernel (nr_kernels_scan.hip).
constexpr int kDeepBucket = kNumBuckets;
constexpr int kMaxDeepLayers = NR_MAX_DEEP_LAYERS;
constexpr int kScanMaxChunk = (kMaxDeepLayers + 1 + 63) / 64;  // levels per lane
inline int bucket_of(int N) {
  for (int b = 0; b < kNumBuckets; ++b)
    if (N <= kBucketLmax[b]) return b;
  return kDeepBucket;
}

struct KernelArgs {
  // work list of one launch (launch order)
  const int32_t* wu_item;
  // split tail units: points | node groups << 16 per unit
  const int32_t* wu_split;
  const int32_t* wu_p0;
  const int64_t* wu_rec;
  // tail work units: per-lane item, point and record (64 per unit)
  const int32_t* tail_item;
  const int32_t* tail_pt;
  const int64_t* tail_rec;
  // batch structure (plan-owned device copies)
  const int32_t* dataset_of_item;
  const int64_t* q_off;
  const int64_t* row_off;
  const double* dq_over_q;
  const int64_t* out_off;
  // resolution (caller-owned, optional): per-point FWHM, per-item dQ/Q
  const double* dq;
  const double* dqq_item;
  // values (caller-owned)
  const double* q;
  const double* r_obs;
  const double* r_err;
  const double* layers;
  const double* scale;
  const double* bkg;
  int32_t* item_status;
  // outputs
  double* out;     // nr_reflectivity
  // nr_reflectivity_vjp: per-point seeds (packed like R_hat); when set, the
  // gradient kernel differentiates sum_i seed_i R_hat_i instead of logL
  const double* seed;
  double* rec;     // workspace records
  const double* consts;  // workspace: per-item layer records (6 doubles per row)
  const float* constsf;  // workspace: their float copies (8 floats per row)
  // plan-owned constants (device): quadrature node offsets in units of
  // sigma_Q and normalised weights (kSmearNodes each), then the tables
  // (sin, cos)(k pi/64) for k = 0..127 interleaved and 2^(j/64), j = 0..63
  const double* rule;
  int zero_mask;  // always 0 (see the layer-record indexing in the kernels)
};

struct ReduceArgs {
  int32_t n_items;
  const int64_t* item_wu_first;
  const int32_t* item_wu_count;
  const int64_t* rec_of_wu;
  const double* rec;
  const int64_t* row_off;
  const double* layers;
  double* logL;
  double* g_rows;
  double* g_inst;
  double* g_res;  // optional: dlogL/d(dQ/Q) per item
  int32_t max_rows;  // the largest rows of any item (record length)
};

hipError_t launch_item_consts(const int64_t* row_off, const double* layers, double* rec,
                              float* recf, int n_items, hipStream_t st);
// precision: NR_F64 or NR_F32
hipError_t launch_forward(int precision, int op, bool split, const KernelArgs& a, int n_wu,
                          hipStream_t st);
// store: the store variant (only for buckets within store_max_layers)
// Forms of the gradient kernel: the recompute form, the store form (buckets up
// to the precision's store limit), and the recompute form that also
// accumulates the derivative with respect to the relative resolution.
enum GradForm { kFormRecompute = 0, kFormStore = 1, kFormRecomputeRes = 2 };
// mode: kModeFull (64 points of one item), kModeTail (packed partial
// groups of several items), kModeSplit (one item's partial group, lanes over
// node groups x points)
enum WuMode { kModeFull = 0, kModeTail = 1, kModeSplit = 2 };
hipError_t launch_grad(int precision, int bucket, int form, int mode, const KernelArgs& a,
                       int n_wu, hipStream_t st);
hipError_t launch_forward_f32(int op, bool split, const KernelArgs& a, int n_wu, hipStream_t st);
hipError_t launch_grad_f32(int bucket, int form, int mode, const KernelArgs& a, int n_wu,
                           hipStream_t st);
// Deep buckets (index >= kFirstDeepBucket): one object per (precision,
// bucket), built from nr_kernels_bucket.hip, each exporting
// launch_grad_deep_<F64|F32>_<layers>.
#define NR_CAT4_(a, b, c, d) a##b##c##d
#define NR_CAT4(a, b, c, d) NR_CAT4_(a, b, c, d)
#define NR_DEEP_LAUNCHER(PREC, LM) NR_CAT4(launch_grad_deep_, PREC, _, LM)
struct F64;
struct F32;
#define NR_DECLARE_DEEP(LM)                                                                  \
  hipError_t NR_DEEP_LAUNCHER(F64, LM)(int form, int mode, const KernelArgs& a, int n_wu,  \
                                       hipStream_t st);                                      \
  hipError_t NR_DEEP_LAUNCHER(F32, LM)(int form, int mode, const KernelArgs& a, int n_wu,  \
                                       hipStream_t st);
NR_BUCKETS_DEEP(NR_DECLARE_DEEP)
#undef NR_DECLARE_DEEP
inline int store_max_layers(int precision) {
  return precision == NR_F32 ? kStoreMaxLayersF32 : kStoreMaxLayers;
}
// Deepest bucket whose default (NR_VARIANT_AUTO) is the store variant.
// Measured on MI355X at 4096 items x 400 points: FP64 store beats the
// recompute form (with its LDS cache of phases and roughness factors, two
// waves per SIMD) up to 4 layers (0.71 vs 0.60 of peak) and loses from 6 on
// (10 layers: 0.56 vs 0.60); FP32 store wins up to 8 layers.
inline int default_store_layers(int precision) { return precision == NR_F32 ? 8 : 4; }
hipError_t launch_reduce(int op, const ReduceArgs& a, hipStream_t st);
// Allows the gradient reduction its dynamic LDS for records of max_rows media.
hipError_t prepare_reduce(int max_rows);
// The scan kernel for items deeper than kMaxLayers: one wave per (item,
// point) unit, ch_max = the largest levels-per-lane of the launch's items.
hipError_t launch_grad_scan(bool res, int ch_max, const KernelArgs& a, int n_wu, hipStream_t st);
size_t scan_lds_bytes(int ch_max);
// Allows the scan kernels their dynamic LDS (over 64 KB for deep chunks).
hipError_t prepare_grad_scan(int ch_max);

hipError_t launch_kick(int64_t n_row_entries, int64_t n_inst, double* mom_rows,
                       const double* g_rows, double* mom_inst, const double* g_inst, double h,
                       hipStream_t st);
hipError_t launch_drift(int64_t n_row_entries, int64_t n_items, const uint8_t* row_kind,
                        double* layers, double* scale, double* bkg, const double* mom_rows,
                        const double* mom_inst, const double* im_rows, const double* im_inst,
                        double dt, hipStream_t st);
hipError_t launch_vi_sample(int64_t n_samples, int P, int rows, const double* mu,
                            const double* omega, const uint8_t* mask, const double* eps,
                            double* layers, double* scale, double* bkg, hipStream_t st);
hipError_t launch_vi_reduce(int64_t n_samples, int P, int rows, const double* omega,
                            const uint8_t* mask, const double* eps, const double* logL,
                            const double* g_rows, const double* g_inst, double* grad_mu,
                            double* grad_omega, double* elbo, hipStream_t st);
hipError_t launch_tie_sum(int64_t n_out, const int64_t* first, const int64_t* src,
                          const double* in, double* out, hipStream_t st);

// Arguments of the per-chain HMC kernels: the caller's chain arrays
// (nr_hmc_chains), the plan's structure, and the driver's own device state.
struct HmcArgs {
  int32_t n_items;
  int64_t n_row_entries;  // 4 x rows; instrument entries follow in the driver's arrays
  const int64_t* row_off;
  const uint8_t* row_kind;
  // caller's chains
  double* z_rows;
  double* z_inst;
  const uint8_t* kind_rows;
  const uint8_t* kind_inst;
  const double* a_rows;
  const double* b_rows;
  const double* a_inst;
  const double* b_inst;
  double* im_rows;
  double* im_inst;
  double* step;
  double* layers;
  double* scale;
  double* bkg;
  double* logL;
  double* g_rows;
  double* g_inst;
  double* U;
  double* accept_prob;
  double* energy_error;
  int32_t* n_accept;
  int32_t* n_divergent;
  // driver state: momentum, saved position and gradient, Welford sums (one
  // per entry each), per-chain scalars, iteration counters
  double* r;
  double* z0;
  double* g0;
  double* wmean;
  double* wm2;
  double* cs;
  uint64_t* iter;
  // configuration
  uint64_t seed;
  double max_energy_error;
  double target_accept;
};
constexpr int kChainScalars = 8;
enum HmcKernel { kHmcTheta, kHmcPotential, kHmcBegin, kHmcDrift, kHmcKick, kHmcEnd, kHmcAdapt };
// arg: from_theta (kHmcTheta), adaptation bits (kHmcEnd), actions (kHmcAdapt);
// frac: the kick's fraction of the step (kHmcKick)
hipError_t launch_hmc(int which, const HmcArgs& h, int arg, double frac, hipStream_t st);

// Arguments of the full-rank Gaussian VI kernels: the caller's variational
// parameters (nr_vi_mvn_params) and the driver's per-draw arrays.
constexpr int kMvnMaxEntries = 4 * (kMaxLayers + 2) + 2;
struct MvnArgs {
  int32_t R, S, P, rows;
  const uint8_t* kind;
  const double* a;
  const double* b;
  const double* theta_fixed;
  double* mu;
  double* omega;
  double* lam;
  double* grad_mu;
  double* grad_omega;
  double* grad_lam;
  double* elbo;
  // driver state: per draw eps, z, h (P each), f; the draws' parameters,
  // logL and gradient; Adam moments; the iteration counter
  double* eps;
  double* z;
  double* h;
  double* f;
  double* layers;
  double* scale;
  double* bkg;
  double* logL;
  double* g_rows;
  double* g_inst;
  double* adam_m;
  double* adam_v;
  uint64_t* iter;
  uint64_t seed;
  double lr, beta1, beta2, adam_eps;
};
enum MvnKernel { kMvnSample, kMvnChain, kMvnReduce, kMvnAdam, kMvnTick };
hipError_t launch_mvn(int which, const MvnArgs& v, hipStream_t st);

}  // namespace nr
