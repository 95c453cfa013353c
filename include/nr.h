/*
 * nr.h — C ABI of the MI355X (gfx950) library for the specular neutron
 * reflectivity log-likelihood and its exact gradient (arXiv 2509.06924).
 *
 * The operation (paper Sec. 2.1 problem statement, Sec. 3 API, Sec. 4.1 chi^2):
 * for every item b (one parameter draw of one slab stack, bound to one
 * dataset), and every data point Q_i of that dataset,
 *
 *   kz0 = Q/2,  kz_j = sqrt(kz0^2 - 4 pi (rho_re,j - rho_re,0) - i 4 pi |rho_im,j|)
 *                  (root with Re >= 0, Im <= 0; fronting rho_im ignored)
 *   r_j  = (kz_j - kz_{j+1}) / (kz_j + kz_{j+1})     interface j = 0..L
 *   r'_j = r_j exp(-2 kz_j kz_{j+1} sigma_{j+1}^2)    (Nevot-Croce roughness)
 *   M = C_0 C_1 ... C_L,  C_j = [[E_j, r'_j E_j], [r'_j/E_j, 1/E_j]],
 *   E_j = exp(i kz_j d_j), E_0 = 1,   R(q) = |M10 / M00|^2      (Abeles)
 *   R_sm(Q) = sum_k w_k R(q_k)   (17-point Gauss-Legendre rule over +-3.5
 *             sigma_Q, sigma_Q = (dQ/Q) Q / (2 sqrt(2 ln 2)), normalised
 *             Gaussian weights; a single node when dQ/Q = 0)
 *   R_hat = scale * R_sm + bkg
 *   logL_b = sum_i [ -1/2 ((R_hat_i - R_obs,i)/e_i)^2 - ln e_i - 1/2 ln 2 pi ]
 *
 * and the gradient of logL_b with respect to every entry of the item's rows
 * and to its scale and background.
 *
 * Layouts (all arrays are caller-owned; "device" means HIP device memory):
 *   Dataset s: points q_off[s] .. q_off[s+1]-1 of the packed arrays q,
 *     r_obs, r_err (Angstrom^-1, absolute reflectivity, its standard error),
 *     resolution dq_over_q[s] (FWHM fraction; 0 = no smearing).
 *   Item b: rows row_off[b] .. row_off[b+1]-1 of `layers` (row-major, 4
 *     doubles per row: [thickness d (A), SLD rho_re (A^-2, absolute), imaginary
 *     SLD rho_im (A^-2), roughness sigma (A) of the interface above the row]);
 *     row 0 = fronting (only rho_re is read), the last row = backing (d is not
 *     read); L = rows - 2 finite layers, 0 <= L <= NR_MAX_DEEP_LAYERS.  The item
 *     reads dataset dataset_of_item[b], scale[b], bkg[b].
 *   Gradient rows are packed exactly like `layers`; entries the model does not
 *     read are written as 0.  Per item g_inst[2b] = d/dscale, g_inst[2b+1] =
 *     d/dbkg.  d/d rho_im uses the one-sided derivative +1 of |x| at 0.
 *
 * Ownership and synchronisation: the library never allocates or frees inside
 * the evaluation calls and never synchronises the stream; every call only
 * enqueues work on `stream` and returns.  Pointers must stay valid until the
 * enqueued work has finished.  A plan holds device copies of the batch
 * structure (offsets, dataset map, work list) and may be used by one stream
 * at a time.
 *
 * Errors: every call returns an nr_status.  Argument errors are detected on
 * the host before anything is enqueued.  Data-dependent faults (non-finite
 * values, Q or a node <= 0, e_i <= 0) cannot be seen without a sync: they set
 * bits in the optional per-item status array and make that item's logL NaN.
 */
#ifndef NR_H_
#define NR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NR_VERSION 2
/* Largest number of finite layers one item may have. */
#define NR_MAX_LAYERS 40
/* Items deeper than NR_MAX_LAYERS (up to NR_MAX_DEEP_LAYERS, e.g. microsliced
 * SLD profiles) are accepted: their value kernels are the same; their gradient
 * uses the parallel-in-layers scan (layer product split across the lanes of
 * one, two or four waves per data point, at most 8 levels per lane), computed
 * in FP64 in both precisions. */
#define NR_MAX_DEEP_LAYERS 2047
/* Number of quadrature nodes per data point when dq_over_q > 0. */
#define NR_SMEAR_NODES 17

typedef int32_t nr_status;
#define NR_OK 0
#define NR_EINVAL 1     /* null pointer, bad count, bad offsets, bad option */
#define NR_EWORKSPACE 2 /* workspace missing or smaller than required */
#define NR_EHIP 3       /* a HIP runtime call or kernel launch failed */
#define NR_ENOMEM 4     /* plan creation could not allocate device memory */
#define NR_ESCRATCH 5   /* nr_loglik_grad_noalloc: the plan needs more workspace than
                         * NR_NOALLOC_SCRATCH_BYTES */

/* Arithmetic precision of the bulk layer product (wavevector roots, interface
 * coefficients, phases, the 2x2 product and its adjoint).  In both, the
 * quadrature nodes, the critical-edge difference kz0^2 - 4 pi (rho_j - rho_0),
 * the smearing sums, chi^2, the likelihood seeds and the per-point gradient
 * accumulation are FP64; NR_F32 rounds that difference to float once and
 * takes the root in float.  Inputs and outputs are FP64 arrays either way. */
#define NR_F64 0
#define NR_F32 1

/* Bits of the optional per-item status array (device int32[n_items]). */
#define NR_ITEM_NONFINITE 1u /* a non-finite R, logL or gradient value */
#define NR_ITEM_BAD_Q 2u     /* a data point or a quadrature node q <= 0 */
#define NR_ITEM_BAD_ERR 4u   /* an error bar e_i <= 0 or non-finite */
#define NR_ITEM_EDGE_SINGULAR 8u /* gradient calls: w_j = kz0^2 - 4 pi (rho_j - rho_0)
                                  * - i 4 pi |rho_im,j| is exactly 0 at some node, where
                                  * dkz/dw is infinite; the item's gradient is finite
                                  * but not meaningful there (logL is unaffected) */

typedef struct nr_plan nr_plan;

/* Batch structure, given as HOST arrays; copied into the plan. */
typedef struct nr_batch_desc {
  int32_t n_datasets;
  const int64_t* q_off;           /* host [n_datasets + 1], q_off[0] = 0, non-decreasing */
  const double* dq_over_q;        /* host [n_datasets], >= 0 and finite */
  int32_t n_items;
  const int32_t* dataset_of_item; /* host [n_items], each in [0, n_datasets) */
  const int64_t* row_off;         /* host [n_items + 1], row_off[0] = 0, 2 <= rows <= NR_MAX_DEEP_LAYERS + 2 */
  int32_t precision;              /* NR_F64 or NR_F32 */
} nr_batch_desc;

/* Values of one evaluation, given as DEVICE pointers. */
typedef struct nr_values {
  const double* q;      /* [q_off[n_datasets]] */
  const double* r_obs;  /* [q_off[n_datasets]] (unused by nr_reflectivity) */
  const double* r_err;  /* [q_off[n_datasets]] (unused by nr_reflectivity) */
  const double* layers; /* [row_off[n_items] * 4] */
  const double* scale;  /* [n_items] */
  const double* bkg;    /* [n_items] */
  int32_t* item_status; /* optional [n_items]; NULL to skip; bits are OR-ed in */
  /* Resolution (Sec. 3 pointwise Gaussian smearing; Sec. 4.1 per-point FWHM;
   * Sec. 4.2 smearing size as a parameter).  Only datasets with
   * dq_over_q > 0 are smeared; for them:
   *   dq        optional [q_off[n_datasets]]: per-point FWHM (A^-1, absolute);
   *             the nodes of point i are Q_i + (dq_i / (2 sqrt(2 ln 2))) t_k;
   *   dqq_item  optional [n_items]: the item's relative FWHM dQ/Q, replacing
   *             the dataset's (used when dq is NULL).
   * NULL for both: (dQ/Q of the dataset) * Q_i. */
  const double* dq;
  const double* dqq_item;
} nr_values;

/* Operation selector for nr_workspace_size. */
#define NR_OP_REFLECTIVITY 0
#define NR_OP_LOGLIK 1
#define NR_OP_LOGLIK_GRAD 2

/* Library version (NR_VERSION). */
int32_t nr_version(void);

/* Human-readable text for a status code, or for NR_EHIP the last HIP error
 * recorded on the calling thread.  Never returns NULL. */
const char* nr_status_string(nr_status status);

/* The resolution quadrature that every smeared evaluation uses (Sec. 3
 * pointwise Gaussian smearing, Sec. 4.1 FWHM): fills HOST t[NR_SMEAR_NODES]
 * with the node offsets in units of sigma_Q (3.5 times the 17-point
 * Gauss-Legendre abscissae on [-1, 1], ascending; the nodes of point Q are
 * Q + sigma_Q t_k, sigma_Q = FWHM / (2 sqrt(2 ln 2))) and w[NR_SMEAR_NODES]
 * with the weights u_k exp(-t_k^2 / 2) normalised to sum 1.  Host only: no
 * device is touched.  NR_EINVAL for NULL. */
nr_status nr_smearing_rule(double* t, double* w);

/* Builds a plan from the host batch description: validates it, builds the
 * work list (one unit = one item x up to 64 consecutive points, ordered by
 * decreasing cost) and uploads it to the current device.  Allocates device
 * memory (owned by the plan; released by nr_plan_destroy).  Synchronous. */
nr_status nr_plan_create(const nr_batch_desc* desc, nr_plan** plan_out);

/* Plan tuning options (nr_plan_create_ex).  None of them changes a result
 * beyond rounding order; they select among equivalent schedules:
 *   grad_variant[k] for layer-count bucket k (nr_bucket_lmax(k) layers):
 *     NR_VARIANT_AUTO       the library's default for the bucket: the store
 *                           form up to 4 layers in NR_F64 and 8 in NR_F32,
 *                           the recompute form deeper (the faster on MI355X);
 *     NR_VARIANT_STORE      forward sweep keeps states, phases and interface
 *                           coefficients for the adjoint (only buckets of at
 *                           most nr_store_max_layers(precision) layers);
 *     NR_VARIANT_RECOMPUTE  the adjoint recomputes wavevectors and interface
 *                           reciprocals (phases and roughness factors of the
 *                           top levels come from an LDS cache).
 *   xcd_run: consecutive work units of the cost-ordered list given to one of
 *     the 8 XCDs (1..64; the default 8 keeps an item's units in one L2).
 *   pack_tails: 1 packs the trailing partial point groups of several items
 *     of equal depth into one wave (default); 0 gives each its own wave.
 *   split_tails (bits): the trailing partial group of an item of at most 10
 *     layers gets a wave of its own when it fills at least 48 of the 64
 *     lanes, which keeps the item's layer records wave-uniform:
 *       NR_TAILS_LONE   by itself (48 points or more);
 *       NR_TAILS_SPLIT  for a smeared item, with the lanes split over 2 to 4
 *                       groups of smearing nodes (lane = node group x point;
 *                       12 to 32 points).
 *     Other tails follow pack_tails.  A third bit serves small problems:
 *       NR_SPLIT_SMALL  when the gradient's full units (64 points each) are
 *                       fewer than one round of the device (two waves per
 *                       SIMD), every point group of a smeared item of at most
 *                       NR_MAX_LAYERS layers is split the same way, over
 *                       G = min(17, round / units) node groups, so that a
 *                       single fit spreads over many waves.
 *     Default: all three bits.
 *   side_stream: 1 (default) runs every second full-unit launch of the
 *     gradient (one launch per layer-count bucket) and its tail and split
 *     launches that hold at most one round of the device (two waves per
 *     SIMD of every compute unit) on a second stream that the plan owns
 *     (default priority, non-blocking), forked from the caller's stream
 *     after the per-layer constants and joined back before the reduction:
 *     small launches run beside the full-unit launches instead of leaving
 *     most of the device idle after them, and consecutive buckets overlap;
 *     0 keeps every launch on the caller's stream.  The fork and join are
 *     event waits, so calls stay ordered on the caller's stream and can be
 *     captured into a HIP graph (the side stream joins the capture).  Calls
 *     on one plan from several host threads are serialised around the fork
 *     and join.
 *   node_groups: the (sample, Q) tiling of the gradient's work units.  0
 *     (default) follows the rules above (64 points per wave, each lane
 *     running all 17 nodes of its point, except the split units); 2..17 puts
 *     every point group of a smeared item of at most NR_MAX_LAYERS layers
 *     into split units of G = node_groups node groups and 64 / G points per
 *     wave (lane = node group x point) whatever the plan's size.  The value
 *     calls are not affected. */
#define NR_TAILS_LONE 1
#define NR_TAILS_SPLIT 2
#define NR_SPLIT_SMALL 4
#define NR_NUM_BUCKETS 16
#define NR_VARIANT_AUTO 0
#define NR_VARIANT_STORE 1
#define NR_VARIANT_RECOMPUTE 2
typedef struct nr_plan_options {
  int32_t grad_variant[NR_NUM_BUCKETS];
  int32_t xcd_run;
  int32_t pack_tails;
  int32_t split_tails;
  int32_t side_stream;
  int32_t node_groups;
} nr_plan_options;

/* Fills *opts with the defaults (all NR_VARIANT_AUTO, xcd_run 8,
 * pack_tails 1, split_tails NR_TAILS_LONE | NR_TAILS_SPLIT | NR_SPLIT_SMALL,
 * side_stream 1, node_groups 0).
 * NR_EINVAL for NULL. */
nr_status nr_plan_options_default(nr_plan_options* opts);

/* Autotuner: chooses plan options for the batch structure *desc by timing
 * nr_loglik_grad on the caller's data `v` (device arrays, as for the
 * evaluation calls) under candidate schedules: per bucket present that has
 * both forms, the store and the recompute form; xcd_run 1, 4, 8, 16, 32;
 * pack_tails, split_tails and side_stream toggled (coordinate search from the defaults,
 * after a 0.3 s warm-up).  A candidate replaces the current one only when its
 * median over `reps` timed calls is at least 3 % lower; a final interleaved
 * comparison keeps the defaults unless the winner holds that margin.  Writes
 * the options to *best and, if ms is not NULL, the median milliseconds of the
 * chosen and of the default schedule to ms[0], ms[1].  Allocates and frees
 * its own plans and device buffers and synchronises `stream` (not for use
 * inside captured work).  The Python module autotune caches its results per
 * structure class. */
nr_status nr_autotune(const nr_batch_desc* desc, const nr_values* v, int32_t reps,
                      nr_plan_options* best, double* ms, void* stream);

/* Largest layer count L of bucket k (0 <= k < NR_NUM_BUCKETS): items with
 * L <= nr_bucket_lmax(k) and L > nr_bucket_lmax(k-1) are evaluated at depth
 * nr_bucket_lmax(k).  Returns -1 for k out of range. */
int32_t nr_bucket_lmax(int32_t k);

/* Deepest bucket (in layers) that NR_VARIANT_STORE supports at `precision`
 * (NR_F64 or NR_F32); -1 for an unknown precision. */
int32_t nr_store_max_layers(int32_t precision);

/* nr_plan_create with options (NULL = defaults).  NR_EINVAL also for an
 * option out of range or NR_VARIANT_STORE on a bucket deeper than
 * nr_store_max_layers(precision). */
nr_status nr_plan_create_ex(const nr_batch_desc* desc, const nr_plan_options* opts,
                            nr_plan** plan_out);

/* Releases a plan and its device memory.  NULL is accepted. */
nr_status nr_plan_destroy(nr_plan* plan);

/* Bytes of caller-provided device workspace that `op` needs for this plan:
 * 80 bytes per row of every item (per-layer constants) plus, for NR_OP_LOGLIK
 * and NR_OP_LOGLIK_GRAD, the per-work-unit partial sums.  Any 8-byte aligned
 * device buffer of at least that size; contents need no initialisation and
 * are overwritten by every call.  Returns NR_EINVAL for an unknown op or a
 * NULL plan. */
nr_status nr_workspace_size(const nr_plan* plan, int32_t op, size_t* bytes);

/* Packed output offsets: R_hat of item b starts at element out_off[b] of the
 * nr_reflectivity output.  Fills host out_off[n_items + 1]. */
nr_status nr_output_offsets(const nr_plan* plan, int64_t* out_off);

/* Model curve (Abeles + smearing + instrument, Sec. 2.1 / Sec. 3): writes
 * R_hat for every point of every item into device r_hat[out_off[n_items]],
 * item-major, in the dataset's point order. */
nr_status nr_reflectivity(const nr_plan* plan, const nr_values* v, double* r_hat,
                          void* workspace, size_t workspace_bytes, void* stream);

/* Gaussian log-likelihood per item (Sec. 2.1, Sec. 4.1 chi^2): writes device
 * logL[n_items]. */
nr_status nr_loglik(const nr_plan* plan, const nr_values* v, double* logL,
                    void* workspace, size_t workspace_bytes, void* stream);

/* logL and its exact gradient (Sec. 2.1 AD figure, Sec. 3 gradient listing),
 * by a hand-written adjoint of the layer product: writes device logL[n_items],
 * g_rows[row_off[n_items] * 4] and g_inst[2 * n_items]. */
nr_status nr_loglik_grad(const nr_plan* plan, const nr_values* v, double* logL,
                         double* g_rows, double* g_inst, void* workspace,
                         size_t workspace_bytes, void* stream);

/* nr_loglik_grad without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving or
 * sampling loops, harnesses that forbid allocation).  The library keeps a
 * fixed scratch array of NR_NOALLOC_SCRATCH_BYTES in device memory, one copy
 * per GPU, reserved when the library is first used on that GPU and held
 * until the process ends; the call uses it in place of the workspace and
 * itself allocates and frees nothing.  Same plan, values, outputs, results
 * and status bits as nr_loglik_grad (the same kernels on the same schedule).
 * The plan's workspace (nr_workspace_size for NR_OP_LOGLIK_GRAD) must fit:
 * otherwise NR_ESCRATCH, before anything is enqueued.  Nothing in the scratch
 * needs to start at zero; it keeps the last call's contents.  Every call on
 * one GPU shares that GPU's scratch, whatever its plan or stream: calls that
 * may overlap on one GPU (other streams, other host threads) race and give
 * wrong results; order them on one stream or use nr_loglik_grad. */
#define NR_NOALLOC_SCRATCH_BYTES (256u << 20)
nr_status nr_loglik_grad_noalloc(const nr_plan* plan, const nr_values* v, double* logL,
                                 double* g_rows, double* g_inst, void* stream);

/* nr_loglik_grad plus the derivative of logL with respect to the relative
 * resolution (Sec. 4.2: the smearing size inferred as a parameter):
 * g_res[b] = dlogL_b / d(dQ/Q)_b (device [n_items]), through the positions
 * of the quadrature nodes q_ik = Q_i (1 + (dQ/Q) t_k / (2 sqrt(2 ln 2))).
 * 0 for items on unsmeared datasets and for all items when values->dq (fixed
 * per-point widths) is given.  Same workspace and status bits. */
nr_status nr_loglik_grad_res(const nr_plan* plan, const nr_values* v, double* logL,
                             double* g_rows, double* g_inst, double* g_res, void* workspace,
                             size_t workspace_bytes, void* stream);

/* Vector-Jacobian product of R_hat (the autograd of nr_reflectivity): for
 * per-point seeds v (device, packed like R_hat, see nr_output_offsets) writes
 * per item b
 *   dot[b]        = sum_i v_i R_hat_i,
 *   g_rows        = sum_i v_i dR_hat_i / d(row entries)  (packed like layers),
 *   g_inst[2b]    = sum_i v_i R_sm_i  (d/dscale),   g_inst[2b+1] = sum_i v_i.
 * The same forward model as nr_reflectivity (Sec. 2.1, Sec. 3); r_obs and
 * r_err are not read.  Uses the NR_OP_LOGLIK_GRAD workspace.  Status bits as
 * for nr_loglik_grad (NONFINITE, BAD_Q, EDGE_SINGULAR). */
nr_status nr_reflectivity_vjp(const nr_plan* plan, const nr_values* values, const double* seed,
                              double* dot, double* g_rows, double* g_inst, void* workspace,
                              size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Integrators and co-fit ties around the gradient.
 * ------------------------------------------------------------------------- */

/* Positions, momenta and gradient of an HMC state (all DEVICE pointers,
 * packed like the rows; instrument pairs [scale, bkg] per item). */
typedef struct nr_hmc_state {
  double* layers;              /* [row_off[n_items] * 4] positions */
  double* scale;               /* [n_items] */
  double* bkg;                 /* [n_items] */
  double* mom_rows;            /* [row_off[n_items] * 4] momenta */
  double* mom_inst;            /* [2 * n_items] momenta of (scale, bkg) */
  const double* inv_mass_rows; /* optional [row_off[n_items] * 4]; NULL = 1 */
  const double* inv_mass_inst; /* optional [2 * n_items]; NULL = 1 */
  double* logL;                /* [n_items] logL at the positions */
  double* g_rows;              /* [row_off[n_items] * 4] gradient of logL */
  double* g_inst;              /* [2 * n_items] */
} nr_hmc_state;

/* n_steps leapfrog steps of Hamiltonian dynamics for every item (Sec. 2.3,
 * leapfrog equations) with potential U = -logL (flat priors) and kinetic
 * energy r^T M^-1 r / 2, M diagonal:
 *   r <- r + (dt/2) g;  theta <- theta + dt M^-1 r;  (logL, g) at theta;
 *   r <- r + (dt/2) g.
 * On entry st->logL, g_rows, g_inst must hold the values at the positions
 * (one nr_loglik_grad call before the first step).  Entries the model does
 * not read are never moved; an inverse mass of 0 freezes an entry.  `data`
 * supplies q, r_obs, r_err and the optional status array (its layers, scale
 * and bkg are ignored).  Uses the NR_OP_LOGLIK_GRAD workspace. */
nr_status nr_leapfrog(const nr_plan* plan, const nr_values* data, const nr_hmc_state* st,
                      double dt, int32_t n_steps, void* workspace, size_t workspace_bytes,
                      void* stream);

/* A captured sequence of launches (HIP graph). */
typedef struct nr_graph nr_graph;

/* Captures nr_leapfrog(plan, data, st, dt, n_steps, ...) into a HIP graph on
 * an internal stream.  Every pointer (including the contents of *data and
 * *st) is baked in and must stay valid until nr_graph_destroy.  Allocates
 * host and device resources for the graph; not graph-capturable itself. */
nr_status nr_leapfrog_graph_create(const nr_plan* plan, const nr_values* data,
                                   const nr_hmc_state* st, double dt, int32_t n_steps,
                                   void* workspace, size_t workspace_bytes, nr_graph** graph_out);

/* Replays a captured graph on `stream`. */
nr_status nr_graph_launch(nr_graph* graph, void* stream);

/* Releases a graph.  NULL is accepted. */
nr_status nr_graph_destroy(nr_graph* graph);

/* ---------------------------------------------------------------------------
 * HMC driver around the leapfrog (Sec. 2.3): per chain, a momentum draw
 * r ~ N(0, M), n_leapfrog leapfrog steps and the Metropolis-Hastings accept
 * alpha = min{1, exp(H(z, r) - H(z', r'))}, in unconstrained coordinates z
 * with potential U(z) = -logL(theta(z)) - sum_p ln|dtheta_p/dz_p| (flat
 * priors) and H = U + r^T M^-1 r / 2, M diagonal.  Each plan item is one
 * chain.  Random numbers come from Philox4x64-10 (Salmon et al., SC'11) with
 * key (seed, 0) and counter (iteration, chain, entry / 4, purpose): Box-Muller
 * normals for the momenta (purpose 0), one uniform for the accept (purpose 1);
 * a 64-bit output x gives ((x >> 11) + 1/2) 2^-53.  Every chain keeps its own
 * iteration counter on the device, so replays of a captured transition draw
 * fresh numbers.
 * ------------------------------------------------------------------------- */

/* Per-entry transform theta(z) (Sec. 2.3: pre-scaling, sampling in log space,
 * hard constraints); a and b are the entry's two constants. */
#define NR_TF_FIXED 0  /* not sampled: theta keeps its value, momentum 0 */
#define NR_TF_AFFINE 1 /* theta = a + b z */
#define NR_TF_LOG 2    /* theta = a + b exp(z), b > 0 */
#define NR_TF_LOGIT 3  /* theta = a + (b - a) / (1 + exp(-z)), a < b */

typedef struct nr_hmc_config {
  int32_t n_leapfrog;      /* leapfrog steps per transition, >= 1 */
  double max_energy_error; /* H' - H above this (or NaN) is divergent: rejected, alpha 0 */
  uint64_t seed;           /* generator key */
  double target_accept;    /* dual-averaging target, in (0, 1) */
} nr_hmc_config;

/* The chains' arrays (all DEVICE pointers).  Entries are packed like the rows
 * (4 per row) and the instrument pairs [scale, bkg] per item.  Entries the
 * model does not read (fronting d, sigma, rho_im; backing d) are never moved,
 * whatever their kind. */
typedef struct nr_hmc_chains {
  double* z_rows;             /* [rows * 4] unconstrained positions (in/out) */
  double* z_inst;             /* [2 * n_items] */
  const uint8_t* kind_rows;   /* [rows * 4] NR_TF_* */
  const uint8_t* kind_inst;   /* [2 * n_items] */
  const double* a_rows;       /* transform constants, same layouts */
  const double* b_rows;
  const double* a_inst;
  const double* b_inst;
  double* inv_mass_rows;      /* diagonal of M^-1 (in; written at a mass window end) */
  double* inv_mass_inst;
  double* step;               /* [n_items] leapfrog step per chain (in; adapted) */
  double* layers;             /* theta: the parameter arrays of nr_values (written on
                                 moving entries; FIXED entries keep the caller's value) */
  double* scale;
  double* bkg;
  double* logL;               /* [n_items] at theta (written) */
  double* g_rows;             /* gradient of logL at theta (written) */
  double* g_inst;
  double* potential;          /* [n_items] U(z) (written) */
  double* accept_prob;        /* [n_items] alpha of the last transition */
  double* energy_error;       /* [n_items] H' - H of the last transition */
  int32_t* n_accept;          /* [n_items] incremented per accepted transition */
  int32_t* n_divergent;       /* [n_items] incremented per divergent transition */
} nr_hmc_chains;

typedef struct nr_hmc nr_hmc;

/* Driver state for the plan's items as chains: momenta, the saved state of a
 * transition, Welford sums and dual-averaging state; iteration counters and
 * adaptation state start at zero.  Allocates device memory (not capturable).
 * The plan must outlive the driver. */
nr_status nr_hmc_create(const nr_plan* plan, const nr_hmc_config* cfg, nr_hmc** out);
nr_status nr_hmc_destroy(nr_hmc* hmc);

/* Evaluates the chains at their positions: theta = theta(z) (with from_theta
 * != 0, z = theta^-1(theta) first), logL and its gradient, U.  Needed before
 * the first transition and after the caller changes z or theta.  `data` gives
 * q, r_obs, r_err (and optional status, resolution); its parameter pointers
 * are ignored.  Uses the NR_OP_LOGLIK_GRAD workspace. */
nr_status nr_hmc_init(nr_hmc* hmc, const nr_values* data, const nr_hmc_chains* ch,
                      int32_t from_theta, void* workspace, size_t workspace_bytes, void* stream);

/* Adaptation during a transition (bits): */
#define NR_HMC_ADAPT_MASS 1 /* push the post-transition z into the Welford window */
#define NR_HMC_ADAPT_STEP 2 /* dual averaging of the step (Hoffman and Gelman 2014,
                               gamma 0.05, t0 10, kappa 0.75) toward target_accept */

/* One transition of every chain.  Same arguments as nr_hmc_init. */
nr_status nr_hmc_transition(nr_hmc* hmc, const nr_values* data, const nr_hmc_chains* ch,
                            int32_t adapt, void* workspace, size_t workspace_bytes,
                            void* stream);

/* Captures n_transitions transitions into a HIP graph (every pointer baked
 * in; see nr_leapfrog_graph_create).  Replays continue the chains. */
nr_status nr_hmc_graph_create(nr_hmc* hmc, const nr_values* data, const nr_hmc_chains* ch,
                              int32_t adapt, int32_t n_transitions, void* workspace,
                              size_t workspace_bytes, nr_graph** graph_out);

/* Warm-up controls between transitions (bits): */
#define NR_HMC_MASS_WINDOW_END 1 /* inverse mass = (n/(n+5)) var + 1e-3 (5/(n+5)) of the
                                    window's positions (n >= 2), window restarts */
#define NR_HMC_STEP_RESTART 2    /* dual averaging restarts at mu = ln(10 step) */
#define NR_HMC_STEP_FINAL 4      /* step = the dual average exp(log eps_bar) */
nr_status nr_hmc_adapt(nr_hmc* hmc, const nr_hmc_chains* ch, int32_t actions, void* stream);

/* ---------------------------------------------------------------------------
 * Full-rank Gaussian variational fit (Sec. 2.4 VI; Sec. 4.2: a multivariate
 * normal surrogate in unconstrained space, Adam, independent restarts, the
 * best ELBO kept).  The plan's items are R restarts x S draws (item r S + s),
 * all with the same number of rows; entry p of a draw is row entry p (4 per
 * row), then scale, bkg (P = 4 rows + 2).  Per restart,
 *   z = mu + L eps, eps ~ N(0, I), theta = theta(z) (the NR_TF_* transforms),
 *   L lower triangular, L_ii = softplus(omega_i), L_ij = lambda_ij (i > j),
 *   ELBO = E[logL(theta(z)) + sum ln|dtheta/dz|] + sum ln L_ii + (n/2) ln(2 pi e)
 * over the n moving entries (transform other than FIXED, read by the model);
 * flat priors.  Draws: Philox4x64-10, counter (iteration, item, entry / 4, 2)
 * (see the HMC driver).  Gradients (h_s = z-gradient of the log target):
 *   dmu_i = mean_s h_si; dlambda_ij = mean_s h_si eps_sj;
 *   domega_i = (mean_s h_si eps_si + 1/L_ii) sigmoid(omega_i).
 * Adam (Kingma and Ba 2015): x += lr mhat / (sqrt(vhat) + eps), ascending.
 * ------------------------------------------------------------------------- */
typedef struct nr_vi_mvn_config {
  int32_t n_restarts; /* R >= 1 */
  int32_t n_draws;    /* S >= 1 draws per restart and step */
  double lr;          /* Adam step (Sec. 4.2: 0.05) */
  double beta1;       /* Adam moment decays and floor (0.9, 0.999, 1e-8) */
  double beta2;
  double adam_eps;
  uint64_t seed;
} nr_vi_mvn_config;

/* Variational parameters and outputs (all DEVICE pointers). */
typedef struct nr_vi_mvn_params {
  const uint8_t* kind;        /* [P] NR_TF_* per entry, shared by the restarts */
  const double* a;            /* [P] transform constants */
  const double* b;            /* [P] */
  const double* theta_fixed;  /* [P] theta of the entries that do not move */
  double* mu;                 /* [R * P] */
  double* omega;              /* [R * P] */
  double* lam;                /* [R * P * P] row-major; row i, columns j < i are lambda_ij */
  double* elbo;               /* [R] estimate at the step's draws (written) */
  double* grad_mu;            /* [R * P] (written; 0 on entries that do not move) */
  double* grad_omega;         /* [R * P] */
  double* grad_lam;           /* [R * P * P] (written; 0 outside j < i) */
} nr_vi_mvn_params;

typedef struct nr_vi_mvn nr_vi_mvn;

/* Driver state for the plan (R x S items, equal rows): the draws, the draws'
 * parameters, logL and gradient, and the Adam moments (zero), iteration 0.
 * Allocates device memory (not capturable).  The plan must outlive it. */
nr_status nr_vi_mvn_create(const nr_plan* plan, const nr_vi_mvn_config* cfg, nr_vi_mvn** out);
nr_status nr_vi_mvn_destroy(nr_vi_mvn* vi);

/* One step: draws for the current iteration, the ELBO estimate and its
 * gradient per restart; with adam != 0, one Adam step of mu, omega and lambda
 * on moving entries.  The iteration advances.  `data` gives q, r_obs, r_err
 * (its parameter pointers are ignored).  Uses the NR_OP_LOGLIK_GRAD
 * workspace. */
nr_status nr_vi_mvn_step(nr_vi_mvn* vi, const nr_values* data, const nr_vi_mvn_params* prm,
                         int32_t adam, void* workspace, size_t workspace_bytes, void* stream);

/* Captures n_steps steps (with Adam) into a HIP graph; replays continue. */
nr_status nr_vi_mvn_graph_create(nr_vi_mvn* vi, const nr_values* data,
                                 const nr_vi_mvn_params* prm, int32_t n_steps, void* workspace,
                                 size_t workspace_bytes, nr_graph** graph_out);

/* Reparameterised Monte-Carlo gradient of the evidence lower bound for a
 * mean-field Gaussian q (Sec. 2.4, Monte-Carlo estimate of the loss and of its
 * gradient; reparameterisation theta = mu + s(omega) eps with
 * s = softplus).  The plan's items are the S samples; each must have the
 * same number of rows `rows`.  P = rows * 4 + 2 entries per sample: the rows
 * of one stack, then scale, bkg.  On variational entries (mask != 0)
 * theta_i = mu + s eps_i, elsewhere theta_i = mu.  Outputs (device):
 *   logL[i], g_rows, g_inst per sample (as nr_loglik_grad);
 *   grad_mu[p] = mean_i g_ip, grad_omega[p] = mean_i g_ip eps_ip s'(omega_p)
 *   + s'(omega_p)/s(omega_p) (0 outside the mask), the gradient of
 *   ELBO = mean_i logL_i + sum_p ln s(omega_p) (+ const), whose estimate is
 *   written to elbo[0].  Flat priors.  Uses the NR_OP_LOGLIK_GRAD workspace. */
typedef struct nr_vi_args {
  const double* mu;     /* [P] */
  const double* omega;  /* [P] */
  const uint8_t* mask;  /* [P] */
  const double* eps;    /* [S * P] standard normal draws (caller's RNG) */
  double* layers;       /* [S * rows * 4] sample positions (written) */
  double* scale;        /* [S] */
  double* bkg;          /* [S] */
  double* logL;         /* [S] */
  double* g_rows;       /* [S * rows * 4] */
  double* g_inst;       /* [2 * S] */
  double* grad_mu;      /* [P] */
  double* grad_omega;   /* [P] */
  double* elbo;         /* [1] */
} nr_vi_args;
nr_status nr_vi_elbo_grad(const nr_plan* plan, const nr_values* data, const nr_vi_args* vi,
                          void* workspace, size_t workspace_bytes, void* stream);

/* Deterministic gather-sum for parameters shared between co-fitted items
 * (Sec. 4.2: instrument and substrate parameters shared across devices):
 *   out[k] = sum of in[src[t]] for t = first[k] .. first[k+1]-1, in order.
 * All arrays on the device; first has n_out + 1 entries. */
nr_status nr_tie_sum(int64_t n_out, const int64_t* first, const int64_t* src, const double* in,
                     double* out, void* stream);

/* Optional timing hooks for profiling: while set, every evaluation call
 * records `start` (a hipEvent_t owned by the caller) on its stream just
 * before its first layer-product kernel and `stop` just after its last one,
 * so that the events bracket the dominant kernels and exclude the per-item
 * reduction.  Pass NULL for both to disable.  Never synchronises. */
nr_status nr_plan_set_timing_events(nr_plan* plan, void* start, void* stop);

#ifdef __cplusplus
}
#endif

#endif /* NR_H_ */
