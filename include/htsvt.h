/*
 * htsvt.h -- C ABI of the MI355X randomized high-order t-SVT library.
 *
 * The library computes, on one GPU, the randomized approximation of the
 * GNHTSVT operator D_{Phi,tau}(A, L) (Def. 4.3 of the paper; the operator that
 * solves  argmin_G tau*||G||_{Phi,L} + ||G - A||_F^2 / 2, Thm. 4.1) for an
 * order-d real tensor under invertible transforms L along modes 3..d
 * (eq. defining L and its inverse), and the per-iteration update of the pure
 * low-rank-prior ADMM solvers for completion and robust completion that call
 * it once per iteration (Sec. V, ADMM updates of L, E, the multiplier and mu).
 *
 * Conventions
 *  - Tensors are dense, real, stored in Fortran order: element (i1,...,id)
 *    (0-based) lives at i1 + n1*(i2 + n2*(i3 + ...)).  Face slice j
 *    (j = i3 + n3*(i4 + ...), the slice index of Sec. II) is therefore the
 *    contiguous column-major n1 x n2 block starting at j*n1*n2.
 *  - All tensor arguments are DEVICE pointers owned by the caller.  The library
 *    never frees them and never keeps them past the call.
 *  - Work is enqueued on the caller's stream (hipStream_t passed as void*;
 *    NULL = the null stream).  Calls return after enqueueing; they do not
 *    synchronize unless stated.  Calls on one plan must not overlap in time
 *    on different host threads.
 *  - Scratch memory is a caller-provided device workspace of at least the
 *    size reported by the matching *_workspace_size call; the library does not
 *    allocate per call.  Plans own small device tables (transform matrices).
 *  - Return value: HT_OK (0) or a negative HT_ERR_* code.  A human-readable
 *    message for the last failure on the calling thread is available from
 *    ht_last_error().  No exception crosses the ABI.
 *  - Numerical breakdowns inside the method (rank-deficient sketches handled
 *    by deflation) are not errors.
 */
#ifndef HTSVT_H
#define HTSVT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HT_MAX_ORDER 8
#define HT_MAX_WIDTH 76    /* largest sketch width l = min(r + p, n1, n2) */
#define HT_MAX_MODE 64     /* largest n_k of a transformed mode */

enum {
  HT_OK = 0,
  HT_ERR_INVALID_ARG = -1,
  HT_ERR_UNSUPPORTED = -2,
  HT_ERR_NONFINITE = -3,
  HT_ERR_WORKSPACE = -4,
  HT_ERR_HIP = -5,
  HT_ERR_ALLOC = -6
};

/* Transform of one mode k = 3..d (the matrices U_{n_k} of the transform L). */
enum {
  HT_DCT2_ORTHO = 0,      /* orthonormal DCT-II, alpha = 1 */
  HT_DFT_UNITARY = 1,     /* unitary DFT F[k][m] = exp(-2 pi i k m / n) / sqrt(n), alpha = 1 */
  HT_CUSTOM_REAL = 2,     /* caller-supplied real U with U U^T = alpha I */
  HT_DFT_UNNORMALIZED = 3 /* plain DFT F[k][m] = exp(-2 pi i k m / n), alpha = n (the FFT of
                             the experiments, Sec. VI); the inverse is F^H / n.  The threshold
                             tau applies unscaled to the transform-domain singular values.
                             The two DFT kinds may be mixed across modes, but a DFT kind must
                             be the transform of every mode 3..d (complex slices; see
                             ht_plan_desc) */
};

/* Arithmetic of the path. */
enum {
  HT_FP64 = 0,        /* tensors double; every step FP64 */
  HT_FP32 = 1,        /* tensors float; sketches/transforms FP32, Gram/Cholesky/eigen FP64 */
  HT_BF16_MIXED = 2   /* tensors float; transformed slices, Omega and Q in BF16 on MFMA
                         with FP32 accumulation; Gram/Cholesky/eigen FP64 */
};

/* Penalty Phi of the low-rank term or psi of the sparse term (the family of the
 * Assumption on Phi, Sec. IV-A).  Every penalty is normalized to slope 1 at 0
 * except LOG; parameters are absolute except FIRM's ratio:
 *   L1         phi(x) = x
 *   MCP        phi(x) = x - x^2/(2 p0) (x <= p0), p0/2 beyond          (p0 = gamma > 0)
 *   SCAD       phi(x) = x (x <= p1), (2 p0 p1 x - x^2 - p1^2)/(2 (p0-1) p1) (x <= p0 p1),
 *              (p0+1) p1 / 2 beyond                                   (p0 = a > 2, p1 = b > 0)
 *   LOG        phi(x) = log(1 + x / p0)                                (p0 = eps > 0)
 *   CAPPED_L1  phi(x) = min(x, p0)                                     (p0 = theta > 0)
 *   FIRM       firm shrinkage (Gao-Bruce) with thresholds (mu, a mu):    (p0 = a > 1)
 *              Prox(v) = 0 (v <= mu), a (v - mu)/(a - 1) (v <= a mu), v beyond; the
 *              proximity operator of MCP with gamma = a mu at the same mu
 * Prox_{phi,mu}(v) = argmin_x mu*phi(x) + (x - v)^2/2 (the proximity operator of
 * Sec. IV-B); ties between two global minimizers resolve to the smaller |x|. */
enum { HT_PEN_L1 = 0, HT_PEN_MCP = 1, HT_PEN_SCAD = 2, HT_PEN_LOG = 3, HT_PEN_CAPPED_L1 = 4, HT_PEN_FIRM = 5 };

typedef struct {
  int kind;
  double p0, p1;
} ht_penalty;

/* Problem description for one tensor.
 *  order       d, 2 <= d <= HT_MAX_ORDER (d = 2: one slice, no transform)
 *  dims[k]     n_{k+1} >= 1
 *  transform[k] for k = 2..d-1: transform kind of mode k+1
 *  custom[k]   HOST pointer to the n x n row-major matrix U (CUSTOM_REAL only;
 *              copied at plan creation)
 *  r, p, q     target rank r >= 1, oversampling p >= 0, power steps q >= 0;
 *              sketch width l = min(r + p, n1, n2) <= HT_MAX_WIDTH, kept k = min(r, l)
 *  precision   HT_FP64 / HT_FP32 / HT_BF16_MIXED
 *  DFT         with a DFT kind (HT_DFT_UNITARY or HT_DFT_UNNORMALIZED) on every
 *              mode 3..d the transformed slices are complex; for real X slice
 *              partner(j) (every transform-domain index negated modulo n_k) is
 *              the conjugate of slice j, so only the canonical member of each
 *              pair (the smaller index) is sketched, with the real Gaussian
 *              Omega (n2 x l) keyed by that index, and the partner's result is
 *              its conjugate (the output is real).  Every product is the
 *              complex one (conjugate transposes where the method transposes);
 *              CholeskyQR and the small SVD run in complex FP64.  Complex slices
 *              need l <= 64.  n_slices, width and kept (ht_plan_info) count
 *              canonical slices and complex columns.  Mixing DFT and real kinds
 *              is UNSUPPORTED, as are ht_transform, ht_omega_fp64 and learned
 *              widths on such plans.
 *  seed, stream_id  key of the Gaussian sketch generator (Philox4x32-10,
 *              counter (group, slice, call, stream_id), key = seed) */
typedef struct {
  int order;
  int64_t dims[HT_MAX_ORDER];
  int transform[HT_MAX_ORDER];
  const double* custom[HT_MAX_ORDER];
  int r, p, q;
  int precision;
  uint64_t seed;
  uint32_t stream_id;
} ht_plan_desc;

typedef struct ht_plan ht_plan;

/* Library version as 10000*major + 100*minor + patch. */
int ht_version(void);

/* Message describing the last failure on the calling thread ("" if none).
 * The pointer stays valid until the next failing call on this thread. */
const char* ht_last_error(void);

/* Create a plan on the current HIP device.  Validates the description and
 * uploads the transform tables.  Errors: INVALID_ARG (bad sizes/ranks/kinds),
 * UNSUPPORTED (a valid request this build does not implement), HIP, ALLOC.
 * The plan is the library's device context: it records the device that was
 * current at creation and owns the tables there; every later call on the plan
 * must run with that device current (INVALID_ARG otherwise). */
int ht_plan_create(const ht_plan_desc* desc, ht_plan** out);
int ht_plan_destroy(ht_plan* plan);

/* HIP device ordinal the plan was created on. */
int ht_plan_device(const ht_plan* plan, int* device);

/* Non-finite detection.  Every t-SVT call records, per slice, whether the FP64
 * Gram matrices of its sketch held a NaN or an infinity (any non-finite entry
 * of the transformed slice reaches them).  This call waits for the stream, and
 * returns HT_ERR_NONFINITE when some slice of the last call on this workspace
 * was flagged (n_bad, optional: how many), HT_OK otherwise. */
int ht_plan_status(const ht_plan* plan, const void* workspace, void* stream, int64_t* n_bad);

/* Bytes of device workspace needed by ht_gnhtsvt on this plan. */
int ht_plan_workspace_size(const ht_plan* plan, size_t* bytes);

/* Number of sketched face slices (P = n3*...*nd, or the number of conjugate
 * pairs and self-conjugate slices under the DFT), the largest sketch width
 * and kept count of the plan. */
int ht_plan_info(const ht_plan* plan, int64_t* n_slices, int* width, int* kept);

/* Offset and size in bytes of a named region of the workspace, for
 * inspecting intermediate results after a call: 0 transformed tensor A,
 * 1 sketch matrices Omega (left unwritten by FP32 plans whose slices are all
 * real with n1 >= 192, n1 a multiple of 4, n2 <= 512 and l <= 64: there the
 * first product draws Omega in place; and by BF16-mixed plans with complex
 * slices, which write only region 24),
 * 2 basis Q1 of the last CholeskyQR pass (n1 x l per
 * slice; the final R2 correction is applied in the l x l space),
 * 3 B^T = A^T Q1 (n2 x l per slice), 4 K' = R2^{-1} U diag(w) U^T R2^{-T}
 * (l x l per slice), 5 Q1 K', 6 reconstructed transformed slices C,
 * 7-9 solver buffers, 10-11 FP64 Gram partials, 12 per-slice widths of the
 * first sketch pass (int pairs l, k), 13 the call index of a replayed graph,
 * learned widths: 14 widths of the redo pass, 15 widths used (l, k),
 * 16 singular values (P x l_max doubles), 17 kept counts (P ints),
 * 18 ||A_j||^2 (previous, current; P x 2 doubles), 19 features (P x 32
 * floats), 20 state (ints: history valid, predicted slices, redone slices),
 * 21 non-finite flags (P ints), 22 RSE partial sums, 23 squared group norms
 * of the tube-wise / slice-wise solver update, and, for BF16-mixed plans
 * with complex slices only (zero bytes otherwise), BF16 copies of the thin
 * operands of the complex products: 24 Omega, 25 the latest left basis Q,
 * 26 the latest right basis (n2 x l per slice).  Thin blocks of slice j start at
 * j * align4(rows * l) elements (align4 rounds up to a multiple of 4).  A
 * complex slice keeps its real and imaginary parts stacked: A and C blocks of
 * 2 n1 x n2, thin blocks of 2 rows x l, K' of 2 l x l (column-major). */
int ht_plan_workspace_region(const ht_plan* plan, int region, size_t* offset, size_t* bytes);

/* Randomized GNHTSVT (Def. 4.3 computed slice-wise on sketches):
 *   out = L^{-1}( slice-wise  Q_j U_k diag(Prox_{Phi,tau}(s_k)) V_k^T )
 * where for each transformed slice A_j = L(X)^<j>:
 *   Y = A_j Omega_j,  Q = orth(Y),  q times { Z = orth(A_j^T Q), Q = orth(A_j Z) },
 *   B = Q^T A_j = U diag(s) V^T,  k = min(r, l).
 * X, out: device tensors of the plan's storage type (double for FP64, float
 * otherwise), N = n1*...*nd elements, may alias.  tau >= 0.  call_index keys the
 * sketch draw (a solver passes its iteration number).  workspace: device buffer
 * of >= ht_plan_workspace_size bytes, 256-byte aligned.
 * stats (optional, device pointers, may be NULL):
 *   sigma_out  P*l doubles, the l singular values of B_j (descending)
 *   kept_out   P ints, how many shrunk values are nonzero
 * Errors: INVALID_ARG (null pointers, tau < 0 or not finite, bad penalty
 * parameters), WORKSPACE (too small or misaligned), HIP. */
int ht_gnhtsvt(ht_plan* plan, const void* X, void* out, double tau, const ht_penalty* penalty,
               uint32_t call_index, void* workspace, size_t workspace_bytes, void* stream,
               double* sigma_out, int* kept_out);

/* Write the FP64 sketch matrices of one call for every slice to dev_out
 * (P * n2 * l doubles, slice-major, each column-major n2 x l), exactly as the
 * t-SVT draws them before rounding to the storage type.  For checking the
 * generator against an independent implementation. */
int ht_omega_fp64(const ht_plan* plan, uint32_t call_index, double* dev_out, void* stream);

/* Forward (inverse != 0: inverse) transform of a whole tensor, out-of-place
 * or in place, in the plan's storage type. */
int ht_transform(const ht_plan* plan, const void* X, void* out, int inverse, void* stream);

/* ---------------------------------------------------------------------------
 * Batches of tensors of different shapes.  Every tensor of a batch is a
 * separate problem (its own transforms, r and p, threshold tau_t); they share
 * q, the precision and the sketch key (seed; the Philox stream word of tensor
 * t is stream_id + t, its slice words are its own slice indices).  Each stage
 * of the method is one launch over every slice of every tensor.
 * The tensors live in one packed device buffer of packed_numel elements:
 * tensor t at element offset offset_t (a multiple of 64), in Fortran order;
 * gaps between tensors are ignored on input and left untouched on output.
 * --------------------------------------------------------------------------- */

/* Create a plan over n_tensors descriptions (q, precision, seed and stream_id
 * must agree).  Errors as ht_plan_create. */
int ht_batch_plan_create(int n_tensors, const ht_plan_desc* descs, ht_plan** out);

/* Packed buffer size (elements) and tensor count of any plan (a single-tensor
 * plan is a batch of one at offset 0). */
int ht_batch_info(const ht_plan* plan, int64_t* packed_numel, int* n_tensors);

/* Offset and size (elements) of tensor t in the packed buffer, its first
 * slice in the plan's slice order, its sketch width l and kept count k. */
int ht_batch_tensor_info(const ht_plan* plan, int t, int64_t* offset, int64_t* numel, int64_t* first_slice,
                         int* width, int* kept);

/* Randomized GNHTSVT of every tensor of a batch plan with threshold
 * tau_dev[t] (DEVICE array of n_tensors doubles, read when the call runs).
 * X, out: packed device buffers; sigma_out (P_total * l_max doubles, rows of
 * l_max with zeros past a slice's own width) and kept_out (P_total ints) are
 * optional, slice order as ht_batch_tensor_info.  Errors as ht_gnhtsvt. */
int ht_batch_gnhtsvt(ht_plan* plan, const void* X, void* out, const double* tau_dev, const ht_penalty* penalty,
                     uint32_t call_index, void* workspace, size_t workspace_bytes, void* stream,
                     double* sigma_out, int* kept_out);

/* Tile choices of a plan: output rows per workgroup of the sketch products
 * (64 or 128; FP64 always 64) and the LDS budget of one transform tile (32, 64
 * or 128 KiB; a budget that does not hold the tensor's face slices fails with
 * UNSUPPORTED).  0 keeps the current value.  Results do not depend on the
 * choice beyond rounding order. */
int ht_plan_set_tuning(ht_plan* plan, int prod_rows, int transform_lds_kib);
int ht_plan_get_tuning(const ht_plan* plan, int* prod_rows, int* transform_lds_kib);

/* Autotuner: times whole t-SVT calls on X (L1, tau = 0; out is overwritten)
 * for every tile choice, one knob at a time (product rows, then transform
 * budget), `repeats` timed calls each after one warm-up, keeps the fastest and
 * reports its milliseconds per call.  Synchronizes the stream. */
int ht_plan_autotune(ht_plan* plan, const void* X, void* out, void* workspace, size_t workspace_bytes,
                     void* stream, int repeats, double* best_ms);

/* Graph replay (on != 0): the next t-SVT call on the plan records its launch
 * sequence as a HIP graph (stream capture); later calls with the same X, out,
 * workspace, stream, tau (or tau_dev), penalty and stats pointers launch the
 * recorded graph, whose first node writes the call index into the workspace.
 * Any other argument set records a new graph.  Per-stage profiling bypasses
 * the graph.  The stream must be a created stream (INVALID_ARG for the null
 * stream, which cannot be captured).  on = 0 drops the graph. */
int ht_plan_graph_enable(ht_plan* plan, int on);

/* ---------------------------------------------------------------------------
 * Learned sketch widths.  A small MLP (32 inputs, two ReLU layers of 128, one
 * output; FP32) predicts from the previous call's statistics of a slice how
 * many of its singular values survive the shrinkage.  Features of slice j
 * (from the previous call on the same workspace, and the current tau):
 *   0-15  sigma_i / sigma_1, i = 1..16 (0 past the width or when sigma_1 = 0)
 *   16    log10(||A_j||^2 + 1e-30) / 10           17  (||A_j||^2 - ||B_j||^2) / ||A_j||^2 in [0, 1]
 *   18    tau / sigma_1 in [0, 10] (10 if sigma_1 = 0)
 *   19    fraction of the sigma above tau         20  kept / width
 *   21-24 log(sigma_k / sigma_{k+1}), k = 2, 4, 8, 16, in [0, 10] (10 when only
 *         sigma_{k+1} is 0, 0 when both are or k >= width)
 *   25    log10(1 / tau) / 10 (1 if tau = 0)      26  min(call index, 200) / 100
 *   27    log(n1 / n2)    28 log2(min(n1, n2)) / 10    29 width / 64
 *   30    (number of sigma above tau) / 64        31  0
 * With z the network output, s = exp(z) - 1, the slice is sketched with
 * l = clamp(ceil(s) + p, p + 1, l_fix) columns and keeps k = min(k_fix, l)
 * values (l_fix, k_fix: the plan's fixed width and kept count).  It is redone at
 * the fixed width when l < l_fix and either every kept value survived
 * (kept >= k) or ||A_j||^2 - ||B_j||^2 > (min(n1, n2) - l) t0^2, where t0 =
 * sup{v : Prox_{Phi,tau}(v) = 0} is the penalty's zero threshold (tau for L1,
 * FIRM and MCP with gamma > tau; sqrt(gamma tau) for MCP with gamma <= tau;
 * min(tau, sqrt(2 tau theta)) for capped-L1; by bisection on the prox for SCAD
 * and LOG): the residual then certainly holds a value that would survive.  The
 * fixed-width method stays the fallback.  The first call after a reset uses the
 * fixed widths.
 *
 * Parameters: one flat FP32 device vector of ht_mlp_param_count() entries,
 * W1 (128 x 32, row-major), b1 (128), W2 (128 x 128), b2 (128), W3 (128), b3.
 * --------------------------------------------------------------------------- */

/* mode 0: fixed widths (default).  mode 1: fixed widths, statistics and
 * features recorded in the workspace (for collecting training traces).
 * mode 2: predicted widths with the network theta (device, caller-owned,
 * read when each call runs).  Applies to ht_gnhtsvt, ht_batch_gnhtsvt and the
 * solver iterations on this plan. */
int ht_plan_learned(ht_plan* plan, int mode, const float* theta);

/* Forget the previous call's statistics and clear the counters (ht_admm_init
 * does this too). */
int ht_plan_learned_reset(const ht_plan* plan, void* workspace, size_t workspace_bytes, void* stream);

/* Read (synchronizing the stream) whether statistics are recorded, and the
 * cumulative numbers of slices sketched at a predicted width and of those
 * redone at the fixed width since the last reset. */
int ht_plan_learned_counts(const ht_plan* plan, const void* workspace, void* stream, int* valid, int* predicted,
                           int* redone);

/* Test hook: redo every slice sketched at a predicted width (the output is then
 * the fixed-width method's). */
int ht_plan_force_fallback(ht_plan* plan, int on);

/* Number of network parameters, and device workspace bytes for a gradient or
 * training step over n samples. */
int ht_mlp_param_count(void);
int ht_mlp_workspace_size(int n, size_t* bytes);

/* z[i] = network(X[i, :]) for n samples (X: n x 32 row-major, device). */
int ht_mlp_forward(const float* theta, const float* X, float* z, int n, void* stream);

/* Gradient of the mean squared error (1/n) sum_i (z_i - y_i)^2 with respect to
 * theta (grad: device, ht_mlp_param_count() floats) and the loss (device
 * float, may be NULL).  Deterministic: partial sums in a fixed order. */
int ht_mlp_grad(const float* theta, const float* X, const float* y, int n, float* grad, float* loss,
                void* workspace, size_t workspace_bytes, void* stream);

/* One Adam step (bias-corrected; step counts from 1) on theta with moment
 * vectors m, v (device, zero before the first step) from the gradient of the
 * mean squared error over the n samples; loss (device, may be NULL) receives
 * the loss before the step. */
int ht_mlp_train_step(float* theta, float* m, float* v, int step, const float* X, const float* y, int n,
                      float lr, float beta1, float beta2, float eps, float* loss, void* workspace,
                      size_t workspace_bytes, void* stream);

/* Per-stage timing: when enabled, every kernel launch of the plan is bracketed
 * by HIP events recorded on the launch stream.  ht_profile_read waits for the
 * recorded events, returns the summed milliseconds and launch counts per stage
 * (0 forward transform, 1 sketch generator, 2 Y = A W, 3 CholeskyQR,
 * 4 Z = A^T Q, 5 small SVD + shrink, 6 Q K, 7 C = (Q K) B, 8 inverse transform,
 * 9 ADMM update) for the first n_stages stages, and clears the records. */
int ht_profile_enable(ht_plan* plan, int on);
int ht_profile_read(ht_plan* plan, double* ms_total, int* count, int n_stages);

/* ---------------------------------------------------------------------------
 * Pure-L ADMM for completion (model = HT_COMPLETION) and robust completion
 * (model = HT_RPCA, HT_RPCA_TUBE, HT_RPCA_SLICE), one iteration per call:
 *   L   <- D_{Phi, 1/mu}(M - E + Y/mu)            (randomized t-SVT above)
 *   H   <- M - L + Y/mu
 *   E   <- off the mask: H;  on the mask: COMPLETION 0, or the GNHTT of
 *          P_mask(H) with Prox_{psi, lambda/mu} (Sec. IV-B):
 *            RPCA        element-wise  Prox(H_i)
 *            RPCA_TUBE   tube-wise     H_t / ||H_t|| Prox(||H_t||) for every tube
 *                        t = (i1, i2) of P_mask(H) (the entries over modes 3..d)
 *            RPCA_SLICE  slice-wise    H^<j> / ||H^<j>|| Prox(||H^<j>||) for
 *                        every face slice j of P_mask(H)
 *          (a group of norm 0 stays 0; group norms summed in FP64)
 *   Y   <- Y + mu (M - L - E)
 *   mu  <- min(mu_max, vartheta * mu)
 * and the stopping terms max|dL|, max|dE|, max|M - L - E| of the iteration.
 * --------------------------------------------------------------------------- */
enum { HT_COMPLETION = 0, HT_RPCA = 1, HT_RPCA_TUBE = 2, HT_RPCA_SLICE = 3 };

typedef struct {
  int model;
  ht_penalty phi;       /* low-rank penalty */
  ht_penalty psi;       /* sparse penalty (robust models only) */
  double lambda;        /* weight of the sparse term (robust models only) */
  double mu0, vartheta, mu_max;
} ht_admm_params;

typedef struct {
  int32_t iteration;    /* iterations completed */
  double mu;            /* mu for the next iteration */
  double dL, dE, resid; /* stopping terms of the last iteration (inf-norms; NaN propagates) */
  double rse;           /* ||L - L*||_F / ||L*||_F after the last ht_admm_iterate call
                           against the registered ground truth L* (NaN if none) */
} ht_admm_stats;

/* Workspace for the ADMM calls (includes the t-SVT workspace). */
int ht_admm_workspace_size(const ht_plan* plan, size_t* bytes);

/* Zero L, E, Y and set mu = mu0, iteration = 0 (state kept in the workspace). */
int ht_admm_init(ht_plan* plan, const ht_admm_params* prm, void* L, void* E, void* Y,
                 void* workspace, size_t workspace_bytes, void* stream);

/* Run n_iter iterations.  M: observed tensor (zero off the mask), mask: N
 * bytes (nonzero = observed).  L, E, Y: solver state in the storage type.
 * The sketch draw of iteration t uses call_index t. */
int ht_admm_iterate(ht_plan* plan, const ht_admm_params* prm, const void* M, const uint8_t* mask,
                    void* L, void* E, void* Y, int n_iter, void* workspace, size_t workspace_bytes,
                    void* stream);

/* Register a ground truth L* (device, storage type, N elements, caller-owned;
 * NULL clears it): every later ht_admm_iterate call ends with the relative
 * recovery error ||L - L*||_F / ||L*||_F (the RSE of the experiments), summed in
 * FP64 in a fixed order, into the solver state. */
int ht_admm_set_truth(ht_plan* plan, const void* truth);

/* Copy the solver scalars to the host (synchronizes the stream).  Returns
 * HT_ERR_NONFINITE (with *out filled) when a stopping term is NaN or infinite
 * or a slice of the last t-SVT was flagged non-finite. */
int ht_admm_get_stats(const ht_plan* plan, const void* workspace, void* stream, ht_admm_stats* out);

/* ---------------------------------------------------------------------------
 * Allocation-free t-SVT, for callers that cannot allocate device memory while
 * they run (code under HIP stream capture, serving loops, harnesses that forbid
 * hipMalloc).  Same operation, arguments and results as ht_gnhtsvt, but the
 * workspace is a device array held by the library: one copy of
 * HT_NOALLOC_SCRATCH_BYTES bytes on every device the library runs on, kept
 * until the process ends.  The call allocates nothing (no hipMalloc, hipFree,
 * events or graphs); its first call on a device looks up that device's copy.
 * Every call on one device shares its copy, which keeps the last call's
 * contents; no part of it needs to start at zero.  Calls that overlap in time
 * on one device (two streams, two threads) race on it and must not be issued.
 * Errors: as ht_gnhtsvt; WORKSPACE when ht_plan_workspace_size of the plan is
 * above HT_NOALLOC_SCRATCH_BYTES; UNSUPPORTED for batch plans and for plans
 * with learned widths, graph replay or per-stage profiling enabled (their
 * state lives in a caller's workspace or allocates).
 * --------------------------------------------------------------------------- */
#define HT_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

int ht_gnhtsvt_noalloc(ht_plan* plan, const void* X, void* out, double tau, const ht_penalty* penalty,
                       uint32_t call_index, void* stream, double* sigma_out, int* kept_out);

#ifdef __cplusplus
}
#endif

#endif /* HTSVT_H */
