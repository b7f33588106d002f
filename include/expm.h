/*
 * expm.h -- C ABI of the MI355X (gfx950) matrix-exponential library.
 *
 * Method (Bader, Blanes, Casas, "An improved algorithm to compute the exponential of a
 * matrix"): scaling and squaring, e^A = (T_m(A / 2^s))^(2^s) (Sec. 1, eq. eses), where the
 * degree-m Taylor polynomial T_m (Sec. 3, eq. tay.exp) is evaluated with the paper's
 * product-reduced sequences -- T_8 with 3 products (eq. Algorithm83eA), T_12 with 4 (eq. poly12),
 * T_18 with 5 (eq. poly.18); T_1, T_2, T_4 with 0, 1, 2 -- and (m, s) is chosen so that the
 * relative backward error stays below the accuracy u (eq. eq.theta; thresholds theta_m of
 * Table 2; product counts of Table 3).
 *
 * Conventions shared by every entry point
 *  - Matrices are n x n, row-major, contiguous (element (i, j) at i*n + j).  Complex matrices
 *    (EXPM_C128) are interleaved (re, im) pairs of doubles.
 *  - Pointers named *_dev are device (HBM) pointers; the caller owns every buffer.  The
 *    library allocates no device memory: scratch space is the caller's workspace, sized by
 *    expm_workspace_bytes() (expm_batched_noalloc uses a fixed device array of the library
 *    instead).  The output must not alias the input.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue work and return;
 *    results, (m, s) and per-matrix status are written to device memory, so nothing is known
 *    on the host until the caller synchronises.  Exception: see expm_taylor for n > 256.
 *  - Return value: EXPM_OK, or an error code for an argument the host can check (null
 *    pointer, n <= 0, n above the supported maximum, unknown enum, workspace too small, u
 *    outside [2^-53, 2^-10]) or a HIP launch failure.  Nothing is launched when an argument
 *    error is returned.  No C++ exception crosses this boundary.
 *  - Per-matrix status (device): EXPM_OK, or EXPM_E_NONFINITE when the input holds a NaN or
 *    an infinity or its 1-norm overflows the double range; then (m, s) = (-1, -1) and the
 *    output is filled with NaN.
 *  - The scaling X = 2^-s A (eq. eses) is applied to the matrix when it is loaded (exactly,
 *    a power of two), before any power is formed, so no intermediate overflows whatever
 *    ||A||_1 is; entries of X that fall below the normal range lose bits (as they would in any
 *    evaluation of 2^-s A).  The global-memory kernel (real orders 144..256) instead puts
 *    2^-ks into the coefficient of A^k (the same exact result) while ||A||_1 <= 2^150, where no
 *    power it forms can overflow, and scales at load above that.
 */
#ifndef EXPM_H_
#define EXPM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define EXPM_API __attribute__((visibility("default")))
#else
#define EXPM_API
#endif

typedef enum {
  EXPM_OK = 0,
  EXPM_E_INVALID_ARG = 1,
  EXPM_E_NONFINITE = 2,
  EXPM_E_WORKSPACE = 3,
  EXPM_E_HIP = 4,
  EXPM_E_UNSUPPORTED = 5
} expm_status_t;

/* Element type of A and e^A.  For EXPM_C128, (m, s) are chosen from the 1-norm of A itself
 * (max over columns of sum_i |a_ij|, |z| the modulus) on every path.  Above complex order 128,
 * in FP64 with the product-reduced Taylor method or Paterson-Stockmeyer, the method runs on
 * complex matrices natively (planar real and imaginary parts, a complex product as four real
 * products; the alpha rule reads the complex norms of the powers).  Up to order 128, and for
 * the reduced-precision forms and Pade, it runs on the real form [[X, -Y], [Y, X]] of
 * A = X + iY (of order 2n): the map is an algebra homomorphism, so the real exponential of the
 * real form is the real form of e^A; there the alpha rule reads the real form's norms of the
 * powers, which bound the complex ones from above (within a factor sqrt(2)). */
typedef enum { EXPM_F64 = 0, EXPM_C128 = 1 } expm_dtype_t;

/* Arithmetic of the polynomial products.  In the reduced forms the powers A^2, A^3 (A^6) and
 * the first product of the product stage use it; the last product of the stage (which carries
 * the O(1) identity part of T_m), the s squarings (error growth 2^s), the norms, the theta
 * comparison and the linear combinations stay FP64.  EXPM_PREC_FP32: operands rounded to
 * FP32, FP32 accumulation.  EXPM_PREC_BF16X3: each FP64 operand is split into three bfloat16
 * terms (hi + mid + lo), six of the nine cross products (lo*lo, mid*lo, lo*mid dropped) are
 * accumulated in FP32.  EXPM_PREC_FP32_ALL: the single-precision form of the paper's second
 * theta row (Table 2, u = 2^-24): every product, the last one of the stage and the squarings
 * included, in FP32 (operands rounded to FP32, FP32 accumulation); norms, selection, linear
 * combinations and storage stay FP64 (O(n^2) work).  Default u: 2^-24 for FP32 and FP32_ALL,
 * 2^-53 for FP64 and BF16X3.  Reduced forms always run the tiled path (any order). */
typedef enum {
  EXPM_PREC_FP64 = 0,
  EXPM_PREC_FP32 = 1,
  EXPM_PREC_BF16X3 = 2,
  EXPM_PREC_FP32_ALL = 3
} expm_prec_t;

/* How (m, s) is chosen.
 *  PLAIN:   from eta = ||A||_1 (Sec. 4: an estimate of the norm drives the choice).
 *  ALPHA:   from alpha_p = max(d_p, d_{p+1}), d_k = ||A^k||_1^(1/k), p (p - 1) <= m + 1
 *           (the power-norm refinement the paper cites in Sec. 1); d_2, d_3 exact from the
 *           powers the method forms, d_4, d_5 by submultiplicative upper bounds.
 *  LEARNED: a small MLP proposes (m, s) from norm features; the proposal is kept only if the
 *           ALPHA bound holds for it, otherwise the PLAIN rule decides (expm_learned_set). */
typedef enum { EXPM_SEL_PLAIN = 0, EXPM_SEL_ALPHA = 1, EXPM_SEL_LEARNED = 2 } expm_sel_t;

/* Evaluation method (expm_opts_t.flags, at most one bit).  0: the product-reduced sequences
 * of the paper (T_8, T_12, T_18 with 3, 4, 5 products).  The two comparison methods, with FP64
 * products and the plain ||A||_1 rule only:
 *  EXPM_FLAG_PS:   the plain Taylor polynomial T_m = sum_k A^k / k! by the Paterson-Stockmeyer
 *                  rule in Horner form (Sec. 4, eq. poli9), m in {1, 2, 4, 6, 9, 12, 16} with
 *                  0..6 products (Table 3), thresholds theta_m(u) of the same definition
 *                  (Table 2), (m, s) by the same cheapest-cost rule.  Any order: real order
 *                  <= 16 on one wave per matrix, larger on the tiled path.
 *  EXPM_FLAG_PADE: diagonal Pade r_10 or r_26 (Sec. 2, eqs. eq.pade10 and eq.pade26): 3 or 6
 *                  products and one linear solve (costed 4/3 of a product), thresholds of
 *                  Table 1 (u = 2^-53 or 2^-24 only); m_dev receives the order 2m (10 or 26).
 *                  Real order <= 16 (one wave per matrix; the solve is Gauss-Jordan with
 *                  partial pivoting).
 * Unsupported combinations, and the calls that only run the product-reduced kernels
 * (expm_batched, expm_batched_stage, expm_features, expm_magnus4_step), return
 * EXPM_E_UNSUPPORTED. */
#define EXPM_FLAG_PS 1
#define EXPM_FLAG_PADE 2

/* Triangular refinement (expm_opts_t.flags = EXPM_FLAG_TRI, on its own; concluding remarks,
 * after the alpha_p paper it cites): when a real input is upper triangular, the diagonal and
 * the first superdiagonal of T_m(2^-s A) and of every squared iterate are overwritten with the
 * exact values of the exponential (exp(2^(r-s) a_ii), and the (1, 2) entry of the exponential
 * of each 2 x 2 diagonal block); other inputs are unaffected.  Real FP64 inputs, any order, on
 * the tiled path (expm_taylor, expm_batched_uniform, expm_select); complex inputs and the other
 * calls return EXPM_E_UNSUPPORTED. */
#define EXPM_FLAG_TRI 4

typedef struct {
  int32_t dtype;  /* expm_dtype_t */
  int32_t prec;   /* expm_prec_t */
  int32_t sel;    /* expm_sel_t */
  int32_t flags;  /* 0 or one of EXPM_FLAG_PS, EXPM_FLAG_PADE, EXPM_FLAG_TRI; anything else:
                     EXPM_E_INVALID_ARG */
  double u;       /* target relative backward error; 0 = the form's default (2^-24 for FP32
                     and FP32_ALL, 2^-53 otherwise) */
} expm_opts_t;

/* Human-readable name of a status code (static storage). */
EXPM_API const char *expm_status_string(expm_status_t st);

/* theta_m(u) (eq. eq.theta): the largest ||X|| for which T_m(X) = e^{X+E} with
 * ||E|| / ||X|| <= u, from the series of log(e^{-x} T_m(x)) cut after 150 terms (Sec. 1).
 * Host-only, no GPU needed.  m in {1, 2, 4, 6, 8, 9, 12, 16, 18}; u in [2^-53, 2^-10]. */
EXPM_API expm_status_t expm_theta(int32_t m, double u, double *theta_out);

/* The selection rule on the host, identical to the device's (for tests and planning).
 * norms[0..2] = ||A||_1, ||A^2||_1, ||A^3||_1 (entries 1 and 2 ignored by the PLAIN rule; a
 * negative entry means "not formed", replaced by its submultiplicative bound).  Host-only. */
EXPM_API expm_status_t expm_select_rule(const double *norms, int32_t sel, double u, int32_t *m_out,
                               int32_t *s_out);

/* Device workspace in bytes for expm_taylor / expm_batched / expm_select with matrices of
 * order up to n_max and `batch` matrices. */
EXPM_API size_t expm_workspace_bytes(int64_t n_max, int64_t batch, const expm_opts_t *opts);

/* (m, s) for one matrix without computing e^A.  PLAIN needs one norm pass; ALPHA and LEARNED
 * also form A^2 and A^3 in the workspace.  m_dev, s_dev: one int32 each (device). */
EXPM_API expm_status_t expm_select(const void *A_dev, int64_t n, const expm_opts_t *opts,
                          int32_t *m_dev, int32_t *s_dev, void *ws_dev, size_t ws_bytes,
                          void *stream);

/* e^A for one n x n matrix: E_dev <- e^{A_dev}; the chosen (m, s) and the status go to
 * m_dev, s_dev, status_dev (one int32 each, device; status_dev may be NULL).
 * Real order n <= 256 (complex n <= 128): one persistent fused launch, no host
 * synchronisation (graph-capturable).  Larger orders: tiled multi-workgroup kernels; the host
 * reads (m, s) back once (8 bytes) to size the launch sequence, so the call synchronises
 * `stream` and is not graph-capturable. */
EXPM_API expm_status_t expm_taylor(const void *A_dev, void *E_dev, int64_t n, const expm_opts_t *opts,
                          int32_t *m_dev, int32_t *s_dev, int32_t *status_dev, void *ws_dev,
                          size_t ws_bytes, void *stream);

/* e^A for `batch` independent matrices of uneven order n_b <= n_max, real order <= 256
 * (complex <= 128), packed: matrix b occupies elements [offsets_dev[b], offsets_dev[b] + n_b^2)
 * of A_dev and E_dev (elements of the dtype, not bytes).  n_dev[b] = n_b (int32).  Outputs per
 * matrix: m_dev[b], s_dev[b], status_dev[b].  Device kernels sort the batch largest order
 * first and, within an order, by a cost estimate from four sampled rows of each matrix
 * (largest first; the order of the work only, every result is computed from its own exact
 * norm); persistent launches walk that work queue; no host synchronisation
 * (graph-capturable).  The sweeps of real orders 112..128 and 17..64 run on `stream`, those
 * of 144..256, 80..96 and <= 16 on a second stream of the device that the library creates once
 * (default priority); it waits for the sort and `stream` waits for it before the call's work
 * ends, so the call behaves as one operation on `stream` (also under graph capture).  Larger orders:
 * EXPM_E_UNSUPPORTED (use expm_batched_uniform). */
EXPM_API expm_status_t expm_batched(const void *A_dev, void *E_dev, const int64_t *offsets_dev,
                           const int32_t *n_dev, int64_t batch, int64_t n_max,
                           const expm_opts_t *opts, int32_t *m_dev, int32_t *s_dev,
                           int32_t *status_dev, void *ws_dev, size_t ws_bytes, void *stream);

/* expm_batched for callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): no workspace argument; the scratch the call needs
 * (work-queue words, the sorted order, cost keys, the 8-wave on-chip kernel's parked matrices)
 * lives in a device array of the library, 64.3 MiB, which every device the library runs on
 * holds until the process ends.  The call allocates nothing (no hipMalloc, no stream or event
 * creation) and runs every sweep on `stream` in turn (expm_batched runs some of them on a
 * second stream beside it).  Results, (m, s) and status are exactly those of expm_batched.
 * Limits: real order n_max <= 128 (complex n_max <= 64) and batch <= 65536, else
 * EXPM_E_WORKSPACE (the scratch is too small); reduced precision, comparison methods:
 * EXPM_E_UNSUPPORTED; other arguments as expm_batched.  All calls on one device share its
 * array, which keeps the last call's contents (every call rewrites what it reads): calls that
 * overlap on one device (concurrent streams or host threads) race and must be serialised by
 * the caller. */
EXPM_API expm_status_t expm_batched_noalloc(const void *A_dev, void *E_dev, const int64_t *offsets_dev,
                                           const int32_t *n_dev, int64_t batch, int64_t n_max,
                                           const expm_opts_t *opts, int32_t *m_dev, int32_t *s_dev,
                                           int32_t *status_dev, void *stream);

/* expm_batched in phases, for callers that time or overlap them: stage 0 sorts the batch into
 * the device work queue (largest real order first, then largest cost estimate); stage 1 runs the 8-wave on-chip kernel
 * over the real orders 112..128 of the queue; stage 2 runs the sweeps of every other order,
 * which are stages 3, 4 and 5 in turn: 3 the real orders 144..256 on the 8-wave global-memory
 * kernel, 4 the orders 80..96 on the split-row on-chip kernel, 5 the orders up to 64 (17..64
 * on the 4-wave on-chip kernel, up to 16 on one wave per matrix, or all on the 4-wave kernel
 * under the learned selector).  Stages 1..5 need stage 0 to have completed and are
 * independent of each other (separate workspace slots and queue ranges, so they may run on
 * different streams).  Calling 0, 1, 2 (or 0, 1, 3, 4, 5) in order on one stream gives
 * exactly the results of expm_batched.  Arguments as expm_batched; stage outside 0..5 is
 * EXPM_E_INVALID_ARG. */
EXPM_API expm_status_t expm_batched_stage(const void *A_dev, void *E_dev, const int64_t *offsets_dev,
                                 const int32_t *n_dev, int64_t batch, int64_t n_max,
                                 const expm_opts_t *opts, int32_t *m_dev, int32_t *s_dev,
                                 int32_t *status_dev, void *ws_dev, size_t ws_bytes, void *stream,
                                 int32_t stage);

/* e^A for `batch` matrices of the same order n stored back to back (matrix b at element
 * b * n^2).  Any order: real order <= 256 (complex <= 128) runs on the fused kernels, without
 * host synchronisation (graph-capturable): a batch larger than one round of the persistent
 * grid walks a device work queue sorted by the cost estimate of expm_batched (largest
 * first), smaller batches and real order <= 16 (one wave per matrix) take a static
 * assignment; larger orders run the tiled path in groups of matrices (about 2048 output tiles
 * per launch), synchronising once per group to read (m, s) back. */
EXPM_API expm_status_t expm_batched_uniform(const void *A_dev, void *E_dev, int64_t n, int64_t batch,
                                   const expm_opts_t *opts, int32_t *m_dev, int32_t *s_dev,
                                   int32_t *status_dev, void *ws_dev, size_t ws_bytes, void *stream);

/* One step of the fourth-order Magnus integrator for `batch` linear systems Y' = F(t) Y with
 * F(t) = S0 + u(t) S1 (an exponential integrator, in which the exponential of the method is
 * the inner stage; concluding remarks of the paper).  Per system b, with the control sampled
 * at the two Gauss points, u1 = u(t + (1/2 - sqrt(3)/6) h) and u2 = u(t + (1/2 + sqrt(3)/6) h):
 *   Omega = h S0 + (h / 2)(u1 + u2) S1 + (sqrt(3) h^2 / 12)(u1 - u2)(S0 S1 - S1 S0)
 * (the midpoint-sum and commutator terms of the two-point Gauss Magnus expansion, written out
 * for this F), then Y_out = e^Omega Y_in with e^Omega by the product-reduced Taylor method
 * ((m, s) of Omega by opts->sel, PLAIN or ALPHA; accuracy opts->u).
 * Real FP64, order 1 <= n <= 16 (one wavefront per system, everything on chip).  Layout:
 * row-major n x n; system b's S0, S1 at element b * s_stride (s_stride = n^2 for per-system
 * matrices, 0 for one pair shared by all), Y_in and Y_out at b * n^2; Y_out may equal Y_in
 * (in place); u1_dev, u2_dev: batch doubles each.  Outputs m_dev[b], s_dev[b] (the (m, s)
 * used for Omega) and status_dev[b] (may be NULL; EXPM_E_NONFINITE and a NaN Y_out when an
 * input of the system is not finite).  Needs no workspace; graph-capturable.  Returns
 * EXPM_E_UNSUPPORTED for complex dtype, reduced precision, the learned selector or n > 16. */
EXPM_API expm_status_t expm_magnus4_step(const double *S0_dev, const double *S1_dev, int64_t s_stride,
                                         const double *Y_in_dev, double *Y_out_dev, const double *u1_dev,
                                         const double *u2_dev, int64_t n, int64_t batch, double h,
                                         const expm_opts_t *opts, int32_t *m_dev, int32_t *s_dev,
                                         int32_t *status_dev, void *stream);

/* ---------------------------------------------------------------------------------------
 * Launch configuration (not part of the paper's method; no effect on any result's
 * definition): what an autotuner picks per order range, precision and selector by timing the
 * candidates on the device (paper_1710_10989_amd/autotune.py keeps the winners in a JSON cache
 * keyed by the GPU architecture and installs them with expm_tune_set).  A zero field means the
 * library's default, which is what an untuned process runs.  Process-wide.
 *  arrangement[sel]     expm_batched with selector sel: 0 (default) the sweeps of real orders
 *                       144..256, 80..96 and <= 16 on a second stream beside 112..128 then
 *                       17..64 on `stream`; 1 every sweep in turn on `stream`; 2 144..256 and
 *                       80..96 beside 112..128, 17..64, <= 16; 3 everything but 112..128 on
 *                       the second stream.
 *  small_kernel         real order <= 16: 0 / 1 one wavefront per matrix (default), 2 the
 *                       4-wave on-chip kernel.
 *  per_cu[k]            persistent workgroups per CU of sweep kernel k (0 global-memory 4-wave,
 *                       1 global-memory 8-wave, 2 on-chip 4-wave, 3 split-row, 4 on-chip 8-wave,
 *                       5 one-wave kernel, in that kernel's workgroups); 0 or more than the
 *                       occupancy maximum means that maximum.
 *  tiles_per_launch[p]  tiled path (orders above 256 and the reduced forms) with expm_prec_t p:
 *                       output tiles per launch, which sets how many matrices a group holds
 *                       (0: 2048).  It changes the workspace expm_workspace_bytes reports, so
 *                       query that after expm_tune_set.
 * Fields out of range: EXPM_E_INVALID_ARG. */
typedef struct {
  int32_t arrangement[3];
  int32_t small_kernel;
  int32_t per_cu[6];
  int32_t tiles_per_launch[4];
} expm_tune_t;

EXPM_API expm_status_t expm_tune_set(const expm_tune_t *t);
/* The installed configuration (zero fields: defaults). */
EXPM_API expm_status_t expm_tune_get(expm_tune_t *t);
/* The candidates' upper limits on the current device: per_cu[k] = occupancy maximum of sweep
 * kernel k, the largest arrangement and small_kernel values, the default tiles_per_launch.
 * EXPM_E_HIP when no device is visible. */
EXPM_API expm_status_t expm_tune_limits(expm_tune_t *t);

/* ---------------------------------------------------------------------------------------
 * Learned (m, s) selector (EXPM_SEL_LEARNED).  Not part of the paper: a small MLP proposes
 * (m, s) from features that exist once A^2 is formed; the proposal is kept only when the
 * alpha_p backward-error bound of eq. eq.theta holds for it (with ||A^3|| when the proposed
 * degree forms A^3, else its submultiplicative bound), otherwise the plain ||A||_1 rule
 * decides.  Classes: 0..4 = (1, 0), (2, 0), (4, 0), (8, 0), (12, 0); 5..15 = (18, 0..10).
 * Features (8, in this order): log2 d_1 .. log2 d_5 with d_k = ||A^k||_1^(1/k) (d_3, d_4, d_5
 * by submultiplicative bounds from ||A||, ||A^2||), log2 n, |tr A| / ||A||_1,
 * ||A - A^T||_1 / (2 ||A||_1).
 * MLP: 8 -> 64 (ReLU) -> 64 (ReLU) -> 16, FP32, parameters packed as W1[64][8], b1[64],
 * W2[64][64], b2[64], W3[16][64], b3[16] (expm_mlp_param_count() floats).
 * Used by the fused path (real order <= 256); the tiled path runs EXPM_SEL_ALPHA instead.
 * --------------------------------------------------------------------------------------- */

/* Feature rows and training labels for a packed batch (arguments as expm_batched; real FP64,
 * order <= 256).  features_dev: 16 doubles per matrix: f0..f7, ||A||_1, ||A^2||_1,
 * ||A^3||_1, label class, plain m, plain s, alpha m, alpha s.  The label is the cheapest
 * (m, s) that passes the acceptance test above; it is also written to m_dev / s_dev.  Forms
 * A^2 and A^3 in the workspace; no e^A. */
EXPM_API expm_status_t expm_features(const void *A_dev, const int64_t *offsets_dev, const int32_t *n_dev,
                                     int64_t batch, int64_t n_max, const expm_opts_t *opts, double *features_dev,
                                     int32_t *m_dev, int32_t *s_dev, void *ws_dev, size_t ws_bytes, void *stream);

/* MLP kernels (device pointers, FP32, row-major batches: x [batch][8], logits [batch][16]).
 * scratch: expm_mlp_scratch_bytes(batch) bytes.  expm_mlp_grad writes the gradient of the
 * mean softmax cross-entropy over the batch (labels y, int32 classes) to grads_dev
 * (expm_mlp_param_count() floats) and the per-sample losses to loss_dev (batch floats).
 * expm_mlp_adam applies one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected,
 * step >= 1) to params_dev with moment buffers m_dev, v_dev.  All deterministic. */
EXPM_API size_t expm_mlp_scratch_bytes(int32_t batch);
EXPM_API int32_t expm_mlp_param_count(void);
EXPM_API expm_status_t expm_mlp_forward(const float *params_dev, const float *x_dev, int32_t batch,
                                        float *logits_dev, void *scratch_dev, size_t scratch_bytes, void *stream);
EXPM_API expm_status_t expm_mlp_grad(const float *params_dev, const float *x_dev, const int32_t *y_dev,
                                     int32_t batch, float *grads_dev, float *loss_dev, void *scratch_dev,
                                     size_t scratch_bytes, void *stream);
EXPM_API expm_status_t expm_mlp_adam(float *params_dev, const float *grads_dev, float *m_dev, float *v_dev,
                                     int32_t step, float lr, void *stream);

/* Installs the selector's parameters (device, copied) and feature normalisation (host:
 * mean[8] then std[8], std > 0; the MLP sees (f - mean) / std), and resets the counters.
 * Process-wide state of the current device; synchronises `stream`. */
EXPM_API expm_status_t expm_learned_set(const float *params_dev, const double *norm_host, void *stream);

/* Proposals accepted / rejected by EXPM_SEL_LEARNED since the last expm_learned_set. */
EXPM_API expm_status_t expm_learned_counts(int64_t *accepted, int64_t *rejected);

#ifdef __cplusplus
}
#endif
#endif /* EXPM_H_ */
