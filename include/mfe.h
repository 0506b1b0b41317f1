/*
 * mfe.h -- stochastic matrix-free equilibration on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libmfe.so.  The library finds diagonal D = diag(e^u), E = diag(e^v) that
 * approximately equilibrate A (rows of DAE with 2-norm alpha, columns with 2-norm
 * beta) by projected stochastic gradient descent on the regularised, box-constrained
 * convex problem of Diamond & Boyd, "Stochastic Matrix-Free Equilibration":
 *
 *   minimise  (1/2) sum_ij A_ij^2 e^(2u_i + 2v_j) - alpha^2 1'u - beta^2 1'v
 *             + (gamma/2) ||(u, v)||^2      subject to ||u||_inf <= M, ||v||_inf <= M
 *
 * (problem (prob:reg-constr-equil), Section 2.3), solved by Algorithm 1 (Section 3.2):
 * at step t, with Rademacher probe blocks S (n x k) and W (m x k),
 *   z_u = e^(2u) * mean_p (A E S)_{:,p}^2,   z_v = e^(2v) * mean_p (A' D W)_{:,p}^2
 *   u  <- clip(u - eta_t (z_u - alpha^2 + gamma u), -M, M)     (v likewise with beta)
 *   u_bar <- 2u/(tau+2) + tau u_bar/(tau+2),  eta_t = 2/(gamma (tau+1)),  tau = t + t0,
 * both updates from the previous iterate (Jacobi order).  Outputs d = e^u_bar, e = e^v_bar.
 * lsqr() is the downstream consumer of Section 5.1: LSQR on (DAE) xbar = D b, x = E xbar.
 *
 * General conventions
 *  - Every call returns an mfe_status; nothing aborts or throws across the ABI.  On a
 *    non-OK status the outputs are unspecified and mfe_last_error() describes the cause.
 *  - "device" pointers are HIP device allocations on the current device; "host"
 *    pointers are ordinary CPU memory.  The caller owns every pointer it passes; the
 *    library never frees caller memory.  Workspaces are library-owned and released
 *    before the call returns, or when the owning plan is destroyed.
 *  - Work is ordered on the HIP stream given in the parameters (NULL = default
 *    stream).  Calls that report a status synchronise that stream once at the end.
 *  - Probe signs are bit-exact and reproducible: probe p of index i at step t is bit
 *    i*k + p of the Philox4x64-10 stream with key (seed, (batch << 34) | (t << 2) | side),
 *    block c evaluated at counter (c+1, 0, 0, 0), 256 bits per block, bit q of a block
 *    = bit (q mod 64) of output word q div 64; bit 1 means -1.  side 0 = s (indexed by
 *    column j), side 1 = w (indexed by row i).  Section 3.1 only asks for iid fair signs.
 *  - Results are deterministic run to run (no floating-point atomics on any path).
 */
#ifndef MFE_H
#define MFE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MFE_OK = 0,
  MFE_EINVAL = -1,       /* invalid parameter value or NULL where a pointer is required */
  MFE_EDIM = -2,         /* inconsistent or unsupported dimensions (e.g. nnz >= 2^31) */
  MFE_ENONFINITE = -3,   /* a gradient estimate or iterate became NaN/Inf (e.g. NaN in A) */
  MFE_EDEVICE = -4,      /* a HIP runtime call failed */
  MFE_ENOMEM = -5,       /* device allocation failed */
  MFE_EUNSUPPORTED = -6  /* valid request the library does not implement */
} mfe_status;

typedef enum {
  MFE_DENSE_F64 = 0,   /* dense row-major FP64: data (device), ld >= n */
  MFE_DENSE_BF16 = 1,  /* dense row-major bfloat16 bit patterns (uint16): data (device), ld >= n */
  MFE_CSR_F32 = 2,     /* CSR: row_ptr int32[m+1], col_idx int32[nnz], val float[nnz] (device);
                          column indices within a row sorted ascending and unique */
  MFE_OPERATOR = 3,    /* matrix-free: only apply() is used */
  MFE_CSR_F64 = 4      /* CSR with FP64 values (val then points to double[nnz]): declared so the
                          kind can be named, not built; every call taking a matrix returns
                          MFE_EUNSUPPORTED for it.  (The sparse engine accumulates in FP64 from
                          FP32 values; a caller holding FP64 values can round them to FP32 or
                          wrap its own product as MFE_OPERATOR.) */
} mfe_kind;

/* Matrix-free operator (the setting of Section 3): Y = A X (trans = 0, X is n x k,
 * Y is m x k) or Y = A' X (trans = 1, X is m x k, Y is n x k).  Row-major blocks:
 * element (i, p) at X[i*ldx + p].  FP64 device pointers (the iteration amplifies
 * rounding in its first steps, so FP32 products cannot track the FP64 method closely),
 * work ordered on `stream` (a hipStream_t).  Returns 0 on success; any other value
 * aborts the run with MFE_EDEVICE. */
typedef int (*mfe_apply_fn)(void* ctx, int trans, int32_t k, const double* X, int64_t ldx,
                            double* Y, int64_t ldy, void* stream);

typedef struct {
  int32_t kind;               /* mfe_kind */
  int64_t m, n;               /* rows, columns (> 0) */
  const void* data;           /* dense kinds */
  int64_t ld;                 /* dense leading dimension (elements) */
  int64_t nnz;                /* CSR */
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const float* val;
  mfe_apply_fn apply;         /* operator kind */
  void* ctx;
} mfe_matrix;

typedef struct {
  double alpha, beta;   /* target row / column norms (> 0); see mfe_default_alpha_beta */
  double gamma;         /* regularisation (> 0); the paper's experiments use 0.1 */
  double box_M;         /* box bound M (> 0): |u_i|, |v_j| <= M */
  int32_t steps;        /* T >= 0; T = 0 returns d = e^u0, e = e^v0 */
  int32_t probes;       /* k probes per step, 1..256 (k = 1 is Algorithm 1 verbatim) */
  uint64_t seed;        /* probe stream seed */
  int32_t t0;           /* step offset >= 0 (0 = Algorithm 1); tau = t + t0 */
  int32_t batch;        /* batch index b of the sign stream (0 for a single matrix) */
  const double* u0;     /* device [m] warm start in [-M, M], or NULL for 0 (EINVAL if outside) */
  const double* v0;     /* device [n] warm start in [-M, M], or NULL for 0 (EINVAL if outside) */
  void* stream;         /* hipStream_t, NULL = default stream */
} mfe_equil_params;

typedef struct {
  int32_t iters;           /* iterations run */
  int32_t stop_reason;     /* 0 max_iter, 1 ||Ax-b||/||b|| <= tol, 2 normal-equation test, 3 breakdown */
  double rel_resid;        /* ||A x - b|| / ||b|| of the original system at the last check */
  double normal_eq;        /* ||Abar' rbar|| / (||Abar|| ||rbar||) estimate at the last check */
} mfe_lsqr_info;

typedef struct {
  int32_t iters;           /* CCP iterations run */
  int32_t norm_iters;      /* bidiagonalisation steps spent on ||D A E||_2 (0 when it was given) */
  double op_norm;          /* ||D A E||_2 used for the step sizes */
  double tau, sigma;       /* step sizes 0.9 / op_norm */
  double objective;        /* ||A x - b||^2 / sqrt(lam) + sqrt(lam) ||x||_1 at the end */
} mfe_ccp_info;

typedef struct mfe_plan mfe_plan;

/* alpha = (n/m)^(1/4), beta = (m/n)^(1/4): the choice of Section 4, which satisfies
 * m alpha^2 = n beta^2 (Section 1) and alpha beta = 1.  Host pointers.
 * EINVAL if m <= 0, n <= 0 or an output is NULL. */
int mfe_default_alpha_beta(int64_t m, int64_t n, double* alpha, double* beta);

/* Section 1: rows of norm alpha and columns of norm beta can only be reached exactly when
 * m alpha^2 = n beta^2 (both sides then sum to ||DAE||_F^2).  Host-only check, no device
 * work.  *rel (host, nullable) receives |m alpha^2 - n beta^2| / max(m alpha^2, n beta^2);
 * above 1e-12 a message starting with "warning:" is left in mfe_last_error().  Returns
 * MFE_OK either way: a mismatch is not an error, since the regularised problem of
 * Section 2.3 has a unique solution for any alpha, beta > 0.  EINVAL: m, n, alpha or
 * beta not positive (or not finite).  mfe_equilibrate, mfe_plan_equilibrate (per
 * matrix), mfe_plan_equilibrate_trace and mfe_plan_autotune run the same check and keep
 * the warning in mfe_last_error() when they return MFE_OK. */
int mfe_check_targets(int64_t m, int64_t n, double alpha, double beta, double* rel);

/* Algorithm 1 on one matrix (any kind).  Outputs are device FP64 arrays:
 * d [m] = e^u_bar, e [n] = e^v_bar (required); u_bar [m], v_bar [n] (nullable).
 * CSR and dense kinds run fused HIP kernels; the operator kind calls apply() twice per
 * step and runs the square/step/project update in the library's kernels.
 * MFE_DENSE_BF16 runs both products on the matrix cores: probe operands are exact signs
 * times bf16(e^x), products accumulate in FP32, iterates stay FP64 (the library keeps
 * two tiled copies of A, 2 x 2mn bytes of device memory, for the call's duration).
 * EINVAL: alpha, beta, gamma or M <= 0 or not finite; steps < 0; probes outside 1..256;
 * t0 < 0; a required pointer NULL.  EDIM: m or n <= 0, nnz >= 2^31, ld < n.
 * EUNSUPPORTED: CSR/dense with probes > 64, MFE_DENSE_BF16 with M > 80 (e^x must stay
 * inside the bf16 range), or a kind not built.
 * ENONFINITE: a non-finite estimate or iterate occurred (the clip would hide a NaN). */
int mfe_equilibrate(const mfe_matrix* A, const mfe_equil_params* p, double* d, double* e,
                    double* u_bar, double* v_bar);

/* mfe_equilibrate for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): MFE_DENSE_F64 only,
 * same kernels and results as mfe_equilibrate, but every workspace is carved from one
 * static device array of 8 MiB (one per device, held until the process ends); no
 * hipMalloc, hipFree or allocating library call, and no host-to-device copy or memset
 * node (scratch that must start at zero is cleared by a kernel).  A run needs
 * 256-byte-aligned pieces of 32 (m + n) bytes of iterates, averages and scales, the sign
 * words (about (m + n) k / 8 bytes), and for the single-workgroup paths (m + n <= 1792) an
 * m x n FP64 transposed copy of A (not for k = 1, m <= 200, n <= 128) and a chunk of
 * staged sign words.  EDIM when that exceeds 8 MiB (nothing is run); otherwise the
 * errors of mfe_equilibrate; EUNSUPPORTED for other kinds.  Calls that overlap on one
 * device (other threads, or other streams before this call's final synchronisation)
 * share the array and race; calls in sequence are independent.  Synchronises p->stream
 * at the end (the status). */
int mfe_equilibrate_noalloc(const mfe_matrix* A, const mfe_equil_params* p, double* d, double* e,
                            double* u_bar, double* v_bar);

/* Plans: preprocessing (CSR -> CSC transpose, sliced-ELL layouts for both products)
 * done once and reused.  count >= 1 CSR matrices are equilibrated together in one
 * launch per step (the batched path).
 * max_probes bounds p->probes of later runs (1..64).  Only MFE_CSR_F32 is accepted. */
int mfe_plan_create(const mfe_matrix* mats, int32_t count, int32_t max_probes, void* stream,
                    mfe_plan** out);

/* Run Algorithm 1 on every matrix of the plan.  Outputs are device FP64 arrays holding
 * all matrices back to back in plan order: d [sum m], e [sum n], u_bar/v_bar nullable.
 * alpha_b/beta_b: host arrays [count] of per-matrix targets, or NULL to use p->alpha,
 * p->beta for every matrix.  Matrix b uses sign-stream batch index p->batch + b.
 * p->u0 / p->v0, when set, are device [sum m] / [sum n].
 * use_graph != 0 captures the T step launches in one HIP graph and replays it. */
int mfe_plan_equilibrate(mfe_plan* plan, const mfe_equil_params* p, const double* alpha_b,
                         const double* beta_b, int32_t use_graph, double* d, double* e,
                         double* u_bar, double* v_bar);

/* Timing of the last mfe_plan_equilibrate (host pointer): milliseconds spent in the
 * step loop (HIP events around it) and in the step kernel alone per launch average. */
int mfe_plan_last_timing(const mfe_plan* plan, double* loop_ms, double* step_kernel_ms);

int mfe_plan_destroy(mfe_plan* plan);

/* Timing of the step loop of the last mfe_equilibrate on the calling thread (dense
 * BF16 path): milliseconds for all T steps and per step (HIP events on the stream).
 * Host pointers (nullable). */
int mfe_last_timing(double* loop_ms, double* step_ms);

/* LSQR (Paige & Saunders) on (D A E) xbar = D b, x = E xbar (Section 5.1), FP64
 * vectors and recurrences, A values FP32 (CSR) or FP64 (dense).  b [m], d [m], e [n]
 * and x [n] are device FP64; d or e NULL means the identity.  Every check_every
 * iterations (and at max_iter) the original residual ||A x - b|| / ||b|| is evaluated;
 * the run stops when it is <= tol (reason 1) or when LSQR's normal-equation estimate is
 * <= tol (reason 2).  info is a host pointer (nullable).  stream: hipStream_t or NULL.
 * Only MFE_CSR_F32 and MFE_DENSE_F64 are accepted. */
int mfe_lsqr(const mfe_matrix* A, const double* b, const double* d, const double* e,
             double tol, int32_t max_iter, int32_t check_every, double* x,
             mfe_lsqr_info* info, void* stream);

/* Same on a single-matrix plan (reuses its preprocessing).  The plan keeps the run's
 * device vectors and its captured iteration block (a HIP graph of up to 25 iterations)
 * from the first call until mfe_plan_destroy, so later calls allocate nothing and
 * capture again only when the captured block length min(check_every, 25) changes; calls
 * on one plan must not overlap (other threads, or other streams before a call's final
 * synchronisation). */
int mfe_plan_lsqr(mfe_plan* plan, const double* b, const double* d, const double* e,
                  double tol, int32_t max_iter, int32_t check_every, double* x,
                  mfe_lsqr_info* info, void* stream);

/* RMS equilibration error of D A E (Section 4):
 *   (1/sqrt(m+n)) sqrt( sum_i (||row_i(DAE)|| - alpha)^2 + sum_j (||col_j(DAE)|| - beta)^2 )
 * evaluated exactly from the entries (one pass over each layout).  d [m], e [n] device
 * FP64 (NULL = identity).  Host outputs: rms over all rows and columns; rms_nonempty over
 * rows/columns of A with at least one stored entry; n_empty the number left out.
 * Only MFE_CSR_F32 and MFE_DENSE_F64 are accepted. */
int mfe_residual(const mfe_matrix* A, const double* d, const double* e, double alpha,
                 double beta, double* rms, double* rms_nonempty, int64_t* n_empty,
                 void* stream);

/* Sign words of the probe stream (Section 3.1 probes, contract above): writes
 * nwords 64-bit words starting at word 0 of the stream (seed, batch, step, side) into
 * device memory `words`.  EINVAL for out-of-range batch (>= 2^30), step (>= 2^32),
 * side (> 3) or NULL. */
int mfe_draw_signs(uint64_t seed, int32_t batch, int64_t step, int32_t side, int64_t nwords,
                   uint64_t* words, void* stream);

/* ---------------------------------------------------------------- learned warm start
 *
 * A warm start (u0, v0) with a step offset t0 > 0 (see mfe_equil_params) replaces the
 * paper's u0 = v0 = 0.  It is built from probe sketches only (matrix-free):
 *   1. sketch: with `probes` Rademacher probes per side (stream sides 2 and 3, step 0,
 *      batch = matrix index) the Section 3.1 estimator at (u, v) = 0 gives r_i ~ row
 *      norm^2, c_j ~ column norm^2;
 *   2. sketch initialisation: u_i = -1/2 log r_i + c, v_j = -1/2 log c_j + c with
 *      e^(4c) = alpha^2 F / n, F = (sum r + sum c)/2 (exact equilibration in expectation
 *      for A = diag(a) G diag(b)); indices without entries get min(M, target/gamma);
 *   3. a width-64, 3-layer tanh MLP maps 8 features per index to a correction; the
 *      warm start is clip(sketch initialisation + correction, -M, M).
 * The feature layout is documented in csrc/warmstart.hip. */

/* Sketch features of every row and column of a plan (all matrices back to back, in
 * plan order).  feat_rows [sum m][8], feat_cols [sum n][8] FP32; u_sketch [sum m],
 * v_sketch [sum n] FP64 sketch initialisations; all device.  alpha_b / beta_b: host
 * [count] or NULL for (n_b/m_b)^(1/4), (m_b/n_b)^(1/4).  probes in {4, 8, 16}. */
int mfe_plan_sketch_features(mfe_plan* plan, uint64_t seed, int32_t probes, const double* alpha_b,
                             const double* beta_b, double gamma, double box_M, float* feat_rows,
                             float* feat_cols, double* u_sketch, double* v_sketch, void* stream);

/* Training set of the warm-start network from a plan whose matrices have been
 * equilibrated: labels u_label [sum m], v_label [sum n] (device FP64, e.g. u_bar, v_bar of a
 * plain Algorithm 1 run), sketch features as mfe_plan_sketch_features(seed, probes,
 * alpha_b, beta_b, gamma, box_M).  From matrix b it takes min(per_matrix, m_b) rows and
 * min(per_matrix, n_b) columns, one per stratum: the c-th of the cnt samples of a side of
 * m_b indices comes from [floor(c m_b / cnt), floor((c+1) m_b / cnt)), at offset
 * Philox4x64-10(counter (c+1, 0, 0, 0), key (sample_seed, (((b << 1) | side) << 2) | 3))
 * word 0 mod the stratum size (side 0 rows, 1 columns), so no index is taken twice.
 * Sample order: the rows of matrix 0, 1, ..., then the columns of matrix 0, 1, ...
 * Outputs (device): X [count][8] FP32 (the sample's features, copied), t [count] FP32
 * (label - sketch initialisation, rounded once from FP64), idx [count] int64 (nullable:
 * the sample's index in the plan's concatenated rows, or columns).  *count (host)
 * receives the number of samples; with X == NULL only *count is computed (no device work).
 * EINVAL: plan, labels or count NULL, per_matrix < 1, probes not in {4, 8, 16};
 * EUNSUPPORTED: a plan with Section 6 settings. */
int mfe_plan_training_set(mfe_plan* plan, uint64_t seed, int32_t probes, const double* alpha_b,
                          const double* beta_b, double gamma, double box_M, const double* u_label,
                          const double* v_label, int64_t per_matrix, uint64_t sample_seed, float* X,
                          float* t, int64_t* idx, int64_t* count, void* stream);

/* Sizes of the warm-start network: parameter count, feature count (8), width (64). */
int mfe_mlp_sizes(int32_t* n_params, int32_t* n_features, int32_t* width);

/* y[i] = MLP(X[i]) for count rows of X [count][8] (device FP32); params device FP32 in the
 * order W1 (8 x 64, row-major), b1 (64), W2 (64 x 64), b2 (64), w3 (64), b3 (1). */
int mfe_mlp_forward(const float* params, const float* X, int64_t count, float* y, void* stream);

/* Mean squared error over all count rows and its gradient grad [n_params] (device FP32);
 * loss is a host pointer (nullable). */
int mfe_mlp_loss_grad(const float* params, const float* X, const float* t, int64_t count, float* grad,
                      double* loss, void* stream);

/* iters Adam steps (lr, beta1 0.9, beta2 0.999, eps 1e-8) on mini-batches of `batch` rows
 * drawn with replacement from X [count][8] / t [count]: row b of step s is
 * Philox(counter (b+1,0,0,0), key (seed, (s << 2) | 3)) word 0 mod count.  params, adam_m,
 * adam_v device FP32 [n_params], updated in place; step0 = steps already taken (for the
 * bias correction and the batch stream).  loss_trace: host [iters] (nullable). */
int mfe_mlp_train(float* params, float* adam_m, float* adam_v, int32_t step0, const float* X, const float* t,
                  int64_t count, int64_t batch, int32_t iters, float lr, uint64_t seed, double* loss_trace,
                  void* stream);

/* The whole warm start in one stream-ordered call: sketch features of every row and
 * column of the plan (as mfe_plan_sketch_features), the network's corrections (when
 * learned != 0; params device FP32 [n_params], else the sketch initialisation alone), and
 * u0 / v0 = clip(sketch + correction, -M, M), device FP64 [sum m] / [sum n], ready for
 * mfe_plan_equilibrate with t0 > 0.  Scratch is kept in the plan between calls.
 * EINVAL: plan or an output NULL, probes not in {4, 8, 16}, learned with params NULL. */
int mfe_plan_warmstart(mfe_plan* plan, const float* params, uint64_t seed, int32_t probes, const double* alpha_b,
                       const double* beta_b, double gamma, double box_M, int32_t learned, double* u0, double* v0,
                       void* stream);

/* out[i] = clip(sketch[i] + delta[i], -M, M) (delta FP32, nullable = 0); device arrays. */
int mfe_warmstart_apply(int64_t n, const double* sketch, const float* delta, double box_M, double* out,
                        void* stream);

/* Algorithm 1 on a single-matrix plan with the RMS equilibration error (Section 4) of the
 * current average recorded after every trace_every steps: rms_trace is a host array of
 * ceil(steps / trace_every) doubles.  Step time is measured without the evaluations
 * (mfe_plan_last_timing). */
int mfe_plan_equilibrate_trace(mfe_plan* plan, const mfe_equil_params* p, int32_t trace_every,
                               double* rms_trace, double* d, double* e, double* u_bar, double* v_bar);

/* Autotuner of a plan's step kernels (the products of Algorithm 1, Section 3.2, in the
 * batched layouts).  Runs trial_steps steps (1..100000, eagerly, results discarded) of
 * every launch configuration with the run parameters p (probes, targets, seed) and keeps
 * the fastest in the plan for its later runs (the default configuration is timed first and
 * kept unless another is more than 1% faster).  Configurations: 1, 2, 4, 8 or 16 entry loads in
 * flight per lane (16 only for p->probes <= 16); both directions of a step in one launch
 * (modes 2, 2: the default) or one launch per direction (mode 0); and, for a
 * single-matrix plan whose gathered table exceeds 6 MB, each such direction also in mode
 * 1 (two launches over the halves of the table, FP64 partial sums in between); and the
 * one-launch form also with the other stream-hint setting, with each fixed slice order
 * and with 512 (p->probes <= 16) and 1024 (p->probes <= 8) threads per workgroup (see
 * mfe_plan_set_tuning).  Every
 * configuration adds the same terms in the same order, so tuning never changes a result
 * bit.  (Plans whose directions have few slices, and plans with Section 6 settings, run
 * their own launch forms whatever the modes.)
 * chosen (host int32[6], nullable): loads in flight, mode of the rows, mode of the columns,
 * stream hints (0 or 1), slice order (-1, 0 or 1), threads per workgroup;
 * best_step_ms, n_candidates: nullable.  Allocates two temporary device arrays.
 * EINVAL: plan NULL, invalid p (as mfe_plan_equilibrate), trial_steps out of range. */
int mfe_plan_autotune(mfe_plan* plan, const mfe_equil_params* p, const double* alpha_b, const double* beta_b,
                      int32_t trial_steps, int32_t* chosen, double* best_step_ms, int32_t* n_candidates);

/* Sets a plan's launch configuration directly (the values mfe_plan_autotune chooses):
 * loads_in_flight 1, 2, 4, 8 or 16; rows_mode / cols_mode both 2 (one launch per step, the
 * default), or each 0 or 1 (1 only for a direction with a two-part layout, see
 * mfe_plan_autotune); stream_hints 1: the entry and per-index state streams use
 * non-temporal loads and stores, 0: plain ones, -1 (the default): non-temporal when the
 * streams of one step exceed 512 MiB (twice the last-level cache; 8 bytes per stored entry
 * and direction plus ~64 bytes per row and column).  Descriptor gathers always use plain
 * loads.  slice_order 1: the wavefronts of a step launch take each matrix's slices (64 rows
 * or columns) in order of decreasing width, which keeps the end of a launch of several
 * rounds of workgroups from running the device half empty; 0: in storage order; -1 (the
 * default): 1 when the one-launch step has more workgroups than five per compute unit or
 * a direction runs one slice per workgroup, else 0.  workgroup_threads: threads per
 * workgroup of the one-launch step (64 rows each per wavefront): 256, 512 or 1024, or 0 for
 * the default 256; a run uses at most 1024 threads up to 8 probes (512 with 16-byte
 * descriptors), 512 up to 16 (256 with one load in flight) and 256 above, and 256 with
 * Section 6 settings.
 * None of these changes a result bit.
 * EINVAL: plan NULL or a value out of range; EUNSUPPORTED: a two-part mode for a
 * direction without the layout. */
int mfe_plan_set_tuning(mfe_plan* plan, int32_t loads_in_flight, int32_t rows_mode, int32_t cols_mode,
                        int32_t stream_hints, int32_t slice_order, int32_t workgroup_threads);

/* ---- Chambolle-Cremers-Pock on the Lasso (Section 5.2), sparse plans ---------------- */

/* ||D A E||_2 of the plan's matrix (block diagonal for a batched plan) by Golub-Kahan
 * bidiagonalisation (the Lanczos process LSQR uses, started from b = 1, one product with
 * D A E and one with its transpose per step): the largest singular value of the i-step
 * bidiagonal matrix is a lower bound that converges to the norm.  Checked every 5 steps;
 * the run stops when it changes by at most tol (relative), when the process ends exactly,
 * or after max_iter steps.  d [sum m], e [sum n]: device FP64, NULL = identity.  norm,
 * iters: host (iters nullable).  EINVAL: NULL plan or norm, max_iter < 1, tol < 0. */
int mfe_plan_op_norm(mfe_plan* plan, const double* d, const double* e, int32_t max_iter, double tol,
                     double* norm, int32_t* iters, void* stream);

/* The Lasso of Section 5.2, minimise ||A x - b||^2 / sqrt(lam) + sqrt(lam) ||x||_1, by the
 * Chambolle-Pock primal-dual method with theta = 1 and tau = sigma = 0.9 / ||D A E||_2 from
 * zero iterates, run on D A E with x = E xbar (D = E = I without equilibration):
 *   y  <- (y + sigma (D A E xt - d b)) / (1 + sigma d^2 sqrt(lam) / 2)   (prox of sigma g*)
 *   x' <- soft(x - tau E A' D y, tau sqrt(lam) e),  xt <- 2 x' - x,  x <- x'
 * One product with D A E and one with its transpose per iteration, each fused with its
 * proximal step; FP64 vectors.  b [sum m], d, e (NULL = identity) and x [sum n] are device
 * FP64; x receives E xbar.  op_norm > 0 is used as ||D A E||_2, otherwise it is estimated
 * (mfe_plan_op_norm, tol 1e-10, at most 1000 steps).  trace (host, nullable) receives
 * the objective every trace_every iterations (iters / trace_every values).  info: host,
 * nullable.  EINVAL: NULL plan, b or x, lam <= 0, iters < 0, trace without trace_every > 0. */
int mfe_plan_ccp_lasso(mfe_plan* plan, const double* b, const double* d, const double* e, double lam,
                       double op_norm, int32_t iters, int32_t trace_every, double* trace, double* x,
                       mfe_ccp_info* info, void* stream);

/* ---- Section 6 variants (sparse plans) ------------------------------------------- */

/* Symmetric equilibration (Section 6, problem (prob:sym-equil), Algorithm 2): a plan for
 * one square CSR FP32 matrix A = A' (pattern and value bits checked on the device).
 * mfe_plan_equilibrate then runs Algorithm 2 with k probes per step: one product
 * D A D s per step, u <- clip(u - eta (z - alpha^2 + gamma u), -M, M) with
 * z_i = e^(2u_i) mean_p (A e^u s_p)_i^2 and the running average as in Algorithm 1.
 * The probes s are the side-0 stream of the probe contract (indexed by j = 0..n-1).
 * p->beta and p->v0 are ignored; d and e both receive e^(u_bar), u_bar and v_bar both
 * u_bar.  Autotuning, LSQR and the residual work as on other plans; the residual
 * trace, warm starts, targets and blocks are EUNSUPPORTED.
 * EDIM: m != n; EINVAL: A not symmetric or invalid CSR; EUNSUPPORTED: another kind. */
int mfe_plan_create_symmetric(const mfe_matrix* A, int32_t max_probes, void* stream, mfe_plan** out);

/* Varying row and column norms (Section 6, problem (prob:equil-vary-norms)): later runs
 * of the plan aim at squared row norms row_target[i] and squared column norms
 * col_target[j] instead of alpha^2 and beta^2 (the gradient is |DAE|^2 1 - r + gamma u).
 * Device FP64 arrays of sum m and sum n values in the plan's concatenated original
 * order, copied into the plan; NULL restores alpha^2 (beta^2) on that side.  The sums
 * of both should agree (sum of squared row norms = sum of squared column norms), as
 * m alpha^2 = n beta^2 does for the standard targets; this is not checked.
 * EINVAL: a value that is not positive and finite (nothing is changed);
 * EUNSUPPORTED: symmetric plan.  Synchronises `stream` (hipStream_t or NULL). */
int mfe_plan_set_targets(mfe_plan* plan, const double* row_target, const double* col_target, void* stream);

/* Block equilibration (Section 6, problem (prob:block-equil)), single-matrix plans:
 * rows [row_ptr[b], row_ptr[b+1]) share one scaling e^(u_b) (row_blocks blocks), and
 * columns likewise; host int64 arrays of blocks + 1 offsets from 0 to m (n), strictly
 * increasing, copied into the plan; NULL for a side without blocks.  Later runs step
 * the block variables with the sum of the block's row estimates (same probes as
 * Algorithm 1) minus the block target (the sum of its rows' squared targets: alpha^2
 * times the block size by default) plus gamma u_b.  In those runs p->u0 / p->v0 hold
 * one value per block, u_bar / v_bar receive one value per block, and d / e one value
 * per row / column (the block's scaling).
 * EINVAL: offsets invalid (nothing is changed); EUNSUPPORTED: plan of several matrices
 * or symmetric plan. */
int mfe_plan_set_blocks(mfe_plan* plan, const int64_t* row_ptr, int64_t row_blocks, const int64_t* col_ptr,
                        int64_t col_blocks);

/* ---- Measurement probes (the ceilings the sparse step is compared against) ---------
 *
 * Each product of Algorithm 1 (Section 3.2) on a sparse matrix reads, per stored entry,
 * one 8-byte descriptor of the other side at a random position, so the step is bounded
 * by the rate of random gathers from a table of the descriptor table's size as well as by
 * the streaming rate.  These calls measure the two rates in isolation on the current
 * device: mean milliseconds per launch over `reps` launches (HIP events, after one
 * untimed launch), written to the host pointer ms.  They allocate and free their own
 * device buffers.  EINVAL for sizes or reps out of range, NULL ms. */

/* `gathers` random 8-byte reads (hashed indices) from a table of table_bytes bytes (>= 8),
 * in_flight (1, 2, 4 or 8) independent reads per lane at a time. */
int mfe_probe_gather(int64_t table_bytes, int64_t gathers, int32_t in_flight, int32_t reps, double* ms,
                     void* stream);

/* `gathers` 8-byte reads from a table of table_bytes bytes (8 .. 32 GiB - 8) in rows of
 * per_row (5, 10, 20 or 40): each thread takes one row of per_row hashed indices, sorts
 * them increasing and reads them one at a time, as a lane of the sparse step walks the
 * sorted entries of one row (the lanes at the same slot then read the same part of the
 * table). */
int mfe_probe_gather_sorted(int64_t table_bytes, int64_t gathers, int32_t per_row, int32_t reps, double* ms,
                            void* stream);

/* One read of a buffer of `bytes` bytes (>= 16) with 16-byte non-temporal loads. */
int mfe_probe_stream(int64_t bytes, int32_t reps, double* ms, void* stream);

/* Thread-local description of the last non-OK status (or a warning), never NULL. */
const char* mfe_last_error(void);

/* Library version string. */
const char* mfe_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MFE_H */
