// C ABI entry points of libmfe: validation, dispatch and error reporting.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "dense.h"
#include "sparse.h"

namespace mfe {

namespace {
thread_local std::string g_last_error;
thread_local double g_loop_ms = 0.0, g_step_ms = 0.0;
}

void record_timing(double loop_ms, double step_ms) {
  g_loop_ms = loop_ms;
  g_step_ms = step_ms;
}

int set_error(int status, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

void clear_error() { g_last_error.clear(); }

void set_warning(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = std::string("warning: ") + buf;
}

// Parameter checks shared by every equilibration entry point (the paper requires
// alpha, beta, gamma, M > 0; Algorithm 1 and Section 2.3).
int check_params(const mfe_equil_params* p, bool check_targets) {
  if (!p) return set_error(MFE_EINVAL, "params is NULL");
  auto pos = [](double x) { return x > 0 && std::isfinite(x); };
  if (check_targets && (!pos(p->alpha) || !pos(p->beta)))
    return set_error(MFE_EINVAL, "alpha and beta must be positive and finite");
  if (!pos(p->gamma)) return set_error(MFE_EINVAL, "gamma must be positive and finite");
  if (!pos(p->box_M)) return set_error(MFE_EINVAL, "box bound M must be positive and finite");
  if (p->steps < 0) return set_error(MFE_EINVAL, "steps must be >= 0");
  if (p->probes < 1 || p->probes > 256) return set_error(MFE_EINVAL, "probes must be in 1..256");
  if (p->t0 < 0) return set_error(MFE_EINVAL, "t0 must be >= 0");
  if (p->batch < 0 || p->batch >= (1 << 30)) return set_error(MFE_EINVAL, "batch must be in [0, 2^30)");
  if ((int64_t)p->steps + (int64_t)p->t0 + 2 >= (int64_t)1 << 32)
    return set_error(MFE_EINVAL, "steps + t0 exceed the sign stream range");
  return MFE_OK;
}

// Section 1: exact equilibration needs m alpha^2 = n beta^2.  A mismatch is reported as
// a warning (the regularised problem is well posed for any positive targets).
int check_targets(int64_t m, int64_t n, double alpha, double beta, double* rel_out) {
  auto pos = [](double x) { return x > 0 && std::isfinite(x); };
  if (m <= 0 || n <= 0) return set_error(MFE_EINVAL, "m and n must be positive");
  if (!pos(alpha) || !pos(beta)) return set_error(MFE_EINVAL, "alpha and beta must be positive and finite");
  const double a = (double)m * alpha * alpha, b = (double)n * beta * beta;
  const double rel = std::fabs(a - b) / std::max(a, b);
  if (rel_out) *rel_out = rel;
  if (rel > 1e-12)
    set_warning("m alpha^2 = %.17g differs from n beta^2 = %.17g (relative %.3g): rows of norm alpha and "
                "columns of norm beta cannot both be reached exactly (Section 1); the regularised problem "
                "is solved as stated",
                a, b, rel);
  return MFE_OK;
}

// The same check for every matrix of a plan (symmetric plans have one target); the
// first mismatched matrix is named.  Invalid values are left to the run to reject.
void check_plan_targets(const mfe_plan* p, const mfe_equil_params* prm, const double* alpha_b,
                        const double* beta_b) {
  if (p->symmetric) return;
  for (int b = 0; b < p->count; ++b) {
    const double al = alpha_b ? alpha_b[b] : prm->alpha;
    const double be = beta_b ? beta_b[b] : prm->beta;
    if (!(al > 0) || !(be > 0) || !std::isfinite(al) || !std::isfinite(be)) return;
    double rel = 0.0;
    (void)check_targets(p->meta[b].m, p->meta[b].n, al, be, &rel);
    if (rel > 1e-12) {
      if (p->count > 1) g_last_error += " (matrix " + std::to_string(b) + " of the plan)";
      return;
    }
  }
}

}  // namespace mfe

using namespace mfe;

extern "C" {

const char* mfe_last_error(void) { return g_last_error.c_str(); }

const char* mfe_version(void) { return "mfe 0.1 (gfx950)"; }

int mfe_check_targets(int64_t m, int64_t n, double alpha, double beta, double* rel) {
  clear_error();
  return check_targets(m, n, alpha, beta, rel);
}

int mfe_default_alpha_beta(int64_t m, int64_t n, double* alpha, double* beta) {
  clear_error();
  if (m <= 0 || n <= 0) return set_error(MFE_EINVAL, "m and n must be positive");
  if (!alpha || !beta) return set_error(MFE_EINVAL, "NULL output");
  *alpha = std::pow((double)n / (double)m, 0.25);
  *beta = std::pow((double)m / (double)n, 0.25);
  return MFE_OK;
}

int mfe_draw_signs(uint64_t seed, int32_t batch, int64_t step, int32_t side, int64_t nwords,
                   uint64_t* words, void* stream) {
  clear_error();
  if (batch < 0 || batch >= (1 << 30)) return set_error(MFE_EINVAL, "batch out of range");
  if (step < 0 || step >= ((int64_t)1 << 32)) return set_error(MFE_EINVAL, "step out of range");
  if (side < 0 || side > 3) return set_error(MFE_EINVAL, "side out of range");
  if (nwords < 0) return set_error(MFE_EINVAL, "nwords < 0");
  if (nwords == 0) return MFE_OK;
  if (!words) return set_error(MFE_EINVAL, "words is NULL");
  hipStream_t st = (hipStream_t)stream;
  // Philox blocks are written whole: draw into a padded scratch area when needed.
  const int64_t nblk = ceil_div(nwords, 4);
  uint64_t* dst = words;
  uint64_t* tmp = nullptr;
  if (nwords % 4) {
    MFE_HIP(hipMalloc((void**)&tmp, sizeof(uint64_t) * nblk * 4));
    dst = tmp;
  }
  SignSeg seg;
  seg.ctrl_lo = ((uint64_t)batch << 34) | (uint64_t)side;
  seg.nblocks = nblk;
  seg.word_off = 0;
  SignSeg* dseg = nullptr;
  int64_t* dpre = nullptr;
  int rc = MFE_OK;
  const int64_t pre[2] = {0, nblk};
  if (hipMalloc((void**)&dseg, sizeof(SignSeg)) != hipSuccess ||
      hipMalloc((void**)&dpre, sizeof(pre)) != hipSuccess) {
    rc = set_error(MFE_ENOMEM, "hipMalloc failed");
  } else if (hipMemcpyAsync(dseg, &seg, sizeof seg, hipMemcpyHostToDevice, st) != hipSuccess ||
             hipMemcpyAsync(dpre, pre, sizeof pre, hipMemcpyHostToDevice, st) != hipSuccess) {
    rc = set_error(MFE_EDEVICE, "hipMemcpyAsync failed");
  } else {
    SignGenDev g;
    g.segs = dseg;
    g.seg_prefix = dpre;
    g.nseg = 1;
    g.nblocks = nblk;
    g.seed = seed;
    g.step = (uint64_t)step;
    g.out = dst;
    rc = launch_signgen(g, st);
    if (rc == MFE_OK && tmp &&
        hipMemcpyAsync(words, tmp, sizeof(uint64_t) * nwords, hipMemcpyDeviceToDevice, st) != hipSuccess)
      rc = set_error(MFE_EDEVICE, "hipMemcpyAsync failed");
    if (rc == MFE_OK && hipStreamSynchronize(st) != hipSuccess) rc = set_error(MFE_EDEVICE, "sync failed");
  }
  (void)hipFree(dseg);
  (void)hipFree(dpre);
  (void)hipFree(tmp);
  return rc;
}

int mfe_plan_create(const mfe_matrix* mats, int32_t count, int32_t max_probes, void* stream, mfe_plan** out) {
  clear_error();
  return plan_build(mats, count, max_probes, (hipStream_t)stream, out);
}

int mfe_plan_equilibrate(mfe_plan* plan, const mfe_equil_params* p, const double* alpha_b,
                         const double* beta_b, int32_t use_graph, double* d, double* e, double* u_bar,
                         double* v_bar) {
  clear_error();
  if (!plan) return set_error(MFE_EINVAL, "plan is NULL");
  MFE_CHECK(check_params(p, alpha_b == nullptr || beta_b == nullptr));
  if (p->probes > 64) return set_error(MFE_EUNSUPPORTED, "sparse path supports at most 64 probes per step");
  check_plan_targets(plan, p, alpha_b, beta_b);
  return plan_run(plan, p, alpha_b, beta_b, use_graph, d, e, u_bar, v_bar);
}

int mfe_last_timing(double* loop_ms, double* step_ms) {
  if (loop_ms) *loop_ms = g_loop_ms;
  if (step_ms) *step_ms = g_step_ms;
  return MFE_OK;
}

int mfe_plan_last_timing(const mfe_plan* plan, double* loop_ms, double* step_kernel_ms) {
  clear_error();
  if (!plan) return set_error(MFE_EINVAL, "plan is NULL");
  if (loop_ms) *loop_ms = plan->last_loop_ms;
  if (step_kernel_ms) *step_kernel_ms = plan->last_step_ms;
  return MFE_OK;
}

int mfe_plan_destroy(mfe_plan* plan) {
  clear_error();
  plan_free(plan);
  return MFE_OK;
}

int mfe_equilibrate(const mfe_matrix* A, const mfe_equil_params* p, double* d, double* e, double* u_bar,
                    double* v_bar) {
  clear_error();
  if (!A) return set_error(MFE_EINVAL, "matrix is NULL");
  MFE_CHECK(check_params(p, true));
  if (!d || !e) return set_error(MFE_EINVAL, "outputs d and e are required");
  if (A->m <= 0 || A->n <= 0) return set_error(MFE_EDIM, "m and n must be positive");
  if (A->kind == MFE_CSR_F64)
    return set_error(MFE_EUNSUPPORTED, "CSR with FP64 values is not built (store the values as FP32, or pass "
                                       "the product as MFE_OPERATOR)");
  MFE_CHECK(check_targets(A->m, A->n, p->alpha, p->beta, nullptr));
  switch (A->kind) {
    case MFE_CSR_F32: {
      if (p->probes > 64) return set_error(MFE_EUNSUPPORTED, "sparse path supports at most 64 probes per step");
      mfe_plan* plan = nullptr;
      MFE_CHECK(plan_build(A, 1, p->probes, (hipStream_t)p->stream, &plan));
      int rc = plan_run(plan, p, nullptr, nullptr, 0, d, e, u_bar, v_bar);
      plan_free(plan);
      return rc;
    }
    case MFE_DENSE_F64:
      return dense_f64_equilibrate(A, p, d, e, u_bar, v_bar);
    case MFE_OPERATOR:
      return operator_equilibrate(A, p, d, e, u_bar, v_bar);
    case MFE_DENSE_BF16:
      return dense_bf16_equilibrate(A, p, d, e, u_bar, v_bar);
    default:
      return set_error(MFE_EINVAL, "unknown matrix kind %d", (int)A->kind);
  }
}

int mfe_equilibrate_noalloc(const mfe_matrix* A, const mfe_equil_params* p, double* d, double* e, double* u_bar,
                            double* v_bar) {
  clear_error();
  if (!A) return set_error(MFE_EINVAL, "matrix is NULL");
  MFE_CHECK(check_params(p, true));
  if (!d || !e) return set_error(MFE_EINVAL, "outputs d and e are required");
  if (A->m <= 0 || A->n <= 0) return set_error(MFE_EDIM, "m and n must be positive");
  if (A->kind != MFE_DENSE_F64)
    return set_error(MFE_EUNSUPPORTED, "the allocation-free entry point takes MFE_DENSE_F64 matrices only");
  MFE_CHECK(check_targets(A->m, A->n, p->alpha, p->beta, nullptr));
  return dense_f64_equilibrate_noalloc(A, p, d, e, u_bar, v_bar);
}

int mfe_plan_lsqr(mfe_plan* plan, const double* b, const double* d, const double* e, double tol,
                  int32_t max_iter, int32_t check_every, double* x, mfe_lsqr_info* info, void* stream) {
  clear_error();
  if (!plan) return set_error(MFE_EINVAL, "plan is NULL");
  if (plan->count != 1) return set_error(MFE_EUNSUPPORTED, "LSQR needs a single-matrix plan");
  if (!b || !x) return set_error(MFE_EINVAL, "b and x are required");
  if (!(tol >= 0) || max_iter < 0 || check_every < 1)
    return set_error(MFE_EINVAL, "need tol >= 0, max_iter >= 0, check_every >= 1");
  return plan_lsqr(plan, b, d, e, tol, max_iter, check_every, x, info, (hipStream_t)stream);
}

int mfe_lsqr(const mfe_matrix* A, const double* b, const double* d, const double* e, double tol,
             int32_t max_iter, int32_t check_every, double* x, mfe_lsqr_info* info, void* stream) {
  clear_error();
  if (!A) return set_error(MFE_EINVAL, "matrix is NULL");
  if (!b || !x) return set_error(MFE_EINVAL, "b and x are required");
  if (!(tol >= 0) || max_iter < 0 || check_every < 1)
    return set_error(MFE_EINVAL, "need tol >= 0, max_iter >= 0, check_every >= 1");
  if (A->m <= 0 || A->n <= 0) return set_error(MFE_EDIM, "m and n must be positive");
  if (A->kind == MFE_CSR_F32) {
    mfe_plan* plan = nullptr;
    MFE_CHECK(plan_build(A, 1, 1, (hipStream_t)stream, &plan));
    int rc = plan_lsqr(plan, b, d, e, tol, max_iter, check_every, x, info, (hipStream_t)stream);
    plan_free(plan);
    return rc;
  }
  if (A->kind == MFE_DENSE_F64) return dense_f64_lsqr(A, b, d, e, tol, max_iter, check_every, x, info, (hipStream_t)stream);
  return set_error(MFE_EUNSUPPORTED, "LSQR accepts CSR FP32 and dense FP64 matrices");
}

int mfe_residual(const mfe_matrix* A, const double* d, const double* e, double alpha, double beta, double* rms,
                 double* rms_nonempty, int64_t* n_empty, void* stream) {
  clear_error();
  if (!A) return set_error(MFE_EINVAL, "matrix is NULL");
  if (!(alpha > 0) || !(beta > 0)) return set_error(MFE_EINVAL, "alpha and beta must be positive");
  if (A->m <= 0 || A->n <= 0) return set_error(MFE_EDIM, "m and n must be positive");
  if (A->kind == MFE_CSR_F32) {
    mfe_plan* plan = nullptr;
    MFE_CHECK(plan_build(A, 1, 1, (hipStream_t)stream, &plan));
    int rc = plan_residual(plan, d, e, alpha, beta, rms, rms_nonempty, n_empty, (hipStream_t)stream);
    plan_free(plan);
    return rc;
  }
  if (A->kind == MFE_DENSE_F64) return dense_f64_residual(A, d, e, alpha, beta, rms, rms_nonempty, n_empty, (hipStream_t)stream);
  return set_error(MFE_EUNSUPPORTED, "residual accepts CSR FP32 and dense FP64 matrices");
}

int mfe_plan_equilibrate_trace(mfe_plan* plan, const mfe_equil_params* p, int32_t trace_every,
                                double* rms_trace, double* d, double* e, double* u_bar, double* v_bar) {
  clear_error();
  if (!plan) return set_error(MFE_EINVAL, "plan is NULL");
  MFE_CHECK(check_params(p, true));
  if (p->probes > plan->max_probes) return set_error(MFE_EINVAL, "probes exceed the plan's max_probes");
  if (plan_has_variant(plan))
    return set_error(MFE_EUNSUPPORTED, "the residual trace measures the standard problem (no variant settings)");
  check_plan_targets(plan, p, nullptr, nullptr);
  return plan_equilibrate_trace(plan, p, trace_every, rms_trace, d, e, u_bar, v_bar);
}

int mfe_plan_warmstart(mfe_plan* plan, const float* params, uint64_t seed, int32_t probes, const double* alpha_b,
                       const double* beta_b, double gamma, double box_M, int32_t learned, double* u0, double* v0,
                       void* stream) {
  clear_error();
  if (!plan) return set_error(MFE_EINVAL, "plan is NULL");
  if (!u0 || !v0) return set_error(MFE_EINVAL, "NULL output");
  if (!(gamma > 0) || !(box_M > 0)) return set_error(MFE_EINVAL, "gamma and M must be positive");
  if (plan_has_variant(plan))
    return set_error(MFE_EUNSUPPORTED, "warm starts are trained for the standard problem (no variant settings)");
  return plan_warmstart(plan, params, seed, probes, alpha_b, beta_b, gamma, box_M, learned, u0, v0,
                        (hipStream_t)stream);
}

int mfe_plan_op_norm(mfe_plan* plan, const double* d, const double* e, int32_t max_iter, double tol, double* norm,
                     int32_t* iters, void* stream) {
  clear_error();
  if (!plan || !norm) return set_error(MFE_EINVAL, "plan or norm is NULL");
  if (max_iter < 1 || !(tol >= 0)) return set_error(MFE_EINVAL, "max_iter must be >= 1 and tol >= 0");
  return plan_op_norm(plan, d, e, max_iter, tol, norm, iters, (hipStream_t)stream);
}

int mfe_plan_ccp_lasso(mfe_plan* plan, const double* b, const double* d, const double* e, double lam,
                       double op_norm, int32_t iters, int32_t trace_every, double* trace, double* x,
                       mfe_ccp_info* info, void* stream) {
  clear_error();
  if (!plan || !b || !x) return set_error(MFE_EINVAL, "plan, b or x is NULL");
  if (!(lam > 0) || !std::isfinite(lam)) return set_error(MFE_EINVAL, "lambda must be positive and finite");
  if (iters < 0) return set_error(MFE_EINVAL, "iters must be >= 0");
  if (trace && trace_every <= 0) return set_error(MFE_EINVAL, "a trace needs trace_every > 0");
  return plan_ccp_lasso(plan, b, d, e, lam, op_norm, iters, trace_every, trace, x, info, (hipStream_t)stream);
}

int mfe_plan_create_symmetric(const mfe_matrix* A, int32_t max_probes, void* stream, mfe_plan** out) {
  clear_error();
  return plan_build_symmetric(A, max_probes, (hipStream_t)stream, out);
}

int mfe_plan_set_targets(mfe_plan* plan, const double* row_target, const double* col_target, void* stream) {
  clear_error();
  if (!plan) return set_error(MFE_EINVAL, "plan is NULL");
  return plan_set_targets(plan, row_target, col_target, (hipStream_t)stream);
}

int mfe_plan_set_blocks(mfe_plan* plan, const int64_t* row_ptr, int64_t row_blocks, const int64_t* col_ptr,
                        int64_t col_blocks) {
  clear_error();
  if (!plan) return set_error(MFE_EINVAL, "plan is NULL");
  return plan_set_blocks(plan, row_ptr, row_blocks, col_ptr, col_blocks, nullptr);
}

int mfe_plan_set_tuning(mfe_plan* plan, int32_t loads_in_flight, int32_t rows_mode, int32_t cols_mode,
                        int32_t stream_hints, int32_t slice_order, int32_t workgroup_threads) {
  clear_error();
  if (!plan) return set_error(MFE_EINVAL, "plan is NULL");
  if (loads_in_flight != 1 && loads_in_flight != 2 && loads_in_flight != 4 && loads_in_flight != 8 &&
      loads_in_flight != 16)
    return set_error(MFE_EINVAL, "loads_in_flight must be 1, 2, 4, 8 or 16");
  const bool both = rows_mode == 2 && cols_mode == 2;
  if (!both && (rows_mode < 0 || rows_mode > 1 || cols_mode < 0 || cols_mode > 1))
    return set_error(MFE_EINVAL, "direction modes must be 0 or 1 each, or 2 for both (one launch per step)");
  if (stream_hints < -1 || stream_hints > 1)
    return set_error(MFE_EINVAL, "stream_hints must be -1 (by the plan's size), 0 or 1");
  if (slice_order < -1 || slice_order > 1)
    return set_error(MFE_EINVAL, "slice_order must be -1 (by the launch shape), 0 or 1");
  if (workgroup_threads != 0 && workgroup_threads != 256 && workgroup_threads != 512 && workgroup_threads != 1024)
    return set_error(MFE_EINVAL, "workgroup_threads must be 0 (the default, 256), 256, 512 or 1024");
  if ((rows_mode == 1 && !plan->rows.len_lo) || (cols_mode == 1 && !plan->cols.len_lo))
    return set_error(MFE_EUNSUPPORTED, "two-part mode requested for a direction without the two-part layout");
  plan->tune_batch = loads_in_flight;
  plan->tune_split[0] = rows_mode;
  plan->tune_split[1] = cols_mode;
  plan->tune_nt = stream_hints;
  plan->tune_sched = slice_order;
  plan->tune_wg = workgroup_threads == 256 ? 0 : workgroup_threads;
  return MFE_OK;
}

int mfe_plan_autotune(mfe_plan* plan, const mfe_equil_params* p, const double* alpha_b, const double* beta_b,
                      int32_t trial_steps, int32_t* chosen, double* best_step_ms, int32_t* n_candidates) {
  clear_error();
  if (!plan) return set_error(MFE_EINVAL, "plan is NULL");
  MFE_CHECK(check_params(p, true));
  if (p->probes > plan->max_probes) return set_error(MFE_EINVAL, "probes exceed the plan's max_probes");
  check_plan_targets(plan, p, alpha_b, beta_b);
  const std::string warn = g_last_error;
  const int rc = plan_autotune(plan, p, alpha_b, beta_b, trial_steps, chosen, best_step_ms, n_candidates);
  if (rc == MFE_OK) g_last_error = warn;
  return rc;
}

int mfe_plan_sketch_features(mfe_plan* plan, uint64_t seed, int32_t probes, const double* alpha_b,
                             const double* beta_b, double gamma, double box_M, float* feat_rows, float* feat_cols,
                             double* u_sketch, double* v_sketch, void* stream) {
  clear_error();
  if (!plan) return set_error(MFE_EINVAL, "plan is NULL");
  if (!(gamma > 0) || !(box_M > 0)) return set_error(MFE_EINVAL, "gamma and M must be positive");
  if (!feat_rows || !feat_cols || !u_sketch || !v_sketch) return set_error(MFE_EINVAL, "NULL output");
  return plan_sketch_features(plan, seed, probes, alpha_b, beta_b, gamma, box_M, feat_rows, feat_cols, u_sketch,
                              v_sketch, (hipStream_t)stream);
}

int mfe_plan_training_set(mfe_plan* plan, uint64_t seed, int32_t probes, const double* alpha_b,
                          const double* beta_b, double gamma, double box_M, const double* u_label,
                          const double* v_label, int64_t per_matrix, uint64_t sample_seed, float* X, float* t,
                          int64_t* idx, int64_t* count, void* stream) {
  clear_error();
  if (!plan || !u_label || !v_label || !count) return set_error(MFE_EINVAL, "plan, labels or count is NULL");
  if (per_matrix < 1) return set_error(MFE_EINVAL, "per_matrix must be >= 1");
  if (!(gamma > 0) || !(box_M > 0)) return set_error(MFE_EINVAL, "gamma and M must be positive");
  if (X && !t) return set_error(MFE_EINVAL, "t is NULL");
  if (plan_has_variant(plan))
    return set_error(MFE_EUNSUPPORTED, "warm starts are trained for the standard problem (no variant settings)");
  return plan_training_set(plan, seed, probes, alpha_b, beta_b, gamma, box_M, u_label, v_label, per_matrix,
                           sample_seed, X, t, idx, count, (hipStream_t)stream);
}

int mfe_mlp_sizes(int32_t* n_params, int32_t* n_features, int32_t* width) {
  clear_error();
  if (n_params) *n_params = mlp_param_count();
  if (n_features) *n_features = mlp_feature_count();
  if (width) *width = 64;
  return MFE_OK;
}

int mfe_mlp_forward(const float* params, const float* X, int64_t count, float* y, void* stream) {
  clear_error();
  if (count < 0) return set_error(MFE_EINVAL, "count < 0");
  if (count > 0 && (!params || !X || !y)) return set_error(MFE_EINVAL, "NULL pointer");
  return mlp_forward(params, X, count, y, (hipStream_t)stream);
}

int mfe_mlp_loss_grad(const float* params, const float* X, const float* t, int64_t count, float* grad,
                      double* loss, void* stream) {
  clear_error();
  if (count < 1 || !params || !X || !t || !grad) return set_error(MFE_EINVAL, "invalid arguments");
  return mlp_grad(params, X, t, count, grad, loss, (hipStream_t)stream);
}

int mfe_mlp_train(float* params, float* adam_m, float* adam_v, int32_t step0, const float* X, const float* t,
                  int64_t count, int64_t batch, int32_t iters, float lr, uint64_t seed, double* loss_trace,
                  void* stream) {
  clear_error();
  if (!params || !adam_m || !adam_v || !X || !t) return set_error(MFE_EINVAL, "NULL pointer");
  if (count < 1 || batch < 1 || iters < 0 || step0 < 0 || !(lr > 0)) return set_error(MFE_EINVAL, "invalid sizes");
  return mlp_train(params, adam_m, adam_v, step0, X, t, count, batch, iters, lr, seed, loss_trace,
                   (hipStream_t)stream);
}

int mfe_warmstart_apply(int64_t n, const double* sketch, const float* delta, double box_M, double* out,
                        void* stream) {
  clear_error();
  if (n < 0 || !(box_M > 0)) return set_error(MFE_EINVAL, "invalid arguments");
  if (n > 0 && (!sketch || !out)) return set_error(MFE_EINVAL, "NULL pointer");
  return warmstart_apply(n, sketch, delta, box_M, out, (hipStream_t)stream);
}

}  // extern "C"
