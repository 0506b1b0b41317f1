// Sparse (CSR) engine of libmfe: layouts, plan and kernel argument blocks.
//
// Both products of Algorithm 1 (Section 3.2) run from one library-built layout per
// direction: the rows of A for Y = A E S and the rows of A' (the CSC of A) for
// X = A' D W.  Each direction is stored as a sliced ELL structure with 64 rows per
// slice (one wavefront, one row per lane): entry (slot q, lane l) of slice s sits at
// ent[slice_off[s] + 64 q + l], so every load of a slot is one contiguous 512-byte
// access.  Within windows of 4096 rows the rows are ordered by decreasing length so
// that the lanes of a slice have similar lengths (little padding, few idle lanes).
// Per-index state (iterates, averages, descriptors) lives in this internal order; the
// entry indices refer to the other direction's internal order.  Several matrices are
// handled as one block-diagonal problem; slices never span two matrices.
#pragma once

#include <vector>

#include "common.h"

namespace mfe {

constexpr int kSlice = 64;       // rows per slice = wavefront size
constexpr int kWindow = 4096;    // rows sorted together by length
constexpr int kBlock = 256;      // threads per workgroup of the step kernel
// Slots whose loads a lane issues together (1, 2, 4, 8 or 16; the autotuner may choose
// another per plan).  One slot at a time -- the entry load, then its gather -- was
// measured fastest on the 1e6 x 5e5 headline: 147 us per step against 173 (2), 177 (4),
// 179 (8) and 187 (16), at the same occupancy for 1 and 8 (grid order, five resident
// workgroups per CU); with the current kernel, 126.7 against 145.4 (2).
#ifndef MFE_BATCH
#define MFE_BATCH 1
#endif
constexpr int kBatch = MFE_BATCH;
// Streams (entries of both directions, per-index state) larger than this -- twice the
// 256 MB last-level cache -- use non-temporal loads and stores by default: caching them
// gains nothing and evicts the gathered descriptor tables.  Smaller plans keep plain
// accesses, whose lines the last-level cache holds from one step to the next (measured
// on the 1e6 x 5e5 headline, ~256 MB of streams: 126.7 us per step plain, 161.5 hinted).
constexpr int64_t kStreamHintBytes = 512ll << 20;

struct SideLayout {
  int64_t norig = 0;   // original indices (sum over matrices)
  int64_t nint = 0;    // internal indices (each matrix padded to whole slices)
  int64_t nslices = 0;
  int64_t nent = 0;    // stored entries including padding
  int64_t* slice_off = nullptr;   // [nslices + 1] first entry of each slice
  int32_t* slice_mat = nullptr;   // [nslices] matrix of the slice
  int32_t* len = nullptr;         // [nint] row length, 0 for padding lanes
  int32_t* orig = nullptr;        // [nint] local original index, -1 for padding lanes
  int32_t* orig2int = nullptr;    // [norig] global original index -> internal index
  int2* ent = nullptr;            // [nent] (other-side internal index, FP32 value bits)
  // Two-part mode (single-matrix plans whose gathered table is larger than one XCD's L2):
  // entries of every row are ordered so that those gathering other-side indices below
  // split_at come first; len_lo[r] counts them.  A step then gathers from one half of
  // the table per launch.
  int64_t split_at = -1;          // -1: no two-part layout
  int32_t* len_lo = nullptr;      // [nint]
  // Launch order of the slices: wavefront w of a step launch takes slice sched[w].  Each
  // matrix's slices in order of decreasing width (stored entries per lane), so that the
  // longest run first and the last wavefronts of a launch are short ones.
  int32_t* sched = nullptr;       // [nslices]
};

// Gathered-table size (at 8 bytes per index) above which a plan builds the two-part
// layout of a direction, so that the autotuner can try it: per launch, half the table
// is gathered, which fits one XCD's 4 MB L2 better than the whole.
constexpr int64_t kSplitBytes = 6ll << 20;

// Per-matrix data the kernels need (device table).
struct MatDev {
  double tgt_row;         // alpha_b^2
  double tgt_col;         // beta_b^2
  int64_t row_orig_base;  // first original row of the matrix in the concatenation
  int64_t col_orig_base;
  int64_t sign_word_row;  // first sign word of the matrix's side-1 segment in a slot
  int64_t sign_word_col;  // first sign word of the matrix's side-0 segment in a slot
};

struct MatMeta {
  int64_t m, n, nnz;
  int64_t row_orig_base, col_orig_base, nnz_base;
  int64_t row_int_base, col_int_base;
};

// One Philox sign segment: all indices of one side of one matrix.
struct SignSeg {
  uint64_t ctrl_lo;   // (batch << 34) | side; the step is or-ed in per launch
  int64_t nblocks;    // Philox blocks of the segment
  int64_t word_off;   // first word of the segment inside a slot
};

struct SideDev {
  const int64_t* slice_off;
  const int32_t* slice_mat;
  const int32_t* len;
  const int32_t* orig;
  const int2* ent;
  int64_t nint;
  double* x;                  // iterate (u or v)
  double* xbar;               // running average
  const void* gather;         // other side's descriptors from the previous step
  void* out;                  // this side's descriptors for the next step
  const uint64_t* next_signs; // slot holding the sign words of step t + 1
  int is_row;                 // 1: rows (targets alpha^2, side-1 signs); 0: columns
  // 0: whole rows; 1: entries [0, len_lo), k partial sums stored to part; 2: partial sums
  // loaded from part, entries [len_lo, len), then the update
  int part_mode;
  const int32_t* len_lo;
  double* part;               // [k][nint] FP64 partial sums
  // Section 6 variants (read by the variant kernel only): per-index squared targets in
  // internal order (null: the matrix's alpha^2 / beta^2), and for a side with blocks the
  // buffer receiving each index's estimate z instead of the update.
  const double* tgt;
  double* zout;
  const int32_t* sched;       // slice taken by each wavefront (null: slice = wavefront)
  // 1: the entry and state streams use non-temporal loads and stores (for working sets
  // well beyond the 256 MB last-level cache, where keeping them would evict the gathered
  // descriptor tables); 0: plain loads and stores
  int nt;
};

// One side of a block-equilibrated plan (Section 6): indices [ptr[b], ptr[b+1]) of the
// original order share the variable x_b.
struct BlockDev {
  const int64_t* ptr;         // [nb + 1]
  int64_t nb;
  const int32_t* orig2int;    // original index -> internal index
  const double* tgt;          // [nb] block targets (sums of the indices' squared targets)
  double* bx;                 // [nb] block iterate
  double* bxbar;              // [nb] running average
  const double* z;            // [nint] per-index estimates of the current step
  int32_t group;              // lanes per block (power of two, 1..64)
};

struct SignGenDev {
  const SignSeg* segs;
  const int64_t* seg_prefix;  // [nseg + 1] prefix sums of blocks
  int32_t nseg;
  int64_t nblocks;            // total Philox blocks
  uint64_t seed;
  uint64_t step;              // step whose signs are generated (0: none)
  uint64_t* out;              // destination slot
};

// Arguments of one launch of the step kernel: one direction of one step.
struct PhaseArgs {
  SideDev side;
  SignGenDev gen;
  const MatDev* mats;
  int32_t k;
  StepScalars sc;
  int64_t side_blocks, gen_blocks;
  int* flag;                  // bit 0: non-finite value seen; bit 1: warm start outside the box
  int32_t split;              // wavefronts per slice wanted for the direction (1: one lane per row)
};

struct mfe_plan_impl;

// LSQR workspace and captured iteration block kept by a plan between calls (lsqr.hip).
struct LsqrCache;
void free_lsqr_cache(LsqrCache* c);

}  // namespace mfe

struct mfe_plan {
  int32_t count = 0;
  int32_t max_probes = 0;
  std::vector<mfe::MatMeta> meta;
  int64_t M = 0, N = 0, NNZ = 0;
  mfe::SideLayout rows, cols;
  // run-time buffers (allocated on first use)
  double *x_row = nullptr, *xbar_row = nullptr, *x_col = nullptr, *xbar_col = nullptr;
  mfe::Desc* desc_row[2] = {nullptr, nullptr};
  mfe::Desc* desc_col[2] = {nullptr, nullptr};
  uint64_t* signs[2] = {nullptr, nullptr};
  double* part[2] = {nullptr, nullptr};  // partial sums of the two-part mode (rows, columns)
  // Launch configuration of the step kernels, chosen by plan_autotune (results are the
  // same bit for bit under every configuration): loads in flight per lane, and how the
  // directions (rows, columns) are launched: {2, 2} both directions of a step in one
  // launch (the default); otherwise one launch per direction (0), or two launches over
  // the halves of its table for a direction with a two-part layout (1); and whether the
  // entry and state streams bypass the caches (1), stay in them (0), or (-1) follow the
  // plan's size (stream_hints); and whether wavefronts take the slices in the layout's
  // longest-first order (1), in grid order (0), or (-1) as slice_schedule decides.
  int32_t tune_batch = mfe::kBatch;
  int32_t tune_split[2] = {2, 2};
  int32_t tune_nt = -1;
  int32_t tune_sched = -1;
  int32_t tune_wg = 0;  // threads per workgroup of the one-launch step (0: kBlock)
  // LSQR workspace and graph of its iteration block, allocated by the first mfe_plan_lsqr
  mfe::LsqrCache* lsqr_cache = nullptr;
  // scratch of the warm-start calls (sketch, features, network outputs)
  void* ws = nullptr;
  size_t ws_bytes = 0;
  std::vector<char> ws_host;  // host staging of the small tables copied into ws
  int64_t sign_words = 0;           // words per slot
  int32_t sign_k = 0;               // k the sign layout was built for
  int64_t sign_batch_base = -1;     // batch index of matrix 0 in that layout
  std::vector<mfe::SignSeg> segs_host;
  mfe::SignSeg* segs = nullptr;
  int64_t* seg_prefix = nullptr;
  int64_t sign_blocks = 0;
  mfe::MatDev* mats = nullptr;
  int* flag = nullptr;
  double last_loop_ms = 0.0, last_step_ms = 0.0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // cached HIP graph of the step loop, valid for the run parameters in graph_key
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  double graph_key[15] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  // ---- Section 6 variants
  // Symmetric plan (Algorithm 2): one square symmetric matrix; the row entries are also
  // stored with indices into the rows' own internal order, and a step is one launch.
  bool symmetric = false;
  int2* ent_sym = nullptr;
  // Varying norms: per-index squared targets, original and internal order (rows, cols).
  double* tgt_orig[2] = {nullptr, nullptr};
  double* tgt_int[2] = {nullptr, nullptr};
  // Block equilibration (single-matrix plans): per side, block offsets and state.
  struct BlockSide {
    int64_t nb = 0;                      // 0: no blocks on this side
    int32_t group = 64;                  // lanes per block in the block kernels
    int64_t* ptr = nullptr;              // [nb + 1] on the device
    double* tgt = nullptr;               // [nb]
    double* bx = nullptr;                // [nb]
    double* bxbar = nullptr;             // [nb]
    double* z = nullptr;                 // [nint]
  } blk[2];
  int64_t variant_epoch = 0;             // bumped by every variant setting (graph key)
};

namespace mfe {

int plan_build(const mfe_matrix* mats, int32_t count, int32_t max_probes, hipStream_t s,
               mfe_plan** out);
void plan_free(mfe_plan* p);
// trace_every > 0 runs the step loop eagerly in chunks of trace_every steps and calls
// on_chunk(t) after each chunk (the residual trace); chunk times are summed.
int plan_run(mfe_plan* p, const mfe_equil_params* prm, const double* alpha_b, const double* beta_b,
             int use_graph, double* d, double* e, double* u_bar, double* v_bar, int trace_every = 0,
             int (*on_chunk)(void* ctx, int t) = nullptr, void* ctx = nullptr);
// Times trial_steps steps of every launch configuration (loads in flight per lane;
// two-part directions where the plan has them) with the run parameters prm and keeps
// the fastest in the plan.  chosen[0..2] = batch, two-part rows, two-part columns.
int plan_autotune(mfe_plan* p, const mfe_equil_params* prm, const double* alpha_b, const double* beta_b,
                  int32_t trial_steps, int32_t* chosen, double* best_step_ms, int32_t* n_candidates);
int plan_equilibrate_trace(mfe_plan* p, const mfe_equil_params* prm, int32_t trace_every, double* rms_trace,
                           double* d, double* e, double* u_bar, double* v_bar);
int plan_sketch_features(mfe_plan* p, uint64_t seed, int32_t ks, const double* alpha_b, const double* beta_b,
                         double gamma, double M, float* feat_rows, float* feat_cols, double* u_sketch,
                         double* v_sketch, hipStream_t st);
int plan_warmstart(mfe_plan* p, const float* params, uint64_t seed, int32_t ks, const double* alpha_b,
                   const double* beta_b, double gamma, double M, int learned, double* u0, double* v0,
                   hipStream_t st);
int plan_training_set(mfe_plan* p, uint64_t seed, int32_t ks, const double* alpha_b, const double* beta_b,
                      double gamma, double M, const double* u_label, const double* v_label, int64_t per_matrix,
                      uint64_t sample_seed, float* X, float* t, int64_t* idx, int64_t* count, hipStream_t st);
int mlp_forward(const float* params, const float* X, int64_t count, float* y, hipStream_t st);
int mlp_train(float* params, float* adam_m, float* adam_v, int32_t step0, const float* X, const float* t,
              int64_t total, int64_t batch, int32_t iters, float lr, uint64_t seed, double* loss_trace,
              hipStream_t st);
int mlp_grad(const float* params, const float* X, const float* t, int64_t count, float* grad, double* loss,
             hipStream_t st);
int warmstart_apply(int64_t n, const double* sketch, const float* delta, double M, double* out, hipStream_t st);
int mlp_param_count();
int mlp_feature_count();
int plan_lsqr(mfe_plan* p, const double* b, const double* d, const double* e, double tol,
              int32_t max_iter, int32_t check_every, double* x, mfe_lsqr_info* info, hipStream_t s);
int plan_residual(mfe_plan* p, const double* d, const double* e, double alpha, double beta,
                  double* rms, double* rms_nonempty, int64_t* n_empty, hipStream_t s);
// Consumer of Section 5.2: CCP on the Lasso, and ||D A E||_2 by power iteration.
int plan_op_norm(mfe_plan* p, const double* d, const double* e, int32_t max_iter, double tol, double* norm,
                 int32_t* iters, hipStream_t s);
int plan_ccp_lasso(mfe_plan* p, const double* b, const double* d, const double* e, double lam, double op_norm,
                   int32_t iters, int32_t trace_every, double* trace, double* x, mfe_ccp_info* info, hipStream_t s);
// Section 6 variants.
int plan_build_symmetric(const mfe_matrix* A, int32_t max_probes, hipStream_t s, mfe_plan** out);
int plan_set_targets(mfe_plan* p, const double* row_target, const double* col_target, hipStream_t s);
int plan_set_blocks(mfe_plan* p, const int64_t* row_ptr, int64_t nrb, const int64_t* col_ptr, int64_t ncb,
                    hipStream_t s);
void plan_free_variants(mfe_plan* p);
inline bool plan_has_variant(const mfe_plan* p) {
  return p->symmetric || p->tgt_int[0] || p->tgt_int[1] || p->blk[0].nb || p->blk[1].nb;
}

// Makes sure the per-matrix device table exists (original-index bases are all that
// LSQR and the residual need from it).
int ensure_mats(mfe_plan* p, hipStream_t s);

// Launches the fused sign-generation for one step into `out` (all segments).
int launch_signgen(const SignGenDev& g, hipStream_t s);

}  // namespace mfe
