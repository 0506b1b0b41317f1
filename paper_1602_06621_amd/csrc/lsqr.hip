// LSQR on the equilibrated system (Section 5.1) and the RMS equilibration error
// (Section 4), for the sparse layouts of a plan and for dense FP64 matrices.
//
// LSQR is the Golub-Kahan bidiagonalisation method of Paige & Saunders applied to
// Abar = D A E, bbar = D b; x = E xbar.  Every iteration is one product with Abar and
// one with Abar' (the cost unit of Section 5.1).  Vectors and recurrences are FP64;
// reductions are two-stage (per-block partials, then one block in a fixed order), so
// results are deterministic.  The scalar recurrence runs on the device; the host only
// reads the scalars at the residual checks.
#include <cmath>
#include <new>
#include <vector>

#include "dense.h"
#include "sparse.h"

namespace mfe {
namespace {

constexpr int kRed = 256;  // threads of the product / reduction kernels

// Device scalars of one LSQR run.
// The bidiagonalisation vectors are kept unnormalised: the row vector p = beta u and the
// column vector q = alpha v, so that no pass over them is needed to divide by a norm; the
// products take the normalisations in their coefficients:
//   p_{i+1} = D A E q_i / alpha_i - (alpha_i / beta_i) p_i        (= beta_{i+1} u_{i+1})
//   q_{i+1} = E A' D p_{i+1} / beta_{i+1} - (beta_{i+1} / alpha_i) q_i  (= alpha_{i+1} v_{i+1})
struct LsqrScal {
  double alpha, beta;          // current alpha_i, beta_{i+1}
  double rhobar, phibar;       // rotation state
  double phi_rho, theta_rho;   // update coefficients of x and w
  double anorm2;               // Frobenius estimate of ||Abar||^2
  double normal_eq;            // ||Abar' r|| / (||Abar|| ||r||) estimate
  double inv_beta, inv_alpha;  // 1 / beta, 1 / alpha (0 when the norm is 0)
  double coef_p, coef_q;       // -alpha_i / beta_i and -beta_{i+1} / alpha_i above
  double bnorm2, res2;         // ||b||^2 and ||A x - b||^2 at the last check
  double neg_one;
  int breakdown;               // iteration at which alpha or beta became 0 (0: none)
  int iter;
};

// Sum of the NT doubles of a block of NT threads, fixed order (tree in LDS).
template <int NT = kRed>
__device__ double block_sum(double v) {
  __shared__ double sh[NT];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// beta_{i+1} = ||p_{i+1}|| (t = ||p_{i+1}||^2).  next_iter != 0 starts the next iteration
// (the count is kept on the device, so that every iteration is the same launches).
__device__ void beta_step(LsqrScal* sc, double t, int next_iter) {
  if (next_iter) sc->iter += 1;
  const double beta = sqrt(t);
  sc->beta = beta;
  sc->anorm2 += sc->alpha * sc->alpha + beta * beta;
  sc->inv_beta = beta > 0.0 ? 1.0 / beta : 0.0;
  sc->coef_q = -beta * sc->inv_alpha;
  if (beta == 0.0 && sc->breakdown == 0) sc->breakdown = sc->iter;
}

// alpha_{i+1} = ||q_{i+1}|| (t = its square) and the plane rotation.  init != 0 is the
// start of the method (alpha_1 v_1 = Abar' u_1, phibar = beta_1, rhobar = alpha_1).
__device__ void alpha_step(LsqrScal* sc, double t, int init) {
  const double an = sqrt(t);
  sc->inv_alpha = an > 0.0 ? 1.0 / an : 0.0;
  sc->coef_p = -an * sc->inv_beta;
  if (init) {
    sc->phibar = sc->beta;
    sc->rhobar = an;
    sc->alpha = an;
    sc->anorm2 = 0.0;
    if (an == 0.0 && sc->breakdown == 0) sc->breakdown = -1;
    return;
  }
  if (sc->breakdown == 0 || sc->breakdown == sc->iter) {
    const double beta = sc->beta;
    const double rho = hypot(sc->rhobar, beta);
    const double c = sc->rhobar / rho, sn = beta / rho;
    const double theta = sn * an;
    sc->rhobar = -c * an;
    const double phi = c * sc->phibar;
    sc->phibar = sn * sc->phibar;
    sc->phi_rho = phi / rho;
    sc->theta_rho = theta / rho;
    sc->normal_eq = an * fabs(c) / sqrt(sc->anorm2);
    if (an == 0.0) sc->breakdown = sc->iter;
  } else {
    sc->phi_rho = 0.0;  // after a breakdown x stays fixed
    sc->theta_rho = 0.0;
  }
  sc->alpha = an;
}

// x += phi/rho w; w = v_{i+1} - theta/rho w for column i, with v_{i+1} = q_{i+1} / alpha_{i+1}
// (init: w = v_1, x = 0); nothing after a breakdown of an earlier iteration.
__device__ __forceinline__ void lsqr_update_at(const LsqrScal* __restrict__ sc, int init, const double* __restrict__ q,
                                               double* __restrict__ w, double* __restrict__ x, int64_t i) {
  const bool frozen = sc->breakdown != 0 && sc->breakdown != sc->iter && !init;
  if (frozen) return;
  const double vi = q[i] * sc->inv_alpha;
  if (init) {
    w[i] = vi;
    x[i] = 0.0;
  } else {
    const double wi = w[i];
    x[i] += sc->phi_rho * wi;
    w[i] = vi - sc->theta_rho * wi;
  }
}

// The x / w update of the previous iteration, run by extra workgroups of the next
// iteration's row product (n = 0: none).  That launch reads and writes none of q, w, x,
// and the update's coefficients come from the alpha step before it.
struct TailUpdate {
  const LsqrScal* sc;
  const double* q;
  double* w;
  double* x;
  int64_t n;
};

// ---------------------------------------------------------------- sliced products
//
// A workgroup holds G groups of P wavefronts; group j takes slice G blockIdx + j (64
// rows), its wavefront w walking the slots [w c, (w+1) c) of every row of the slice
// (c = ceil(width / P)), and the group's first wavefront adding the P partial sums in
// order.  Plans with many slices run P = 1, G = 4 (one sequential sum per row); long rows
// in few slices (the Lasso of Section 5.2: 10,000 rows of ~200 entries are 157 slices)
// get P up to 16, so that thousands of wavefronts share the work instead of 157.
constexpr int kMaxSplit = 16;

struct SliceMap {
  int P, G;  // wavefronts per slice, slices per workgroup
};

// Wavefronts per slice for a direction with `nslices` slices: enough to give the device
// about 4096 wavefronts, at most kMaxSplit per slice; four slices per workgroup when one
// wavefront per slice suffices.
inline SliceMap slice_map(int64_t nslices) {
  const int64_t p = nslices > 0 ? ceil_div(4096, nslices) : 1;
  SliceMap m;
  m.P = (int)std::max<int64_t>(1, std::min<int64_t>(kMaxSplit, p));
  m.G = std::max(1, 4 / m.P);
  return m;
}

// sum over slots [q0, q1) of a_q f(a_q) g[idx_q] for one lane's row (f = 1, or a_q when
// SQ: the squared entries of the residual pass), in slot order.  One slot at a time:
// batching the entry loads and the gathers (4 or 8 slots in flight per lane, with or
// without non-temporal entry loads) was measured slower on the headline matrix (195-210
// against 173 us per LSQR iteration).
template <bool SQ>
__device__ __forceinline__ double row_dot(const int2* __restrict__ e, int q0, int q1, const double* __restrict__ g) {
  double acc = 0.0;
  for (int q = q0; q < q1; ++q) {
    const int2 en = e[(int64_t)q * kSlice];
    const double a = (double)__int_as_float(en.y);
    acc += SQ ? a * a * g[en.x] : a * g[en.x];
  }
  return acc;
}

// Slice taken by slice slot i of a launch (the layout's longest-first order when it has
// one); slots past the last slice stay out of range.
__device__ __forceinline__ int64_t launch_slice(const SideDev& S, int64_t i, int64_t nslices) {
  return (S.sched && i < nslices) ? (int64_t)S.sched[i] : i;
}

// Row sums sum_q a_q g[idx_q] of slice s for lane `lane`, returned in the group's first
// wavefront (wsub = 0; 0 elsewhere and for s >= nslices).  Every thread of the workgroup
// must call it (it has a barrier when P > 1).
__device__ double slice_row_sum(const SideDev& S, const double* __restrict__ g, int64_t s, int64_t nslices, int P,
                                int wave, int wsub, int lane) {
  __shared__ double part[kMaxSplit][kSlice];
  double acc = 0.0;
  if (s < nslices) {
    const int64_t base = S.slice_off[s];
    const int len = S.len[s * kSlice + lane];
    const int width = (int)((S.slice_off[s + 1] - base) / kSlice);
    const int chunk = (width + P - 1) / P;
    const int q0 = wsub * chunk, q1 = min(len, q0 + chunk);
    acc = row_dot<false>(S.ent + base + lane, q0, q1, g);
  }
  if (P == 1) return acc;
  part[wave][lane] = acc;
  __syncthreads();
  double tot = 0.0;
  if (wsub == 0)
    for (int i = 0; i < P; ++i) tot += part[wave + i][lane];
  return tot;
}

// y_r = sout_r * inv * sum_q a_q g[idx_q] + coef * yprev_r  over the rows r of one
// direction of a plan (internal order); gout_r = sout_r * y_r when requested; one
// partial of sum y_r^2 per workgroup.  inv and coef are read from device memory
// (nullable = 1, 0).  Grid: ceil(nslices / G) workgroups of 64 G P threads.
__global__ __launch_bounds__(kSlice * kMaxSplit) void k_sell_product(SideDev S, SliceMap sm,
                                                                     const double* __restrict__ sout,
                                                                     const double* __restrict__ g, const double* inv,
                                                                     const double* coef,
                                                                     const double* __restrict__ yprev,
                                                                     double* __restrict__ y, double* __restrict__ gout,
                                                                     double* __restrict__ partial, int64_t pblocks,
                                                                     TailUpdate tu) {
  __shared__ double gsum[kMaxSplit];
  if ((int64_t)blockIdx.x >= pblocks) {  // whole workgroups past the product: the tail update
    const int64_t i = ((int64_t)blockIdx.x - pblocks) * blockDim.x + threadIdx.x;
    if (i < tu.n) lsqr_update_at(tu.sc, 0, tu.q, tu.w, tu.x, i);
    return;
  }
  const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int wsub = wave % sm.P;
  const int64_t nslices = S.nint / kSlice;
  const int64_t s = launch_slice(S, (int64_t)blockIdx.x * sm.G + wave / sm.P, nslices);
  const double acc = slice_row_sum(S, g, s, nslices, sm.P, wave, wsub, lane);
  double contrib = 0.0;
  if (wsub == 0 && s < nslices) {
    const int64_t r = s * kSlice + lane;
    if (S.orig[r] >= 0) {
      const double so = sout ? sout[r] : 1.0;
      double v = so * (acc * (inv ? *inv : 1.0));
      if (coef) v += *coef * yprev[r];
      y[r] = v;
      if (gout) gout[r] = so * v;
      contrib = v * v;
    }
  }
  const double ws = wave_sum(contrib);
  if (lane == 0) gsum[wave] = ws;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < sm.G; ++i) t += gsum[i * sm.P];
    partial[blockIdx.x] = t;
  }
}

// RMS-residual pass over one direction: s_r = sum_q a_q^2 g2[idx_q] (g2 = squared scales
// of the other side), r_r = own2_r * s_r; partials of (sqrt(r) - target)^2 over all
// rows, over non-empty rows, and the count of empty rows.
__global__ __launch_bounds__(kRed) void k_sell_rownorm(SideDev S, const double* __restrict__ own2,
                                                       const double* __restrict__ g2, double target,
                                                       double* __restrict__ p_all, double* __restrict__ p_ne,
                                                       double* __restrict__ p_empty) {
  const int64_t r = (int64_t)blockIdx.x * kRed + threadIdx.x;
  double all = 0.0, ne = 0.0, em = 0.0;
  if (r < S.nint && S.orig[r] >= 0) {
    const int64_t s = r >> 6;
    const int lane = (int)(r & 63);
    const int len = S.len[r];
    const double acc = row_dot<true>(S.ent + S.slice_off[s] + lane, 0, len, g2);
    const double dev = sqrt((own2 ? own2[r] : 1.0) * acc) - target;
    all = dev * dev;
    if (len > 0) ne = all;
    else em = 1.0;
  }
  const double a = block_sum(all), b = block_sum(ne), c = block_sum(em);
  if (threadIdx.x == 0) {
    p_all[blockIdx.x] = a;
    p_ne[blockIdx.x] = b;
    p_empty[blockIdx.x] = c;
  }
}

// Original order <-> internal order of one direction.  op: 0 copy, 1 square.
__global__ void k_to_internal(SideDev S, const MatDev* __restrict__ mats, const double* __restrict__ src,
                              double fill, int op, double* __restrict__ dst) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= S.nint) return;
  const int32_t li = S.orig[r];
  if (li < 0) {
    dst[r] = 0.0;
    return;
  }
  const MatDev mt = mats[S.slice_mat[r >> 6]];
  const int64_t gi = (S.is_row ? mt.row_orig_base : mt.col_orig_base) + li;
  const double v = src ? src[gi] : fill;
  dst[r] = op == 1 ? v * v : v;
}

__global__ void k_from_internal(SideDev S, const MatDev* __restrict__ mats, const double* __restrict__ src,
                                const double* __restrict__ scale, double* __restrict__ dst) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= S.nint) return;
  const int32_t li = S.orig[r];
  if (li < 0) return;
  const MatDev mt = mats[S.slice_mat[r >> 6]];
  const int64_t gi = (S.is_row ? mt.row_orig_base : mt.col_orig_base) + li;
  dst[gi] = scale ? scale[r] * src[r] : src[r];
}

// ---------------------------------------------------------------- dense FP64 products
//
// Row-major A (m x n, leading dimension ld).  Forward: one wavefront per row.
__global__ __launch_bounds__(kRed) void k_dense_fwd(const double* __restrict__ A, int64_t m, int64_t n, int64_t ld,
                                                    const double* __restrict__ sout, const double* __restrict__ g,
                                                    const double* inv, const double* coef,
                                                    const double* __restrict__ yprev, double* __restrict__ y,
                                                    double* __restrict__ gout, double* __restrict__ partial) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (kRed / 64) + wave;
  double contrib = 0.0;
  if (i < m) {
    double acc = 0.0;
    for (int64_t j = lane; j < n; j += 64) acc += A[i * ld + j] * g[j];
    acc = wave_sum(acc);
    if (lane == 0) {
      const double so = sout ? sout[i] : 1.0;
      double v = so * (acc * (inv ? *inv : 1.0));
      if (coef) v += *coef * yprev[i];
      y[i] = v;
      if (gout) gout[i] = so * v;
      contrib = v * v;
    }
  }
  const double bs = block_sum(contrib);
  if (threadIdx.x == 0) partial[blockIdx.x] = bs;
}

// Transposed: one thread per column, coalesced across the columns of a row.
__global__ __launch_bounds__(kRed) void k_dense_bwd(const double* __restrict__ A, int64_t m, int64_t n, int64_t ld,
                                                    const double* __restrict__ sout, const double* __restrict__ g,
                                                    const double* inv, const double* coef,
                                                    const double* __restrict__ yprev, double* __restrict__ y,
                                                    double* __restrict__ gout, double* __restrict__ partial) {
  const int64_t j = (int64_t)blockIdx.x * kRed + threadIdx.x;
  double contrib = 0.0;
  if (j < n) {
    double acc = 0.0;
    for (int64_t i = 0; i < m; ++i) acc += A[i * ld + j] * g[i];
    const double so = sout ? sout[j] : 1.0;
    double v = so * (acc * (inv ? *inv : 1.0));
    if (coef) v += *coef * yprev[j];
    y[j] = v;
    if (gout) gout[j] = so * v;
    contrib = v * v;
  }
  const double bs = block_sum(contrib);
  if (threadIdx.x == 0) partial[blockIdx.x] = bs;
}

// Dense residual passes (squared entries).
__global__ __launch_bounds__(kRed) void k_dense_rownorm(const double* __restrict__ A, int64_t m, int64_t n, int64_t ld,
                                                        int trans, const double* __restrict__ own, const double* __restrict__ other,
                                                        double target, double* p_all, double* p_ne, double* p_empty) {
  const int64_t i = (int64_t)blockIdx.x * kRed + threadIdx.x;
  const int64_t cnt = trans ? n : m, len = trans ? m : n;
  double all = 0.0, ne = 0.0, em = 0.0;
  if (i < cnt) {
    double acc = 0.0;
    int64_t nz = 0;
    for (int64_t q = 0; q < len; ++q) {
      const double a = trans ? A[q * ld + i] : A[i * ld + q];
      const double o = other ? other[q] : 1.0;
      acc += a * a * o * o;
      nz += (a != 0.0);
    }
    const double w = own ? own[i] : 1.0;
    const double dev = sqrt(w * w * acc) - target;
    all = dev * dev;
    if (nz > 0) ne = all;
    else em = 1.0;
  }
  const double a = block_sum(all), b = block_sum(ne), c = block_sum(em);
  if (threadIdx.x == 0) {
    p_all[blockIdx.x] = a;
    p_ne[blockIdx.x] = b;
    p_empty[blockIdx.x] = c;
  }
}

// ---------------------------------------------------------------- reductions + scalars

// out[0] = sum of partial[0..n) in a fixed order.
__global__ __launch_bounds__(kRed) void k_reduce(const double* __restrict__ partial, int64_t n, double* out) {
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kRed) s += partial[i];
  const double t = block_sum(s);
  if (threadIdx.x == 0) *out = t;
}

// First stage of a long sum: one partial per block of kRed values.
__global__ __launch_bounds__(kRed) void k_block_partials(const double* __restrict__ v, int64_t n,
                                                         double* __restrict__ partial) {
  const int64_t i = (int64_t)blockIdx.x * kRed + threadIdx.x;
  const double t = block_sum(i < n ? v[i] : 0.0);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// out = sum of v[0..n) in a fixed order, in two stages (scratch: ceil(n / kRed) values).
void reduce_long(const double* v, int64_t n, double* scratch, double* out, hipStream_t st) {
  const int64_t nb = ceil_div(n, kRed);
  k_block_partials<<<dim3((unsigned)std::max<int64_t>(nb, 1)), dim3(kRed), 0, st>>>(v, n, scratch);
  k_reduce<<<1, kRed, 0, st>>>(scratch, nb, out);
}

// The scalar step after a product, over that product's n per-workgroup partial sums of
// y^2 (one workgroup, fixed order): kind 1 the beta step (flag: count a new iteration),
// kind 2 the alpha step and rotation (flag: the start of the method).  A separate launch:
// folding it into the product's last workgroup needs a device-scope release per
// workgroup, which writes back the L2 of every XCD and measured 362 us per iteration
// against 150.
constexpr int kScal = 1024;
__global__ __launch_bounds__(kScal) void k_scal_step(const double* __restrict__ partial, int64_t n, LsqrScal* sc,
                                                     int kind, int flag) {
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kScal) s += partial[i];
  const double t = block_sum<kScal>(s);
  if (threadIdx.x == 0) {
    if (kind == 1) beta_step(sc, t, flag);
    else alpha_step(sc, t, flag);
  }
}

// Elementwise over the columns, after the alpha step: v_{i+1} = q_{i+1} / alpha_{i+1},
// x += phi/rho w; w = v_{i+1} - theta/rho w.  init: w = v_1, x = 0.
__global__ void k_lsqr_update(int64_t ncol, const LsqrScal* __restrict__ sc, int init, const double* __restrict__ q,
                              double* __restrict__ w, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ncol) lsqr_update_at(sc, init, q, w, x, i);
}

// y = escale (x + phi/rho w): the solution with the pending update of the last iteration
// (the one the next row product would apply), for the residual checks.
__global__ void k_x_pending(int64_t ncol, const LsqrScal* __restrict__ sc, const double* __restrict__ escale,
                            const double* __restrict__ x, const double* __restrict__ w, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncol) return;
  const bool frozen = sc->breakdown != 0 && sc->breakdown != sc->iter;
  const double xi = frozen ? x[i] : x[i] + sc->phi_rho * w[i];
  y[i] = (escale ? escale[i] : 1.0) * xi;
}

__global__ void k_scal_init(LsqrScal* sc) {
  LsqrScal z;
  z.alpha = z.beta = z.rhobar = z.phibar = z.phi_rho = z.theta_rho = 0.0;
  z.anorm2 = z.normal_eq = z.coef_p = z.coef_q = 0.0;
  z.inv_beta = z.inv_alpha = 1.0;
  z.bnorm2 = z.res2 = 0.0;
  z.neg_one = -1.0;
  z.breakdown = 0;
  z.iter = 0;
  *sc = z;
}


__global__ void k_mul(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (a ? a[i] : 1.0) * b[i];
}

// ---------------------------------------------------------------- operator abstraction

struct Work {
  std::vector<void*> bufs;
  ~Work() {
    for (void* p : bufs) (void)hipFree(p);
  }
  template <class T>
  int alloc(T** p, int64_t n) {
    hipError_t e = hipMalloc((void**)p, sizeof(T) * (size_t)std::max<int64_t>(n, 1));
    if (e != hipSuccess)
      return set_error(e == hipErrorOutOfMemory ? MFE_ENOMEM : MFE_EDEVICE, "hipMalloc failed: %s",
                       hipGetErrorString(e));
    bufs.push_back(*p);
    return MFE_OK;
  }
};

// Products y = sout * inv * (A or A') g + coef * yprev, with partial sums of y^2; the row
// product also runs a pending LSQR x / w update (TailUpdate) in the same stream order.
struct Ops {
  virtual ~Ops() {}
  virtual int64_t rows() const = 0;  // length of row-direction vectors
  virtual int64_t cols() const = 0;
  virtual int64_t fwd_blocks() const = 0;
  virtual int64_t bwd_blocks() const = 0;
  virtual void fwd(const double* sout, const double* g, const double* inv, const double* coef, const double* yprev,
                   double* y, double* gout, double* partial, const TailUpdate& tu, hipStream_t st) const = 0;
  virtual void bwd(const double* sout, const double* g, const double* inv, const double* coef, const double* yprev,
                   double* y, double* gout, double* partial, hipStream_t st) const = 0;
  // original <-> operator order
  virtual void to_op(bool row, const double* src, double fill, int op, double* dst, hipStream_t st) const = 0;
  virtual void from_op(bool row, const double* src, const double* scale, double* dst, hipStream_t st) const = 0;
  virtual const int32_t* col_valid() const { return nullptr; }
};

struct SellOps : Ops {
  mfe_plan* p;
  SideDev R, C;
  explicit SellOps(mfe_plan* plan) : p(plan) {
    R = SideDev{};
    C = SideDev{};
    R.slice_off = p->rows.slice_off;
    R.slice_mat = p->rows.slice_mat;
    R.len = p->rows.len;
    R.orig = p->rows.orig;
    R.ent = p->rows.ent;
    R.nint = p->rows.nint;
    R.sched = p->rows.sched;
    R.is_row = 1;
    C.slice_off = p->cols.slice_off;
    C.slice_mat = p->cols.slice_mat;
    C.len = p->cols.len;
    C.orig = p->cols.orig;
    C.ent = p->cols.ent;
    C.nint = p->cols.nint;
    C.sched = p->cols.sched;
    C.is_row = 0;
    MR = slice_map(p->rows.nslices);
    MC = slice_map(p->cols.nslices);
  }
  int64_t rows() const override { return p->rows.nint; }
  int64_t cols() const override { return p->cols.nint; }
  SliceMap MR{1, 4}, MC{1, 4};  // slice maps of the two directions
  int64_t fwd_blocks() const override { return ceil_div(p->rows.nslices, MR.G); }
  int64_t bwd_blocks() const override { return ceil_div(p->cols.nslices, MC.G); }
  void fwd(const double* sout, const double* g, const double* inv, const double* coef, const double* yprev, double* y,
           double* gout, double* partial, const TailUpdate& tu, hipStream_t st) const override {
    const int threads = kSlice * MR.P * MR.G;
    const int64_t pb = fwd_blocks(), tb = ceil_div(tu.n, threads);
    k_sell_product<<<dim3((unsigned)(pb + tb)), dim3(threads), 0, st>>>(R, MR, sout, g, inv, coef, yprev, y, gout,
                                                                        partial, pb, tu);
  }
  void bwd(const double* sout, const double* g, const double* inv, const double* coef, const double* yprev, double* y,
           double* gout, double* partial, hipStream_t st) const override {
    k_sell_product<<<dim3((unsigned)bwd_blocks()), dim3(kSlice * MC.P * MC.G), 0, st>>>(C, MC, sout, g, inv, coef,
                                                                                          yprev, y, gout, partial,
                                                                                          bwd_blocks(), TailUpdate{});
  }
  void to_op(bool row, const double* src, double fill, int op, double* dst, hipStream_t st) const override {
    const SideDev& S = row ? R : C;
    k_to_internal<<<dim3((unsigned)ceil_div(S.nint, 256)), dim3(256), 0, st>>>(S, p->mats, src, fill, op, dst);
  }
  void from_op(bool row, const double* src, const double* scale, double* dst, hipStream_t st) const override {
    const SideDev& S = row ? R : C;
    k_from_internal<<<dim3((unsigned)ceil_div(S.nint, 256)), dim3(256), 0, st>>>(S, p->mats, src, scale, dst);
  }
  const int32_t* col_valid() const override { return p->cols.orig; }
};

__global__ void k_copy_scaled(int64_t n, const double* __restrict__ src, double fill, int op, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = src ? src[i] : fill;
  dst[i] = op == 1 ? v * v : v;
}

__global__ void k_mul_into(int64_t n, const double* __restrict__ src, const double* __restrict__ scale,
                           double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = scale ? scale[i] * src[i] : src[i];
}

struct DenseOps : Ops {
  const double* A;
  int64_t m, n, ld;
  DenseOps(const double* a, int64_t m_, int64_t n_, int64_t ld_) : A(a), m(m_), n(n_), ld(ld_) {}
  int64_t rows() const override { return m; }
  int64_t cols() const override { return n; }
  int64_t fwd_blocks() const override { return ceil_div(m, kRed / 64); }
  int64_t bwd_blocks() const override { return ceil_div(n, kRed); }
  void fwd(const double* sout, const double* g, const double* inv, const double* coef, const double* yprev, double* y,
           double* gout, double* partial, const TailUpdate& tu, hipStream_t st) const override {
    if (tu.n > 0)
      k_lsqr_update<<<dim3((unsigned)ceil_div(tu.n, 256)), dim3(256), 0, st>>>(tu.n, tu.sc, 0, tu.q, tu.w, tu.x);
    k_dense_fwd<<<dim3((unsigned)fwd_blocks()), dim3(kRed), 0, st>>>(A, m, n, ld, sout, g, inv, coef, yprev, y, gout,
                                                                     partial);
  }
  void bwd(const double* sout, const double* g, const double* inv, const double* coef, const double* yprev, double* y,
           double* gout, double* partial, hipStream_t st) const override {
    k_dense_bwd<<<dim3((unsigned)bwd_blocks()), dim3(kRed), 0, st>>>(A, m, n, ld, sout, g, inv, coef, yprev, y, gout,
                                                                     partial);
  }
  void to_op(bool row, const double* src, double fill, int op, double* dst, hipStream_t st) const override {
    const int64_t cnt = row ? m : n;
    k_copy_scaled<<<dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, st>>>(cnt, src, fill, op, dst);
  }
  void from_op(bool row, const double* src, const double* scale, double* dst, hipStream_t st) const override {
    const int64_t cnt = row ? m : n;
    k_mul_into<<<dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, st>>>(cnt, src, scale, dst);
  }
};

// LSQR driver over any Ops (see the stopping rule in mfe.h).
// A captured graph and its capture stream, released on every return path.
struct GraphHolder {
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int iters = 0;  // iterations in the captured block
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
    exec = nullptr;
    graph = nullptr;
    cap = nullptr;
    iters = 0;
  }
  ~GraphHolder() { reset(); }
};

// Device vectors of one LSQR run (rows nr, columns nc, pb reduction partials).
struct LsqrBufs {
  double *bb, *dd, *ee, *u, *du, *v, *w, *x, *ev, *res, *part, *w_tmp;
  LsqrScal* sc;
  int alloc(Work& W, int64_t nr, int64_t nc, int64_t pb) {
    MFE_CHECK(W.alloc(&w_tmp, nc));
    MFE_CHECK(W.alloc(&bb, nr));
    MFE_CHECK(W.alloc(&dd, nr));
    MFE_CHECK(W.alloc(&ee, nc));
    MFE_CHECK(W.alloc(&u, nr));
    MFE_CHECK(W.alloc(&du, nr));
    MFE_CHECK(W.alloc(&v, nc));
    MFE_CHECK(W.alloc(&w, nc));
    MFE_CHECK(W.alloc(&x, nc));
    MFE_CHECK(W.alloc(&ev, nc));
    MFE_CHECK(W.alloc(&res, nr));
    MFE_CHECK(W.alloc(&part, pb));
    MFE_CHECK(W.alloc(&sc, 1));
    return MFE_OK;
  }
};

// Iterations per captured block: a block between two residual checks is replayed as
// whole graphs of at most this many iterations, the rest of it launched eagerly.
constexpr int kLsqrGraphIters = 25;

}  // namespace

// A plan's LSQR workspace and captured iteration block, kept between calls: the plan's
// layouts, and so every pointer the graph holds, are fixed for the plan's lifetime, and a
// call rewrites every vector it reads before reading it.
struct LsqrCache {
  int64_t nr = -1, nc = -1, pb = -1;
  Work W;
  LsqrBufs B;
  GraphHolder G;
};

void free_lsqr_cache(LsqrCache* c) { delete c; }

namespace {

int run_lsqr(const Ops& ops, const double* b, const double* d, const double* e, double tol, int32_t max_iter,
             int32_t check_every, double* x_out, mfe_lsqr_info* info, hipStream_t st, LsqrCache* cache = nullptr) {
  const int64_t nr = ops.rows(), nc = ops.cols();
  const int64_t pb = std::max(ops.fwd_blocks(), ops.bwd_blocks()) + ceil_div(nr, kRed) + 1;
  // Vectors and the captured block: the plan's cache when given (allocated on its first
  // use), else this call's own.
  Work Wl;
  GraphHolder Gl;
  LsqrBufs B;
  GraphHolder* Gp = &Gl;
  if (cache) {
    if (cache->nr != nr || cache->nc != nc || cache->pb != pb) {
      Work fresh;
      LsqrBufs nb;
      MFE_CHECK(nb.alloc(fresh, nr, nc, pb));
      cache->G.reset();
      for (void* q : cache->W.bufs) (void)hipFree(q);
      cache->W.bufs.swap(fresh.bufs);
      cache->B = nb;
      cache->nr = nr;
      cache->nc = nc;
      cache->pb = pb;
    }
    B = cache->B;
    Gp = &cache->G;
  } else {
    MFE_CHECK(B.alloc(Wl, nr, nc, pb));
  }
  GraphHolder& G = *Gp;
  double *bb = B.bb, *dd = B.dd, *ee = B.ee, *u = B.u, *du = B.du, *v = B.v, *w = B.w, *x = B.x, *ev = B.ev,
         *res = B.res, *part = B.part, *w_tmp = B.w_tmp;
  LsqrScal* sc = B.sc;
  for (double* z : {u, du, res}) MFE_HIP(hipMemsetAsync(z, 0, sizeof(double) * nr, st));
  for (double* z : {v, w, x, ev}) MFE_HIP(hipMemsetAsync(z, 0, sizeof(double) * nc, st));
  ops.to_op(true, b, 0.0, 0, bb, st);
  ops.to_op(true, d, 1.0, 0, dd, st);
  ops.to_op(false, e, 1.0, 0, ee, st);
  k_scal_init<<<1, 1, 0, st>>>(sc);
  const unsigned upd_grid = (unsigned)ceil_div(nc, 256);
  const unsigned row_grid = (unsigned)ceil_div(nr, 256);
  // ||b||^2 for the relative residual of the original system
  k_mul<<<row_grid, 256, 0, st>>>(nr, bb, bb, res);
  reduce_long(res, nr, part, &sc->bnorm2, st);
  // start: p_1 = D b (= beta_1 u_1), q_1 = E A' D p_1 / beta_1 (= alpha_1 v_1)
  k_mul<<<row_grid, 256, 0, st>>>(nr, dd, bb, u);   // p_1
  k_mul<<<row_grid, 256, 0, st>>>(nr, dd, u, du);   // D p_1, gathered by the transposed product
  k_mul<<<row_grid, 256, 0, st>>>(nr, u, u, res);
  reduce_long(res, nr, part + ceil_div(nr, kRed), part, st);
  k_scal_step<<<1, kScal, 0, st>>>(part, 1, sc, 1, 0);
  ops.bwd(ee, du, &sc->inv_beta, nullptr, nullptr, v, ev, part, st);
  k_scal_step<<<1, kScal, 0, st>>>(part, ops.bwd_blocks(), sc, 2, 1);
  k_lsqr_update<<<upd_grid, 256, 0, st>>>(nc, sc, 1, v, w, x);
  MFE_HIP(hipGetLastError());

  LsqrScal h;
  MFE_HIP(hipMemcpyAsync(&h, sc, sizeof h, hipMemcpyDeviceToHost, st));
  MFE_HIP(hipStreamSynchronize(st));
  const double bnorm = std::sqrt(h.bnorm2);
  mfe_lsqr_info inf;
  inf.iters = 0;
  inf.stop_reason = 0;
  inf.rel_resid = bnorm > 0 ? 1.0 : 0.0;
  inf.normal_eq = 0.0;
  if (bnorm == 0.0 || h.beta == 0.0 || h.breakdown != 0) {
    MFE_HIP(hipMemsetAsync(x, 0, sizeof(double) * nc, st));
    inf.stop_reason = 3;
    max_iter = 0;
  }
  // One iteration: four launches with no host involvement.  The x / w update of an
  // iteration runs in the next iteration's row product (at the first iteration its
  // coefficients are zero and it rewrites w = v_1); the residual checks read x with the
  // pending update added, and the last one is applied after the loop.
  const TailUpdate tail{sc, v, w, x, nc};
  auto iteration = [&](hipStream_t s) {
    // p_{i+1} = D A (E q_i) / alpha_i - (alpha_i / beta_i) p_i, du = D p_{i+1} (and the
    // previous iteration's x / w update); then beta and the iteration count
    ops.fwd(dd, ev, &sc->inv_alpha, &sc->coef_p, u, u, du, part, tail, s);
    k_scal_step<<<1, kScal, 0, s>>>(part, ops.fwd_blocks(), sc, 1, 1);
    // q_{i+1} = E A' du / beta_{i+1} - (beta_{i+1} / alpha_i) q_i, ev = E q_{i+1}; then
    // alpha and the rotation
    ops.bwd(ee, du, &sc->inv_beta, &sc->coef_q, v, v, ev, part, s);
    k_scal_step<<<1, kScal, 0, s>>>(part, ops.bwd_blocks(), sc, 2, 0);
  };
  // The iterations between two residual checks are replayed as whole captured blocks of
  // g iterations (the launches are identical from one block to the next), the rest
  // eagerly; the block is captured once per call, or once per plan.
  const int g = std::min<int>(check_every, kLsqrGraphIters);
  for (int it = 1; it <= max_iter;) {
    const int block_end =
        (int)std::min<int64_t>(max_iter, ((int64_t)(it - 1) / check_every + 1) * (int64_t)check_every);
    const int nblk = block_end - it + 1;
    int done = 0;
    if (g > 1 && nblk >= g) {
      if (!G.exec || G.iters != g) {
        G.reset();
        MFE_HIP(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
        MFE_HIP(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < g; ++i) iteration(G.cap);
        MFE_HIP(hipStreamEndCapture(G.cap, &G.graph));
        MFE_HIP(hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0));
        G.iters = g;
      }
      for (; done + g <= nblk; done += g) MFE_HIP(hipGraphLaunch(G.exec, st));
    }
    for (; done < nblk; ++done) iteration(st);
    MFE_HIP(hipGetLastError());
    it = block_end + 1;
    {
      // residual of the original system: A (E xbar) - b, reduced over the rows
      k_x_pending<<<dim3((unsigned)ceil_div(nc, 256)), dim3(256), 0, st>>>(nc, sc, ee, x, w, w_tmp);
      ops.fwd(nullptr, w_tmp, nullptr, &sc->neg_one, bb, res, nullptr, part, TailUpdate{}, st);
      k_reduce<<<1, kRed, 0, st>>>(part, ops.fwd_blocks(), &sc->res2);
      MFE_HIP(hipGetLastError());
      MFE_HIP(hipMemcpyAsync(&h, sc, sizeof h, hipMemcpyDeviceToHost, st));
      MFE_HIP(hipStreamSynchronize(st));
      const double rel = std::sqrt(h.res2) / bnorm;
      inf.iters = h.breakdown > 0 ? h.breakdown : block_end;
      inf.rel_resid = rel;
      inf.normal_eq = h.normal_eq;
      if (rel <= tol) {
        inf.stop_reason = 1;
        break;
      }
      if (h.normal_eq <= tol) {
        inf.stop_reason = 2;
        break;
      }
      if (h.breakdown != 0) {
        inf.stop_reason = 3;
        break;
      }
    }
  }
  k_lsqr_update<<<upd_grid, 256, 0, st>>>(nc, sc, 0, v, w, x);  // the last iteration's update
  ops.from_op(false, x, ee, x_out, st);
  MFE_HIP(hipGetLastError());
  MFE_HIP(hipStreamSynchronize(st));
  if (info) *info = inf;
  return MFE_OK;
}

int run_residual_sell(mfe_plan* p, const double* d, const double* e, double alpha, double beta, double* rms,
                      double* rms_nonempty, int64_t* n_empty, hipStream_t st) {
  SellOps ops(p);
  Work W;
  double *d2, *e2, *pa, *pn, *pe, *out;
  const int64_t nr = p->rows.nint, nc = p->cols.nint;
  const int64_t br = ceil_div(nr, kRed), bc = ceil_div(nc, kRed);
  MFE_CHECK(W.alloc(&d2, nr));
  MFE_CHECK(W.alloc(&e2, nc));
  MFE_CHECK(W.alloc(&pa, br + bc));
  MFE_CHECK(W.alloc(&pn, br + bc));
  MFE_CHECK(W.alloc(&pe, br + bc));
  MFE_CHECK(W.alloc(&out, 3));
  ops.to_op(true, d, 1.0, 1, d2, st);
  ops.to_op(false, e, 1.0, 1, e2, st);
  k_sell_rownorm<<<dim3((unsigned)br), dim3(kRed), 0, st>>>(ops.R, d2, e2, alpha, pa, pn, pe);
  k_sell_rownorm<<<dim3((unsigned)bc), dim3(kRed), 0, st>>>(ops.C, e2, d2, beta, pa + br, pn + br, pe + br);
  k_reduce<<<1, kRed, 0, st>>>(pa, br + bc, out);
  k_reduce<<<1, kRed, 0, st>>>(pn, br + bc, out + 1);
  k_reduce<<<1, kRed, 0, st>>>(pe, br + bc, out + 2);
  MFE_HIP(hipGetLastError());
  double h[3];
  MFE_HIP(hipMemcpyAsync(h, out, sizeof h, hipMemcpyDeviceToHost, st));
  MFE_HIP(hipStreamSynchronize(st));
  const double total = (double)(p->M + p->N);
  const int64_t ne = (int64_t)llround(h[2]);
  if (rms) *rms = std::sqrt(h[0] / total);
  if (rms_nonempty) *rms_nonempty = total - ne > 0 ? std::sqrt(h[1] / (total - ne)) : 0.0;
  if (n_empty) *n_empty = ne;
  return MFE_OK;
}

__global__ void k_exp2(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = exp(2.0 * x[i]);
}

struct TraceCtx {
  mfe_plan* p;
  SideDev R, C;
  double alpha, beta;
  double *d2, *e2, *pa, *pn, *pe, *out;
  int64_t br, bc;
  double* trace;
  int idx;
  hipStream_t st;
};

// RMS equilibration error (Section 4) of the current averages, appended to the trace.
int trace_chunk(void* c, int /*t*/) {
  TraceCtx* x = (TraceCtx*)c;
  mfe_plan* p = x->p;
  k_exp2<<<dim3((unsigned)ceil_div(p->rows.nint, 256)), dim3(256), 0, x->st>>>(p->rows.nint, p->xbar_row, x->d2);
  k_exp2<<<dim3((unsigned)ceil_div(p->cols.nint, 256)), dim3(256), 0, x->st>>>(p->cols.nint, p->xbar_col, x->e2);
  k_sell_rownorm<<<dim3((unsigned)x->br), dim3(kRed), 0, x->st>>>(x->R, x->d2, x->e2, x->alpha, x->pa, x->pn, x->pe);
  k_sell_rownorm<<<dim3((unsigned)x->bc), dim3(kRed), 0, x->st>>>(x->C, x->e2, x->d2, x->beta, x->pa + x->br,
                                                                 x->pn + x->br, x->pe + x->br);
  k_reduce<<<1, kRed, 0, x->st>>>(x->pa, x->br + x->bc, x->out);
  MFE_HIP(hipGetLastError());
  double h = 0.0;
  MFE_HIP(hipMemcpyAsync(&h, x->out, sizeof(double), hipMemcpyDeviceToHost, x->st));
  MFE_HIP(hipStreamSynchronize(x->st));
  x->trace[x->idx++] = std::sqrt(h / (double)(p->M + p->N));
  return MFE_OK;
}

}  // namespace

int plan_equilibrate_trace(mfe_plan* p, const mfe_equil_params* prm, int32_t trace_every, double* rms_trace,
                           double* d, double* e, double* u_bar, double* v_bar) {
  if (p->count != 1) return set_error(MFE_EUNSUPPORTED, "the residual trace needs a single-matrix plan");
  if (trace_every < 1 || !rms_trace) return set_error(MFE_EINVAL, "trace_every >= 1 and a trace buffer are required");
  MFE_CHECK(ensure_mats(p, (hipStream_t)prm->stream));
  SellOps ops(p);
  Work W;
  TraceCtx c;
  c.p = p;
  c.R = ops.R;
  c.C = ops.C;
  c.alpha = prm->alpha;
  c.beta = prm->beta;
  c.br = ceil_div(p->rows.nint, kRed);
  c.bc = ceil_div(p->cols.nint, kRed);
  MFE_CHECK(W.alloc(&c.d2, p->rows.nint));
  MFE_CHECK(W.alloc(&c.e2, p->cols.nint));
  MFE_CHECK(W.alloc(&c.pa, c.br + c.bc));
  MFE_CHECK(W.alloc(&c.pn, c.br + c.bc));
  MFE_CHECK(W.alloc(&c.pe, c.br + c.bc));
  MFE_CHECK(W.alloc(&c.out, 1));
  c.trace = rms_trace;
  c.idx = 0;
  c.st = (hipStream_t)prm->stream;
  return plan_run(p, prm, nullptr, nullptr, 0, d, e, u_bar, v_bar, trace_every, trace_chunk, &c);
}

int plan_lsqr(mfe_plan* p, const double* b, const double* d, const double* e, double tol, int32_t max_iter,
              int32_t check_every, double* x, mfe_lsqr_info* info, hipStream_t st) {
  MFE_CHECK(ensure_mats(p, st));
  SellOps ops(p);
  if (!p->lsqr_cache) {
    p->lsqr_cache = new (std::nothrow) LsqrCache();
    if (!p->lsqr_cache) return set_error(MFE_ENOMEM, "out of host memory for the LSQR workspace");
  }
  return run_lsqr(ops, b, d, e, tol, max_iter, check_every, x, info, st, p->lsqr_cache);
}

int plan_residual(mfe_plan* p, const double* d, const double* e, double alpha, double beta, double* rms,
                  double* rms_nonempty, int64_t* n_empty, hipStream_t st) {
  if (p->count != 1) return set_error(MFE_EUNSUPPORTED, "residual needs a single-matrix plan");
  MFE_CHECK(ensure_mats(p, st));
  return run_residual_sell(p, d, e, alpha, beta, rms, rms_nonempty, n_empty, st);
}

int dense_f64_lsqr(const mfe_matrix* A, const double* b, const double* d, const double* e, double tol,
                   int32_t max_iter, int32_t check_every, double* x, mfe_lsqr_info* info, hipStream_t st) {
  if (!A->data) return set_error(MFE_EINVAL, "dense data is NULL");
  if (A->ld < A->n) return set_error(MFE_EDIM, "ld < n");
  DenseOps ops((const double*)A->data, A->m, A->n, A->ld);
  return run_lsqr(ops, b, d, e, tol, max_iter, check_every, x, info, st);
}

int dense_f64_residual(const mfe_matrix* A, const double* d, const double* e, double alpha, double beta, double* rms,
                       double* rms_nonempty, int64_t* n_empty, hipStream_t st) {
  if (!A->data) return set_error(MFE_EINVAL, "dense data is NULL");
  if (A->ld < A->n) return set_error(MFE_EDIM, "ld < n");
  const int64_t m = A->m, n = A->n;
  const int64_t br = ceil_div(m, kRed), bc = ceil_div(n, kRed);
  Work W;
  double *pa, *pn, *pe, *out;
  MFE_CHECK(W.alloc(&pa, br + bc));
  MFE_CHECK(W.alloc(&pn, br + bc));
  MFE_CHECK(W.alloc(&pe, br + bc));
  MFE_CHECK(W.alloc(&out, 3));
  const double* Ad = (const double*)A->data;
  k_dense_rownorm<<<dim3((unsigned)br), dim3(kRed), 0, st>>>(Ad, m, n, A->ld, 0, d, e, alpha, pa, pn, pe);
  k_dense_rownorm<<<dim3((unsigned)bc), dim3(kRed), 0, st>>>(Ad, m, n, A->ld, 1, e, d, beta, pa + br, pn + br, pe + br);
  k_reduce<<<1, kRed, 0, st>>>(pa, br + bc, out);
  k_reduce<<<1, kRed, 0, st>>>(pn, br + bc, out + 1);
  k_reduce<<<1, kRed, 0, st>>>(pe, br + bc, out + 2);
  MFE_HIP(hipGetLastError());
  double h[3];
  MFE_HIP(hipMemcpyAsync(h, out, sizeof h, hipMemcpyDeviceToHost, st));
  MFE_HIP(hipStreamSynchronize(st));
  const double total = (double)(m + n);
  const int64_t ne = (int64_t)llround(h[2]);
  if (rms) *rms = std::sqrt(h[0] / total);
  if (rms_nonempty) *rms_nonempty = total - ne > 0 ? std::sqrt(h[1] / (total - ne)) : 0.0;
  if (n_empty) *n_empty = ne;
  return MFE_OK;
}


// ------------------------------------------- Chambolle-Cremers-Pock on the Lasso (Section 5.2)
//
// minimise ||A x - b||^2 / sqrt(lam) + sqrt(lam) ||x||_1 by the first-order primal-dual
// method with theta = 1 on Abar = D A E (x = E xbar): per iteration one product with Abar
// and one with Abar', each fused with its proximal step (closed forms of the separable
// functions; see mfe.h).  FP64 throughout; vectors in the plan's internal order.

// Dual step over the rows: y <- (y + sigma D A gx - sigma d b) / (1 + sigma d^2 sqrt(lam)/2),
// gy = d y (gathered by the primal step); gx = e xt in the columns' internal order.
// Workgroups as for k_sell_product.
__global__ __launch_bounds__(kSlice * kMaxSplit) void k_ccp_dual(SideDev S, SliceMap sm,
                                                                 const double* __restrict__ gx,
                                                                 const double* __restrict__ d,
                                                                 const double* __restrict__ b, double sigma,
                                                                 double half_sqrt_lam, double* __restrict__ y,
                                                                 double* __restrict__ gy) {
  const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int wsub = wave % sm.P;
  const int64_t nslices = S.nint / kSlice;
  const int64_t s = launch_slice(S, (int64_t)blockIdx.x * sm.G + wave / sm.P, nslices);
  const double acc = slice_row_sum(S, gx, s, nslices, sm.P, wave, wsub, lane);
  if (wsub != 0 || s >= nslices) return;
  const int64_t r = s * kSlice + lane;
  if (S.orig[r] < 0) return;
  const double dr = d[r];
  const double yn = (y[r] + sigma * (dr * acc) - sigma * dr * b[r]) / (1.0 + sigma * dr * dr * half_sqrt_lam);
  y[r] = yn;
  gy[r] = dr * yn;
}

// Primal step over the columns: u = x - tau e A' gy, x' = soft(u, tau sqrt(lam) e),
// xt = x' + theta (x' - x), gx = e xt.
__global__ __launch_bounds__(kSlice * kMaxSplit) void k_ccp_primal(SideDev S, SliceMap sm,
                                                                   const double* __restrict__ gy,
                                                                   const double* __restrict__ e_sc, double tau,
                                                                   double thr, double theta, double* __restrict__ x,
                                                                   double* __restrict__ gx) {
  const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int wsub = wave % sm.P;
  const int64_t nslices = S.nint / kSlice;
  const int64_t s = launch_slice(S, (int64_t)blockIdx.x * sm.G + wave / sm.P, nslices);
  const double acc = slice_row_sum(S, gy, s, nslices, sm.P, wave, wsub, lane);
  if (wsub != 0 || s >= nslices) return;
  const int64_t c = s * kSlice + lane;
  if (S.orig[c] < 0) return;
  const double ec = e_sc[c];
  const double u = x[c] - tau * (ec * acc);
  const double t = thr * ec;
  const double xn = u > t ? u - t : (u < -t ? u + t : 0.0);
  const double xt = xn + theta * (xn - x[c]);
  x[c] = xn;
  gx[c] = ec * xt;
}

// Block partials of sum_c |e_c x_c| (the l1 term of the objective at x = E xbar).
__global__ __launch_bounds__(kRed) void k_l1_partial(int64_t n, const double* __restrict__ e_sc,
                                                     const double* __restrict__ x, double* __restrict__ partial) {
  const int64_t c = (int64_t)blockIdx.x * kRed + threadIdx.x;
  const double v = c < n ? fabs(e_sc[c] * x[c]) : 0.0;
  const double bs = block_sum(v);
  if (threadIdx.x == 0) partial[blockIdx.x] = bs;
}

__global__ void k_set1(double* p, double v) { *p = v; }

__global__ void k_fill_valid(int64_t n, const int32_t* __restrict__ orig, double v, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = orig[i] >= 0 ? v : 0.0;
}

// hist[2 it] = beta, hist[2 it + 1] = alpha of the current bidiagonalisation step.
__global__ void k_record(const LsqrScal* __restrict__ sc, double* __restrict__ hist, int it) {
  hist[2 * it] = sc->beta;
  hist[2 * it + 1] = sc->alpha;
}

// Largest eigenvalue of the symmetric tridiagonal matrix (diag, off) by bisection on the
// Sturm count (the number of negative pivots of T - x I = L D L').
double tridiag_max_eig(const std::vector<double>& dg, const std::vector<double>& off) {
  const size_t k = dg.size();
  double lo = 0.0, hi = 0.0;
  for (size_t j = 0; j < k; ++j) {
    const double r = (j > 0 ? std::fabs(off[j - 1]) : 0.0) + (j + 1 < k ? std::fabs(off[j]) : 0.0);
    hi = std::max(hi, dg[j] + r);
    lo = std::min(lo, dg[j] - r);
  }
  auto count_above = [&](double x) {  // eigenvalues > x
    int neg = 0;
    double dpiv = 1.0;
    for (size_t j = 0; j < k; ++j) {
      const double o2 = j > 0 ? off[j - 1] * off[j - 1] : 0.0;
      dpiv = (dg[j] - x) - (j > 0 ? o2 / dpiv : 0.0);
      if (dpiv == 0.0) dpiv = -1e-300;
      if (dpiv < 0.0) ++neg;
    }
    return (int)k - neg;
  };
  for (int i = 0; i < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++i) {
    const double mid = 0.5 * (lo + hi);
    if (count_above(mid) >= 1) lo = mid;
    else hi = mid;
  }
  return hi;
}

// ||D A E||_2 by Golub-Kahan bidiagonalisation (the Lanczos process of LSQR, started
// from b = 1): after i steps the lower bidiagonal B_i (alpha_1..alpha_i on the diagonal,
// beta_2..beta_{i+1} below it) has largest singular value at most ||D A E||_2 and
// converging to it; it is the square root of the largest eigenvalue of the tridiagonal
// B_i' B_i, found by bisection.  Checked every 5 steps; stops when it changes by at most
// tol (relative), when the process ends exactly (alpha or beta = 0), or at max_iter.
int run_op_norm(const SellOps& ops, const double* dd, const double* ee, int32_t max_iter, double tol, double* norm,
                int32_t* iters, hipStream_t st) {
  const int64_t nr = ops.rows(), nc = ops.cols();
  const int64_t pb = std::max(ops.fwd_blocks(), ops.bwd_blocks()) + ceil_div(nr, kRed) + 1;
  Work W;
  double *bb, *u, *du, *v, *ev, *res, *part, *hist;
  LsqrScal* sc;
  MFE_CHECK(W.alloc(&bb, nr));
  MFE_CHECK(W.alloc(&u, nr));
  MFE_CHECK(W.alloc(&du, nr));
  MFE_CHECK(W.alloc(&res, nr));
  MFE_CHECK(W.alloc(&v, nc));
  MFE_CHECK(W.alloc(&ev, nc));
  MFE_CHECK(W.alloc(&part, pb));
  MFE_CHECK(W.alloc(&hist, 2 * ((int64_t)max_iter + 1)));
  MFE_CHECK(W.alloc(&sc, 1));
  for (double* z : {v, ev}) MFE_HIP(hipMemsetAsync(z, 0, sizeof(double) * nc, st));
  const unsigned row_grid = (unsigned)ceil_div(nr, 256);
  k_fill_valid<<<row_grid, 256, 0, st>>>(nr, ops.R.orig, 1.0, bb);
  k_scal_init<<<1, 1, 0, st>>>(sc);
  k_mul<<<row_grid, 256, 0, st>>>(nr, dd, bb, u);  // p_1 = D 1 (= beta_1 u_1)
  k_mul<<<row_grid, 256, 0, st>>>(nr, dd, u, du);
  k_mul<<<row_grid, 256, 0, st>>>(nr, u, u, res);
  reduce_long(res, nr, part + ceil_div(nr, kRed), part, st);
  k_scal_step<<<1, kScal, 0, st>>>(part, 1, sc, 1, 0);
  // q_1 = E A' D p_1 / beta_1 (= alpha_1 v_1), then alpha_1
  ops.bwd(ee, du, &sc->inv_beta, nullptr, nullptr, v, ev, part, st);
  k_scal_step<<<1, kScal, 0, st>>>(part, ops.bwd_blocks(), sc, 2, 1);
  k_record<<<1, 1, 0, st>>>(sc, hist, 0);
  MFE_HIP(hipGetLastError());
  std::vector<double> h;
  double est = 0.0, prev = -1.0;
  int it = 0;
  for (it = 1; it <= max_iter; ++it) {
    // beta u = Abar v - alpha u, then beta (and the iteration count)
    ops.fwd(dd, ev, &sc->inv_alpha, &sc->coef_p, u, u, du, part, TailUpdate{}, st);
    k_scal_step<<<1, kScal, 0, st>>>(part, ops.fwd_blocks(), sc, 1, 1);
    // alpha v = Abar' u - beta v, then alpha
    ops.bwd(ee, du, &sc->inv_beta, &sc->coef_q, v, v, ev, part, st);
    k_scal_step<<<1, kScal, 0, st>>>(part, ops.bwd_blocks(), sc, 2, 0);
    k_record<<<1, 1, 0, st>>>(sc, hist, it);
    MFE_HIP(hipGetLastError());
    if (it % 5 != 0 && it != max_iter) continue;
    h.resize(2 * (size_t)(it + 1));
    MFE_HIP(hipMemcpyAsync(h.data(), hist, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
    MFE_HIP(hipStreamSynchronize(st));
    // columns j = 1..i of B_i: alpha_j = h[2(j-1)+1], beta_{j+1} = h[2j]
    std::vector<double> dg, off;
    bool ended = false;
    for (int j = 1; j <= it; ++j) {
      const double a = h[2 * (j - 1) + 1], bnext = h[2 * j];
      if (!(a > 0.0)) {
        ended = true;
        break;
      }
      dg.push_back(a * a + bnext * bnext);
      const double anext = h[2 * j + 1];
      if (j < it) off.push_back(anext * bnext);
      if (!(bnext > 0.0)) {
        ended = true;
        break;
      }
    }
    if (dg.empty()) break;
    off.resize(dg.size() - 1);
    est = std::sqrt(tridiag_max_eig(dg, off));
    if (ended || (prev > 0.0 && std::fabs(est - prev) <= tol * est)) break;
    prev = est;
  }
  *norm = est;
  if (iters) *iters = std::min(it, max_iter);
  return MFE_OK;
}

int plan_op_norm(mfe_plan* p, const double* d, const double* e, int32_t max_iter, double tol, double* norm,
                 int32_t* iters, hipStream_t st) {
  MFE_CHECK(ensure_mats(p, st));
  SellOps ops(p);
  Work W;
  double *dd, *ee;
  MFE_CHECK(W.alloc(&dd, ops.rows()));
  MFE_CHECK(W.alloc(&ee, ops.cols()));
  ops.to_op(true, d, 1.0, 0, dd, st);
  ops.to_op(false, e, 1.0, 0, ee, st);
  return run_op_norm(ops, dd, ee, max_iter, tol, norm, iters, st);
}

int plan_ccp_lasso(mfe_plan* p, const double* b, const double* d, const double* e, double lam, double op_norm,
                   int32_t iters, int32_t trace_every, double* trace, double* x_out, mfe_ccp_info* info,
                   hipStream_t st) {
  MFE_CHECK(ensure_mats(p, st));
  SellOps ops(p);
  const int64_t nr = ops.rows(), nc = ops.cols();
  const int64_t pb = std::max(ops.fwd_blocks(), ops.bwd_blocks()) + ceil_div(nc, kRed);
  Work W;
  double *bb, *dd, *ee, *y, *gy, *x, *gx, *res, *wx, *part, *obj, *neg1;
  MFE_CHECK(W.alloc(&neg1, 1));
  k_set1<<<1, 1, 0, st>>>(neg1, -1.0);
  MFE_CHECK(W.alloc(&bb, nr));
  MFE_CHECK(W.alloc(&dd, nr));
  MFE_CHECK(W.alloc(&ee, nc));
  MFE_CHECK(W.alloc(&y, nr));
  MFE_CHECK(W.alloc(&gy, nr));
  MFE_CHECK(W.alloc(&x, nc));
  MFE_CHECK(W.alloc(&gx, nc));
  MFE_CHECK(W.alloc(&res, nr));
  MFE_CHECK(W.alloc(&wx, nc));
  MFE_CHECK(W.alloc(&part, pb));
  MFE_CHECK(W.alloc(&obj, 2));
  ops.to_op(true, b, 0.0, 0, bb, st);
  ops.to_op(true, d, 1.0, 0, dd, st);
  ops.to_op(false, e, 1.0, 0, ee, st);
  for (double* v : {y, gy}) MFE_HIP(hipMemsetAsync(v, 0, sizeof(double) * nr, st));
  for (double* v : {x, gx}) MFE_HIP(hipMemsetAsync(v, 0, sizeof(double) * nc, st));
  mfe_ccp_info inf{};
  if (!(op_norm > 0)) {
    MFE_CHECK(run_op_norm(ops, dd, ee, 1000, 1e-10, &op_norm, &inf.norm_iters, st));
    if (!(op_norm > 0)) return set_error(MFE_EINVAL, "the scaled matrix is zero");
  }
  const double tau = 0.9 / op_norm, sigma = 0.9 / op_norm, sl = std::sqrt(lam);
  const unsigned cg = (unsigned)ceil_div(nc, kRed);
  // f(x) at x = E xbar: ||A x - b||^2 / sqrt(lam) + sqrt(lam) ||x||_1
  auto objective = [&](double* out) -> int {
    k_mul<<<dim3((unsigned)ceil_div(nc, 256)), dim3(256), 0, st>>>(nc, ee, x, wx);
    ops.fwd(nullptr, wx, nullptr, neg1, bb, res, nullptr, part, TailUpdate{}, st);
    k_reduce<<<1, kRed, 0, st>>>(part, ops.fwd_blocks(), obj);
    k_l1_partial<<<cg, kRed, 0, st>>>(nc, ee, x, part);
    k_reduce<<<1, kRed, 0, st>>>(part, cg, obj + 1);
    MFE_HIP(hipGetLastError());
    double h[2];
    MFE_HIP(hipMemcpyAsync(h, obj, sizeof h, hipMemcpyDeviceToHost, st));
    MFE_HIP(hipStreamSynchronize(st));
    *out = h[0] / sl + sl * h[1];
    return MFE_OK;
  };
  int tr = 0;
  for (int it = 1; it <= iters; ++it) {
    k_ccp_dual<<<dim3((unsigned)ops.fwd_blocks()), dim3(kSlice * ops.MR.P * ops.MR.G), 0, st>>>(
        ops.R, ops.MR, gx, dd, bb, sigma, 0.5 * sl, y, gy);
    k_ccp_primal<<<dim3((unsigned)ops.bwd_blocks()), dim3(kSlice * ops.MC.P * ops.MC.G), 0, st>>>(
        ops.C, ops.MC, gy, ee, tau, tau * sl, 1.0, x, gx);
    MFE_HIP(hipGetLastError());
    if (trace && trace_every > 0 && it % trace_every == 0) MFE_CHECK(objective(&trace[tr++]));
  }
  MFE_CHECK(objective(&inf.objective));
  inf.iters = iters;
  inf.op_norm = op_norm;
  inf.tau = tau;
  inf.sigma = sigma;
  ops.from_op(false, x, ee, x_out, st);
  MFE_HIP(hipGetLastError());
  MFE_HIP(hipStreamSynchronize(st));
  if (info) *info = inf;
  return MFE_OK;
}

}  // namespace mfe
