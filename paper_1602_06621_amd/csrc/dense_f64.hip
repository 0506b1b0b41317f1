// Algorithm 1 (Section 3.2) for dense FP64 matrices and for matrix-free operators.
//
// Dense: one launch per direction and step, Jacobi order (both read the scales of step
// t-1).  Row direction: one wavefront per row, lanes stride the columns (coalesced),
// the k probe sums are reduced across the wavefront.  Column direction: one thread per
// column, a wavefront reads 64 consecutive columns of each row (coalesced).  The scale
// e^x of every index is kept in FP64 (ping-pong by step parity); probe signs come from
// the same Philox stream contract as the sparse engine.
//
// Operator: per step the library forms the probe blocks E S (n x k) and D W (m x k) in
// FP64, calls apply() for A (E S) and A' (D W), and runs the square/step/project update
// in its own kernels (the unfused path).
#include <cmath>
#include <vector>

#include "dense.h"
#include "sparse.h"

namespace mfe {
namespace {

struct DenseSide {
  double* x;
  double* xbar;
  const double* scale_in;   // other side's e^x from step t-1
  double* scale_out;        // this side's e^x of step t
  const uint64_t* sign_in;  // sign words (of the other side's indices) of step t
  double target;
};

template <int KP>
__global__ __launch_bounds__(256) void k_dense_rows(const double* __restrict__ A, int64_t m, int64_t n, int64_t ld,
                                                   DenseSide S, int k, StepScalars sc, int* flag) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + wave;
  if (i >= m) return;
  double acc[KP];
#pragma unroll
  for (int p = 0; p < KP; ++p) acc[p] = 0.0;
  for (int64_t j = lane; j < n; j += 64)
    accumulate_signed<KP>(acc, A[i * ld + j] * S.scale_in[j], extract_bits(S.sign_in, j * k, k));
#pragma unroll
  for (int p = 0; p < KP; ++p)
    for (int off = 32; off > 0; off >>= 1) acc[p] += __shfl_xor(acc[p], off);
  if (lane != 0) return;
  double ss = 0.0;
#pragma unroll
  for (int p = 0; p < KP; ++p)
    if (p < k) ss += acc[p] * acc[p];
  double x = S.x[i], xb = S.xbar[i];
  if (!sgd_update(ss, k, S.target, sc, x, xb)) atomicOr(flag, 1);
  S.x[i] = x;
  S.xbar[i] = xb;
  S.scale_out[i] = exp(x);
}

template <int KP>
__global__ __launch_bounds__(256) void k_dense_cols(const double* __restrict__ A, int64_t m, int64_t n, int64_t ld,
                                                   DenseSide S, int k, StepScalars sc, int* flag) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  double acc[KP];
#pragma unroll
  for (int p = 0; p < KP; ++p) acc[p] = 0.0;
  for (int64_t i = 0; i < m; ++i)
    accumulate_signed<KP>(acc, A[i * ld + j] * S.scale_in[i], extract_bits(S.sign_in, i * k, k));
  double ss = 0.0;
#pragma unroll
  for (int p = 0; p < KP; ++p)
    if (p < k) ss += acc[p] * acc[p];
  double x = S.x[j], xb = S.xbar[j];
  if (!sgd_update(ss, k, S.target, sc, x, xb)) atomicOr(flag, 1);
  S.x[j] = x;
  S.xbar[j] = xb;
  S.scale_out[j] = exp(x);
}

__global__ void k_dense_init(int64_t cnt, const double* __restrict__ x0, double M, double* __restrict__ x,
                             double* __restrict__ xbar, double* __restrict__ scale, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  double v = x0 ? x0[i] : 0.0;
  if (!(fabs(v) <= M)) {
    atomicOr(flag, 2);
    v = 0.0;
  }
  x[i] = v;
  xbar[i] = v;
  scale[i] = exp(v);
}

__global__ void k_dense_output(int64_t cnt, const double* __restrict__ xbar, double* __restrict__ dout,
                               double* __restrict__ xbar_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  dout[i] = exp(xbar[i]);
  if (xbar_out) xbar_out[i] = xbar[i];
}

// Operator path: probe block Z[i, p] = scale[i] * (-1)^bit(i*k + p), row-major, ld = k.
__global__ void k_probe_block(int64_t cnt, int k, const double* __restrict__ scale, const uint64_t* __restrict__ sw,
                              double* __restrict__ Z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const uint64_t bits = extract_bits(sw, i * k, k);
  for (int p = 0; p < k; ++p) Z[i * k + p] = ((bits >> p) & 1ull) ? -scale[i] : scale[i];
}

// Operator path: update from the product block Y (cnt x k, row-major, ld = k).
__global__ void k_block_update(int64_t cnt, int k, const double* __restrict__ Y, double target, StepScalars sc,
                               double* __restrict__ x, double* __restrict__ xbar, double* __restrict__ scale_out,
                               int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  double ss = 0.0;
  for (int p = 0; p < k; ++p) ss += Y[i * k + p] * Y[i * k + p];
  double xi = x[i], xb = xbar[i];
  if (!sgd_update(ss, k, target, sc, xi, xb)) atomicOr(flag, 1);
  x[i] = xi;
  xbar[i] = xb;
  scale_out[i] = exp(xi);
}

struct Bufs {
  std::vector<void*> p;
  ~Bufs() {
    for (void* q : p) (void)hipFree(q);
  }
  template <class T>
  int alloc(T** out, int64_t n) {
    hipError_t e = hipMalloc((void**)out, sizeof(T) * (size_t)std::max<int64_t>(n, 1));
    if (e != hipSuccess)
      return set_error(e == hipErrorOutOfMemory ? MFE_ENOMEM : MFE_EDEVICE, "hipMalloc failed: %s",
                       hipGetErrorString(e));
    p.push_back(*out);
    return MFE_OK;
  }
};

// Sign words of one matrix: side 0 (columns, n*k bits) and side 1 (rows, m*k bits) in
// one slot; the slot is refilled every step.
struct DenseSigns {
  SignSeg* segs = nullptr;
  int64_t* prefix = nullptr;
  uint64_t* words = nullptr;
  int64_t nblocks = 0, off_rows = 0;
  int setup(Bufs& B, int64_t m, int64_t n, int k, int64_t batch, hipStream_t st) {
    SignSeg h[2];
    h[0].ctrl_lo = ((uint64_t)batch << 34) | 0ull;
    h[0].nblocks = ceil_div(n * k, 256);
    h[0].word_off = 0;
    h[1].ctrl_lo = ((uint64_t)batch << 34) | 1ull;
    h[1].nblocks = ceil_div(m * k, 256);
    h[1].word_off = 4 * h[0].nblocks + 4;
    off_rows = h[1].word_off;
    nblocks = h[0].nblocks + h[1].nblocks;
    const int64_t pre[3] = {0, h[0].nblocks, nblocks};
    MFE_CHECK(B.alloc(&segs, 2));
    MFE_CHECK(B.alloc(&prefix, 3));
    MFE_CHECK(B.alloc(&words, h[1].word_off + 4 * h[1].nblocks + 4));
    MFE_HIP(hipMemsetAsync(words, 0, sizeof(uint64_t) * (h[1].word_off + 4 * h[1].nblocks + 4), st));
    MFE_HIP(hipMemcpyAsync(segs, h, sizeof h, hipMemcpyHostToDevice, st));
    MFE_HIP(hipMemcpyAsync(prefix, pre, sizeof pre, hipMemcpyHostToDevice, st));
    return MFE_OK;
  }
  int draw(uint64_t seed, uint64_t step, hipStream_t st) const {
    SignGenDev g;
    g.segs = segs;
    g.seg_prefix = prefix;
    g.nseg = 2;
    g.nblocks = nblocks;
    g.seed = seed;
    g.step = step;
    g.out = words;
    return launch_signgen(g, st);
  }
};

StepScalars scalars(const mfe_equil_params* p, int t) {
  StepScalars sc;
  sc.tau = (double)t + (double)p->t0;
  sc.eta = 2.0 / (p->gamma * (sc.tau + 1.0));
  sc.gamma = p->gamma;
  sc.M = p->box_M;
  return sc;
}

template <int KP>
void launch_dense_step(const double* A, int64_t m, int64_t n, int64_t ld, const DenseSide& R, const DenseSide& C,
                       int k, const StepScalars& sc, int* flag, hipStream_t st) {
  k_dense_rows<KP><<<dim3((unsigned)ceil_div(m, 4)), dim3(256), 0, st>>>(A, m, n, ld, R, k, sc, flag);
  k_dense_cols<KP><<<dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st>>>(A, m, n, ld, C, k, sc, flag);
}

int finish(int* flag, hipStream_t st) {
  int h = 0;
  MFE_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  MFE_HIP(hipStreamSynchronize(st));
  if (h & 2) return set_error(MFE_EINVAL, "warm start u0/v0 outside the box [-M, M] (or NaN)");
  if (h & 1) return set_error(MFE_ENONFINITE, "non-finite gradient estimate or iterate (NaN/Inf in A?)");
  return MFE_OK;
}

}  // namespace

int dense_f64_equilibrate(const mfe_matrix* A, const mfe_equil_params* p, double* d, double* e, double* u_bar,
                          double* v_bar) {
  if (!A->data) return set_error(MFE_EINVAL, "dense data is NULL");
  if (A->ld < A->n) return set_error(MFE_EDIM, "ld < n");
  if (p->probes > 64) return set_error(MFE_EUNSUPPORTED, "dense FP64 path supports at most 64 probes per step");
  hipStream_t st = (hipStream_t)p->stream;
  const int64_t m = A->m, n = A->n;
  const int k = p->probes;
  Bufs B;
  double *u, *ub, *v, *vb, *su[2], *sv[2];
  int* flag;
  MFE_CHECK(B.alloc(&u, m));
  MFE_CHECK(B.alloc(&ub, m));
  MFE_CHECK(B.alloc(&v, n));
  MFE_CHECK(B.alloc(&vb, n));
  for (int i = 0; i < 2; ++i) {
    MFE_CHECK(B.alloc(&su[i], m));
    MFE_CHECK(B.alloc(&sv[i], n));
  }
  MFE_CHECK(B.alloc(&flag, 1));
  DenseSigns S;
  MFE_CHECK(S.setup(B, m, n, k, p->batch, st));
  MFE_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
  k_dense_init<<<dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st>>>(m, p->u0, p->box_M, u, ub, su[0], flag);
  k_dense_init<<<dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st>>>(n, p->v0, p->box_M, v, vb, sv[0], flag);
  const double* Ad = (const double*)A->data;
  for (int t = 1; t <= p->steps; ++t) {
    MFE_CHECK(S.draw(p->seed, (uint64_t)t, st));
    const int cur = t & 1, prev = cur ^ 1;
    DenseSide R{u, ub, sv[prev], su[cur], S.words, p->alpha * p->alpha};              // gathers s (side 0)
    DenseSide C{v, vb, su[prev], sv[cur], S.words + S.off_rows, p->beta * p->beta};  // gathers w (side 1)
    const StepScalars sc = scalars(p, t);
    if (k <= 1) launch_dense_step<1>(Ad, m, n, A->ld, R, C, k, sc, flag, st);
    else if (k <= 2) launch_dense_step<2>(Ad, m, n, A->ld, R, C, k, sc, flag, st);
    else if (k <= 4) launch_dense_step<4>(Ad, m, n, A->ld, R, C, k, sc, flag, st);
    else if (k <= 8) launch_dense_step<8>(Ad, m, n, A->ld, R, C, k, sc, flag, st);
    else if (k <= 16) launch_dense_step<16>(Ad, m, n, A->ld, R, C, k, sc, flag, st);
    else if (k <= 32) launch_dense_step<32>(Ad, m, n, A->ld, R, C, k, sc, flag, st);
    else launch_dense_step<64>(Ad, m, n, A->ld, R, C, k, sc, flag, st);
  }
  MFE_HIP(hipGetLastError());
  k_dense_output<<<dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st>>>(m, ub, d, u_bar);
  k_dense_output<<<dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st>>>(n, vb, e, v_bar);
  MFE_HIP(hipGetLastError());
  return finish(flag, st);
}

int operator_equilibrate(const mfe_matrix* A, const mfe_equil_params* p, double* d, double* e, double* u_bar,
                         double* v_bar) {
  if (!A->apply) return set_error(MFE_EINVAL, "operator apply() is NULL");
  hipStream_t st = (hipStream_t)p->stream;
  const int64_t m = A->m, n = A->n;
  const int k = p->probes;
  Bufs B;
  double *u, *ub, *v, *vb, *su[2], *sv[2], *Z, *Wd, *Y, *X;
  int* flag;
  MFE_CHECK(B.alloc(&u, m));
  MFE_CHECK(B.alloc(&ub, m));
  MFE_CHECK(B.alloc(&v, n));
  MFE_CHECK(B.alloc(&vb, n));
  for (int i = 0; i < 2; ++i) {
    MFE_CHECK(B.alloc(&su[i], m));
    MFE_CHECK(B.alloc(&sv[i], n));
  }
  MFE_CHECK(B.alloc(&Z, n * k));
  MFE_CHECK(B.alloc(&Wd, m * k));
  MFE_CHECK(B.alloc(&Y, m * k));
  MFE_CHECK(B.alloc(&X, n * k));
  MFE_CHECK(B.alloc(&flag, 1));
  DenseSigns S;
  MFE_CHECK(S.setup(B, m, n, k, p->batch, st));
  MFE_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
  k_dense_init<<<dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st>>>(m, p->u0, p->box_M, u, ub, su[0], flag);
  k_dense_init<<<dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st>>>(n, p->v0, p->box_M, v, vb, sv[0], flag);
  for (int t = 1; t <= p->steps; ++t) {
    MFE_CHECK(S.draw(p->seed, (uint64_t)t, st));
    const int cur = t & 1, prev = cur ^ 1;
    k_probe_block<<<dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st>>>(n, k, sv[prev], S.words, Z);
    k_probe_block<<<dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st>>>(m, k, su[prev], S.words + S.off_rows, Wd);
    MFE_HIP(hipGetLastError());
    if (A->apply(A->ctx, 0, k, Z, k, Y, k, (void*)st) != 0)
      return set_error(MFE_EDEVICE, "operator apply(trans=0) failed at step %d", t);
    if (A->apply(A->ctx, 1, k, Wd, k, X, k, (void*)st) != 0)
      return set_error(MFE_EDEVICE, "operator apply(trans=1) failed at step %d", t);
    const StepScalars sc = scalars(p, t);
    k_block_update<<<dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st>>>(m, k, Y, p->alpha * p->alpha, sc, u, ub,
                                                                          su[cur], flag);
    k_block_update<<<dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st>>>(n, k, X, p->beta * p->beta, sc, v, vb,
                                                                          sv[cur], flag);
    MFE_HIP(hipGetLastError());
  }
  k_dense_output<<<dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st>>>(m, ub, d, u_bar);
  k_dense_output<<<dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st>>>(n, vb, e, v_bar);
  MFE_HIP(hipGetLastError());
  return finish(flag, st);
}

}  // namespace mfe
