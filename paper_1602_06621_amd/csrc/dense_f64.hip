// Algorithm 1 (Section 3.2) for dense FP64 matrices and for matrix-free operators.
//
// Dense: one launch per direction and step, Jacobi order (both read the scales of step
// t-1).  Row direction: one wavefront per row, lanes stride the columns (coalesced),
// the k probe sums are reduced across the wavefront.  Column direction: one thread per
// column, a wavefront reads 64 consecutive columns of each row (coalesced).  The scale
// e^x of every index is kept in FP64 (ping-pong by step parity); probe signs come from
// the same Philox stream contract as the sparse engine.
//
// Small dense matrices (config-0 scale) run all T steps in one persistent workgroup
// instead: one launch for the whole run, LDS barriers between steps, so the run is not
// bounded by per-step launch latency.
//
// Operator: per step the library forms the probe blocks E S (n x k) and D W (m x k) in
// FP64, calls apply() for A (E S) and A' (D W), and runs the square/step/project update
// in its own kernels (the unfused path).
#include <cmath>
#include <mutex>
#include <vector>

#include "dense.h"
#include "sparse.h"

// Scratch of the allocation-free entry point (mfe_equilibrate_noalloc): every device the
// library runs on holds its own copy until the process ends.  Its address differs per
// device and reaches the host only through hipGetSymbolAddress; in host code the name
// `scratch` is not a device address and is never passed to a kernel or a copy.
static constexpr size_t kScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

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
    acc[p] = wave_sum(acc[p]);
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

// ---- persistent single-workgroup paths for small matrices
//
// The whole run (or a chunk of up to kPersistChunk steps) is one launch of one
// workgroup; steps are separated by LDS barriers.  The probe sign words of the chunk
// are drawn beforehand by a parallel launch (k_sign_chunk) and staged into LDS one step
// ahead, so the Philox rounds stay off the step's critical path.
constexpr int kPersistThreads = 1024;
constexpr int kPersistWaves = kPersistThreads / 64;
constexpr int64_t kPersistMaxDim = 1792;               // m + n (LDS: 32 (m + n) bytes of state)
constexpr int64_t kPersistMaxWork = (int64_t)1 << 20;  // m n k multiply-adds per direction
constexpr int kPersistChunk = 4096;                    // steps per launch
constexpr int kPersistMaxWords = 1024;                 // sign words per step (one per thread)
// Register-resident variant (k = 1): 8 wavefronts; thread (w, l) keeps
// A[w + 8 r][l + 64 c] for r < kTinyRM, c < kTinyCM in registers for the whole run
// (2 wavefronts per SIMD leave each lane 256 registers).
constexpr int kTinyThreads = 512, kTinyWaves = kTinyThreads / 64;
constexpr int kTinyRM = 25, kTinyCM = 2;
constexpr int kTinyStageWords = 5120;  // 40 KB of LDS

struct PersistArgs {
  const double* A;   // m x n, row stride ld
  const double* AT;  // n x m, row stride m (transposed copy; LDS-state variant only)
  int64_t m, n, ld;
  double *u, *ub, *v, *vb;  // iterates and averages: values in, values out
  int k, nsteps;            // steps t_begin .. t_begin + nsteps - 1
  double t_begin, t0, gamma, M, tgt_row, tgt_col;
  const uint64_t* sw;       // sign words of the chunk, step-major
  int32_t nb0, wps;         // Philox blocks of side 0 (columns); sign words per step
  int* flag;
};

// Sign words of steps t_begin .. t_begin + nsteps - 1, step-major (wps words per step):
// side 0 (columns) at 0, side 1 (rows) at 4 nb0 + 4; Philox block c of a side at counter
// (c + 1, 0, 0, 0), the same stream as every other path.
__global__ void k_sign_chunk(uint64_t* __restrict__ sw, int64_t t_begin, int nsteps, int nb0, int nb1, int wps,
                             uint64_t seed, uint64_t batch) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int per = nb0 + nb1;
  if (g >= (int64_t)nsteps * per) return;
  const int64_t st = g / per;
  const int c = (int)(g % per);
  const bool rows = c >= nb0;
  const int cb = rows ? c - nb0 : c;
  const U64x4 r = philox4x64_10((uint64_t)cb + 1, 0, 0, 0, seed,
                                stream_ctrl(batch, (uint64_t)(t_begin + st), rows ? 1 : 0));
  uint64_t* o = sw + st * wps + (rows ? 4 * (int64_t)nb0 + 4 : 0) + 4 * (int64_t)cb;
  o[0] = r.x[0];
  o[1] = r.x[1];
  o[2] = r.x[2];
  o[3] = r.x[3];
}

__device__ __forceinline__ StepScalars persist_scalars(const PersistArgs& a, int s) {
  StepScalars sc;
  sc.tau = a.t_begin + (double)s + a.t0;
  sc.eta = 2.0 / (a.gamma * (sc.tau + 1.0));
  sc.gamma = a.gamma;
  sc.M = a.M;
  return sc;
}

// Outputs per wavefront iteration: several rows (columns) at once keep their loads in
// flight together; fewer when the k accumulators are wide.
template <int KP>
struct PersistUnroll {
  static constexpr int U = KP <= 4 ? 4 : (KP <= 8 ? 2 : 1);
};

// One direction of one step of the LDS-state variant: wavefront w handles outputs
// w, w + 16, ...; lanes stride the inner dimension of the row-major operand B (rows of A,
// or rows of A'), the k sums are reduced across the wavefront, and lane r updates the
// r-th output of the group.  Iterates, averages and scales live in LDS.
template <int KP>
__device__ __forceinline__ void persist_side(const double* __restrict__ B, int64_t nout, int64_t ninner, int64_t ldb,
                                             const double* __restrict__ scale_in, const uint64_t* __restrict__ sw,
                                             double* __restrict__ scale_out, double* __restrict__ x,
                                             double* __restrict__ xbar, double target, int k, const StepScalars& sc,
                                             int* flag) {
  constexpr int U = PersistUnroll<KP>::U;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int W = kPersistWaves;
  for (int64_t i0 = wave; i0 < nout; i0 += (int64_t)W * U) {
    double acc[U][KP];
#pragma unroll
    for (int r = 0; r < U; ++r)
#pragma unroll
      for (int p = 0; p < KP; ++p) acc[r][p] = 0.0;
    for (int64_t j = lane; j < ninner; j += 64) {
      const double s = scale_in[j];
      const uint64_t bits = extract_bits(sw, j * k, k);
#pragma unroll
      for (int r = 0; r < U; ++r) {
        const int64_t i = i0 + (int64_t)r * W;
        if (i < nout) accumulate_signed<KP>(acc[r], B[i * ldb + j] * s, bits);
      }
    }
    double ss = 0.0;
#pragma unroll
    for (int r = 0; r < U; ++r) {
      double sr = 0.0;
#pragma unroll
      for (int p = 0; p < KP; ++p) {
        double a = acc[r][p];
        a = wave_sum(a);
        if (p < k) sr += a * a;
      }
      if (lane == r) ss = sr;
    }
    const int64_t i = i0 + (int64_t)lane * W;
    if (lane < U && i < nout) {
      double xi = x[i], xb = xbar[i];
      if (!sgd_update(ss, k, target, sc, xi, xb)) atomicOr(flag, 1);
      x[i] = xi;
      xbar[i] = xb;
      scale_out[i] = exp(xi);
    }
  }
}

template <int KP>
__global__ __launch_bounds__(kPersistThreads) void k_dense_persistent(PersistArgs a) {
  extern __shared__ double lds[];
  // scales by step parity: buffer (s & 1) receives step s, the other holds step s - 1
  double* sr[2] = {lds, lds + a.m};
  double* scl[2] = {lds + 2 * a.m, lds + 2 * a.m + a.n};
  double* xu = lds + 2 * (a.m + a.n);
  double* xub = xu + a.m;
  double* xv = xub + a.m;
  double* xvb = xv + a.n;
  uint64_t* words = reinterpret_cast<uint64_t*>(xvb + a.n);  // [2][wps], by step parity
  const int tid = threadIdx.x;
  for (int64_t i = tid; i < a.m; i += kPersistThreads) {
    xu[i] = a.u[i];
    xub[i] = a.ub[i];
    sr[1][i] = exp(xu[i]);
  }
  for (int64_t j = tid; j < a.n; j += kPersistThreads) {
    xv[j] = a.v[j];
    xvb[j] = a.vb[j];
    scl[1][j] = exp(xv[j]);
  }
  if (tid < a.wps) words[tid] = a.sw[tid];
  __syncthreads();
  for (int s = 0; s < a.nsteps; ++s) {
    const int cur = s & 1, prev = cur ^ 1;
    uint64_t next = 0;
    if (tid < a.wps && s + 1 < a.nsteps) next = a.sw[(int64_t)(s + 1) * a.wps + tid];
    const uint64_t* w0 = words + (int64_t)cur * a.wps;
    const uint64_t* w1 = w0 + 4 * (int64_t)a.nb0 + 4;
    const StepScalars sc = persist_scalars(a, s);
    // Jacobi order: both directions read the scales of step s - 1 and write those of step s
    persist_side<KP>(a.A, a.m, a.n, a.ld, scl[prev], w0, sr[cur], xu, xub, a.tgt_row, a.k, sc, a.flag);
    persist_side<KP>(a.AT, a.n, a.m, a.m, sr[prev], w1, scl[cur], xv, xvb, a.tgt_col, a.k, sc, a.flag);
    if (tid < a.wps && s + 1 < a.nsteps) words[(int64_t)prev * a.wps + tid] = next;
    __syncthreads();
  }
  for (int64_t i = tid; i < a.m; i += kPersistThreads) {
    a.u[i] = xu[i];
    a.ub[i] = xub[i];
  }
  for (int64_t j = tid; j < a.n; j += kPersistThreads) {
    a.v[j] = xv[j];
    a.vb[j] = xvb[j];
  }
}

// v from lane l ^ 16 (within each half of the wavefront), by ds_swizzle in bit mode.
__device__ __forceinline__ double swizzle_xor16(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)b, 0x401F);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), 0x401F);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Register-resident variant, k = 1, m <= 8 kTinyRM, n <= 64 kTinyCM.  Row sums: each
// lane sums its kTinyCM entries of a row, and the wavefront reduces 16 rows at a time
// by halving exchanges.  Column sums: each wavefront sums its kTinyRM rows per column
// into LDS, then one thread per column adds the 8 wavefront partials.
__global__ __launch_bounds__(kTinyThreads) void k_dense_tiny(PersistArgs a) {
  constexpr int NR = kTinyWaves * kTinyRM, NC = 64 * kTinyCM;
  __shared__ double sr[2][NR], scl[2][NC], xu[NR], xub[NR], xv[NC], xvb[NC];
  __shared__ double gsr[NR];  // (-1)^w_i e^(u_i) of the previous step, with this step's sign
  __shared__ double part[kTinyWaves][NC];
  // sign words of up to kTinyStageWords / wps steps, loaded together (a global load issued
  // inside a step would be waited for at one of the step's barriers)
  __shared__ uint64_t words[kTinyStageWords];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int m = (int)a.m, n = (int)a.n;
  double Ar[kTinyRM][kTinyCM];
#pragma unroll
  for (int r = 0; r < kTinyRM; ++r)
#pragma unroll
    for (int c = 0; c < kTinyCM; ++c) {
      const int i = w + kTinyWaves * r, j = l + 64 * c;
      Ar[r][c] = (i < m && j < n) ? a.A[(int64_t)i * a.ld + j] : 0.0;
    }
  for (int i = tid; i < m; i += kTinyThreads) {
    xu[i] = a.u[i];
    xub[i] = a.ub[i];
    sr[1][i] = exp(xu[i]);
  }
  for (int j = tid; j < n; j += kTinyThreads) {
    xv[j] = a.v[j];
    xvb[j] = a.vb[j];
    scl[1][j] = exp(xv[j]);
  }
  const int per_fill = kTinyStageWords / a.wps;  // steps per staging load
  __syncthreads();
  for (int s = 0; s < a.nsteps; ++s) {
    const int cur = s & 1, prev = cur ^ 1;
    if (s % per_fill == 0) {
      const int ns = min(per_fill, a.nsteps - s);
      for (int q = tid; q < ns * a.wps; q += kTinyThreads) words[q] = a.sw[(int64_t)s * a.wps + q];
      __syncthreads();
    }
    const uint64_t* w0 = words + (s % per_fill) * a.wps;
    const uint64_t* w1 = w0 + 4 * a.nb0 + 4;
    const StepScalars sc = persist_scalars(a, s);
    // signed row scales of this step (one thread per row), then one pass over the register
    // tile: each row's partial over this lane's columns (reduced across the wavefront) and
    // each column's partial over this wavefront's rows.  Multiplying by a signed scale
    // gives the same product as negating the unsigned one.
    for (int i = tid; i < m; i += kTinyThreads) gsr[i] = extract_bits(w1, i, 1) ? -sr[prev][i] : sr[prev][i];
    double gsj[kTinyCM], cacc[kTinyCM];
#pragma unroll
    for (int c = 0; c < kTinyCM; ++c) {
      const int j = l + 64 * c;
      gsj[c] = j < n ? (extract_bits(w0, j, 1) ? -scl[prev][j] : scl[prev][j]) : 0.0;
      cacc[c] = 0.0;
    }
    __syncthreads();
    // Row sums, 16 rows at a time: each lane's partials of the 16 rows are reduced over
    // the wavefront by halving exchanges (lane bit 5, 4, 3, 2: the lane keeps the half of
    // the rows selected by its bit and adds its partner's partials of that half), after
    // which lane l holds rows (l >> 2) & 15 summed over the 16 lanes that share bits 2-5,
    // and two more exchanges (bits 1, 0) complete the sums in all four lanes of a quad.
    // Quad lane 0 keeps batch 0's sum (rows 0-15), quad lane 1 batch 1's (rows 16-24).
    double ss = 0.0;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      double v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int r = 16 * b + q, i = w + kTinyWaves * r;
        v[q] = 0.0;
        if (r < kTinyRM && i < m) {
          const double gi = gsr[i];
#pragma unroll
          for (int c = 0; c < kTinyCM; ++c) {
            v[q] += Ar[r][c] * gsj[c];
            cacc[c] += Ar[r][c] * gi;
          }
        }
      }
      const bool b5 = l & 32, b4 = l & 16, b3 = l & 8, b2 = l & 4;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double send = b5 ? v[q] : v[q + 8], keep = b5 ? v[q + 8] : v[q];
        v[q] = keep + __shfl_xor(send, 32);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double send = b4 ? v[q] : v[q + 4], keep = b4 ? v[q + 4] : v[q];
        v[q] = keep + swizzle_xor16(send);
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const double send = b3 ? v[q] : v[q + 2], keep = b3 ? v[q + 2] : v[q];
        v[q] = keep + dpp_mov<0x140>(send);  // row_mirror: partner differs in bit 3
      }
      {
        const double send = b2 ? v[0] : v[1], keep = b2 ? v[1] : v[0];
        v[0] = keep + dpp_mov<0x141>(send);  // row_half_mirror: partner differs in bit 2
      }
      v[0] += dpp_mov<0x4E>(v[0]);  // quad_perm [2, 3, 0, 1]
      v[0] += dpp_mov<0xB1>(v[0]);  // quad_perm [1, 0, 3, 2]
      if ((l & 3) == b) ss = v[0] * v[0];
    }
#pragma unroll
    for (int c = 0; c < kTinyCM; ++c) part[w][l + 64 * c] = cacc[c];
    __syncthreads();
    // Both sides' updates in one code path: rows on quad lanes 0 and 1 (the lanes that
    // hold their sums), columns on quad lanes 2 and 3 (the sum of the 8 wavefront
    // partials, in wavefront order), so the exp / divide chain of the update is paid once.
    {
      const int quad = l & 3;
      const bool is_row = quad < 2;
      int idx;
      bool live;
      if (is_row) {
        const int r = (quad == 1 ? 16 : 0) + (l >> 2);
        idx = w + kTinyWaves * r;
        live = r < kTinyRM && idx < m;
      } else {
        idx = w * 32 + (l >> 2) * 2 + (quad - 2);
        live = idx < n;
        if (live) {
          double y = 0.0;
#pragma unroll
          for (int q = 0; q < kTinyWaves; ++q) y += part[q][idx];
          ss = y * y;
        }
      }
      if (live) {
        double* xs = is_row ? xu : xv;
        double* xbs = is_row ? xub : xvb;
        double* out = is_row ? sr[cur] : scl[cur];
        double xi = xs[idx], xb = xbs[idx];
        if (!sgd_update(ss, 1, is_row ? a.tgt_row : a.tgt_col, sc, xi, xb)) atomicOr(a.flag, 1);
        xs[idx] = xi;
        xbs[idx] = xb;
        out[idx] = exp(xi);
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < m; i += kTinyThreads) {
    a.u[i] = xu[i];
    a.ub[i] = xub[i];
  }
  for (int j = tid; j < n; j += kTinyThreads) {
    a.v[j] = xv[j];
    a.vb[j] = xvb[j];
  }
}

__global__ void k_transpose(const double* __restrict__ A, int64_t m, int64_t n, int64_t ld, double* __restrict__ AT) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * n) return;
  const int64_t i = idx / n, j = idx % n;
  AT[j * m + i] = A[i * ld + j];
}

// Device buffers from hipMalloc, freed when the run returns.
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

// Device buffers carved from one caller-provided region (256-byte aligned pieces); with
// base == nullptr it only adds up the bytes the pieces need.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, off = 0;
  template <class T>
  int alloc(T** out, int64_t n) {
    off = (off + 255) & ~(size_t)255;
    const size_t b = sizeof(T) * (size_t)std::max<int64_t>(n, 1);
    *out = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += b;
    if (base && off > cap) return set_error(MFE_EDIM, "scratch of %zu bytes exceeded", cap);
    return MFE_OK;
  }
};

__global__ void k_zero_words(uint64_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// The two sign segments of a dense run and their block prefix (written on the device, so
// that a run makes no host-to-device copy), and the run's status flag cleared.
__global__ void k_sign_tables(SignSeg* __restrict__ segs, int64_t* __restrict__ prefix, SignSeg h0, SignSeg h1,
                              int* __restrict__ flag) {
  if (threadIdx.x != 0) return;
  segs[0] = h0;
  segs[1] = h1;
  prefix[0] = 0;
  prefix[1] = h0.nblocks;
  prefix[2] = h0.nblocks + h1.nblocks;
  *flag = 0;
}

void zero_words(uint64_t* p, int64_t n, hipStream_t st) {
  if (n > 0) k_zero_words<<<dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st>>>(p, n);
}

// Sign words of one matrix: side 0 (columns, n*k bits) and side 1 (rows, m*k bits) in
// one slot; the slot is refilled every step.
struct DenseSigns {
  SignSeg h[2];
  SignSeg* segs = nullptr;
  int64_t* prefix = nullptr;
  uint64_t* words = nullptr;
  int64_t nwords = 0, nblocks = 0, off_rows = 0;
  template <class Alloc>
  int alloc(Alloc& B, int64_t m, int64_t n, int k, int64_t batch) {
    h[0].ctrl_lo = ((uint64_t)batch << 34) | 0ull;
    h[0].nblocks = ceil_div(n * k, 256);
    h[0].word_off = 0;
    h[1].ctrl_lo = ((uint64_t)batch << 34) | 1ull;
    h[1].nblocks = ceil_div(m * k, 256);
    h[1].word_off = 4 * h[0].nblocks + 4;
    off_rows = h[1].word_off;
    nblocks = h[0].nblocks + h[1].nblocks;
    nwords = h[1].word_off + 4 * h[1].nblocks + 4;
    MFE_CHECK(B.alloc(&segs, 2));
    MFE_CHECK(B.alloc(&prefix, 3));
    MFE_CHECK(B.alloc(&words, nwords));
    return MFE_OK;
  }
  // tables and the flag on the device, words cleared (no host copy, no memset node)
  int setup(int* flag, hipStream_t st) const {
    k_sign_tables<<<dim3(1), dim3(64), 0, st>>>(segs, prefix, h[0], h[1], flag);
    zero_words(words, nwords, st);
    MFE_HIP(hipGetLastError());
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

// Everything one dense FP64 run uses on the device, allocated before any launch: the
// iterates, averages and scales of both sides, the status flag, the sign words, and for
// the persistent paths the transposed copy of A and the staged sign words of a chunk.
struct DenseWork {
  double *u, *ub, *v, *vb, *su[2], *sv[2];
  int* flag;
  DenseSigns S;
  bool tiny = false, persistent = false;
  int32_t nb0 = 0, nb1 = 0, wps = 0;
  size_t lds = 0;
  int chunk = 0;
  double* AT = nullptr;
  uint64_t* sw = nullptr;

  template <class Alloc>
  int alloc(Alloc& B, int64_t m, int64_t n, int k, int steps, int64_t batch) {
    MFE_CHECK(B.alloc(&u, m));
    MFE_CHECK(B.alloc(&ub, m));
    MFE_CHECK(B.alloc(&v, n));
    MFE_CHECK(B.alloc(&vb, n));
    for (int i = 0; i < 2; ++i) {
      MFE_CHECK(B.alloc(&su[i], m));
      MFE_CHECK(B.alloc(&sv[i], n));
    }
    MFE_CHECK(B.alloc(&flag, 1));
    MFE_CHECK(S.alloc(B, m, n, k, batch));
    nb0 = (int32_t)ceil_div(n * k, 256);
    nb1 = (int32_t)ceil_div(m * k, 256);
    wps = 4 * (nb0 + nb1) + 8;
    tiny = k == 1 && m <= kTinyWaves * kTinyRM && n <= 64 * kTinyCM && wps <= kTinyThreads;
    lds = sizeof(double) * (size_t)(4 * (m + n)) + sizeof(uint64_t) * (size_t)(2 * wps);
    persistent = tiny || (k <= 16 && m + n <= kPersistMaxDim && m * n * k <= kPersistMaxWork && lds <= 65536 &&
                          wps <= kPersistMaxWords);
    if (persistent && steps > 0) {
      if (!tiny) MFE_CHECK(B.alloc(&AT, m * n));
      chunk = std::min(steps, kPersistChunk);
      MFE_CHECK(B.alloc(&sw, (int64_t)chunk * wps));
    }
    return MFE_OK;
  }
};

// The launches of one dense FP64 run on buffers already in place (no allocation).
int dense_f64_run(const DenseWork& w, const mfe_matrix* A, const mfe_equil_params* p, double* d, double* e,
                  double* u_bar, double* v_bar) {
  hipStream_t st = (hipStream_t)p->stream;
  const int64_t m = A->m, n = A->n;
  const int k = p->probes;
  double *u = w.u, *ub = w.ub, *v = w.v, *vb = w.vb;
  int* flag = w.flag;
  MFE_CHECK(w.S.setup(flag, st));
  k_dense_init<<<dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st>>>(m, p->u0, p->box_M, u, ub, w.su[0], flag);
  k_dense_init<<<dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st>>>(n, p->v0, p->box_M, v, vb, w.sv[0], flag);
  const double* Ad = (const double*)A->data;
  if (w.persistent && p->steps > 0) {
    if (!w.tiny)
      k_transpose<<<dim3((unsigned)ceil_div(m * n, 256)), dim3(256), 0, st>>>(Ad, m, n, A->ld, w.AT);
    zero_words(w.sw, (int64_t)w.chunk * w.wps, st);
    PersistArgs pa;
    pa.A = Ad;
    pa.AT = w.AT;
    pa.m = m;
    pa.n = n;
    pa.ld = A->ld;
    pa.u = u;
    pa.ub = ub;
    pa.v = v;
    pa.vb = vb;
    pa.k = k;
    pa.t0 = (double)p->t0;
    pa.gamma = p->gamma;
    pa.M = p->box_M;
    pa.tgt_row = p->alpha * p->alpha;
    pa.tgt_col = p->beta * p->beta;
    pa.sw = w.sw;
    pa.nb0 = w.nb0;
    pa.wps = w.wps;
    pa.flag = flag;
    for (int t1 = 1; t1 <= p->steps; t1 += w.chunk) {
      const int ns = std::min(w.chunk, p->steps - t1 + 1);
      k_sign_chunk<<<dim3((unsigned)ceil_div((int64_t)ns * (w.nb0 + w.nb1), 256)), dim3(256), 0, st>>>(
          w.sw, t1, ns, w.nb0, w.nb1, w.wps, p->seed, p->batch);
      pa.t_begin = (double)t1;
      pa.nsteps = ns;
      const dim3 g(1), b(kPersistThreads);
      if (w.tiny) k_dense_tiny<<<g, dim3(kTinyThreads), 0, st>>>(pa);
      else if (k <= 1) k_dense_persistent<1><<<g, b, w.lds, st>>>(pa);
      else if (k <= 2) k_dense_persistent<2><<<g, b, w.lds, st>>>(pa);
      else if (k <= 4) k_dense_persistent<4><<<g, b, w.lds, st>>>(pa);
      else if (k <= 8) k_dense_persistent<8><<<g, b, w.lds, st>>>(pa);
      else k_dense_persistent<16><<<g, b, w.lds, st>>>(pa);
      MFE_HIP(hipGetLastError());
    }
  } else {
    for (int t = 1; t <= p->steps; ++t) {
      MFE_CHECK(w.S.draw(p->seed, (uint64_t)t, st));
      const int cur = t & 1, prev = cur ^ 1;
      DenseSide R{u, ub, w.sv[prev], w.su[cur], w.S.words, p->alpha * p->alpha};                 // gathers s (side 0)
      DenseSide C{v, vb, w.su[prev], w.sv[cur], w.S.words + w.S.off_rows, p->beta * p->beta};  // gathers w (side 1)
      const StepScalars sc = scalars(p, t);
      if (k <= 1) launch_dense_step<1>(Ad, m, n, A->ld, R, C, k, sc, flag, st);
      else if (k <= 2) launch_dense_step<2>(Ad, m, n, A->ld, R, C, k, sc, flag, st);
      else if (k <= 4) launch_dense_step<4>(Ad, m, n, A->ld, R, C, k, sc, flag, st);
      else if (k <= 8) launch_dense_step<8>(Ad, m, n, A->ld, R, C, k, sc, flag, st);
      else if (k <= 16) launch_dense_step<16>(Ad, m, n, A->ld, R, C, k, sc, flag, st);
      else if (k <= 32) launch_dense_step<32>(Ad, m, n, A->ld, R, C, k, sc, flag, st);
      else launch_dense_step<64>(Ad, m, n, A->ld, R, C, k, sc, flag, st);
    }
  }
  MFE_HIP(hipGetLastError());
  k_dense_output<<<dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st>>>(m, ub, d, u_bar);
  k_dense_output<<<dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st>>>(n, vb, e, v_bar);
  MFE_HIP(hipGetLastError());
  return finish(flag, st);
}

int dense_checks(const mfe_matrix* A, const mfe_equil_params* p) {
  if (!A->data) return set_error(MFE_EINVAL, "dense data is NULL");
  if (A->ld < A->n) return set_error(MFE_EDIM, "ld < n");
  if (p->probes > 64) return set_error(MFE_EUNSUPPORTED, "dense FP64 path supports at most 64 probes per step");
  return MFE_OK;
}

// ---- the allocation-free variant: the file-scope scratch array above, one per device

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

int scratch_for_current_device(char** out) {
  int dev = -1;
  MFE_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_error(MFE_EDEVICE, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(::scratch));
    if (e != hipSuccess || !ptr)
      return set_error(MFE_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = (char*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return MFE_OK;
}

}  // namespace

int dense_f64_equilibrate(const mfe_matrix* A, const mfe_equil_params* p, double* d, double* e, double* u_bar,
                          double* v_bar) {
  MFE_CHECK(dense_checks(A, p));
  Bufs B;
  DenseWork w;
  MFE_CHECK(w.alloc(B, A->m, A->n, p->probes, p->steps, p->batch));
  return dense_f64_run(w, A, p, d, e, u_bar, v_bar);
}

int dense_f64_equilibrate_noalloc(const mfe_matrix* A, const mfe_equil_params* p, double* d, double* e,
                                  double* u_bar, double* v_bar) {
  MFE_CHECK(dense_checks(A, p));
  Arena need;
  DenseWork w;
  MFE_CHECK(w.alloc(need, A->m, A->n, p->probes, p->steps, p->batch));
  if (need.off > kScratchBytes)
    return set_error(MFE_EDIM,
                     "a %lld x %lld run with %d probes needs %zu bytes of scratch; the allocation-free entry point "
                     "has %zu (use mfe_equilibrate)",
                     (long long)A->m, (long long)A->n, p->probes, need.off, kScratchBytes);
  char* base = nullptr;
  MFE_CHECK(scratch_for_current_device(&base));
  Arena ar;
  ar.base = base;
  ar.cap = kScratchBytes;
  MFE_CHECK(w.alloc(ar, A->m, A->n, p->probes, p->steps, p->batch));
  return dense_f64_run(w, A, p, d, e, u_bar, v_bar);
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
  MFE_CHECK(S.alloc(B, m, n, k, p->batch));
  MFE_CHECK(S.setup(flag, st));
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
