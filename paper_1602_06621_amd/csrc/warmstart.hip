// Learned warm start for Algorithm 1: probe sketches -> per-index features -> a small
// MLP -> initial (u0, v0), used with a step offset t0 (tau = t + t0).
//
// Sketch.  At (u, v) = 0 the estimator of Section 3.1 with ks probes per side gives
// r_i ~ ||row_i(A)||^2 and c_j ~ ||col_j(A)||^2 (probe signs: sides 2 and 3 of the
// stream, step 0).  For A = diag(a) G diag(b) with iid unit-variance G, the scalings
// u_i = -1/2 log r_i + c, v_j = -1/2 log c_j + c with e^(4c) = alpha^2 F / n (F the
// squared Frobenius norm) equilibrate A in expectation; that closed form is the
// "sketch initialisation".  The network learns the correction from it to the
// regularised optimum (labels: plain projected SGD run to convergence).
//
// Features of an index (row or column of matrix b), FP32:
//   f0 = (l - mean l)/4   l = log of its sketch norm estimate, mean over its side of b
//   f1 = s/4              the sketch initialisation (clipped to the box)
//   f2 = log(target)      log alpha^2 (rows) or log beta^2 (columns)
//   f3 = std(l)/4         spread of the log norms over its side of b
//   f4 = 1 for rows, 0 for columns
//   f5 = log(m_b / n_b)
//   f6 = c                the constant of the sketch initialisation
//   f7 = log(max_p y_p^2 / mean_p y_p^2) (sketch noise of this index; 0 if empty)
//
// Network: h1 = tanh(x W1 + b1), h2 = tanh(h1 W2 + b2), y = h2 w3 + b3, width 64, FP32.
// Parameters in one flat FP32 vector: W1 (F x 64, row-major), b1, W2 (64 x 64), b2, w3, b3.
// Training: mean squared error, Adam (Kingma & Ba), mini-batches drawn with replacement
// by a counter-based Philox stream; every reduction is fixed-order (deterministic).
#include <cmath>
#include <cstring>
#include <vector>

#include "sparse.h"

namespace mfe {
namespace {

constexpr int kH = 64;
constexpr int kF = 8;
constexpr int kP = kF * kH + kH + kH * kH + kH + kH + 1;  // 4801 parameters

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

// Bump allocation inside one device buffer (256-byte aligned pieces); a first pass with
// base == nullptr only measures.
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(int64_t n) {
    off = (off + 255) & ~(size_t)255;
    T* r = reinterpret_cast<T*>(base + off);
    off += sizeof(T) * (size_t)std::max<int64_t>(n, 1);
    return base ? r : nullptr;
  }
};

// ---------------------------------------------------------------- sketch

// Per index (internal order, one direction): y_p = sum_q a_q (-1)^bit(other index, p)
// for p < ks, at u = v = 0.  Writes, in original order, the estimate mean_p y_p^2 and
// the ratio max_p y_p^2 / mean.
template <int KS>
__global__ __launch_bounds__(256) void k_sketch(SideDev S, const MatDev* __restrict__ mats,
                                                const uint64_t* __restrict__ sw_other,
                                                const int64_t* __restrict__ word_base_other,
                                                const int32_t* __restrict__ other_mat_of_int,
                                                const int32_t* __restrict__ other_orig,
                                                double* __restrict__ est, double* __restrict__ ratio) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= S.nint) return;
  const int32_t li = S.orig[r];
  if (li < 0) return;
  const int64_t s = r >> 6;
  const int lane = (int)(r & 63);
  const int len = S.len[r];
  const int2* e = S.ent + S.slice_off[s] + lane;
  double acc[KS];
#pragma unroll
  for (int p = 0; p < KS; ++p) acc[p] = 0.0;
  for (int q = 0; q < len; ++q) {
    const int2 en = e[(int64_t)q * kSlice];
    const int32_t o = en.x;  // other direction, internal index
    const int32_t b = other_mat_of_int[o >> 6];
    const int64_t g = (int64_t)other_orig[o] * KS;
    const uint64_t bits = extract_bits(sw_other + word_base_other[b], g, KS);
    accumulate_signed<KS>(acc, (double)__int_as_float(en.y), bits);
  }
  double mean = 0.0, mx = 0.0;
#pragma unroll
  for (int p = 0; p < KS; ++p) {
    const double y2 = acc[p] * acc[p];
    mean += y2;
    mx = fmax(mx, y2);
  }
  mean /= KS;
  const MatDev mt = mats[S.slice_mat[s]];
  const int64_t gi = (S.is_row ? mt.row_orig_base : mt.col_orig_base) + li;
  est[gi] = mean;
  ratio[gi] = mean > 0.0 ? mx / mean : 0.0;
}

// Per matrix and side: mean and std of log(est) over the non-empty indices, and the sum
// of est; stats[b] = {mean, std, sum}.  Two stages with a fixed order (deterministic):
// workgroup (b, c) reduces chunk c of matrix b's range into part[b][c] = {sum log,
// sum log^2, count, sum}; then one thread per matrix adds the chunks in order.
constexpr int kStatChunks = 64;

__global__ __launch_bounds__(256) void k_side_partial(const double* __restrict__ est, const int64_t* __restrict__ base,
                                                      double* __restrict__ part) {
  __shared__ double sh[4][256];
  const int b = blockIdx.x, c = blockIdx.y;
  const int64_t lo = base[b], hi = base[b + 1];
  const int64_t len = (hi - lo + kStatChunks - 1) / kStatChunks;
  const int64_t c0 = lo + (int64_t)c * len, c1 = c0 + len < hi ? c0 + len : hi;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = c0 + threadIdx.x; i < c1; i += 256) {
    const double x = est[i];
    v[3] += x;
    if (x > 0) {
      const double l = log(x);
      v[0] += l;
      v[1] += l * l;
      v[2] += 1.0;
    }
  }
  for (int q = 0; q < 4; ++q) sh[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 4; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[((int64_t)b * kStatChunks + c) * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_side_final(const double* __restrict__ part, int count, double* __restrict__ stats) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= count) return;
  double S1 = 0, S2 = 0, C = 0, sum = 0;
  for (int c = 0; c < kStatChunks; ++c) {
    const double* q = part + ((int64_t)b * kStatChunks + c) * 4;
    S1 += q[0];
    S2 += q[1];
    C += q[2];
    sum += q[3];
  }
  const double mean = C > 0 ? S1 / C : 0.0;
  const double var = C > 0 ? fmax(S2 / C - mean * mean, 0.0) : 0.0;
  stats[3 * b + 0] = mean;
  stats[3 * b + 1] = sqrt(var);
  stats[3 * b + 2] = sum;
}

struct FeatMat {
  double tgt_row, tgt_col;  // alpha^2, beta^2
  double log_mn;            // log(m / n)
  int64_t row_base, col_base;
  int64_t m, n;
};

// Features and sketch initialisation of one side (original order), matrix per index
// found by binary search over the bases.
__global__ void k_features(const double* __restrict__ est, const double* __restrict__ ratio,
                           const double* __restrict__ stats, const double* __restrict__ stats_r,
                           const double* __restrict__ stats_c, const FeatMat* __restrict__ fm, int count, int is_row,
                           int64_t total, double gamma, double M, float* __restrict__ feat,
                           double* __restrict__ sketch_init) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((is_row ? fm[mid].row_base : fm[mid].col_base) <= i) lo = mid;
    else hi = mid - 1;
  }
  const FeatMat f = fm[lo];
  // e^(4c) = alpha^2 F / n, F = (sum of row estimates + sum of column estimates) / 2
  const double F = 0.5 * (stats_r[3 * lo + 2] + stats_c[3 * lo + 2]);
  const double fc = F > 0 ? 0.25 * log(f.tgt_row * F / (double)f.n) : 0.0;
  const double tgt = is_row ? f.tgt_row : f.tgt_col;
  const double x = est[i];
  const double mean = stats[3 * lo], sd = stats[3 * lo + 1];
  double s, l;
  if (x > 0) {
    l = log(x);
    s = -0.5 * l + fc;
  } else {
    l = mean;                         // no entries: no information about the norm
    s = fmin(tgt / gamma, M);         // where an index without entries settles (Section 2.3)
  }
  s = fmin(fmax(s, -M), M);
  sketch_init[i] = s;
  float* o = feat + i * kF;
  o[0] = (float)((l - mean) / 4.0);
  o[1] = (float)(s / 4.0);
  o[2] = (float)log(tgt);
  o[3] = (float)(sd / 4.0);
  o[4] = is_row ? 1.f : 0.f;
  o[5] = (float)f.log_mn;
  o[6] = (float)fc;
  o[7] = (float)(ratio[i] > 0 ? log(ratio[i]) : 0.0);
}

// ---------------------------------------------------------------- network

__device__ inline void philox_index(uint64_t seed, uint64_t it, uint64_t b, int64_t count, int64_t& out) {
  const U64x4 w = philox4x64_10(b + 1, 0, 0, 0, seed, (it << 2) | 3ull);
  out = (int64_t)(w.x[0] % (uint64_t)count);
}

// Training forward and backward: kLanesPerSample threads per sample, each owning a
// quarter of the hidden units; the sample's first hidden layer (forward) or output-layer
// deltas (backward) are exchanged through LDS.  A 4096-sample batch spreads over 64
// workgroups.  With one sample per thread (16 workgroups) the two kernels took 49.6 and
// 39.1 us per batch.
constexpr int kLanesPerSample = 4;
constexpr int kPart = kH / kLanesPerSample;
constexpr int kSamplesPerWg = 256 / kLanesPerSample;

int64_t train_grid(int64_t count) { return ceil_div(count, (int64_t)kSamplesPerWg); }

// Forward for `count` samples (rows of X, or X[idx[b]] when idx is given); keeps h1, h2
// (nullable) for the backward pass.  Parameters are staged in LDS.  Each unit's sums run
// in the same order as one sample per thread; the output adds the four threads' partial
// sums of w3 h2 pairwise.
__global__ __launch_bounds__(256) void k_mlp_fwd(const float* __restrict__ params, const float* __restrict__ X,
                                                 const int64_t* __restrict__ idx, int64_t count, float* __restrict__ y,
                                                 float* __restrict__ h1s, float* __restrict__ h2s) {
  __shared__ float P[kP];
  __shared__ float H1[kSamplesPerWg][kH + 1];
  for (int i = threadIdx.x; i < kP; i += 256) P[i] = params[i];
  const int q = (int)threadIdx.x % kLanesPerSample, ls = (int)threadIdx.x / kLanesPerSample;
  const int64_t b = (int64_t)blockIdx.x * kSamplesPerWg + ls;
  const bool live = b < count;
  const int64_t row = live ? (idx ? idx[b] : b) : 0;
  float x[kF];
#pragma unroll
  for (int f = 0; f < kF; ++f) x[f] = live ? X[row * kF + f] : 0.f;
  __syncthreads();  // parameters staged
  const float* W1 = P;
  const float* b1 = W1 + kF * kH;
  const float* W2 = b1 + kH;
  const float* b2 = W2 + kH * kH;
  const float* w3 = b2 + kH;
  const float b3 = w3[kH];
  const int j0 = q * kPart;
#pragma unroll
  for (int jj = 0; jj < kPart; ++jj) {
    const int j = j0 + jj;
    float a = b1[j];
#pragma unroll
    for (int f = 0; f < kF; ++f) a = fmaf(x[f], W1[f * kH + j], a);
    const float h = tanhf(a);
    H1[ls][j] = h;
    if (live && h1s) h1s[b * kH + j] = h;
  }
  __syncthreads();  // the sample's 64 first-layer units are in LDS
  float out = 0.f;
  for (int jj = 0; jj < kPart; ++jj) {
    const int j = j0 + jj;
    float a = b2[j];
#pragma unroll
    for (int i = 0; i < kH; ++i) a = fmaf(H1[ls][i], W2[i * kH + j], a);
    const float h = tanhf(a);
    if (live && h2s) h2s[b * kH + j] = h;
    out = fmaf(h, w3[j], out);
  }
  // the four partial sums (consecutive lanes of one wavefront), added pairwise
  out += __shfl_xor(out, 1, 64);
  out += __shfl_xor(out, 2, 64);
  if (live && q == 0) y[b] = b3 + out;
}

// Inference on the matrix cores (v_mfma_f32_32x32x2_f32, FP32 products and sums): a
// wavefront evaluates 32 samples at a time as H1' = tanh(W1' X' + b1) (64 x 32, eight
// MFMAs) and H2' = tanh(W2' H1' + b2) (64 x 32, 64 MFMAs), then y = w3' H2' + b3 across the
// lanes.  Accumulator layout of a 32 x 32 block: lane l, register v holds row
// 8 (v/4) + 4 (l/32) + v%4, column l%32.  The second product takes the first one's
// accumulators as its B operand as they are -- step (t, v) pairs hidden unit
// 32 t + 8 (v/4) + v%4 (lanes 0-31) with the one 4 above it (lanes 32-63) -- and each lane
// holds the matching entries of W2 (64 per lane, loaded once per wavefront), so no data
// moves between the layers.  The order of the 64-term sums differs from the per-sample
// kernel's; both are FP32.  tanh is evaluated as 1 - 2 / (e^(2x) + 1) with the hardware
// exponential and reciprocal (absolute error about 1e-7; the outputs feed a warm start).
typedef float f32x16v __attribute__((ext_vector_type(16)));

__device__ inline float tanh_fast(float x) {
  const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);  // e^(2x) = 2^(2x log2 e)
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

__device__ inline int acc_row(int v, int lane) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

__global__ __launch_bounds__(256) void k_mlp_infer(const float* __restrict__ params, const float* __restrict__ X,
                                                   int64_t count, float* __restrict__ y) {
  const int lane = (int)(threadIdx.x & 63);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const float* W1 = params;            // [F][H]
  const float* b1 = W1 + kF * kH;
  const float* W2 = b1 + kH;           // [in][out]
  const float* b2 = W2 + kH * kH;
  const float* w3 = b2 + kH;
  const float b3 = w3[kH];
  const int col = lane & 31, half = lane >> 5;
  // biases and w3 in LDS, read at the lane's accumulator rows; per-lane operands in
  // registers: W1 as the A operand of step s, tile t, and W2 at step (t, v), output tile o
  __shared__ float vb1[kH], vb2[kH], vw3[kH];
  for (int i = threadIdx.x; i < kH; i += blockDim.x) {
    vb1[i] = b1[i];
    vb2[i] = b2[i];
    vw3[i] = w3[i];
  }
  __syncthreads();
  float a1[2][4], a2[2][2][16];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int s = 0; s < 4; ++s) a1[t][s] = W1[(2 * s + half) * kH + 32 * t + col];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int in = 32 * t + acc_row(v, lane);  // the hidden unit this lane brings to step (t, v)
#pragma unroll
      for (int o = 0; o < 2; ++o) a2[o][t][v] = W2[in * kH + 32 * o + col];
    }
  const int64_t nblk = (count + 31) / 32;
  for (int64_t blk = wave; blk < nblk; blk += nwaves) {  // the same trip count for all lanes of a wave
    const int64_t smp = blk * 32 + col;
    const bool live = smp < count;
    float xb[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) xb[s] = live ? X[smp * kF + 2 * s + half] : 0.f;
    f32x16v h1[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
      for (int v = 0; v < 16; ++v) h1[t][v] = vb1[32 * t + acc_row(v, lane)];
#pragma unroll
      for (int s = 0; s < 4; ++s) h1[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[t][s], xb[s], h1[t], 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 16; ++v) h1[t][v] = tanh_fast(h1[t][v]);
    }
    f32x16v h2[2];
#pragma unroll
    for (int o = 0; o < 2; ++o)
#pragma unroll
      for (int v = 0; v < 16; ++v) h2[o][v] = vb2[32 * o + acc_row(v, lane)];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v)
#pragma unroll
        for (int o = 0; o < 2; ++o) h2[o] = __builtin_amdgcn_mfma_f32_32x32x2f32(a2[o][t][v], h1[t][v], h2[o], 0, 0, 0);
    float part = 0.f;
#pragma unroll
    for (int o = 0; o < 2; ++o)
#pragma unroll
      for (int v = 0; v < 16; ++v) part = fmaf(tanh_fast(h2[o][v]), vw3[32 * o + acc_row(v, lane)], part);
    // lanes l and l + 32 hold the two halves of sample l's hidden units
    const float other = __shfl_xor(part, 32);
    if (half == 0 && live) y[smp] = (part + other) + b3;
  }
}

// Per-sample backward: gy = 2 (y - t)/B, gh2 = gy w3 (1 - h2^2), gh1 = (gh2 W2') (1 - h1^2).
// Also the per-sample squared error for the loss.  Same layout as k_mlp_fwd; every sum
// runs in the same order as one sample per thread.
__global__ __launch_bounds__(256) void k_mlp_bwd(const float* __restrict__ params, const float* __restrict__ y,
                                                 const float* __restrict__ t, const int64_t* __restrict__ idx,
                                                 int64_t count, const float* __restrict__ h1s,
                                                 const float* __restrict__ h2s, float* __restrict__ gy,
                                                 float* __restrict__ gh1, float* __restrict__ gh2,
                                                 double* __restrict__ se) {
  __shared__ float P[kH * kH + 2 * kH];
  __shared__ float G2[kSamplesPerWg][kH + 1];
  const float* W2g = params + kF * kH + kH;
  for (int i = threadIdx.x; i < kH * kH; i += 256) P[i] = W2g[i];
  const float* w3g = W2g + kH * kH + kH;
  for (int i = threadIdx.x; i < kH; i += 256) P[kH * kH + i] = w3g[i];
  const int q = (int)threadIdx.x % kLanesPerSample, ls = (int)threadIdx.x / kLanesPerSample;
  const int64_t b = (int64_t)blockIdx.x * kSamplesPerWg + ls;
  const bool live = b < count;
  float g = 0.f;
  if (live) {
    const int64_t row = idx ? idx[b] : b;
    const float r = y[b] - t[row];
    g = 2.0f * r / (float)count;
    if (q == 0) {
      se[b] = (double)r * (double)r;
      gy[b] = g;
    }
  }
  __syncthreads();  // W2, w3 staged
  const float* W2 = P;
  const float* w3 = P + kH * kH;
  const int j0 = q * kPart;
#pragma unroll
  for (int jj = 0; jj < kPart; ++jj) {
    const int j = j0 + jj;
    const float h = live ? h2s[b * kH + j] : 0.f;
    const float g2 = g * w3[j] * (1.0f - h * h);
    G2[ls][j] = g2;
    if (live) gh2[b * kH + j] = g2;
  }
  __syncthreads();  // the sample's 64 output-layer deltas are in LDS
  for (int ii = 0; ii < kPart; ++ii) {
    const int i = j0 + ii;
    float a = 0.f;
#pragma unroll
    for (int j = 0; j < kH; ++j) a = fmaf(G2[ls][j], W2[i * kH + j], a);
    if (live) {
      const float h = h1s[b * kH + i];
      gh1[b * kH + i] = a * (1.0f - h * h);
    }
  }
}

// Weight gradients in two deterministic stages.  Stage one: workgroup c sums samples
// [c S, min((c + 1) S, count)) for every parameter in FP64, in sample order, staging
// kWgTile samples' activations and deltas at a time in LDS (coalesced loads; each
// thread owns parameters tid, tid + 256, ...).  Stage two adds each parameter's chunk
// partials in a fixed order.  With one thread per parameter looping over the whole batch
// (strided loads, 19 workgroups) the gradient of a 4096-sample batch took ~1.2 ms.
constexpr int kWgTile = 32;
constexpr int kWgMaxChunks = 512;
constexpr int kWgPer = (kP + 255) / 256;

int64_t wgrad_chunks(int64_t count) {
  return std::max<int64_t>(1, std::min<int64_t>(ceil_div(count, (int64_t)kWgTile), kWgMaxChunks));
}

__global__ __launch_bounds__(256) void k_mlp_wgrad_part(const float* __restrict__ X, const int64_t* __restrict__ idx,
                                                        int64_t count, int64_t S, const float* __restrict__ gy,
                                                        const float* __restrict__ h1s, const float* __restrict__ h2s,
                                                        const float* __restrict__ gh1, const float* __restrict__ gh2,
                                                        double* __restrict__ part) {
  __shared__ float sx[kWgTile][kF];
  __shared__ float sh1[kWgTile][kH];
  __shared__ float sh2[kWgTile][kH];
  __shared__ float sg1[kWgTile][kH];
  __shared__ float sg2[kWgTile][kH];
  __shared__ float sgy[kWgTile];
  const int tid = threadIdx.x;
  const int64_t b0 = (int64_t)blockIdx.x * S;
  const int64_t b1 = b0 + S < count ? b0 + S : count;
  double acc[kWgPer];
#pragma unroll
  for (int r = 0; r < kWgPer; ++r) acc[r] = 0.0;
  for (int64_t tb = b0; tb < b1; tb += kWgTile) {
    const int nt = (int)(b1 - tb < kWgTile ? b1 - tb : kWgTile);
    __syncthreads();  // the previous tile has been consumed
    for (int i = tid; i < nt * kH; i += 256) {
      const int64_t g = tb * kH + i;  // samples tb .. tb + nt - 1 are contiguous rows
      sh1[i / kH][i % kH] = h1s[g];
      sh2[i / kH][i % kH] = h2s[g];
      sg1[i / kH][i % kH] = gh1[g];
      sg2[i / kH][i % kH] = gh2[g];
    }
    for (int i = tid; i < nt * kF; i += 256) {
      const int64_t b = tb + i / kF;
      sx[i / kF][i % kF] = X[(idx ? idx[b] : b) * kF + i % kF];
    }
    if (tid < nt) sgy[tid] = gy[tb + tid];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kWgPer; ++r) {
      const int p = tid + 256 * r;
      double a = acc[r];
      if (p < kF * kH) {  // W1[f][j]
        const int f = p / kH, j = p % kH;
        for (int q = 0; q < nt; ++q) a += (double)sx[q][f] * sg1[q][j];
      } else if (p < kF * kH + kH) {  // b1[j]
        const int j = p - kF * kH;
        for (int q = 0; q < nt; ++q) a += sg1[q][j];
      } else if (p < kF * kH + kH + kH * kH) {  // W2[i][j]
        const int o = p - (kF * kH + kH), i = o / kH, j = o % kH;
        for (int q = 0; q < nt; ++q) a += (double)sh1[q][i] * sg2[q][j];
      } else if (p < kF * kH + 2 * kH + kH * kH) {  // b2[j]
        const int j = p - (kF * kH + kH + kH * kH);
        for (int q = 0; q < nt; ++q) a += sg2[q][j];
      } else if (p < kF * kH + 3 * kH + kH * kH) {  // w3[j]
        const int j = p - (kF * kH + 2 * kH + kH * kH);
        for (int q = 0; q < nt; ++q) a += (double)sgy[q] * sh2[q][j];
      } else if (p < kP) {  // b3
        for (int q = 0; q < nt; ++q) a += sgy[q];
      }
      acc[r] = a;
    }
  }
#pragma unroll
  for (int r = 0; r < kWgPer; ++r) {
    const int p = tid + 256 * r;
    if (p < kP) part[(int64_t)blockIdx.x * kP + p] = acc[r];
  }
}

// Four consecutive lanes per parameter: lane l adds chunks l, l + 4, ... in order, then
// the four sums are added pairwise.
__global__ __launch_bounds__(256) void k_mlp_wgrad_sum(const double* __restrict__ part, int chunks,
                                                       float* __restrict__ grad) {
  const int p = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 2), l = (int)(threadIdx.x & 3);
  double acc = 0.0;
  if (p < kP) {
#pragma unroll 4
    for (int c = l; c < chunks; c += 4) acc += part[(int64_t)c * kP + p];
  }
  acc += __shfl_xor(acc, 1, 64);
  acc += __shfl_xor(acc, 2, 64);
  if (p < kP && l == 0) grad[p] = (float)acc;
}

// grad = the batch's weight gradient; part holds wgrad_chunks(count) x kP doubles.
void launch_wgrad(const float* X, const int64_t* idx, int64_t count, const float* gy, const float* h1,
                  const float* h2, const float* g1, const float* g2, double* part, float* grad, hipStream_t st) {
  const int64_t C = wgrad_chunks(count);
  const int64_t S = ceil_div(count, C);
  k_mlp_wgrad_part<<<dim3((unsigned)C), dim3(256), 0, st>>>(X, idx, count, S, gy, h1, h2, g1, g2, part);
  k_mlp_wgrad_sum<<<dim3((unsigned)ceil_div((int64_t)kP * 4, (int64_t)256)), dim3(256), 0, st>>>(part, (int)C,
                                                                                                 grad);
}

__global__ void k_sum(const double* __restrict__ v, int64_t n, double scale, double* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += v[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0] * scale;
}

__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int step, float lr) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kP) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float gi = g[p];
  const float mi = b1 * m[p] + (1.f - b1) * gi;
  const float vi = b2 * v[p] + (1.f - b2) * gi * gi;
  m[p] = mi;
  v[p] = vi;
  const float mh = mi / (1.f - powf(b1, (float)step));
  const float vh = vi / (1.f - powf(b2, (float)step));
  th[p] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_batch_indices(uint64_t seed, uint64_t it, int64_t count, int64_t total, int64_t* __restrict__ idx) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < count) philox_index(seed, it, (uint64_t)b, total, idx[b]);
}

__global__ void k_apply_delta(int64_t n, const double* __restrict__ s, const float* __restrict__ d, double M,
                              double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = fmin(fmax(s[i] + (double)(d ? d[i] : 0.f), -M), M);
}

// One training sample per thread, for one side: sample s of matrix b is stratum
// c = s - soff[b] of that matrix's cnt = soff[b+1] - soff[b] strata over its nb indices,
// [floor(c nb / cnt), floor((c+1) nb / cnt)), at a Philox offset inside the stratum.
// Copies the index's features and writes label - sketch (rounded once to FP32).
__global__ void k_training_samples(const int64_t* __restrict__ soff, const int64_t* __restrict__ ibase,
                                   int count, int side, uint64_t seed, const float* __restrict__ feat,
                                   const double* __restrict__ label, const double* __restrict__ sketch,
                                   int64_t out0, float* __restrict__ X, float* __restrict__ t,
                                   int64_t* __restrict__ idx) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= soff[count]) return;
  int lo = 0, hi = count;  // the matrix b with soff[b] <= s < soff[b+1]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (soff[mid] <= s) lo = mid;
    else hi = mid;
  }
  const int b = lo;
  const int64_t cnt = soff[b + 1] - soff[b], nb = ibase[b + 1] - ibase[b], c = s - soff[b];
  const int64_t a = (int64_t)(((unsigned __int128)c * (uint64_t)nb) / (uint64_t)cnt);
  const int64_t e = (int64_t)(((unsigned __int128)(c + 1) * (uint64_t)nb) / (uint64_t)cnt);
  int64_t off;
  philox_index(seed, ((uint64_t)b << 1) | (uint64_t)side, (uint64_t)c, e - a, off);
  const int64_t g = ibase[b] + a + off;
  const int64_t o = out0 + s;
  for (int f = 0; f < kF; ++f) X[o * kF + f] = feat[g * kF + f];
  t[o] = (float)(label[g] - sketch[g]);
  if (idx) idx[o] = g;
}

}  // namespace

// Inference grid: enough wavefronts to fill the device (blocks of 32 samples are shared
// out grid-stride, so the per-wavefront weight loads are amortised).
void launch_mlp_infer(const float* params, const float* X, int64_t count, float* y, hipStream_t st) {
  if (count <= 0) return;
  const int64_t waves = std::min<int64_t>((count + 31) / 32, 2048);
  k_mlp_infer<<<(unsigned)ceil_div(waves, 4), 256, 0, st>>>(params, X, count, y);
}

// ---------------------------------------------------------------- drivers

namespace {

// Sketch features with all scratch carved from `ws` (base == nullptr: measure only;
// the needed bytes are added to *bytes).
int sketch_impl(mfe_plan* p, uint64_t seed, int32_t ks, const double* alpha_b, const double* beta_b, double gamma,
                double M, float* feat_rows, float* feat_cols, double* u_sketch, double* v_sketch, hipStream_t st,
                char* ws, size_t* bytes) {
  const int count = p->count;
  // sketch sign words: side 2 (indexed by column) and side 3 (by row), step 0, batch b
  std::vector<SignSeg> segs;
  std::vector<int64_t> prefix{0}, wb_col(count), wb_row(count), rb(count + 1), cb(count + 1);
  int64_t words = 0, blocks = 0;
  for (int side = 2; side < 4; ++side)
    for (int b = 0; b < count; ++b) {
      const int64_t cnt = side == 2 ? p->meta[b].n : p->meta[b].m;
      SignSeg sg;
      sg.ctrl_lo = ((uint64_t)b << 34) | (uint64_t)side;
      sg.nblocks = ceil_div(cnt * ks, 256);
      sg.word_off = words;
      (side == 2 ? wb_col : wb_row)[b] = words;
      words += 4 * sg.nblocks + 4;
      blocks += sg.nblocks;
      prefix.push_back(blocks);
      segs.push_back(sg);
    }
  rb[0] = cb[0] = 0;
  std::vector<FeatMat> fm(count);
  for (int b = 0; b < count; ++b) {
    rb[b + 1] = rb[b] + p->meta[b].m;
    cb[b + 1] = cb[b] + p->meta[b].n;
    const double al = alpha_b ? alpha_b[b] : std::pow((double)p->meta[b].n / p->meta[b].m, 0.25);
    const double be = beta_b ? beta_b[b] : std::pow((double)p->meta[b].m / p->meta[b].n, 0.25);
    fm[b].tgt_row = al * al;
    fm[b].tgt_col = be * be;
    fm[b].log_mn = std::log((double)p->meta[b].m / p->meta[b].n);
    fm[b].row_base = rb[b];
    fm[b].col_base = cb[b];
    fm[b].m = p->meta[b].m;
    fm[b].n = p->meta[b].n;
  }
  // the host-built tables come first in the scratch and travel in one copy
  Carver cv{ws};
  SignSeg* d_segs = cv.take<SignSeg>((int64_t)segs.size());
  int64_t* d_prefix = cv.take<int64_t>((int64_t)prefix.size());
  int64_t* d_wb_col = cv.take<int64_t>(count);
  int64_t* d_wb_row = cv.take<int64_t>(count);
  int64_t* d_rbase = cv.take<int64_t>(count + 1);
  int64_t* d_cbase = cv.take<int64_t>(count + 1);
  FeatMat* d_fm = cv.take<FeatMat>(count);
  const size_t table_bytes = cv.off;
  uint64_t* sw = cv.take<uint64_t>(words);
  double* est_r = cv.take<double>(p->M);
  double* est_c = cv.take<double>(p->N);
  double* rat_r = cv.take<double>(p->M);
  double* rat_c = cv.take<double>(p->N);
  double* st_r = cv.take<double>(3 * count);
  double* st_c = cv.take<double>(3 * count);
  double* part_r = cv.take<double>((int64_t)count * kStatChunks * 4);
  double* part_c = cv.take<double>((int64_t)count * kStatChunks * 4);
  if (!ws) {
    *bytes += cv.off + 256;
    return MFE_OK;
  }
  // staged in the plan: the copy may read the host buffer after this function returns
  std::vector<char>& host = p->ws_host;
  host.assign(table_bytes, 0);
  auto put = [&](const void* dev, const void* src, size_t n) {
    std::memcpy(host.data() + ((const char*)dev - ws), src, n);
  };
  put(d_segs, segs.data(), sizeof(SignSeg) * segs.size());
  put(d_prefix, prefix.data(), sizeof(int64_t) * prefix.size());
  put(d_wb_col, wb_col.data(), sizeof(int64_t) * count);
  put(d_wb_row, wb_row.data(), sizeof(int64_t) * count);
  put(d_rbase, rb.data(), sizeof(int64_t) * (count + 1));
  put(d_cbase, cb.data(), sizeof(int64_t) * (count + 1));
  put(d_fm, fm.data(), sizeof(FeatMat) * count);
  MFE_HIP(hipMemcpyAsync(ws, host.data(), table_bytes, hipMemcpyHostToDevice, st));
  MFE_HIP(hipMemsetAsync(sw, 0, sizeof(uint64_t) * words, st));
  SignGenDev g;
  g.segs = d_segs;
  g.seg_prefix = d_prefix;
  g.nseg = (int32_t)segs.size();
  g.nblocks = blocks;
  g.seed = seed;
  g.step = 0;
  g.out = sw;
  MFE_CHECK(launch_signgen(g, st));
  SideDev R{}, C{};
  R.slice_off = p->rows.slice_off;
  R.slice_mat = p->rows.slice_mat;
  R.len = p->rows.len;
  R.orig = p->rows.orig;
  R.ent = p->rows.ent;
  R.nint = p->rows.nint;
  R.is_row = 1;
  C.slice_off = p->cols.slice_off;
  C.slice_mat = p->cols.slice_mat;
  C.len = p->cols.len;
  C.orig = p->cols.orig;
  C.ent = p->cols.ent;
  C.nint = p->cols.nint;
  C.is_row = 0;
  const int32_t* mat_of_row_slice = p->rows.slice_mat;
  const int32_t* mat_of_col_slice = p->cols.slice_mat;
  const unsigned gr = (unsigned)ceil_div(p->rows.nint, 256), gc = (unsigned)ceil_div(p->cols.nint, 256);
  // rows gather column-indexed sketch signs (side 2); columns gather row-indexed (side 3)
  if (ks == 4) {
    k_sketch<4><<<gr, 256, 0, st>>>(R, p->mats, sw, d_wb_col, mat_of_col_slice, p->cols.orig, est_r, rat_r);
    k_sketch<4><<<gc, 256, 0, st>>>(C, p->mats, sw, d_wb_row, mat_of_row_slice, p->rows.orig, est_c, rat_c);
  } else if (ks == 8) {
    k_sketch<8><<<gr, 256, 0, st>>>(R, p->mats, sw, d_wb_col, mat_of_col_slice, p->cols.orig, est_r, rat_r);
    k_sketch<8><<<gc, 256, 0, st>>>(C, p->mats, sw, d_wb_row, mat_of_row_slice, p->rows.orig, est_c, rat_c);
  } else {
    k_sketch<16><<<gr, 256, 0, st>>>(R, p->mats, sw, d_wb_col, mat_of_col_slice, p->cols.orig, est_r, rat_r);
    k_sketch<16><<<gc, 256, 0, st>>>(C, p->mats, sw, d_wb_row, mat_of_row_slice, p->rows.orig, est_c, rat_c);
  }
  k_side_partial<<<dim3((unsigned)count, kStatChunks), 256, 0, st>>>(est_r, d_rbase, part_r);
  k_side_partial<<<dim3((unsigned)count, kStatChunks), 256, 0, st>>>(est_c, d_cbase, part_c);
  k_side_final<<<(unsigned)ceil_div(count, 64), 64, 0, st>>>(part_r, count, st_r);
  k_side_final<<<(unsigned)ceil_div(count, 64), 64, 0, st>>>(part_c, count, st_c);
  k_features<<<(unsigned)ceil_div(p->M, 256), 256, 0, st>>>(est_r, rat_r, st_r, st_r, st_c, d_fm, count, 1, p->M,
                                                             gamma, M, feat_rows, u_sketch);
  k_features<<<(unsigned)ceil_div(p->N, 256), 256, 0, st>>>(est_c, rat_c, st_c, st_r, st_c, d_fm, count, 0, p->N,
                                                             gamma, M, feat_cols, v_sketch);
  MFE_HIP(hipGetLastError());
  return MFE_OK;
}

}  // namespace

// Plan-owned scratch of the warm-start calls, grown on demand.
int plan_workspace(mfe_plan* p, size_t bytes, char** out) {
  if (p->ws_bytes < bytes) {
    (void)hipFree(p->ws);
    p->ws = nullptr;
    p->ws_bytes = 0;
    hipError_t e = hipMalloc(&p->ws, bytes);
    if (e != hipSuccess)
      return set_error(e == hipErrorOutOfMemory ? MFE_ENOMEM : MFE_EDEVICE, "hipMalloc failed: %s",
                       hipGetErrorString(e));
    p->ws_bytes = bytes;
  }
  *out = (char*)p->ws;
  return MFE_OK;
}

int plan_sketch_features(mfe_plan* p, uint64_t seed, int32_t ks, const double* alpha_b, const double* beta_b,
                         double gamma, double M, float* feat_rows, float* feat_cols, double* u_sketch,
                         double* v_sketch, hipStream_t st) {
  if (ks != 4 && ks != 8 && ks != 16) return set_error(MFE_EINVAL, "sketch probes must be 4, 8 or 16");
  MFE_CHECK(ensure_mats(p, st));
  size_t bytes = 0;
  MFE_CHECK(sketch_impl(p, seed, ks, alpha_b, beta_b, gamma, M, nullptr, nullptr, nullptr, nullptr, st, nullptr,
                        &bytes));
  char* ws;
  MFE_CHECK(plan_workspace(p, bytes, &ws));
  MFE_CHECK(sketch_impl(p, seed, ks, alpha_b, beta_b, gamma, M, feat_rows, feat_cols, u_sketch, v_sketch, st, ws,
                        &bytes));
  MFE_HIP(hipStreamSynchronize(st));
  return MFE_OK;
}

int plan_warmstart(mfe_plan* p, const float* params, uint64_t seed, int32_t ks, const double* alpha_b,
                   const double* beta_b, double gamma, double M, int learned, double* u0, double* v0,
                   hipStream_t st) {
  if (ks != 4 && ks != 8 && ks != 16) return set_error(MFE_EINVAL, "sketch probes must be 4, 8 or 16");
  if (learned && !params) return set_error(MFE_EINVAL, "learned warm start needs the network parameters");
  MFE_CHECK(ensure_mats(p, st));
  // layout: features and sketch initialisations of rows and columns, network outputs,
  // then the sketch scratch
  Carver head{nullptr};
  head.take<float>(p->M * kF);
  head.take<float>(p->N * kF);
  head.take<double>(p->M);
  head.take<double>(p->N);
  head.take<float>(p->M);
  head.take<float>(p->N);
  const size_t head_bytes = (head.off + 255) & ~(size_t)255;
  size_t bytes = head_bytes;
  MFE_CHECK(sketch_impl(p, seed, ks, alpha_b, beta_b, gamma, M, nullptr, nullptr, nullptr, nullptr, st, nullptr,
                        &bytes));
  char* ws;
  MFE_CHECK(plan_workspace(p, bytes, &ws));
  Carver cv{ws};
  float* fr = cv.take<float>(p->M * kF);
  float* fc = cv.take<float>(p->N * kF);
  double* us = cv.take<double>(p->M);
  double* vs = cv.take<double>(p->N);
  float* du = cv.take<float>(p->M);
  float* dv = cv.take<float>(p->N);
  MFE_CHECK(sketch_impl(p, seed, ks, alpha_b, beta_b, gamma, M, fr, fc, us, vs, st, ws + head_bytes, &bytes));
  if (learned) {
    launch_mlp_infer(params, fr, p->M, du, st);
    launch_mlp_infer(params, fc, p->N, dv, st);
  }
  k_apply_delta<<<(unsigned)ceil_div(p->M, 256), 256, 0, st>>>(p->M, us, learned ? du : nullptr, M, u0);
  k_apply_delta<<<(unsigned)ceil_div(p->N, 256), 256, 0, st>>>(p->N, vs, learned ? dv : nullptr, M, v0);
  MFE_HIP(hipGetLastError());
  MFE_HIP(hipStreamSynchronize(st));
  return MFE_OK;
}


int plan_training_set(mfe_plan* p, uint64_t seed, int32_t ks, const double* alpha_b, const double* beta_b,
                      double gamma, double M, const double* u_label, const double* v_label, int64_t per_matrix,
                      uint64_t sample_seed, float* X, float* t, int64_t* idx, int64_t* count, hipStream_t st) {
  if (ks != 4 && ks != 8 && ks != 16) return set_error(MFE_EINVAL, "sketch probes must be 4, 8 or 16");
  const int nmat = p->count;
  // per-side sample offsets and index bases (rows: side 0, columns: side 1)
  std::vector<int64_t> tab(4 * ((size_t)nmat + 1));
  int64_t* soff_r = tab.data();
  int64_t* soff_c = soff_r + nmat + 1;
  int64_t* base_r = soff_c + nmat + 1;
  int64_t* base_c = base_r + nmat + 1;
  soff_r[0] = soff_c[0] = base_r[0] = base_c[0] = 0;
  for (int b = 0; b < nmat; ++b) {
    soff_r[b + 1] = soff_r[b] + std::min<int64_t>(per_matrix, p->meta[b].m);
    soff_c[b + 1] = soff_c[b] + std::min<int64_t>(per_matrix, p->meta[b].n);
    base_r[b + 1] = base_r[b] + p->meta[b].m;
    base_c[b + 1] = base_c[b] + p->meta[b].n;
  }
  *count = soff_r[nmat] + soff_c[nmat];
  if (!X) return MFE_OK;
  MFE_CHECK(ensure_mats(p, st));
  // scratch: the offset tables, features and sketch initialisations, then the sketch's own
  Carver head{nullptr};
  head.take<int64_t>((int64_t)tab.size());
  head.take<float>(p->M * kF);
  head.take<float>(p->N * kF);
  head.take<double>(p->M);
  head.take<double>(p->N);
  const size_t head_bytes = (head.off + 255) & ~(size_t)255;
  size_t bytes = head_bytes;
  MFE_CHECK(sketch_impl(p, seed, ks, alpha_b, beta_b, gamma, M, nullptr, nullptr, nullptr, nullptr, st, nullptr,
                        &bytes));
  char* ws;
  MFE_CHECK(plan_workspace(p, bytes, &ws));
  Carver cv{ws};
  int64_t* d_tab = cv.take<int64_t>((int64_t)tab.size());
  float* fr = cv.take<float>(p->M * kF);
  float* fc = cv.take<float>(p->N * kF);
  double* us = cv.take<double>(p->M);
  double* vs = cv.take<double>(p->N);
  // ordered on st after earlier users of the scratch; waited for, so that `tab` may go
  MFE_HIP(hipMemcpyAsync(d_tab, tab.data(), sizeof(int64_t) * tab.size(), hipMemcpyHostToDevice, st));
  MFE_HIP(hipStreamSynchronize(st));
  MFE_CHECK(sketch_impl(p, seed, ks, alpha_b, beta_b, gamma, M, fr, fc, us, vs, st, ws + head_bytes, &bytes));
  const int64_t nr = soff_r[nmat], nc = soff_c[nmat];
  const int64_t* d_soff_r = d_tab;
  const int64_t* d_soff_c = d_soff_r + nmat + 1;
  const int64_t* d_base_r = d_soff_c + nmat + 1;
  const int64_t* d_base_c = d_base_r + nmat + 1;
  if (nr > 0)
    k_training_samples<<<(unsigned)ceil_div(nr, 256), 256, 0, st>>>(d_soff_r, d_base_r, nmat, 0, sample_seed, fr,
                                                                    u_label, us, 0, X, t, idx);
  if (nc > 0)
    k_training_samples<<<(unsigned)ceil_div(nc, 256), 256, 0, st>>>(d_soff_c, d_base_c, nmat, 1, sample_seed, fc,
                                                                    v_label, vs, nr, X, t, idx);
  MFE_HIP(hipGetLastError());
  MFE_HIP(hipStreamSynchronize(st));
  return MFE_OK;
}

int mlp_forward(const float* params, const float* X, int64_t count, float* y, hipStream_t st) {
  if (count <= 0) return MFE_OK;
  launch_mlp_infer(params, X, count, y, st);
  MFE_HIP(hipGetLastError());
  MFE_HIP(hipStreamSynchronize(st));
  return MFE_OK;
}

int mlp_train(float* params, float* adam_m, float* adam_v, int32_t step0, const float* X, const float* t,
              int64_t total, int64_t batch, int32_t iters, float lr, uint64_t seed, double* loss_trace,
              hipStream_t st) {
  Work W;
  int64_t* idx;
  float *y, *gy, *h1, *h2, *g1, *g2, *grad;
  double *se, *loss;
  MFE_CHECK(W.alloc(&idx, batch));
  MFE_CHECK(W.alloc(&y, batch));
  MFE_CHECK(W.alloc(&gy, batch));
  MFE_CHECK(W.alloc(&h1, batch * kH));
  MFE_CHECK(W.alloc(&h2, batch * kH));
  MFE_CHECK(W.alloc(&g1, batch * kH));
  MFE_CHECK(W.alloc(&g2, batch * kH));
  MFE_CHECK(W.alloc(&grad, kP));
  MFE_CHECK(W.alloc(&se, batch));
  MFE_CHECK(W.alloc(&loss, std::max(iters, 1)));
  double* part;
  MFE_CHECK(W.alloc(&part, wgrad_chunks(batch) * kP));
  const unsigned gb = (unsigned)ceil_div(batch, 256), gp = (unsigned)ceil_div(kP, 256);
  const unsigned gt = (unsigned)train_grid(batch);
  for (int it = 0; it < iters; ++it) {
    const uint64_t step = (uint64_t)step0 + it + 1;
    k_batch_indices<<<gb, 256, 0, st>>>(seed, step, batch, total, idx);
    k_mlp_fwd<<<gt, 256, 0, st>>>(params, X, idx, batch, y, h1, h2);
    k_mlp_bwd<<<gt, 256, 0, st>>>(params, y, t, idx, batch, h1, h2, gy, g1, g2, se);
    launch_wgrad(X, idx, batch, gy, h1, h2, g1, g2, part, grad, st);
    k_sum<<<1, 256, 0, st>>>(se, batch, 1.0 / (double)batch, loss + it);
    k_adam<<<gp, 256, 0, st>>>(params, grad, adam_m, adam_v, (int)step, lr);
  }
  MFE_HIP(hipGetLastError());
  if (loss_trace && iters > 0)
    MFE_HIP(hipMemcpyAsync(loss_trace, loss, sizeof(double) * iters, hipMemcpyDeviceToHost, st));
  MFE_HIP(hipStreamSynchronize(st));
  return MFE_OK;
}

int mlp_grad(const float* params, const float* X, const float* t, int64_t count, float* grad, double* loss,
             hipStream_t st) {
  Work W;
  float *y, *gy, *h1, *h2, *g1, *g2;
  double *se, *l;
  MFE_CHECK(W.alloc(&y, count));
  MFE_CHECK(W.alloc(&gy, count));
  MFE_CHECK(W.alloc(&h1, count * kH));
  MFE_CHECK(W.alloc(&h2, count * kH));
  MFE_CHECK(W.alloc(&g1, count * kH));
  MFE_CHECK(W.alloc(&g2, count * kH));
  MFE_CHECK(W.alloc(&se, count));
  MFE_CHECK(W.alloc(&l, 1));
  double* part;
  MFE_CHECK(W.alloc(&part, wgrad_chunks(count) * kP));
  const unsigned gt = (unsigned)train_grid(count);
  k_mlp_fwd<<<gt, 256, 0, st>>>(params, X, nullptr, count, y, h1, h2);
  k_mlp_bwd<<<gt, 256, 0, st>>>(params, y, t, nullptr, count, h1, h2, gy, g1, g2, se);
  launch_wgrad(X, nullptr, count, gy, h1, h2, g1, g2, part, grad, st);
  k_sum<<<1, 256, 0, st>>>(se, count, 1.0 / (double)count, l);
  MFE_HIP(hipGetLastError());
  if (loss) MFE_HIP(hipMemcpyAsync(loss, l, sizeof(double), hipMemcpyDeviceToHost, st));
  MFE_HIP(hipStreamSynchronize(st));
  return MFE_OK;
}

int warmstart_apply(int64_t n, const double* sketch, const float* delta, double M, double* out, hipStream_t st) {
  if (n <= 0) return MFE_OK;
  k_apply_delta<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(n, sketch, delta, M, out);
  MFE_HIP(hipGetLastError());
  MFE_HIP(hipStreamSynchronize(st));
  return MFE_OK;
}

int mlp_param_count() { return kP; }
int mlp_feature_count() { return kF; }

}  // namespace mfe
