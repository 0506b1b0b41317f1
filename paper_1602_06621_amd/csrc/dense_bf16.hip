// Algorithm 1 (Section 3.2) for dense bfloat16 A on the matrix cores (MFMA).
//
// Per step the two products are GEMMs against the probe block: Y = A (E S) (m x k) and
// X = A' (D W) (n x k), k <= 64.  Probe operands are exact signs times bf16(e^x);
// products accumulate in FP32 on v_mfma_f32_32x32x16_bf16; the square / step /
// project / average epilogue runs in FP64 inside the same kernel.
//
// Layout.  The library keeps two copies of A in an MFMA-native tiled layout: tile
// (row block rb of 32 rows, k chunk kc of 16 columns) is 1 KiB, lane l holding the 8
// values A[32 rb + l%32][16 kc + 8 (l/32) + j], j < 8, in 16 consecutive bytes, so a
// wavefront reads each tile with one fully coalesced 16-byte load per lane.  The second
// copy is A' in the same layout, which turns the transposed product into the same
// kernel.  Probe blocks use the matching operand layout (per k chunk, lane l holds probe
// 32 nb + l%32 at the same 8 k values).  Both are padded with zeros to whole tiles.
//
// Work split: a workgroup of 4 wavefronts covers 4 consecutive 32-row blocks over one k
// range (the k chunks are split into `splits` ranges so that a pass launches ~512
// workgroups).  The four wavefronts walk the same chunks, so each probe tile is fetched
// from L2 once per workgroup and read by the other wavefronts from L1 (probe loads were
// two thirds of the L2 requests when every wavefront walked its own chunks; the pass is
// bound by L2 requests in flight per CU).  Each wavefront stores its 32 x 32 NB FP32
// accumulator as the partial of its block and range; a second launch adds the ranges in
// FP64 and runs the square / step / project / average update.
#include <cmath>
#include <vector>

#include "dense.h"
#include "sparse.h"

namespace mfe {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kRows = 32;   // rows per tile / workgroup
constexpr int kChunk = 16;  // k per MFMA
constexpr int kWaves = 4;

// FP64 -> bfloat16 bits, round to nearest even, for finite normal values in range.
__device__ inline uint16_t bf16_rne(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  const uint64_t sign = u >> 63;
  int64_t ex = (int64_t)((u >> 52) & 0x7FF) - 1023;
  uint64_t mant = u & ((1ull << 52) - 1ull);
  // keep 7 fraction bits: round the 45 dropped bits to nearest even
  uint64_t keep = mant >> 45;
  const uint64_t rest = mant & ((1ull << 45) - 1ull);
  const uint64_t half = 1ull << 44;
  if (rest > half || (rest == half && (keep & 1ull))) {
    keep += 1;
    if (keep == 128) {
      keep = 0;
      ex += 1;
    }
  }
  const uint32_t e8 = (uint32_t)(ex + 127);
  return (uint16_t)((sign << 15) | (e8 << 7) | keep);
}

// Tiles of A (trans = 0) or A' (trans = 1) from the row-major input (bf16 bits).
// R x C is the tiled matrix (R = m, C = n for A; R = n, C = m for A').
__global__ void k_tile(const uint16_t* __restrict__ A, int64_t m, int64_t n, int64_t ld, int trans, int64_t RB,
                       int64_t KC, u32x4* __restrict__ tiles) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (rb, kc, lane)
  if (gid >= RB * KC * 64) return;
  const int lane = (int)(gid & 63);
  const int64_t t = gid >> 6;
  const int64_t rb = t / KC, kc = t % KC;
  const int64_t r = rb * kRows + (lane & 31);
  const int64_t c0 = kc * kChunk + (lane >> 5) * 8;
  uint16_t v[8];
  for (int j = 0; j < 8; ++j) {
    const int64_t c = c0 + j;
    uint16_t x = 0;
    if (!trans) {
      if (r < m && c < n) x = A[r * ld + c];
    } else {
      if (r < n && c < m) x = A[c * ld + r];
    }
    v[j] = x;
  }
  u32x4 w;
  w.x = v[0] | ((uint32_t)v[1] << 16);
  w.y = v[2] | ((uint32_t)v[3] << 16);
  w.z = v[4] | ((uint32_t)v[5] << 16);
  w.w = v[6] | ((uint32_t)v[7] << 16);
  tiles[gid] = w;
}

// Probe operand tiles: per k chunk kc and probe block nb (32 probes), lane l holds
// probe p = 32 nb + l%32 at k = 16 kc + 8 (l/32) + j:  +-bf16(scale[k]), sign bit k*K + p.
__global__ void k_probe_tiles(const double* __restrict__ scale, const uint64_t* __restrict__ sw, int64_t C, int K,
                              int64_t KC, int NB, u32x4* __restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (kc, nb, lane)
  if (gid >= KC * NB * 64) return;
  const int lane = (int)(gid & 63);
  const int64_t t = gid >> 6;
  const int nb = (int)(t % NB);
  const int64_t kc = t / NB;
  const int p = nb * 32 + (lane & 31);
  const int64_t k0 = kc * kChunk + (lane >> 5) * 8;
  uint16_t v[8];
  for (int j = 0; j < 8; ++j) {
    const int64_t kk = k0 + j;
    uint16_t x = 0;
    if (kk < C && p < K) {
      x = bf16_rne(scale[kk]);
      const uint64_t g = (uint64_t)kk * (uint64_t)K + (uint64_t)p;
      if ((sw[g >> 6] >> (g & 63)) & 1ull) x ^= 0x8000;
    }
    v[j] = x;
  }
  u32x4 w;
  w.x = v[0] | ((uint32_t)v[1] << 16);
  w.y = v[2] | ((uint32_t)v[3] << 16);
  w.z = v[4] | ((uint32_t)v[5] << 16);
  w.w = v[6] | ((uint32_t)v[7] << 16);
  out[gid] = w;
}

struct Bf16Side {
  const u32x4* tiles;   // [RB][KC][64]
  const u32x4* probes;  // [KC][NB][64]
  int64_t R, RB, KC;
  int splits;           // k ranges per row block
  float* part;          // [splits][RB * 32][32 NB] partial products
  double* x;
  double* xbar;
  double* scale_out;
  double target;
};

__device__ inline bf16x8 as_bf16x8(u32x4 v) {
  bf16x8 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}

// Wavefront w of workgroup (g, split): row block 4 g + w, chunks of range `split`;
// partial Y (32 x 32 NB) = tiles . probes.
template <int NB>
struct ChunkGroup {
  static constexpr int F = 4;  // chunks per group; two groups are in flight
  u32x4 a[F];
  u32x4 p[F][NB];
  __device__ __forceinline__ void load(const u32x4* __restrict__ at, const u32x4* __restrict__ pt, int64_t kc) {
#pragma unroll
    for (int u = 0; u < F; ++u) {
      a[u] = __builtin_nontemporal_load(at + (kc + u) * 64);
#pragma unroll
      for (int b = 0; b < NB; ++b) p[u][b] = pt[((kc + u) * NB + b) * 64];
    }
  }
  __device__ __forceinline__ void mma(f32x16 (&acc)[NB]) const {
#pragma unroll
    for (int u = 0; u < F; ++u)
#pragma unroll
      for (int b = 0; b < NB; ++b)
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(a[u]), as_bf16x8(p[u][b]), acc[b], 0, 0, 0);
  }
};

template <int NB>
__global__ __launch_bounds__(256) void k_bf16_pass(Bf16Side S) {
  constexpr int F = ChunkGroup<NB>::F;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t rb = (int64_t)blockIdx.x * kWaves + wave;
  if (rb >= S.RB) return;
  const int split = blockIdx.y;
  const int64_t per = (S.KC + S.splits - 1) / S.splits;
  const int64_t kbeg = (int64_t)split * per, kend = kbeg + per < S.KC ? kbeg + per : S.KC;
  f32x16 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[b][v] = 0.f;
  const u32x4* __restrict__ at = S.tiles + rb * S.KC * 64 + lane;
  const u32x4* __restrict__ pt = S.probes + lane;
  // double-buffered groups: the loads of group g + 1 are issued before the products of g
  const int64_t ngroups = (kend - kbeg) / F;
  ChunkGroup<NB> g0, g1;
  int64_t kc = kbeg;
  if (ngroups > 0) g0.load(at, pt, kc);
  for (int64_t g = 0; g < ngroups; g += 2) {
    if (g + 1 < ngroups) g1.load(at, pt, kc + F);
    g0.mma(acc);
    if (g + 1 >= ngroups) {
      kc += F;
      break;
    }
    if (g + 2 < ngroups) g0.load(at, pt, kc + 2 * F);
    g1.mma(acc);
    kc += 2 * F;
  }
  for (; kc < kend; ++kc) {
    const u32x4 a = __builtin_nontemporal_load(at + kc * 64);
#pragma unroll
    for (int b = 0; b < NB; ++b)
      acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(a), as_bf16x8(pt[(kc * NB + b) * 64]), acc[b], 0,
                                                       0, 0);
  }
  // accumulator layout: lane l, register v -> row 8 (v/4) + 4 (l/32) + v%4, column l%32
  float* __restrict__ out = S.part + ((int64_t)split * S.RB + rb) * kRows * 32 * NB;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 16; ++v)
      out[((v >> 2) * 8 + (lane >> 5) * 4 + (v & 3)) * 32 * NB + b * 32 + (lane & 31)] = acc[b][v];
}

// Update of every index from the FP32 partials: one wavefront per row, lane p adds the
// ranges of probe p in FP64 (coalesced over the probes), the squares are summed across
// the wavefront, and lane 0 updates the iterate.
template <int NB>
__global__ __launch_bounds__(256) void k_bf16_update(Bf16Side S, int k, StepScalars sc, int* flag) {
  const int lane = threadIdx.x & 63;
  const int64_t r = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  if (r >= S.R) return;  // whole wavefronts leave together
  const int64_t stride = S.RB * kRows * 32 * NB;
  double y = 0.0;
  if (lane < 32 * NB && lane < k) {
    const float* __restrict__ base = S.part + r * 32 * NB + lane;
    for (int sp = 0; sp < S.splits; ++sp) y += (double)base[sp * stride];
  }
  const double ss = wave_sum(y * y);
  if (lane == 0) {
    double x = S.x[r], xb = S.xbar[r];
    if (!sgd_update(ss, k, S.target, sc, x, xb)) atomicOr(flag, 1);
    S.x[r] = x;
    S.xbar[r] = xb;
    S.scale_out[r] = exp(x);
  }
}

__global__ void k_bf_init(int64_t cnt, const double* __restrict__ x0, double M, double* __restrict__ x,
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

__global__ void k_bf_output(int64_t cnt, const double* __restrict__ xbar, double* __restrict__ dout,
                            double* __restrict__ xbar_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  dout[i] = exp(xbar[i]);
  if (xbar_out) xbar_out[i] = xbar[i];
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

template <int NB>
void launch_pass(const Bf16Side& S, int k, const StepScalars& sc, int* flag, hipStream_t st) {
  k_bf16_pass<NB><<<dim3((unsigned)ceil_div(S.RB, kWaves), (unsigned)S.splits), dim3(256), 0, st>>>(S);
  k_bf16_update<NB><<<dim3((unsigned)ceil_div(S.R * 64, 256)), dim3(256), 0, st>>>(S, k, sc, flag);
}

// k ranges per row block: about 512 workgroups (of 4 row blocks) per pass, at least 32
// chunks per range.
int bf16_splits(int64_t RB, int64_t KC) {
  int64_t s = 1;
  while (ceil_div(RB, kWaves) * s < 512 && KC / (2 * s) >= 32) s *= 2;
  return (int)s;
}

}  // namespace

int dense_bf16_equilibrate(const mfe_matrix* A, const mfe_equil_params* p, double* d, double* e, double* u_bar,
                           double* v_bar) {
  if (!A->data) return set_error(MFE_EINVAL, "dense data is NULL");
  if (A->ld < A->n) return set_error(MFE_EDIM, "ld < n");
  if (p->probes > 64) return set_error(MFE_EUNSUPPORTED, "BF16 path supports at most 64 probes per step");
  if (p->box_M > 80.0) return set_error(MFE_EUNSUPPORTED, "BF16 path needs M <= 80 (e^x inside the bf16 range)");
  hipStream_t st = (hipStream_t)p->stream;
  const int64_t m = A->m, n = A->n;
  const int k = p->probes;
  const int NB = k <= 32 ? 1 : 2;
  const int64_t RBu = ceil_div(m, kRows), KCu = ceil_div(n, kChunk);  // tiles of A
  const int64_t RBv = ceil_div(n, kRows), KCv = ceil_div(m, kChunk);  // tiles of A'
  Bufs B;
  u32x4 *tu, *tv, *pu, *pv;
  double *u, *ub, *v, *vb, *su[2], *sv[2];
  int* flag;
  MFE_CHECK(B.alloc(&tu, RBu * KCu * 64));
  MFE_CHECK(B.alloc(&tv, RBv * KCv * 64));
  MFE_CHECK(B.alloc(&pu, KCu * NB * 64));  // probes for the row pass: columns, side 0
  MFE_CHECK(B.alloc(&pv, KCv * NB * 64));  // probes for the column pass: rows, side 1
  MFE_CHECK(B.alloc(&u, m));
  MFE_CHECK(B.alloc(&ub, m));
  MFE_CHECK(B.alloc(&v, n));
  MFE_CHECK(B.alloc(&vb, n));
  for (int i = 0; i < 2; ++i) {
    MFE_CHECK(B.alloc(&su[i], m));
    MFE_CHECK(B.alloc(&sv[i], n));
  }
  MFE_CHECK(B.alloc(&flag, 1));
  const int Su = bf16_splits(RBu, KCu), Sv = bf16_splits(RBv, KCv);
  float *partu, *partv;
  MFE_CHECK(B.alloc(&partu, (int64_t)Su * RBu * kRows * 32 * NB));
  MFE_CHECK(B.alloc(&partv, (int64_t)Sv * RBv * kRows * 32 * NB));
  // sign words: side 0 (n * k bits) then side 1 (m * k bits), one slot refilled per step
  SignSeg segs_h[2];
  segs_h[0].ctrl_lo = ((uint64_t)p->batch << 34) | 0ull;
  segs_h[0].nblocks = ceil_div(n * k, 256);
  segs_h[0].word_off = 0;
  segs_h[1].ctrl_lo = ((uint64_t)p->batch << 34) | 1ull;
  segs_h[1].nblocks = ceil_div(m * k, 256);
  segs_h[1].word_off = 4 * segs_h[0].nblocks + 4;
  const int64_t words = segs_h[1].word_off + 4 * segs_h[1].nblocks + 4;
  const int64_t pre[3] = {0, segs_h[0].nblocks, segs_h[0].nblocks + segs_h[1].nblocks};
  SignSeg* segs;
  int64_t* prefix;
  uint64_t* sw;
  MFE_CHECK(B.alloc(&segs, 2));
  MFE_CHECK(B.alloc(&prefix, 3));
  MFE_CHECK(B.alloc(&sw, words));
  MFE_HIP(hipMemcpyAsync(segs, segs_h, sizeof segs_h, hipMemcpyHostToDevice, st));
  MFE_HIP(hipMemcpyAsync(prefix, pre, sizeof pre, hipMemcpyHostToDevice, st));
  MFE_HIP(hipMemsetAsync(sw, 0, sizeof(uint64_t) * words, st));
  MFE_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));

  const uint16_t* Ad = (const uint16_t*)A->data;
  k_tile<<<dim3((unsigned)ceil_div(RBu * KCu * 64, 256)), dim3(256), 0, st>>>(Ad, m, n, A->ld, 0, RBu, KCu, tu);
  k_tile<<<dim3((unsigned)ceil_div(RBv * KCv * 64, 256)), dim3(256), 0, st>>>(Ad, m, n, A->ld, 1, RBv, KCv, tv);
  k_bf_init<<<dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st>>>(m, p->u0, p->box_M, u, ub, su[0], flag);
  k_bf_init<<<dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st>>>(n, p->v0, p->box_M, v, vb, sv[0], flag);
  MFE_HIP(hipGetLastError());

  hipEvent_t e0, e1;
  MFE_HIP(hipEventCreate(&e0));
  MFE_HIP(hipEventCreate(&e1));
  MFE_HIP(hipEventRecord(e0, st));
  for (int t = 1; t <= p->steps; ++t) {
    SignGenDev g;
    g.segs = segs;
    g.seg_prefix = prefix;
    g.nseg = 2;
    g.nblocks = pre[2];
    g.seed = p->seed;
    g.step = (uint64_t)t;
    g.out = sw;
    MFE_CHECK(launch_signgen(g, st));
    const int cur = t & 1, prev = cur ^ 1;
    // probe operands from the scales of step t-1 (Jacobi order)
    k_probe_tiles<<<dim3((unsigned)ceil_div(KCu * NB * 64, 256)), dim3(256), 0, st>>>(sv[prev], sw, n, k, KCu, NB, pu);
    k_probe_tiles<<<dim3((unsigned)ceil_div(KCv * NB * 64, 256)), dim3(256), 0, st>>>(
        su[prev], sw + segs_h[1].word_off, m, k, KCv, NB, pv);
    StepScalars sc;
    sc.tau = (double)t + (double)p->t0;
    sc.eta = 2.0 / (p->gamma * (sc.tau + 1.0));
    sc.gamma = p->gamma;
    sc.M = p->box_M;
    Bf16Side R{tu, pu, m, RBu, KCu, Su, partu, u, ub, su[cur], p->alpha * p->alpha};
    Bf16Side Cc{tv, pv, n, RBv, KCv, Sv, partv, v, vb, sv[cur], p->beta * p->beta};
    if (NB == 1) {
      launch_pass<1>(R, k, sc, flag, st);
      launch_pass<1>(Cc, k, sc, flag, st);
    } else {
      launch_pass<2>(R, k, sc, flag, st);
      launch_pass<2>(Cc, k, sc, flag, st);
    }
  }
  MFE_HIP(hipGetLastError());
  MFE_HIP(hipEventRecord(e1, st));
  k_bf_output<<<dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st>>>(m, ub, d, u_bar);
  k_bf_output<<<dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st>>>(n, vb, e, v_bar);
  MFE_HIP(hipGetLastError());
  int h = 0;
  MFE_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  MFE_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  MFE_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  record_timing(ms, p->steps > 0 ? ms / p->steps : 0.0);
  if (h & 2) return set_error(MFE_EINVAL, "warm start u0/v0 outside the box [-M, M] (or NaN)");
  if (h & 1) return set_error(MFE_ENONFINITE, "non-finite gradient estimate or iterate (NaN/Inf in A?)");
  return MFE_OK;
}

}  // namespace mfe
