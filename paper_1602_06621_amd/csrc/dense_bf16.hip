// Algorithm 1 (Section 3.2) for dense bfloat16 A on the matrix cores (MFMA).
//
// Per step the two products are GEMMs against the probe block: Y = A (E S) (m x k) and
// X = A' (D W) (n x k), k <= 64.  The scale e^x of a probe operand is carried as two
// bf16 numbers, hi = bf16(e^x) and lo = bf16(e^x - hi) (relative error of hi + lo at most
// about 2^-17 instead of bf16's 2^-9), each times the exact sign: two MFMA products per
// tile, accumulated together in FP32 on v_mfma_f32_32x32x16_bf16.  The square / step /
// project / average update runs in FP64.
//
// Layout.  The library keeps two copies of A in an MFMA-native tiled layout: tile
// (row block rb of 32 rows, k chunk kc of 16 columns) is 1 KiB, lane l holding the 8
// values A[32 rb + l%32][16 kc + 8 (l/32) + j], j < 8, in 16 consecutive bytes, so a
// wavefront reads each tile with one fully coalesced 16-byte load per lane.  The second
// copy is A' in the same layout, which turns the transposed product into the same
// kernel.  Tiles are padded with zeros.  The probe operands of a chunk have the matching
// layout (lane l holds probe 32 nb + l%32 at the same 8 k values), but are not stored as
// tiles: per k chunk the pass loads the 16 hi and 16 lo bf16 scales and one sign byte per
// (probe, half chunk), 64 + 64 NB bytes, and assembles the two MFMA operands in registers
// (sign bit XORed into each scale).  A step is two launches:
// both passes (rows over A, then columns over A'), and the update of both sides, which
// also writes the bf16 scales and (extra workgroups) the Philox sign bytes of the next
// step.  A separate probe build makes the operands of the first step.
//
// Work split: a workgroup of 4 wavefronts covers 4 RW consecutive 32-row blocks over one
// k range (the k chunks are split into `splits` ranges so that a pass launches about
// MFE_BF16_WG workgroups).  Each wavefront keeps two groups of F chunks in flight and
// stores its 32 RW x 32 NB FP32 accumulator as the partial of its blocks and range; the
// update adds the ranges in FP64 and runs the square / step / project / average update.
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
#ifndef MFE_BF16_WAVES
#define MFE_BF16_WAVES 4
#endif
constexpr int kWaves = MFE_BF16_WAVES;

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

// The low part of a two-term bf16 scale: bf16(x - hi), where hi = bf16_rne(x).  Values
// below the smallest normal bf16 (2^-126) are flushed to zero; for the scales here
// (x >= e^-80) that happens only when x - hi is below 2^-126, i.e. the two terms are
// then exact to at least 2^-11 relative (2^-17 or better for x >= 2^-108).
__device__ inline uint16_t bf16_lo(double x, uint16_t hi) {
  const double h = (double)__uint_as_float((uint32_t)hi << 16);
  const double r = x - h;  // exact in FP64: h has 8 significant bits and |r| <= ulp(h) / 2
  if (!(fabs(r) >= 0x1p-126)) return (uint16_t)0;
  return bf16_rne(r);
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

// Probe operands, kept compressed in memory and expanded into MFMA operands in
// registers by the pass: per k chunk kc, the two-term bf16 scales of its 16 indices
// (scl[16 kc + i] = hi, slo[16 kc + i] = lo; zero past the end) and one sign byte per
// (half h, probe p):
// sgn[((2 kc + h) 32 + p % 32) NB + p / 32] holds in bit j the sign of probe p at
// index 16 kc + 8 h + j, which is bit k*K + p of the side's Philox stream (the layout
// of the library's sign words); zero for p >= K or past the end.  Per chunk that is
// 64 + 64 NB bytes instead of two 1 KiB operand tiles per 32 probes.
struct ProbeSide {
  const double* scale;  // e^x of the indices of this side (first step), or null: sign bytes only
  int64_t C, KC;        // indices, k chunks
  uint64_t ctrl;        // Philox key word: (batch << 34) | (t << 2) | side
  uint16_t* scl;        // [KC * 16] hi parts
  uint16_t* slo;        // [KC * 16] lo parts
  uint8_t* sgn;         // [KC][2][32][NB]
  int64_t groups;       // workgroups of kProbeChunks chunks
};

constexpr int kProbeChunks = 4;                                       // k chunks per workgroup
constexpr int kProbeBlocks = kProbeChunks * kChunk * 64 / 256 + 2;  // Philox blocks per workgroup (K <= 64)

// One workgroup of the probe build: draws the Philox blocks that hold the sign bits of
// its 64 indices into LDS, then writes its chunks' sign bytes and, when P.scale is set,
// their bf16 scales.  Called by every thread of the workgroup.
__device__ __forceinline__ void probe_group(const ProbeSide& P, int64_t grp, int K, int NB, uint64_t seed,
                                            uint64_t* words) {
  const int64_t kk0 = grp * kProbeChunks * kChunk;
  const int64_t kk1 = kk0 + kProbeChunks * kChunk < P.C ? kk0 + kProbeChunks * kChunk : P.C;
  const int64_t c0 = (kk0 * K) >> 8;  // first Philox block
  const int64_t nblk = kk1 > kk0 ? (((kk1 * K + 255) >> 8) - c0) : 0;
  for (int64_t i = threadIdx.x; i < nblk; i += 256) {
    const U64x4 w = philox4x64_10((uint64_t)(c0 + i) + 1, 0, 0, 0, seed, P.ctrl);
#pragma unroll
    for (int q = 0; q < 4; ++q) words[4 * i + q] = w.x[q];
  }
  if (P.scale && threadIdx.x < kProbeChunks * kChunk) {
    const int64_t kk = kk0 + threadIdx.x;
    if (kk < P.KC * kChunk) {
      const uint16_t hi = kk < P.C ? bf16_rne(P.scale[kk]) : (uint16_t)0;
      P.scl[kk] = hi;
      P.slo[kk] = kk < P.C ? bf16_lo(P.scale[kk], hi) : (uint16_t)0;
    }
  }
  __syncthreads();
  const int nout = kProbeChunks * 64 * NB;
  for (int o = threadIdx.x; o < nout; o += 256) {
    const int nb = o % NB;
    const int hq = (o / NB) & 63;  // 32 h + p % 32
    const int64_t kc = grp * kProbeChunks + o / (64 * NB);
    if (kc >= P.KC) continue;
    const int p = nb * 32 + (hq & 31);
    const int64_t k0 = kc * kChunk + (hq >> 5) * 8;
    uint32_t byte = 0;
    if (p < K) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t kk = k0 + j;
        if (kk < P.C) {
          const int64_t g = kk * K + p - c0 * 256;
          byte |= (uint32_t)((words[g >> 6] >> (g & 63)) & 1ull) << j;
        }
      }
    }
    P.sgn[kc * 64 * NB + o % (64 * NB)] = (uint8_t)byte;
  }
}

// Probe operands of the first step for both sides (scales from the initial iterates).
__global__ __launch_bounds__(256) void k_probe_build(ProbeSide P0, ProbeSide P1, int K, int NB, uint64_t seed) {
  __shared__ uint64_t words[4 * kProbeBlocks];
  const bool first = blockIdx.x < P0.groups;
  probe_group(first ? P0 : P1, first ? blockIdx.x : blockIdx.x - P0.groups, K, NB, seed, words);
}

struct Bf16Side {
  const u32x4* tiles;   // [RB][KC][64]
  const uint16_t* scl;  // probe operands, compressed (see ProbeSide): hi, lo, signs
  const uint16_t* slo;
  const uint8_t* sgn;
  int64_t R, RB, KC;
  int splits;           // k ranges per row block
  int64_t groups;       // workgroups per k range (kWaves * RW row blocks each)
  float* part;          // [splits][RB * 32][32 NB] partial products
  double* x;
  double* xbar;
  uint16_t* scl_out;    // hi and lo of e^x of this side: the other pass's probe scales next step
  uint16_t* slo_out;
  double target;
};

__device__ inline bf16x8 as_bf16x8(u32x4 v) {
  bf16x8 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}

// Sign masks of the probe operands: entry y (a sign byte) holds, for each index j < 8 of
// the byte, bit 15 of slot j set when bit j of y is set (slots 2i and 2i+1 share 32-bit
// word i).  XORed into the 16 bytes of 8 bf16 scales it gives the signed operand.  Kept in
// LDS (4 KiB per workgroup) so that a chunk's operands cost one LDS read and eight XORs per
// probe block instead of the bit shuffling.
__device__ inline u32x4 sign_mask(uint32_t y) {
  u32x4 m;
  m.x = ((y & 1u) << 15) | (((y >> 1) & 1u) << 31);
  m.y = (((y >> 2) & 1u) << 15) | (((y >> 3) & 1u) << 31);
  m.z = (((y >> 4) & 1u) << 15) | (((y >> 5) & 1u) << 31);
  m.w = (((y >> 6) & 1u) << 15) | (((y >> 7) & 1u) << 31);
  return m;
}

// Probe operands of one chunk for lane l from its 8 hi and 8 lo scales (16 bytes each) and
// its sign bytes (byte b: probe block b).
template <int NB>
__device__ __forceinline__ void expand_probes(const u32x4& sc, const u32x4& sl, uint32_t sg,
                                              const u32x4* __restrict__ masks, u32x4 (&oh)[NB], u32x4 (&ol)[NB]) {
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const u32x4 mk = masks[(sg >> (8 * b)) & 0xFFu];
    oh[b] = sc ^ mk;
    ol[b] = sl ^ mk;
  }
}

// Wavefront w of workgroup (g, split): row blocks RW (4 g + w) .. + RW - 1, chunks of
// range `split`; partial Y (32 RW x 32 NB) = tiles . probes.  The probe operands of a
// chunk are expanded once per wavefront and used for all RW row blocks.
template <int NB, int RW, int F>
struct ChunkGroup {
  u32x4 a[F][RW];
  u32x4 sc[F];    // hi bf16 scales of the lane's 8 indices
  u32x4 sl[F];    // lo bf16 scales
  uint32_t sg[F]; // sign bytes of the lane's NB probes
  // ps, pl: hi and lo scales as 16-byte groups, offset by the lane's half; pg: sign bytes
  // (NB per lane), offset by the lane
  __device__ __forceinline__ void load(const u32x4* const (&at)[RW], const u32x4* __restrict__ ps,
                                       const u32x4* __restrict__ pl, const uint8_t* __restrict__ pg, int64_t kc) {
#pragma unroll
    for (int u = 0; u < F; ++u) {
#pragma unroll
      for (int r = 0; r < RW; ++r) a[u][r] = __builtin_nontemporal_load(at[r] + (kc + u) * 64);
      sc[u] = ps[(kc + u) * 2];
      sl[u] = pl[(kc + u) * 2];
      if (NB == 2) sg[u] = *(const uint16_t*)(pg + (kc + u) * 128);
      else sg[u] = pg[(kc + u) * 64];
    }
  }
  // per chunk: the hi product, then the lo product, into the same FP32 accumulator
  __device__ __forceinline__ void mma(f32x16 (&acc)[RW][NB], const u32x4* __restrict__ masks) const {
#pragma unroll
    for (int u = 0; u < F; ++u) {
      u32x4 oh[NB], ol[NB];
      expand_probes<NB>(sc[u], sl[u], sg[u], masks, oh, ol);
#pragma unroll
      for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          acc[r][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(a[u][r]), as_bf16x8(oh[b]), acc[r][b], 0, 0,
                                                              0);
          acc[r][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(a[u][r]), as_bf16x8(ol[b]), acc[r][b], 0, 0,
                                                              0);
        }
    }
  }
};

template <int NB, int RW, int F>
__device__ __forceinline__ void bf16_pass(const Bf16Side& S, int64_t grp, int split, const u32x4* __restrict__ masks) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t rb0 = (grp * kWaves + wave) * RW;
  if (rb0 >= S.RB) return;
  const int64_t per = (S.KC + S.splits - 1) / S.splits;
  const int64_t kbeg = (int64_t)split * per, kend = kbeg + per < S.KC ? kbeg + per : S.KC;
  f32x16 acc[RW][NB];
#pragma unroll
  for (int r = 0; r < RW; ++r)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[r][b][v] = 0.f;
  // row blocks past the end re-read the last one; their results are not stored
  const u32x4* at[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) at[r] = S.tiles + (rb0 + r < S.RB ? rb0 + r : S.RB - 1) * S.KC * 64 + lane;
  const u32x4* __restrict__ ps = (const u32x4*)S.scl + (lane >> 5);
  const u32x4* __restrict__ pl = (const u32x4*)S.slo + (lane >> 5);
  const uint8_t* __restrict__ pg = S.sgn + lane * NB;
  // double-buffered groups: the loads of group g + 1 are issued before the products of g
  const int64_t ngroups = (kend - kbeg) / F;
  ChunkGroup<NB, RW, F> g0, g1;
  int64_t kc = kbeg;
  if (ngroups > 0) g0.load(at, ps, pl, pg, kc);
  int64_t g = 0;
  for (; g + 2 <= ngroups; g += 2) {
    g1.load(at, ps, pl, pg, kc + F);
    g0.mma(acc, masks);
    if (g + 2 < ngroups) g0.load(at, ps, pl, pg, kc + 2 * F);
    g1.mma(acc, masks);
    kc += 2 * F;
  }
  if (g < ngroups) {  // odd number of groups: the last one is in g0
    g0.mma(acc, masks);
    kc += F;
  }
  for (; kc < kend; ++kc) {
    ChunkGroup<NB, RW, 1> one;
    one.load(at, ps, pl, pg, kc);
    one.mma(acc, masks);
  }
  // accumulator layout: lane l, register v -> row 8 (v/4) + 4 (l/32) + v%4, column l%32
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    if (rb0 + r >= S.RB) break;
    float* __restrict__ out = S.part + ((int64_t)split * S.RB + rb0 + r) * kRows * 32 * NB;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v)
        out[((v >> 2) * 8 + (lane >> 5) * 4 + (v & 3)) * 32 * NB + b * 32 + (lane & 31)] = acc[r][b][v];
  }
}

// Both products of one step in one launch: the row pass over the tiles of A, then the
// column pass over the tiles of A' (Jacobi order: each reads the operands of step t-1).
// Workgroup b < R.groups * R.splits belongs to the row pass.
template <int NB, int RW, int F>
__global__ __launch_bounds__(kWaves * 64) void k_bf16_pass(Bf16Side R, Bf16Side C) {
  __shared__ u32x4 masks[256];
  for (int y = threadIdx.x; y < 256; y += kWaves * 64) masks[y] = sign_mask((uint32_t)y);
  __syncthreads();
  const int64_t nr = R.groups * R.splits;
  const int64_t b = blockIdx.x;
  if (b < nr) bf16_pass<NB, RW, F>(R, b % R.groups, (int)(b / R.groups), masks);
  else bf16_pass<NB, RW, F>(C, (b - nr) % C.groups, (int)((b - nr) / C.groups), masks);
}

// Sum over the eight lanes of an aligned group (every lane gets the sum).
__device__ __forceinline__ double octet_sum(double v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1, 0, 3, 2]: pairs
  v += dpp_mov<0x4E>(v);   // quad_perm [2, 3, 0, 1]: quads
  v += dpp_mov<0x141>(v);  // row_half_mirror: groups of 8
  return v;
}

// Index r with eight lanes: lane j of the eight adds the ranges of probes
// 4 NB j .. 4 NB j + 4 NB - 1 in FP64 (in range order), the squares of the probes p < k
// are summed across the eight lanes, and lane 0 of the eight updates the iterate.
template <int NB>
__device__ __forceinline__ void bf16_update(const Bf16Side& S, int64_t r, int j, int k, const StepScalars& sc,
                                            int* flag) {
  constexpr int PPL = 4 * NB;  // probes per lane
  const bool live = r < S.R;
  double ss = 0.0;
  if (live) {
    const int64_t stride = S.RB * kRows * 32 * NB / 4;  // float4 units
    const float4* __restrict__ base = (const float4*)(S.part + r * 32 * NB + j * PPL);
    double y[PPL];
#pragma unroll
    for (int i = 0; i < PPL; ++i) y[i] = 0.0;
    // four ranges' loads in flight at a time, added in range order
    for (int s0 = 0; s0 < S.splits; s0 += 4) {
      float4 q[4][NB];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int b = 0; b < NB; ++b)
          q[u][b] = s0 + u < S.splits ? base[(int64_t)(s0 + u) * stride + b] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (s0 + u >= S.splits) break;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          y[4 * b + 0] += (double)q[u][b].x;
          y[4 * b + 1] += (double)q[u][b].y;
          y[4 * b + 2] += (double)q[u][b].z;
          y[4 * b + 3] += (double)q[u][b].w;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < PPL; ++i)
      if (j * PPL + i < k) ss += y[i] * y[i];
  }
  ss = octet_sum(ss);
  if (live && j == 0) {
    double x = S.x[r], xb = S.xbar[r];
    if (!sgd_update(ss, k, S.target, sc, x, xb)) atomicOr(flag, 1);
    S.x[r] = x;
    S.xbar[r] = xb;
    const double ex = exp(x);
    const uint16_t hi = bf16_rne(ex);
    S.scl_out[r] = hi;
    S.slo_out[r] = bf16_lo(ex, hi);
  }
}

// Update of every index of both sides from the FP32 partials, 32 indices per workgroup
// (workgroups b < ceil(R.R / 32) take the rows), followed by the workgroups that write
// the sign bytes of the next step (they depend on the step only, and the passes of this
// step have finished reading the current ones).
template <int NB>
__global__ __launch_bounds__(256) void k_bf16_update(Bf16Side R, Bf16Side C, int k, StepScalars sc, int* flag,
                                                     ProbeSide N0, ProbeSide N1, uint64_t seed) {
  __shared__ uint64_t words[4 * kProbeBlocks];
  const int64_t rw = (R.R + 31) / 32, cw = (C.R + 31) / 32;
  const int64_t b = blockIdx.x;
  const int64_t i = threadIdx.x >> 3;
  const int j = threadIdx.x & 7;
  if (b < rw) bf16_update<NB>(R, b * 32 + i, j, k, sc, flag);
  else if (b < rw + cw) bf16_update<NB>(C, (b - rw) * 32 + i, j, k, sc, flag);
  else if (b < rw + cw + N0.groups) probe_group(N0, b - rw - cw, k, NB, seed, words);
  else probe_group(N1, b - rw - cw - N0.groups, k, NB, seed, words);
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

// Timing events released on every return path.
struct Events {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~Events() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

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

// Launch shape (compile-time; measured on the 16384 x 8192, k = 64 workload: one row
// block per wavefront, eight chunks per load group and about 128 workgroups per pass
// gave the shortest step).
#ifndef MFE_BF16_RW
#define MFE_BF16_RW 1
#endif
#ifndef MFE_BF16_F
#define MFE_BF16_F 8
#endif
#ifndef MFE_BF16_WG
#define MFE_BF16_WG 128
#endif
constexpr int kRW = MFE_BF16_RW;   // row blocks per wavefront
constexpr int kF = MFE_BF16_F;     // chunks per load group (two groups in flight)

// One step: both passes, then the updates with the sign bytes of the next step (none
// after the last step: N0.groups = N1.groups = 0).
template <int NB>
void launch_step(const Bf16Side& R, const Bf16Side& C, int k, const StepScalars& sc, int* flag,
                 const ProbeSide& N0, const ProbeSide& N1, uint64_t seed, hipStream_t st) {
  const int64_t wgs = R.groups * R.splits + C.groups * C.splits;
  k_bf16_pass<NB, kRW, kF><<<dim3((unsigned)wgs), dim3(kWaves * 64), 0, st>>>(R, C);
  const int64_t ub = ceil_div(R.R, 32) + ceil_div(C.R, 32) + N0.groups + N1.groups;
  k_bf16_update<NB><<<dim3((unsigned)ub), dim3(256), 0, st>>>(R, C, k, sc, flag, N0, N1, seed);
}

// k ranges per row block: about MFE_BF16_WG workgroups (of kWaves * kRW row blocks) per
// pass, at least 32 chunks per range.
int bf16_splits(int64_t RB, int64_t KC) {
  int64_t s = 1;
  while (ceil_div(RB, kWaves * kRW) * s < MFE_BF16_WG && KC / (2 * s) >= 32) s *= 2;
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
  u32x4 *tu, *tv;
  uint16_t *scu, *scv, *slu, *slv;
  uint8_t *sgu, *sgv;
  double *u, *ub, *v, *vb, *su, *sv;
  int* flag;
  MFE_CHECK(B.alloc(&tu, RBu * KCu * 64));
  MFE_CHECK(B.alloc(&tv, RBv * KCv * 64));
  // probe operands for the row pass (columns, side 0) and the column pass (rows, side 1)
  MFE_CHECK(B.alloc(&scu, KCu * kChunk));
  MFE_CHECK(B.alloc(&slu, KCu * kChunk));
  MFE_CHECK(B.alloc(&sgu, KCu * 64 * NB));
  MFE_CHECK(B.alloc(&scv, KCv * kChunk));
  MFE_CHECK(B.alloc(&slv, KCv * kChunk));
  MFE_CHECK(B.alloc(&sgv, KCv * 64 * NB));
  MFE_CHECK(B.alloc(&u, m));
  MFE_CHECK(B.alloc(&ub, m));
  MFE_CHECK(B.alloc(&v, n));
  MFE_CHECK(B.alloc(&vb, n));
  MFE_CHECK(B.alloc(&su, m));  // initial scales e^x (FP64), read by the first probe build
  MFE_CHECK(B.alloc(&sv, n));
  MFE_CHECK(B.alloc(&flag, 1));
  const int Su = bf16_splits(RBu, KCu), Sv = bf16_splits(RBv, KCv);
  float *partu, *partv;
  MFE_CHECK(B.alloc(&partu, (int64_t)Su * RBu * kRows * 32 * NB));
  MFE_CHECK(B.alloc(&partv, (int64_t)Sv * RBv * kRows * 32 * NB));
  MFE_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));

  const uint16_t* Ad = (const uint16_t*)A->data;
  k_tile<<<dim3((unsigned)ceil_div(RBu * KCu * 64, 256)), dim3(256), 0, st>>>(Ad, m, n, A->ld, 0, RBu, KCu, tu);
  k_tile<<<dim3((unsigned)ceil_div(RBv * KCv * 64, 256)), dim3(256), 0, st>>>(Ad, m, n, A->ld, 1, RBv, KCv, tv);
  k_bf_init<<<dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st>>>(m, p->u0, p->box_M, u, ub, su, flag);
  k_bf_init<<<dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st>>>(n, p->v0, p->box_M, v, vb, sv, flag);
  MFE_HIP(hipGetLastError());

  Events ev;
  MFE_HIP(hipEventCreate(&ev.e0));
  MFE_HIP(hipEventCreate(&ev.e1));
  MFE_HIP(hipEventRecord(ev.e0, st));
  const int64_t groups_u = ceil_div(RBu, kWaves * kRW), groups_v = ceil_div(RBv, kWaves * kRW);
  const int64_t pg_u = ceil_div(KCu, kProbeChunks), pg_v = ceil_div(KCv, kProbeChunks);
  const uint64_t bt = (uint64_t)p->batch;
  // probe operands of step 1 from the initial scales (Jacobi order): the row pass takes
  // the column scales and side-0 signs, the column pass the row scales and side-1 signs;
  // later steps get their scales from the updates and their sign bytes from the update
  // launch of the step before
  if (p->steps > 0) {
    ProbeSide P0{sv, n, KCu, stream_ctrl(bt, 1, 0), scu, slu, sgu, pg_u};
    ProbeSide P1{su, m, KCv, stream_ctrl(bt, 1, 1), scv, slv, sgv, pg_v};
    k_probe_build<<<dim3((unsigned)(pg_u + pg_v)), dim3(256), 0, st>>>(P0, P1, k, NB, p->seed);
  }
  for (int t = 1; t <= p->steps; ++t) {
    StepScalars sc;
    sc.tau = (double)t + (double)p->t0;
    sc.eta = 2.0 / (p->gamma * (sc.tau + 1.0));
    sc.gamma = p->gamma;
    sc.M = p->box_M;
    const bool more = t < p->steps;
    ProbeSide N0{nullptr, n, KCu, stream_ctrl(bt, (uint64_t)t + 1, 0), scu, slu, sgu, more ? pg_u : 0};
    ProbeSide N1{nullptr, m, KCv, stream_ctrl(bt, (uint64_t)t + 1, 1), scv, slv, sgv, more ? pg_v : 0};
    Bf16Side R{tu, scu, slu, sgu, m, RBu, KCu, Su, groups_u, partu, u, ub, scv, slv, p->alpha * p->alpha};
    Bf16Side Cc{tv, scv, slv, sgv, n, RBv, KCv, Sv, groups_v, partv, v, vb, scu, slu, p->beta * p->beta};
    if (NB == 1) launch_step<1>(R, Cc, k, sc, flag, N0, N1, p->seed, st);
    else launch_step<2>(R, Cc, k, sc, flag, N0, N1, p->seed, st);
  }
  MFE_HIP(hipGetLastError());
  MFE_HIP(hipEventRecord(ev.e1, st));
  k_bf_output<<<dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st>>>(m, ub, d, u_bar);
  k_bf_output<<<dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st>>>(n, vb, e, v_bar);
  MFE_HIP(hipGetLastError());
  int h = 0;
  MFE_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  MFE_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  MFE_HIP(hipEventElapsedTime(&ms, ev.e0, ev.e1));
  record_timing(ms, p->steps > 0 ? ms / p->steps : 0.0);
  if (h & 2) return set_error(MFE_EINVAL, "warm start u0/v0 outside the box [-M, M] (or NaN)");
  if (h & 1) return set_error(MFE_ENONFINITE, "non-finite gradient estimate or iterate (NaN/Inf in A?)");
  return MFE_OK;
}

}  // namespace mfe
