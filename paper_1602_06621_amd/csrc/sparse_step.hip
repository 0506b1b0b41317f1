// Step kernels of the sparse engine and their driver (Algorithm 1, Section 3.2).
//
// Step t is two launches, one per direction; both read the descriptors of step t-1
// (Jacobi order) and write those of step t (double-buffered):
//   rows:    Y_i = sum_j A_ij e^(v_j) s_jp        (p < k)  -> z_i = e^(2u_i) mean_p Y_ip^2
//            u_i <- clip(u_i - eta (z_i - alpha^2 + gamma u_i), -M, M),  u_bar update,
//            descriptor_i <- (e^(u_i), probe bits w_i of step t+1)
//   columns: X_j = sum_i A_ij e^(u_i) w_ip                -> z_j = e^(2v_j) mean_p X_jp^2
//            v_j update with beta, v_bar update, descriptor_j <- (e^(v_j), bits s_j of t+1)
//   extra workgroups of the row launch: Philox sign words of step t+2 for all indices.
// Arithmetic: matrix values FP32 (exact in FP64), scales, products, sums and iterates
// FP64.  Early steps of Algorithm 1 have eta gamma close to 1 and amplify rounding, so
// FP32 accumulation cannot track the FP64 iteration to 1e-5 (measured, see the
// design notes); FP64 costs no more VALU issue slots than unpacked FP32 on gfx950.
#include <cmath>
#include <vector>

#include "sparse.h"

namespace mfe {
namespace {

// acc_p += (-1)^bit_p * t for p < KP.  The sign of t is folded into the probe bits so
// each probe costs one shift, one and-or on the high word and one FP64 add.
template <int KP>
__device__ __forceinline__ void accumulate(double (&acc)[KP], double t, uint64_t bits) {
  const uint64_t tb = (uint64_t)__double_as_longlong(t);
  const uint32_t lo = (uint32_t)tb;
  const uint32_t hi_abs = (uint32_t)(tb >> 32) & 0x7FFFFFFFu;
  if (tb >> 63) bits = ~bits;
  const uint32_t b0 = (uint32_t)bits;
  const uint32_t b1 = (uint32_t)(bits >> 32);
#pragma unroll
  for (int p = 0; p < KP; ++p) {
    const uint32_t sb = p < 32 ? ((b0 << (31 - (p & 31))) & 0x80000000u)
                               : ((b1 << (31 - (p & 31))) & 0x80000000u);
    acc[p] += __longlong_as_double((long long)(((uint64_t)(hi_abs | sb) << 32) | lo));
  }
}

// Descriptor codecs.  Wide: {FP64 scale, 64 sign bits} (16 B).  Packed (8 B, KP <= 16 and
// |x| <= 11): e^x has an unbiased binary exponent in [-16, 15], stored in 5 bits; the
// low KP bits hold the probe signs and the mantissa keeps 52 - max(0, KP - 7) bits
// (rounded to nearest: relative error at most 2^-44 for KP = 16, exact for KP <= 7; a
// carry out of the mantissa moves into the exponent, which stays in range because
// e^11 < 2^16).  Halving the gathered table keeps more of it in each XCD's L2, which
// sets the gather rate.
template <int KP, bool PACKED>
struct Codec;

template <int KP>
struct Codec<KP, false> {
  using T = Desc;
  __device__ static inline void decode(const T& d, double& scale, uint64_t& bits) {
    scale = d.scale;
    bits = d.bits;
  }
  __device__ static inline T encode(double scale, uint64_t bits) {
    T d;
    d.scale = scale;
    d.bits = bits;
    return d;
  }
};

template <int KP>
struct Codec<KP, true> {
  using T = uint64_t;
  static constexpr int kDrop = KP > 7 ? KP - 7 : 0;
  static constexpr int kMant = 52 - kDrop;
  __device__ static inline void decode(const T& d, double& scale, uint64_t& bits) {
    bits = d & ((1ull << KP) - 1ull);
    const uint64_t mant = ((d >> KP) & ((1ull << kMant) - 1ull)) << kDrop;
    const uint64_t ex = (d >> 59) + 1007ull;
    scale = __longlong_as_double((long long)((ex << 52) | mant));
  }
  __device__ static inline T encode(double scale, uint64_t bits) {
    uint64_t u = (uint64_t)__double_as_longlong(scale);
    if constexpr (kDrop > 0) u += 1ull << (kDrop - 1);  // round half up on the dropped bits
    const uint64_t ex = ((u >> 52) & 0x7FFull) - 1007ull;
    const uint64_t mant = (u & ((1ull << 52) - 1ull)) >> kDrop;
    return (ex << 59) | (mant << KP) | bits;
  }
};

// Entry streams and per-index state are read and written with non-temporal hints (nt,
// uniform over a launch, chosen per plan by stream_hints) or with plain accesses.  Plain
// accesses are faster when the step's streams fit the 256 MB Infinity Cache, which the
// hinted streams bypass (1e6 x 5e5 headline, ~250 MB: 192.4 us per step with both hinted,
// 182.0 with plain entry loads, 179.7 with both plain, at 8 slots in flight), so that the
// entries of step t+1 are partly served from it; a plan whose streams do not fit (512
// matrices, 4.4 GB per step: 2.25 ms hinted against 2.33 ms plain) keeps them out of the
// way of the gathered tables.
// NT is a template parameter, and each kernel branches once on the plan's flag: a run-time
// choice between a hinted and a plain load of the same address is merged by the compiler
// into one plain load.
template <bool NT, class T>
__device__ __forceinline__ T ld_stream(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, class T>
__device__ __forceinline__ void st_stream(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
template <bool NT>
__device__ __forceinline__ void st_stream(Desc* p, Desc v) {
  u64x2 w;
  w.x = (unsigned long long)__double_as_longlong(v.scale);
  w.y = v.bits;
  st_stream<NT>(reinterpret_cast<u64x2*>(p), w);
}

// Sums of the signed products of slots [q_beg, q_end) of one row into acc.  Batches of
// NB slots: all entry loads of a batch are issued, then all descriptor gathers, then the
// accumulation, so a wavefront keeps 2 x NB independent memory requests in flight
// instead of one dependent load/gather pair per slot.
template <int KP, bool PACKED, int NB, bool NT>
__device__ __forceinline__ void gather_rows(const long long* __restrict__ e,
                                            const typename Codec<KP, PACKED>::T* __restrict__ gather, int q_beg,
                                            int q_end, double (&acc)[KP]) {
  using C = Codec<KP, PACKED>;
  using DT = typename C::T;
  for (int q0 = q_beg; q0 < q_end; q0 += NB) {
    long long en[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u)
      en[u] = (q0 + u < q_end) ? ld_stream<NT>(e + (int64_t)(q0 + u) * kSlice) : 0ll;
    DT d[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (q0 + u < q_end) d[u] = gather[(int32_t)(en[u] & 0xFFFFFFFFll)];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      if (q0 + u < q_end) {
        double scale;
        uint64_t bits;
        C::decode(d[u], scale, bits);
        const float a = __int_as_float((int32_t)(en[u] >> 32));
        accumulate<KP>(acc, (double)a * scale, bits);
      }
    }
  }
}

// Update of internal index r from its k probe sums (a5-a7 and the next descriptor).
// VAR (the Section 6 variant kernel): per-index target, or the estimate z written out for
// the block update instead of the update itself.
template <int KP, bool PACKED, bool VAR, bool NT>
__device__ __forceinline__ void finish_update(const SideDev& S, const MatDev* __restrict__ mats, int k,
                                              const StepScalars& sc, int64_t r, int32_t li, int32_t mi,
                                              double x_old, double xbar_old, double tgt_r, const double (&acc)[KP],
                                              int* flag) {
  // Every product and sum of the update is rounded on its own (no fused multiply-add),
  // as in the plain definition, so that all kernels that finish an update agree bit
  // for bit.
#pragma clang fp contract(off)
  using C = Codec<KP, PACKED>;
  using DT = typename C::T;
  const MatDev mt = mats[mi];
  double ss = 0.0;
#pragma unroll
  for (int p = 0; p < KP; ++p)
    if (p < k) ss += acc[p] * acc[p];
  const double z = exp(2.0 * x_old) * (ss / (double)k);
  double tgt = S.is_row ? mt.tgt_row : mt.tgt_col;
  if constexpr (VAR) {
    if (S.zout) {  // block side: the estimate goes to the block update
      if (!isfinite(z)) atomicOr(flag, 1);
      st_stream<NT>(S.zout + r, z);
      return;
    }
    if (S.tgt) tgt = tgt_r;
  }
  const double g = (z - tgt) + sc.gamma * x_old;
  double xn = x_old - sc.eta * g;
  xn = fmin(fmax(xn, -sc.M), sc.M);
  const bool bad = !isfinite(z) || !isfinite(xn);
  if (bad) {
    atomicOr(flag, 1);
    xn = 0.0;  // keep the descriptor encodable; the run reports MFE_ENONFINITE
  }
  st_stream<NT>(S.x + r, xn);
  st_stream<NT>(S.xbar + r, 2.0 * xn / (sc.tau + 2.0) + sc.tau * xbar_old / (sc.tau + 2.0));
  const int64_t wbase = S.is_row ? mt.sign_word_row : mt.sign_word_col;
  st_stream<NT>(reinterpret_cast<DT*>(S.out) + r,
            C::encode(exp(xn), extract_bits(S.next_signs + wbase, (int64_t)li * k, k)));
}

// One lane per row.  part_mode (two-part layouts, see SideDev): 0 whole rows; 1 entries
// [0, len_lo) to the partial sums; 2 partial sums plus entries [len_lo, len), then the
// update.
template <int KP, bool PACKED, int NB, bool VAR, bool NT, int WT = kBlock>
__device__ __forceinline__ void side_update(const SideDev& S, const MatDev* __restrict__ mats, int k,
                                            const StepScalars& sc, int64_t blk, int* flag) {
  // WT: threads per workgroup when fixed at compile time (0: the launch's blockDim)
  using C = Codec<KP, PACKED>;
  using DT = typename C::T;
  const int64_t wv = blk * ((WT ? WT : (int)blockDim.x) / kSlice) + (threadIdx.x >> 6);  // wavefront of the launch
  if (wv * kSlice >= S.nint) return;  // whole wavefronts leave together
  const int64_t s = S.sched ? (int64_t)S.sched[wv] : wv;
  const int64_t r = s * kSlice + (threadIdx.x & 63);
  const int lane = (int)(threadIdx.x & 63);
  const int mode = S.part_mode;  // uniform over the launch
  const bool partial_out = mode == 1;
  const int len = ld_stream<NT>(S.len + r);
  const int split = mode != 0 ? ld_stream<NT>(S.len_lo + r) : 0;
  const int q_beg = mode == 2 ? split : 0;
  const int q_end = mode == 1 ? split : len;
  // The epilogue's operands are loaded before the gather loop so their latency overlaps
  // it -- except in the Section 6 kernels, where loading them after the loop shortens
  // their live range enough for the one-launch variant kernel to run eight waves per SIMD
  // without spilling (per-index targets 137-139 -> 130-132 us per step on the 1e6 x 5e5
  // matrix, 16 x 8 blocks 142 -> 137 us; results unchanged bit for bit).
  int32_t li = 0, mi = 0;
  double x_old = 0.0, xbar_old = 0.0, tgt_r = 0.0;
  auto load_epilogue = [&]() {
    li = ld_stream<NT>(S.orig + r);
    x_old = ld_stream<NT>(S.x + r);
    if (!VAR || !S.zout) xbar_old = ld_stream<NT>(S.xbar + r);
    mi = S.slice_mat[s];
    if constexpr (VAR) {
      if (S.tgt) tgt_r = ld_stream<NT>(S.tgt + r);
    }
  };
  if (!partial_out && !VAR) load_epilogue();
  const long long* __restrict__ e = reinterpret_cast<const long long*>(S.ent + S.slice_off[s] + lane);
  const DT* __restrict__ gather = reinterpret_cast<const DT*>(S.gather);
  double acc[KP];
#pragma unroll
  for (int p = 0; p < KP; ++p) acc[p] = (mode == 2 && p < k) ? ld_stream<NT>(S.part + (int64_t)p * S.nint + r) : 0.0;
  gather_rows<KP, PACKED, NB, NT>(e, gather, q_beg, q_end, acc);
  if (partial_out) {
#pragma unroll
    for (int p = 0; p < KP; ++p)
      if (p < k) st_stream<NT>(S.part + (int64_t)p * S.nint + r, acc[p]);
    return;
  }
  if (VAR) load_epilogue();
  if (li < 0) return;
  finish_update<KP, PACKED, VAR, NT>(S, mats, k, sc, r, li, mi, x_old, xbar_old, tgt_r, acc, flag);
}

// Long rows in few slices: a workgroup of P wavefronts per slice, wavefront w walking
// the slots [w c, (w+1) c) of every row of the slice (c = ceil(width / P)); wavefront 0
// adds the P partial sums in order through LDS and finishes the update.  P is at most
// split_max<KP>() so that the partial sums fit in 64 KB of LDS.
template <int KP>
constexpr int split_max() {
  return 1 + 65536 / (KP * kSlice * 8) < 16 ? 1 + 65536 / (KP * kSlice * 8) : 16;
}

template <int KP, bool PACKED, bool VAR, bool NT>
__device__ __forceinline__ void side_update_split(const SideDev& S, const MatDev* __restrict__ mats, int k,
                                                  const StepScalars& sc, int64_t s, int P, int* flag) {
  using C = Codec<KP, PACKED>;
  using DT = typename C::T;
  constexpr int PM = split_max<KP>();
  __shared__ double part[(PM > 1 ? PM - 1 : 1) * KP * kSlice];
  const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int64_t r = s * kSlice + lane;
  const int len = ld_stream<NT>(S.len + r);
  int32_t li = 0, mi = 0;
  double x_old = 0.0, xbar_old = 0.0, tgt_r = 0.0;
  if (w == 0) {
    li = ld_stream<NT>(S.orig + r);
    x_old = ld_stream<NT>(S.x + r);
    if (!VAR || !S.zout) xbar_old = ld_stream<NT>(S.xbar + r);
    mi = S.slice_mat[s];
    if constexpr (VAR) {
      if (S.tgt) tgt_r = ld_stream<NT>(S.tgt + r);
    }
  }
  const int64_t base = S.slice_off[s];
  const int width = (int)((S.slice_off[s + 1] - base) / kSlice);
  const int chunk = (width + P - 1) / P;
  const int q0 = min(len, w * chunk), q1 = min(len, w * chunk + chunk);
  const long long* __restrict__ e = reinterpret_cast<const long long*>(S.ent + base + lane);
  const DT* __restrict__ gather = reinterpret_cast<const DT*>(S.gather);
  double acc[KP];
#pragma unroll
  for (int p = 0; p < KP; ++p) acc[p] = 0.0;
  gather_rows<KP, PACKED, kBatch, NT>(e, gather, q0, q1, acc);
  if (w > 0) {
#pragma unroll
    for (int p = 0; p < KP; ++p)
      if (p < k) part[((w - 1) * KP + p) * kSlice + lane] = acc[p];
  }
  __syncthreads();
  if (w != 0) return;
  for (int i = 1; i < P; ++i) {
#pragma unroll
    for (int p = 0; p < KP; ++p)
      if (p < k) acc[p] += part[((i - 1) * KP + p) * kSlice + lane];
  }
  if (li < 0) return;
  finish_update<KP, PACKED, VAR, NT>(S, mats, k, sc, r, li, mi, x_old, xbar_old, tgt_r, acc, flag);
}

__device__ __forceinline__ void signgen_block(const SignGenDev& g, int64_t gblk, int64_t bsize = kBlock) {
  const int64_t c = gblk * bsize + threadIdx.x;
  if (c >= g.nblocks) return;
  int lo = 0, hi = g.nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g.seg_prefix[mid] <= c) lo = mid;
    else hi = mid - 1;
  }
  const SignSeg sg = g.segs[lo];
  const int64_t cb = c - g.seg_prefix[lo];
  const U64x4 w = philox4x64_10((uint64_t)cb + 1, 0, 0, 0, g.seed, sg.ctrl_lo | (g.step << 2));
  uint64_t* o = g.out + sg.word_off + 4 * cb;
  o[0] = w.x[0];
  o[1] = w.x[1];
  o[2] = w.x[2];
  o[3] = w.x[3];
}

// Minimum waves per SIMD the one-launch step kernel is compiled for.  One slot in flight
// with at most 16 probes: 8 (64 VGPRs, 12 bytes spilled), which keeps eight workgroups per
// CU resident instead of five (85 VGPRs): 131.3 -> 126.1 us per step on the 1e6 x 5e5
// headline (131 at six waves); the 2e5 x 1e5 warm-start matrix is unchanged (40.2 us).
// The same bound on the single-direction kernels made them slower (the symmetric product
// 75.8 -> 83.5 us: 28-44 bytes spilled; 77.6 us with their epilogue operands loaded after
// the gather loop, 12 bytes spilled, and one launch per direction on the headline 133.5 ->
// 138.5 us), so they keep the compiler's choice; the Section 6
// one-launch kernel spilled as well (per-index targets 132.7 -> 140.2 us) until its
// epilogue operands were loaded after the gather loop (var_step_waves).  Other probe
// counts and loads in flight keep the compiler's choice too (more accumulators or loads):
// with 8 probes and 16 loads in flight a bound of
// five waves (96 VGPRs instead of 107, 52 bytes spilled) took the 512-matrix batched
// step from 2.07 to 2.53 ms.
template <int KP, int NB>
constexpr int step_waves() {
  return (KP <= 16 && NB == 1) ? 8 : 1;
}

// The same bound for the one-launch Section 6 kernel up to 16 probes (64 VGPRs, no spill
// with its epilogue operands loaded after the gather loop).
template <int KP>
constexpr int var_step_waves() {
  return KP <= 16 ? 8 : 1;
}

// Largest workgroup of the one-launch step kernel (the launch size is a plan tuning, 256
// threads by default): 1024 threads up to 8 probes with 8-byte descriptors, 512 up to
// 16, 256 above -- and 256 for
// 16 probes at one slot in flight, the headline form: a larger bound caps the registers
// the compiler may give a lane, which raised that kernel's spill from 12 to 20 bytes and
// its step from 126 to 130 us (the 200k x 100k warm-start matrix gained 1 us at 512
// threads); at 1024 threads the 16-probe forms spilled 20-212 bytes.  The batched
// workload (8 probes, 16 slots in flight) runs 2.08 ms per step at 512 threads against
// 2.25 at 256 and 2.23 at 1024.
template <int KP, int NB, bool PACKED>
constexpr int step_max_threads() {
  return KP <= 8 && PACKED ? 1024 : (KP <= 16 && NB > 1 ? 512 : kBlock);
}

// One direction of one step; extra workgroups past side_blocks draw the sign words
// of step t+2 (the row launch carries them).
template <int KP, bool PACKED, int NB>
__global__ __launch_bounds__(kBlock) void k_phase(PhaseArgs a) {
  const int64_t b = blockIdx.x;
  if (b >= a.side_blocks) signgen_block(a.gen, b - a.side_blocks);
  else if (a.side.nt) side_update<KP, PACKED, NB, false, true>(a.side, a.mats, a.k, a.sc, b, a.flag);
  else side_update<KP, PACKED, NB, false, false>(a.side, a.mats, a.k, a.sc, b, a.flag);
}

// Both directions of one step in one launch (row workgroups, then column workgroups,
// then the sign words): for plans too small to fill the device with one direction.  The
// directions read the other's descriptors of step t-1 and write their own of step t, so
// they are independent within a step.
template <int KP, bool PACKED, int NB, bool VAR, bool NT, int WT = kBlock>
__device__ __forceinline__ void phase_both(const PhaseArgs& a, const SideDev& C, int64_t b) {
  if (b < a.side_blocks) side_update<KP, PACKED, NB, VAR, NT, WT>(a.side, a.mats, a.k, a.sc, b, a.flag);
  else side_update<KP, PACKED, NB, VAR, NT, WT>(C, a.mats, a.k, a.sc, b - a.side_blocks, a.flag);
}

template <int KP, bool PACKED, int NB>
__global__ __launch_bounds__((step_max_threads<KP, NB, PACKED>()), (step_waves<KP, NB>())) void k_phase_both(PhaseArgs a, SideDev C,
                                                                            int64_t col_blocks) {
  // workgroup size fixed at compile time where the bound allows only kBlock threads (the
  // constant keeps that kernel's register allocation), else read from the launch
  constexpr int WT = step_max_threads<KP, NB, PACKED>() == kBlock ? kBlock : 0;
  const int64_t b = blockIdx.x;
  if (b >= a.side_blocks + col_blocks)
    signgen_block(a.gen, b - a.side_blocks - col_blocks, (int64_t)(WT ? WT : (int)blockDim.x));
  else if (a.side.nt) phase_both<KP, PACKED, NB, false, true, WT>(a, C, b);
  else phase_both<KP, PACKED, NB, false, false, WT>(a, C, b);
}

// The same with the Section 6 variant update (per-index targets, block sides).
template <int KP, bool PACKED>
__global__ __launch_bounds__(kBlock, (var_step_waves<KP>())) void k_phase_both_var(PhaseArgs a, SideDev C,
                                                                          int64_t col_blocks) {
  const int64_t b = blockIdx.x;
  if (b >= a.side_blocks + col_blocks) signgen_block(a.gen, b - a.side_blocks - col_blocks, (int64_t)blockDim.x);
  else if (a.side.nt) phase_both<KP, PACKED, kBatch, true, true>(a, C, b);
  else phase_both<KP, PACKED, kBatch, true, false>(a, C, b);
}

// The same for the Section 6 variants (per-index targets, block sides, symmetric plans).
template <int KP, bool PACKED>
__global__ __launch_bounds__(kBlock) void k_phase_var(PhaseArgs a) {
  const int64_t b = blockIdx.x;
  if (b >= a.side_blocks) signgen_block(a.gen, b - a.side_blocks);
  else if (a.side.nt) side_update<KP, PACKED, kBatch, true, true>(a.side, a.mats, a.k, a.sc, b, a.flag);
  else side_update<KP, PACKED, kBatch, true, false>(a.side, a.mats, a.k, a.sc, b, a.flag);
}

__global__ __launch_bounds__(kBlock) void k_signgen(SignGenDev g) { signgen_block(g, blockIdx.x); }

// One slice per workgroup of 64 P threads (side_update_split); workgroups past
// side_blocks (= slices) draw the sign words of step t+2, 64 P Philox blocks each.
template <int KP, bool PACKED, bool VAR>
__global__ __launch_bounds__(kSlice * split_max<KP>()) void k_phase_split(PhaseArgs a, int P) {
  const int64_t b = blockIdx.x;
  if (b >= a.side_blocks) {
    signgen_block(a.gen, b - a.side_blocks, (int64_t)blockDim.x);
    return;
  }
  const int64_t s = a.side.sched ? (int64_t)a.side.sched[b] : b;
  if (a.side.nt) side_update_split<KP, PACKED, VAR, true>(a.side, a.mats, a.k, a.sc, s, P, a.flag);
  else side_update_split<KP, PACKED, VAR, false>(a.side, a.mats, a.k, a.sc, s, P, a.flag);
}

// Lane groups of the block kernels: G lanes (a power of two, 1..64, chosen from the
// mean block size) share one block; the wavefront holds 64 / G blocks.  group_sum adds
// the G lanes' values in a fixed butterfly order and returns the group's first lane's
// result in every lane of the group, so the value is the same on every run.
__device__ __forceinline__ double group_sum(double v, int G) {
  for (int off = G >> 1; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = (int)(threadIdx.x & 63);
  return G > 1 ? __shfl(v, lane & ~(G - 1), 64) : v;
}

// Block update of one side (Section 6, block equilibration): the sum of the indices'
// estimates over each block (original index order, each lane of the block's group a
// strided part, then the group sum), the projected step and the average of the block
// variable, then every index of the block gets the new value and its descriptor for
// the next step.  init != 0: the block variables start from x0 (or 0) instead.
template <int KP, bool PACKED>
__device__ __forceinline__ void block_step(const SideDev& S, const BlockDev& B, int k, const StepScalars& sc,
                                           int64_t wbase, const double* __restrict__ x0, int init, int* flag,
                                           int64_t gt) {
#pragma clang fp contract(off)
  using C = Codec<KP, PACKED>;
  const int G = B.group;
  const int64_t b = gt / G;
  const int sub = (int)(gt % G);
  const bool valid = b < B.nb;
  const int64_t j0 = valid ? B.ptr[b] : 0, j1 = valid ? B.ptr[b + 1] : 0;
  double xn = 0.0;
  if (init) {
    if (valid) {
      xn = x0 ? x0[b] : 0.0;
      if (!(fabs(xn) <= sc.M)) {
        if (sub == 0) atomicOr(flag, 2);
        xn = 0.0;
      }
      if (sub == 0) {
        B.bx[b] = xn;
        B.bxbar[b] = xn;
      }
    }
  } else {
    double part = 0.0;
    for (int64_t j = j0 + sub; j < j1; j += G) part += B.z[B.orig2int[j]];
    const double zb = group_sum(part, G);  // every lane takes part
    if (valid) {
      const double x_old = B.bx[b];
      const double g = (zb - B.tgt[b]) + sc.gamma * x_old;
      xn = x_old - sc.eta * g;
      xn = fmin(fmax(xn, -sc.M), sc.M);
      if (!isfinite(zb) || !isfinite(xn)) {
        if (sub == 0) atomicOr(flag, 1);
        xn = 0.0;
      }
      if (sub == 0) {
        B.bx[b] = xn;
        B.bxbar[b] = 2.0 * xn / (sc.tau + 2.0) + sc.tau * B.bxbar[b] / (sc.tau + 2.0);
      }
    }
  }
  if (!valid) return;
  const double sx = exp(xn);
  for (int64_t j = j0 + sub; j < j1; j += G) {
    const int32_t r = B.orig2int[j];
    S.x[r] = xn;
    reinterpret_cast<typename C::T*>(S.out)[r] = C::encode(sx, extract_bits(S.next_signs + wbase, j * k, k));
  }
}

template <int KP, bool PACKED>
__global__ __launch_bounds__(256) void k_block_step(SideDev S, BlockDev B, int k, StepScalars sc,
                                                    int64_t wbase, const double* __restrict__ x0, int init,
                                                    int* flag) {
  block_step<KP, PACKED>(S, B, k, sc, wbase, x0, init, flag, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Both sides' block updates of a step in one launch (they are independent within a step:
// each reads its own side's estimates and writes its own side's state): the first row_wgs
// workgroups take the row blocks, the rest the column blocks.
template <int KP, bool PACKED>
__global__ __launch_bounds__(256) void k_block_step_both(SideDev S0, BlockDev B0, StepScalars sc0, int64_t wbase0,
                                                         SideDev S1, BlockDev B1, StepScalars sc1, int64_t wbase1,
                                                         int k, int64_t row_wgs, int* flag) {
  const int64_t w = blockIdx.x;
  if (w < row_wgs)
    block_step<KP, PACKED>(S0, B0, k, sc0, wbase0, nullptr, 0, flag, w * blockDim.x + threadIdx.x);
  else
    block_step<KP, PACKED>(S1, B1, k, sc1, wbase1, nullptr, 0, flag, (w - row_wgs) * blockDim.x + threadIdx.x);
}

// Targets of the blocks of one side: the sum over each block of the indices' squared
// targets (t2 each when no per-index targets are set), one lane group per block.
__global__ __launch_bounds__(256) void k_block_targets(const int64_t* __restrict__ ptr, int64_t nb, int G,
                                                       const double* __restrict__ tgt, double t2,
                                                       double* __restrict__ out) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t b = gt / G;
  const int sub = (int)(gt % G);
  const bool valid = b < nb;
  double part = 0.0;
  if (valid)
    for (int64_t j = ptr[b] + sub; j < ptr[b + 1]; j += G) part += tgt ? tgt[j] : t2;
  const double sum = group_sum(part, G);
  if (valid && sub == 0) out[b] = sum;
}

// Per-index outputs of a block side: e^(x_bar) of the index's block.
__global__ void k_block_output(BlockDev B, double* __restrict__ dout, double* __restrict__ xbar_out) {
  const int G = B.group;
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t b = gt / G;
  const int sub = (int)(gt % G);
  if (b >= B.nb) return;
  const double xb = B.bxbar[b];
  const double dv = exp(xb);
  for (int64_t j = B.ptr[b] + sub; j < B.ptr[b + 1]; j += G) dout[j] = dv;
  if (sub == 0 && xbar_out) xbar_out[b] = xb;
}

// Workgroups of 256 threads covering nb blocks of G lanes.
inline unsigned block_grid(int64_t nb, int G) { return (unsigned)ceil_div(nb * G, 256); }


template <int KP, bool PACKED>
__global__ void k_init(SideDev S, const MatDev* __restrict__ mats, const double* __restrict__ x0, int k, double M,
                       int* flag) {
  using C = Codec<KP, PACKED>;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= S.nint) return;
  const int32_t li = S.orig[r];
  if (li < 0) return;
  const MatDev mt = mats[S.slice_mat[r >> 6]];
  const int64_t g = (S.is_row ? mt.row_orig_base : mt.col_orig_base) + li;
  double x = x0 ? x0[g] : 0.0;
  if (!(fabs(x) <= M)) {
    atomicOr(flag, 2);  // warm start outside the box (or NaN)
    x = 0.0;
  }
  S.x[r] = x;
  S.xbar[r] = x;
  const uint64_t bits = extract_bits(S.next_signs + (S.is_row ? mt.sign_word_row : mt.sign_word_col), (int64_t)li * k, k);
  reinterpret_cast<typename C::T*>(S.out)[r] = C::encode(exp(x), bits);
}

__global__ void k_output(SideDev S, const MatDev* __restrict__ mats, double* __restrict__ dout,
                         double* __restrict__ xbar_out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= S.nint) return;
  const int32_t li = S.orig[r];
  if (li < 0) return;
  const MatDev mt = mats[S.slice_mat[r >> 6]];
  const int64_t g = (S.is_row ? mt.row_orig_base : mt.col_orig_base) + li;
  const double xb = S.xbar[r];
  dout[g] = exp(xb);
  if (xbar_out) xbar_out[g] = xb;
}

template <class T>
int ensure(T** ptr, int64_t count) {
  if (*ptr) return MFE_OK;
  hipError_t e = hipMalloc((void**)ptr, sizeof(T) * (size_t)std::max<int64_t>(count, 1));
  if (e != hipSuccess)
    return set_error(e == hipErrorOutOfMemory ? MFE_ENOMEM : MFE_EDEVICE, "hipMalloc failed: %s",
                     hipGetErrorString(e));
  return MFE_OK;
}

// Sign stream layout of a plan for k probes: per matrix, one segment for side 0
// (columns) and one for side 1 (rows), each starting on a Philox block boundary.
int build_sign_layout(mfe_plan* p, int k, int64_t batch_base) {
  if (p->sign_k == k && p->sign_batch_base == batch_base) return MFE_OK;
  // A cached graph holds the addresses of the sign buffers freed below: drop it, so
  // that the next graph run captures the new ones (its key alone cannot tell, since a
  // later run may come back to the same k and batch).
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->graph_exec = nullptr;
  p->graph = nullptr;
  for (int i = 0; i < 2; ++i) {
    (void)hipFree(p->signs[i]);
    p->signs[i] = nullptr;
  }
  (void)hipFree(p->segs);
  (void)hipFree(p->seg_prefix);
  p->segs = nullptr;
  p->seg_prefix = nullptr;
  p->segs_host.clear();
  std::vector<int64_t> prefix;
  int64_t words = 0, blocks = 0;
  prefix.push_back(0);
  for (int side = 0; side < 2; ++side) {
    for (int b = 0; b < p->count; ++b) {
      const int64_t cnt = side == 0 ? p->meta[b].n : p->meta[b].m;
      SignSeg sg;
      sg.ctrl_lo = ((uint64_t)(batch_base + b) << 34) | (uint64_t)side;
      sg.nblocks = ceil_div(cnt * k, 256);
      sg.word_off = words;
      words += 4 * sg.nblocks + 4;  // one spare block: bit extraction may read one word past the end
      blocks += sg.nblocks;
      prefix.push_back(blocks);
      p->segs_host.push_back(sg);
    }
  }
  p->sign_words = words;
  p->sign_blocks = blocks;
  MFE_CHECK(ensure(&p->signs[0], words));
  MFE_CHECK(ensure(&p->signs[1], words));
  MFE_HIP(hipMemset(p->signs[0], 0, sizeof(uint64_t) * words));
  MFE_HIP(hipMemset(p->signs[1], 0, sizeof(uint64_t) * words));
  MFE_CHECK(ensure(&p->segs, (int64_t)p->segs_host.size()));
  MFE_CHECK(ensure(&p->seg_prefix, (int64_t)prefix.size()));
  MFE_HIP(hipMemcpy(p->segs, p->segs_host.data(), sizeof(SignSeg) * p->segs_host.size(), hipMemcpyHostToDevice));
  MFE_HIP(hipMemcpy(p->seg_prefix, prefix.data(), sizeof(int64_t) * prefix.size(), hipMemcpyHostToDevice));
  p->sign_k = k;
  p->sign_batch_base = batch_base;
  return MFE_OK;
}

SignGenDev make_gen(const mfe_plan* p, uint64_t seed, uint64_t step, uint64_t* out) {
  SignGenDev g;
  g.segs = p->segs;
  g.seg_prefix = p->seg_prefix;
  g.nseg = (int32_t)p->segs_host.size();
  g.nblocks = p->sign_blocks;
  g.seed = seed;
  g.step = step;
  g.out = out;
  return g;
}

// Whether a run's entry and state streams use non-temporal accesses: the plan's tuning,
// else by the size of the streams one step moves (8-byte entries of both directions, and
// about 64 bytes of state, descriptors and layout per internal index).
int stream_hints(const mfe_plan* p) {
  if (p->tune_nt >= 0) return p->tune_nt;
  const int64_t bytes = 8 * (p->rows.nent + p->cols.nent) + 64 * (p->rows.nint + p->cols.nint);
  return bytes > kStreamHintBytes ? 1 : 0;
}

// Whether a run's step launches take the slices in the layout's longest-first order: the
// plan's tuning, else when the order has a tail to shorten -- the one-launch step has more
// workgroups than one round of the device's resident workgroups (about 5 per CU), or a
// direction runs the split kernels (one slice per workgroup).  Measured, µs per step: 1e6
// x 5e5 headline (5,861 workgroups) 130.8 with the order against 148.7 without; 5e4 x
// 2.5e4 (split kernels) 31.5 against 33.1; 2e5 x 1e5 with U{8..16} entries per row (1,173
// workgroups, one round) 42.1 against 40.2.
int slice_schedule(const mfe_plan* p, int64_t row_blocks, int64_t col_blocks, bool split) {
  if (p->tune_sched >= 0) return p->tune_sched;
  if (split) return 1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  return row_blocks + col_blocks > 5ll * cus ? 1 : 0;
}

SideDev make_side(const SideLayout& L, double* x, double* xbar, const void* gather, void* out,
                  const uint64_t* next_signs, int is_row) {
  SideDev S;
  S.slice_off = L.slice_off;
  S.slice_mat = L.slice_mat;
  S.len = L.len;
  S.orig = L.orig;
  S.ent = L.ent;
  S.nint = L.nint;
  S.x = x;
  S.xbar = xbar;
  S.gather = gather;
  S.out = out;
  S.next_signs = next_signs;
  S.is_row = is_row;
  S.part_mode = 0;
  S.len_lo = L.len_lo;
  S.part = nullptr;
  S.tgt = nullptr;
  S.zout = nullptr;
  S.sched = L.sched;
  S.nt = 0;
  return S;
}

template <int KP, bool PACKED, int NB>
void launch_phase(const PhaseArgs& a, hipStream_t st) {
  k_phase<KP, PACKED, NB><<<dim3((unsigned)(a.side_blocks + a.gen_blocks)), dim3(kBlock), 0, st>>>(a);
}

template <int KP, bool PACKED>
void launch_init(const SideDev& S, const MatDev* mats, const double* x0, int k, double M, int* flag, hipStream_t st) {
  k_init<KP, PACKED><<<dim3((unsigned)ceil_div(S.nint, 256)), dim3(256), 0, st>>>(S, mats, x0, k, M, flag);
}

// Dispatch on the probe bucket KP >= k and on the descriptor format.
template <template <int, bool> class F, class... Args>
void dispatch(int k, bool packed, Args&&... args) {
  if (packed) {
    if (k <= 1) F<1, true>::run(args...);
    else if (k <= 2) F<2, true>::run(args...);
    else if (k <= 4) F<4, true>::run(args...);
    else if (k <= 8) F<8, true>::run(args...);
    else F<16, true>::run(args...);
  } else {
    if (k <= 1) F<1, false>::run(args...);
    else if (k <= 2) F<2, false>::run(args...);
    else if (k <= 4) F<4, false>::run(args...);
    else if (k <= 8) F<8, false>::run(args...);
    else if (k <= 16) F<16, false>::run(args...);
    else if (k <= 32) F<32, false>::run(args...);
    else F<64, false>::run(args...);
  }
}

// Loads in flight per lane: 4, 8 or 16 slots (16 only up to 16 probes, where the
// accumulators leave room for it).
template <int KP, bool PACKED>
struct PhaseLauncher {
  static void run(const PhaseArgs& a, int nb, hipStream_t st) {
    const int P = std::min(a.split, split_max<KP>());
    if (a.side.part_mode == 0 && P > 1) {
      // few slices: one workgroup of P wavefronts per slice (grid in slices, not rows)
      PhaseArgs b = a;
      b.side_blocks = a.side.nint / kSlice;
      b.gen_blocks = a.gen_blocks > 0 ? ceil_div(a.gen.nblocks, (int64_t)kSlice * P) : 0;
      const dim3 grid((unsigned)(b.side_blocks + b.gen_blocks)), block((unsigned)(kSlice * P));
      if (a.side.tgt || a.side.zout) k_phase_split<KP, PACKED, true><<<grid, block, 0, st>>>(b, P);
      else k_phase_split<KP, PACKED, false><<<grid, block, 0, st>>>(b, P);
    } else if (a.side.tgt || a.side.zout) {
      k_phase_var<KP, PACKED><<<dim3((unsigned)(a.side_blocks + a.gen_blocks)), dim3(kBlock), 0, st>>>(a);
    } else if (nb <= 1) {
      launch_phase<KP, PACKED, 1>(a, st);
    } else if (nb <= 2) {
      launch_phase<KP, PACKED, 2>(a, st);
    } else if (nb <= 4) {
      launch_phase<KP, PACKED, 4>(a, st);
    } else if constexpr (KP <= 16) {
      if (nb >= 16) launch_phase<KP, PACKED, 16>(a, st);
      else launch_phase<KP, PACKED, 8>(a, st);
    } else {
      launch_phase<KP, PACKED, 8>(a, st);
    }
  }
};

template <int KP, bool PACKED>
struct BothLauncher {
  // threads: workgroup size of the plain kernel (256, 512 or 1024, at most
  // step_max_threads; 256 for the Section 6 variant kernel); the row and sign-word block
  // counts of a0 are for kBlock-thread workgroups and are recomputed here, with the
  // column block count.
  static void run(const PhaseArgs& a0, const SideDev& C, int nb, int threads, hipStream_t st) {
    const bool var = a0.side.tgt || a0.side.zout || C.tgt || C.zout;
    int wg = kBlock;
    if (!var) {
      const int cap = nb <= 1 ? step_max_threads<KP, 1, PACKED>() : step_max_threads<KP, 2, PACKED>();
      wg = std::min(threads, cap);
    }
    PhaseArgs a = a0;
    a.side_blocks = ceil_div(a0.side.nint, wg);
    a.gen_blocks = a0.gen_blocks > 0 ? ceil_div(a0.gen.nblocks, wg) : 0;
    const int64_t col_blocks = ceil_div(C.nint, wg);
    const dim3 grid((unsigned)(a.side_blocks + col_blocks + a.gen_blocks)), block((unsigned)wg);
    if (var) {
      k_phase_both_var<KP, PACKED><<<grid, block, 0, st>>>(a, C, col_blocks);
    } else if (nb <= 1) {
      k_phase_both<KP, PACKED, 1><<<grid, block, 0, st>>>(a, C, col_blocks);
    } else if (nb <= 2) {
      k_phase_both<KP, PACKED, 2><<<grid, block, 0, st>>>(a, C, col_blocks);
    } else if (nb <= 4) {
      k_phase_both<KP, PACKED, 4><<<grid, block, 0, st>>>(a, C, col_blocks);
    } else if constexpr (KP <= 16) {
      if (nb >= 16) k_phase_both<KP, PACKED, 16><<<grid, block, 0, st>>>(a, C, col_blocks);
      else k_phase_both<KP, PACKED, 8><<<grid, block, 0, st>>>(a, C, col_blocks);
    } else {
      k_phase_both<KP, PACKED, 8><<<grid, block, 0, st>>>(a, C, col_blocks);
    }
  }
};

template <int KP, bool PACKED>
struct BlockLauncher {
  static void run(const SideDev& S, const BlockDev& B, int k, const StepScalars& sc, int64_t wbase,
                  const double* x0, int init, int* flag, hipStream_t st) {
    k_block_step<KP, PACKED><<<dim3(block_grid(B.nb, B.group)), dim3(256), 0, st>>>(S, B, k, sc, wbase, x0,
                                                                                       init, flag);
  }
};

template <int KP, bool PACKED>
struct BlockBothLauncher {
  static void run(const SideDev& S0, const BlockDev& B0, const StepScalars& sc0, int64_t wbase0, const SideDev& S1,
                  const BlockDev& B1, const StepScalars& sc1, int64_t wbase1, int k, int* flag, hipStream_t st) {
    const unsigned g0 = block_grid(B0.nb, B0.group), g1 = block_grid(B1.nb, B1.group);
    k_block_step_both<KP, PACKED><<<dim3(g0 + g1), dim3(256), 0, st>>>(S0, B0, sc0, wbase0, S1, B1, sc1, wbase1, k,
                                                                        (int64_t)g0, flag);
  }
};

template <int KP, bool PACKED>
struct InitLauncher {
  static void run(const SideDev& S, const MatDev* mats, const double* x0, int k, double M, int* flag,
                  hipStream_t st) {
    launch_init<KP, PACKED>(S, mats, x0, k, M, flag, st);
  }
};

}  // namespace

int ensure_mats(mfe_plan* p, hipStream_t st) {
  if (p->mats) return MFE_OK;
  MFE_CHECK(ensure(&p->mats, p->count));
  std::vector<MatDev> md(p->count);
  int64_t ro = 0, co = 0;
  for (int b = 0; b < p->count; ++b) {
    md[b] = MatDev{};
    md[b].row_orig_base = ro;
    md[b].col_orig_base = co;
    ro += p->meta[b].m;
    co += p->meta[b].n;
  }
  MFE_HIP(hipMemcpyAsync(p->mats, md.data(), sizeof(MatDev) * p->count, hipMemcpyHostToDevice, st));
  return MFE_OK;
}

int launch_signgen(const SignGenDev& g, hipStream_t st) {
  if (g.nblocks <= 0) return MFE_OK;
  k_signgen<<<dim3((unsigned)ceil_div(g.nblocks, kBlock)), dim3(kBlock), 0, st>>>(g);
  MFE_HIP(hipGetLastError());
  return MFE_OK;
}

int plan_run(mfe_plan* p, const mfe_equil_params* prm, const double* alpha_b, const double* beta_b,
             int use_graph, double* d, double* e, double* u_bar, double* v_bar, int trace_every,
             int (*on_chunk)(void* ctx, int t), void* ctx) {
  hipStream_t st = (hipStream_t)prm->stream;
  const int k = prm->probes;
  if (k < 1 || k > p->max_probes)
    return set_error(MFE_EINVAL, "probes = %d outside 1..%d (the plan's max_probes)", k, p->max_probes);
  if (!d || !e) return set_error(MFE_EINVAL, "outputs d and e are required");
  const int64_t nr = p->rows.nint, nc = p->cols.nint;
  MFE_CHECK(ensure(&p->x_row, nr));
  MFE_CHECK(ensure(&p->xbar_row, nr));
  MFE_CHECK(ensure(&p->x_col, nc));
  MFE_CHECK(ensure(&p->xbar_col, nc));
  for (int i = 0; i < 2; ++i) {
    MFE_CHECK(ensure(&p->desc_row[i], nr));
    MFE_CHECK(ensure(&p->desc_col[i], nc));
  }
  MFE_CHECK(ensure(&p->flag, 1));
  MFE_CHECK(ensure(&p->mats, p->count));
  if ((int64_t)prm->batch + p->count > ((int64_t)1 << 30))
    return set_error(MFE_EINVAL, "batch + count exceeds 2^30");
  MFE_CHECK(build_sign_layout(p, k, prm->batch));

  // per-matrix targets and sign offsets
  std::vector<MatDev> md(p->count);
  int64_t ro = 0, co = 0;
  for (int b = 0; b < p->count; ++b) {
    const double al = alpha_b ? alpha_b[b] : prm->alpha;
    const double be = beta_b ? beta_b[b] : prm->beta;
    if (!(al > 0) || !(be > 0) || !std::isfinite(al) || !std::isfinite(be))
      return set_error(MFE_EINVAL, "matrix %d: alpha and beta must be positive and finite", b);
    md[b].tgt_row = al * al;
    md[b].tgt_col = be * be;
    md[b].row_orig_base = ro;
    md[b].col_orig_base = co;
    md[b].sign_word_col = p->segs_host[b].word_off;              // side 0
    md[b].sign_word_row = p->segs_host[p->count + b].word_off;   // side 1
    // Algorithm 2 draws one probe block s, indexed like the columns (side 0)
    if (p->symmetric) md[b].sign_word_row = md[b].sign_word_col;
    ro += p->meta[b].m;
    co += p->meta[b].n;
  }
  MFE_HIP(hipMemcpyAsync(p->mats, md.data(), sizeof(MatDev) * p->count, hipMemcpyHostToDevice, st));
  MFE_HIP(hipMemsetAsync(p->flag, 0, sizeof(int), st));

  // Block sides: targets of this run (sums of the indices' squared targets), state.
  const bool blocked[2] = {p->blk[0].nb > 0, p->blk[1].nb > 0};
  BlockDev bd[2];
  for (int i = 0; i < 2; ++i) {
    if (!blocked[i]) continue;
    mfe_plan::BlockSide& bs = p->blk[i];
    const SideLayout& L = i == 0 ? p->rows : p->cols;
    MFE_CHECK(ensure(&bs.tgt, bs.nb));
    MFE_CHECK(ensure(&bs.bx, bs.nb));
    MFE_CHECK(ensure(&bs.bxbar, bs.nb));
    MFE_CHECK(ensure(&bs.z, L.nint));
    const double t2 = i == 0 ? md[0].tgt_row : md[0].tgt_col;
    k_block_targets<<<dim3(block_grid(bs.nb, bs.group)), dim3(256), 0, st>>>(bs.ptr, bs.nb, bs.group,
                                                                               p->tgt_orig[i], t2, bs.tgt);
    MFE_HIP(hipGetLastError());
    bd[i].ptr = bs.ptr;
    bd[i].nb = bs.nb;
    bd[i].orig2int = L.orig2int;
    bd[i].tgt = bs.tgt;
    bd[i].bx = bs.bx;
    bd[i].bxbar = bs.bxbar;
    bd[i].z = bs.z;
    bd[i].group = bs.group;
  }
  const int64_t wbase[2] = {md[0].sign_word_row, md[0].sign_word_col};

  const uint64_t seed = prm->seed;
  const int T = prm->steps;
  // 8-byte descriptors whenever k <= 16 and the box keeps e^x inside the packed range
  const bool packed = k <= 16 && prm->box_M <= 11.0;
  // signs of step 1 -> slot 1, of step 2 -> slot 0
  MFE_CHECK(launch_signgen(make_gen(p, seed, 1, p->signs[1]), st));
  MFE_CHECK(launch_signgen(make_gen(p, seed, 2, p->signs[0]), st));
  {
    SideDev R = make_side(p->rows, p->x_row, p->xbar_row, nullptr, p->desc_row[0], p->signs[1], 1);
    SideDev C = make_side(p->cols, p->x_col, p->xbar_col, nullptr, p->desc_col[0], p->signs[1], 0);
    StepScalars sc0{};
    sc0.M = prm->box_M;
    if (blocked[0])
      dispatch<BlockLauncher>(k, packed, R, bd[0], k, sc0, wbase[0], prm->u0, 1, p->flag, st);
    else
      dispatch<InitLauncher>(k, packed, R, (const MatDev*)p->mats, prm->u0, k, prm->box_M, p->flag, st);
    if (blocked[1])
      dispatch<BlockLauncher>(k, packed, C, bd[1], k, sc0, wbase[1], prm->v0, 1, p->flag, st);
    else if (!p->symmetric)
      dispatch<InitLauncher>(k, packed, C, (const MatDev*)p->mats, prm->v0, k, prm->box_M, p->flag, st);
    MFE_HIP(hipGetLastError());
  }

  // Step t (Jacobi order: both directions read the descriptors of step t-1): by default
  // one launch holding the row direction (plus the sign words of step t+2) and the
  // column direction; otherwise, as the plan's tuning says, one launch per direction, and
  // a direction with a two-part layout as two launches, each gathering from one half of
  // its table.
  // (Symmetric plans gather with their own entries, which have no two-part layout.)
  const int split_rows = p->rows.len_lo && !p->symmetric && p->tune_split[0] == 1 ? 1 : 0;  // 1: two launches
  const int split_cols = p->cols.len_lo && p->tune_split[1] == 1 ? 1 : 0;
  const int nb = p->tune_batch;
  const int nt = stream_hints(p);
  int sched = 1;  // slice order (slice_schedule), set below
  const int32_t wg_threads = p->tune_wg > 0 ? p->tune_wg : kBlock;  // one-launch step workgroups
  for (int i = 0; i < 2; ++i) {
    const bool need = (i == 0 ? split_rows : split_cols) != 0;
    if (need && !p->part[i]) {
      const int64_t n = (i == 0 ? p->rows.nint : p->cols.nint) * (int64_t)p->max_probes;
      MFE_CHECK(ensure(&p->part[i], n));
    }
  }
  auto phase_args = [&](int t, bool rows, int mode) {
    PhaseArgs a;
    const int par = t & 1, prev = par ^ 1;
    if (rows && p->symmetric) {
      // Algorithm 2: D A D s, the row entries gathering the rows' own descriptors
      a.side = make_side(p->rows, p->x_row, p->xbar_row, p->desc_row[prev], p->desc_row[par],
                         p->signs[(t + 1) & 1], 1);
      a.side.ent = p->ent_sym;
    } else if (rows) {
      a.side = make_side(p->rows, p->x_row, p->xbar_row, p->desc_col[prev], p->desc_row[par],
                         p->signs[(t + 1) & 1], 1);
    } else {
      a.side = make_side(p->cols, p->x_col, p->xbar_col, p->desc_row[prev], p->desc_col[par],
                         p->signs[(t + 1) & 1], 0);
    }
    a.side.part_mode = mode;
    a.side.part = p->part[rows ? 0 : 1];
    a.side.nt = nt;
    if (!sched) a.side.sched = nullptr;
    const int si = rows ? 0 : 1;
    if (blocked[si]) a.side.zout = p->blk[si].z;
    else a.side.tgt = p->tgt_int[si];
    const uint64_t gen_step = (uint64_t)t + 2;
    const bool gen = rows && mode != 2 && (int64_t)gen_step <= (int64_t)T + 1;
    a.gen = make_gen(p, seed, gen_step, p->signs[t & 1]);
    a.mats = p->mats;
    a.k = k;
    const double tau = (double)t + (double)prm->t0;
    a.sc.tau = tau;
    a.sc.eta = 2.0 / (prm->gamma * (tau + 1.0));
    a.sc.gamma = prm->gamma;
    a.sc.M = prm->box_M;
    a.side_blocks = ceil_div(rows ? nr : nc, kBlock);
    a.gen_blocks = gen ? ceil_div(p->sign_blocks, kBlock) : 0;
    a.flag = p->flag;
    // few slices (rows of a small matrix, or long rows): several wavefronts per slice,
    // so that about 2048 slices' worth of wavefronts are in flight
    const int64_t ns = (rows ? p->rows.nslices : p->cols.nslices);
    a.split = mode == 0 ? (int)std::max<int64_t>(1, std::min<int64_t>(16, 2048 / std::max<int64_t>(ns, 1))) : 1;
    return a;
  };
  // A block side adds one launch after its direction: the block sums, steps and the
  // descriptors of the block's indices (which the other direction reads at step t+1).
  // Both directions in one launch (tuning modes 2 / 2) where neither needs another form;
  // block sides then run their block launches after it.
  const bool fused = p->tune_split[0] == 2 && p->tune_split[1] == 2 && !p->symmetric;
  {
    // the launch shapes phase_args chooses: split kernels below 1024 slices
    const bool split = p->rows.nslices < 1024 || (!p->symmetric && p->cols.nslices < 1024);
    sched = slice_schedule(p, ceil_div(nr, kBlock), p->symmetric ? 0 : ceil_div(nc, kBlock), split);
  }
  auto launch_step = [&](int t, hipStream_t s) {
    if (fused) {
      const PhaseArgs a = phase_args(t, true, 0), c = phase_args(t, false, 0);
      if (a.split <= 1 && c.split <= 1) {
        dispatch<BothLauncher>(k, packed, a, c.side, nb, (int)wg_threads, s);
        if (blocked[0] && blocked[1]) {
          dispatch<BlockBothLauncher>(k, packed, a.side, bd[0], a.sc, wbase[0], c.side, bd[1], c.sc, wbase[1], k,
                                      p->flag, s);
          return;
        }
        for (int si = 0; si < 2; ++si)
          if (blocked[si]) {
            const PhaseArgs& x = si == 0 ? a : c;
            dispatch<BlockLauncher>(k, packed, x.side, bd[si], k, x.sc, wbase[si], nullptr, 0, p->flag, s);
          }
        return;
      }
    }
    for (const bool rows : {true, false}) {
      if (!rows && p->symmetric) break;
      if (rows ? split_rows : split_cols) {
        dispatch<PhaseLauncher>(k, packed, phase_args(t, rows, 1), nb, s);
        dispatch<PhaseLauncher>(k, packed, phase_args(t, rows, 2), nb, s);
      } else {
        dispatch<PhaseLauncher>(k, packed, phase_args(t, rows, 0), nb, s);
      }
      const int si = rows ? 0 : 1;
      if (blocked[si]) {
        const PhaseArgs a = phase_args(t, rows, 0);
        dispatch<BlockLauncher>(k, packed, a.side, bd[si], k, a.sc, wbase[si], nullptr, 0, p->flag, s);
      }
    }
  };
  auto launch_steps = [&](hipStream_t s) {
    for (int t = 1; t <= T; ++t) launch_step(t, s);
  };

  // The step loop runs either as 2T (or more) launches or as one cached HIP graph of
  // those launches (captured once per (k, T, t0, gamma, M, seed, batch, tuning, hints,
  // slice order, workgroup size)).
  hipStream_t run_st = st;
  if (use_graph && T > 0) {
    const double key[15] = {(double)k, (double)T, (double)prm->t0, prm->gamma, prm->box_M,
                            (double)(seed >> 32), (double)(seed & 0xFFFFFFFFull), (double)prm->batch,
                            (double)nb, (double)p->tune_split[0], (double)p->tune_split[1],
                            (double)p->variant_epoch, (double)nt, (double)sched, (double)wg_threads};
    bool hit = p->graph_exec != nullptr;
    for (int i = 0; i < 15 && hit; ++i) hit = (key[i] == p->graph_key[i]);
    if (!p->cap_stream) MFE_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    if (!hit) {
      if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
      if (p->graph) (void)hipGraphDestroy(p->graph);
      p->graph_exec = nullptr;
      p->graph = nullptr;
      MFE_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
      launch_steps(p->cap_stream);
      MFE_HIP(hipStreamEndCapture(p->cap_stream, &p->graph));
      MFE_HIP(hipGraphInstantiate(&p->graph_exec, p->graph, nullptr, nullptr, 0));
      for (int i = 0; i < 15; ++i) p->graph_key[i] = key[i];
    }
    if (st == nullptr) {
      // graphs are replayed on the plan's own stream, ordered after the default stream
      MFE_HIP(hipStreamSynchronize(nullptr));
      run_st = p->cap_stream;
    }
    MFE_HIP(hipEventRecord(p->ev0, run_st));
    MFE_HIP(hipGraphLaunch(p->graph_exec, run_st));
    MFE_HIP(hipEventRecord(p->ev1, run_st));
  } else if (trace_every > 0) {
    // chunks of steps with the caller's evaluation in between; only step time is summed
    double total_ms = 0.0;
    for (int t0 = 1; t0 <= T; t0 += trace_every) {
      const int t1 = std::min(T, t0 + trace_every - 1);
      MFE_HIP(hipEventRecord(p->ev0, run_st));
      for (int t = t0; t <= t1; ++t) launch_step(t, run_st);
      MFE_HIP(hipGetLastError());
      MFE_HIP(hipEventRecord(p->ev1, run_st));
      MFE_HIP(hipEventSynchronize(p->ev1));
      float ms = 0.f;
      MFE_HIP(hipEventElapsedTime(&ms, p->ev0, p->ev1));
      total_ms += ms;
      if (on_chunk) MFE_CHECK(on_chunk(ctx, t1));
    }
    p->last_loop_ms = total_ms;
    p->last_step_ms = T > 0 ? total_ms / T : 0.0;
  } else {
    MFE_HIP(hipEventRecord(p->ev0, run_st));
    launch_steps(run_st);
    MFE_HIP(hipGetLastError());
    MFE_HIP(hipEventRecord(p->ev1, run_st));
  }
  {
    const int par = T & 1;
    SideDev R = make_side(p->rows, p->x_row, p->xbar_row, nullptr, p->desc_row[par], nullptr, 1);
    SideDev C = make_side(p->cols, p->x_col, p->xbar_col, nullptr, p->desc_col[par], nullptr, 0);
    if (blocked[0]) k_block_output<<<dim3(block_grid(bd[0].nb, bd[0].group)), dim3(256), 0, run_st>>>(bd[0], d, u_bar);
    else k_output<<<dim3((unsigned)ceil_div(nr, 256)), dim3(256), 0, run_st>>>(R, p->mats, d, u_bar);
    if (blocked[1]) k_block_output<<<dim3(block_grid(bd[1].nb, bd[1].group)), dim3(256), 0, run_st>>>(bd[1], e, v_bar);
    else if (p->symmetric) k_output<<<dim3((unsigned)ceil_div(nr, 256)), dim3(256), 0, run_st>>>(R, p->mats, e, v_bar);
    else k_output<<<dim3((unsigned)ceil_div(nc, 256)), dim3(256), 0, run_st>>>(C, p->mats, e, v_bar);
    MFE_HIP(hipGetLastError());
  }
  int flag = 0;
  MFE_HIP(hipMemcpyAsync(&flag, p->flag, sizeof(int), hipMemcpyDeviceToHost, run_st));
  MFE_HIP(hipStreamSynchronize(run_st));
  if (trace_every <= 0 || use_graph) {
    float ms = 0.f;
    MFE_HIP(hipEventElapsedTime(&ms, p->ev0, p->ev1));
    p->last_loop_ms = ms;
    p->last_step_ms = T > 0 ? ms / T : 0.0;
  }
  if (flag & 2) return set_error(MFE_EINVAL, "warm start u0/v0 outside the box [-M, M] (or NaN)");
  if (flag & 1) return set_error(MFE_ENONFINITE, "non-finite gradient estimate or iterate (NaN/Inf in A?)");
  return MFE_OK;
}

}  // namespace mfe

namespace mfe {

int plan_autotune(mfe_plan* p, const mfe_equil_params* prm, const double* alpha_b, const double* beta_b,
                  int32_t trial_steps, int32_t* chosen, double* best_step_ms, int32_t* n_candidates) {
  if (trial_steps < 1 || trial_steps > 100000) return set_error(MFE_EINVAL, "trial_steps must be in 1..100000");
  const int k = prm->probes;
  if (k < 1 || k > p->max_probes)
    return set_error(MFE_EINVAL, "probes = %d outside 1..%d (the plan's max_probes)", k, p->max_probes);
  struct Cand {
    int nb, sr, sc, nt, sched, wg;
  };
  // The default configuration is timed first and kept unless another is more than 1%
  // faster, so the choice does not flip on timing noise.
  std::vector<Cand> cands;
  std::vector<int> nbs{kBatch};
  for (int nb : {1, 2, 4, 8, 16})
    if (nb != kBatch) nbs.push_back(nb);
  // Stream hints: the plan's size-based default for every form, and the other setting for
  // the one-launch form.
  // Slice order: the default rule (-1) for every form, and both fixed orders for the
  // one-launch form.
  const int32_t keep_nt = p->tune_nt, keep_sched = p->tune_sched, keep_wg = p->tune_wg;
  p->tune_nt = -1;
  const int nt0 = stream_hints(p);
  p->tune_nt = keep_nt;
  for (int nb : nbs) {
    if (nb == 16 && k > 16) continue;
    cands.push_back({nb, 2, 2, nt0, -1, 0});  // both directions in one launch
    for (int sr = 0; sr <= (p->rows.len_lo ? 1 : 0); ++sr)
      for (int sc = 0; sc <= (p->cols.len_lo ? 1 : 0); ++sc) cands.push_back({nb, sr, sc, nt0, -1, 0});
    cands.push_back({nb, 2, 2, 1 - nt0, -1, 0});
    cands.push_back({nb, 2, 2, nt0, 0, 0});
    cands.push_back({nb, 2, 2, nt0, 1, 0});
    if (k <= 16) cands.push_back({nb, 2, 2, nt0, -1, 512});  // larger workgroups of the one-launch kernel
    if (k <= 8) cands.push_back({nb, 2, 2, nt0, -1, 1024});
  }
  double *d = nullptr, *e = nullptr;
  MFE_CHECK(ensure(&d, p->M));
  struct Free {
    double*& a;
    double*& b;
    ~Free() {
      (void)hipFree(a);
      (void)hipFree(b);
    }
  } fr{d, e};
  MFE_CHECK(ensure(&e, p->N));
  mfe_equil_params trial = *prm;
  trial.steps = trial_steps;
  const int32_t keep_batch = p->tune_batch, keep_sr = p->tune_split[0], keep_sc = p->tune_split[1];
  double best = 0.0;
  int best_i = -1;
  for (size_t i = 0; i < cands.size(); ++i) {
    p->tune_batch = cands[i].nb;
    p->tune_split[0] = cands[i].sr;
    p->tune_split[1] = cands[i].sc;
    p->tune_nt = cands[i].nt;
    p->tune_sched = cands[i].sched;
    p->tune_wg = cands[i].wg;
    double t = 0.0;
    for (int rep = 0; rep < 2; ++rep) {  // the first run warms caches and code objects
      const int rc = plan_run(p, &trial, alpha_b, beta_b, 0, d, e, nullptr, nullptr);
      if (rc != MFE_OK) {
        p->tune_batch = keep_batch;
        p->tune_split[0] = keep_sr;
        p->tune_split[1] = keep_sc;
        p->tune_nt = keep_nt;
        p->tune_sched = keep_sched;
        p->tune_wg = keep_wg;
        return rc;
      }
      t = p->last_step_ms;
    }
    if (best_i < 0 || t < 0.99 * best) {
      best = t;
      best_i = (int)i;
    }
  }
  p->tune_batch = cands[best_i].nb;
  p->tune_split[0] = cands[best_i].sr;
  p->tune_split[1] = cands[best_i].sc;
  p->tune_nt = cands[best_i].nt;
  p->tune_sched = cands[best_i].sched;
  p->tune_wg = cands[best_i].wg;
  if (chosen) {
    chosen[0] = p->tune_batch;
    chosen[1] = p->tune_split[0];
    chosen[2] = p->tune_split[1];
    chosen[3] = p->tune_nt;
    chosen[4] = p->tune_sched;
    chosen[5] = p->tune_wg > 0 ? p->tune_wg : kBlock;
  }
  if (best_step_ms) *best_step_ms = best;
  if (n_candidates) *n_candidates = (int32_t)cands.size();
  return MFE_OK;
}

}  // namespace mfe
