// Shared host/device definitions of libmfe (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/mfe.h"

namespace mfe {

// ----------------------------------------------------------------- errors

// Records a message for mfe_last_error() and returns the status.
int set_error(int status, const char* fmt, ...);
void clear_error();
// Step-loop timing of the last equilibration on this thread (HIP events on its stream).
void record_timing(double loop_ms, double step_ms);
void set_warning(const char* fmt, ...);

#define MFE_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t _e = (call);                                                             \
    if (_e != hipSuccess)                                                               \
      return ::mfe::set_error(_e == hipErrorOutOfMemory ? MFE_ENOMEM : MFE_EDEVICE,     \
                              "%s failed: %s (%s:%d)", #call, hipGetErrorString(_e),    \
                              __FILE__, __LINE__);                                      \
  } while (0)

#define MFE_CHECK(status_expr)        \
  do {                                \
    int _s = (status_expr);           \
    if (_s != MFE_OK) return _s;      \
  } while (0)

// Per-step scalars, computed on the host exactly as the oracle writes them.
struct StepScalars {
  double eta;   // 2 / (gamma (tau + 1))
  double tau;   // t + t0
  double gamma;
  double M;
};
using StepScalarsFwd = StepScalars;

// ----------------------------------------------------------------- probe signs
//
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).  One block = 4 x 64 bits for a
// counter (c+1, 0, 0, 0) and key (seed, ctrl).  The stream bit layout is documented in
// mfe.h.

struct U64x4 {
  uint64_t x[4];
};

__host__ __device__ inline uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

__host__ __device__ inline U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = mulhi64(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = mulhi64(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  U64x4 o;
  o.x[0] = c0;
  o.x[1] = c1;
  o.x[2] = c2;
  o.x[3] = c3;
  return o;
}

__host__ __device__ inline uint64_t stream_ctrl(uint64_t batch, uint64_t step, uint64_t side) {
  return (batch << 34) | (step << 2) | side;
}

// k (<= 64) bits starting at bit g of a word array.
__device__ inline uint64_t extract_bits(const uint64_t* __restrict__ words, int64_t g, int k) {
  const int64_t w = g >> 6;
  const int sh = (int)(g & 63);
  uint64_t v = words[w] >> sh;
  if (sh + k > 64) v |= words[w + 1] << (64 - sh);
  return k == 64 ? v : (v & ((1ull << k) - 1ull));
}

// acc_p += (-1)^bit_p * t for p < KP.  The sign of t is folded into the probe bits so
// each probe costs one shift, one and-or on the high word and one FP64 add.
template <int KP>
__device__ __forceinline__ void accumulate_signed(double (&acc)[KP], double t, uint64_t bits) {
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

// Projected step of Algorithm 1 for one index: z = e^(2x) * (sum of squares / k),
// x <- clip(x - eta (z - target + gamma x), -M, M), average update with weight tau.
// Returns false if z or the new iterate is not finite.
__device__ __forceinline__ bool sgd_update(double ss, int k, double target, const StepScalarsFwd& sc,
                                           double& x, double& xbar) {
  const double x_old = x;
  const double z = exp(2.0 * x_old) * (ss / (double)k);
  const double g = (z - target) + sc.gamma * x_old;
  double xn = x_old - sc.eta * g;
  xn = fmin(fmax(xn, -sc.M), sc.M);
  const bool ok = isfinite(z) && isfinite(xn);
  if (!ok) xn = 0.0;
  x = xn;
  xbar = 2.0 * xn / (sc.tau + 2.0) + sc.tau * xbar / (sc.tau + 2.0);
  return ok;
}

// Sum of a double over the 64 lanes of a wavefront, returned to every lane.  Data
// parallel primitives (DPP) add within quads, half rows and rows of 16 lanes on the
// vector ALU; the four row sums are then read as wavefront-uniform values.  Must be
// called with all 64 lanes active.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double read_lane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1, 0, 3, 2]: pairs
  v += dpp_mov<0x4E>(v);   // quad_perm [2, 3, 0, 1]: quads
  v += dpp_mov<0x141>(v);  // row_half_mirror: groups of 8
  v += dpp_mov<0x140>(v);  // row_mirror: rows of 16
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Gathered per-index record of the sparse path: the scale e^x of the index (FP64) and
// the sign bits of its probes for the step that consumes it.
struct __align__(16) Desc {
  double scale;
  uint64_t bits;
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }


}  // namespace mfe
