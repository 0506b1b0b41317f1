// Measurement probes for the ceilings the sparse engine's step is compared against.
//
// Every product of Algorithm 1 (Section 3.2) on a sparse matrix needs, per stored entry,
// one random 8-byte read of the other side's descriptor table, so the step is bounded by
// two rates of the memory system rather than by the HBM peak alone:
//   * the rate of random 8-byte gathers from a table of a given size (which decides how
//     much of it the L2 of each XCD holds), and
//   * the rate of a plain streaming read (the entry streams).
// These kernels measure both in isolation: the gather probe reads hashed indices (no
// index stream) with 1, 2, 4 or 8 gathers in flight per lane; the sorted gather probe
// gives each thread the L indices of one row of a uniformly random sparse matrix, in
// increasing order, gathered one at a time (the step's pattern: a lane walks one row's
// sorted entries, so the lanes at the same slot gather from the same part of the table);
// the stream probe reads a buffer once with 16-byte non-temporal loads.  All fold what
// they read into one word per thread so nothing is optimised away.
#include "common.h"

namespace mfe {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kProbeThreads = 256;

// 64-bit finaliser of MurmurHash3 (Appleby): a bijective mix, used to spread indices.
__device__ inline uint64_t mix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

__global__ void k_fill_table(uint64_t* __restrict__ t, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] = mix64((uint64_t)i + 1);
}

// Thread g performs gathers g, g + G, g + 2G, ... (G = grid size) below `total`, in
// batches of B independent loads.
template <int B>
__global__ __launch_bounds__(kProbeThreads) void k_gather_probe(const uint64_t* __restrict__ table, int64_t n,
                                                                int64_t total, uint64_t salt,
                                                                uint64_t* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t G = (int64_t)gridDim.x * blockDim.x;
  uint64_t acc = 0;
  for (int64_t q0 = g; q0 < total; q0 += G * B) {
    uint64_t v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int64_t q = q0 + (int64_t)u * G;
      v[u] = q < total ? table[mix64((uint64_t)q ^ salt) % (uint64_t)n] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < B; ++u) acc ^= v[u];
  }
  out[g] = acc;
}

void launch_gather_probe(int in_flight, int blocks, const uint64_t* table, int64_t n, int64_t total, uint64_t salt,
                         uint64_t* out, hipStream_t st) {
  switch (in_flight) {
    case 1: k_gather_probe<1><<<blocks, kProbeThreads, 0, st>>>(table, n, total, salt, out); break;
    case 2: k_gather_probe<2><<<blocks, kProbeThreads, 0, st>>>(table, n, total, salt, out); break;
    case 4: k_gather_probe<4><<<blocks, kProbeThreads, 0, st>>>(table, n, total, salt, out); break;
    default: k_gather_probe<8><<<blocks, kProbeThreads, 0, st>>>(table, n, total, salt, out); break;
  }
}

// Thread g gathers the L hashed indices of "row" g (row g < rows), sorted increasing, one
// at a time: each index depends on the value gathered before it (plus a term that is
// almost surely zero, the sum clamped into the table) so the loads cannot overlap.
template <int L>
__global__ __launch_bounds__(kProbeThreads) void k_gather_sorted(const uint64_t* __restrict__ table, uint32_t n,
                                                                 int64_t rows, uint64_t salt,
                                                                 uint64_t* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= rows) return;
  uint32_t idx[L];
#pragma unroll
  for (int q = 0; q < L; ++q) idx[q] = (uint32_t)(mix64(((uint64_t)g * L + q) ^ salt) % n);
#pragma unroll
  for (int i = 0; i < L; ++i)
#pragma unroll
    for (int j = 0; j < L - 1 - i; ++j) {
      const uint32_t a = idx[j], b = idx[j + 1];
      idx[j] = a < b ? a : b;
      idx[j + 1] = a < b ? b : a;
    }
  uint64_t acc = 0;
#pragma unroll
  for (int q = 0; q < L; ++q) {
    const uint32_t j = min(idx[q] + (uint32_t)(acc == 0x5bd1e9955bd1e995ull), n - 1u);
    acc += table[j] * (uint64_t)(q + 1);
  }
  out[g] = acc;
}

void launch_gather_sorted(int L, const uint64_t* table, uint32_t n, int64_t rows, uint64_t salt, uint64_t* out,
                          hipStream_t st) {
  const unsigned blocks = (unsigned)ceil_div(rows, kProbeThreads);
  switch (L) {
    case 5: k_gather_sorted<5><<<blocks, kProbeThreads, 0, st>>>(table, n, rows, salt, out); break;
    case 10: k_gather_sorted<10><<<blocks, kProbeThreads, 0, st>>>(table, n, rows, salt, out); break;
    case 20: k_gather_sorted<20><<<blocks, kProbeThreads, 0, st>>>(table, n, rows, salt, out); break;
    default: k_gather_sorted<40><<<blocks, kProbeThreads, 0, st>>>(table, n, rows, salt, out); break;
  }
}

__global__ __launch_bounds__(kProbeThreads) void k_stream_probe(const u32x4* __restrict__ buf, int64_t n16,
                                                                uint32_t* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t G = (int64_t)gridDim.x * blockDim.x;
  uint32_t acc = 0;
  int64_t i = g;
  for (; i + 3 * G < n16; i += 4 * G) {
    const u32x4 a = __builtin_nontemporal_load(buf + i);
    const u32x4 b = __builtin_nontemporal_load(buf + i + G);
    const u32x4 c = __builtin_nontemporal_load(buf + i + 2 * G);
    const u32x4 d = __builtin_nontemporal_load(buf + i + 3 * G);
    acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
  }
  for (; i < n16; i += G) {
    const u32x4 a = __builtin_nontemporal_load(buf + i);
    acc ^= a.x ^ a.y ^ a.z ^ a.w;
  }
  out[g] = acc;
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

}  // namespace

int probe_gather(int64_t table_bytes, int64_t gathers, int32_t in_flight, int32_t reps, double* ms, hipStream_t st) {
  const int64_t n = table_bytes / 8;
  const int blocks = 2048;
  DevBuf tab, out;
  MFE_HIP(hipMalloc(&tab.p, sizeof(uint64_t) * (size_t)n));
  MFE_HIP(hipMalloc(&out.p, sizeof(uint64_t) * (size_t)blocks * kProbeThreads));
  k_fill_table<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>((uint64_t*)tab.p, n);
  EventPair ev;
  MFE_HIP(hipEventCreate(&ev.a));
  MFE_HIP(hipEventCreate(&ev.b));
  // one untimed launch warms the table into the caches, as the step's tables are
  launch_gather_probe(in_flight, blocks, (const uint64_t*)tab.p, n, gathers, 0, (uint64_t*)out.p, st);
  MFE_HIP(hipEventRecord(ev.a, st));
  for (int r = 0; r < reps; ++r)
    launch_gather_probe(in_flight, blocks, (const uint64_t*)tab.p, n, gathers, (uint64_t)r + 1, (uint64_t*)out.p, st);
  MFE_HIP(hipGetLastError());
  MFE_HIP(hipEventRecord(ev.b, st));
  MFE_HIP(hipEventSynchronize(ev.b));
  float t = 0.f;
  MFE_HIP(hipEventElapsedTime(&t, ev.a, ev.b));
  *ms = (double)t / reps;
  return MFE_OK;
}

int probe_gather_sorted(int64_t table_bytes, int64_t gathers, int32_t per_row, int32_t reps, double* ms,
                        hipStream_t st) {
  const int64_t n = table_bytes / 8;
  const int64_t rows = ceil_div(gathers, per_row);
  DevBuf tab, out;
  MFE_HIP(hipMalloc(&tab.p, sizeof(uint64_t) * (size_t)n));
  MFE_HIP(hipMalloc(&out.p, sizeof(uint64_t) * (size_t)rows));
  k_fill_table<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>((uint64_t*)tab.p, n);
  EventPair ev;
  MFE_HIP(hipEventCreate(&ev.a));
  MFE_HIP(hipEventCreate(&ev.b));
  launch_gather_sorted(per_row, (const uint64_t*)tab.p, (uint32_t)n, rows, 0, (uint64_t*)out.p, st);
  MFE_HIP(hipEventRecord(ev.a, st));
  for (int r = 0; r < reps; ++r)
    launch_gather_sorted(per_row, (const uint64_t*)tab.p, (uint32_t)n, rows, (uint64_t)r + 1, (uint64_t*)out.p, st);
  MFE_HIP(hipGetLastError());
  MFE_HIP(hipEventRecord(ev.b, st));
  MFE_HIP(hipEventSynchronize(ev.b));
  float t = 0.f;
  MFE_HIP(hipEventElapsedTime(&t, ev.a, ev.b));
  *ms = (double)t / reps;
  return MFE_OK;
}

int probe_stream(int64_t bytes, int32_t reps, double* ms, hipStream_t st) {
  const int64_t n16 = bytes / 16;
  const int blocks = 8192;
  DevBuf buf, out;
  MFE_HIP(hipMalloc(&buf.p, (size_t)n16 * 16));
  MFE_HIP(hipMalloc(&out.p, sizeof(uint32_t) * (size_t)blocks * kProbeThreads));
  MFE_HIP(hipMemsetAsync(buf.p, 1, (size_t)n16 * 16, st));
  EventPair ev;
  MFE_HIP(hipEventCreate(&ev.a));
  MFE_HIP(hipEventCreate(&ev.b));
  k_stream_probe<<<blocks, kProbeThreads, 0, st>>>((const u32x4*)buf.p, n16, (uint32_t*)out.p);
  MFE_HIP(hipEventRecord(ev.a, st));
  for (int r = 0; r < reps; ++r)
    k_stream_probe<<<blocks, kProbeThreads, 0, st>>>((const u32x4*)buf.p, n16, (uint32_t*)out.p);
  MFE_HIP(hipGetLastError());
  MFE_HIP(hipEventRecord(ev.b, st));
  MFE_HIP(hipEventSynchronize(ev.b));
  float t = 0.f;
  MFE_HIP(hipEventElapsedTime(&t, ev.a, ev.b));
  *ms = (double)t / reps;
  return MFE_OK;
}

}  // namespace mfe

extern "C" {

int mfe_probe_gather(int64_t table_bytes, int64_t gathers, int32_t in_flight, int32_t reps, double* ms,
                     void* stream) {
  mfe::clear_error();
  if (table_bytes < 8 || gathers < 1 || reps < 1 || !ms)
    return mfe::set_error(MFE_EINVAL, "need table_bytes >= 8, gathers >= 1, reps >= 1 and ms");
  if (in_flight != 1 && in_flight != 2 && in_flight != 4 && in_flight != 8)
    return mfe::set_error(MFE_EINVAL, "in_flight must be 1, 2, 4 or 8");
  return mfe::probe_gather(table_bytes, gathers, in_flight, reps, ms, (hipStream_t)stream);
}

int mfe_probe_gather_sorted(int64_t table_bytes, int64_t gathers, int32_t per_row, int32_t reps, double* ms,
                            void* stream) {
  mfe::clear_error();
  if (table_bytes < 8 || table_bytes > (8ll << 32) - 8 || gathers < 1 || reps < 1 || !ms)
    return mfe::set_error(MFE_EINVAL, "need 8 <= table_bytes < 32 GiB, gathers >= 1, reps >= 1 and ms");
  if (per_row != 5 && per_row != 10 && per_row != 20 && per_row != 40)
    return mfe::set_error(MFE_EINVAL, "per_row must be 5, 10, 20 or 40");
  return mfe::probe_gather_sorted(table_bytes, gathers, per_row, reps, ms, (hipStream_t)stream);
}

int mfe_probe_stream(int64_t bytes, int32_t reps, double* ms, void* stream) {
  mfe::clear_error();
  if (bytes < 16 || reps < 1 || !ms) return mfe::set_error(MFE_EINVAL, "need bytes >= 16, reps >= 1 and ms");
  return mfe::probe_stream(bytes, reps, ms, (hipStream_t)stream);
}

}  // extern "C"
