// Preprocessing of the sparse engine: concatenation of the input CSR matrices, the
// transpose (CSC) by a stable radix sort on column index, and the sliced-ELL layouts of
// both products (see sparse.h).  Runs once per plan; deterministic.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <new>
#include <vector>

#include "sparse.h"

namespace mfe {
namespace {

// Device-side per-matrix bases of one direction.
struct SideMat {
  int64_t orig_base;  // first original index of the matrix
  int64_t int_base;   // first internal index of the matrix
  int64_t win_base;   // first sort window of the matrix
  int64_t count;      // original indices of the matrix
};

struct Buf {
  void* p = nullptr;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
};

template <class T>
int dalloc(T** ptr, int64_t count) {
  *ptr = nullptr;
  if (count <= 0) count = 1;
  hipError_t e = hipMalloc((void**)ptr, sizeof(T) * (size_t)count);
  if (e != hipSuccess)
    return set_error(e == hipErrorOutOfMemory ? MFE_ENOMEM : MFE_EDEVICE,
                     "hipMalloc(%lld bytes) failed: %s", (long long)(sizeof(T) * count),
                     hipGetErrorString(e));
  return MFE_OK;
}

template <class T>
int talloc(Buf& b, T** ptr, int64_t count) {
  MFE_CHECK(dalloc(ptr, count));
  b.p = *ptr;
  return MFE_OK;
}

inline unsigned grid_for(int64_t n, int block = 256) { return (unsigned)std::max<int64_t>(1, ceil_div(n, block)); }

// ------------------------------------------------------------------ kernels

// Checks one input CSR: row_ptr[0] = 0, non-decreasing, row_ptr[m] = nnz, 0 <= col < n,
// columns strictly increasing within a row.  Sets bits of *bad.
__global__ void k_validate_csr(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                               int64_t m, int64_t n, int64_t nnz, int* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > m) return;
  const int32_t a = ptr[i];
  if (i == 0 && a != 0) atomicOr(bad, 1);
  if (i == m) {
    if (a != nnz) atomicOr(bad, 2);
    return;
  }
  const int32_t b = ptr[i + 1];
  if (b < a || a < 0 || b > nnz) {
    atomicOr(bad, 4);
    return;
  }
  for (int32_t q = a; q < b; ++q) {
    const int32_t c = col[q];
    if (c < 0 || c >= n) atomicOr(bad, 8);
    if (q > a && c <= col[q - 1]) atomicOr(bad, 16);
  }
}

__global__ void k_concat_ptr(const int32_t* __restrict__ ptr, int64_t m, int64_t nnz_base,
                             int64_t* __restrict__ gptr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= m) gptr[i] = nnz_base + (int64_t)ptr[i];
}

__global__ void k_concat_col(const int32_t* __restrict__ col, int64_t nnz, int32_t col_base,
                             int32_t* __restrict__ gcol) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nnz) gcol[q] = col_base + col[q];
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_iota(int32_t* __restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (int32_t)i;
}

__global__ void k_row_len(const int64_t* __restrict__ gptr, int64_t M, int32_t* __restrict__ len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) len[i] = (int32_t)(gptr[i + 1] - gptr[i]);
}

__global__ void k_row_ids(const int64_t* __restrict__ gptr, int64_t M, int32_t* __restrict__ rowid) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  for (int64_t q = gptr[i]; q < gptr[i + 1]; ++q) rowid[q] = (int32_t)i;
}

__global__ void k_col_hist(const int32_t* __restrict__ gcol, int64_t nnz, int32_t* __restrict__ cnt) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nnz) atomicAdd(&cnt[gcol[q]], 1);
}

__global__ void k_widen(const int32_t* __restrict__ a, int64_t n, int64_t* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
  if (i == n) b[n] = 0;
}

__global__ void k_csc_gather(const int32_t* __restrict__ perm, const int32_t* __restrict__ rowid,
                             const float* __restrict__ val, int64_t nnz, int32_t* __restrict__ crow,
                             float* __restrict__ cval) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nnz) return;
  const int32_t p = perm[q];
  crow[q] = rowid[p];
  cval[q] = val[p];
}

// Sort key: window in the high word, (2^32 - 1 - length) in the low word, so an ascending
// stable sort orders windows, then lengths decreasing, then original index increasing.
__global__ void k_window_keys(const int32_t* __restrict__ len, const int32_t* __restrict__ mat,
                              const SideMat* __restrict__ sm, int64_t n, uint64_t* __restrict__ key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const SideMat s = sm[mat[i]];
  const uint64_t win = (uint64_t)(s.win_base + (i - s.orig_base) / kWindow);
  key[i] = (win << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)len[i]);
}

__global__ void k_assign(const int32_t* __restrict__ order, const int32_t* __restrict__ len,
                         const int32_t* __restrict__ mat, const SideMat* __restrict__ sm, int64_t n,
                         int32_t* __restrict__ orig2int, int32_t* __restrict__ int_orig,
                         int32_t* __restrict__ int_len) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= n) return;
  const int32_t i = order[pos];
  const SideMat s = sm[mat[i]];
  const int64_t r = s.int_base + (pos - s.orig_base);
  orig2int[i] = (int32_t)r;
  int_orig[r] = (int32_t)(i - s.orig_base);
  int_len[r] = len[i];
}

__global__ void k_slice_width(const int32_t* __restrict__ int_len, int64_t nslices,
                              int64_t* __restrict__ cnt) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s > nslices) return;
  if (s == nslices) {
    cnt[s] = 0;
    return;
  }
  int w = 0;
  for (int l = 0; l < kSlice; ++l) w = max(w, int_len[s * kSlice + l]);
  cnt[s] = (int64_t)w * kSlice;
}

// One thread per internal index: writes its row of the sliced layout (and its padding).
__global__ void k_fill_entries(const int64_t* __restrict__ slice_off, const int32_t* __restrict__ slice_mat,
                               const int32_t* __restrict__ int_orig, const int32_t* __restrict__ int_len,
                               const SideMat* __restrict__ sm, const int64_t* __restrict__ src_ptr,
                               const int32_t* __restrict__ src_idx, const float* __restrict__ src_val,
                               const int32_t* __restrict__ other_orig2int, int64_t nint,
                               int2* __restrict__ ent) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nint) return;
  const int64_t s = r / kSlice;
  const int lane = (int)(r % kSlice);
  const int64_t base = slice_off[s];
  const int64_t w = (slice_off[s + 1] - base) / kSlice;
  const int32_t li = int_orig[r];
  const int32_t len = int_len[r];
  int64_t src = 0;
  if (li >= 0) src = src_ptr[sm[slice_mat[s]].orig_base + li];
  for (int64_t q = 0; q < w; ++q) {
    int2 e = make_int2(0, 0);
    if (q < len) {
      e.x = other_orig2int[src_idx[src + q]];
      e.y = __float_as_int(src_val[src + q]);
    }
    ent[base + q * kSlice + lane] = e;
  }
}

// Two-part layout: per internal index, the number of entries gathering other-side
// indices below h; flags rows whose entries are not in that order (they always are for
// a single matrix split at a window boundary, since windows keep original order).
__global__ void k_split_len(const int64_t* __restrict__ slice_off, const int32_t* __restrict__ int_len,
                            const int2* __restrict__ ent, int64_t nint, int64_t h, int32_t* __restrict__ len_lo,
                            int* __restrict__ bad) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nint) return;
  const int64_t base = slice_off[r / kSlice] + r % kSlice;
  const int32_t len = int_len[r];
  int32_t lo = 0;
  bool high = false;
  for (int32_t q = 0; q < len; ++q) {
    const bool below = ent[base + (int64_t)q * kSlice].x < h;
    if (below && high) *bad = 1;
    if (below) ++lo;
    else high = true;
  }
  len_lo[r] = lo;
}

__global__ void k_fill_slice_mat(int32_t* __restrict__ slice_mat, int64_t first, int64_t count, int32_t b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) slice_mat[first + i] = b;
}

int bits_for(uint64_t v) {
  int b = 1;
  while (b < 64 && (v >> b) != 0) ++b;
  return b;
}

// Launch order of the slices (SideLayout::sched): stable sort by matrix, then by width
// decreasing.  Longest-first ordering shortens the tail of a launch whose slices differ in
// width: the 500,000 columns of the 1e6 x 5e5 headline (Poisson widths around 20) filled
// 1.5 rounds of the device's workgroup slots, and the half-full second round left the
// device under 90% occupied for the last ~65 us of a step.  Keeping each matrix's slices
// together keeps the gathers of consecutive workgroups within one matrix's table.  Step
// launches use it as the plan's tuning says (slice_schedule).
int build_slice_schedule(SideLayout& L, hipStream_t st) {
  std::vector<int64_t> off(L.nslices + 1);
  std::vector<int32_t> smat(L.nslices);
  MFE_HIP(hipMemcpyAsync(off.data(), L.slice_off, sizeof(int64_t) * (L.nslices + 1), hipMemcpyDeviceToHost, st));
  MFE_HIP(hipMemcpyAsync(smat.data(), L.slice_mat, sizeof(int32_t) * L.nslices, hipMemcpyDeviceToHost, st));
  MFE_HIP(hipStreamSynchronize(st));
  std::vector<int32_t> ord(L.nslices);
  for (int64_t i = 0; i < L.nslices; ++i) ord[i] = (int32_t)i;
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
    if (smat[a] != smat[b]) return smat[a] < smat[b];
    return off[a + 1] - off[a] > off[b + 1] - off[b];
  });
  MFE_CHECK(dalloc(&L.sched, L.nslices));
  MFE_HIP(hipMemcpyAsync(L.sched, ord.data(), sizeof(int32_t) * L.nslices, hipMemcpyHostToDevice, st));
  MFE_HIP(hipStreamSynchronize(st));
  return MFE_OK;
}

// Builds the ordering and slice structure of one direction; entries are filled later.
int build_side_order(SideLayout& L, const std::vector<int64_t>& counts, const int32_t* len,
                     const int32_t* mat, hipStream_t st) {
  const int count = (int)counts.size();
  std::vector<SideMat> sm(count);
  int64_t orig = 0, inb = 0, win = 0;
  for (int b = 0; b < count; ++b) {
    sm[b].orig_base = orig;
    sm[b].int_base = inb;
    sm[b].win_base = win;
    sm[b].count = counts[b];
    orig += counts[b];
    inb += ceil_div(counts[b], kSlice) * kSlice;
    win += ceil_div(counts[b], kWindow);
  }
  L.norig = orig;
  L.nint = inb;
  L.nslices = inb / kSlice;
  if (inb >= (int64_t)INT32_MAX) return set_error(MFE_EDIM, "too many rows or columns for int32 indices");

  Buf b_sm, b_key, b_key2, b_val, b_val2, b_tmp, b_cnt;
  SideMat* d_sm;
  MFE_CHECK(talloc(b_sm, &d_sm, count));
  MFE_HIP(hipMemcpyAsync(d_sm, sm.data(), sizeof(SideMat) * count, hipMemcpyHostToDevice, st));
  uint64_t *key, *key2;
  int32_t *val, *val2;
  MFE_CHECK(talloc(b_key, &key, orig));
  MFE_CHECK(talloc(b_key2, &key2, orig));
  MFE_CHECK(talloc(b_val, &val, orig));
  MFE_CHECK(talloc(b_val2, &val2, orig));
  k_window_keys<<<grid_for(orig), 256, 0, st>>>(len, mat, d_sm, orig, key);
  k_iota<<<grid_for(orig), 256, 0, st>>>(val, orig);
  size_t tmp_bytes = 0;
  const int end_bit = 32 + bits_for((uint64_t)win);
  MFE_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, key, key2, val, val2, (int)orig, 0, end_bit, st));
  void* tmp;
  MFE_CHECK(talloc(b_tmp, (char**)&tmp, (int64_t)tmp_bytes));
  MFE_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, key, key2, val, val2, (int)orig, 0, end_bit, st));

  MFE_CHECK(dalloc(&L.orig2int, orig));
  MFE_CHECK(dalloc(&L.orig, inb));
  MFE_CHECK(dalloc(&L.len, inb));
  MFE_CHECK(dalloc(&L.slice_mat, L.nslices));
  MFE_CHECK(dalloc(&L.slice_off, L.nslices + 1));
  k_fill_i32<<<grid_for(inb), 256, 0, st>>>(L.orig, inb, -1);
  k_fill_i32<<<grid_for(inb), 256, 0, st>>>(L.len, inb, 0);
  k_assign<<<grid_for(orig), 256, 0, st>>>(val2, len, mat, d_sm, orig, L.orig2int, L.orig, L.len);
  for (int b = 0; b < count; ++b) {
    const int64_t first = sm[b].int_base / kSlice, ns = ceil_div(counts[b], kSlice);
    k_fill_slice_mat<<<grid_for(ns), 256, 0, st>>>(L.slice_mat, first, ns, b);
  }
  int64_t* cnt;
  MFE_CHECK(talloc(b_cnt, &cnt, L.nslices + 1));
  k_slice_width<<<grid_for(L.nslices + 1), 256, 0, st>>>(L.len, L.nslices, cnt);
  size_t scan_bytes = 0;
  MFE_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, cnt, L.slice_off, (int)(L.nslices + 1), st));
  Buf b_tmp2;
  void* tmp2;
  MFE_CHECK(talloc(b_tmp2, (char**)&tmp2, (int64_t)scan_bytes));
  MFE_HIP(hipcub::DeviceScan::ExclusiveSum(tmp2, scan_bytes, cnt, L.slice_off, (int)(L.nslices + 1), st));
  MFE_HIP(hipMemcpyAsync(&L.nent, L.slice_off + L.nslices, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MFE_HIP(hipStreamSynchronize(st));
  return build_slice_schedule(L, st);
}

int fill_side(SideLayout& L, const std::vector<int64_t>& counts, const int64_t* src_ptr,
              const int32_t* src_idx, const float* src_val, const int32_t* other_orig2int,
              hipStream_t st) {
  const int count = (int)counts.size();
  std::vector<SideMat> sm(count);
  int64_t orig = 0;
  for (int b = 0; b < count; ++b) {
    sm[b].orig_base = orig;
    orig += counts[b];
  }
  Buf b_sm;
  SideMat* d_sm;
  MFE_CHECK(talloc(b_sm, &d_sm, count));
  MFE_HIP(hipMemcpyAsync(d_sm, sm.data(), sizeof(SideMat) * count, hipMemcpyHostToDevice, st));
  MFE_CHECK(dalloc(&L.ent, L.nent));
  k_fill_entries<<<grid_for(L.nint), 256, 0, st>>>(L.slice_off, L.slice_mat, L.orig, L.len, d_sm, src_ptr,
                                                     src_idx, src_val, other_orig2int, L.nint, L.ent);
  MFE_HIP(hipGetLastError());
  MFE_HIP(hipStreamSynchronize(st));
  return MFE_OK;
}

// Two-part layout of direction L, whose entries gather from `other`, if that table (at
// 8 bytes per index) exceeds kSplitBytes.  Single-matrix plans only: in a batched plan
// the slices running at one time belong to a few matrices, whose tables are small.
int build_split(SideLayout& L, const SideLayout& other, int count, hipStream_t st) {
  if (count != 1 || other.nint * 8 <= kSplitBytes) return MFE_OK;
  const int64_t h = (other.norig / 2 / kWindow) * kWindow;
  if (h <= 0) return MFE_OK;
  Buf b_bad;
  int* bad;
  MFE_CHECK(talloc(b_bad, &bad, 1));
  MFE_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
  MFE_CHECK(dalloc(&L.len_lo, L.nint));
  k_split_len<<<grid_for(L.nint), 256, 0, st>>>(L.slice_off, L.len, L.ent, L.nint, h, L.len_lo, bad);
  MFE_HIP(hipGetLastError());
  int bad_h = 0;
  MFE_HIP(hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  MFE_HIP(hipStreamSynchronize(st));
  if (bad_h) {
    (void)hipFree(L.len_lo);
    L.len_lo = nullptr;
    return MFE_OK;
  }
  L.split_at = h;
  return MFE_OK;
}

void free_side(SideLayout& L) {
  (void)hipFree(L.sched);
  (void)hipFree(L.len_lo);
  (void)hipFree(L.slice_off);
  (void)hipFree(L.slice_mat);
  (void)hipFree(L.len);
  (void)hipFree(L.orig);
  (void)hipFree(L.orig2int);
  (void)hipFree(L.ent);
  L = SideLayout();
}

}  // namespace

void plan_free(mfe_plan* p) {
  if (!p) return;
  free_side(p->rows);
  free_side(p->cols);
  (void)hipFree(p->x_row);
  (void)hipFree(p->xbar_row);
  (void)hipFree(p->x_col);
  (void)hipFree(p->xbar_col);
  for (int i = 0; i < 2; ++i) {
    (void)hipFree(p->desc_row[i]);
    (void)hipFree(p->desc_col[i]);
    (void)hipFree(p->signs[i]);
    (void)hipFree(p->part[i]);
  }
  (void)hipFree(p->ws);
  mfe::free_lsqr_cache(p->lsqr_cache);
  plan_free_variants(p);
  (void)hipFree(p->segs);
  (void)hipFree(p->seg_prefix);
  (void)hipFree(p->mats);
  (void)hipFree(p->flag);
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->ev0) (void)hipEventDestroy(p->ev0);
  if (p->ev1) (void)hipEventDestroy(p->ev1);
  delete p;
}

int plan_build(const mfe_matrix* mats, int32_t count, int32_t max_probes, hipStream_t st,
               mfe_plan** out) {
  if (!out) return set_error(MFE_EINVAL, "plan output pointer is NULL");
  *out = nullptr;
  if (!mats || count < 1) return set_error(MFE_EINVAL, "need at least one matrix");
  if (max_probes < 1 || max_probes > 64)
    return set_error(MFE_EUNSUPPORTED, "sparse plans support 1..64 probes per step (got %d)", max_probes);
  mfe_plan* p = new (std::nothrow) mfe_plan();
  if (!p) return set_error(MFE_ENOMEM, "host allocation failed");
  struct Guard {
    mfe_plan*& p;
    bool keep = false;
    ~Guard() {
      if (!keep) plan_free(p);
    }
  } guard{p};
  p->count = count;
  p->max_probes = max_probes;
  p->meta.resize(count);
  int64_t M = 0, N = 0, NNZ = 0;
  for (int b = 0; b < count; ++b) {
    const mfe_matrix& A = mats[b];
    if (A.kind != MFE_CSR_F32) return set_error(MFE_EUNSUPPORTED, "plans accept CSR FP32 matrices only");
    if (A.m <= 0 || A.n <= 0) return set_error(MFE_EDIM, "matrix %d: m and n must be positive", b);
    if (A.nnz < 0 || A.nnz >= (int64_t)INT32_MAX)
      return set_error(MFE_EDIM, "matrix %d: nnz must be in [0, 2^31-1)", b);
    if (!A.row_ptr || (A.nnz > 0 && (!A.col_idx || !A.val)))
      return set_error(MFE_EINVAL, "matrix %d: NULL CSR array", b);
    MatMeta& mm = p->meta[b];
    mm.m = A.m;
    mm.n = A.n;
    mm.nnz = A.nnz;
    mm.row_orig_base = M;
    mm.col_orig_base = N;
    mm.nnz_base = NNZ;
    M += A.m;
    N += A.n;
    NNZ += A.nnz;
  }
  if (NNZ >= (int64_t)INT32_MAX || M >= (int64_t)INT32_MAX / 2 || N >= (int64_t)INT32_MAX / 2)
    return set_error(MFE_EDIM, "total size exceeds the int32 index range");
  p->M = M;
  p->N = N;
  p->NNZ = NNZ;

  // ---- concatenate and validate
  Buf b_gptr, b_gcol, b_gval, b_rmat, b_cmat, b_bad;
  int64_t* gptr;
  int32_t *gcol, *rmat, *cmat;
  float* gval;
  int* bad;
  MFE_CHECK(talloc(b_gptr, &gptr, M + 1));
  MFE_CHECK(talloc(b_gcol, &gcol, NNZ));
  MFE_CHECK(talloc(b_gval, &gval, NNZ));
  MFE_CHECK(talloc(b_rmat, &rmat, M));
  MFE_CHECK(talloc(b_cmat, &cmat, N));
  MFE_CHECK(talloc(b_bad, &bad, count));
  MFE_HIP(hipMemsetAsync(bad, 0, sizeof(int) * count, st));
  for (int b = 0; b < count; ++b) {
    const mfe_matrix& A = mats[b];
    const MatMeta& mm = p->meta[b];
    k_validate_csr<<<grid_for(A.m + 1), 256, 0, st>>>(A.row_ptr, A.col_idx, A.m, A.n, A.nnz, bad + b);
    k_concat_ptr<<<grid_for(A.m + 1), 256, 0, st>>>(A.row_ptr, A.m, mm.nnz_base, gptr + mm.row_orig_base);
    if (A.nnz > 0) {
      k_concat_col<<<grid_for(A.nnz), 256, 0, st>>>(A.col_idx, A.nnz, (int32_t)mm.col_orig_base, gcol + mm.nnz_base);
      MFE_HIP(hipMemcpyAsync(gval + mm.nnz_base, A.val, sizeof(float) * A.nnz, hipMemcpyDeviceToDevice, st));
    }
    k_fill_i32<<<grid_for(A.m), 256, 0, st>>>(rmat + mm.row_orig_base, A.m, b);
    k_fill_i32<<<grid_for(A.n), 256, 0, st>>>(cmat + mm.col_orig_base, A.n, b);
  }
  MFE_HIP(hipGetLastError());
  std::vector<int> bad_h(count);
  MFE_HIP(hipMemcpyAsync(bad_h.data(), bad, sizeof(int) * count, hipMemcpyDeviceToHost, st));
  MFE_HIP(hipStreamSynchronize(st));
  for (int b = 0; b < count; ++b)
    if (bad_h[b])
      return set_error(MFE_EINVAL,
                       "matrix %d: invalid CSR (code %d: 1 row_ptr[0]!=0, 2 row_ptr[m]!=nnz, 4 decreasing "
                       "row_ptr, 8 column out of range, 16 columns not strictly increasing)",
                       b, bad_h[b]);

  // ---- transpose: stable sort of (column, position)
  Buf b_rlen, b_rowid, b_ckey, b_perm0, b_perm, b_crow, b_cval, b_ccnt, b_cptr, b_tmp;
  int32_t *rlen, *rowid, *ckey, *perm0, *perm, *crow, *ccnt;
  float* cval;
  int64_t* cptr;
  MFE_CHECK(talloc(b_rlen, &rlen, M));
  MFE_CHECK(talloc(b_rowid, &rowid, NNZ));
  MFE_CHECK(talloc(b_ckey, &ckey, NNZ));
  MFE_CHECK(talloc(b_perm0, &perm0, NNZ));
  MFE_CHECK(talloc(b_perm, &perm, NNZ));
  MFE_CHECK(talloc(b_crow, &crow, NNZ));
  MFE_CHECK(talloc(b_cval, &cval, NNZ));
  MFE_CHECK(talloc(b_ccnt, &ccnt, N));
  MFE_CHECK(talloc(b_cptr, &cptr, N + 1));
  k_row_len<<<grid_for(M), 256, 0, st>>>(gptr, M, rlen);
  k_row_ids<<<grid_for(M), 256, 0, st>>>(gptr, M, rowid);
  k_iota<<<grid_for(NNZ), 256, 0, st>>>(perm0, NNZ);
  MFE_HIP(hipMemsetAsync(ccnt, 0, sizeof(int32_t) * N, st));
  k_col_hist<<<grid_for(NNZ), 256, 0, st>>>(gcol, NNZ, ccnt);
  if (NNZ > 0) {
    size_t tb = 0;
    const int end_bit = bits_for((uint64_t)N);
    const uint32_t* kin = reinterpret_cast<const uint32_t*>(gcol);
    uint32_t* kout = reinterpret_cast<uint32_t*>(ckey);
    MFE_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, kin, kout, perm0, perm, (int)NNZ, 0, end_bit, st));
    void* tmp;
    MFE_CHECK(talloc(b_tmp, (char**)&tmp, (int64_t)tb));
    MFE_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, kin, kout, perm0, perm, (int)NNZ, 0, end_bit, st));
    k_csc_gather<<<grid_for(NNZ), 256, 0, st>>>(perm, rowid, gval, NNZ, crow, cval);
  }
  {
    Buf b_c64, b_t;
    int64_t* c64;
    MFE_CHECK(talloc(b_c64, &c64, N + 1));
    k_widen<<<grid_for(N + 1), 256, 0, st>>>(ccnt, N, c64);
    size_t tb = 0;
    MFE_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, c64, cptr, (int)(N + 1), st));
    void* tmp;
    MFE_CHECK(talloc(b_t, (char**)&tmp, (int64_t)tb));
    MFE_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, c64, cptr, (int)(N + 1), st));
    MFE_HIP(hipStreamSynchronize(st));
  }

  // ---- sliced layouts of both directions
  std::vector<int64_t> mcount(count), ncount(count);
  for (int b = 0; b < count; ++b) {
    mcount[b] = p->meta[b].m;
    ncount[b] = p->meta[b].n;
  }
  MFE_CHECK(build_side_order(p->rows, mcount, rlen, rmat, st));
  MFE_CHECK(build_side_order(p->cols, ncount, ccnt, cmat, st));
  MFE_CHECK(fill_side(p->rows, mcount, gptr, gcol, gval, p->cols.orig2int, st));
  MFE_CHECK(fill_side(p->cols, ncount, cptr, crow, cval, p->rows.orig2int, st));
  MFE_CHECK(build_split(p->rows, p->cols, count, st));
  MFE_CHECK(build_split(p->cols, p->rows, count, st));
  {
    int64_t rb = 0, cb = 0;
    for (int b = 0; b < count; ++b) {
      p->meta[b].row_int_base = rb;
      p->meta[b].col_int_base = cb;
      rb += ceil_div(p->meta[b].m, kSlice) * kSlice;
      cb += ceil_div(p->meta[b].n, kSlice) * kSlice;
    }
  }
  MFE_HIP(hipEventCreate(&p->ev0));
  MFE_HIP(hipEventCreate(&p->ev1));
  guard.keep = true;
  *out = p;
  return MFE_OK;
}

}  // namespace mfe
