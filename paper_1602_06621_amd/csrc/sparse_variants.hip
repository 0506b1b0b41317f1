// Section 6 variants on sparse plans: symmetric equilibration (Algorithm 2), varying
// row and column norms, block equilibration.  The step kernels are those of
// sparse_step.hip; this file builds and checks what the variants add to a plan.
#include <cmath>
#include <vector>

#include "sparse.h"

namespace mfe {
namespace {

template <class T>
int dev_alloc(T** ptr, int64_t count) {
  hipError_t e = hipMalloc((void**)ptr, sizeof(T) * (size_t)std::max<int64_t>(count, 1));
  if (e != hipSuccess)
    return set_error(e == hipErrorOutOfMemory ? MFE_ENOMEM : MFE_EDEVICE, "hipMalloc failed: %s",
                     hipGetErrorString(e));
  return MFE_OK;
}

template <class T>
void dev_free(T*& ptr) {
  (void)hipFree(ptr);
  ptr = nullptr;
}

inline unsigned grid256(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, 256)); }

// Symmetry of a CSR matrix with strictly increasing columns per row: every entry
// (i, j, a) has an entry (j, i) with the same value bits (binary search in row j).
__global__ void k_check_symmetric(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                  const float* __restrict__ val, int64_t m, int* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  for (int32_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
    const int32_t j = col[q];
    int32_t lo = row_ptr[j], hi = row_ptr[j + 1] - 1;
    bool found = false;
    while (lo <= hi) {
      const int32_t mid = lo + ((hi - lo) >> 1);
      const int32_t c = col[mid];
      if (c == (int32_t)i) {
        found = __float_as_int(val[mid]) == __float_as_int(val[q]);
        break;
      }
      if (c < (int32_t)i) lo = mid + 1;
      else hi = mid - 1;
    }
    if (!found) {
      atomicOr(bad, 1);
      return;
    }
  }
}

// Row entries re-indexed from the columns' internal order to the rows' own.
__global__ void k_sym_entries(const int2* __restrict__ ent, int64_t nent, const int32_t* __restrict__ col_orig,
                              const int32_t* __restrict__ row_orig2int, int2* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nent) return;
  const int2 e = ent[q];
  const int32_t o = col_orig[e.x];
  out[q] = make_int2(o >= 0 ? row_orig2int[o] : 0, e.y);
}

__global__ void k_check_targets(const double* __restrict__ t, int64_t n, int* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = t[i];
  if (!(v > 0.0) || !isfinite(v)) atomicOr(bad, 1);
}

// Per-index targets to internal order: padding lanes get 1 (never used), then every
// original index its own.
__global__ void k_fill_one(double* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = 1.0;
}

__global__ void k_scatter_targets(const double* __restrict__ t, const int32_t* __restrict__ orig2int,
                                  int64_t norig, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < norig) out[orig2int[i]] = t[i];
}

int check_block_ptr(const int64_t* ptr, int64_t nb, int64_t count, const char* side) {
  if (nb < 1 || nb > count) return set_error(MFE_EINVAL, "%s blocks: count %lld outside 1..%lld", side,
                                             (long long)nb, (long long)count);
  if (ptr[0] != 0 || ptr[nb] != count)
    return set_error(MFE_EINVAL, "%s blocks: offsets must start at 0 and end at %lld", side, (long long)count);
  for (int64_t b = 0; b < nb; ++b)
    if (ptr[b + 1] <= ptr[b]) return set_error(MFE_EINVAL, "%s blocks: offsets must increase strictly", side);
  return MFE_OK;
}

void free_block_side(mfe_plan::BlockSide& bs) {
  dev_free(bs.ptr);
  dev_free(bs.tgt);
  dev_free(bs.bx);
  dev_free(bs.bxbar);
  dev_free(bs.z);
  bs.nb = 0;
}

}  // namespace

int plan_build_symmetric(const mfe_matrix* A, int32_t max_probes, hipStream_t st, mfe_plan** out) {
  if (!out) return set_error(MFE_EINVAL, "plan output pointer is NULL");
  *out = nullptr;
  if (!A) return set_error(MFE_EINVAL, "matrix is NULL");
  if (A->kind != MFE_CSR_F32) return set_error(MFE_EUNSUPPORTED, "symmetric plans accept CSR FP32 matrices only");
  if (A->m != A->n) return set_error(MFE_EDIM, "symmetric equilibration needs a square matrix (%lld x %lld)",
                                     (long long)A->m, (long long)A->n);
  mfe_plan* p = nullptr;
  MFE_CHECK(plan_build(A, 1, max_probes, st, &p));  // validates the CSR arrays
  struct Guard {
    mfe_plan*& p;
    bool keep = false;
    ~Guard() {
      if (!keep) plan_free(p);
    }
  } guard{p};
  int* bad = nullptr;
  MFE_CHECK(dev_alloc(&bad, 1));
  MFE_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
  k_check_symmetric<<<grid256(A->m), 256, 0, st>>>(A->row_ptr, A->col_idx, A->val, A->m, bad);
  int bad_h = 0;
  hipError_t e1 = hipGetLastError();
  hipError_t e2 = hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, st);
  hipError_t e3 = hipStreamSynchronize(st);
  (void)hipFree(bad);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
    return set_error(MFE_EDEVICE, "symmetry check failed on the device");
  if (bad_h) return set_error(MFE_EINVAL, "matrix is not symmetric (pattern or values differ from the transpose)");
  MFE_CHECK(dev_alloc(&p->ent_sym, p->rows.nent));
  if (p->rows.nent > 0)
    k_sym_entries<<<grid256(p->rows.nent), 256, 0, st>>>(p->rows.ent, p->rows.nent, p->cols.orig, p->rows.orig2int,
                                                         p->ent_sym);
  MFE_HIP(hipGetLastError());
  MFE_HIP(hipStreamSynchronize(st));
  p->symmetric = true;
  guard.keep = true;
  *out = p;
  return MFE_OK;
}

int plan_set_targets(mfe_plan* p, const double* row_target, const double* col_target, hipStream_t st) {
  if (p->symmetric) return set_error(MFE_EUNSUPPORTED, "per-index targets are not available on symmetric plans");
  int* bad = nullptr;
  if (row_target || col_target) {
    MFE_CHECK(dev_alloc(&bad, 1));
    MFE_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
    if (row_target) k_check_targets<<<grid256(p->rows.norig), 256, 0, st>>>(row_target, p->rows.norig, bad);
    if (col_target) k_check_targets<<<grid256(p->cols.norig), 256, 0, st>>>(col_target, p->cols.norig, bad);
    int bad_h = 0;
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, st);
    hipError_t e3 = hipStreamSynchronize(st);
    (void)hipFree(bad);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
      return set_error(MFE_EDEVICE, "target check failed on the device");
    if (bad_h) return set_error(MFE_EINVAL, "targets must be positive and finite");
  }
  for (int i = 0; i < 2; ++i) {
    const double* t = i == 0 ? row_target : col_target;
    const SideLayout& L = i == 0 ? p->rows : p->cols;
    if (!t) {
      dev_free(p->tgt_orig[i]);
      dev_free(p->tgt_int[i]);
      continue;
    }
    if (!p->tgt_orig[i]) MFE_CHECK(dev_alloc(&p->tgt_orig[i], L.norig));
    if (!p->tgt_int[i]) MFE_CHECK(dev_alloc(&p->tgt_int[i], L.nint));
    MFE_HIP(hipMemcpyAsync(p->tgt_orig[i], t, sizeof(double) * L.norig, hipMemcpyDeviceToDevice, st));
    k_fill_one<<<grid256(L.nint), 256, 0, st>>>(p->tgt_int[i], L.nint);
    k_scatter_targets<<<grid256(L.norig), 256, 0, st>>>(t, L.orig2int, L.norig, p->tgt_int[i]);
    MFE_HIP(hipGetLastError());
  }
  MFE_HIP(hipStreamSynchronize(st));
  ++p->variant_epoch;
  return MFE_OK;
}

int plan_set_blocks(mfe_plan* p, const int64_t* row_ptr, int64_t nrb, const int64_t* col_ptr, int64_t ncb,
                    hipStream_t st) {
  if (p->symmetric) return set_error(MFE_EUNSUPPORTED, "blocks are not available on symmetric plans");
  if ((row_ptr || col_ptr) && p->count != 1)
    return set_error(MFE_EUNSUPPORTED, "block equilibration needs a single-matrix plan");
  if (row_ptr) MFE_CHECK(check_block_ptr(row_ptr, nrb, p->rows.norig, "row"));
  if (col_ptr) MFE_CHECK(check_block_ptr(col_ptr, ncb, p->cols.norig, "column"));
  for (int i = 0; i < 2; ++i) {
    mfe_plan::BlockSide& bs = p->blk[i];
    free_block_side(bs);
    const int64_t* ptr = i == 0 ? row_ptr : col_ptr;
    const int64_t nb = i == 0 ? nrb : ncb;
    if (!ptr) continue;
    MFE_CHECK(dev_alloc(&bs.ptr, nb + 1));
    MFE_HIP(hipMemcpyAsync(bs.ptr, ptr, sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice, st));
    bs.nb = nb;
    // lanes per block: the power of two at or above the mean block size, at most 64
    const int64_t mean = ceil_div(ptr[nb], nb);
    bs.group = 1;
    while (bs.group < 64 && bs.group < mean) bs.group *= 2;
  }
  MFE_HIP(hipStreamSynchronize(st));
  ++p->variant_epoch;
  return MFE_OK;
}

void plan_free_variants(mfe_plan* p) {
  dev_free(p->ent_sym);
  for (int i = 0; i < 2; ++i) {
    dev_free(p->tgt_orig[i]);
    dev_free(p->tgt_int[i]);
    free_block_side(p->blk[i]);
  }
}

}  // namespace mfe
