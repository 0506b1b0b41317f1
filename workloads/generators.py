"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws problem data (matrices, right-hand sides, warm starts).  It
holds none of the equilibration arithmetic: no probes, no scalings, no updates.
Every generator is a pure function of its arguments and a numpy PCG64 seed.

Workload shapes follow the experiments of the paper (Section 4, Section 5.1):
a base matrix with i.i.d. standard-normal entries, multiplied on the left and
right by diagonal matrices of log-normal scales, so that row and column norms
spread over several orders of magnitude.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class CSR:
    """A CSR matrix with FP32 values and int32 indices (sorted, unique columns per row)."""

    m: int
    n: int
    row_ptr: np.ndarray  # int32 [m+1]
    col_idx: np.ndarray  # int32 [nnz]
    val: np.ndarray  # float32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self, dtype=np.float64) -> sp.csr_matrix:
        """Exact FP64 (or other) copy as a scipy CSR matrix."""
        return sp.csr_matrix(
            (self.val.astype(dtype), self.col_idx.astype(np.int64), self.row_ptr.astype(np.int64)),
            shape=(self.m, self.n),
        )


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def scaled_dense(m: int, n: int, sigma: float, seed: int) -> np.ndarray:
    """Dense FP64 A = diag(e^r) G diag(e^c), G iid N(0,1), r, c iid N(0, sigma^2)."""
    g = rng(seed)
    G = g.standard_normal((m, n))
    r = g.normal(0.0, sigma, m)
    c = g.normal(0.0, sigma, n)
    return (np.exp(r)[:, None] * G) * np.exp(c)[None, :]


def _distinct_columns(g: np.random.Generator, lengths: np.ndarray, n: int) -> np.ndarray:
    """Per row, `lengths[i]` distinct uniform columns in [0, n), sorted; concatenated."""
    m = lengths.shape[0]
    out = []
    lmax = int(lengths.max()) if m else 0
    # Rows are drawn in groups of equal length; duplicates are redrawn.
    for L in np.unique(lengths):
        L = int(L)
        rows = np.nonzero(lengths == L)[0]
        if L == 0:
            continue
        if L > n:
            raise ValueError("row longer than the number of columns")
        if 4 * L > n:
            # dense-ish rows: draw a permutation prefix per row
            cols = np.stack([np.sort(g.permutation(n)[:L]) for _ in rows]) if len(rows) else np.zeros((0, L), np.int64)
        else:
            cols = np.sort(g.integers(0, n, size=(len(rows), L)), axis=1)
            while True:
                dup = np.any(cols[:, 1:] == cols[:, :-1], axis=1) if L > 1 else np.zeros(len(rows), bool)
                if not dup.any():
                    break
                cols[dup] = np.sort(g.integers(0, n, size=(int(dup.sum()), L)), axis=1)
        out.append((rows, cols))
    del lmax
    col_idx = np.empty(int(lengths.sum()), dtype=np.int32)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lengths, out=row_ptr[1:])
    for rows, cols in out:
        L = cols.shape[1]
        dst = row_ptr[rows][:, None] + np.arange(L)[None, :]
        col_idx[dst.ravel()] = cols.ravel()
    return col_idx


def scaled_sparse(
    m: int,
    n: int,
    nnz_per_row,
    sigma: float,
    seed: int,
) -> CSR:
    """Sparse CSR FP32 with uniform random distinct columns per row.

    nnz_per_row: an int (every row has that many entries), or an int array of
    per-row lengths.  Values are N(0,1) * exp(r_i + c_j) with r, c iid N(0, sigma^2),
    computed in FP64 and rounded once to FP32.
    """
    g = rng(seed)
    if np.isscalar(nnz_per_row):
        lengths = np.full(m, int(nnz_per_row), dtype=np.int64)
    else:
        lengths = np.asarray(nnz_per_row, dtype=np.int64)
        assert lengths.shape == (m,)
    col_idx = _distinct_columns(g, lengths, n)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lengths, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32 row pointers")
    r = g.normal(0.0, sigma, m)
    c = g.normal(0.0, sigma, n)
    rows = np.repeat(np.arange(m), lengths)
    vals = g.standard_normal(row_ptr[-1]) * np.exp(r[rows] + c[col_idx])
    return CSR(m, n, row_ptr.astype(np.int32), col_idx, vals.astype(np.float32))


def symmetric_sparse(n: int, half_nnz_per_row: int, sigma: float, seed: int) -> CSR:
    """Square symmetric CSR FP32: G with half_nnz_per_row uniform random distinct columns
    per row and N(0,1) values, A = diag(e^r) (G + G') diag(e^r) with r iid N(0, sigma^2),
    computed in FP64 (entry (i, j) and (j, i) by the same operations) and rounded once to
    FP32, so that A equals its transpose bit for bit.  About 2 half_nnz_per_row entries
    per row."""
    g = rng(seed)
    lengths = np.full(n, int(half_nnz_per_row), dtype=np.int64)
    cols = _distinct_columns(g, lengths, n)
    rows = np.repeat(np.arange(n), lengths)
    vals = g.standard_normal(rows.size)
    G = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    S = (G + G.T).tocsr()
    S.sum_duplicates()
    S.sort_indices()
    r = g.normal(0.0, sigma, n)
    er = np.exp(r)
    ri = np.repeat(np.arange(n), np.diff(S.indptr))
    data = (S.data * er[ri]) * er[S.indices]
    keep = data != 0.0
    A = sp.csr_matrix((data[keep], S.indices[keep], np.concatenate([[0], np.cumsum(
        np.bincount(ri[keep], minlength=n))])), shape=(n, n))
    if A.nnz >= 2**31:
        raise ValueError("nnz does not fit int32 row pointers")
    return CSR(n, n, A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float32))


def paper_sparse(m: int, n: int, density: float, seed: int) -> CSR:
    """The construction of the paper's experiments (Section 4): a sparse matrix with each
    entry nonzero with probability `density` (per-row counts Binomial(n, density), distinct
    uniform columns), N(0,1) nonzeros, scaled as diag(e^u) A diag(e^v) with u, v iid
    N(1, 1); FP64, rounded once to FP32."""
    g = rng(seed)
    lengths = g.binomial(n, density, size=m).astype(np.int64)
    col_idx = _distinct_columns(g, lengths, n)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lengths, out=row_ptr[1:])
    u = g.normal(1.0, 1.0, m)
    v = g.normal(1.0, 1.0, n)
    rows = np.repeat(np.arange(m), lengths)
    vals = g.standard_normal(row_ptr[-1]) * np.exp(u[rows] + v[col_idx])
    return CSR(m, n, row_ptr.astype(np.int32), col_idx, vals.astype(np.float32))


def lasso_rhs(A, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Right-hand side of the Lasso experiment (Section 5.2): x_hat with n/10 nonzero
    entries at uniform random positions, drawn N(0,1); b = A x_hat + nu, nu iid N(0,1).
    A is any matrix with a product (values taken as stored, in FP64)."""
    g = rng(seed)
    m, n = A.shape
    x_hat = np.zeros(n)
    idx = g.choice(n, n // 10, replace=False)
    x_hat[idx] = g.standard_normal(idx.size)
    b = np.asarray(A @ x_hat, dtype=np.float64).ravel() + g.standard_normal(m)
    return b, x_hat


def poisson_lengths(m: int, mean: float, n: int, seed: int) -> np.ndarray:
    """Per-row nonzero counts ~ Poisson(mean), capped at n (empty rows allowed)."""
    g = rng(seed)
    return np.minimum(g.poisson(mean, m), n).astype(np.int64)


def batched_shapes(count: int, seed: int, m_lo=1000, m_hi=64000):
    """Shapes of a batch of uneven problems: m ~ U[m_lo, m_hi], n ~ U[m/4, m].
    Drawn matrix by matrix, so the first c shapes do not depend on count."""
    g = rng(seed)
    ms, ns = [], []
    for _ in range(count):
        mm = int(g.integers(m_lo, m_hi + 1))
        ms.append(mm)
        ns.append(int(g.integers(max(1, mm // 4), mm + 1)))
    return np.array(ms, dtype=np.int64), np.array(ns, dtype=np.int64)


def batched_sparse(count: int, seed: int, mean_nnz=12.0, sigma=2.0, m_lo=1000, m_hi=64000):
    """A list of CSR matrices with Poisson(mean_nnz) row lengths and log-normal scales."""
    ms, ns = batched_shapes(count, seed, m_lo, m_hi)
    mats = []
    for b in range(count):
        L = poisson_lengths(int(ms[b]), mean_nnz, int(ns[b]), seed * 7919 + 2 * b + 1)
        mats.append(scaled_sparse(int(ms[b]), int(ns[b]), L, sigma, seed * 7919 + 2 * b + 2))
    return mats


def rhs_consistent(A, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """x* ~ N(0,1) and b = A x* (FP64; A as FP64 dense or scipy)."""
    g = rng(seed)
    x = g.standard_normal(A.shape[1])
    return A @ x, x


def rhs_noisy(A, seed: int, noise=1e-3) -> tuple[np.ndarray, np.ndarray]:
    """x* ~ N(0,1) and b = A x* + noise * N(0,1) (FP64)."""
    g = rng(seed)
    x = g.standard_normal(A.shape[1])
    return A @ x + noise * g.standard_normal(A.shape[0]), x


def round_to_bf16(x: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Round FP64 values directly to bfloat16 (8 significant bits, round-half-even).

    Returns (bits uint16, values as FP64).  No intermediate FP32 rounding, so no
    double rounding.  Values must lie inside the FP32 normal range.
    """
    x = np.asarray(x, dtype=np.float64)
    mant, ex = np.frexp(x)  # x = mant * 2**ex, 0.5 <= |mant| < 1
    r = np.ldexp(np.rint(np.ldexp(mant, 8)), ex - 8)
    f32 = r.astype(np.float32)
    if not np.array_equal(f32.astype(np.float64), r):
        raise ValueError("value outside the bfloat16 normal range")
    bits = (f32.view(np.uint32) >> 16).astype(np.uint16)
    return bits, r


def csr_from_dense(A: np.ndarray) -> CSR:
    """CSR FP32 copy of the nonzeros of a dense array (values rounded to FP32)."""
    S = sp.csr_matrix(A)
    S.sort_indices()
    return CSR(A.shape[0], A.shape[1], S.indptr.astype(np.int32), S.indices.astype(np.int32),
               S.data.astype(np.float32))


def warmstart_matrix(m: int, n: int, sigma: float, seed: int, lo: int = 8, hi: int = 16) -> CSR:
    """Sparse CSR with U{lo..hi} entries per row and log-normal scales sigma (the
    learned-warm-start workloads)."""
    g = rng(seed)
    lengths = g.integers(lo, hi + 1, size=m)
    return scaled_sparse(m, n, lengths, sigma, seed + 1)


def warmstart_training_set(count: int, seed: int, m_lo=10_000, m_hi=50_000, s_lo=0.5, s_hi=3.0):
    """Training matrices for the warm start: m ~ U[m_lo, m_hi], n = m/2, sigma ~ U[s_lo, s_hi]."""
    g = rng(seed)
    out = []
    for b in range(count):
        m = int(g.integers(m_lo, m_hi + 1))
        s = float(g.uniform(s_lo, s_hi))
        out.append(warmstart_matrix(m, max(1, m // 2), s, seed * 1009 + 3 * b))
    return out
