"""Section 6 variants of the equilibration problem, in FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

  * Symmetric equilibration (problem (prob:sym-equil), Algorithm 2): square symmetric
    A, one scaling D = E = diag(e^u); each step pushes probes s through D A D.
  * Varying row and column norms (problem (prob:equil-vary-norms)): per-row and
    per-column targets in place of alpha and beta.
  * Block equilibration (problem (prob:block-equil)): u is constant on blocks of
    consecutive rows and v on blocks of consecutive columns.

Readings of the paper taken here:
  * Targets are given as squared norms (row_target[i] = r_i^2).  The problem as printed
    has linear terms r^T u + c^T v next to the condition r^T r = c^T c; the gradient
    |DAE|^2 1 - r + gamma u would make r the squared norm, while the condition (sum
    of squared row norms = sum of squared column norms = ||DAE||_F^2) and the standard
    case r = alpha 1 (linear term alpha^2 1^T u) make r the norm itself.  The reading
    that keeps both is the linear term sum_i r_i^2 u_i, i.e. targets r_i^2.
  * Block problem: the regularisation is (gamma/2)(||u||^2 + ||v||^2) on the block
    variables (u in R^p, v in R^q), as in problem (prob:reg-constr-equil) with the block
    variables as the optimisation variables.  The gradient estimate of block i is the
    sum of the row estimates of Algorithm 1 over the rows of the block, minus the
    block's target (alpha^2 m_i, or the sum of the rows' targets) plus gamma u_i.  The
    probes stay per row and column of A, drawn exactly as in Algorithm 1.
  * Symmetric problem: the probes of Algorithm 2 are drawn like Algorithm 1's s (stream
    side 0, indexed by the column j = 0..n-1).  k probes are averaged, and the step
    offset t0 and the starting average are read as for Algorithm 1.
  * Everything else (Jacobi order, step size 2/(gamma (tau + 1)), the running average,
    the box, non-finite estimates as errors) is read as in algorithm1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import signs as _signs
from .algorithm1 import NonFiniteError, as_operator, step_size
from .theory import _sq


# ------------------------------------------------------------------ block helpers

def block_sizes(ptr, count):
    """Sizes of the blocks [ptr[b], ptr[b+1]); None means one block per index."""
    if ptr is None:
        return np.ones(count, dtype=np.int64)
    ptr = np.asarray(ptr, dtype=np.int64)
    if ptr[0] != 0 or ptr[-1] != count or np.any(np.diff(ptr) <= 0):
        raise ValueError("block pointers must start at 0, end at the dimension and increase")
    return np.diff(ptr)


def expand(x, sizes):
    """Per-index values of a per-block vector (each block's value repeated)."""
    return np.repeat(np.asarray(x, dtype=np.float64), sizes)


def block_sum(z, sizes):
    """Sum of a per-index vector over each block, in index order."""
    out = np.zeros(len(sizes))
    start = 0
    for b, s in enumerate(sizes):
        acc = 0.0
        for i in range(start, start + s):
            acc += z[i]
        out[b] = acc
        start += s
    return out


def _targets(target, default, count):
    if target is None:
        return np.full(count, float(default))
    t = np.asarray(target, dtype=np.float64)
    if t.shape != (count,) or not np.all(t > 0) or not np.all(np.isfinite(t)):
        raise ValueError("targets must be positive and finite, one per index")
    return t


# ------------------------------------------------ general (block, varying targets)

def general_objective(A, u, v, row_ptr=None, col_ptr=None, row_target=None, col_target=None,
                      alpha=1.0, beta=1.0, gamma=0.0):
    """Objective of problems (prob:equil-vary-norms) and (prob:block-equil) with the
    regularisation of (prob:reg-constr-equil): u, v are block variables (one per block;
    with no blocks, one per row / column).  Targets are squared norms per row / column
    (default alpha^2, beta^2); a block's target is the sum over its rows."""
    A = as_operator(A)
    m, n = A.shape
    rs, cs = block_sizes(row_ptr, m), block_sizes(col_ptr, n)
    rt = block_sum(_targets(row_target, alpha**2, m), rs)
    ct = block_sum(_targets(col_target, beta**2, n), cs)
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    B = _sq(A)
    du = np.exp(2.0 * expand(u, rs))
    ev = np.exp(2.0 * expand(v, cs))
    total = float(du @ np.asarray(B @ ev).ravel())
    return 0.5 * total - rt @ u - ct @ v + 0.5 * gamma * (u @ u + v @ v)


def general_gradient(A, u, v, row_ptr=None, col_ptr=None, row_target=None, col_target=None,
                     alpha=1.0, beta=1.0, gamma=0.0):
    """Exact gradient of general_objective: per block, the sum of the squared row (column)
    norms of DAE over the block, minus the block target, plus gamma times the variable."""
    A = as_operator(A)
    m, n = A.shape
    rs, cs = block_sizes(row_ptr, m), block_sizes(col_ptr, n)
    B = _sq(A)
    du = np.exp(2.0 * expand(u, rs))
    ev = np.exp(2.0 * expand(v, cs))
    r = du * np.asarray(B @ ev).ravel()
    c = ev * np.asarray(B.T @ du).ravel()
    gu = block_sum(r, rs) - block_sum(_targets(row_target, alpha**2, m), rs) + gamma * np.asarray(u)
    gv = block_sum(c, cs) - block_sum(_targets(col_target, beta**2, n), cs) + gamma * np.asarray(v)
    return gu, gv


def general_gradient_estimate(A, u, v, S, W, row_ptr=None, col_ptr=None, row_target=None,
                              col_target=None, alpha=1.0, beta=1.0, gamma=0.0):
    """Gradient estimate of the block / varying-norm problem from the probe blocks
    S [n, k] and W [m, k] of Algorithm 1: the row estimates e^(2u_i) mean_p (A E S)_ip^2
    summed over each block, minus the block target, plus gamma u.  Returns
    (g_u, g_v, z_u, z_v) with z the per-block sums."""
    A = as_operator(A)
    m, n = A.shape
    rs, cs = block_sizes(row_ptr, m), block_sizes(col_ptr, n)
    ur, vc = expand(u, rs), expand(v, cs)
    S = np.asarray(S, dtype=np.float64).reshape(n, -1)
    W = np.asarray(W, dtype=np.float64).reshape(m, -1)
    Y = np.asarray(A @ (np.exp(vc)[:, None] * S))
    X = np.asarray(A.T @ (np.exp(ur)[:, None] * W))
    z_u = block_sum(np.exp(2.0 * ur) * np.mean(Y * Y, axis=1), rs)
    z_v = block_sum(np.exp(2.0 * vc) * np.mean(X * X, axis=1), cs)
    t_u = block_sum(_targets(row_target, alpha**2, m), rs)
    t_v = block_sum(_targets(col_target, beta**2, n), cs)
    return z_u - t_u + gamma * np.asarray(u), z_v - t_v + gamma * np.asarray(v), z_u, z_v


def equilibrate_general(A, gamma, M, steps, k=1, seed=0, t0=0, row_ptr=None, col_ptr=None,
                        row_target=None, col_target=None, alpha=1.0, beta=1.0, u0=None, v0=None,
                        batch=0):
    """Algorithm 1 applied to the block and varying-norm problems (Section 6): the same
    probes, step size, projection and running average, with the gradient estimate of
    general_gradient_estimate.  u0 / v0 and the returned u_bar / v_bar / u / v are block
    variables; d and e are the per-row and per-column scalings e^u_bar expanded."""
    if not (gamma > 0 and M > 0):
        raise ValueError("gamma and M must be positive")
    if steps < 0 or k < 1:
        raise ValueError("steps must be >= 0 and k >= 1")
    A = as_operator(A)
    m, n = A.shape
    rs, cs = block_sizes(row_ptr, m), block_sizes(col_ptr, n)
    u = np.zeros(len(rs)) if u0 is None else np.array(u0, dtype=np.float64)
    v = np.zeros(len(cs)) if v0 is None else np.array(v0, dtype=np.float64)
    u_bar, v_bar = u.copy(), v.copy()
    for t in range(1, steps + 1):
        tau = t + t0
        S = _signs.signs(seed, batch, t, 0, n, k)
        W = _signs.signs(seed, batch, t, 1, m, k)
        g_u, g_v, z_u, z_v = general_gradient_estimate(A, u, v, S, W, row_ptr, col_ptr, row_target,
                                                       col_target, alpha, beta, gamma)
        if not (np.all(np.isfinite(z_u)) and np.all(np.isfinite(z_v))):
            raise NonFiniteError(f"non-finite gradient estimate at step {t}")
        eta = step_size(gamma, tau)
        u_new = np.clip(u - eta * g_u, -M, M)
        v_new = np.clip(v - eta * g_v, -M, M)
        u_bar = 2.0 * u_new / (tau + 2.0) + tau * u_bar / (tau + 2.0)
        v_bar = 2.0 * v_new / (tau + 2.0) + tau * v_bar / (tau + 2.0)
        u, v = u_new, v_new
    return dict(u_bar=u_bar, v_bar=v_bar, u=u, v=v, d=np.exp(expand(u_bar, rs)), e=np.exp(expand(v_bar, cs)))


def compress(A, row_ptr=None, col_ptr=None):
    """The matrix of block norms: entry (a, b) = sqrt of the sum of A_ij^2 over the rows
    of block a and the columns of block b.  Its (unblocked) problem has the same
    objective as the block problem of A, since the scaling is constant on each block."""
    A = as_operator(A)
    m, n = A.shape
    rs, cs = block_sizes(row_ptr, m), block_sizes(col_ptr, n)
    B = _sq(A)
    B = B.toarray() if sp.issparse(B) else B
    rb = np.repeat(np.arange(len(rs)), rs)
    cb = np.repeat(np.arange(len(cs)), cs)
    C = np.zeros((len(rs), len(cs)))
    np.add.at(C, (rb[:, None], cb[None, :]), B)
    return np.sqrt(C)


# ------------------------------------------------------------------- symmetric

def sym_objective(A, u, alpha, gamma=0.0):
    """(1/4) sum_ij A_ij^2 e^(2u_i + 2u_j) - alpha^2 1^T u + (gamma/2) ||u||^2
    (problem (prob:sym-equil) with the regularisation of (prob:reg-constr-equil))."""
    A = as_operator(A)
    u = np.asarray(u, dtype=np.float64)
    e2 = np.exp(2.0 * u)
    return 0.25 * float(e2 @ np.asarray(_sq(A) @ e2).ravel()) - alpha**2 * u.sum() + 0.5 * gamma * (u @ u)


def sym_gradient(A, u, alpha, gamma):
    """Exact gradient of sym_objective for symmetric A: |DAD|^2 1 - alpha^2 + gamma u."""
    A = as_operator(A)
    u = np.asarray(u, dtype=np.float64)
    e2 = np.exp(2.0 * u)
    return e2 * np.asarray(_sq(A) @ e2).ravel() - alpha**2 + gamma * u


def sym_gradient_estimate(A, u, S, alpha, gamma):
    """Algorithm 2's estimate |D A D s|^2 - alpha^2 + gamma u, averaged over the k
    columns of S [n, k].  Returns (g, z)."""
    A = as_operator(A)
    u = np.asarray(u, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64).reshape(A.shape[0], -1)
    Y = np.asarray(A @ (np.exp(u)[:, None] * S))
    z = np.exp(2.0 * u) * np.mean(Y * Y, axis=1)
    return z - alpha**2 + gamma * u, z


def equilibrate_symmetric(A, alpha, gamma, M, steps, k=1, seed=0, t0=0, u0=None, batch=0):
    """Algorithm 2 (Section 6): projected stochastic gradient for symmetric equilibration.
    Returns u_bar, u and d = e^u_bar (D = E)."""
    if not (alpha > 0 and gamma > 0 and M > 0):
        raise ValueError("alpha, gamma and M must be positive")
    if steps < 0 or k < 1:
        raise ValueError("steps must be >= 0 and k >= 1")
    A = as_operator(A)
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("symmetric equilibration needs a square matrix")
    u = np.zeros(n) if u0 is None else np.array(u0, dtype=np.float64)
    u_bar = u.copy()
    for t in range(1, steps + 1):
        tau = t + t0
        S = _signs.signs(seed, batch, t, 0, n, k)
        g, z = sym_gradient_estimate(A, u, S, alpha, gamma)
        if not np.all(np.isfinite(z)):
            raise NonFiniteError(f"non-finite gradient estimate at step {t}")
        u_new = np.clip(u - step_size(gamma, tau) * g, -M, M)
        u_bar = 2.0 * u_new / (tau + 2.0) + tau * u_bar / (tau + 2.0)
        u = u_new
    return dict(u_bar=u_bar, u=u, d=np.exp(u_bar))
