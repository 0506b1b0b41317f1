"""Objective, gradients and exact solvers of the equilibration problems (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

A is a dense FP64 ndarray or a scipy sparse matrix; all arithmetic is FP64.
Notation follows the paper: u (rows), v (columns), D = diag(e^u), E = diag(e^v),
alpha and beta the target row and column norms, gamma the regularisation weight
and M the box bound of problem (prob:reg-constr-equil), Section 2.3.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.special


def _sq(A):
    """Elementwise square |A|^2 as the same kind of matrix."""
    if sp.issparse(A):
        B = A.copy().astype(np.float64)
        B.data = B.data * B.data
        return B
    A = np.asarray(A, dtype=np.float64)
    return A * A


def scaled_sq(A, u, v):
    """|DAE|^2 (the m x n matrix with entries A_ij^2 e^(2u_i + 2v_j))."""
    B = _sq(A)
    du = np.exp(2.0 * np.asarray(u, dtype=np.float64))
    ev = np.exp(2.0 * np.asarray(v, dtype=np.float64))
    if sp.issparse(B):
        return sp.diags(du) @ B @ sp.diags(ev)
    return du[:, None] * B * ev[None, :]


def row_col_sq_norms(A, u, v):
    """Row and column squared norms of DAE: (|DAE|^2 1, |E A^T D|^2 1)."""
    S = scaled_sq(A, u, v)
    r = np.asarray(S.sum(axis=1)).ravel()
    c = np.asarray(S.sum(axis=0)).ravel()
    return r, c


def objective(A, u, v, alpha, beta, gamma=0.0):
    """f(u, v) of problem (prob:reg-constr-equil); gamma = 0 gives (prob:equil), Section 2."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    S = scaled_sq(A, u, v)
    return (0.5 * float(S.sum()) - alpha**2 * u.sum() - beta**2 * v.sum()
            + 0.5 * gamma * (u @ u + v @ v))


def gradient(A, u, v, alpha, beta, gamma):
    """Exact gradient (Section 3.1): |DAE|^2 1 - alpha^2 + gamma u, and the v analogue."""
    r, c = row_col_sq_norms(A, u, v)
    return r - alpha**2 + gamma * np.asarray(u), c - beta**2 + gamma * np.asarray(v)


def gradient_estimate(A, u, v, S, W, alpha, beta, gamma):
    """Unbiased gradient estimate from probe blocks (Section 3.1, Algorithm 1).

    S: [n, k] probes pushed through A (entries +-1), W: [m, k] probes pushed
    through A^T.  With k > 1 the squared products are averaged over the k
    columns, i.e. the mean of k independent single-probe estimates.
    Returns (g_u, g_v, z_u, z_v) where z are the row-norm estimates.
    """
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64).reshape(A.shape[1], -1)
    W = np.asarray(W, dtype=np.float64).reshape(A.shape[0], -1)
    Y = A @ (np.exp(v)[:, None] * S)  # A E S, [m, k]
    X = A.T @ (np.exp(u)[:, None] * W)  # A^T D W, [n, k]
    Y = np.asarray(Y)
    X = np.asarray(X)
    z_u = np.exp(2.0 * u) * np.mean(Y * Y, axis=1)  # |D A E s|^2, averaged over probes
    z_v = np.exp(2.0 * v) * np.mean(X * X, axis=1)  # |E A^T D w|^2
    return z_u - alpha**2 + gamma * u, z_v - beta**2 + gamma * v, z_u, z_v


def second_moment(A, u, v, alpha, beta, gamma):
    """E_{s,w} ||g~||^2 for single probes (k = 1), in closed form.

    Section 3.2 prints a constant 3 in front of the squared row/column-norm term;
    expanding E[(b^T s)^4] = 3 sum b^4 + ... gives, per row, Var[(b^T s)^2]
    = 2 (sum b^2)^2 - 2 sum b^4, so the identity that holds is
      ||grad f||^2 + 2 sum_i r_i^2 + 2 sum_j c_j^2 - 4 sum_ij |DAE|_ij^4,
    with r, c the row and column squared norms of DAE.  Enumeration over all
    sign vectors confirms this (tests/test_oracle_estimator.py).
    """
    gu, gv = gradient(A, u, v, alpha, beta, gamma)
    S = scaled_sq(A, u, v)
    r = np.asarray(S.sum(axis=1)).ravel()
    c = np.asarray(S.sum(axis=0)).ravel()
    if sp.issparse(S):
        s4 = float(S.multiply(S).sum())
    else:
        s4 = float((S * S).sum())
    return float(gu @ gu + gv @ gv + 2.0 * (r @ r) + 2.0 * (c @ c) - 4.0 * s4)


# ---------------------------------------------------------------- exact solvers

def sinkhorn_knopp(A, alpha, beta, iters=5000, tol=1e-13):
    """Alternating exact minimisation of (prob:equil) over u and v (Section 2.1).

    D_ii = alpha (sum_j A_ij^2 E_jj^2)^(-1/2), then E_jj = beta (sum_i A_ij^2 D_ii^2)^(-1/2).
    Returns (u, v, iterations).  Requires A to be equilibratable (no zero rows/cols).
    """
    B = _sq(A)
    m, n = B.shape
    e2 = np.ones(n)
    d2 = np.ones(m)
    for it in range(1, iters + 1):
        d2 = alpha**2 / np.asarray(B @ e2).ravel()
        e2_new = beta**2 / np.asarray(B.T @ d2).ravel()
        done = np.max(np.abs(np.log(e2_new) - np.log(e2))) < tol
        e2 = e2_new
        if done:
            break
    return 0.5 * np.log(d2), 0.5 * np.log(e2), it


def lambertw_exp(L):
    """Principal Lambert W evaluated at exp(L), for real L (vectorised, FP64).

    Solves w + log(w) = L.  For moderate L this is scipy's W(e^L); for large L
    (where e^L overflows) Newton's method on h(w) = w + log w - L is used,
    started at L - log L.
    """
    L = np.asarray(L, dtype=np.float64)
    out = np.empty_like(L)
    small = L < 600.0
    if np.any(small):
        out[small] = np.real(scipy.special.lambertw(np.exp(L[small])))
    big = ~small
    if np.any(big):
        Lb = L[big]
        w = Lb - np.log(Lb)
        for _ in range(50):
            step = (w + np.log(w) - Lb) / (1.0 + 1.0 / w)
            w = w - step
            if np.max(np.abs(step)) < 1e-15 * np.max(np.abs(w)):
                break
        out[big] = w
    return out


def bcd_regularized(A, alpha, beta, gamma, M, iters=20000, tol=1e-14):
    """Block coordinate minimisation of (prob:reg-constr-equil) (Section 2.3).

    The exact minimiser over u with v fixed: with c_i = sum_j A_ij^2 e^(2 v_j),
    c_i e^(2u) - alpha^2 + gamma u = 0 gives 2u = 2alpha^2/gamma - W(z_i),
    z_i = (2/gamma) e^(2alpha^2/gamma) c_i, then u is clipped to [-M, M]
    (the one-dimensional objective is strictly convex).  The printed formula in
    the paper omits the exponential around (2alpha^2/gamma - W); this is the
    reading that satisfies the optimality condition.  Rows with c_i = 0 give
    u = min(M, alpha^2/gamma).  Returns (u, v, iterations).
    """
    B = _sq(A)
    m, n = B.shape
    u = np.zeros(m)
    v = np.zeros(n)

    def block(c, target):
        out = np.full(c.shape, min(M, target / gamma))
        pos = c > 0
        L = np.log(2.0 / gamma) + 2.0 * target / gamma + np.log(c[pos])
        out[pos] = np.clip(0.5 * (2.0 * target / gamma - lambertw_exp(L)), -M, M)
        return out

    for it in range(1, iters + 1):
        u = block(np.asarray(B @ np.exp(2.0 * v)).ravel(), alpha**2)
        v_new = block(np.asarray(B.T @ np.exp(2.0 * u)).ravel(), beta**2)
        done = np.max(np.abs(v_new - v)) < tol
        v = v_new
        if done:
            break
    return u, v, it


def newton_regularized(A, alpha, beta, gamma, iters=200, tol=1e-12):
    """Newton's method with backtracking line search for (prob:reg-constr-equil)
    without the box (Section 4 obtains p* this way and checks the box is inactive).

    Dense Hessian of size (m + n); for small problems only.
    Hessian: d2f/du_i^2 = 2 r_i + gamma, d2f/dv_j^2 = 2 c_j + gamma,
    d2f/du_i dv_j = 2 |DAE|^2_ij.  Returns (u, v, iterations).
    """
    m, n = A.shape
    u = np.zeros(m)
    v = np.zeros(n)
    f = objective(A, u, v, alpha, beta, gamma)
    for it in range(1, iters + 1):
        gu, gv = gradient(A, u, v, alpha, beta, gamma)
        g = np.concatenate([gu, gv])
        S = scaled_sq(A, u, v)
        S = S.toarray() if sp.issparse(S) else S
        H = np.zeros((m + n, m + n))
        H[:m, :m] = np.diag(2.0 * S.sum(axis=1) + gamma)
        H[m:, m:] = np.diag(2.0 * S.sum(axis=0) + gamma)
        H[:m, m:] = 2.0 * S
        H[m:, :m] = 2.0 * S.T
        dx = -np.linalg.solve(H, g)
        lam2 = -g @ dx
        if lam2 / 2.0 <= tol:
            break
        s = 1.0
        while True:
            un, vn = u + s * dx[:m], v + s * dx[m:]
            fn = objective(A, un, vn, alpha, beta, gamma)
            if fn <= f - 0.25 * s * lam2 or s < 1e-12:
                break
            s *= 0.5
        u, v, f = un, vn, fn
    return u, v, it


# ------------------------------------------------------- condition-number bound

def log_phi(U):
    """log Phi(U) = ||U||_F^2 / 2 - sum_i log sigma_i (Section 2.2), via SVD."""
    s = np.linalg.svd(np.asarray(U, dtype=np.float64), compute_uv=False)
    return 0.5 * float(np.sum(s * s)) - float(np.sum(np.log(s)))


def kappa(U):
    s = np.linalg.svd(np.asarray(U, dtype=np.float64), compute_uv=False)
    return float(s[0] / s[-1])


def log_kappa_upper_bound(U):
    """log of 2 e^(-n/2) Phi(U), the upper bound on kappa(U) of Theorem 2.2."""
    n = np.asarray(U).shape[0]
    return np.log(2.0) - 0.5 * n + log_phi(U)


def kappa_norm_ratio_lower_bound(U):
    """Ratio of largest to smallest column (and row) 2-norm, a lower bound on kappa (Section 1)."""
    U = np.asarray(U, dtype=np.float64)
    cn = np.linalg.norm(U, axis=0)
    rn = np.linalg.norm(U, axis=1)
    return float(cn.max() / cn.min()), float(rn.max() / rn.min())
