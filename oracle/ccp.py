"""Chambolle-Cremers-Pock (CCP) on the Lasso with and without equilibration
(Section 5.2), in FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Problem (Section 5.2): minimise ||A x - b||^2 / sqrt(lam) + sqrt(lam) ||x||_1, as
f(x) + g(A x) with f = sqrt(lam) ||.||_1 and g(y) = ||y - b||^2 / sqrt(lam).

Readings taken here:
  * Equilibration enters as the change of variables x = E xbar: CCP runs on
    Abar = D A E with fbar(xbar) = sqrt(lam) ||E xbar||_1 and gbar(ybar) = g(D^-1 ybar),
    which has the same optimal value; x = E xbar is reported.  D = E = I is the plain run.
  * The iteration is Chambolle and Pock's first-order primal-dual method with
    theta = 1 (the paper gives only its parameters: tau = sigma = 0.9 / ||Abar||_2,
    theta = 1, all initial iterates 0):
        y  <- prox_{sigma gbar*}(y + sigma Abar xt)
        x' <- prox_{tau fbar}(x - tau Abar' y)
        xt <- x' + theta (x' - x),  x <- x'
  * The proximal maps are the closed forms of these separable functions:
        prox_{sigma gbar*}(v)_i = (v_i - sigma d_i b_i) / (1 + sigma d_i^2 sqrt(lam) / 2)
        prox_{tau fbar}(u)_j    = sign(u_j) max(|u_j| - tau sqrt(lam) e_j, 0)
    (gbar*(z) = sum_i d_i b_i z_i + d_i^2 sqrt(lam) z_i^2 / 4 is the conjugate of gbar).
  * ||Abar||_2 is the largest singular value (computed here by a dense SVD).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def objective(A, b, lam, x):
    """f(x) + g(A x) = ||A x - b||^2 / sqrt(lam) + sqrt(lam) ||x||_1."""
    r = np.asarray(A @ x).ravel() - b
    s = np.sqrt(lam)
    return float(r @ r) / s + s * float(np.abs(x).sum())


def default_lambda(A, b):
    """lam = 1e-3 ||A' b||_inf (Section 5.2)."""
    return 1e-3 * float(np.abs(np.asarray(A.T @ b).ravel()).max())


def scaled(A, d, e):
    """D A E as an FP64 matrix of the same kind."""
    if sp.issparse(A):
        return (sp.diags(d) @ sp.csr_matrix(A, dtype=np.float64) @ sp.diags(e)).tocsr()
    return d[:, None] * np.asarray(A, dtype=np.float64) * e[None, :]


def op_norm(A, d=None, e=None):
    """||D A E||_2: the largest singular value, by a dense SVD for small matrices and by
    scipy's sparse partial SVD (ARPACK) for large sparse ones."""
    m, n = A.shape
    d = np.ones(m) if d is None else np.asarray(d, dtype=np.float64)
    e = np.ones(n) if e is None else np.asarray(e, dtype=np.float64)
    B = scaled(A, d, e)
    if sp.issparse(B) and min(m, n) > 2000:
        from scipy.sparse.linalg import svds

        return float(svds(B, k=1, tol=1e-14, return_singular_vectors=False, random_state=0)[0])
    B = B.toarray() if sp.issparse(B) else B
    return float(np.linalg.svd(B, compute_uv=False)[0])


def prox_dual(v, sigma, d, b, lam):
    """prox of sigma gbar* (see the module docstring)."""
    return (v - sigma * d * b) / (1.0 + sigma * d * d * np.sqrt(lam) / 2.0)


def prox_primal(u, tau, e, lam):
    """prox of tau fbar: soft threshold at tau sqrt(lam) e_j."""
    return np.sign(u) * np.maximum(np.abs(u) - tau * np.sqrt(lam) * e, 0.0)


def ccp_lasso(A, b, lam, iters, d=None, e=None, norm=None, theta=1.0, trace_every=0):
    """CCP on the (optionally equilibrated) Lasso.  Returns x = E xbar after `iters`
    iterations, the step sizes and, when trace_every > 0, f(x) every trace_every
    iterations."""
    m, n = A.shape
    d = np.ones(m) if d is None else np.asarray(d, dtype=np.float64)
    e = np.ones(n) if e is None else np.asarray(e, dtype=np.float64)
    B = scaled(A, d, e)
    L = op_norm(A, d, e) if norm is None else float(norm)
    tau = sigma = 0.9 / L
    x = np.zeros(n)
    xt = np.zeros(n)
    y = np.zeros(m)
    trace = []
    for it in range(1, iters + 1):
        y = prox_dual(y + sigma * np.asarray(B @ xt).ravel(), sigma, d, b, lam)
        xn = prox_primal(x - tau * np.asarray(B.T @ y).ravel(), tau, e, lam)
        xt = xn + theta * (xn - x)
        x = xn
        if trace_every and it % trace_every == 0:
            trace.append(objective(A, b, lam, e * x))
    return dict(x=e * x, xbar=x, y=y, tau=tau, sigma=sigma, norm=L, trace=np.array(trace))
