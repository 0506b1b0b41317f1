"""LSQR on the equilibrated system of Section 5.1, in FP64.  TEST INFRASTRUCTURE ONLY.

Section 5.1 solves (D A E) x_bar = D b with LSQR and recovers x = E x_bar; the
accuracy that counts is the residual of the original system, ||A x - b|| / ||b||.
LSQR itself is the Golub-Kahan bidiagonalisation method of Paige & Saunders
(ACM TOMS 8(1), 1982); the recurrences below follow that paper's description.

Stopping rule (shared with the GPU library): every `check_every` iterations and at
max_iter, stop when ||A x - b|| / ||b|| <= tol (reason 1) or when LSQR's
normal-equation estimate ||Abar^T rbar|| / (||Abar||_F-estimate ||rbar||) <= tol
(reason 2); otherwise stop at max_iter (reason 0).  Reason 3: the
bidiagonalisation broke down (alpha or beta exactly 0: the current x is exact).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _op(A):
    if sp.issparse(A):
        return sp.csr_matrix(A, dtype=np.float64)
    return np.asarray(A, dtype=np.float64)


def lsqr(A, b, d=None, e=None, tol=1e-6, max_iter=100, check_every=1):
    A = _op(A)
    m, n = A.shape
    b = np.asarray(b, dtype=np.float64)
    d = np.ones(m) if d is None else np.asarray(d, dtype=np.float64)
    e = np.ones(n) if e is None else np.asarray(e, dtype=np.float64)

    def mv(x):  # Abar x = D A E x
        return d * (A @ (e * x))

    def rmv(y):  # Abar^T y = E A^T D y
        return e * (A.T @ (d * y))

    bnorm = float(np.linalg.norm(b))
    x = np.zeros(n)
    info = dict(iters=0, rel_resid=1.0 if bnorm > 0 else 0.0, normal_eq=0.0, stop_reason=0,
                history=[])
    if bnorm == 0.0:
        info["stop_reason"] = 3
        return x, info
    u = d * b
    beta = float(np.linalg.norm(u))
    if beta == 0.0:
        info["stop_reason"] = 3
        return x, info
    u = u / beta
    v = rmv(u)
    alpha = float(np.linalg.norm(v))
    if alpha == 0.0:
        info["stop_reason"] = 3
        return x, info
    v = v / alpha
    w = v.copy()
    phibar = beta
    rhobar = alpha
    anorm2 = 0.0
    it = 0
    while it < max_iter:
        it += 1
        # bidiagonalisation
        u = mv(v) - alpha * u
        beta_next = float(np.linalg.norm(u))
        anorm2 += alpha * alpha + beta_next * beta_next
        if beta_next > 0.0:
            u = u / beta_next
        v = rmv(u) - beta_next * v
        alpha_next = float(np.linalg.norm(v))
        if alpha_next > 0.0:
            v = v / alpha_next
        # plane rotation
        rho = float(np.hypot(rhobar, beta_next))
        c = rhobar / rho
        s = beta_next / rho
        theta = s * alpha_next
        rhobar = -c * alpha_next
        phi = c * phibar
        phibar = s * phibar
        # update x and w
        x = x + (phi / rho) * w
        w = v - (theta / rho) * w
        alpha = alpha_next
        normal_eq = alpha_next * abs(c) / np.sqrt(anorm2)
        breakdown = beta_next == 0.0 or alpha_next == 0.0
        if it % check_every == 0 or it == max_iter or breakdown:
            r = b - A @ (e * x)
            rel = float(np.linalg.norm(r)) / bnorm
            info["history"].append((it, rel))
            info.update(iters=it, rel_resid=rel, normal_eq=float(normal_eq))
            if rel <= tol:
                info["stop_reason"] = 1
                break
            if normal_eq <= tol:
                info["stop_reason"] = 2
                break
            if breakdown:
                info["stop_reason"] = 3
                break
    return e * x, info
