"""FP64 reference of the warm-start sketch and features.  TEST INFRASTRUCTURE ONLY.

With ks Rademacher probes per side (stream sides 2 and 3, step 0) the estimator of
Section 3.1 at (u, v) = 0 gives r_i ~ ||row_i(A)||^2 and c_j ~ ||col_j(A)||^2.  For
A = diag(a) G diag(b) (G iid, unit variance) the scalings u_i = -1/2 log r_i + c,
v_j = -1/2 log c_j + c with e^(4c) = alpha^2 F / n equilibrate A in expectation (rows of
DAE then have squared norm n e^(4c)/F = alpha^2, columns m alpha^2 / n = beta^2); this is
the sketch initialisation.  Indices without entries get min(M, target/gamma), the point
where Algorithm 1 leaves them (Section 2.3).  Feature layout: see `features`.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import signs as _signs


def sketch(A, seed, ks=4, batch=0):
    """(r, c, ratio_r, ratio_c): mean over ks probes of the squared products, and the
    ratio max / mean (0 where the estimate is 0)."""
    A = sp.csr_matrix(A, dtype=np.float64) if sp.issparse(A) else np.asarray(A, dtype=np.float64)
    m, n = A.shape
    S = _signs.signs(seed, batch, 0, 2, n, ks)
    W = _signs.signs(seed, batch, 0, 3, m, ks)
    Y = np.asarray(A @ S) ** 2
    X = np.asarray(A.T @ W) ** 2
    r, c = Y.mean(axis=1), X.mean(axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        rr = np.where(r > 0, Y.max(axis=1) / r, 0.0)
        rc = np.where(c > 0, X.max(axis=1) / c, 0.0)
    return r, c, rr, rc


def init_from_norms(r, c, alpha, n, gamma, M, beta=None):
    """Sketch initialisation from (estimated) squared row and column norms r, c."""
    F = 0.5 * (np.sum(r) + np.sum(c))
    cc = 0.25 * np.log(alpha**2 * F / n)
    beta = alpha * np.sqrt(len(r) / n) if beta is None else beta
    u = np.full(np.shape(r), min(alpha**2 / gamma, M))
    v = np.full(np.shape(c), min(beta**2 / gamma, M))
    u[r > 0] = -0.5 * np.log(r[r > 0]) + cc
    v[c > 0] = -0.5 * np.log(c[c > 0]) + cc
    return np.clip(u, -M, M), np.clip(v, -M, M)


def features(A, seed, ks, alpha, beta, gamma, M, batch=0):
    """Features (rows [m, 8], columns [n, 8]) and sketch initialisations (u_s, v_s):
      f0 = (l - mean l)/4, l = log of the estimate (mean over the side's non-empty indices)
      f1 = s/4 (sketch initialisation), f2 = log target, f3 = std l / 4, f4 = is_row,
      f5 = log(m/n), f6 = c, f7 = log(max_p y_p^2 / mean_p y_p^2) (0 if empty)."""
    m, n = A.shape
    r, c, rr, rc = sketch(A, seed, ks, batch)
    F = 0.5 * (r.sum() + c.sum())
    cc = 0.25 * np.log(alpha**2 * F / n) if F > 0 else 0.0

    def side(est, ratio, tgt, is_row):
        nz = est > 0
        l_nz = np.log(est[nz])
        mean = l_nz.mean() if nz.any() else 0.0
        sd = l_nz.std() if nz.any() else 0.0
        l = np.full(est.shape, mean)
        l[nz] = l_nz
        s = np.full(est.shape, min(tgt / gamma, M))
        s[nz] = -0.5 * l_nz + cc
        s = np.clip(s, -M, M)
        f = np.zeros((est.size, 8))
        f[:, 0] = (l - mean) / 4.0
        f[:, 1] = s / 4.0
        f[:, 2] = np.log(tgt)
        f[:, 3] = sd / 4.0
        f[:, 4] = 1.0 if is_row else 0.0
        f[:, 5] = np.log(m / n)
        f[:, 6] = cc
        with np.errstate(divide="ignore"):
            f[:, 7] = np.where(ratio > 0, np.log(np.where(ratio > 0, ratio, 1.0)), 0.0)
        return f, s

    fr, us = side(r, rr, alpha**2, True)
    fc, vs = side(c, rc, beta**2, False)
    return fr, fc, us, vs
