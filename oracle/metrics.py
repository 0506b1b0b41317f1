"""Quality measures of Section 4 (FP64).  TEST INFRASTRUCTURE ONLY."""
from __future__ import annotations

import numpy as np

from .theory import objective, row_col_sq_norms


def rms_equilibration_error(A, u, v, alpha, beta, skip_empty=False):
    """RMS equilibration error of DAE (Section 4):

        (1/sqrt(m+n)) * sqrt( sum_i (sqrt(r_i) - alpha)^2 + sum_j (sqrt(c_j) - beta)^2 )

    with r, c the row and column squared norms of DAE.  With skip_empty, rows and
    columns of A with no nonzero are left out (they cannot be equilibrated) and
    the normaliser counts only the remaining ones.  Returns (rms, n_empty).
    """
    r, c = row_col_sq_norms(A, u, v)
    if skip_empty:
        r0, c0 = row_col_sq_norms(A, np.zeros_like(u), np.zeros_like(v))
        rk, ck = r0 > 0, c0 > 0
        n_empty = int((~rk).sum() + (~ck).sum())
        r, c = r[rk], c[ck]
    else:
        n_empty = 0
    s = np.sum((np.sqrt(r) - alpha) ** 2) + np.sum((np.sqrt(c) - beta) ** 2)
    return float(np.sqrt(s / (r.size + c.size))), n_empty


def relative_gap(A, u, v, alpha, beta, gamma, p_star):
    """(f(u, v) - p*) / f(0, 0) (Section 4)."""
    f0 = objective(A, np.zeros(A.shape[0]), np.zeros(A.shape[1]), alpha, beta, gamma)
    return (objective(A, u, v, alpha, beta, gamma) - p_star) / f0
