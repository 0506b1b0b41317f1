"""Pins for the warm-start sketch reference (closed form and estimator behaviour)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import algorithm1 as A1
from oracle import warmstart as WS
from workloads import scaled_sparse, warmstart_matrix


def test_sketch_initialisation_equilibrates_rank_one_structure():
    """A = diag(a) S diag(b) with S = +-1: exact norms give exact equilibration."""
    rng = np.random.default_rng(1)
    m, n = 40, 20
    a, b = np.exp(rng.normal(0, 2, m)), np.exp(rng.normal(0, 2, n))
    A = a[:, None] * rng.choice([-1.0, 1.0], (m, n)) * b[None, :]
    al, be = A1.default_alpha_beta(m, n)
    r, c = (A * A).sum(1), (A * A).sum(0)
    u, v = WS.init_from_norms(r, c, al, n, 0.1, 50.0, be)
    B = np.exp(u)[:, None] * A * np.exp(v)[None, :]
    assert np.allclose(np.linalg.norm(B, axis=1), al, rtol=1e-12)
    assert np.allclose(np.linalg.norm(B, axis=0), be, rtol=1e-12)


def test_sketch_estimates_norms_unbiasedly():
    c = scaled_sparse(300, 200, 6, 1.0, 5)
    A = c.to_scipy()
    exact = np.asarray(A.multiply(A).sum(1)).ravel()
    errs = []
    for ks in (4, 64):
        r, _, _, _ = WS.sketch(A, 11, ks)
        errs.append(np.median(np.abs(r / exact - 1)))
    assert errs[1] < errs[0] / 2.5  # 1/sqrt(k) scaling: sqrt(16) = 4


def test_features_match_their_definition():
    c = warmstart_matrix(500, 250, 1.5, 7)
    A = c.to_scipy()
    al, be = A1.default_alpha_beta(500, 250)
    fr, fc, us, vs = WS.features(A, 3, 4, al, be, 0.1, 10.0)
    r, cc, rr, rc = WS.sketch(A, 3, 4)
    u2, v2 = WS.init_from_norms(r, cc, al, 250, 0.1, 10.0, be)
    assert np.allclose(us, u2) and np.allclose(vs, v2)
    assert np.allclose(fr[:, 1], us / 4) and np.allclose(fc[:, 1], vs / 4)
    assert np.all(fr[:, 4] == 1) and np.all(fc[:, 4] == 0)
    assert np.allclose(fr[:, 0].mean(), 0.0, atol=1e-12)
    assert fr.shape == (500, 8) and fc.shape == (250, 8)


def test_empty_rows_get_the_algorithm1_limit():
    A = sp.csr_matrix(np.array([[1.0, 2.0], [0.0, 0.0], [3.0, 0.0]]))
    fr, fc, us, vs = WS.features(A, 1, 4, 0.8, 1.1, 0.1, 5.0)
    assert us[1] == pytest.approx(min(0.8**2 / 0.1, 5.0))
