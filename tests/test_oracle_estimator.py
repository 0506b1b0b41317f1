"""Pins for the gradient, the randomized row-norm estimator and its moments (Section 3)."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import theory


def _all_signs(n):
    return np.array(list(itertools.product([-1.0, 1.0], repeat=n)))


def _tiny():
    # integer entries and integer log-scalings of 0 keep every product exact in FP64
    return np.array([[1.0, -2.0, 0.0, 3.0, 1.0],
                     [0.0, 1.0, 2.0, -1.0, 0.0],
                     [4.0, 0.0, -1.0, 0.0, 2.0],
                     [1.0, 1.0, 1.0, 1.0, -3.0]])


def test_estimator_unbiased_by_enumeration():
    """E[|B s|^2] = |B|^2 1 over all sign vectors (Section 3.1), exactly."""
    A = _tiny()
    m, n = A.shape
    u = np.zeros(m)
    v = np.zeros(n)
    al, be, ga = 0.7, 1.3, 0.1
    Ss, Ws = _all_signs(n), _all_signs(m)
    acc_u = np.zeros(m)
    acc_v = np.zeros(n)
    for s in Ss:
        for w in Ws:
            _, _, zu, zv = theory.gradient_estimate(A, u, v, s[:, None], w[:, None], al, be, ga)
            acc_u += zu
            acc_v += zv
    N = len(Ss) * len(Ws)
    # exact row/column squared norms written out for this integer matrix
    rows = np.array([1 + 4 + 0 + 9 + 1, 0 + 1 + 4 + 1 + 0, 16 + 0 + 1 + 0 + 4, 1 + 1 + 1 + 1 + 9], float)
    cols = np.array([1 + 0 + 16 + 1, 4 + 1 + 0 + 1, 0 + 4 + 1 + 1, 9 + 1 + 0 + 1, 1 + 0 + 4 + 9], float)
    assert np.array_equal(acc_u / N, rows)
    assert np.array_equal(acc_v / N, cols)
    gu, gv = theory.gradient(A, u, v, al, be, ga)
    assert np.allclose(gu, rows - al**2, rtol=0, atol=1e-14)
    assert np.allclose(gv, cols - be**2, rtol=0, atol=1e-14)


def test_estimator_unbiased_with_scalings():
    """Same, at non-zero (u, v): the mean of the estimator is the exact gradient."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((3, 4))
    u = rng.normal(0, 0.5, 3)
    v = rng.normal(0, 0.5, 4)
    Ss, Ws = _all_signs(4), _all_signs(3)
    acc = [np.zeros(3), np.zeros(4)]
    for s in Ss:
        for w in Ws:
            gu, gv, _, _ = theory.gradient_estimate(A, u, v, s[:, None], w[:, None], 1.0, 1.0, 0.3)
            acc[0] += gu
            acc[1] += gv
    N = len(Ss) * len(Ws)
    gu, gv = theory.gradient(A, u, v, 1.0, 1.0, 0.3)
    assert np.allclose(acc[0] / N, gu, rtol=1e-12, atol=1e-12)
    assert np.allclose(acc[1] / N, gv, rtol=1e-12, atol=1e-12)


def test_second_moment_constant_is_two():
    """E ||g~||^2 by enumeration matches the identity with constant 2, not the printed 3."""
    rng = np.random.default_rng(4)
    A = rng.standard_normal((3, 4))
    u = rng.normal(0, 0.3, 3)
    v = rng.normal(0, 0.3, 4)
    al, be, ga = 1.0, np.sqrt(3 / 4), 0.2
    Ss, Ws = _all_signs(4), _all_signs(3)
    tot = 0.0
    for s in Ss:
        for w in Ws:
            gu, gv, _, _ = theory.gradient_estimate(A, u, v, s[:, None], w[:, None], al, be, ga)
            tot += gu @ gu + gv @ gv
    enum = tot / (len(Ss) * len(Ws))
    closed = theory.second_moment(A, u, v, al, be, ga)
    assert enum == pytest.approx(closed, rel=1e-12)
    # the printed constant 3 would add sum r_i^2 + sum c_j^2 more
    S = theory.scaled_sq(A, u, v)
    extra = np.sum(S.sum(1) ** 2) + np.sum(S.sum(0) ** 2)
    assert abs(enum - (closed + extra)) > 1e-3 * enum


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((6, 4)) * np.exp(rng.normal(0, 1, (6, 1)))
    u = rng.normal(0, 0.5, 6)
    v = rng.normal(0, 0.5, 4)
    al, be, ga = 0.8, 1.1, 0.3
    gu, gv = theory.gradient(A, u, v, al, be, ga)
    h = 1e-6
    for i in range(6):
        e = np.zeros(6)
        e[i] = h
        fd = (theory.objective(A, u + e, v, al, be, ga) - theory.objective(A, u - e, v, al, be, ga)) / (2 * h)
        assert fd == pytest.approx(gu[i], rel=1e-7, abs=1e-7)
    for j in range(4):
        e = np.zeros(4)
        e[j] = h
        fd = (theory.objective(A, u, v + e, al, be, ga) - theory.objective(A, u, v - e, al, be, ga)) / (2 * h)
        assert fd == pytest.approx(gv[j], rel=1e-7, abs=1e-7)


def test_objective_sparse_equals_dense():
    rng = np.random.default_rng(6)
    A = rng.standard_normal((5, 7)) * (rng.random((5, 7)) < 0.4)
    u, v = rng.normal(0, 1, 5), rng.normal(0, 1, 7)
    f1 = theory.objective(A, u, v, 1.0, 0.9, 0.1)
    f2 = theory.objective(sp.csr_matrix(A), u, v, 1.0, 0.9, 0.1)
    assert f1 == pytest.approx(f2, rel=1e-13)


def test_multi_probe_estimate_is_mean_of_single_probes():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((5, 6))
    u, v = rng.normal(0, 0.4, 5), rng.normal(0, 0.4, 6)
    S = rng.choice([-1.0, 1.0], size=(6, 8))
    W = rng.choice([-1.0, 1.0], size=(5, 8))
    gu, gv, zu, zv = theory.gradient_estimate(A, u, v, S, W, 1.0, 1.0, 0.1)
    singles = [theory.gradient_estimate(A, u, v, S[:, [p]], W[:, [p]], 1.0, 1.0, 0.1) for p in range(8)]
    assert np.allclose(zu, np.mean([s[2] for s in singles], axis=0), rtol=1e-13)
    assert np.allclose(zv, np.mean([s[3] for s in singles], axis=0), rtol=1e-13)


def test_monte_carlo_converges_at_root_n():
    """Averages of N estimates approach the exact squared row norms like 1/sqrt(N)."""
    rng = np.random.default_rng(8)
    A = rng.standard_normal((20, 30))
    u, v = np.zeros(20), np.zeros(30)
    r_exact = (A * A).sum(1)
    errs = []
    for N in (64, 4096):
        S = rng.choice([-1.0, 1.0], size=(30, N))
        W = rng.choice([-1.0, 1.0], size=(20, N))
        _, _, zu, _ = theory.gradient_estimate(A, u, v, S, W, 1.0, 1.0, 0.1)
        errs.append(np.linalg.norm(zu - r_exact) / np.linalg.norm(r_exact))
    assert errs[1] < errs[0] / 4  # sqrt(64) = 8x fewer; allow slack
