"""Pins for the exact solvers and the condition-number results (Sections 1, 2)."""
import numpy as np
import pytest
import scipy.special

from oracle import algorithm1 as A1
from oracle import theory
from workloads import scaled_dense


def test_sinkhorn_equilibrates_exactly():
    """Alternating minimisation (Section 2.1) gives row norms alpha and column norms beta."""
    A = scaled_dense(12, 8, 1.0, 31)
    al, be = A1.default_alpha_beta(12, 8)
    u, v, it = theory.sinkhorn_knopp(A, al, be)
    B = np.exp(u)[:, None] * A * np.exp(v)[None, :]
    assert np.allclose(np.linalg.norm(B, axis=1), al, rtol=1e-10)
    assert np.allclose(np.linalg.norm(B, axis=0), be, rtol=1e-10)
    # m alpha^2 = ||DAE||_F^2 = n beta^2
    assert np.sum(B * B) == pytest.approx(12 * al**2, rel=1e-10)
    # the optimality condition of (prob:equil): gradient with gamma = 0 vanishes
    gu, gv = theory.gradient(A, u, v, al, be, 0.0)
    assert np.max(np.abs(gu)) < 1e-9 and np.max(np.abs(gv)) < 1e-9


def test_sinkhorn_square_is_sinkhorn_knopp():
    """m = n, alpha = beta = 1: |DAE|^2 becomes doubly stochastic (Sinkhorn-Knopp)."""
    A = np.abs(scaled_dense(6, 6, 0.5, 32)) + 0.1
    u, v, _ = theory.sinkhorn_knopp(A, 1.0, 1.0)
    P = (np.exp(u)[:, None] * A * np.exp(v)[None, :]) ** 2
    assert np.allclose(P.sum(0), 1.0, atol=1e-10) and np.allclose(P.sum(1), 1.0, atol=1e-10)


def test_lambertw_exp_matches_library_and_equation():
    L = np.array([-3.0, 0.0, 1.0, 10.0, 100.0, 500.0])
    w = theory.lambertw_exp(L)
    assert np.allclose(w, np.real(scipy.special.lambertw(np.exp(L))), rtol=1e-14)
    Lb = np.array([700.0, 1e4, 1e8])
    wb = theory.lambertw_exp(Lb)
    assert np.allclose(wb + np.log(wb), Lb, rtol=1e-15)


def test_block_minimisation_agrees_with_newton():
    """Two independent exact solvers of (prob:reg-constr-equil) agree (Sections 2.3, 4)."""
    A = scaled_dense(15, 10, 1.0, 33)
    al, be = A1.default_alpha_beta(15, 10)
    ub, vb, _ = theory.bcd_regularized(A, al, be, 0.1, 10.0)
    un, vn, _ = theory.newton_regularized(A, al, be, 0.1)
    assert np.allclose(ub, un, atol=1e-9) and np.allclose(vb, vn, atol=1e-9)
    gu, gv = theory.gradient(A, ub, vb, al, be, 0.1)
    assert np.max(np.abs(gu)) < 1e-9 and np.max(np.abs(gv)) < 1e-9


def test_gauge_invariant_at_regularized_optimum():
    """Box inactive and m alpha^2 = n beta^2  =>  1^T u* = 1^T v* (Section 2.3)."""
    A = scaled_dense(9, 14, 1.0, 34)
    al, be = A1.default_alpha_beta(9, 14)
    u, v, _ = theory.newton_regularized(A, al, be, 0.1)
    assert np.abs(u).max() < 10 and np.abs(v).max() < 10
    assert u.sum() == pytest.approx(v.sum(), abs=1e-9)
    # product of D entries equals product of E entries
    assert np.sum(u) - np.sum(v) == pytest.approx(0.0, abs=1e-9)


def test_block_minimisation_with_active_box():
    """When the box is active, BCD returns the clipped coordinate minimiser."""
    A = scaled_dense(6, 5, 3.0, 35)
    al, be = A1.default_alpha_beta(6, 5)
    M = 1.0
    u, v, _ = theory.bcd_regularized(A, al, be, 0.1, M)
    assert np.abs(u).max() <= M + 1e-15 and np.abs(v).max() <= M + 1e-15
    gu, gv = theory.gradient(A, u, v, al, be, 0.1)
    # KKT: interior coordinates have zero gradient; at +M gradient <= 0, at -M >= 0
    for x, g in ((u, gu), (v, gv)):
        inner = np.abs(x) < M - 1e-12
        assert np.all(np.abs(g[inner]) < 1e-8)
        assert np.all(g[x >= M - 1e-12] <= 1e-8) and np.all(g[x <= -M + 1e-12] >= -1e-8)


def test_bcd_tends_to_sinkhorn_as_gamma_vanishes():
    """M = inf, m = n, alpha = beta = 1: as gamma -> 0 the regularised solution equilibrates
    (Section 2.3); compare in the gauge 1^T u = 1^T v."""
    A = scaled_dense(7, 7, 0.5, 36)
    us, vs, _ = theory.sinkhorn_knopp(A, 1.0, 1.0)
    c = 0.5 * (us.sum() - vs.sum()) / 7
    us, vs = us - c, vs + c
    errs = []
    for g in (1e-2, 1e-3):
        u, v, _ = theory.bcd_regularized(A, 1.0, 1.0, g, 1e6, iters=200000, tol=1e-13)
        errs.append(max(np.abs(u - us).max(), np.abs(v - vs).max()))
    assert errs[1] < errs[0] / 5 and errs[1] < 2e-2


def test_condition_bound_holds_on_random_matrices():
    """kappa <= 2 e^(-n/2) Phi(U) (Theorem 2.2), brute-force SVD."""
    rng = np.random.default_rng(37)
    for n in (2, 3, 5, 10, 30):
        for _ in range(5):
            U = rng.standard_normal((n, n)) * np.exp(rng.normal(0, 1, (n, 1)))
            assert np.log(theory.kappa(U)) <= theory.log_kappa_upper_bound(U) + 1e-12


def test_condition_bound_tight_case():
    """Singular values sqrt(2k^2/(1+k^2)), 1, ..., 1, sqrt(2/(1+k^2)) give
    Phi = (e^(n/2)/2)(kappa + 1/kappa) exactly (proof of Theorem 2.2)."""
    rng = np.random.default_rng(38)
    for n, k in ((3, 10.0), (8, 1e3), (5, 1.5)):
        s = np.ones(n)
        s[0] = np.sqrt(2 * k * k / (1 + k * k))
        s[-1] = np.sqrt(2 / (1 + k * k))
        Q1, _ = np.linalg.qr(rng.standard_normal((n, n)))
        Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
        U = Q1 @ np.diag(s) @ Q2
        assert theory.kappa(U) == pytest.approx(k, rel=1e-8)
        assert theory.log_phi(U) == pytest.approx(n / 2 + np.log((k + 1 / k) / 2), rel=1e-10)
        # within a factor 2 of kappa (inequality ineq:cond2)
        assert np.exp(theory.log_kappa_upper_bound(U)) <= 2 * k * (1 + 1e-9)


def test_psi_minimum_value():
    """min over sigma_n of exp(sigma_n^2 (1+k^2)/2)/(k sigma_n^2) = (e/2)(k + 1/k)
    at sigma_n^2 = 2/(1+k^2) (proof of Theorem 2.2), checked on a grid."""
    for k in (1.0, 3.0, 100.0):
        z = np.linspace(1e-4, 4 / (1 + k * k), 200001)
        f = np.exp(z * (1 + k * k) / 2) / (k * z)
        assert f.min() == pytest.approx(np.e / 2 * (k + 1 / k), rel=1e-8)
        assert z[np.argmin(f)] == pytest.approx(2 / (1 + k * k), rel=1e-3)


def test_equilibration_minimises_phi():
    """Theorem 2.1: the equilibrating (D, E) minimise Phi(DAE) over positive diagonals."""
    rng = np.random.default_rng(39)
    A = scaled_dense(6, 6, 1.0, 40)
    u, v, _ = theory.sinkhorn_knopp(A, 1.0, 1.0)
    base = theory.log_phi(np.exp(u)[:, None] * A * np.exp(v)[None, :])
    for _ in range(50):
        du, dv = rng.normal(0, 0.05, 6), rng.normal(0, 0.05, 6)
        pert = theory.log_phi(np.exp(u + du)[:, None] * A * np.exp(v + dv)[None, :])
        assert pert >= base - 1e-12


def test_norm_ratio_is_lower_bound_on_kappa():
    rng = np.random.default_rng(41)
    for _ in range(20):
        U = rng.standard_normal((5, 5)) * np.exp(rng.normal(0, 1, (1, 5)))
        cr, rr = theory.kappa_norm_ratio_lower_bound(U)
        k = theory.kappa(U)
        assert cr <= k * (1 + 1e-12) and rr <= k * (1 + 1e-12)
