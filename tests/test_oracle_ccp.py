"""Pins for the CCP Lasso oracle (Section 5.2): proximal maps against direct numerical
minimisation, the limit against scikit-learn's coordinate-descent Lasso and the
optimality (KKT) conditions, with and without equilibration."""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from oracle import algorithm1 as A1
from oracle import ccp
from workloads import lasso_rhs, paper_sparse


def _problem(m=60, n=90, seed=3):
    A = paper_sparse(m, n, 0.2, seed).to_scipy()
    b, _ = lasso_rhs(A, seed + 1)
    return A, b, ccp.default_lambda(A, b)


def test_prox_maps_match_numerical_minimisation():
    rng = np.random.default_rng(0)
    lam, sigma, tau = 0.7, 0.3, 0.45
    for _ in range(20):
        d, e, b = rng.uniform(0.2, 3.0), rng.uniform(0.2, 3.0), rng.normal()
        v, u = rng.normal(0, 3), rng.normal(0, 3)
        # dual prox through Moreau: prox_{sigma g*}(v) = v - sigma prox_{g/sigma}(v/sigma),
        # with gbar(y) = (y/d - b)^2 / sqrt(lam) minimised directly
        w = v / sigma
        res = minimize_scalar(lambda y: (y / d - b) ** 2 / np.sqrt(lam) + 0.5 * sigma * (y - w) ** 2,
                              bracket=(w - 10, w + 10), tol=1e-14)
        ref = v - sigma * res.x
        got = ccp.prox_dual(np.array([v]), sigma, np.array([d]), np.array([b]), lam)[0]
        assert abs(got - ref) < 1e-7 * max(1.0, abs(ref))
        res = minimize_scalar(lambda x: tau * np.sqrt(lam) * e * abs(x) + 0.5 * (x - u) ** 2,
                              bounds=(u - 10, u + 10), method="bounded", options={"xatol": 1e-12})
        got = ccp.prox_primal(np.array([u]), tau, np.array([e]), lam)[0]
        assert abs(got - res.x) < 1e-7


def test_objective_and_lambda():
    A, b, lam = _problem()
    assert np.isclose(ccp.objective(A, b, lam, np.zeros(A.shape[1])), (b @ b) / np.sqrt(lam))
    assert np.isclose(lam, 1e-3 * np.abs(A.T @ b).max())
    assert np.isclose(ccp.op_norm(A), np.sqrt(np.linalg.eigvalsh((A.T @ A).toarray()).max()), rtol=1e-10)


@pytest.mark.parametrize("equilibrated", [False, True])
def test_ccp_reaches_the_lasso_optimum(equilibrated):
    """The CCP limit, with and without equilibration, is the Lasso solution of
    scikit-learn's coordinate descent (alpha = lam / (2 m), which rescales the same
    objective), and satisfies the optimality conditions."""
    from sklearn.linear_model import Lasso

    A, b, lam = _problem()
    m, n = A.shape
    d = e = None
    if equilibrated:
        al, be = A1.default_alpha_beta(m, n)
        out = A1.equilibrate(A, al, be, 0.1, np.log(1e4), 100, k=1, seed=7)
        d, e = out["d"], out["e"]
    res = ccp.ccp_lasso(A, b, lam, 20000, d=d, e=e)
    x = res["x"]
    sk = Lasso(alpha=lam / (2 * m), fit_intercept=False, tol=1e-14, max_iter=200000).fit(A.toarray(), b)
    p_sk = ccp.objective(A, b, lam, sk.coef_)
    p = ccp.objective(A, b, lam, x)
    assert abs(p - p_sk) <= 1e-9 * p_sk
    assert np.max(np.abs(x - sk.coef_)) < 1e-5
    # KKT: (2/sqrt(lam)) A'(Ax - b) + sqrt(lam) s = 0 with s in the subdifferential of ||.||_1
    g = (2.0 / np.sqrt(lam)) * np.asarray(A.T @ (A @ x - b)).ravel()
    nz = np.abs(x) > 1e-9
    assert np.max(np.abs(g[nz] + np.sqrt(lam) * np.sign(x[nz]))) < 1e-5 * np.sqrt(lam)
    assert np.max(np.abs(g[~nz])) <= np.sqrt(lam) * (1 + 1e-5)


def test_equilibration_does_not_change_the_problem():
    """x = E xbar: the equilibrated iteration solves the same problem (same optimum),
    and with D = E = I it is the plain iteration."""
    A, b, lam = _problem(40, 70, 5)
    r1 = ccp.ccp_lasso(A, b, lam, 50)
    r2 = ccp.ccp_lasso(A, b, lam, 50, d=np.ones(40), e=np.ones(70))
    assert np.array_equal(r1["x"], r2["x"])


def test_sparse_norm_path_equals_dense_svd():
    """The operator norm of large sparse inputs (ARPACK partial SVD) is the dense SVD's."""
    A = paper_sparse(2100, 2200, 0.01, 9).to_scipy()
    d = np.exp(np.random.default_rng(1).normal(0, 0.5, 2100))
    ref = np.linalg.svd(d[:, None] * A.toarray(), compute_uv=False)[0]
    assert abs(ccp.op_norm(A, d=d) - ref) <= 1e-12 * ref
