"""Pins for the oracle's Section 6 variants (symmetric, varying norms, block) against
Algorithm 1's pinned oracle, sign enumeration, finite differences, closed forms and an
independent Newton solve."""
import itertools

import numpy as np
import pytest

from oracle import algorithm1 as A1
from oracle import theory
from oracle import variants as V
from workloads import scaled_dense, scaled_sparse


def _fd_grad(f, x, h=1e-6):
    g = np.zeros_like(x)
    for i in range(len(x)):
        e = np.zeros_like(x)
        e[i] = h
        g[i] = (f(x + e) - f(x - e)) / (2 * h)
    return g


def _all_signs(count):
    return [np.array(s, dtype=np.float64) for s in itertools.product((1.0, -1.0), repeat=count)]


A_INT = np.array([[1, -2, 0, 3, 1],
                  [0, 1, 2, -1, 0],
                  [2, 0, -1, 1, 3],
                  [-1, 1, 1, 0, 2]], dtype=np.float64)
ROW_PTR = [0, 1, 4]          # blocks of 1 and 3 rows
COL_PTR = [0, 2, 3, 5]       # blocks of 2, 1 and 2 columns


@pytest.mark.parametrize("A", [scaled_dense(30, 20, 1.0, 5), scaled_sparse(300, 120, 5, 1.5, 6).to_scipy()])
@pytest.mark.parametrize("k,t0", [(1, 0), (4, 9)])
def test_singletons_with_uniform_targets_equal_algorithm1(A, k, t0):
    """No blocks and targets alpha^2, beta^2: the variant oracle is Algorithm 1, bit for bit."""
    m, n = A.shape
    al, be = A1.default_alpha_beta(m, n)
    ref = A1.equilibrate(A, al, be, 0.1, 10.0, 25, k=k, seed=3, t0=t0)
    out = V.equilibrate_general(A, 0.1, 10.0, 25, k=k, seed=3, t0=t0, alpha=al, beta=be)
    for key in ("u_bar", "v_bar", "u", "v", "d", "e"):
        assert np.array_equal(out[key], ref[key])
    # explicit per-index targets equal to alpha^2 give the same run
    out2 = V.equilibrate_general(A, 0.1, 10.0, 25, k=k, seed=3, t0=t0,
                                 row_target=np.full(m, al**2), col_target=np.full(n, be**2))
    assert np.array_equal(out2["u_bar"], ref["u_bar"])


def test_block_estimator_unbiased_by_enumeration():
    """Mean of the block / varying-norm estimate over all 2^5 x 2^4 sign vectors (k = 1)
    equals the exact gradient, which matches finite differences of the objective."""
    rng = np.random.default_rng(1)
    rt = rng.uniform(0.5, 2.0, 4)
    ct = rng.uniform(0.5, 2.0, 5)
    u = np.array([0.3, -0.2])
    v = np.array([0.1, -0.4, 0.25])
    kw = dict(row_ptr=ROW_PTR, col_ptr=COL_PTR, row_target=rt, col_target=ct, gamma=0.3)
    gu_sum = np.zeros(2)
    gv_sum = np.zeros(3)
    cnt = 0
    for S in _all_signs(5):
        for W in _all_signs(4):
            gu, gv, _, _ = V.general_gradient_estimate(A_INT, u, v, S[:, None], W[:, None], **kw)
            gu_sum += gu
            gv_sum += gv
            cnt += 1
    gu_ex, gv_ex = V.general_gradient(A_INT, u, v, **kw)
    assert np.allclose(gu_sum / cnt, gu_ex, rtol=1e-13, atol=1e-13)
    assert np.allclose(gv_sum / cnt, gv_ex, rtol=1e-13, atol=1e-13)
    fu = _fd_grad(lambda x: V.general_objective(A_INT, x, v, **kw), u)
    fv = _fd_grad(lambda x: V.general_objective(A_INT, u, x, **kw), v)
    assert np.allclose(fu, gu_ex, rtol=1e-7, atol=1e-7)
    assert np.allclose(fv, gv_ex, rtol=1e-7, atol=1e-7)


def test_block_problem_is_problem_of_block_norm_matrix():
    """With the scaling constant on blocks, the block problem of A has the objective and
    gradient of the unblocked problem of the matrix of block norms, with the blocks'
    summed targets (computed through a different route: explicit compression)."""
    rng = np.random.default_rng(2)
    A = scaled_dense(9, 7, 1.0, 8)
    rp, cp = [0, 2, 3, 7, 9], [0, 3, 4, 7]
    rt = rng.uniform(0.5, 2.0, 9)
    ct = rng.uniform(0.5, 2.0, 7)
    u = rng.normal(0, 0.5, 4)
    v = rng.normal(0, 0.5, 3)
    C = V.compress(A, rp, cp)
    rtc = np.array([rt[0:2].sum(), rt[2:3].sum(), rt[3:7].sum(), rt[7:9].sum()])
    ctc = np.array([ct[0:3].sum(), ct[3:4].sum(), ct[4:7].sum()])
    kwb = dict(row_ptr=rp, col_ptr=cp, row_target=rt, col_target=ct, gamma=0.2)
    kwc = dict(row_target=rtc, col_target=ctc, gamma=0.2)
    assert np.isclose(V.general_objective(A, u, v, **kwb), V.general_objective(C, u, v, **kwc), rtol=1e-13)
    gb = V.general_gradient(A, u, v, **kwb)
    gc = V.general_gradient(C, u, v, **kwc)
    assert np.allclose(gb[0], gc[0], rtol=1e-12, atol=1e-13)
    assert np.allclose(gb[1], gc[1], rtol=1e-12, atol=1e-13)


def _vary_diag_optimum(a, R, C, gamma):
    """Diagonal square A with squared targets R_i, C_i: a^2 e^(2u+2v) - R + gamma u = 0 and
    a^2 e^(2u+2v) - C + gamma v = 0 give u - v = (R - C)/gamma and, with s = u + v and
    P = R + C, s = P/gamma - W((4a^2/gamma) e^(2P/gamma))/2."""
    P = R + C
    s = P / gamma - 0.5 * theory.lambertw_exp(np.log(4.0 * a**2 / gamma) + 2.0 * P / gamma)
    d = (R - C) / gamma
    return 0.5 * (s + d), 0.5 * (s - d)


def test_varying_norms_diagonal_reaches_closed_form():
    """One nonzero per row and column: the estimate is sign-independent, the method is
    projected gradient descent and converges to the closed-form optimum."""
    a = np.array([0.05, 0.4, 1.0, 3.0, 20.0])
    R = np.array([0.6, 1.0, 1.4, 0.8, 1.2])
    C = np.array([1.1, 0.7, 1.0, 1.3, 0.9])
    gamma = 0.5
    us, vs = _vary_diag_optimum(a, R, C, gamma)
    assert np.all(np.abs(us) < 10) and np.all(np.abs(vs) < 10)
    # the u - v mode has curvature gamma, so with eta gamma = 2/(t+1) its error falls
    # like 2/(T(T+1)): about 1e-6 after 1500 steps, 4x less after twice as many
    errs = []
    for T in (1500, 3000):
        out = V.equilibrate_general(np.diag(a), gamma, 10.0, T, k=1, seed=4, row_target=R, col_target=C)
        errs.append(max(np.max(np.abs(out["u"] - us)), np.max(np.abs(out["v"] - vs))))
    assert errs[0] < 1e-5
    assert 3.5 < errs[0] / errs[1] < 4.5, errs
    g = V.general_gradient(np.diag(a), us, vs, row_target=R, col_target=C, gamma=gamma)
    assert np.max(np.abs(g[0])) < 1e-10 and np.max(np.abs(g[1])) < 1e-10
    # sign independence: another seed gives the same run
    out2 = V.equilibrate_general(np.diag(a), gamma, 10.0, 50, k=3, seed=99, row_target=R, col_target=C)
    out3 = V.equilibrate_general(np.diag(a), gamma, 10.0, 50, k=3, seed=5, row_target=R, col_target=C)
    assert np.allclose(out2["u_bar"], out3["u_bar"], rtol=0, atol=1e-14)


def test_block_sgd_approaches_newton_optimum_of_block_norm_matrix():
    """Equal-size row blocks make every block target 2 alpha^2, so the block optimum is the
    regularised optimum of the block-norm matrix with alpha' = sqrt(2) alpha, found by
    Newton's method (theory).  The block SGD average approaches it (fixed seed)."""
    A = scaled_dense(12, 8, 0.7, 21)
    rp = list(range(0, 13, 2))
    al, be = 1.0, np.sqrt(12 / 8 / 2) * np.sqrt(2)   # 6 alpha'^2 = 8 beta^2 with alpha'^2 = 2
    ur, vr, _ = theory.newton_regularized(V.compress(A, rp, None), np.sqrt(2) * al, be, 0.1)
    out = V.equilibrate_general(A, 0.1, 10.0, 4000, k=16, seed=8, row_ptr=rp, alpha=al, beta=be)
    err = max(np.max(np.abs(out["u_bar"] - ur)), np.max(np.abs(out["v_bar"] - vr)))
    assert err < 0.05, err
    # and it is far closer than the start
    assert err < 0.2 * max(np.max(np.abs(ur)), np.max(np.abs(vr)))


A_SYM = np.array([[2, -1, 0, 3],
                  [-1, 0, 2, 1],
                  [0, 2, 1, -2],
                  [3, 1, -2, 1]], dtype=np.float64)


def test_symmetric_estimator_unbiased_by_enumeration():
    """Algorithm 2: the mean of |DADs|^2 - alpha^2 + gamma u over all 2^4 sign vectors is
    the exact gradient, which matches finite differences of the symmetric objective."""
    u = np.array([0.2, -0.3, 0.1, 0.4])
    acc = np.zeros(4)
    S_all = _all_signs(4)
    for S in S_all:
        acc += V.sym_gradient_estimate(A_SYM, u, S[:, None], 1.3, 0.2)[0]
    g = V.sym_gradient(A_SYM, u, 1.3, 0.2)
    assert np.allclose(acc / len(S_all), g, rtol=1e-13, atol=1e-13)
    assert np.allclose(_fd_grad(lambda x: V.sym_objective(A_SYM, x, 1.3, 0.2), u), g, rtol=1e-7, atol=1e-7)


def test_symmetric_optimum_is_standard_optimum():
    """For symmetric A and alpha = beta the regularised standard problem at u = v is twice
    the symmetric one and its unique optimum has u = v, so Newton's u* (theory) zeroes
    the symmetric gradient."""
    rng = np.random.default_rng(3)
    G = rng.normal(size=(7, 7)) * np.exp(rng.normal(0, 0.8, 7))[:, None]
    A = G + G.T
    u, v, _ = theory.newton_regularized(A, 1.0, 1.0, 0.1)
    assert np.max(np.abs(u - v)) < 1e-9
    g_std = theory.gradient(A, u, v, 1.0, 1.0, 0.1)
    g_sym = V.sym_gradient(A, u, 1.0, 0.1)
    # zero up to Newton's own stopping point, where the standard gradient is as small
    assert np.max(np.abs(g_sym)) < 1e-6
    assert np.max(np.abs(g_sym)) < 10 * max(np.max(np.abs(g_std[0])), 1e-12)
    # at any point u = v the two gradients coincide
    w = rng.normal(0, 0.5, 7)
    for gs in theory.gradient(A, w, w, 1.0, 1.0, 0.1):
        assert np.allclose(V.sym_gradient(A, w, 1.0, 0.1), gs, rtol=1e-13, atol=1e-13)
    assert np.isclose(theory.objective(A, u, u, 1.0, 1.0, 0.1), 2 * V.sym_objective(A, u, 1.0, 0.1), rtol=1e-13)


def test_symmetric_diagonal_reaches_closed_form():
    """Diagonal A: z_i = a_i^2 e^(4 u_i) does not depend on the signs; the fixed point
    a^2 e^(4x) = alpha^2 - gamma x is x = (alpha^2 - q)/gamma, q = (gamma/4) W((4a^2/gamma)
    e^(4 alpha^2/gamma))."""
    a = np.array([0.01, 0.3, 1.0, 2.0, 50.0])
    gamma, al = 0.1, 1.2
    q = (gamma / 4.0) * theory.lambertw_exp(np.log(4.0 * a**2 / gamma) + 4.0 * al**2 / gamma)
    xs = (al**2 - q) / gamma
    out = V.equilibrate_symmetric(np.diag(a), al, gamma, 12.0, 1000, k=2, seed=1)
    assert np.max(np.abs(out["u"] - xs)) < 1e-12
    assert np.max(np.abs(V.sym_gradient(np.diag(a), xs, al, gamma))) < 1e-11


def test_symmetric_sgd_approaches_optimum():
    """Algorithm 2's average approaches the Newton optimum (fixed seed, k = 16)."""
    rng = np.random.default_rng(4)
    G = rng.normal(size=(10, 10)) * np.exp(rng.normal(0, 0.7, 10))[:, None]
    A = G + G.T
    u, _, _ = theory.newton_regularized(A, 1.0, 1.0, 0.1)
    out = V.equilibrate_symmetric(A, 1.0, 0.1, 10.0, 4000, k=16, seed=2)
    err = np.max(np.abs(out["u_bar"] - u))
    assert err < 0.05, err


def test_block_pointers_validated():
    with pytest.raises(ValueError):
        V.block_sizes([0, 2, 2, 4], 4)
    with pytest.raises(ValueError):
        V.block_sizes([1, 4], 4)
    with pytest.raises(ValueError):
        V.equilibrate_general(A_INT, 0.1, 10.0, 1, row_target=-np.ones(4))
