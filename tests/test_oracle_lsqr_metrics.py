"""Pins for the LSQR consumer (Section 5.1) and the RMS equilibration error (Section 4)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import algorithm1 as A1
from oracle import lsqr as L
from oracle import metrics, theory
from workloads import rhs_consistent, rhs_noisy, scaled_dense, scaled_sparse


def test_lsqr_iterates_match_scipy():
    """Same Golub-Kahan recurrences: the k-th iterate equals scipy's with iter_lim = k.

    Krylov recurrences amplify rounding differences (loss of orthogonality), so the
    comparison is tight for a well-conditioned A and early iterations only."""
    A = scaled_sparse(80, 50, 5, 0.3, 51).to_scipy()
    b, _ = rhs_noisy(A, 52, noise=1e-2)
    for k, tol in ((1, 1e-13), (3, 1e-13), (10, 1e-11), (25, 1e-4)):
        x, info = L.lsqr(A, b, tol=0.0, max_iter=k)
        xs = spla.lsqr(A, b, atol=0, btol=0, conlim=0, iter_lim=k)[0]
        assert np.max(np.abs(x - xs)) <= tol * np.abs(xs).max()
        assert info["iters"] == k


def test_lsqr_converges_to_least_squares_solution():
    A = scaled_dense(60, 20, 0.5, 53)
    b, _ = rhs_noisy(A, 54, noise=0.1)
    x, info = L.lsqr(A, b, tol=1e-13, max_iter=500)
    xl = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.allclose(x, xl, rtol=1e-8, atol=1e-10)
    assert info["stop_reason"] == 2


def test_scaled_lsqr_solves_consistent_system():
    """(DAE) x_bar = D b, x = E x_bar recovers x* of a consistent system (Section 5.1)."""
    A = scaled_dense(40, 25, 1.0, 55)
    b, xs = rhs_consistent(A, 56)
    al, be = A1.default_alpha_beta(40, 25)
    o = A1.equilibrate(A, al, be, 0.1, 10.0, 200, seed=3)
    x, info = L.lsqr(A, b, o["d"], o["e"], tol=1e-10, max_iter=2000)
    assert info["stop_reason"] == 1
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) <= 1e-10
    assert np.allclose(x, xs, rtol=1e-6, atol=1e-6)


def test_equilibration_speeds_up_lsqr():
    """Qualitative claim of Section 5.1: fewer LSQR iterations after equilibration
    (the paper's matrices and seeds are not available, so no counts are compared)."""
    csr = scaled_sparse(400, 400, 8, 1.0, 57)
    A = csr.to_scipy()
    b, _ = rhs_consistent(A, 58)
    al, be = A1.default_alpha_beta(400, 400)
    _, plain = L.lsqr(A, b, tol=1e-4, max_iter=20000)
    o = A1.equilibrate(A, al, be, 0.1, np.log(1e4), 100, seed=4)
    _, pre = L.lsqr(A, b, o["d"], o["e"], tol=1e-4, max_iter=20000)
    assert pre["stop_reason"] == 1
    assert pre["iters"] < plain["iters"]


def test_lsqr_zero_rhs_and_breakdown():
    A = scaled_dense(5, 3, 0.5, 59)
    x, info = L.lsqr(A, np.zeros(5))
    assert np.all(x == 0) and info["stop_reason"] == 3
    # A with one column: exact after one iteration (alpha_2 = 0)
    a = np.arange(1.0, 6.0)[:, None]
    x, info = L.lsqr(a, 2 * a[:, 0], max_iter=10, tol=0.0)
    assert x[0] == pytest.approx(2.0, rel=1e-14)
    assert info["stop_reason"] in (1, 3)


def test_rms_error_zero_when_equilibrated():
    A = scaled_dense(10, 6, 1.0, 60)
    al, be = A1.default_alpha_beta(10, 6)
    u, v, _ = theory.sinkhorn_knopp(A, al, be)
    rms, _ = metrics.rms_equilibration_error(A, u, v, al, be)
    assert rms < 1e-10


def test_rms_error_hand_example():
    """A = diag(3, 4) with D = E = I: rows have norms 3, 4 and columns 3, 4."""
    A = np.diag([3.0, 4.0])
    rms, _ = metrics.rms_equilibration_error(A, np.zeros(2), np.zeros(2), 1.0, 1.0)
    assert rms == pytest.approx(np.sqrt((4 + 9 + 4 + 9) / 4.0), rel=1e-15)
    rms2, _ = metrics.rms_equilibration_error(sp.csr_matrix(A), np.log([1 / 3, 1 / 4]), np.zeros(2), 1.0, 1.0)
    # rows now have norm 1; columns too
    assert rms2 == pytest.approx(0.0, abs=1e-15)


def test_rms_error_skips_empty():
    A = np.array([[1.0, 0.0], [0.0, 0.0]])
    rms, n_empty = metrics.rms_equilibration_error(A, np.zeros(2), np.zeros(2), 1.0, 1.0, skip_empty=True)
    assert n_empty == 2 and rms == 0.0
    rms_all, _ = metrics.rms_equilibration_error(A, np.zeros(2), np.zeros(2), 1.0, 1.0)
    assert rms_all == pytest.approx(np.sqrt(2 / 4))
