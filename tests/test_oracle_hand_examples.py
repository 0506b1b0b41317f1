"""Hand-worked examples that pin single oracle functions against values written out
by hand (not recomputed by the oracle's own vectorised code), each chosen so that a
plausible slip in that function fails it:

* Algorithm 1's update order (Section 3.2): both updates of step t use D and E of
  step t-1.  A Gauss-Seidel oracle (the v step from the new u, or the u step from the
  new v) reaches the same fixed points, so only a worked trajectory tells them apart.
* the warm-start feature map f0..f7, including an empty row;
* the relative optimality gap (f(u, v) - p*) / f(0, 0) of Section 4;
* the norm-ratio lower bound on the condition number (Section 1).
"""
import math

import numpy as np
import pytest

from oracle import algorithm1 as A1
from oracle import metrics, theory
from oracle import warmstart as WS

# 2 x 3 integer matrix and fixed one-probe sign blocks for steps 1 and 2
A23 = np.array([[1.0, 2.0, 0.0],
                [0.0, 1.0, 3.0]])
S_STEP = {1: [1.0, -1.0, 1.0], 2: [-1.0, 1.0, 1.0]}    # s (indexed by column)
W_STEP = {1: [1.0, 1.0], 2: [1.0, -1.0]}              # w (indexed by row)


def _fixed_probes(seed, batch, t, m, n, k):
    assert (m, n, k) == (2, 3, 1)
    return np.array(S_STEP[t])[:, None], np.array(W_STEP[t])[:, None]


def _hand_trajectory():
    """alpha = beta = gamma = 1, M = 50 (never active), u0 = v0 = 0, t0 = 0.

    Step 1 (tau = 1, eta = 2/(gamma (tau+1)) = 1, D = E = I):
      A s1 = (1 - 2, -1 + 3) = (-1, 2)              z_u = (1, 4)
      A' w1 = (1, 2 + 1, 3) = (1, 3, 3)             z_v = (1, 9, 9)
      u1 = -(z_u - 1) = (0, -3),   v1 = -(z_v - 1) = (0, -8, -8)
      u_bar1 = 2 u1 / 3 = (0, -2), v_bar1 = (0, -16/3, -16/3)
    Step 2 (tau = 2, eta = 2/3), E1 = diag(1, e^-8, e^-8), D1 = diag(1, e^-3):
      A E1 s2 = (-1 + 2 e^-8, e^-8 + 3 e^-8)
      z_u = e^(2 u1) (A E1 s2)^2 = ((1 - 2e^-8)^2, e^-6 16 e^-16)
      A' D1 w2 = (1, 2 - e^-3, -3 e^-3)
      z_v = e^(2 v1) (A' D1 w2)^2 = (1, e^-16 (2 - e^-3)^2, e^-16 9 e^-6)
      u2 = u1 - (2/3)(z_u - 1 + u1),  v2 = v1 - (2/3)(z_v - 1 + v1)
      u_bar2 = 2 u2 / 4 + 2 u_bar1 / 4
    """
    e = math.exp
    u1 = [0.0, -3.0]
    v1 = [0.0, -8.0, -8.0]
    ub1 = [0.0, -2.0]
    vb1 = [0.0, -16.0 / 3.0, -16.0 / 3.0]
    zu2 = [(1.0 - 2.0 * e(-8.0)) ** 2, 16.0 * e(-22.0)]
    zv2 = [1.0, e(-16.0) * (2.0 - e(-3.0)) ** 2, 9.0 * e(-22.0)]
    u2 = [u1[0] - (2.0 / 3.0) * (zu2[0] - 1.0 + u1[0]),
          u1[1] - (2.0 / 3.0) * (zu2[1] - 1.0 + u1[1])]
    v2 = [v1[0] - (2.0 / 3.0) * (zv2[0] - 1.0 + v1[0]),
          v1[1] - (2.0 / 3.0) * (zv2[1] - 1.0 + v1[1]),
          v1[2] - (2.0 / 3.0) * (zv2[2] - 1.0 + v1[2])]
    ub2 = [0.5 * u2[0] + 0.5 * ub1[0], 0.5 * u2[1] + 0.5 * ub1[1]]
    vb2 = [0.5 * v2[j] + 0.5 * vb1[j] for j in range(3)]
    return dict(u1=u1, v1=v1, ub1=ub1, vb1=vb1, u2=u2, v2=v2, ub2=ub2, vb2=vb2)


def test_algorithm1_two_steps_by_hand_jacobi_order(monkeypatch):
    monkeypatch.setattr(A1, "probes", _fixed_probes)
    h = _hand_trajectory()
    seen = {}
    A1.equilibrate(A23, 1.0, 1.0, 1.0, 50.0, 2, k=1,
                   on_step=lambda t, u, v, ub, vb: seen.__setitem__(t, (u.copy(), v.copy(), ub.copy(), vb.copy())))
    u, v, ub, vb = seen[1]
    np.testing.assert_allclose(u, h["u1"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(v, h["v1"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(ub, h["ub1"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(vb, h["vb1"], rtol=0, atol=1e-15)
    u, v, ub, vb = seen[2]
    np.testing.assert_allclose(u, h["u2"], rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(v, h["v2"], rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(ub, h["ub2"], rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(vb, h["vb2"], rtol=1e-14, atol=1e-15)
    # outputs after T = 2 are the averages
    out = A1.equilibrate(A23, 1.0, 1.0, 1.0, 50.0, 2, k=1)
    np.testing.assert_allclose(out["u_bar"], h["ub2"], rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(out["d"], np.exp(h["ub2"]), rtol=1e-14)
    np.testing.assert_allclose(out["e"], np.exp(h["vb2"]), rtol=1e-14)


def test_hand_trajectory_separates_jacobi_from_gauss_seidel():
    """The worked example is a real discriminator: the v step of step 1 taken from the
    new u1 = (0, -3) instead of u0 = 0 changes v1 by far more than rounding."""
    Dn = np.diag(np.exp([0.0, -3.0]))
    zv_gs = (A23.T @ Dn @ np.array(W_STEP[1])) ** 2
    v1_gs = -(zv_gs - 1.0)
    assert np.max(np.abs(v1_gs - np.array(_hand_trajectory()["v1"]))) > 1.0


def test_warmstart_features_by_hand(monkeypatch):
    """4 x 2 matrix with an empty last row, ks = 2 fixed sketch probes,
    alpha = 1, beta = sqrt(2) (m alpha^2 = n beta^2), gamma = 0.1, M = 20.

      S (columns x probes) = [[1, 1], [1, -1]],  W (rows x probes) = [[1, -1], [1, 1], [-1, 1], [1, 1]]
      A S = [[1, 1], [3, 1], [3, -3], [0, 0]]:   r = (1, 5, 9, 0),  max/mean = (1, 9/5, 1, -)
      A' W = [[3, 1], [-2, 4]]:                  c = (5, 10),       max/mean = (9/5, 8/5)
      F = (15 + 15)/2 = 15, cc = log(alpha^2 F / n)/4 = log(7.5)/4
      rows: l = (0, log 5, log 9) over the non-empty rows, mean = log(45)/3,
            sd = population std of (0, log 5, log 9); the empty row takes l = mean,
            s = min(alpha^2/gamma, M) = 10 and f7 = 0
      cols: l = (log 5, log 10), mean = log(50)/2, sd = log(2)/2
    """
    S = np.array([[1.0, 1.0], [1.0, -1.0]])
    W = np.array([[1.0, -1.0], [1.0, 1.0], [-1.0, 1.0], [1.0, 1.0]])

    def fake_signs(seed, batch, t, side, count, k):
        assert (t, k) == (0, 2)
        return {2: S, 3: W}[side][:count]

    monkeypatch.setattr(WS._signs, "signs", fake_signs)
    A = np.array([[1.0, 0.0], [2.0, 1.0], [0.0, 3.0], [0.0, 0.0]])
    al, be, g, M = 1.0, math.sqrt(2.0), 0.1, 20.0
    fr, fc, us, vs = WS.features(A, 0, 2, al, be, g, M)

    L = math.log
    cc = L(7.5) / 4.0
    lr = [0.0, L(5.0), L(9.0)]
    mr = L(45.0) / 3.0
    sdr = math.sqrt(sum((x - mr) ** 2 for x in lr) / 3.0)
    rows = [
        [(0.0 - mr) / 4, cc / 4, 0.0, sdr / 4, 1.0, L(2.0), cc, 0.0],
        [(L(5.0) - mr) / 4, (cc - 0.5 * L(5.0)) / 4, 0.0, sdr / 4, 1.0, L(2.0), cc, L(9.0 / 5.0)],
        [(L(9.0) - mr) / 4, (cc - 0.5 * L(9.0)) / 4, 0.0, sdr / 4, 1.0, L(2.0), cc, 0.0],
        [0.0, 10.0 / 4, 0.0, sdr / 4, 1.0, L(2.0), cc, 0.0],
    ]
    mc = L(50.0) / 2.0
    cols = [
        [(L(5.0) - mc) / 4, (cc - 0.5 * L(5.0)) / 4, L(2.0), L(2.0) / 8, 0.0, L(2.0), cc, L(9.0 / 5.0)],
        [(L(10.0) - mc) / 4, (cc - 0.5 * L(10.0)) / 4, L(2.0), L(2.0) / 8, 0.0, L(2.0), cc, L(8.0 / 5.0)],
    ]
    np.testing.assert_allclose(fr, rows, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(fc, cols, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(us, [cc, cc - 0.5 * L(5.0), cc - L(3.0), 10.0], rtol=1e-14)
    np.testing.assert_allclose(vs, [cc - 0.5 * L(5.0), cc - 0.5 * L(10.0)], rtol=1e-14)


def test_relative_gap_by_hand():
    """A = [[2]], alpha = beta = gamma = 1: f(0, 0) = A^2/2 = 2 and
    f(1/2, -1/4) = 2 e^(1/2) - 1/2 + 1/4 + (1/4 + 1/16)/2; with p* = 1 the gap is (f - 1)/2."""
    A = np.array([[2.0]])
    f = 2.0 * math.exp(0.5) - 0.5 + 0.25 + 0.5 * (0.25 + 0.0625)
    got = metrics.relative_gap(A, np.array([0.5]), np.array([-0.25]), 1.0, 1.0, 1.0, 1.0)
    assert got == pytest.approx((f - 1.0) / 2.0, rel=1e-15)


def test_norm_ratio_lower_bound_by_hand():
    """U = [[3, 0], [4, 1]]: column norms (5, 1), row norms (3, sqrt 17)."""
    col, row = theory.kappa_norm_ratio_lower_bound(np.array([[3.0, 0.0], [4.0, 1.0]]))
    assert col == pytest.approx(5.0, rel=1e-15)
    assert row == pytest.approx(math.sqrt(17.0) / 3.0, rel=1e-15)
    assert theory.kappa(np.array([[3.0, 0.0], [4.0, 1.0]])) >= max(col, row) * (1 - 1e-12)
