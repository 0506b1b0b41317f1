"""GPU parity of the dense bfloat16 MFMA path.

The problem is rounded once, FP64 -> bf16 (round-to-nearest-even), and the oracle runs
in FP64 on the rounded matrix.  The GPU's own arithmetic error comes from the probe
operand (exact sign times the two-term scale hi + lo, hi = bf16(e^v), lo = bf16(e^v - hi):
relative error <= 2^-16) and FP32 accumulation.

Checks:
  * whole runs long enough for the averaged output to be well posed (T >= 500): the
    early steps of Algorithm 1 amplify any perturbation chaotically, and their weight in
    u_bar decays like 1/T^2 -- on short runs even the oracle on the FP64 matrix and the
    oracle on the rounded matrix differ by O(0.1-1) (measured), so those runs say nothing
    about the kernel; the 2e-2 bound is asserted on the long ones.
  * one step from oracle states (any size, including the full 16384 x 8192): the GPU
    result must lie within a rigorous bound derived from the two rounding sources.
  * the benchmarked workload at full size (16384 x 8192, sigma = 3, k = 64): 10 whole
    steps at gamma = 1, where the oracle is well posed (its own spread under 1e-16
    perturbations is 4e-11), elementwise at 5e-3; and the benchmarked 500-step run at
    gamma = 0.1 against the stored oracle result (tests/golden/make_long_runs.py) at 2e-2.
"""
import os
import sys

import numpy as np
import pytest
import torch

from oracle import algorithm1 as A1
from workloads import round_to_bf16, scaled_dense

pytestmark = pytest.mark.gpu
TOL = 2e-2


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _bf16(A):
    from paper_1602_06621_amd import Dense

    bits, vals = round_to_bf16(A)
    return Dense(torch.tensor(bits.view(np.int16), device="cuda")), vals


@pytest.mark.parametrize("m,n,k,T", [(300, 170, 16, 1000), (1024, 512, 64, 500), (1000, 333, 40, 600)])
def test_bf16_whole_run(m, n, k, T):
    from paper_1602_06621_amd import equilibrate

    A = scaled_dense(m, n, 3.0, 300 + k)
    D, Ab = _bf16(A)
    al, be = A1.default_alpha_beta(m, n)
    g = equilibrate(D, al, be, 0.1, 10.0, T, k, 17)
    o = A1.equilibrate(Ab, al, be, 0.1, 10.0, T, k=k, seed=17)
    ub, vb = g["u_bar"].cpu().numpy(), g["v_bar"].cpu().numpy()
    err = max(np.abs(ub - o["u_bar"]).max(), np.abs(vb - o["v_bar"]).max())
    o64 = A1.equilibrate(A, al, be, 0.1, 10.0, T, k=k, seed=17)
    prob = max(np.abs(o64["u_bar"] - o["u_bar"]).max(), np.abs(o64["v_bar"] - o["v_bar"]).max())
    _say(f"bf16 {m}x{n} k={k} T={T}: arithmetic error {err:.3e}, problem rounding {prob:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("m,n,k,T,sigma", [(1024, 512, 64, 300, 3.0), (300, 170, 16, 600, 3.0),
                                           (1000, 333, 40, 300, 1.0)])
def test_bf16_whole_run_without_chaos(m, n, k, T, sigma):
    """With gamma = 1 the iteration contracts perturbations, so a whole run stays within
    the bf16 path's per-step arithmetic error of the oracle on the rounded matrix
    (measured 1.8e-4 to 1.9e-3) while the oracle with another seed lands 2.4e-2 to 3.2e-2
    away: 5e-3 checks every step's probes and update, not only the statistics."""
    from paper_1602_06621_amd import equilibrate

    A = scaled_dense(m, n, sigma, 300 + k)
    D, Ab = _bf16(A)
    al, be = A1.default_alpha_beta(m, n)
    g = equilibrate(D, al, be, 1.0, 10.0, T, k, 17)
    o = A1.equilibrate(Ab, al, be, 1.0, 10.0, T, k=k, seed=17)
    err = max(np.abs(g["u_bar"].cpu().numpy() - o["u_bar"]).max(), np.abs(g["v_bar"].cpu().numpy() - o["v_bar"]).max())
    _say(f"bf16 {m}x{n} k={k} T={T} gamma=1: error {err:.3e}")
    assert err <= 5e-3


def _one_step_bound(Ab, u, v, S, W, k, eta, tau):
    """Rigorous bound on |u_bar_gpu - u_bar_oracle| (and v) after one step from (u, v).

    |Y_gpu - Y| <= (2^-16 (1 + g) + g) sum_j |A_ij| e^(v_j), g = K 2^-24 / (1 - K 2^-24)
    (two-term bf16 probe scale: hi within 2^-8 of e^v, lo within 2^-8 of e^v - hi; FP32
    accumulation of the K = 2n + 3 products and partial sums); then
    |dz| <= e^(2u)/k sum_p (2 |Y_p| d + d^2), |du| <= eta |dz| (the clip is 1-Lipschitz)
    and the average moves by 2/(tau + 2) of that."""
    def side(M, x, y, P):
        K = 2 * M.shape[1] + 3
        g = K * 2.0**-24 / (1 - K * 2.0**-24)
        c = 2.0**-16 * (1 + g) + g
        Y = M @ (np.exp(y)[:, None] * P)
        d = c * (np.abs(M) @ np.exp(y))
        dz = np.exp(2 * x) / k * np.sum(2 * np.abs(Y) * d[:, None] + d[:, None] ** 2, axis=1)
        return 2.0 / (tau + 2.0) * eta * dz * (1 + 1e-9) + 1e-12 * (1 + np.abs(x))
    return side(Ab, u, v, S), side(Ab.T, v, u, W)


def _one_step_check(D, Ab, states, k, seed, al, be):
    from paper_1602_06621_amd import equilibrate

    m, n = Ab.shape
    S, W = A1.probes(seed, 0, 1, m, n, k)
    worst = 0.0
    for t, (u, v) in states.items():
        tu, tv = torch.tensor(u, device="cuda"), torch.tensor(v, device="cuda")
        g = equilibrate(D, al, be, 0.1, 10.0, 1, k, seed, t0=t, u0=tu, v0=tv)
        o = A1.equilibrate(Ab, al, be, 0.1, 10.0, 1, k=k, seed=seed, t0=t, u0=u, v0=v)
        tau = 1 + t
        bu, bv = _one_step_bound(Ab, u, v, S, W, k, 2.0 / (0.1 * (tau + 1)), tau)
        du = np.abs(g["u_bar"].cpu().numpy() - o["u_bar"])
        dv = np.abs(g["v_bar"].cpu().numpy() - o["v_bar"])
        assert np.all(du <= bu) and np.all(dv <= bv), (t, (du / bu).max(), (dv / bv).max())
        worst = max(worst, (du / bu).max(), (dv / bv).max())
    return worst


@pytest.mark.parametrize("m,n,k", [(300, 170, 16), (67, 45, 5), (33, 1000, 33), (256, 256, 64)])
def test_bf16_one_step_within_rounding_bound(m, n, k):
    A = scaled_dense(m, n, 3.0, 300 + k)
    D, Ab = _bf16(A)
    al, be = A1.default_alpha_beta(m, n)
    states = {0: (np.zeros(m), np.zeros(n))}
    A1.equilibrate(Ab, al, be, 0.1, 10.0, 40, k=k, seed=9,
                   on_step=lambda t, u, v, ub, vb: states.__setitem__(t, (u.copy(), v.copy())))
    worst = _one_step_check(D, Ab, {t: states[t] for t in (0, 1, 3, 10, 40)}, k, 21, al, be)
    _say(f"bf16 {m}x{n} k={k}: worst error / bound = {worst:.3f}")


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (1, 40, 7), (40, 1, 64), (17, 3, 33), (31, 17, 64)])
def test_bf16_degenerate_shapes_one_step(m, n, k):
    """Single rows or columns and shapes smaller than one tile (32 x 16) or one probe
    block: one step from oracle states within the rounding bound."""
    A = scaled_dense(m, n, 3.0, 500 + k)
    D, Ab = _bf16(A)
    al, be = A1.default_alpha_beta(m, n)
    states = {0: (np.zeros(m), np.zeros(n))}
    A1.equilibrate(Ab, al, be, 0.1, 10.0, 5, k=k, seed=9,
                   on_step=lambda t, u, v, ub, vb: states.__setitem__(t, (u.copy(), v.copy())))
    worst = _one_step_check(D, Ab, {t: states[t] for t in (0, 2, 5)}, k, 23, al, be)
    _say(f"bf16 {m}x{n} k={k}: worst error / bound = {worst:.3f}")


def test_bf16_zero_steps_and_warm_start():
    """steps = 0 returns u_bar = u0, v_bar = v0 exactly and d = e^u0, e = e^v0 (to the
    last bit of FP64 exp); a warm start outside the box is rejected."""
    from paper_1602_06621_amd import MfeError, equilibrate

    A = scaled_dense(70, 50, 3.0, 77)
    D, _ = _bf16(A)
    rng = np.random.default_rng(5)
    u0, v0 = rng.uniform(-2, 2, 70), rng.uniform(-2, 2, 50)
    g = equilibrate(D, 1.0, 1.0, 0.1, 10.0, 0, 8, 3, u0=torch.tensor(u0, device="cuda"),
                    v0=torch.tensor(v0, device="cuda"))
    assert np.array_equal(g["u_bar"].cpu().numpy(), u0) and np.array_equal(g["v_bar"].cpu().numpy(), v0)
    assert np.allclose(g["d"].cpu().numpy(), np.exp(u0), rtol=4e-16, atol=0)
    assert np.allclose(g["e"].cpu().numpy(), np.exp(v0), rtol=4e-16, atol=0)
    bad = u0.copy()
    bad[3] = 11.0
    with pytest.raises(MfeError):
        equilibrate(D, 1.0, 1.0, 0.1, 10.0, 5, 8, 3, u0=torch.tensor(bad, device="cuda"),
                    v0=torch.tensor(v0, device="cuda"))


@pytest.mark.parametrize("batch", [0, 7])
def test_bf16_exact_products(batch):
    """+-1 and power-of-two entries with u = v = 0: every product is exact in bf16 and
    FP32, so one GPU step equals the oracle's step up to the FP64 epilogue (also with a
    nonzero batch index of the sign stream)."""
    from paper_1602_06621_amd import equilibrate

    rng = np.random.default_rng(4)
    A = rng.choice([-2.0, -1.0, -0.5, 0.0, 0.5, 1.0, 2.0], size=(96, 80))
    D, Ab = _bf16(A)
    g = equilibrate(D, 1.0, 1.0, 0.1, 10.0, 1, 8, 3, batch=batch)
    o = A1.equilibrate(Ab, 1.0, 1.0, 0.1, 10.0, 1, k=8, seed=3, batch=batch)
    assert np.abs(g["u_bar"].cpu().numpy() - o["u_bar"]).max() < 1e-13
    assert np.abs(g["v_bar"].cpu().numpy() - o["v_bar"]).max() < 1e-13


@pytest.fixture(scope="module")
def config3():
    """Dense 16384 x 8192 generated in FP64 (sigma = 3), rounded to bf16."""
    A = scaled_dense(16384, 8192, 3.0, 1003)
    bits, vals = round_to_bf16(A)
    del A
    return bits, vals


def test_bf16_full_size_one_step(config3):
    """Full size, k = 64: one step from oracle states t = 0, 1, 2 within the rounding bound."""
    from paper_1602_06621_amd import Dense

    bits, Ab = config3
    al, be = A1.default_alpha_beta(16384, 8192)
    D = Dense(torch.tensor(bits.view(np.int16), device="cuda"))
    states = {0: (np.zeros(16384), np.zeros(8192))}
    A1.equilibrate(Ab, al, be, 0.1, 10.0, 2, k=64, seed=2003,
                   on_step=lambda t, u, v, ub, vb: states.__setitem__(t, (u.copy(), v.copy())))
    worst = _one_step_check(D, Ab, states, 64, 2003, al, be)
    _say(f"full bf16 one step: worst error / bound = {worst:.3f}")


def test_bf16_full_size_500_steps_properties(config3):
    from paper_1602_06621_amd import Dense, equilibrate, last_timing

    bits, _ = config3
    al, be = A1.default_alpha_beta(16384, 8192)
    D = Dense(torch.tensor(bits.view(np.int16), device="cuda"))
    g = equilibrate(D, al, be, 0.1, 10.0, 500, 64, 2003)
    _say("timing", last_timing())
    ub, vb = g["u_bar"].cpu().numpy(), g["v_bar"].cpu().numpy()
    assert np.all(np.isfinite(ub)) and np.all(np.isfinite(vb))
    assert ub.max() <= al**2 / 0.1 and vb.max() <= be**2 / 0.1
    assert np.abs(ub).max() <= 10 and np.abs(vb).max() <= 10
    g2 = equilibrate(D, al, be, 0.1, 10.0, 500, 64, 2003)
    assert torch.equal(g["u_bar"], g2["u_bar"])


def test_bf16_full_size_10_steps_without_chaos(config3):
    """The benchmarked matrix and launch, 10 whole steps at gamma = 1: elementwise within
    5e-3 of the oracle on the rounded matrix.  (With one-term bf16 scales this run was
    5.4e-2 away: rows with large z turn the 2^-9 scale rounding into steps of a few
    1e-2; the two-term scale removes that.)"""
    from paper_1602_06621_amd import Dense, equilibrate

    bits, Ab = config3
    m, n = Ab.shape
    al, be = A1.default_alpha_beta(m, n)
    D = Dense(torch.tensor(bits.view(np.int16), device="cuda"))
    _say("full bf16 10 steps gamma 1")
    g = equilibrate(D, al, be, 1.0, 10.0, 10, 64, 2003)
    o = A1.equilibrate(Ab, al, be, 1.0, 10.0, 10, k=64, seed=2003)
    err = max(np.abs(g["u_bar"].cpu().numpy() - o["u_bar"]).max(), np.abs(g["v_bar"].cpu().numpy() - o["v_bar"]).max())
    _say(f"full bf16 10 steps gamma 1: error {err:.3e}")
    assert err <= 5e-3


def test_bf16_full_size_500_steps_benchmarked_run(config3):
    """The benchmarked run itself (16384 x 8192, k = 64, gamma = 0.1, M = 10, seed 2003,
    500 steps) against the stored 500-step oracle run on the rounded matrix: 2e-2."""
    from paper_1602_06621_amd import Dense, equilibrate

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_bf16.npz")
    ref = np.load(path)
    bits, Ab = config3
    m, n = Ab.shape
    al, be = A1.default_alpha_beta(m, n)
    D = Dense(torch.tensor(bits.view(np.int16), device="cuda"))
    _say("full bf16 500 steps")
    g = equilibrate(D, al, be, 0.1, 10.0, int(ref["steps"]), 64, 2003)
    eu = np.abs(g["u_bar"].cpu().numpy() - ref["u_bar"]).max()
    ev = np.abs(g["v_bar"].cpu().numpy() - ref["v_bar"]).max()
    _say(f"full bf16 500 steps: error u {eu:.3e} v {ev:.3e}")
    assert max(eu, ev) <= TOL
