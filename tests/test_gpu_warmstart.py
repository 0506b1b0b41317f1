"""GPU parity and gain of the learned warm start (sketch features, MLP kernels, training)."""
import sys

import numpy as np
import pytest
import torch

from oracle import algorithm1 as A1
from oracle import mlp as OM
from oracle import warmstart as OW
from tests.philox_ref import philox4x64
from workloads import warmstart_matrix, warmstart_training_set

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gpu(c):
    from paper_1602_06621_amd import Csr

    return Csr.from_arrays(c.m, c.n, c.row_ptr, c.col_idx, c.val)


def test_sketch_features_match_oracle():
    from paper_1602_06621_amd import Plan

    mats = [warmstart_matrix(700, 350, 1.5, 3), warmstart_matrix(130, 400, 2.5, 4, lo=1, hi=3)]
    with Plan([_gpu(c) for c in mats], max_probes=4) as plan:
        f = plan.sketch_features(99, 4, 0.1, 10.0)
        fr, fc = f["feat_rows"].cpu().numpy(), f["feat_cols"].cpu().numpy()
        us, vs = f["u_sketch"].cpu().numpy(), f["v_sketch"].cpu().numpy()
    r0 = c0 = 0
    for b, c in enumerate(mats):
        al, be = A1.default_alpha_beta(c.m, c.n)
        ofr, ofc, ous, ovs = OW.features(c.to_scipy(), 99, 4, al, be, 0.1, 10.0, batch=b)
        assert np.allclose(us[r0:r0 + c.m], ous, rtol=1e-12, atol=1e-12)
        assert np.allclose(vs[c0:c0 + c.n], ovs, rtol=1e-12, atol=1e-12)
        assert np.allclose(fr[r0:r0 + c.m], ofr, rtol=1e-5, atol=1e-6)
        assert np.allclose(fc[c0:c0 + c.n], ofc, rtol=1e-5, atol=1e-6)
        r0 += c.m
        c0 += c.n


def test_mlp_forward_and_gradient_match_oracle():
    from paper_1602_06621_amd import mlp_forward, mlp_loss_grad
    from paper_1602_06621_amd.warmstart import init_params

    rng = np.random.default_rng(5)
    X = rng.normal(0, 1, (1000, 8)).astype(np.float32)
    t = rng.normal(0, 1, 1000).astype(np.float32)
    th0 = init_params(7).cpu().numpy().astype(np.float64)
    th = th0 + rng.normal(0, 0.05, th0.size)
    thg = torch.tensor(th, dtype=torch.float32, device="cuda")
    y = mlp_forward(thg, torch.tensor(X, device="cuda")).cpu().numpy()
    th32 = thg.cpu().numpy().astype(np.float64)
    yo, _ = OM.forward(th32, X.astype(np.float64), 64)
    assert np.abs(y - yo).max() <= 1e-5 * max(1.0, np.abs(yo).max())
    loss, g = mlp_loss_grad(thg, torch.tensor(X, device="cuda"), torch.tensor(t, device="cuda"))
    lo, go = OM.loss_and_grad(th32, X.astype(np.float64), t.astype(np.float64), 64)
    assert loss == pytest.approx(lo, rel=1e-5)
    assert np.abs(g.cpu().numpy() - go).max() <= 1e-4 * np.abs(go).max()


def test_mlp_training_steps_match_oracle_adam():
    """Three Adam steps on Philox-drawn mini-batches: same batches, same updates."""
    from paper_1602_06621_amd import mlp_train
    from paper_1602_06621_amd.warmstart import init_params

    rng = np.random.default_rng(6)
    N, B, seed = 500, 64, 1234
    X = rng.normal(0, 1, (N, 8)).astype(np.float32)
    t = (np.sin(X[:, 0]) + 0.3 * X[:, 1]).astype(np.float32)
    thg = init_params(8)
    th = thg.cpu().numpy().astype(np.float64)
    m = torch.zeros_like(thg)
    v = torch.zeros_like(thg)
    losses = mlp_train(thg, m, v, 0, torch.tensor(X, device="cuda"), torch.tensor(t, device="cuda"), B, 3, 1e-2, seed)
    mo, vo = np.zeros_like(th), np.zeros_like(th)
    for s in range(1, 4):
        idx = [philox4x64([b + 1, 0, 0, 0], [seed, (s << 2) | 3])[0] % N for b in range(B)]
        L, g = OM.loss_and_grad(th, X[idx].astype(np.float64), t[idx].astype(np.float64), 64)
        assert losses[s - 1] == pytest.approx(L, rel=1e-4)
        th, mo, vo = OM.adam_step(th, g, mo, vo, s, 1e-2)
    assert np.abs(thg.cpu().numpy() - th).max() <= 1e-4


def test_learned_warm_start_reaches_plain_residual_sooner():
    """Train on small generated matrices, evaluate on held-out ones.  Target: 1.2 x the RMS
    equilibration error of the plain run after 2000 steps (the regularised floor).  The
    learned start (t0 = 20) must reach it in fewer steps than plain Algorithm 1, and must
    start closer to equilibrium than the sketch-only initialisation."""
    from paper_1602_06621_amd import Plan
    from paper_1602_06621_amd import warmstart as W

    train_mats = warmstart_training_set(24, 31, m_lo=5000, m_hi=20000)
    with Plan([_gpu(c) for c in train_mats], max_probes=16) as plan:
        lab = plan.equilibrate(None, None, 0.1, 10.0, 2000, 16, 77, use_graph=True)
        X, t = W.training_set(plan, 5, lab, per_matrix=2048)
    params, loss = W.train(X, t, iters=1500, batch=4096, lr=2e-3, seed=3)
    _say("train loss first/last", float(loss[:20].mean()), float(loss[-20:].mean()))
    assert loss[-20:].mean() < 0.5 * loss[:20].mean()
    every = 5
    for sigma in (1.0, 2.0):
        c = warmstart_matrix(40000, 20000, sigma, 900 + int(10 * sigma))
        al, be = A1.default_alpha_beta(c.m, c.n)
        with Plan([_gpu(c)], max_probes=16) as plan:
            _, plain = plan.equilibrate_trace(al, be, 0.1, 10.0, 2000, 16, 11, trace_every=every)
            target = 1.2 * plain[-1]
            res = {"plain": (W.steps_to_residual(plain, target, every), None)}
            for name, learned, t0 in (("sketch", False, 10), ("mlp", True, 20)):
                u0, v0 = W.warm_start(plan, params, 5, learned=learned)
                _, start = plan.equilibrate_trace(al, be, 0.1, 10.0, 1, 16, 11, t0=10**9, u0=u0, v0=v0,
                                                  trace_every=1)
                _, tr = plan.equilibrate_trace(al, be, 0.1, 10.0, 2000, 16, 11, t0=t0, u0=u0, v0=v0,
                                               trace_every=every)
                res[name] = (W.steps_to_residual(tr, target, every), float(start[0]))
        _say(f"sigma {sigma}: target {target:.4g}; (steps, start residual):", res)
        assert res["mlp"][0] is not None and res["mlp"][0] < res["plain"][0]
        assert res["mlp"][1] < res["sketch"][1]


def test_one_call_warm_start_equals_composed_steps():
    """mfe_plan_warmstart (sketch, network, clip in one call) gives the same (u0, v0) bit for
    bit as the separate calls, learned and sketch-only, on a batched plan."""
    from paper_1602_06621_amd import Plan, mlp_forward, warmstart_apply
    from paper_1602_06621_amd.warmstart import init_params

    mats = [warmstart_matrix(900, 450, 1.5, 21), warmstart_matrix(300, 600, 2.5, 22, lo=1, hi=4)]
    params = init_params(4)
    with Plan([_gpu(c) for c in mats], max_probes=4) as plan:
        for learned in (True, False):
            u0, v0 = plan.warm_start(params, 77, 4, 0.1, 10.0, learned=learned)
            f = plan.sketch_features(77, 4, 0.1, 10.0)
            du = mlp_forward(params, f["feat_rows"]) if learned else None
            dv = mlp_forward(params, f["feat_cols"]) if learned else None
            assert torch.equal(u0, warmstart_apply(f["u_sketch"], du, 10.0))
            assert torch.equal(v0, warmstart_apply(f["v_sketch"], dv, 10.0))


def test_warm_start_full_size_evaluation_matrix():
    """The one-call warm start on the 200,000 x 100,000 evaluation matrix of the warm-start
    benchmark (U{8..16} entries per row, sigma 2, seed 9001; sketch seed 5, 4 probes):
    sketch initialisation and features against the oracle as in the small test, and the
    learned start clip(sketch + MLP(features), -M, M) against the oracle's network applied
    to the library's FP32 features (the network runs in FP32 on the matrix cores: 1e-5 of
    the largest correction)."""
    from paper_1602_06621_amd import Plan
    from paper_1602_06621_amd.warmstart import init_params

    c = warmstart_matrix(200_000, 100_000, 2.0, 9001)
    al, be = A1.default_alpha_beta(c.m, c.n)
    params = init_params(6)
    with Plan([_gpu(c)], max_probes=16) as plan:
        f = plan.sketch_features(5, 4, 0.1, 10.0)
        u0, v0 = plan.warm_start(params, 5, 4, 0.1, 10.0, learned=True)
        fr, fc = f["feat_rows"].cpu().numpy(), f["feat_cols"].cpu().numpy()
        us, vs = f["u_sketch"].cpu().numpy(), f["v_sketch"].cpu().numpy()
        u0, v0 = u0.cpu().numpy(), v0.cpu().numpy()
    ofr, ofc, ous, ovs = OW.features(c.to_scipy(), 5, 4, al, be, 0.1, 10.0)
    assert np.allclose(us, ous, rtol=1e-12, atol=1e-12) and np.allclose(vs, ovs, rtol=1e-12, atol=1e-12)
    assert np.allclose(fr, ofr, rtol=1e-5, atol=1e-6) and np.allclose(fc, ofc, rtol=1e-5, atol=1e-6)
    theta = params.cpu().numpy().astype(np.float64)
    worst = 0.0
    for x0, feat, sk in ((u0, fr, us), (v0, fc, vs)):
        d, _ = OM.forward(theta, feat.astype(np.float64), 64)
        ref = np.clip(sk + d, -10.0, 10.0)
        worst = max(worst, np.abs(x0 - ref).max() / max(1.0, np.abs(d).max()))
    _say("full-size warm start: worst |u0 - oracle| / max(1, |correction|)", worst)
    assert worst <= 1e-5


def test_training_set_call_samples_strata_and_targets():
    """mfe_plan_training_set: every sample lies in its own stratum at the Philox offset the
    header states (recomputed here from the published Philox definition), its features are
    the sketch features of that index bit for bit, and its target is label - sketch
    initialisation rounded once to FP32.  Matrices smaller than per_matrix give every index."""
    from paper_1602_06621_amd import Plan

    mats = [warmstart_matrix(900, 450, 1.5, 31), warmstart_matrix(100, 300, 2.5, 32, lo=1, hi=4)]
    per, sseed = 256, 17
    with Plan([_gpu(c) for c in mats], max_probes=4) as plan:
        lab = plan.equilibrate(None, None, 0.1, 10.0, 50, 4, 5)
        X, t, idx = plan.training_set(5, lab["u_bar"], lab["v_bar"], per_matrix=per, sample_seed=sseed)
        f = plan.sketch_features(5, 4, 0.1, 10.0)
        X, t, idx = X.cpu().numpy(), t.cpu().numpy(), idx.cpu().numpy()
        fr, fc = f["feat_rows"].cpu().numpy(), f["feat_cols"].cpu().numpy()
        us, vs = f["u_sketch"].cpu().numpy(), f["v_sketch"].cpu().numpy()
        ub, vb = lab["u_bar"].cpu().numpy(), lab["v_bar"].cpu().numpy()
    want, s = [], 0
    for side, sizes in ((0, [c.m for c in mats]), (1, [c.n for c in mats])):
        base = 0
        for b, nb in enumerate(sizes):
            cnt = min(per, nb)
            for c in range(cnt):
                a, e = c * nb // cnt, (c + 1) * nb // cnt
                off = philox4x64([c + 1, 0, 0, 0], [sseed, (((b << 1) | side) << 2) | 3])[0] % (e - a)
                want.append((side, base + a + off))
            base += nb
    assert len(want) == len(idx)
    nr = sum(min(per, c.m) for c in mats)
    for s, (side, g) in enumerate(want):
        assert idx[s] == g
    ri, ci = idx[:nr], idx[nr:]
    assert len(set(ri.tolist())) == len(ri) and len(set(ci.tolist())) == len(ci)
    assert np.array_equal(X[:nr], fr[ri]) and np.array_equal(X[nr:], fc[ci])
    assert np.array_equal(t[:nr], (ub[ri] - us[ri]).astype(np.float32))
    assert np.array_equal(t[nr:], (vb[ci] - vs[ci]).astype(np.float32))
    # the second matrix has 100 rows < per: all of them, in order
    assert np.array_equal(ri[per:], 900 + np.arange(100))
