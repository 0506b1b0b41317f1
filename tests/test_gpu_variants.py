"""GPU parity of the Section 6 variants (symmetric equilibration / Algorithm 2, varying
row and column norms, block equilibration) against the FP64 oracle, through the C ABI.

Tolerance as for the standard sparse path: 1e-5 max-abs on the averaged log scalings
(elementwise relative on d, e).  Whole runs are compared only where the oracle itself
is stable: for each whole-run case below, the oracle's own spread under 1e-16 relative
perturbations of the targets was measured (values in the docstrings); rows whose
estimate z is large make the early steps expanding (|1 - eta (2z + gamma)| > 1), and
such runs are checked one step at a time instead, from random in-box states.  Where the
variant reduces to the standard problem (targets alpha^2, singleton blocks) the results
must be the standard path's bit for bit.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import algorithm1 as A1
from oracle import variants as V
from workloads import scaled_sparse, symmetric_sparse

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gpu(csr):
    from paper_1602_06621_amd import Csr

    return Csr.from_arrays(csr.m, csr.n, csr.row_ptr, csr.col_idx, csr.val)


def _np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def _random_blocks(count, max_size, seed):
    g = np.random.default_rng(seed)
    ptr = [0]
    while ptr[-1] < count:
        ptr.append(min(count, ptr[-1] + int(g.integers(1, max_size + 1))))
    return ptr


@pytest.mark.parametrize("k", [3, 16])
def test_targets_equal_to_alpha_are_bitwise_standard(k):
    from paper_1602_06621_amd import Plan

    csr = scaled_sparse(700, 380, 6, 1.5, 41)
    al, be = A1.default_alpha_beta(csr.m, csr.n)
    _say("targets = alpha^2, k", k)
    with Plan([_gpu(csr)], max_probes=k) as plan:
        ref = _np(plan.equilibrate(al, be, 0.1, 10.0, 30, k, 7))
        plan.set_targets(torch.full((csr.m,), al * al, dtype=torch.float64, device="cuda"),
                         torch.full((csr.n,), be * be, dtype=torch.float64, device="cuda"))
        got = _np(plan.equilibrate(al, be, 0.1, 10.0, 30, k, 7))
        got_g = _np(plan.equilibrate(al, be, 0.1, 10.0, 30, k, 7, use_graph=True))
    for key in ("u_bar", "v_bar", "d", "e"):
        assert np.array_equal(got[key], ref[key])
        assert np.array_equal(got_g[key], ref[key])


@pytest.mark.parametrize("k", [3, 16])
def test_varying_norms_parity(k):
    """300 x 170, 7 entries per row, per-row and per-column squared targets, t0 = 30
    (oracle spread 2.8e-11 for k = 3, 4.7e-14 for k = 16; with t0 = 0 it is 1.3e-2 and
    1.1e-4, covered by the one-step test)."""
    from paper_1602_06621_amd import Plan

    csr = scaled_sparse(300, 170, 7, 1.5, 51 + k)
    al, be = A1.default_alpha_beta(csr.m, csr.n)
    g = np.random.default_rng(k)
    rt = al**2 * g.uniform(0.5, 2.0, csr.m)
    ct = be**2 * g.uniform(0.5, 2.0, csr.n)
    ct *= rt.sum() / ct.sum()   # sum of squared row norms = sum of squared column norms
    _say("varying norms k", k)
    with Plan([_gpu(csr)], max_probes=k) as plan:
        plan.set_targets(torch.tensor(rt, device="cuda"), torch.tensor(ct, device="cuda"))
        out = _np(plan.equilibrate(al, be, 0.1, 10.0, 60, k, 3001 + k, t0=30))
    o = V.equilibrate_general(csr.to_scipy(), 0.1, 10.0, 60, k=k, seed=3001 + k, t0=30, row_target=rt,
                              col_target=ct)
    err = max(np.abs(out["u_bar"] - o["u_bar"]).max(), np.abs(out["v_bar"] - o["v_bar"]).max())
    _say("max err", err)
    assert err <= TOL
    assert np.allclose(out["d"], o["d"], rtol=TOL, atol=0)


def test_singleton_blocks_are_bitwise_standard():
    from paper_1602_06621_amd import Plan

    csr = scaled_sparse(700, 380, 6, 1.5, 43)
    al, be = A1.default_alpha_beta(csr.m, csr.n)
    _say("singleton blocks")
    with Plan([_gpu(csr)], max_probes=16) as plan:
        ref = _np(plan.equilibrate(al, be, 0.1, 10.0, 30, 16, 9))
        plan.set_blocks(range(csr.m + 1), range(csr.n + 1))
        got = _np(plan.equilibrate(al, be, 0.1, 10.0, 30, 16, 9))
        got_g = _np(plan.equilibrate(al, be, 0.1, 10.0, 30, 16, 9, use_graph=True))
    for key in ("u_bar", "v_bar", "d", "e"):
        assert np.array_equal(got[key], ref[key])
        assert np.array_equal(got_g[key], ref[key])


@pytest.mark.parametrize("rows,cols,targets,k", [(True, True, False, 16), (False, True, True, 16),
                                                 (True, True, True, 8)])
def test_block_parity(rows, cols, targets, k):
    """300 x 170 with blocks of 1-20 rows and 1-10 columns (ragged), optionally with
    per-index targets; block variables and per-index scalings against the oracle
    (oracle spreads 2.2e-10, 1.2e-10, 7.2e-12)."""
    from paper_1602_06621_amd import Plan

    csr = scaled_sparse(300, 170, 7, 1.5, 61 + k)
    al, be = A1.default_alpha_beta(csr.m, csr.n)
    rp = _random_blocks(csr.m, 20, 5) if rows else None
    cp = _random_blocks(csr.n, 10, 6) if cols else None
    rt = ct = None
    if targets:
        g = np.random.default_rng(9)
        rt = al**2 * g.uniform(0.5, 2.0, csr.m)
        ct = be**2 * g.uniform(0.5, 2.0, csr.n)
    _say("blocks", rows, cols, targets, k)
    with Plan([_gpu(csr)], max_probes=k) as plan:
        if targets:
            plan.set_targets(torch.tensor(rt, device="cuda"), torch.tensor(ct, device="cuda"))
        plan.set_blocks(rp, cp)
        out = _np(plan.equilibrate(al, be, 0.1, 10.0, 60, k, 77, use_graph=True))
    o = V.equilibrate_general(csr.to_scipy(), 0.1, 10.0, 60, k=k, seed=77, row_ptr=rp, col_ptr=cp,
                              row_target=rt, col_target=ct, alpha=al, beta=be)
    assert out["u_bar"].shape == o["u_bar"].shape and out["v_bar"].shape == o["v_bar"].shape
    err = max(np.abs(out["u_bar"] - o["u_bar"]).max(), np.abs(out["v_bar"] - o["v_bar"]).max())
    _say("max err", err)
    assert err <= TOL
    assert np.allclose(out["d"], o["d"], rtol=TOL, atol=0)
    assert np.allclose(out["e"], o["e"], rtol=TOL, atol=0)


@pytest.mark.parametrize("k", [1, 16])
def test_variants_whole_run_without_chaos(k):
    """With a large enough gamma the iterations contract perturbations, so 400 steps of
    each Section 6 variant are compared elementwise at 1e-10 (with k = 1 too, where
    gamma = 0.1 runs are chaotic): blocks of 1-20 rows and 1-10 columns with per-index
    targets at gamma = 4 (a block sums up to 20 rows' estimates; at gamma = 1 the
    oracle's own spread under 1e-15 perturbations of A is still 2.2e-7 for k = 1, at
    gamma = 4 it is 1.7e-14, and another seed moves u_bar by 0.13), and Algorithm 2 on a
    symmetric matrix at gamma = 1."""
    from paper_1602_06621_amd import Plan

    csr = scaled_sparse(300, 170, 7, 1.5, 61 + k)
    al, be = A1.default_alpha_beta(csr.m, csr.n)
    rp, cp = _random_blocks(csr.m, 20, 5), _random_blocks(csr.n, 10, 6)
    g = np.random.default_rng(9)
    rt, ct = al**2 * g.uniform(0.5, 2.0, csr.m), be**2 * g.uniform(0.5, 2.0, csr.n)
    with Plan([_gpu(csr)], max_probes=k) as plan:
        plan.set_targets(torch.tensor(rt, device="cuda"), torch.tensor(ct, device="cuda"))
        plan.set_blocks(rp, cp)
        out = _np(plan.equilibrate(al, be, 4.0, 10.0, 400, k, 77, use_graph=True))
    o = V.equilibrate_general(csr.to_scipy(), 4.0, 10.0, 400, k=k, seed=77, row_ptr=rp, col_ptr=cp,
                              row_target=rt, col_target=ct, alpha=al, beta=be)
    err = max(np.abs(out["u_bar"] - o["u_bar"]).max(), np.abs(out["v_bar"] - o["v_bar"]).max())
    sym = symmetric_sparse(300, 4, 1.5, 390 + k)
    with Plan.symmetric_plan(_gpu(sym), max_probes=k) as plan:
        so = _np(plan.equilibrate(1.0, 1.0, 1.0, 10.0, 400, k, 4001, use_graph=True))
    os_ = V.equilibrate_symmetric(sym.to_scipy(), 1.0, 1.0, 10.0, 400, k=k, seed=4001)
    serr = np.abs(so["u_bar"] - os_["u_bar"]).max()
    _say("400 steps: blocks+targets (gamma 4)", err, "symmetric (gamma 1)", serr)
    assert err <= 1e-10 and serr <= 1e-10


def _one_step_cases(m_blocks, n_blocks, seed):
    g = np.random.default_rng(seed)
    for t0 in (0, 7, 100):
        yield t0, np.clip(g.normal(0, 1.5, m_blocks), -10, 10), np.clip(g.normal(0, 1.5, n_blocks), -10, 10)


@pytest.mark.parametrize("case", ["targets", "row_blocks_k3", "blocks_targets"])
def test_variant_one_step_from_random_states(case):
    """One step from random in-box states (u0 = u_bar0 as the warm start sets them), t0 in
    {0, 7, 100}, against one oracle step: relative 1e-11.  Covers the regimes where whole
    runs are chaotic (large z, t0 = 0)."""
    from paper_1602_06621_amd import Plan

    csr = scaled_sparse(300, 170, 7, 1.5, 63)
    al, be = A1.default_alpha_beta(csr.m, csr.n)
    g = np.random.default_rng(2)
    rt = al**2 * g.uniform(0.5, 2.0, csr.m) if case != "row_blocks_k3" else None
    ct = be**2 * g.uniform(0.5, 2.0, csr.n) if case != "row_blocks_k3" else None
    rp = _random_blocks(csr.m, 20, 5) if case != "targets" else None
    cp = _random_blocks(csr.n, 10, 6) if case == "blocks_targets" else None
    k = 3 if case == "row_blocks_k3" else 16
    nu = len(rp) - 1 if rp else csr.m
    nv = len(cp) - 1 if cp else csr.n
    A = csr.to_scipy()
    worst = 0.0
    _say("one step", case)
    with Plan([_gpu(csr)], max_probes=k) as plan:
        if rt is not None:
            plan.set_targets(torch.tensor(rt, device="cuda"), torch.tensor(ct, device="cuda"))
        plan.set_blocks(rp, cp)
        for t0, u, v in _one_step_cases(nu, nv, 11):
            out = _np(plan.equilibrate(al, be, 0.1, 10.0, 1, k, 17, t0=t0, u0=torch.tensor(u, device="cuda"),
                                       v0=torch.tensor(v, device="cuda")))
            o = V.equilibrate_general(A, 0.1, 10.0, 1, k=k, seed=17, t0=t0, row_ptr=rp, col_ptr=cp, row_target=rt,
                                      col_target=ct, alpha=al, beta=be, u0=u, v0=v)
            for key in ("u_bar", "v_bar"):
                d = np.abs(out[key] - o[key]) / np.maximum(1.0, np.abs(o[key]))
                worst = max(worst, d.max())
    _say("worst", worst)
    assert worst <= 1e-11


def test_block_warm_start_with_offset():
    """Block warm start (one value per block, inside the box) and t0 > 0 (oracle spread
    1.9e-8)."""
    from paper_1602_06621_amd import Plan

    csr = scaled_sparse(400, 230, 6, 1.0, 71)
    al, be = A1.default_alpha_beta(csr.m, csr.n)
    rp = _random_blocks(csr.m, 12, 1)
    cp = _random_blocks(csr.n, 7, 2)
    g = np.random.default_rng(3)
    u0 = np.clip(g.normal(0, 1.0, len(rp) - 1), -10, 10)
    v0 = np.clip(g.normal(0, 1.0, len(cp) - 1), -10, 10)
    _say("block warm start")
    with Plan([_gpu(csr)], max_probes=16) as plan:
        plan.set_blocks(rp, cp)
        out = _np(plan.equilibrate(al, be, 0.1, 10.0, 25, 16, 5, t0=20, u0=torch.tensor(u0, device="cuda"),
                                   v0=torch.tensor(v0, device="cuda")))
    o = V.equilibrate_general(csr.to_scipy(), 0.1, 10.0, 25, k=16, seed=5, t0=20, row_ptr=rp, col_ptr=cp,
                              alpha=al, beta=be, u0=u0, v0=v0)
    err = max(np.abs(out["u_bar"] - o["u_bar"]).max(), np.abs(out["v_bar"] - o["v_bar"]).max())
    _say("max err", err)
    assert err <= TOL


def test_block_parity_large():
    """100,000 x 50,000, 10 entries per row, row blocks of 8 and column blocks of 1-6
    (many slices and windows, ragged tails), k = 16, 20 steps (oracle spread 2.0e-12)."""
    from paper_1602_06621_amd import Plan

    csr = scaled_sparse(100_000, 50_000, 10, 2.0, 81)
    al, be = A1.default_alpha_beta(csr.m, csr.n)
    rp = list(range(0, csr.m, 8)) + [csr.m]
    cp = _random_blocks(csr.n, 6, 4)
    _say("blocks large")
    with Plan([_gpu(csr)], max_probes=16) as plan:
        plan.set_blocks(rp, cp)
        out = _np(plan.equilibrate(al, be, 0.1, 10.0, 20, 16, 91, use_graph=True))
    o = V.equilibrate_general(csr.to_scipy(), 0.1, 10.0, 20, k=16, seed=91, row_ptr=rp, col_ptr=cp,
                              alpha=al, beta=be)
    err = max(np.abs(out["u_bar"] - o["u_bar"]).max(), np.abs(out["v_bar"] - o["v_bar"]).max())
    _say("max err", err)
    assert err <= TOL


@pytest.mark.parametrize("n,half,k,T", [(300, 4, 16, 60), (300, 4, 3, 60), (513, 2, 8, 40)])
def test_symmetric_parity(n, half, k, T):
    """Algorithm 2 on a symmetric sparse matrix (ragged slices) against the oracle (oracle
    spreads 1.7e-9, 6.2e-9, 1.5e-9)."""
    from paper_1602_06621_amd import Plan

    csr = symmetric_sparse(n, half, 1.5, 90 + n + k)
    _say("symmetric", n, half, k, T)
    with Plan.symmetric_plan(_gpu(csr), max_probes=k) as plan:
        out = _np(plan.equilibrate(1.0, 1.0, 0.1, 10.0, T, k, 4001, use_graph=True))
    o = V.equilibrate_symmetric(csr.to_scipy(), 1.0, 0.1, 10.0, T, k=k, seed=4001)
    err = np.abs(out["u_bar"] - o["u_bar"]).max()
    _say("max err", err)
    assert err <= TOL
    assert np.array_equal(out["d"], out["e"]) and np.array_equal(out["u_bar"], out["v_bar"])
    assert np.allclose(out["d"], o["d"], rtol=TOL, atol=0)


def test_symmetric_parity_large():
    """200,000 x 200,000 symmetric, ~10 entries per row, k = 16, 20 steps (oracle spread
    4.3e-8)."""
    from paper_1602_06621_amd import Plan

    csr = symmetric_sparse(200_000, 5, 2.0, 95)
    _say("symmetric large")
    with Plan.symmetric_plan(_gpu(csr), max_probes=16) as plan:
        out = _np(plan.equilibrate(1.0, 1.0, 0.1, 10.0, 20, 16, 4002, use_graph=True))
    o = V.equilibrate_symmetric(csr.to_scipy(), 1.0, 0.1, 10.0, 20, k=16, seed=4002)
    err = np.abs(out["u_bar"] - o["u_bar"]).max()
    _say("max err", err)
    assert err <= TOL


@pytest.mark.parametrize("k", [1, 16])
def test_symmetric_one_step_from_random_states(k):
    """Algorithm 2, one step from random in-box states, t0 in {0, 7, 100}: relative 1e-11."""
    from paper_1602_06621_amd import Plan

    csr = symmetric_sparse(700, 4, 2.0, 97)
    A = csr.to_scipy()
    g = np.random.default_rng(k)
    worst = 0.0
    _say("symmetric one step", k)
    with Plan.symmetric_plan(_gpu(csr), max_probes=k) as plan:
        for t0 in (0, 7, 100):
            u = np.clip(g.normal(0, 1.5, csr.n), -10, 10)
            out = _np(plan.equilibrate(1.3, 1.3, 0.1, 10.0, 1, k, 23, t0=t0, u0=torch.tensor(u, device="cuda")))
            o = V.equilibrate_symmetric(A, 1.3, 0.1, 10.0, 1, k=k, seed=23, t0=t0, u0=u)
            d = np.abs(out["u_bar"] - o["u_bar"]) / np.maximum(1.0, np.abs(o["u_bar"]))
            worst = max(worst, d.max())
    _say("worst", worst)
    assert worst <= 1e-11


def test_variant_settings_rejected():
    from paper_1602_06621_amd import Plan
    from paper_1602_06621_amd._ffi import MfeError

    csr = scaled_sparse(300, 200, 4, 1.0, 3)
    other = scaled_sparse(200, 100, 4, 1.0, 4)
    _say("variant rejections")
    # not symmetric / not square
    with pytest.raises(MfeError, match="EINVAL"):
        Plan.symmetric_plan(_gpu(scaled_sparse(200, 200, 4, 1.0, 5)))
    with pytest.raises(MfeError, match="EDIM"):
        Plan.symmetric_plan(_gpu(csr))
    with Plan.symmetric_plan(_gpu(symmetric_sparse(200, 3, 1.0, 6))) as sym:
        with pytest.raises(MfeError, match="EUNSUPPORTED"):
            sym.set_blocks([0, 100, 200], None)
        with pytest.raises(MfeError, match="EUNSUPPORTED"):
            sym.set_targets(torch.ones(200, dtype=torch.float64, device="cuda"), None)
    with Plan([_gpu(csr), _gpu(other)]) as batched:
        with pytest.raises(MfeError, match="EUNSUPPORTED"):
            batched.set_blocks([0, 300], None)
    with Plan([_gpu(csr)]) as plan:
        for bad in ([0, 150, 150, 300], [1, 300], [0, 299], [0, 200, 100, 300]):
            with pytest.raises(MfeError, match="EINVAL"):
                plan.set_blocks(bad, None)
        t = torch.ones(300, dtype=torch.float64, device="cuda")
        t[17] = -1.0
        with pytest.raises(MfeError, match="EINVAL"):
            plan.set_targets(t, None)
        t[17] = float("nan")
        with pytest.raises(MfeError, match="EINVAL"):
            plan.set_targets(t, None)
        plan.set_blocks([0, 100, 300], None)
        with pytest.raises(MfeError, match="EUNSUPPORTED"):
            plan.equilibrate_trace(1.0, 1.0, steps=10, probes=4, trace_every=5)
        # clearing the settings restores the standard problem
        plan.set_blocks(None, None)
        plan.set_targets(None, None)
        out = plan.equilibrate(None, None, 0.1, 10.0, 10, 4, 1)
        assert out["u_bar"].numel() == 300


def test_targets_on_a_batched_plan():
    """Per-index targets on a plan of three matrices (targets concatenated in plan order,
    matrix b on sign batch b): each matrix against its own oracle run, t0 = 30 (oracle
    spread 4.4e-13)."""
    from paper_1602_06621_amd import Plan

    mats = [scaled_sparse(240, 130, 6, 1.0, 300 + i) for i in range(3)]
    g = np.random.default_rng(12)
    rts, cts = [], []
    for c in mats:
        al, be = A1.default_alpha_beta(c.m, c.n)
        rts.append(al**2 * g.uniform(0.5, 2.0, c.m))
        cts.append(be**2 * g.uniform(0.5, 2.0, c.n))
    _say("batched targets")
    with Plan([_gpu(c) for c in mats], max_probes=16) as plan:
        plan.set_targets(torch.tensor(np.concatenate(rts), device="cuda"),
                         torch.tensor(np.concatenate(cts), device="cuda"))
        out = _np(plan.equilibrate(None, None, 0.1, 10.0, 40, 16, 61, t0=30))
    r0 = np.concatenate([[0], np.cumsum([c.m for c in mats])])
    c0 = np.concatenate([[0], np.cumsum([c.n for c in mats])])
    worst = 0.0
    for b, c in enumerate(mats):
        o = V.equilibrate_general(c.to_scipy(), 0.1, 10.0, 40, k=16, seed=61, t0=30, row_target=rts[b],
                                  col_target=cts[b], batch=b)
        worst = max(worst, np.abs(out["u_bar"][r0[b]:r0[b + 1]] - o["u_bar"]).max(),
                    np.abs(out["v_bar"][c0[b]:c0[b + 1]] - o["v_bar"]).max())
    _say("max err", worst)
    assert worst <= TOL


def test_symmetric_wide_descriptors_one_step():
    """Algorithm 2 with k = 64 (16-byte descriptors, the widest probe bucket), one step
    from random in-box states: relative 1e-11."""
    from paper_1602_06621_amd import Plan

    csr = symmetric_sparse(500, 3, 1.5, 98)
    A = csr.to_scipy()
    g = np.random.default_rng(64)
    worst = 0.0
    with Plan.symmetric_plan(_gpu(csr), max_probes=64) as plan:
        for t0 in (0, 50):
            u = np.clip(g.normal(0, 1.5, csr.n), -10, 10)
            out = _np(plan.equilibrate(1.0, 1.0, 0.1, 10.0, 1, 64, 29, t0=t0, u0=torch.tensor(u, device="cuda")))
            o = V.equilibrate_symmetric(A, 1.0, 0.1, 10.0, 1, k=64, seed=29, t0=t0, u0=u)
            worst = max(worst, (np.abs(out["u_bar"] - o["u_bar"]) / np.maximum(1.0, np.abs(o["u_bar"]))).max())
    _say("worst", worst)
    assert worst <= 1e-11


def test_graph_recaptured_after_variant_settings():
    """A plan's cached HIP graph is rebuilt when the variant settings change: graph runs
    before and after set_blocks / set_targets equal the eager runs with the same settings."""
    from paper_1602_06621_amd import Plan

    csr = scaled_sparse(500, 300, 6, 1.0, 44)
    al, be = A1.default_alpha_beta(csr.m, csr.n)
    rp = _random_blocks(csr.m, 9, 3)
    g = np.random.default_rng(4)
    rt = torch.tensor(al**2 * g.uniform(0.5, 2.0, csr.m), device="cuda")
    _say("graph recapture")
    with Plan([_gpu(csr)], max_probes=8) as plan:
        res = {}
        for label in ("plain", "blocks", "targets", "plain2"):
            if label == "blocks":
                plan.set_blocks(rp, None)
            elif label == "targets":
                plan.set_blocks(None, None)
                plan.set_targets(rt, None)
            elif label == "plain2":
                plan.set_targets(None, None)
            gr = _np(plan.equilibrate(al, be, 0.1, 10.0, 20, 8, 5, use_graph=True))
            ea = _np(plan.equilibrate(al, be, 0.1, 10.0, 20, 8, 5, use_graph=False))
            for key in ("u_bar", "v_bar", "d", "e"):
                assert np.array_equal(gr[key], ea[key]), (label, key)
            res[label] = gr
    assert np.array_equal(res["plain"]["d"], res["plain2"]["d"])
    assert not np.array_equal(res["plain"]["d"], res["blocks"]["d"])
    assert not np.array_equal(res["plain"]["d"], res["targets"]["d"])
