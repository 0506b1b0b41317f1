"""GPU parity of the sparse (CSR) path against the FP64 oracle, through the C ABI.

Tolerance: the target bound for (u, v) is 1e-5 (max-abs on u_bar, v_bar, which is
the elementwise relative error of d, e).  The GPU path accumulates in FP64, so the
measured error is far smaller; chaotic amplification of rounding in the first steps
(eta_1 gamma = 1) is what separates the two at all.

With a single probe per step (k = 1, Algorithm 1 verbatim) the iteration is chaotic:
the oracle itself moves u_bar by O(0.1) under 1e-16 relative perturbations of the
estimate (measured; it decays like 1/T^2).  Whole-run elementwise parity is then not
a property any second implementation can have, so k = 1 is checked step by step: from
states on the oracle's own trajectory, one GPU step must equal one oracle step.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import algorithm1 as A1
from oracle import signs as S
from workloads import poisson_lengths, scaled_sparse

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gpu(csr):
    from paper_1602_06621_amd import Csr

    return Csr.from_arrays(csr.m, csr.n, csr.row_ptr, csr.col_idx, csr.val)


def _both(csr, k, T, seed, t0=0, u0=None, v0=None, gamma=0.1, M=10.0):
    from paper_1602_06621_amd import equilibrate

    al, be = A1.default_alpha_beta(csr.m, csr.n)
    g = equilibrate(_gpu(csr), al, be, gamma, M, T, k, seed, t0,
                    u0=None if u0 is None else torch.tensor(u0, device="cuda"),
                    v0=None if v0 is None else torch.tensor(v0, device="cuda"))
    o = A1.equilibrate(csr.to_scipy(), al, be, gamma, M, T, k=k, seed=seed, t0=t0, u0=u0, v0=v0)
    return {k_: v.cpu().numpy() for k_, v in g.items()}, o


def _err(g, o):
    return max(np.abs(g["u_bar"] - o["u_bar"]).max(), np.abs(g["v_bar"] - o["v_bar"]).max())


@pytest.mark.parametrize("seed,batch,step,side,nwords", [
    (0, 0, 1, 0, 1), (2001, 0, 7, 1, 5), (2**63 + 11, 3, 123456, 2, 1001), (5, 2**30 - 1, 2**32 - 1, 3, 64)])
def test_sign_words_bit_exact(seed, batch, step, side, nwords):
    from paper_1602_06621_amd import draw_signs

    _say("signs", seed, batch, step, side, nwords)
    w = draw_signs(seed, batch, step, side, nwords).cpu().numpy().view(np.uint64)
    ref = S.stream_words(seed, batch, step, side, nwords)
    assert np.array_equal(w, ref)


@pytest.mark.parametrize("k", [3, 16, 33, 64])
def test_small_parity_several_tiles(k):
    """300 x 170 (5 row slices, 3 column slices, ragged tails), 7 entries per row."""
    csr = scaled_sparse(300, 170, 7, 1.5, 101 + k)
    _say("small parity k", k)
    g, o = _both(csr, k, 60, 2001 + k)
    err = _err(g, o)
    _say("max err", err)
    assert err <= TOL
    assert np.allclose(g["d"], np.exp(o["u_bar"]), rtol=TOL, atol=0)
    assert np.allclose(g["e"], np.exp(o["v_bar"]), rtol=TOL, atol=0)


@pytest.mark.parametrize("k", [1, 2])
def test_whole_run_without_chaos_few_probes(k):
    """One and two probes per step are chaotic over whole runs at gamma = 0.1; with
    gamma = 1 the iteration contracts perturbations (the oracle's own u_bar moves by 1e-14
    under 1e-16 perturbations of z, by 0.2 with another seed), so 500 steps of the
    one-launch path (3,000 x 1,500, 8 entries per row) are compared elementwise."""
    csr = scaled_sparse(3000, 1500, 8, 2.0, 77)
    g, o = _both(csr, k, 500, 5, gamma=1.0)
    err = _err(g, o)
    _say("k", k, "gamma 1, 500 steps: max err", err)
    assert err <= 1e-10


@pytest.mark.parametrize("k", [1, 2, 16])
def test_one_step_map_along_oracle_trajectory(k):
    """From the oracle's states (u^t, v^t, u_bar^t, v_bar^t), one GPU step with t0 = t equals
    one oracle step (same probes: step index 1 of the stream) -- well posed for any k."""
    from paper_1602_06621_amd import equilibrate

    csr = scaled_sparse(300, 170, 7, 1.5, 101 + k)
    al, be = A1.default_alpha_beta(csr.m, csr.n)
    A = csr.to_scipy()
    states = {0: (np.zeros(300), np.zeros(170))}
    A1.equilibrate(A, al, be, 0.1, 10.0, 60, k=k, seed=2001,
                   on_step=lambda t, u, v, ub, vb: states.__setitem__(t, (u.copy(), v.copy())))
    G = _gpu(csr)
    worst = 0.0
    for t in (0, 1, 2, 3, 5, 10, 30, 59):
        u, v = states[t]
        g = equilibrate(G, al, be, 0.1, 10.0, 1, k, 77, t0=t, u0=torch.tensor(u, device="cuda"),
                        v0=torch.tensor(v, device="cuda"))
        o = A1.equilibrate(A, al, be, 0.1, 10.0, 1, k=k, seed=77, t0=t, u0=u, v0=v)
        for key in ("u_bar", "v_bar"):
            d = np.abs(g[key].cpu().numpy() - o[key]) / np.maximum(1.0, np.abs(o[key]))
            worst = max(worst, d.max())
    _say("one-step worst rel err", worst)
    assert worst <= 1e-11


def test_ragged_rows_with_empty_rows_and_columns():
    """Poisson(3) row lengths: empty rows and columns, many slice widths."""
    m, n = 1500, 700
    L = poisson_lengths(m, 3.0, n, 7)
    csr = scaled_sparse(m, n, L, 2.0, 8)
    assert (np.diff(csr.row_ptr) == 0).any()
    _say("ragged")
    g, o = _both(csr, 8, 150, 9)
    err = _err(g, o)
    _say("max err", err)
    assert err <= TOL
    # empty rows sit at min(M, alpha^2/gamma) times the average weight (closed form)
    al, _ = A1.default_alpha_beta(m, n)
    empty = np.diff(csr.row_ptr) == 0
    T = 150
    assert np.allclose(g["u_bar"][empty], (1 - 2 / ((T + 1) * (T + 2))) * al**2 / 0.1, rtol=1e-12)


def test_long_rows_and_columns():
    """A few rows far longer than the rest (wide slices), dense-ish columns."""
    m, n = 400, 90
    L = np.full(m, 3)
    L[[0, 77, 399]] = [90, 60, 45]
    csr = scaled_sparse(m, n, L, 1.0, 10)
    g, o = _both(csr, 8, 60, 11)
    assert _err(g, o) <= TOL


def test_warm_start_and_offset():
    csr = scaled_sparse(257, 129, 5, 1.0, 12)
    rng = np.random.default_rng(13)
    u0 = rng.normal(0, 0.5, 257)
    v0 = rng.normal(0, 0.5, 129)
    g, o = _both(csr, 4, 50, 14, t0=25, u0=u0, v0=v0)
    assert _err(g, o) <= TOL


@pytest.mark.parametrize("k,M", [(8, 20.0), (16, 12.0)])
def test_wide_descriptors_for_few_probes_and_a_large_box(k, M):
    """With M > 11, e^x leaves the range of the 8-byte descriptor, so even k <= 16 runs
    with 16-byte descriptors (FP64 scale, 64 sign bits); parity at T = 80 (the oracle's
    own spread here is ~1e-10)."""
    csr = scaled_sparse(300, 170, 7, 1.5, 112 + k)
    g, o = _both(csr, k, 80, 5, M=M)
    err = _err(g, o)
    _say("wide descriptors k", k, "M", M, "err", err)
    assert err <= TOL


def test_warm_start_outside_box_rejected():
    from paper_1602_06621_amd import MfeError, equilibrate

    csr = scaled_sparse(40, 30, 3, 1.0, 16)
    u0 = np.zeros(40)
    u0[7] = 10.5
    with pytest.raises(MfeError, match="outside the box"):
        equilibrate(_gpu(csr), None, None, 0.1, 10.0, 5, 2, 1, u0=torch.tensor(u0, device="cuda"),
                    v0=torch.zeros(30, dtype=torch.float64, device="cuda"))


def test_zero_steps_returns_warm_start():
    csr = scaled_sparse(70, 65, 3, 1.0, 15)
    u0 = np.linspace(-1, 1, 70)
    v0 = np.linspace(2, -2, 65)
    g, _ = _both(csr, 2, 0, 1, u0=u0, v0=v0)
    assert np.array_equal(g["u_bar"], u0) and np.array_equal(g["v_bar"], v0)
    assert np.allclose(g["d"], np.exp(u0), rtol=1e-15)


def test_diagonal_matrix_matches_closed_form():
    """Deterministic special case: one entry per row and column (independent of the RNG)."""
    from oracle import theory

    a = np.array([0.01, 0.3, 1.0, 2.0, 50.0, 1e3] * 20)
    m = a.size
    import scipy.sparse as sp

    from workloads import csr_from_dense

    csr = csr_from_dense(np.diag(a))
    from paper_1602_06621_amd import equilibrate

    af = csr.val.astype(np.float64)
    q = (0.1 / 4.0) * theory.lambertw_exp(np.log(4.0 * af**2 / 0.1) + 4.0 / 0.1)
    xs = (1 - q) / 0.1
    g = equilibrate(_gpu(csr), 1.0, 1.0, 0.1, 10.0, 1000, 3, 5)
    ub = g["u_bar"].cpu().numpy()
    o = A1.equilibrate(sp.csr_matrix(np.diag(af)), 1.0, 1.0, 0.1, 10.0, 1000, k=3, seed=5)
    assert np.max(np.abs(ub - o["u_bar"])) < 1e-10
    assert np.max(np.abs(ub - xs)) < 3e-3


def test_nonfinite_input_reported():
    from paper_1602_06621_amd import MfeError, equilibrate

    csr = scaled_sparse(100, 50, 4, 1.0, 16)
    csr.val[17] = np.nan
    with pytest.raises(MfeError) as ei:
        equilibrate(_gpu(csr), steps=5, probes=2)
    assert ei.value.name == "MFE_ENONFINITE"


def test_invalid_csr_rejected():
    from paper_1602_06621_amd import Csr, MfeError, equilibrate

    csr = scaled_sparse(50, 40, 4, 1.0, 17)
    bad = csr.col_idx.copy()
    bad[5] = 40  # out of range
    with pytest.raises(MfeError) as ei:
        equilibrate(Csr.from_arrays(50, 40, csr.row_ptr, bad, csr.val), steps=2)
    assert ei.value.name == "MFE_EINVAL"
    unsorted = csr.col_idx.copy()
    unsorted[0], unsorted[1] = unsorted[1], unsorted[0]
    with pytest.raises(MfeError):
        equilibrate(Csr.from_arrays(50, 40, csr.row_ptr, unsorted, csr.val), steps=2)


def test_deterministic_and_graph_replay_identical():
    from paper_1602_06621_amd import Plan

    csr = scaled_sparse(3000, 1700, 6, 2.0, 18)
    with Plan([_gpu(csr)], max_probes=16) as plan:
        a = plan.equilibrate(steps=80, probes=16, seed=3)
        a = {k: v.clone() for k, v in a.items()}
        b = plan.equilibrate(steps=80, probes=16, seed=3)
        c = plan.equilibrate(steps=80, probes=16, seed=3, use_graph=True)
        for key in ("u_bar", "v_bar", "d", "e"):
            assert torch.equal(a[key], b[key])
            assert torch.equal(a[key], c[key])


def test_graph_recaptured_after_sign_buffers_change():
    """A cached graph must not replay with sign buffers that a run with another k (or
    another batch index) has freed and reallocated: graph k = 16, then an ungraphed
    k = 8 run, then a traced run with k = 4, then graph k = 16 again, all bitwise equal to
    a fresh plan's graph run."""
    from paper_1602_06621_amd import Plan

    csr = scaled_sparse(3000, 1700, 6, 2.0, 19)
    _say("graph recapture 3000x1700")
    with Plan([_gpu(csr)], max_probes=16) as fresh:
        ref = fresh.equilibrate(steps=60, probes=16, seed=4, use_graph=True)
        ref = {k: v.clone() for k, v in ref.items()}
    with Plan([_gpu(csr)], max_probes=16) as plan:
        plan.equilibrate(steps=60, probes=16, seed=4, use_graph=True)
        plan.equilibrate(steps=60, probes=8, seed=4)
        al, be = A1.default_alpha_beta(csr.m, csr.n)
        plan.equilibrate_trace(al, be, steps=20, probes=4, seed=4, trace_every=10)
        plan.equilibrate(steps=60, probes=16, seed=4, batch=2)
        again = plan.equilibrate(steps=60, probes=16, seed=4, use_graph=True)
        torch.cuda.synchronize()
        for key in ("u_bar", "v_bar", "d", "e"):
            assert torch.equal(again[key], ref[key]), key


def test_batched_plan_matches_per_matrix_oracle():
    """Several uneven matrices in one plan: matrix b uses sign batch index b."""
    from paper_1602_06621_amd import Plan

    shapes = [(130, 40), (64, 64), (1, 7), (257, 200), (90, 23)]
    mats = []
    for i, (m, n) in enumerate(shapes):
        L = poisson_lengths(m, 4.0, n, 50 + i)
        mats.append(scaled_sparse(m, n, L, 2.0, 60 + i))
    with Plan([_gpu(c) for c in mats], max_probes=8) as plan:
        out = plan.equilibrate(steps=70, probes=8, seed=77)
        ub = out["u_bar"].cpu().numpy()
        vb = out["v_bar"].cpu().numpy()
    r0 = c0 = 0
    for b, c in enumerate(mats):
        al, be = A1.default_alpha_beta(c.m, c.n)
        o = A1.equilibrate(c.to_scipy(), al, be, 0.1, 10.0, 70, k=8, seed=77, batch=b)
        assert np.abs(ub[r0:r0 + c.m] - o["u_bar"]).max() <= TOL
        assert np.abs(vb[c0:c0 + c.n] - o["v_bar"]).max() <= TOL
        r0 += c.m
        c0 += c.n


def test_batched_plan_one_probe_whole_run_without_chaos():
    """The same batch with one probe per step over 400 steps at gamma = 1 (no chaos):
    every matrix elementwise at 1e-10 against the oracle with its own batch index."""
    from paper_1602_06621_amd import Plan

    shapes = [(130, 40), (64, 64), (1, 7), (257, 200), (90, 23)]
    mats = [scaled_sparse(m, n, poisson_lengths(m, 4.0, n, 50 + i), 2.0, 60 + i) for i, (m, n) in enumerate(shapes)]
    with Plan([_gpu(c) for c in mats], max_probes=1) as plan:
        out = plan.equilibrate(gamma=1.0, steps=400, probes=1, seed=77, use_graph=True)
        ub = out["u_bar"].cpu().numpy()
        vb = out["v_bar"].cpu().numpy()
    r0 = c0 = 0
    worst = 0.0
    for b, c in enumerate(mats):
        al, be = A1.default_alpha_beta(c.m, c.n)
        o = A1.equilibrate(c.to_scipy(), al, be, 1.0, 10.0, 400, k=1, seed=77, batch=b)
        worst = max(worst, np.abs(ub[r0:r0 + c.m] - o["u_bar"]).max(), np.abs(vb[c0:c0 + c.n] - o["v_bar"]).max())
        r0 += c.m
        c0 += c.n
    _say("batched k=1 gamma=1: worst", worst)
    assert worst <= 1e-10


def test_batched_plan_with_batch_base_warm_start_and_offset():
    """Batched plan run with sign batch base 5, per-matrix warm starts (concatenated in plan
    order) and t0 = 10: matrix b must equal the oracle with batch 5 + b and its slice of
    the warm start."""
    from paper_1602_06621_amd import Plan

    shapes = [(150, 60), (40, 90), (1, 5), (300, 120)]
    mats = [scaled_sparse(m, n, poisson_lengths(m, 4.0, n, 70 + i), 1.5, 80 + i) for i, (m, n) in enumerate(shapes)]
    rng = np.random.default_rng(3)
    u0s = [rng.normal(0, 0.5, m) for m, _ in shapes]
    v0s = [rng.normal(0, 0.5, n) for _, n in shapes]
    with Plan([_gpu(c) for c in mats], max_probes=8) as plan:
        out = plan.equilibrate(None, None, 0.1, 10.0, 60, 8, 9, t0=10, batch=5,
                               u0=torch.tensor(np.concatenate(u0s), device="cuda"),
                               v0=torch.tensor(np.concatenate(v0s), device="cuda"), use_graph=True)
        ub, vb = out["u_bar"].cpu().numpy(), out["v_bar"].cpu().numpy()
    r0 = c0 = 0
    for b, c in enumerate(mats):
        al, be = A1.default_alpha_beta(c.m, c.n)
        o = A1.equilibrate(c.to_scipy(), al, be, 0.1, 10.0, 60, k=8, seed=9, t0=10, u0=u0s[b], v0=v0s[b],
                           batch=5 + b)
        assert np.abs(ub[r0:r0 + c.m] - o["u_bar"]).max() <= TOL
        assert np.abs(vb[c0:c0 + c.n] - o["v_bar"]).max() <= TOL
        r0 += c.m
        c0 += c.n


@pytest.fixture(scope="module")
def config1():
    """The headline workload at full size: CSR 1e6 x 5e5, 10 uniform columns per row,
    values N(0,1) e^(r_i + c_j), r, c ~ N(0, 2^2)."""
    return scaled_sparse(10**6, 5 * 10**5, 10, 2.0, 1001)


def test_full_size_first_steps_elementwise(config1):
    """Full-size parity on every output after 3 steps (the oracle takes ~1 s per step)."""
    from paper_1602_06621_amd import Plan

    _say("full size, 3 steps")
    al, be = A1.default_alpha_beta(config1.m, config1.n)
    with Plan([_gpu(config1)], max_probes=16) as plan:
        g = plan.equilibrate(al, be, 0.1, 10.0, steps=3, probes=16, seed=2001, use_graph=True)
        ub, vb = g["u_bar"].cpu().numpy(), g["v_bar"].cpu().numpy()
    o = A1.equilibrate(config1.to_scipy(), al, be, 0.1, 10.0, 3, k=16, seed=2001)
    err = max(np.abs(ub - o["u_bar"]).max(), np.abs(vb - o["v_bar"]).max())
    _say("max err", err)
    assert err <= TOL


def test_full_size_benchmarked_run(config1):
    """The benchmarked run itself (full size, k = 16, gamma = 0.1, M = 10, seed 2001, one
    launch per step under graph replay) after 500, 1000 and all 2000 steps, against the
    stored oracle run (tests/golden/make_long_runs.py; every 13th row and column):
    elementwise at 1e-5.  (The running average after T steps does not depend on the steps
    that follow.)  Shorter prefixes are not well posed at this tolerance: under random
    relative perturbations of z of 2^-43 per step -- the size of the 8-byte descriptors'
    rounding -- the oracle's own u_bar moves by 3.9e-5 after 100 steps and 1.0e-5 after 200
    (the early steps amplify perturbations and keep a weight of order 1/T^2 in u_bar); at
    the stored checkpoints the same experiment gives 1.6e-6, 4.0e-7 and 1.0e-7, and the GPU
    run was measured at 1.4e-6, 3.5e-7 and 8.7e-8."""
    import os

    from paper_1602_06621_amd import Plan

    ref = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c1_prefix.npz"))
    st = int(ref["stride"])
    al, be = A1.default_alpha_beta(config1.m, config1.n)
    with Plan([_gpu(config1)], max_probes=16) as plan:
        for T in ref["checkpoints"]:
            _say(f"full size, benchmarked run, {T} steps")
            g = plan.equilibrate(al, be, 0.1, 10.0, steps=int(T), probes=16, seed=2001, use_graph=True)
            eu = np.abs(g["u_bar"].cpu().numpy()[::st] - ref[f"u_bar_{T}"]).max()
            ev = np.abs(g["v_bar"].cpu().numpy()[::st] - ref[f"v_bar_{T}"]).max()
            _say(f"T = {T}: max err u {eu:.3e} v {ev:.3e}")
            assert max(eu, ev) <= TOL


def test_full_size_20_steps_without_chaos(config1):
    """Full size, the benchmarked launch (one launch per step, graph replay), 20 steps at
    gamma = 1, where perturbations are not amplified: every output elementwise at 1e-9."""
    from paper_1602_06621_amd import Plan

    _say("full size, 20 steps, gamma 1")
    al, be = A1.default_alpha_beta(config1.m, config1.n)
    with Plan([_gpu(config1)], max_probes=16) as plan:
        g = plan.equilibrate(al, be, 1.0, 10.0, steps=20, probes=16, seed=2001, use_graph=True)
        ub, vb = g["u_bar"].cpu().numpy(), g["v_bar"].cpu().numpy()
    o = A1.equilibrate(config1.to_scipy(), al, be, 1.0, 10.0, 20, k=16, seed=2001)
    err = max(np.abs(ub - o["u_bar"]).max(), np.abs(vb - o["v_bar"]).max())
    _say("max err", err)
    assert err <= 1e-9


def test_full_size_bench_configuration_properties(config1):
    """2000 steps, k = 16, graph replay (the benchmarked launch): invariants that hold at
    any size -- box, iterate bound alpha^2/gamma carried to the average, finiteness,
    bitwise determinism."""
    from paper_1602_06621_amd import Plan

    al, be = A1.default_alpha_beta(config1.m, config1.n)
    _say("full size, 2000 steps")
    with Plan([_gpu(config1)], max_probes=16) as plan:
        g = plan.equilibrate(al, be, 0.1, 10.0, steps=2000, probes=16, seed=2001, use_graph=True)
        ub1 = g["u_bar"].clone()
        g2 = plan.equilibrate(al, be, 0.1, 10.0, steps=2000, probes=16, seed=2001, use_graph=True)
        assert torch.equal(ub1, g2["u_bar"])
        ub, vb = g["u_bar"].cpu().numpy(), g["v_bar"].cpu().numpy()
        _say("timing", plan.last_timing())
    assert np.all(np.isfinite(ub)) and np.all(np.isfinite(vb))
    assert np.abs(ub).max() <= 10.0 and np.abs(vb).max() <= 10.0
    assert ub.max() <= al**2 / 0.1 + 1e-12 and vb.max() <= be**2 / 0.1 + 1e-12


def test_batched_512_matrices_config2():
    """The batched workload at full size: 512 uneven CSR matrices (m ~ U[1k, 64k],
    n ~ U[m/4, m], Poisson(12) entries per row, sigma = 2) in one plan and one graph,
    k = 8, T = 1000 (the benchmarked run).  Eight matrices across the batch are compared
    elementwise with the oracle (matrix b uses sign batch index b); all 512 are checked for finiteness,
    box and iterate bounds.  (At T = 100 the oracle's own spread under 1e-16 perturbations
    reaches 3e-6 on some of these matrices; at T = 1000 it is ~1e-8.)"""
    from paper_1602_06621_amd import Csr, Plan
    from workloads import batched_sparse

    mats = batched_sparse(512, 1002)
    G = [Csr.from_arrays(c.m, c.n, c.row_ptr, c.col_idx, c.val) for c in mats]
    _say("config2 generated", sum(c.nnz for c in mats))
    with Plan(G, max_probes=8) as plan:
        out = plan.equilibrate(None, None, 0.1, 10.0, 1000, 8, 2002, use_graph=True)
        ub, vb = out["u_bar"].cpu().numpy(), out["v_bar"].cpu().numpy()
        _say("config2 timing", plan.last_timing())
    r0 = np.concatenate([[0], np.cumsum([c.m for c in mats])])
    c0 = np.concatenate([[0], np.cumsum([c.n for c in mats])])
    worst = 0.0
    for b in (0, 73, 146, 255, 300, 402, 509, 511):
        c = mats[b]
        al, be = A1.default_alpha_beta(c.m, c.n)
        o = A1.equilibrate(c.to_scipy(), al, be, 0.1, 10.0, 1000, k=8, seed=2002, batch=b)
        worst = max(worst, np.abs(ub[r0[b]:r0[b + 1]] - o["u_bar"]).max(), np.abs(vb[c0[b]:c0[b + 1]] - o["v_bar"]).max())
        _say("config2 matrix", b, "err", worst)
    assert worst <= TOL
    assert np.all(np.isfinite(ub)) and np.all(np.isfinite(vb))
    assert np.abs(ub).max() <= 10 and np.abs(vb).max() <= 10
    for b in range(512):
        al, be = A1.default_alpha_beta(mats[b].m, mats[b].n)
        assert ub[r0[b]:r0[b + 1]].max() <= al**2 / 0.1 + 1e-12
        assert vb[c0[b]:c0[b + 1]].max() <= be**2 / 0.1 + 1e-12


def _two_part_case(m, n, mean, seed):
    L = poisson_lengths(m, mean, n, seed)
    return scaled_sparse(m, n, L, 2.0, seed + 1)


def _split_modes(m, n, mode):
    """(rows mode, columns mode) with `mode` on the direction(s) that have a two-part
    layout: a direction gets one when the table it gathers (8 bytes per index of the
    other direction, padded to whole slices) exceeds 6 MiB."""
    big = lambda cnt: -(-cnt // 64) * 64 * 8 > 6 * 2**20
    return (mode if big(n) else 0), (mode if big(m) else 0)


@pytest.mark.parametrize("m,n,k", [(900_000, 250_000, 8), (200_000, 850_000, 8), (900_000, 250_000, 24)])
def test_two_part_mode_bitwise_equal_one_part(m, n, k):
    """A single matrix whose gathered table exceeds one XCD's L2 has a two-part layout for
    that direction.  Mode 1 (two launches over the halves of the table, FP64 partial sums
    in between) keeps the entry order of the sums, so it equals mode 0 bit for bit."""
    from paper_1602_06621_amd import Plan

    _say(f"two-part {m}x{n} k={k}")
    A = _two_part_case(m, n, 5.0, 700 + k)
    with Plan([_gpu(A)], max_probes=k) as plan:
        out = {}
        for mode in (0, 1):
            plan.set_tuning(8, *_split_modes(m, n, mode))
            g = plan.equilibrate(None, None, 0.1, 10.0, 25, k, 31, use_graph=True)
            out[mode] = {key: v.clone() for key, v in g.items()}
    for key in ("u_bar", "v_bar"):
        assert torch.equal(out[0][key], out[1][key])


@pytest.mark.parametrize("k,mode", [(16, 1), (24, 1), (16, 0)])
def test_two_part_one_step_matches_oracle(k, mode):
    """Two-part column direction (row table 7.2 MB) with empty rows: one step from random
    in-box states (t0 > 0 as in a warm start) against one oracle step.  Whole runs at this
    size are not comparable elementwise at short T: the oracle's own u_bar moves by 3e-5
    after 40 steps under 1e-16 relative perturbations of z (measured on this matrix and
    on a fixed-length one of the same size)."""
    from paper_1602_06621_amd import Plan

    A = _two_part_case(900_000, 250_000, 5.0, 811)
    al, be = A1.default_alpha_beta(A.m, A.n)
    As = A.to_scipy()
    rng = np.random.default_rng(k)
    worst = 0.0
    with Plan([_gpu(A)], max_probes=k) as plan:
        plan.set_tuning(8, *_split_modes(A.m, A.n, mode))
        for t0 in (0, 7, 100):
            u = np.clip(rng.normal(0, 1.5, A.m), -10, 10)
            v = np.clip(rng.normal(0, 1.5, A.n), -10, 10)
            g = plan.equilibrate(al, be, 0.1, 10.0, 1, k, 43, t0=t0, u0=torch.tensor(u, device="cuda"),
                                 v0=torch.tensor(v, device="cuda"))
            o = A1.equilibrate(As, al, be, 0.1, 10.0, 1, k=k, seed=43, t0=t0, u0=u, v0=v)
            for key in ("u_bar", "v_bar"):
                d = np.abs(g[key].cpu().numpy() - o[key]) / np.maximum(1.0, np.abs(o[key]))
                worst = max(worst, d.max())
    _say("two-part one-step worst rel err", mode, worst)
    assert worst <= 1e-11


def test_set_tuning_rejects_missing_layout():
    from paper_1602_06621_amd import Plan
    from paper_1602_06621_amd._ffi import MfeError

    with Plan([_gpu(scaled_sparse(300, 200, 4, 1.0, 3))], max_probes=4) as plan:
        with pytest.raises(MfeError):
            plan.set_tuning(8, 1, 0)
        with pytest.raises(MfeError):
            plan.set_tuning(5, 0, 0)
        with pytest.raises(MfeError):
            plan.set_tuning(1, 2, 2, 2)
        with pytest.raises(MfeError):
            plan.set_tuning(1, 2, 2, -1, 2)
        with pytest.raises(MfeError):
            plan.set_tuning(1, 2, 2, -1, -1, 384)
        plan.set_tuning(16, 0, 0)
        plan.set_tuning(1, 2, 2, 1)
        plan.set_tuning(1, 2, 2, -1, 0)


def test_autotune_keeps_results_bitwise():
    """The autotuner times every launch configuration and keeps the fastest; results after
    tuning equal those before, bit for bit (batched plan, and a single matrix whose
    column direction has a two-part layout)."""
    from paper_1602_06621_amd import Plan

    shapes = [(2000, 900), (513, 512), (7, 3), (4000, 1500)]
    mats = [scaled_sparse(m, n, poisson_lengths(m, 6.0, n, 90 + i), 2.0, 95 + i) for i, (m, n) in enumerate(shapes)]
    big = _two_part_case(900_000, 250_000, 5.0, 811)
    for group, k in ((mats, 8), ([big], 16)):
        with Plan([_gpu(c) for c in group], max_probes=k) as plan:
            a = plan.equilibrate(None, None, 0.1, 10.0, 30, k, 5, use_graph=True)
            a = {key: v.clone() for key, v in a.items()}
            choice = plan.autotune(None, None, 0.1, 10.0, k, 5, trial_steps=5)
            _say("autotune", choice)
            assert choice["loads_in_flight"] in (1, 2, 4, 8, 16)
            assert choice["stream_hints"] in (0, 1)
            assert choice["slice_order"] in (-1, 0, 1)
            assert choice["workgroup_threads"] in (256, 512, 1024)
            # 1, 2, 4, 8, 16 loads x (one launch per step with either stream-hint setting,
            # with each fixed slice order and with 512 threads per workgroup (and 1024 for
            # k = 8), one launch per direction, and for the single matrix (k = 16) its column
            # direction's two-part form)
            assert choice["candidates"] == (35 if len(group) == 1 else 35)
            b = plan.equilibrate(None, None, 0.1, 10.0, 30, k, 5, use_graph=True)
            b = {key: v.clone() for key, v in b.items()}
            c = plan.equilibrate(None, None, 0.1, 10.0, 30, k, 5, use_graph=False)
            for key in ("u_bar", "v_bar"):
                assert torch.equal(b[key], c[key])
                assert torch.equal(a[key], b[key])


def test_slice_order_bitwise_equal():
    """The longest-first slice order only changes which wavefront takes which slice: runs
    with either fixed order (and the default rule) give the same results bit for bit,
    through the one-launch step and through the split kernels of a small plan."""
    from paper_1602_06621_amd import Plan

    for csr, k in ((scaled_sparse(140_000, 70_000, poisson_lengths(140_000, 9.0, 70_000, 41), 2.0, 42), 16),
                   (scaled_sparse(3000, 1100, poisson_lengths(3000, 7.0, 1100, 43), 2.0, 44), 8)):
        with Plan([_gpu(csr)], max_probes=k) as plan:
            out = {}
            for order in (-1, 0, 1):
                plan.set_tuning(1, 2, 2, -1, order)
                g = plan.equilibrate(None, None, 0.1, 10.0, 40, k, 3, use_graph=True)
                out[order] = {key: v.clone() for key, v in g.items()}
        for key in ("u_bar", "v_bar"):
            assert torch.equal(out[0][key], out[1][key])
            assert torch.equal(out[-1][key], out[1][key])


def test_workgroup_size_bitwise_equal():
    """256, 512 and 1024 threads per workgroup of the one-launch step change only which
    workgroup runs which slices: results are equal bit for bit (one slot in flight, and
    16; a single matrix with k = 16, where 1024 runs as 512, and a batch of uneven matrices
    with k = 8)."""
    from paper_1602_06621_amd import Plan

    single = [scaled_sparse(140_000, 70_000, poisson_lengths(140_000, 9.0, 70_000, 47), 2.0, 48)]
    batch = [scaled_sparse(m, n, poisson_lengths(m, 8.0, n, 60 + i), 2.0, 70 + i)
             for i, (m, n) in enumerate(((70_000, 30_000), (66_000, 66_000), (90_000, 25_000)))]
    for group, k in ((single, 16), (batch, 8)):
        with Plan([_gpu(c) for c in group], max_probes=k) as plan:
            out = {}
            for nb in (1, 16):
                for wg in (0, 512, 1024):
                    plan.set_tuning(nb, 2, 2, -1, -1, wg)
                    g = plan.equilibrate(None, None, 0.1, 10.0, 30, k, 7, use_graph=True)
                    out[(nb, wg)] = {key: v.clone() for key, v in g.items()}
        ref = out[(1, 0)]
        for cfg, g in out.items():
            for key in ("u_bar", "v_bar"):
                assert torch.equal(g[key], ref[key]), cfg


def test_stream_hints_bitwise_equal():
    """Non-temporal and plain loads and stores of the entry and state streams read and
    write the same values: runs under either setting (and the size rule) are equal bit
    for bit, for the one-slot kernel and for 16 slots in flight."""
    from paper_1602_06621_amd import Plan

    csr = scaled_sparse(140_000, 70_000, poisson_lengths(140_000, 9.0, 70_000, 45), 2.0, 46)
    with Plan([_gpu(csr)], max_probes=16) as plan:
        out = {}
        for nb in (1, 16):
            for hint in (-1, 0, 1):
                plan.set_tuning(nb, 2, 2, hint)
                g = plan.equilibrate(None, None, 0.1, 10.0, 30, 16, 9, use_graph=True)
                out[(nb, hint)] = {key: v.clone() for key, v in g.items()}
    ref = out[(1, 0)]
    for cfg, g in out.items():
        for key in ("u_bar", "v_bar"):
            assert torch.equal(g[key], ref[key]), cfg


def test_ceiling_probes_measure():
    """The ceiling probes run and return positive times; a sorted-row gather from a table
    that fits one XCD's L2 is not slower than twice the uniformly random one."""
    import paper_1602_06621_amd as mfe

    t_rand = mfe.probe_gather(1 << 20, 1_000_000, 1, reps=2)
    t_sort = mfe.probe_gather_sorted(1 << 20, 1_000_000, 10, reps=2)
    t_stream = mfe.probe_stream(64 << 20, reps=2)
    _say("probes", t_rand, t_sort, t_stream)
    assert t_rand > 0 and t_sort > 0 and t_stream > 0
    assert t_sort < 2 * t_rand


def test_mismatched_targets_run_with_a_warning():
    """m alpha^2 != n beta^2 (Section 1): the run succeeds and mfe_last_error holds a
    warning naming the relation; with the paper's alpha, beta it holds nothing."""
    from paper_1602_06621_amd import Plan, equilibrate, last_error

    csr = scaled_sparse(400, 200, 5, 1.0, 23)
    A = _gpu(csr)
    equilibrate(A, 1.0, 1.0, 0.1, 10.0, 5, 4, 1)
    assert last_error().startswith("warning:") and "Section 1" in last_error()
    al, be = A1.default_alpha_beta(csr.m, csr.n)
    equilibrate(A, al, be, 0.1, 10.0, 5, 4, 1)
    assert last_error() == ""
    with Plan([A, _gpu(scaled_sparse(300, 300, 4, 1.0, 24))], max_probes=4) as plan:
        plan.equilibrate([al, 1.0], [be, 1.0], steps=3, probes=4, seed=1)
        assert last_error() == ""
        plan.equilibrate([al, 1.0], [be, 2.0], steps=3, probes=4, seed=1)
        assert last_error().startswith("warning:") and "matrix 1" in last_error()
