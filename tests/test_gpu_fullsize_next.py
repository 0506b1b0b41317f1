"""Full-size parity of the Section 6 variants and of the CCP consumer, at the sizes and in
the launch configuration bench.py measures (graph replay): the headline matrix
(1,000,000 x 500,000) with per-index targets and with 16 x 8 blocks, Algorithm 2 on the
symmetric 1,000,000 x 1,000,000 matrix, and CCP on the 10,000 x 20,000 Lasso matrix.
The FP64 oracle runs the first steps at full size (~1-5 s per step); elementwise
comparison at 1e-5 as elsewhere (the oracle's spread over three steps from the zero
start is far below it)."""
import os
import sys

import numpy as np
import pytest
import torch

from oracle import algorithm1 as A1
from oracle import ccp
from oracle import variants as V
from workloads import lasso_rhs, paper_sparse, scaled_sparse, symmetric_sparse

pytestmark = pytest.mark.gpu
TOL = 1e-5
# 500-step runs at gamma = 4, where the oracle's own spread under 1e-13 relative changes
# of the estimates peaks below 5e-10 and is ~1e-13 to 3e-12 at step 500
TOL_CONTRACTING = 1e-9
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gpu(csr):
    from paper_1602_06621_amd import Csr

    return Csr.from_arrays(csr.m, csr.n, csr.row_ptr, csr.col_idx, csr.val)


@pytest.fixture(scope="module")
def headline():
    return scaled_sparse(1_000_000, 500_000, 10, 2.0, 1001)


def test_full_size_targets_and_blocks(headline):
    """The bench's variant runs on the headline matrix, 3 graph-replayed steps each."""
    from paper_1602_06621_amd import Plan

    c = headline
    al, be = A1.default_alpha_beta(c.m, c.n)
    g = np.random.default_rng(5)
    rt = al**2 * g.uniform(0.5, 2.0, c.m)
    ct = be**2 * g.uniform(0.5, 2.0, c.n)
    rp = list(range(0, c.m, 16)) + [c.m]
    cp = list(range(0, c.n, 8)) + [c.n]
    As = c.to_scipy()
    with Plan([_gpu(c)], max_probes=16) as plan:
        _say("full size targets")
        plan.set_targets(torch.tensor(rt, device="cuda"), torch.tensor(ct, device="cuda"))
        out = plan.equilibrate(al, be, 0.1, 10.0, 3, 16, 2001, use_graph=True)
        ut, vt = out["u_bar"].cpu().numpy(), out["v_bar"].cpu().numpy()
        plan.set_targets(None, None)
        _say("full size blocks")
        plan.set_blocks(rp, cp)
        out = plan.equilibrate(al, be, 0.1, 10.0, 3, 16, 2001, use_graph=True)
        ubl, vbl, dbl = out["u_bar"].cpu().numpy(), out["v_bar"].cpu().numpy(), out["d"].cpu().numpy()
    o = V.equilibrate_general(As, 0.1, 10.0, 3, k=16, seed=2001, row_target=rt, col_target=ct)
    err = max(np.abs(ut - o["u_bar"]).max(), np.abs(vt - o["v_bar"]).max())
    _say("targets err", err)
    assert err <= TOL
    o = V.equilibrate_general(As, 0.1, 10.0, 3, k=16, seed=2001, row_ptr=rp, col_ptr=cp, alpha=al, beta=be)
    err = max(np.abs(ubl - o["u_bar"]).max(), np.abs(vbl - o["v_bar"]).max())
    _say("blocks err", err)
    assert err <= TOL
    assert np.allclose(dbl, o["d"], rtol=TOL, atol=0)


def _variant_inputs(c):
    """Targets and block boundaries of the variant runs (as tests/golden/make_long_runs.py
    draws them)."""
    al, be = A1.default_alpha_beta(c.m, c.n)
    g = np.random.default_rng(5)
    rt = al**2 * g.uniform(0.5, 2.0, c.m)
    ct = be**2 * g.uniform(0.5, 2.0, c.n)
    rp = list(range(0, c.m, 16)) + [c.m]
    cp = list(range(0, c.n, 8)) + [c.n]
    return al, be, rt, ct, rp, cp


@pytest.mark.parametrize("kind", ["var_targets", "var_blocks"])
def test_full_size_variants_500_steps(headline, kind):
    """The variant runs at the bench's size over 500 graph-replayed steps, against the
    stored oracle runs (every 13th index; written by tests/golden/make_long_runs.py, which
    calls only the oracle).  The runs use gamma = 4: at the bench's gamma = 0.1 both
    variants are chaotic at this size (1e-13 relative changes of the estimates move the
    oracle's own u_bar by 0.6 within 50 steps with targets and 0.05 within 100 with
    blocks), while at gamma = 4 such changes stay below 5e-10 and die out."""
    from paper_1602_06621_amd import Plan

    ref = np.load(os.path.join(GOLDEN, kind + ".npz"))
    st, T, gamma = int(ref["stride"]), int(ref["steps"]), float(ref["gamma"])
    al, be, rt, ct, rp, cp = _variant_inputs(headline)
    with Plan([_gpu(headline)], max_probes=16) as plan:
        if kind == "var_targets":
            plan.set_targets(torch.tensor(rt, device="cuda"), torch.tensor(ct, device="cuda"))
        else:
            plan.set_blocks(rp, cp)
        out = plan.equilibrate(al, be, gamma, 10.0, T, 16, 2001, use_graph=True)
        ub, vb = out["u_bar"].cpu().numpy(), out["v_bar"].cpu().numpy()
    err = max(np.abs(ub[::st] - ref["u_bar"]).max(), np.abs(vb[::st] - ref["v_bar"]).max())
    _say(kind, T, "steps err", err)
    assert err <= TOL_CONTRACTING


def test_full_size_symmetric_500_steps():
    """Algorithm 2 at the bench's size over 500 graph-replayed steps, against the stored
    oracle run (every 13th index), at gamma = 4 (at gamma = 0.1 this run is chaotic too:
    1e-13 relative changes of the estimates move u_bar by 2e-3 within 50 steps)."""
    from paper_1602_06621_amd import Plan

    ref = np.load(os.path.join(GOLDEN, "var_symmetric.npz"))
    st, T, gamma = int(ref["stride"]), int(ref["steps"]), float(ref["gamma"])
    S = symmetric_sparse(1_000_000, 5, 2.0, 1005)
    with Plan.symmetric_plan(_gpu(S), max_probes=16) as plan:
        out = plan.equilibrate(1.0, 1.0, gamma, 10.0, T, 16, 2001, use_graph=True)
        ub = out["u_bar"].cpu().numpy()
    err = np.abs(ub[::st] - ref["u_bar"]).max()
    _say("symmetric", T, "steps err", err)
    assert err <= TOL_CONTRACTING


def test_full_size_symmetric():
    """Algorithm 2 on the bench's symmetric 1,000,000 x 1,000,000 matrix, 3 steps."""
    from paper_1602_06621_amd import Plan

    S = symmetric_sparse(1_000_000, 5, 2.0, 1005)
    _say("full size symmetric", S.nnz)
    with Plan.symmetric_plan(_gpu(S), max_probes=16) as plan:
        out = plan.equilibrate(1.0, 1.0, 0.1, 10.0, 3, 16, 2001, use_graph=True)
        ub = out["u_bar"].cpu().numpy()
    o = V.equilibrate_symmetric(S.to_scipy(), 1.0, 0.1, 10.0, 3, k=16, seed=2001)
    err = np.abs(ub - o["u_bar"]).max()
    _say("symmetric err", err)
    assert err <= TOL


def test_full_size_ccp():
    """CCP on the bench's Lasso (10,000 x 20,000, 1% dense), equilibrated by 100 steps of
    the oracle's Algorithm 1: the estimated norm against ARPACK's, then 300 iterations
    with the oracle's norm, x elementwise."""
    from paper_1602_06621_amd import Plan

    c = paper_sparse(10_000, 20_000, 0.01, 1006)
    As = c.to_scipy()
    b, _ = lasso_rhs(As, 1007)
    lam = ccp.default_lambda(As, b)
    al, be = A1.default_alpha_beta(c.m, c.n)
    eq = A1.equilibrate(As, al, be, 0.1, np.log(1e4), 100, k=1, seed=2006)
    d, e = eq["d"], eq["e"]
    ref_norm = ccp.op_norm(As, d, e)
    o = ccp.ccp_lasso(As, b, lam, 300, d=d, e=e, norm=ref_norm)
    _say("full size ccp")
    with Plan([_gpu(c)], max_probes=1) as plan:
        nrm, it = plan.op_norm(torch.tensor(d, device="cuda"), torch.tensor(e, device="cuda"))
        x, info, _ = plan.ccp_lasso(torch.tensor(b, device="cuda"), lam, torch.tensor(d, device="cuda"),
                                    torch.tensor(e, device="cuda"), iters=300, op_norm=ref_norm)
    _say("norm", nrm, ref_norm, it)
    assert abs(nrm - ref_norm) <= 1e-8 * ref_norm
    x = x.cpu().numpy()
    err = np.max(np.abs(x - o["x"])) / np.max(np.abs(o["x"]))
    _say("ccp err", err)
    assert err <= 1e-9
