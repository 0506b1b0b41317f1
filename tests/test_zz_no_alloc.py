"""The allocation-free entry point (mfe_equilibrate_noalloc, dense FP64) against
mfe_equilibrate through the C ABI: two calls in a row, the second on a smaller input, on
each of the three dense launch paths (register-resident single workgroup, LDS single
workgroup, one launch per direction and step).  Both entry points run the same kernels,
so the outputs must agree bit for bit; the scratch array keeps the previous call's
contents, which a smaller second call must not see."""
import sys

import numpy as np
import pytest
import torch

from oracle import algorithm1 as A1
from workloads import scaled_dense

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dense(A):
    from paper_1602_06621_amd import Dense

    return Dense(torch.tensor(A, device="cuda"))


@pytest.mark.parametrize("first,second", [
    ((200, 100, 1, 300), (150, 80, 1, 200)),      # register-resident path (k = 1, m <= 200, n <= 128)
    ((600, 300, 4, 100), (300, 200, 4, 60)),      # one workgroup, LDS state
    ((3000, 700, 4, 20), (2000, 500, 3, 15)),     # one launch per direction and step
])
def test_noalloc_matches_allocating_entry_point(first, second):
    from paper_1602_06621_amd import equilibrate, equilibrate_noalloc

    for i, (m, n, k, T) in enumerate((first, second)):
        _say(f"noalloc call {i + 1}: {m}x{n} k={k} T={T}")
        A = _dense(scaled_dense(m, n, 1.5, 40 + m))
        al, be = A1.default_alpha_beta(m, n)
        ref = equilibrate(A, al, be, 0.1, 10.0, T, k, 7)
        got = equilibrate_noalloc(A, al, be, 0.1, 10.0, T, k, 7)
        torch.cuda.synchronize()
        for key in ("d", "e", "u_bar", "v_bar"):
            assert torch.equal(got[key], ref[key]), (i, key)


def test_noalloc_warm_start_and_rejections():
    """A warm start with a step offset agrees too; a shape beyond the scratch is refused
    with EDIM before any work, and other kinds with EUNSUPPORTED."""
    from paper_1602_06621_amd import Csr, MfeError, equilibrate, equilibrate_noalloc

    m, n = 200, 100
    A = _dense(scaled_dense(m, n, 1.5, 41))
    rng = np.random.default_rng(3)
    u0 = torch.tensor(rng.uniform(-1, 1, m), device="cuda")
    v0 = torch.tensor(rng.uniform(-1, 1, n), device="cuda")
    ref = equilibrate(A, None, None, 0.1, 10.0, 50, 1, 9, t0=20, u0=u0, v0=v0)
    got = equilibrate_noalloc(A, None, None, 0.1, 10.0, 50, 1, 9, t0=20, u0=u0, v0=v0)
    torch.cuda.synchronize()
    assert torch.equal(got["u_bar"], ref["u_bar"]) and torch.equal(got["v_bar"], ref["v_bar"])
    big = _dense(np.zeros((300000, 10)))
    with pytest.raises(MfeError, match="scratch") as ei:
        equilibrate_noalloc(big, None, None, 0.1, 10.0, 5, 1, 1)
    assert ei.value.status == -2
    csr = Csr.from_arrays(2, 2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32),
                          np.array([1.0, 2.0], np.float32))
    with pytest.raises(MfeError) as ei:
        equilibrate_noalloc(csr, None, None, 0.1, 10.0, 5, 1, 1)
    assert ei.value.status == -6
