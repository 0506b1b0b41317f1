"""Pins for the probe-sign stream used by the oracle (Section 3.1 asks for iid fair signs)."""
import os

import numpy as np
import pytest

from oracle import signs
from tests.philox_ref import philox4x64, stream_bit

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x64_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_python_philox_matches_published_kat():
    for ctr, key, out in _kat():
        assert philox4x64(ctr, key) == out


@pytest.mark.parametrize("seed,batch,step,side", [(0, 0, 1, 0), (2001, 0, 7, 1), (2**63 + 5, 3, 123456, 2)])
def test_oracle_words_are_philox_blocks(seed, batch, step, side):
    words = signs.stream_words(seed, batch, step, side, 12)
    ctrl = signs.stream_ctrl(batch, step, side)
    for c in range(3):
        assert [int(w) for w in words[4 * c:4 * c + 4]] == philox4x64([c + 1, 0, 0, 0], [seed, ctrl])


@pytest.mark.parametrize("k", [1, 3, 16, 64, 100])
def test_sign_bit_layout(k):
    seed, batch, step, side, count = 99, 1, 5, 1, 37
    bits = signs.sign_bits(seed, batch, step, side, count, k)
    ctrl = signs.stream_ctrl(batch, step, side)
    rng = np.random.default_rng(k)
    for _ in range(40):
        i = int(rng.integers(count))
        p = int(rng.integers(k))
        assert bits[i, p] == stream_bit(seed, ctrl, i * k + p)


def test_streams_differ_by_side_step_batch():
    base = signs.sign_bits(1, 0, 1, 0, 64, 16)
    for args in [(1, 0, 1, 1), (1, 0, 2, 0), (1, 1, 1, 0), (2, 0, 1, 0)]:
        other = signs.sign_bits(args[0], args[1], args[2], args[3], 64, 16)
        assert not np.array_equal(base, other)


def test_signs_are_fair_and_pairwise_independent():
    s = signs.signs(7, 0, 3, 0, 20000, 16)
    assert set(np.unique(s)) == {-1.0, 1.0}
    assert abs(s.mean()) < 0.01
    c = (s.T @ s) / s.shape[0]
    off = c - np.diag(np.diag(c))
    assert np.max(np.abs(off)) < 0.03


def test_ctrl_range_checks():
    with pytest.raises(ValueError):
        signs.stream_ctrl(0, 2**32, 0)
    with pytest.raises(ValueError):
        signs.stream_ctrl(2**30, 0, 0)
    with pytest.raises(ValueError):
        signs.stream_ctrl(0, 0, 4)
