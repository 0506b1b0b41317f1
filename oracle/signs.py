"""Probe signs for Algorithm 1 (Section 3.1: entries iid uniform on {-1, +1}).

The paper only asks for iid fair signs.  The library and this oracle agree on one
counter-based stream so that both see the same probes (the oracle side uses
numpy's Philox, the GPU side its own Philox4x64-10 written from Salmon et al.,
"Parallel random numbers: as easy as 1, 2, 3", SC'11):

  key     = (seed, ctrl),  ctrl = (batch << 34) | (step << 2) | side
  block c = Philox4x64-10(key, counter = (c + 1, 0, 0, 0)) -> words x0..x3
  stream bit g = 256*c + q  is bit (q mod 64) of word x_(q div 64)
  sign of (index i, probe p) with k probes per index = stream bit i*k + p;
  bit 1 means -1, bit 0 means +1.

side 0: s, indexed by column j (probes pushed through A);
side 1: w, indexed by row i (probes pushed through A^T);
sides 2 and 3 are free for sketch probes.
numpy's Philox increments its counter before each block, so starting it at
counter 0 yields block c at counter c + 1.
"""
from __future__ import annotations

import numpy as np

MAX_BATCH = 1 << 30
MAX_STEP = 1 << 32


def stream_ctrl(batch: int, step: int, side: int) -> int:
    if not (0 <= batch < MAX_BATCH and 0 <= step < MAX_STEP and 0 <= side < 4):
        raise ValueError("batch, step or side out of range")
    return (batch << 34) | (step << 2) | side


def stream_words(seed: int, batch: int, step: int, side: int, nwords: int) -> np.ndarray:
    """First `nwords` 64-bit words of the stream (whole Philox blocks are drawn)."""
    key = np.array([seed & ((1 << 64) - 1), stream_ctrl(batch, step, side)], dtype=np.uint64)
    gen = np.random.Philox(key=key)
    nblk = (nwords + 3) // 4
    return gen.random_raw(4 * nblk).astype(np.uint64)[:nwords]


def sign_bits(seed: int, batch: int, step: int, side: int, count: int, k: int) -> np.ndarray:
    """uint8 array [count, k] of sign bits (1 -> -1) for indices 0..count-1."""
    nbits = count * k
    words = stream_words(seed, batch, step, side, (nbits + 63) // 64)
    bits = np.unpackbits(words.astype("<u8").view(np.uint8), bitorder="little")[:nbits]
    return bits.reshape(count, k)


def signs(seed: int, batch: int, step: int, side: int, count: int, k: int) -> np.ndarray:
    """FP64 array [count, k] of +-1 probe entries."""
    return 1.0 - 2.0 * sign_bits(seed, batch, step, side, count, k).astype(np.float64)
