"""Pure-Python Philox4x64-10, written from the published definition (Salmon et al., SC'11).

Test-side reference used to pin the oracle's sign stream (which draws its words
from numpy) and the GPU's sign words.  Round: with multipliers M0, M1,
(hi0, lo0) = M0 * x0, (hi1, lo1) = M1 * x2 as 128-bit products, the new state is
(hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0); the key is bumped by the Weyl
constants before every round but the first.
"""

MASK = (1 << 64) - 1
M0, M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
W0, W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B


def philox4x64(counter, key, rounds=10):
    x0, x1, x2, x3 = counter
    k0, k1 = key
    for r in range(rounds):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * x0
        p1 = M1 * x2
        x0, x1, x2, x3 = (p1 >> 64) ^ x1 ^ k0, p1 & MASK, (p0 >> 64) ^ x3 ^ k1, p0 & MASK
    return [x0, x1, x2, x3]


def stream_bit(seed, ctrl, g):
    """Bit g of the sign stream for key (seed, ctrl): block g // 256 at counter block+1."""
    blk, q = divmod(g, 256)
    words = philox4x64([blk + 1, 0, 0, 0], [seed, ctrl])
    return (words[q // 64] >> (q % 64)) & 1
