"""Oracle: the seeded start vector drawn when the caller gives none (test infrastructure).

Section V shows that the polynomial built from v0 = b can be useless (its
residual polynomial swings far below zero on the Laplacian) and recommends a
random start vector with entries uniform on (-1, 1).  When no v0 is passed,
the library draws one itself, so both sides must produce the same vector from
a seed: each implements the same counter-based generator from its published
definition.

Generator: Philox4x64-10 (J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011).  A block maps a
256-bit counter (four 64-bit words, the first the least significant) and a
128-bit key (two words) to four 64-bit words by ten rounds; each round
multiplies words 0 and 2 by two fixed constants, takes the high and low
halves of the 128-bit products, swaps and XORs them with words 1 and 3 and the
key, and the key is advanced by two fixed Weyl increments between rounds.

Vector: entry i is word (i mod 4) of the block at counter floor(i/4) + 1 with
key (seed, 0) -- the same stream numpy's ``Philox(key=(seed, 0))`` bit
generator emits, whose counter is advanced before each block -- mapped to
(-1, 1) as 2 * (w >> 11) * 2^-53 - 1 (exact in float64).

Pinned in tests/test_oracle_rng.py against the generator's published
known-answer block (counter 0, key 0), against numpy's independent Philox
implementation, and by the statistics of U(-1, 1).
"""
from __future__ import annotations

import numpy as np

__all__ = ["philox4x64_10", "philox_words", "uniform_pm1"]

# round multipliers and Weyl key increments of Philox4x64 (published constants)
M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
ROUNDS = 10
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b):
    """(high, low) 64-bit halves of the 128-bit products a * b (uint64 arrays)."""
    a_lo, a_hi = a & _LO32, a >> _S32
    b_lo, b_hi = b & _LO32, b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _LO32) + (hl & _LO32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    lo = (mid << _S32) | (ll & _LO32)
    return hi, lo


def philox4x64_10(ctr, key):
    """Philox4x64-10 blocks.  ctr: uint64 array (..., 4); key: (2,) -> uint64 (..., 4)."""
    ctr = np.asarray(ctr, dtype=np.uint64)
    x0, x1, x2, x3 = (ctr[..., q].copy() for q in range(4))
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    with np.errstate(over="ignore"):
        for r in range(ROUNDS):
            hi0, lo0 = _mulhilo(M0, x0)
            hi1, lo1 = _mulhilo(M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
            if r + 1 < ROUNDS:
                k0 = k0 + W0
                k1 = k1 + W1
    return np.stack([x0, x1, x2, x3], axis=-1)


def philox_words(n, seed):
    """The first n 64-bit words of the stream with key (seed, 0), counters 1, 2, ..."""
    n = int(n)
    nblk = (n + 3) // 4
    ctr = np.zeros((nblk, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(1, nblk + 1, dtype=np.uint64)
    key = (np.uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), np.uint64(0))
    return philox4x64_10(ctr, key).reshape(-1)[:n]


def uniform_pm1(n, seed):
    """n float64 entries in (-1, 1): 2 * (w >> 11) * 2^-53 - 1 of the stream's words."""
    w = philox_words(n, seed)
    u = (w >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0
