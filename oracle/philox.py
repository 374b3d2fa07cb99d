"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC 2011).

TEST INFRASTRUCTURE ONLY (see the package docstring).

One block maps a 128-bit counter (c0..c3) and a 64-bit key (k0, k1) to four 32-bit words by
ten rounds of: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 (full 64-bit products),
c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key is bumped by the Weyl constants
(W0, W1) between rounds.

Draws of the approximate count (both sides follow this layout):
  key = (seed mod 2^32, seed div 2^32);
  uniform coordinate q = p*d + k of sample point p in trial t after s splits:
      block (q div 2, s, t, 1), words (0,1) for even q and (2,3) for odd q,
      u = ((a >> 5) * 2^26 + (b >> 6)) / 2^53 in [0, 1);
  split dimension of trial t after s splits: block (0, s, t, 2), word 0, dim = (w * d) >> 32;
  kept half: same block, word 1, bit 0 (0 keeps the lower part).
"""
from __future__ import annotations

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF

TAG_SAMPLE = 1
TAG_SPLIT = 2


def philox4x32_10(counter, key):
    c0, c1, c2, c3 = (int(v) & MASK for v in counter)
    k0, k1 = (int(v) & MASK for v in key)
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def seed_key(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & MASK, seed >> 32


def uniform53(a: int, b: int) -> float:
    return ((a >> 5) * 67108864 + (b >> 6)) / 9007199254740992.0


def sample_uniforms(seed: int, trial: int, split: int, n_points: int, d: int):
    """[n_points][d] uniforms in [0, 1) as a list of lists of Python floats."""
    key = seed_key(seed)
    out = [[0.0] * d for _ in range(n_points)]
    cache = {}
    for p in range(n_points):
        for k in range(d):
            q = p * d + k
            blk = q >> 1
            if blk not in cache:
                cache = {blk: philox4x32_10((blk, split, trial, TAG_SAMPLE), key)}
            w = cache[blk]
            a, b = (w[0], w[1]) if (q & 1) == 0 else (w[2], w[3])
            out[p][k] = uniform53(a, b)
    return out


def split_choice(seed: int, trial: int, split: int, d: int):
    """(dimension, side) of the split of trial ``trial`` after ``split`` splits."""
    w = philox4x32_10((0, split, trial, TAG_SPLIT), seed_key(seed))
    return (w[0] * d) >> 32, w[1] & 1
