"""Counter-based random numbers (oracle; test infrastructure only).

Philox4x32-10 follows Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
as easy as 1, 2, 3" (SC'11): a 4 x 32-bit counter and a 2 x 32-bit key, ten
rounds, each round multiplying counter words 0 and 2 by the published
multipliers and mixing the high halves with the other words and the key; the
key is bumped by the published Weyl constants between rounds.

Bounded integers use Lemire's multiply-shift method with rejection ("Fast
random integer generation in an interval", ACM TOMACS 2019): for bound s,
x * s is a 64-bit product; its high word is the draw unless its low word falls
below (2^32 - s) mod s, in which case the next 32-bit word is tried.

Stream layout used by the walk estimators (the same on both sides):
  key  = (seed mod 2^32, seed >> 32)
  ctr  = (c0, c1, c2, (step << 8) | j)
  one Philox call yields 4 words; a draw consumes words in order, moving to
  j + 1 when all four are used.  Each (c0, c1, c2, step) names a fresh stream.
"""
from __future__ import annotations

import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10; inputs are arrays (or scalars) of 32-bit
    values, returned as four uint64 arrays holding 32-bit words."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & _MASK for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def key_of(seed: int):
    seed = int(seed)
    return seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF


def stream_words(seed, c0, c1, c2, step, j):
    k0, k1 = key_of(seed)
    c3 = (np.asarray(step, dtype=np.uint64) << np.uint64(8)) | np.asarray(j, dtype=np.uint64)
    return np.stack(philox4x32_10(c0, c1, c2, c3, k0, k1), axis=0)  # (4, ...)


def bounded(seed, c0, c1, c2, step, bound):
    """Lemire draw in [0, bound) from stream (c0, c1, c2, step), vectorised.
    `bound` must be in [1, 2^32)."""
    c0 = np.atleast_1d(np.asarray(c0, dtype=np.uint64))
    shape = c0.shape
    c1 = np.broadcast_to(np.asarray(c1, dtype=np.uint64), shape)
    c2 = np.broadcast_to(np.asarray(c2, dtype=np.uint64), shape)
    step = np.broadcast_to(np.asarray(step, dtype=np.uint64), shape)
    s = np.broadcast_to(np.asarray(bound, dtype=np.uint64), shape)
    if np.any(s == 0) or np.any(s >= np.uint64(1 << 32)):
        raise ValueError("bound outside [1, 2^32)")
    out = np.zeros(shape, dtype=np.uint64)
    todo = np.ones(shape, dtype=bool)
    thresh = (np.uint64(1 << 32) - s) % s
    j = 0
    while todo.any():
        idx = np.nonzero(todo)
        words = stream_words(seed, c0[idx], c1[idx], c2[idx], step[idx], j)
        pending = np.ones(idx[0].shape[0], dtype=bool)
        res = np.zeros(idx[0].shape[0], dtype=np.uint64)
        for wi in range(4):
            m = words[wi] * s[idx]
            lo = m & _MASK
            ok = pending & ~((lo < s[idx]) & (lo < thresh[idx]))
            res[ok] = m[ok] >> np.uint64(32)
            pending &= ~ok
        done_here = ~pending
        sel = tuple(ax[done_here] for ax in idx)
        out[sel] = res[done_here]
        todo[sel] = False
        j += 1
        if j > 255:
            raise RuntimeError("Lemire stream exhausted")
    return out.astype(np.int64)


def uniform53(seed, c0, c1, c2, step):
    """Uniform double in [0, 1) with 53 random bits: (w0 * 2^21 + (w1 >> 11)) * 2^-53,
    words 0 and 1 of stream (c0, c1, c2, step) at j = 0."""
    w = stream_words(seed, c0, c1, c2, step, 0)
    top = (w[0] << np.uint64(21)) + (w[1] >> np.uint64(11))
    return top.astype(np.float64) * (2.0 ** -53)
