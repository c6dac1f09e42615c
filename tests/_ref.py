"""Integer-only references for the builder (no floating point, no oracle).

feistel_order: the counter-based epoch order from its definition -- a
4-round balanced Feistel network on 2h bits with the SplitMix64 finaliser as
round function (Steele, Lea & Flood 2014), round keys the SplitMix64 stream
from the key, restricted to [0, n) by cycle walking (Black & Rogaway 2002).

minibatch_sort: per minibatch and mode, the positions sorted stably by row.
"""
import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z):
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def epoch_key(shuffle_seed, epoch, salt=0):
    with np.errstate(over="ignore"):
        return np.uint64(shuffle_seed) ^ (
            GOLDEN * np.uint64(2 * epoch + 1 + 2 * salt))


def feistel_order(n, key):
    key = np.uint64(key)
    with np.errstate(over="ignore"):
        ks = []
        st = key
        for _ in range(4):
            st = st + GOLDEN
            ks.append(_mix64(np.array([st], dtype=np.uint64))[0])
        bits = 2
        while (1 << bits) < n:
            bits += 1
        if bits & 1:
            bits += 1
        h = np.uint64(bits // 2)
        mask = np.uint64((1 << (bits // 2)) - 1)

        def enc(x):
            L = x >> h
            R = x & mask
            for k in ks:
                L, R = R, L ^ (_mix64(R ^ k) & mask)
            return (L << h) | R

        x = enc(np.arange(n, dtype=np.uint64))
        bad = x >= np.uint64(n)
        while bad.any():
            x[bad] = enc(x[bad])
            bad = x >= np.uint64(n)
    return x.astype(np.int64)


def minibatch_sort(rows_in_order):
    """Stable sort of one minibatch's rows: (positions, sorted rows)."""
    pos = np.argsort(rows_in_order, kind="stable").astype(np.int32)
    return pos, rows_in_order[pos].astype(np.int32)
