"""Integer-only references for the builder (no floating point, no oracle).

feistel_order: the counter-based epoch order from its definition -- a
4-round Feistel network on the mixed-radix domain Z_a x Z_b, a = ceil(sqrt n),
b = ceil(n / a) (Black & Rogaway 2002): x = L b + R, a round maps
(L in Z_p, R in Z_q) to (R, (L + F(R)) mod p) and swaps the moduli; F is the
MurmurHash3 32-bit finaliser of R ^ k scaled into [0, p) by (h p) >> 32; round
keys are the high halves of the SplitMix64 stream from the key (Steele, Lea &
Flood 2014); values >= n are cycle-walked.

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


def _fmix32(h):
    m = np.uint64(0xFFFFFFFF)
    h = h ^ (h >> np.uint64(16))
    h = (h * np.uint64(0x85EBCA6B)) & m
    h = h ^ (h >> np.uint64(13))
    h = (h * np.uint64(0xC2B2AE35)) & m
    return h ^ (h >> np.uint64(16))


def feistel_order(n, key):
    key = np.uint64(key)
    with np.errstate(over="ignore"):
        ks = []
        st = key
        for _ in range(4):
            st = st + GOLDEN
            ks.append(_mix64(np.array([st], dtype=np.uint64))[0]
                      >> np.uint64(32))
    a = 1
    while a * a < n:
        a += 1
    b = -(-n // a)
    A, B = np.uint64(a), np.uint64(b)

    def enc(x):
        L, R = x // B, x % B
        p, q = A, B
        for k in ks:
            f = (_fmix32(R ^ k) * p) >> np.uint64(32)
            L, R = R, (L + f) % p
            p, q = q, p
        return L * B + R

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
