"""FP8 (OCP e4m3) quantisation written from the format definition, used to
emulate the inputs of the FP8 contraction (no oracle arithmetic here).

e4m3: 1 sign bit, 4 exponent bits (bias 7), 3 mantissa bits; exponent 0 is
subnormal (m/8 * 2^-6), code S.1111.111 is NaN, there are no infinities and
the largest finite value is 448. Rounding is to nearest, ties to the even
code. A vector x is stored as codes q and one FP32 scale s with
    s = max|x| / 448,   q = e4m3(clamp(x * (448 / max|x|), -448, 448)),
every step in FP32 arithmetic, x ~= s * value(q) (an all-zero x has s = 0).
"""
import numpy as np


def _code_values():
    v = np.empty(128)
    for c in range(128):
        e, m = c >> 3, c & 7
        v[c] = (m / 8.0) * 2.0 ** -6 if e == 0 else (1 + m / 8.0) * 2.0 ** (e - 7)
    return v[:127]          # code 0x7f is NaN


_VALS = _code_values()


def e4m3_round(x):
    """Nearest e4m3 value of each entry of x (|x| <= 448), ties to even."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    hi = np.clip(np.searchsorted(_VALS, a), 1, len(_VALS) - 1)
    lo = hi - 1
    dlo, dhi = a - _VALS[lo], _VALS[hi] - a
    pick = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi,
                                            np.where(lo % 2 == 0, lo, hi)))
    return np.sign(x) * _VALS[pick]


def quantize(x, axis):
    """Dequantised FP8 form of x with one scale per slice along `axis`."""
    x = np.asarray(x, dtype=np.float32)
    m = np.max(np.abs(x), axis=axis, keepdims=True).astype(np.float32)
    with np.errstate(divide="ignore"):
        inv = np.where(m > 0, np.float32(448.0) / m, np.float32(0.0))
    inv = inv.astype(np.float32)
    y = np.clip((x * inv).astype(np.float32), -448.0, 448.0)
    s = (m / np.float32(448.0)).astype(np.float32)
    return e4m3_round(y) * s.astype(np.float64)
