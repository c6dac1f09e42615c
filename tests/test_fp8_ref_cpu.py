"""The e4m3 emulation used by the FP8 GPU tests, against values fixed by
the format definition (largest value, subnormal spacing, ties to even)."""
import numpy as np

from tests import _fp8


def test_code_table_spans_the_format():
    v = _fp8._VALS
    assert len(v) == 127 and v[0] == 0.0
    assert v[1] == 2.0 ** -9          # smallest subnormal
    assert v[8] == 2.0 ** -6          # smallest normal
    assert v[-1] == 448.0             # largest finite value
    assert np.all(np.diff(v) > 0)


def test_round_to_nearest_ties_to_even():
    x = np.array([1.0625, 1.1875, 440.0, -3.3, 2.0 ** -10, 1.5 * 2.0 ** -9,
                  0.0])
    y = np.array([1.0, 1.25, 448.0, -3.25, 0.0, 2.0 ** -8, 0.0])
    assert np.array_equal(_fp8.e4m3_round(x), y)


def test_quantize_scales_the_largest_entry_to_448():
    x = np.array([[0.5, -2.0, 1.0], [0.0, 0.0, 0.0]], dtype=np.float32)
    q = _fp8.quantize(x, axis=1)
    s = np.float64(np.float32(2.0) / np.float32(448.0))
    assert q[0, 1] == -448.0 * s            # the max maps to code 448
    assert np.all(q[1] == 0.0)              # all-zero row: scale 0
    assert np.allclose(q[0], x[0], rtol=2 ** -4)
