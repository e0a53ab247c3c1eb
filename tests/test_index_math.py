"""Host checks of arithmetic tricks in the kernels.

The tile step's loops and its parity-class loops split an item index q into a row and
a column with a float reciprocal of the row length n: row = trunc((q + 1/2) * fl(1/n)),
all in IEEE single precision (correctly rounded reciprocal and product, truncating
conversion).  The kernels assert at compile time that rows hold at most 64 points and
that q stays below 4096; the first test checks every such pair against the integer
quotient.  The second checks the reductions' 64-bit integer maximum of |detail| values.
"""
import numpy as np


def test_float_row_split_is_exact_for_the_kernel_sizes():
    q = np.arange(4096, dtype=np.int64)
    qf = q.astype(np.float32) + np.float32(0.5)
    for n in range(1, 65):
        rn = np.float32(1.0) / np.float32(n)
        row = (qf * rn).astype(np.float32).astype(np.int64)   # float32 product, truncation
        assert np.array_equal(row, q // n), n


def test_unsigned_maximum_of_detail_magnitudes_propagates_nan():
    """The workgroup reductions take the maximum of |detail| values (sign bit clear) as
    64-bit unsigned integers: that is the value maximum, and any NaN wins."""
    rng = np.random.default_rng(7)
    for trial in range(200):
        v = np.abs(rng.standard_normal(64)) * 10.0 ** rng.integers(-300, 300)
        v[rng.integers(0, 64, 3)] = 0.0
        if trial % 3 == 0:
            v[rng.integers(0, 64)] = np.inf
        if trial % 4 == 0:
            v[rng.integers(0, 64)] = abs(np.float64(np.nan))
        u = np.abs(v).view(np.uint64).max().view(np.float64)
        if np.isnan(v).any():
            assert np.isnan(u)
        else:
            assert u == np.max(v)
