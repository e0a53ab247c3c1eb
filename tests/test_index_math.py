"""Host checks of arithmetic tricks in the kernels.

The tile step's loops and its parity-class loops split an item index q into a row and
a column with a float reciprocal of the row length n: row = trunc((q + 1/2) * fl(1/n)),
all in IEEE single precision (correctly rounded reciprocal and product, truncating
conversion).  The kernels assert at compile time that rows hold at most 64 points and
that q stays below 4096; the first test checks every such pair against the integer
quotient.  The other index splits (parity classes, gathers, write-backs) divide by row
and plane sizes known only at run time, with the same formula; the second test checks
it for every divisor of a tile (rows and planes of up to 64 x 64 points) and indices
below 2^14, and near the bound 2^21 the error analysis gives.  The third checks the
reductions' 64-bit integer maximum of |detail| values.
"""
import numpy as np


def test_float_row_split_is_exact_for_the_kernel_sizes():
    q = np.arange(4096, dtype=np.int64)
    qf = q.astype(np.float32) + np.float32(0.5)
    for n in range(1, 65):
        rn = np.float32(1.0) / np.float32(n)
        row = (qf * rn).astype(np.float32).astype(np.int64)   # float32 product, truncation
        assert np.array_equal(row, q // n), n


def _fdiv(p, d):
    pf = p.astype(np.float32) + np.float32(0.5)
    return (pf * (np.float32(1.0) / np.float32(d))).astype(np.float32).astype(np.int64)


def test_float_split_by_run_time_sizes_is_exact():
    p = np.arange(1 << 14, dtype=np.int64)
    for n0 in range(1, 65):
        assert np.array_equal(_fdiv(p, n0), p // n0), n0
        for n1 in range(1, 65):
            d = n0 * n1
            assert np.array_equal(_fdiv(p, d), p // d), (n0, n1)
    # near the bound, for divisors up to 4096
    top = np.arange((1 << 21) - 4096, 1 << 21, dtype=np.int64)
    for d in range(1, 4097):
        assert np.array_equal(_fdiv(top, d), top // d), d


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
