"""Host checks of integer arithmetic the kernels do in floating point.

The tile step's loops and its parity-class loops split an item index q into a row and
a column with a float reciprocal of the row length n: row = trunc((q + 1/2) * fl(1/n)),
all in IEEE single precision (correctly rounded reciprocal and product, truncating
conversion).  The kernels assert at compile time that rows hold at most 64 points and
that q stays below 4096; this test checks every such pair against the integer quotient.
"""
import numpy as np


def test_float_row_split_is_exact_for_the_kernel_sizes():
    q = np.arange(4096, dtype=np.int64)
    qf = q.astype(np.float32) + np.float32(0.5)
    for n in range(1, 65):
        rn = np.float32(1.0) / np.float32(n)
        row = (qf * rn).astype(np.float32).astype(np.int64)   # float32 product, truncation
        assert np.array_equal(row, q // n), n
