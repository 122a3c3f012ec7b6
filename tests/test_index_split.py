"""The calibration kernel splits flat indices i (below m*n <= 256*32 and
n*n*C <= 32*32*4) by run-time divisors d (n, C, n*n, ceil(n/2)) with a float32
quotient and one integer correction instead of an integer division.  This
checks that method in float32 arithmetic (IEEE multiply and correctly rounded
reciprocal, as on the device): the uncorrected quotient is within one of the
exact one, and the corrected quotient and remainder equal divmod, for every
index up to 2^14 and every divisor that the kernel can use."""
import numpy as np


def split(i, d):
    inv = np.float32(1.0) / np.float32(d)
    q = (i.astype(np.float32) * inv).astype(np.int64)   # truncation, i >= 0
    r = i - q * d
    q_fix = q + np.where(r >= d, 1, np.where(r < 0, -1, 0))
    return q, q_fix


def test_float_quotient_within_one_and_corrected_exactly():
    i = np.arange(1 << 14, dtype=np.int64)
    divisors = sorted(set(range(1, 33)) | {n * n for n in range(1, 33)} | {(n + 1) // 2 for n in range(1, 33)})
    for d in divisors:
        q, q_fix = split(i, d)
        exact = i // d
        assert np.all(np.abs(q - exact) <= 1), d
        assert np.array_equal(q_fix, exact), d
        assert np.all((i - q_fix * d >= 0) & (i - q_fix * d < d)), d
