"""Arithmetic facts the sieve kernel's setup relies on, checked exhaustively
on the host in the same IEEE single precision the GPU uses (round to nearest
even for the conversion and the product, truncation back to an integer).

floor(x / 3) for x < 2^23 is computed as (uint32)((float)x * fl(1/3)); the
start of a prime's strikes in a class uses j + k*p < 2^23 with j < 2^21 and
p < 2^21 (or p <= 2^11 in the one-prime-per-wave tier).
"""
import numpy as np


def test_float_divide_by_three_is_exact_below_2_23():
    third = np.float32(1.0) / np.float32(3.0)
    for lo in range(0, 1 << 23, 1 << 21):
        x = np.arange(lo, lo + (1 << 21), dtype=np.uint32)
        q = (x.astype(np.float32) * third).astype(np.uint32)
        assert np.array_equal(q, x // 3), lo


def test_float_divide_by_three_fails_later():
    # the bound is real: the trick breaks soon above 2^23, so the kernel's
    # operand bounds matter
    third = np.float32(1.0) / np.float32(3.0)
    x = np.arange(1 << 23, 1 << 24, dtype=np.uint32)
    q = (x.astype(np.float32) * third).astype(np.uint32)
    assert not np.array_equal(q, x // 3)
