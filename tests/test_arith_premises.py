"""Arithmetic facts the sieve kernel's setup relies on, checked exhaustively
on the host in the same IEEE single precision the GPU uses (round to nearest
even for the conversion and the product, truncation back to an integer).

floor(x / 3) for x < 2^23 is computed as (uint32)((float)x * fl(1/3)); the
start of a prime's strikes in a class uses j + k*p < 2^23 with j < 2^21 and
p < 2^21 (or p <= 2^11 in the one-prime-per-wave tier).

The first odd multiple of p at or above a window start is computed in double
precision, exactly (gb_first_odd_multiple and the segment kernel's form below
2^52); tests/first_multiple_premise.c checks that arithmetic on the host,
compiled with gcc with contraction off as in the kernels, against 128-bit
integer remainders.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest


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


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_double_first_multiple_is_exact():
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "first_multiple_premise.c")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "fm")
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-o", exe, src, "-lm"], check=True)
        r = subprocess.run([exe, "3000000"], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().splitlines()[-1] == "0", r.stdout
