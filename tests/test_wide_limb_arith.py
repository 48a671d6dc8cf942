"""Host check of the arithmetic the Baillie-PSW test past 2^64 runs on, compiled
here with g++ as plain C++: the Montgomery product over N = 3, 4, 5 28-bit
limbs (gb_wide_limbs.h, R = 2^(28 N), by tests/wide_limb_arith.cpp) -- for
seeded moduli of the sizes each N serves and operands at the limits of the
documented bounds (limbs up to 2^30 - 1, values up to 8q - 1) the product is
congruent to a b / R mod q, its limbs below the top one are normalized and its
value is below a b / R + q, and the reduction and subtraction helpers give the
exact residues, and the product by a small signed Q gives Q x mod q at most
3q -- and the 128-bit helpers (gb_wide_u128.h).  Exact integers
decide."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def val(limbs):
    return sum(x << (28 * j) for j, x in enumerate(limbs))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_limb_montgomery_product_and_helpers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "limbs")
        subprocess.run(["g++", "-O2", "-std=c++17", "-o", exe,
                        os.path.join(HERE, "wide_limb_arith.cpp")], check=True)
        out = subprocess.run([exe, "40000", "7"], capture_output=True, text=True, timeout=600,
                             check=True).stdout.splitlines()
    assert len(out) == 120000
    lazy = 0
    sizes = set()
    qs = set()
    for mline, hline, qline in zip(out[0::3], out[1::3], out[2::3]):
        f = mline.split()
        assert f[0] == "mont"
        N, qi = int(f[1]), int(f[2], 16)
        R = 1 << (28 * N)
        ql, al, bl, rl = ([int(x, 16) for x in f[3 + N * k:3 + N * (k + 1)]] for k in range(4))
        q, a, b, r = val(ql), val(al), val(bl), val(rl)
        assert q % 2 == 1 and (1 << 60) < q < R >> 12
        sizes.add(N)
        assert (qi * q) % (1 << 28) == (1 << 28) - 1          # qi = -q^-1 mod 2^28
        assert max(al + bl) < (1 << 30) and a < 8 * q and b < 8 * q
        lazy += max(al + bl) >= (1 << 28)
        assert (r * R - a * b) % q == 0
        assert max(rl[:N - 1]) < (1 << 28)
        assert r * R < a * b + q * R                          # r < a b / R + q
        h = hline.split()
        assert h[0] == "help"
        yl, zl, sl = ([int(x, 16) for x in h[1 + N * k:1 + N * (k + 1)]] for k in range(3))
        assert val(yl) == r % q and max(yl[:N - 1]) < (1 << 28)   # canonical
        assert val(zl) == 2 * q - r and max(zl[:N - 1]) < (1 << 28)
        assert val(sl) == (r + 3 * (2 * q - r)) % q
        g = qline.split()
        assert g[0] == "mulq"
        Q = int(g[1])
        ml = [int(x, 16) for x in g[2:2 + N]]
        m = val(ml)
        assert 0 < abs(Q) <= (1 << 14) + 1
        assert (m - Q * r) % q == 0 and 0 <= m <= 3 * q   # Q r mod q, at most 3q
        assert max(ml[:N - 1]) < (1 << 28)
        qs.add(Q)
    assert sizes == {3, 4, 5}
    assert {1, -1, (1 << 14) + 1, -(1 << 14) - 1} <= qs
    assert lazy > 10000   # the lazy operand forms were exercised


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_u128_small_product_and_montgomery_one():
    """gb_wide_u128.h on the host: x * c mod q for residues x (random, next to
    q, next to multiples of q over c) and constants c of 1 to 40 bits, and
    2^(28 N) mod q for the limb count N of q, for seeded moduli of 64 to 128
    bits; exact integers decide."""
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "u128")
        subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-o", exe,
                        os.path.join(HERE, "wide_u128_arith.cpp")], check=True)
        out = subprocess.run([exe, "200000", "11"], capture_output=True, text=True, timeout=600,
                             check=True).stdout.splitlines()
    assert len(out) == 200000
    near = 0
    for line in out:
        f = line.split()
        qh, ql, xh, xl, k, rh, rl = (int(v, 16) for v in f[:7])
        rbits, oh, ol = int(f[7]), int(f[8], 16), int(f[9], 16)
        q, x, r, one = (qh << 64) | ql, (xh << 64) | xl, (rh << 64) | rl, (oh << 64) | ol
        assert 0 <= x < q and 1 <= k < (1 << 40)
        assert r == (x * k) % q, (q, x, k)
        assert rbits in (84, 112, 140) and q < (1 << (rbits - 12))
        assert one == (1 << rbits) % q, q
        near += min((x * k) % q, q - (x * k) % q) < (q >> 40)
    assert near > 1000   # products next to multiples of q were exercised
