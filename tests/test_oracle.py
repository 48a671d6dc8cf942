"""Pins for the CPU oracle against facts that do not come from the oracle itself.

Each test checks the oracle against the definition of the problem (paper Sec. 1,
Sec. 3.3), published constants (prime counts, known pseudoprimes), brute force
on small inputs, an independent library (sympy) and invariants of the method
(merge of disjoint ranges, independence from the segment size).  A plausible
slip in the oracle -- a dropped base, an off-by-one window, a wrong halo, a
swapped tie-break -- fails at least one of them.
"""
import math
import os
import random

import numpy as np
import pytest

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U64 = (1 << 64) - 1


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(x) for x in line.split()])
    return rows


def _td_is_prime(q):
    """Textbook trial division, written independently of the oracle."""
    if q < 2:
        return False
    if q % 2 == 0:
        return q == 2
    d = 3
    while d * d <= q:
        if q % d == 0:
            return False
        d += 2
    return True


def _td_table(limit):
    return [q for q in range(limit + 1) if _td_is_prime(q)]


# --- base-prime sieve ---------------------------------------------------------

@pytest.mark.parametrize("row", [r for r in _golden_rows("prime_counts.txt") if r[0] <= 10**8])
def test_prime_counts(row):
    x, count, largest = row
    p = O.primes(x)
    assert len(p) == count
    assert int(p[-1]) == largest
    assert int(p[0]) == 2


@pytest.mark.slow
@pytest.mark.parametrize("row", [r for r in _golden_rows("prime_counts.txt") if r[0] > 10**8])
def test_prime_counts_large(row):
    x, count, largest = row
    p = O.primes(x)
    assert len(p) == count
    assert int(p[-1]) == largest


def test_primes_match_trial_division():
    p = O.primes(20000)
    assert [int(x) for x in p] == _td_table(20000)


def test_isqrt_exact():
    cases = [0, 1, 2, 3, 4, 15, 16, 17, U64, (1 << 64) - (1 << 33) + 1, ((1 << 32) - 1) ** 2,
             ((1 << 32) - 1) ** 2 - 1, 10**12, 10**12 - 1]
    rng = random.Random(7)
    cases += [rng.getrandbits(64) for _ in range(2000)]
    for x in cases:
        assert O.isqrt(x) == math.isqrt(x), x


# --- primality (Phase 2 test, Sec. 3.3/3.4) -----------------------------------

def test_is_prime_small_vs_trial_division():
    for q in range(0, 30000):
        assert O.is_prime(q) == _td_is_prime(q), q


def test_is_prime_known_values():
    assert not O.is_prime(561)               # Carmichael 3*11*17
    assert not O.is_prime(2047)              # strong pseudoprime to base 2 (23*89)
    assert 151 * 751 * 28351 == 3215031751
    assert not O.is_prime(3215031751)        # strong pseudoprime to bases 2, 3, 5, 7
    # strong pseudoprime to every prime base up to 23; only bases 29, 31, 37
    # of the twelve reject it
    assert 149491 * 747451 * 34233211 == 3825123056546413051
    assert not O.is_prime(3825123056546413051)
    assert 3 * 5 * 17 * 257 * 641 * 65537 * 6700417 == U64
    assert not O.is_prime(U64)
    assert O.is_prime(4294967291)            # largest prime below 2^32
    assert O.is_prime(U64 - 58)              # 2^64 - 59, largest prime below 2^64
    assert O.is_prime(2**61 - 1)             # Mersenne prime
    assert not O.is_prime((2**32 + 15) * (2**31 - 1))


def test_is_prime_large_vs_sympy():
    sympy = pytest.importorskip("sympy")
    rng = random.Random(11)
    vals = [rng.getrandbits(64) | 1 for _ in range(1500)]
    vals += [rng.randrange(1 << 32, 1 << 40) | 1 for _ in range(500)]
    vals += [int(sympy.randprime(1 << 63, 1 << 64)) for _ in range(100)]
    vals += [int(sympy.randprime(1 << 32, 1 << 33)) * 3 for _ in range(20)]
    for q in vals:
        assert O.is_prime(q) == bool(sympy.isprime(q)), q


# --- the verification itself --------------------------------------------------

def test_worked_values_4_to_30():
    rows = _golden_rows("pmin_4_30.txt")
    r = O.verify_range(4, 30, 65521, 3163, want_pmin=True)
    assert [int(x) for x in r["pmin"]] == [row[1] for row in rows]
    for n, p, q in rows:
        assert n == p + q and _td_is_prime(p) and _td_is_prime(q)
    assert r["verified"] == 14 and r["checksum"] == 53
    assert (r["max_p"], r["max_p_n"]) == (7, 30)
    assert r["n_unresolved"] == 0 and r["n_failed"] == 0


def _brute_pmin(nmax):
    table = _td_table(nmax)
    isp = bytearray(nmax + 1)
    for q in table:
        isp[q] = 1
    out = {}
    for n in range(4, nmax + 1, 2):
        for p in table:
            if isp[n - p]:
                out[n] = p
                break
    return out, isp, table


@pytest.fixture(scope="module")
def brute_1e5():
    return _brute_pmin(100000)


def test_pmin_brute_force_all_even_up_to_1e5(brute_1e5):
    bp, _, _ = brute_1e5
    r = O.verify_range(4, 100000, 65521, 3163, want_pmin=True, seg_evens=4096)
    assert [int(x) for x in r["pmin"]] == [bp[n] for n in range(4, 100001, 2)]
    assert r["verified"] == len(bp)
    assert r["checksum"] == sum(bp.values())
    mx = max(bp.values())
    assert (r["max_p"], r["max_p_n"]) == (mx, min(n for n, p in bp.items() if p == mx))


@pytest.mark.parametrize("P_max", [2, 3, 7, 31, 100])
def test_tiny_pmax_unresolved_matches_definition(brute_1e5, P_max):
    bp, isp, table = brute_1e5
    N = 40000
    r = O.verify_range(4, N, P_max, 1000, cap=N)
    expect_unres = []
    for n in range(4, N + 1, 2):
        ok = any(p <= P_max and p <= n - 2 and isp[n - p] for p in table if p <= P_max)
        if not ok:
            expect_unres.append(n)
    assert r["unresolved"] == expect_unres
    assert r["n_unresolved"] == len(expect_unres)
    # Phase 2 completes every miss: totals equal the unrestricted definition
    assert r["n_failed"] == 0
    assert r["verified"] == (N - 4) // 2 + 1
    assert r["checksum"] == sum(bp[n] for n in range(4, N + 1, 2))


def test_merge_and_segment_size_invariance():
    base = O.verify_range(4, 2_000_000, 65536, 2000, seg_evens=1 << 16)
    for seg in (1, 3, 1000, 77777, 1 << 20):
        if seg < 100:
            r = O.verify_range(4, 20000, 65536, 2000, seg_evens=seg)
            assert r == O.verify_range(4, 20000, 65536, 2000, seg_evens=1 << 16)
        else:
            assert O.verify_range(4, 2_000_000, 65536, 2000, seg_evens=seg) == base
    for M in (4, 1000, 123456, 1_999_998):
        lo = O.verify_range(4, M, 65536, 2000)
        hi = O.verify_range(M + 2, 2_000_000, 65536, 2000)
        m = O.merge(lo, hi)
        for f in O.FIELDS:
            assert m[f] == base[f], f
    assert base["verified"] + base["n_failed"] == (2_000_000 - 4) // 2 + 1


def test_normalization_edges():
    r = O.verify_range(0, 3, 100, 100)
    assert r["A"] > r["B"] and r["verified"] == 0
    r = O.verify_range(0, 4, 100, 100)
    assert (r["A"], r["B"], r["verified"], r["checksum"]) == (4, 4, 1, 2)
    r = O.verify_range(5, 9, 100, 100)
    assert (r["A"], r["B"], r["verified"], r["checksum"]) == (6, 8, 2, 6)
    r = O.verify_range(100, 50, 100, 100)
    assert r["verified"] == 0 and r["status"] == 0
    r = O.verify_range(U64, U64, 100, 2**32 - 1)
    assert r["A"] > r["B"] and r["verified"] == 0
    # invalid arguments
    assert O.verify_range(4, 100, 1, 100)["status"] == 1
    assert O.verify_range(4, 10**12, 100, 100)["status"] == 2   # table below isqrt(B)


def test_window_halo_is_needed():
    # p_min(n) can exceed the distance to the segment start: a one-even segment
    # still has to see q = n - p far below it.
    r1 = O.verify_range(4, 200000, 65536, 1000, seg_evens=1)
    r2 = O.verify_range(4, 200000, 65536, 1000, seg_evens=1 << 18)
    assert r1 == r2


def _mr_pmin(n, table_iter):
    for p in table_iter:
        if p > n // 2:
            return 0
        if O.is_prime(n - p):
            return p
    return 0


@pytest.mark.slow
def test_near_2_64_two_methods():
    """Sieve with primes to 2^32 against per-q Miller-Rabin on the top window."""
    T = 2**32 - 1
    count = 20000
    q0 = U64 - 2 * (count - 1)
    a = O.sieve_window(q0, count, T)
    b = O.is_prime_window(q0, count)
    assert np.array_equal(a, b)
    assert a.sum() > 0
    # and per-n minimal p at the very top of the u64 range
    small = [int(x) for x in O.primes(65536)[1:2000]]
    r = O.verify_range(U64 - 2 * 1500, U64, 65536, T, want_pmin=True)
    assert r["B"] == U64 - 1
    ns = range(r["A"], r["B"] + 1, 2)
    exp = [_mr_pmin(n, small) for n in ns]
    assert [int(x) for x in r["pmin"]] == exp
    assert r["checksum"] == sum(exp) % (1 << 64)


def test_mid_range_two_methods():
    T = 1 << 28
    count = 50000
    q0 = (1 << 56) + 1
    assert np.array_equal(O.sieve_window(q0, count, T), O.is_prime_window(q0, count))
    small = [int(x) for x in O.primes(65536)[1:3000]]
    A = (1 << 56) + 1000
    r = O.verify_range(A, A + 4000, 65536, T, want_pmin=True, seg_evens=333)
    exp = [_mr_pmin(n, small) for n in range(A, A + 4001, 2)]
    assert [int(x) for x in r["pmin"]] == exp
