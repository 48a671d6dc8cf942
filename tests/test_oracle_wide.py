"""Pins of the wide oracle (oracle/gb_oracle_wide.c): Goldbach verification
past 2^64 with primality of n - p decided by Baillie-PSW.

The oracle is pinned against what mathematics fixes: known primes and known
composites (Mersenne numbers with published factorizations), pseudoprimes of
each half of the test (strong pseudoprimes to base 2 must be caught by the
Lucas half, strong Lucas pseudoprimes by the base-2 half), an independent
library (sympy) on random 65..127-bit values, the deterministic 64-bit oracle
wherever both apply (BPSW has no pseudoprime below 2^64, so both must agree
exactly there), trial-division brute force on small ranges, and invariants
(merge of split ranges, normalization of the bounds)."""
import random

import pytest

from oracle import oracle as O

U64 = (1 << 64) - 1
FIELDS = ("A", "B", "P_max", "verified", "max_p", "max_p_n", "checksum", "n_unresolved",
          "n_failed", "unresolved")


def test_known_primes_and_composites():
    for e in (61, 89, 107, 127):            # Mersenne primes
        assert O.bpsw(2**e - 1), e
    # 2^67 - 1 = 193707721 * 761838257287 (Cole, 1903)
    assert 193707721 * 761838257287 == 2**67 - 1
    assert not O.bpsw(2**67 - 1)
    for e in (71, 73, 79, 83, 97, 101, 103, 109, 113):   # composite Mersenne numbers
        assert not O.bpsw(2**e - 1), e
    assert O.bpsw(2**64 + 13) and not O.bpsw(2**64 + 1)  # 2^64 + 1 = 274177 * 67280421310721
    assert 274177 * 67280421310721 == 2**64 + 1
    assert O.bpsw(U64 - 58) and not O.bpsw(U64)
    assert O.bpsw(2**128 - 159)                          # largest prime below 2^128


def test_each_half_of_the_test_is_needed():
    # strong pseudoprimes to base 2 (pass the first half): the Lucas half rejects them
    for n in (2047, 3277, 4033, 4681, 8321, 15841, 29341, 42799, 49141, 52633,
              3215031751, 3825123056546413051):
        assert not O.bpsw(n), n
    # strong Lucas pseudoprimes with Selfridge's parameters (pass the second
    # half): the base-2 half rejects them
    for n in (5459, 5777, 10877, 16109, 18971, 22499, 24569, 25199, 40309, 58519):
        assert not O.bpsw(n), n
    # perfect squares of primes have no Selfridge D; they are composite
    for p in (1000003, 4294967291, 2**61 - 1):
        assert not O.bpsw(p * p), p


def test_bpsw_vs_sympy_random_wide():
    sympy = pytest.importorskip("sympy")
    rng = random.Random(17)
    vals = [rng.getrandbits(rng.randrange(65, 128)) | 1 for _ in range(1500)]
    vals += [int(sympy.randprime(1 << 64, 1 << 65)) for _ in range(50)]
    vals += [int(sympy.randprime(1 << 126, 1 << 127)) for _ in range(30)]
    # products of two primes near 2^32..2^63, which trial division never catches
    vals += [int(sympy.randprime(1 << 32, 1 << 60)) * int(sympy.randprime(1 << 33, 1 << 64))
             for _ in range(40)]
    for q in vals:
        assert O.bpsw(q) == bool(sympy.isprime(q)), q


def test_bpsw_equals_deterministic_64bit_test():
    rng = random.Random(3)
    vals = list(range(0, 3000)) + [U64 - 2 * i for i in range(4000)]
    vals += [rng.getrandbits(64) | 1 for _ in range(4000)]
    for q in vals:
        assert O.bpsw(q) == O.is_prime(q), q


def test_isqrt128():
    rng = random.Random(5)
    import math
    for x in [0, 1, 2, 3, 4, 2**64, 2**64 - 1, 2**128 - 1, 2**126] + \
             [rng.getrandbits(128) for _ in range(300)]:
        assert O.isqrt128(x) == math.isqrt(x)


def _brute_pmin(n):
    def isprime(q):
        if q < 2:
            return False
        d = 2
        while d * d <= q:
            if q % d == 0:
                return False
            d += 1
        return True
    for p in range(2, n // 2 + 1):
        if isprime(p) and isprime(n - p):
            return p
    return 0


def test_small_range_against_trial_division():
    r = O.verify_range_wide(4, 3000, 65536, 100000, want_pmin=True)
    want = [_brute_pmin(n) for n in range(4, 3001, 2)]
    assert list(r["pmin"]) == want
    assert r["verified"] == len(want) and r["checksum"] == sum(want)
    m = max(want)
    assert r["max_p"] == m and r["max_p_n"] == 4 + 2 * want.index(m)


@pytest.mark.parametrize("AB,P", [((4, 20000), 65536), ((4, 20000), 7), ((10**12, 10**12 + 4000), 65536),
                                   ((U64 - 1 - 2 * 1500, U64), 65536), ((U64 - 2 * 300, U64), 31)])
def test_equals_64bit_oracle_below_2_64(AB, P):
    a = O.verify_range_wide(AB[0], AB[1], P, 2**32 - 1 if AB[1] > 10**13 else 10**6, cap=1 << 14)
    b = O.verify_range(AB[0], AB[1], P, 2**32 - 1 if AB[1] > 10**13 else 10**6, cap=1 << 14,
                       seg_evens=1 << 22)
    for f in FIELDS:
        assert a[f] == b[f], (f, a[f], b[f])


@pytest.mark.parametrize("A", [2**64, 2**64 + 2 * 98765, 2**80 + 2, 2**100, 2**127 + 2**64,
                               2**128 - 2 * 60 - 2])
def test_wide_windows_against_sympy(A):
    sympy = pytest.importorskip("sympy")
    B = min(A + 2 * 59, 2**128 - 2)
    r = O.verify_range_wide(A, B, 65536, 10**6, want_pmin=True)
    odd = [int(p) for p in O.primes(65536)[1:]]
    want = []
    for n in range(A, B + 1, 2):
        want.append(next((p for p in odd if sympy.isprime(n - p)), 0))
    assert list(r["pmin"]) == want
    assert r["checksum"] == sum(want) % 2**64 and r["verified"] == len(want)


def test_split_merge_and_normalization():
    A, B = 2**64 + 4, 2**64 + 2 * 1200
    whole = O.verify_range_wide(A, B, 65536, 10**6)
    cut = A + 2 * 577
    a = O.verify_range_wide(A, cut, 65536, 10**6)
    b = O.verify_range_wide(cut + 2, B, 65536, 10**6)
    m = O.merge(a, b)
    for f in ("verified", "checksum", "max_p", "max_p_n", "n_unresolved", "n_failed"):
        assert m[f] == whole[f], f
    # bounds round inward; 2^128 - 1 is odd, so the range ends at 2^128 - 2
    r = O.verify_range_wide(2**128 - 7, 2**128 - 1, 65536, 10**6)
    assert (r["A"], r["B"], r["verified"]) == (2**128 - 6, 2**128 - 2, 3)
    r = O.verify_range_wide(2**128 - 1, 2**128 - 1, 65536, 10**6)
    assert r["A"] > r["B"] and r["verified"] == 0


def test_tiny_pmax_unresolved_and_phase2():
    """With P_max = 7 most evens go to Phase 2 (BPSW over the next table
    primes): the list is the evens whose p_min exceeds 7, in order."""
    A, B = 2**70, 2**70 + 2 * 150
    full = O.verify_range_wide(A, B, 65536, 10**6, want_pmin=True)
    tiny = O.verify_range_wide(A, B, 7, 10**6, cap=1000)
    want = [A + 2 * i for i, p in enumerate(full["pmin"]) if p > 7]
    assert tiny["unresolved"] == want and tiny["n_unresolved"] == len(want)
    for f in ("verified", "checksum", "max_p", "max_p_n", "n_failed"):
        assert tiny[f] == full[f], f
