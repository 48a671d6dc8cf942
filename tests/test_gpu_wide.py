"""GPU parity past 2^64: gb_verify_range_u128 and gb_is_prime_u128 through the
C ABI against the wide CPU oracle (oracle/gb_oracle_wide.c), field by field,
bit-exact: windows just above 2^64, at and across 2^72 and 2^100 (where the
arithmetic changes its limb count), at 2^80, 2^127 and at the top of the u128
range, a range straddling 2^64 (the part below goes through the
64-bit path), one range cut into chunks of three sizes with ragged tails, tiny P_max with
Phase 2 and unresolved lists, normalization and refusals."""
import concurrent.futures as cf
import random

import pytest

pytestmark = pytest.mark.gpu

FIELDS = ("A", "B", "P_max", "verified", "max_p", "max_p_n", "checksum", "n_unresolved",
          "n_failed", "unresolved")
THREADS = 16


@pytest.fixture(scope="module")
def gb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2603_07850_amd as g
    g.lib()
    print("[gpu-wide] gb_base_primes(10^7)", flush=True)
    g.base_primes(10**7)
    return g


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    return oracle


def oracle_split(O, A, B, P_max, limit, pieces=THREADS, cap=1 << 12):
    """The wide oracle over [A, B] (even bounds), cut into pieces run on a thread
    pool and merged in order."""
    n = (B - A) // 2 + 1
    cuts = [A + 2 * ((n * i) // pieces) for i in range(pieces + 1)]
    jobs = [(cuts[i], cuts[i + 1] - 2) for i in range(pieces) if cuts[i + 1] - 2 >= cuts[i]]
    with cf.ThreadPoolExecutor(THREADS) as ex:
        parts = list(ex.map(lambda j: O.verify_range_wide(j[0], j[1], P_max, limit, cap=cap), jobs))
    out = parts[0]
    for p in parts[1:]:
        out = O.merge(out, p)
    out["A"], out["B"] = A, B
    return out


def same(g, o, what):
    for f in FIELDS:
        assert g[f] == o[f], (what, f, g[f], o[f])


def test_device_primality_u128(gb, O):
    import sympy
    rng = random.Random(23)
    vals = [2**89 - 1, 2**67 - 1, 2**127 - 1, 2**128 - 159, 2**64 + 13, 2**64 + 1, 2**64 - 59,
            2**107 - 1, 2**101 - 1, 4294967291, 2047, 3215031751]
    vals += [rng.getrandbits(rng.randrange(65, 128)) | 1 for _ in range(1500)]
    vals += [int(sympy.randprime(1 << 64, 1 << 127)) for _ in range(200)]
    # composites without small factors, and squares of primes above 2^32
    vals += [int(sympy.randprime(1 << 33, 1 << 62)) * int(sympy.randprime(1 << 33, 1 << 64))
             for _ in range(200)]
    vals += [int(sympy.randprime(1 << 33, 1 << 63)) ** 2 for _ in range(50)]
    vals += [rng.getrandbits(64) | 1 for _ in range(300)]
    print("[gpu-wide] is_prime_u128 on %d values" % len(vals), flush=True)
    got = gb.is_prime_u128(vals)
    for v, g in zip(vals, got):
        assert g == O.bpsw(v), v


# 2^72 and 2^100 are where the probe's arithmetic moves from 3 to 4 and from 4
# to 5 limbs (chosen per chunk by its last n): windows ending just below them
# and windows across them
WINDOWS = [2**64, 2**64 + 2 * 123457, 2**72 - 2 * 1500, 2**72 - 2 * 700, 2**80 + 2 * 77,
           2**100 - 2 * 1500, 2**100 - 2 * 700, 2**100, 2**127 + 2**64 + 6, 2**128 - 2 * 1500]


@pytest.mark.parametrize("A", WINDOWS, ids=lambda a: "2^%.2f" % (a.bit_length() - 1))
def test_windows_against_oracle(gb, O, A):
    B = min(A + 2 * 1499, 2**128 - 1)
    print("[gpu-wide] verify_range_u128(%d, %d)" % (A, B), flush=True)
    g = gb.verify_range_u128(A, B, 65536)
    o = oracle_split(O, A, B - (B & 1), 65536, 10**7)
    o["B"] = g["B"]
    same(g, o, A)
    assert g["verified"] == (g["B"] - g["A"]) // 2 + 1


def test_straddles_2_64(gb, O):
    """The part below 2^64 goes through the 64-bit path, which needs the table
    up to isqrt(2^64 - 2) = 2^32 - 1; every even resolves among the candidates
    p <= 2^16 (n_unresolved = 0), so the oracle's smaller table gives the same
    result."""
    A, B = 2**64 - 2 * 3000, 2**64 + 2 * 3000
    print("[gpu-wide] straddling 2^64", flush=True)
    gb.base_primes(2**32 - 1)
    try:
        g = gb.verify_range_u128(A, B, 65536)
        low = gb.verify_range(A, 2**64 - 1, 65536)
    finally:
        gb.base_primes(10**7)
    o = oracle_split(O, A, B, 65536, 10**7)
    assert o["n_unresolved"] == 0
    same(g, o, "straddle")
    # the part below 2^64 equals the 64-bit entry point's result
    lo = O.verify_range_wide(A, 2**64 - 1, 65536, 10**7)
    for f in ("verified", "checksum", "max_p", "max_p_n"):
        assert low[f] == lo[f]


def test_chunks_ragged(gb, O):
    """One range in one chunk (the default 2^26 evens), in chunks of 2^16 (two
    full and a ragged third) and of 2^12 (34, the last ragged): every split
    gives the oracle's result."""
    A = 2**64 + 2 * 10**9
    B = A + 2 * (2 * 65536 + 4321 - 1)
    o = oracle_split(O, A, B, 65536, 10**7)
    assert gb.get_wide_chunk_log2() == 26
    try:
        for lg, chunks in ((26, 1), (16, 3), (12, 34)):
            print("[gpu-wide] chunks of 2^%d evens" % lg, flush=True)
            gb.set_wide_chunk_log2(lg)
            g = gb.verify_range_u128(A, B, 65536)
            same(g, o, "chunks of 2^%d" % lg)
            assert gb.last_stats()["segments"] == chunks
    finally:
        gb.set_wide_chunk_log2(26)


@pytest.mark.parametrize("P", [7, 31, 1000])
def test_tiny_pmax_phase2(gb, O, P):
    A, B = 2**70, 2**70 + 2 * 700
    print("[gpu-wide] P_max %d" % P, flush=True)
    g = gb.verify_range_u128(A, B, P, unresolved_cap=1000)
    o = oracle_split(O, A, B, P, 10**7, cap=1000)
    same(g, o, "P_max %d" % P)


def test_normalization_and_refusals(gb, O):
    top = 2**128 - 1
    g = gb.verify_range_u128(top - 6, top, 65536)
    o = O.verify_range_wide(top - 6, top, 65536, 10**7)
    same(g, o, "top")
    assert (g["A"], g["B"], g["verified"]) == (top - 5, top - 1, 3)
    g = gb.verify_range_u128(top, top, 65536)
    assert g["verified"] == 0 and g["A"] > g["B"]
    g = gb.verify_range_u128(2**64 + 10, 2**64 + 4, 65536)
    assert g["verified"] == 0 and g["A"] > g["B"]
    with pytest.raises(gb.GoldbachError) as e:
        gb.verify_range_u128(2**64, 2**64 + 2**42, 65536)
    assert e.value.name == "GB_EINVAL"
    with pytest.raises(gb.GoldbachError) as e:
        gb.verify_range_u128(2**64, 2**64 + 100, 2 * 10**7)
    assert e.value.name == "GB_ERANGE"
    # and the library still gives exact results afterwards
    g = gb.verify_range_u128(2**64 + 2, 2**64 + 200, 65536)
    same(g, O.verify_range_wide(2**64 + 2, 2**64 + 200, 65536, 10**7), "after refusals")


def test_bench_size_window_split_and_samples(gb, O):
    """At the bench's size (2^22-even windows, here a 2^24-even range from 2^64
    + 2 * 10^6 on the table to 2^32 - 1): the whole range in one chunk, in
    chunks of 2^22 and as the merge of eight separate calls all agree field
    by field, and eight seeded 512-even sub-windows equal the wide oracle."""
    A = 2**64 + 2 * 10**6
    n = 1 << 24
    B = A + 2 * (n - 1)
    print("[gpu-wide] 2^24 evens from 2^64 + 2e6, table to 2^32 - 1", flush=True)
    gb.base_primes(2**32 - 1)
    try:
        whole = gb.verify_range_u128(A, B, 65536)
        assert whole["verified"] == n and whole["n_failed"] == 0
        gb.set_wide_chunk_log2(22)
        try:
            chunked = gb.verify_range_u128(A, B, 65536)
            assert gb.last_stats()["segments"] == 4
        finally:
            gb.set_wide_chunk_log2(26)
        same(chunked, whole, "chunks of 2^22")
        merged = None
        step = n // 8
        for j in range(8):
            a = A + 2 * step * j
            r = gb.verify_range_u128(a, a + 2 * (step - 1), 65536)
            merged = r if merged is None else O.merge(merged, r)
        for f in ("verified", "checksum", "max_p", "max_p_n", "n_unresolved", "n_failed"):
            assert merged[f] == whole[f], f
        rng = random.Random(2024)
        for _ in range(8):
            a = A + 2 * rng.randrange(n - 512)
            g = gb.verify_range_u128(a, a + 2 * 511, 65536)
            same(g, O.verify_range_wide(a, a + 2 * 511, 65536, 10**7), ("sample", a))
    finally:
        gb.base_primes(10**7)


def test_spill_cap_refusal_and_recovery(gb, O):
    """P_max = 3 over 2^17 evens from 2^64 leaves far more than 65536 evens to
    Phase 2: the call refuses with GB_ENOMEM and says why, and the next call is
    exact."""
    A = 2**64 + 2 * 10**5
    print("[gpu-wide] P_max 3 over 2^17 evens", flush=True)
    with pytest.raises(gb.GoldbachError) as e:
        gb.verify_range_u128(A, A + 2 * ((1 << 17) - 1), 3)
    assert e.value.name == "GB_ENOMEM" and "raise P_max" in str(e.value)
    g = gb.verify_range_u128(A, A + 2 * 999, 65536)
    same(g, O.verify_range_wide(A, A + 2 * 999, 65536, 10**7), "after the refusal")
