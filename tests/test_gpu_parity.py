"""GPU parity: the HIP path through the C ABI against the CPU oracle, field by
field (integer work, so bit-exact), on seeded ranges that span several
segments and a ragged tail, at every launch shape the library supports, and
on the edge cases of the method (n = 4, tiny P_max, ranges at 2^64 - 2,
empty and single-even ranges, batches mixing all of these)."""
import os
import random

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FIELDS = ("A", "B", "P_max", "verified", "max_p", "max_p_n", "checksum", "n_unresolved",
          "n_failed", "unresolved")
U64 = (1 << 64) - 1


@pytest.fixture(scope="module")
def gb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2603_07850_amd as g
    g.lib()
    return g


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    return oracle


_current = {"limit": None}


def table(gb, limit):
    if _current["limit"] != limit:
        print("[gpu] gb_base_primes(%d)" % limit, flush=True)
        gb.base_primes(limit)
        _current["limit"] = limit


_oracle_memo = {}


def oracle_range(O, A, B, P_max, limit, cap, seg_evens):
    key = (A, B, P_max, limit, cap)
    if key not in _oracle_memo:
        _oracle_memo[key] = O.verify_range(A, B, P_max, limit, cap=cap, seg_evens=seg_evens)
    return _oracle_memo[key]


def check(gb, O, A, B, P_max, limit, cap=1 << 16, seg_evens=1 << 16):
    table(gb, limit)
    print("[gpu] verify_range(%d, %d, %d) params=%s" % (A, B, P_max, gb.get_params()), flush=True)
    g = gb.verify_range(A, B, P_max, unresolved_cap=cap)
    o = oracle_range(O, A, B, P_max, limit, cap, seg_evens)
    for f in FIELDS:
        assert g[f] == o[f], (f, A, B, P_max, g[f], o[f])
    return g


# --- prime table ---------------------------------------------------------------

@pytest.mark.parametrize("limit", [3163, 100000, 1000000, 10**8])
def test_base_primes_exact(gb, O, limit):
    table(gb, limit)
    T = max(limit, 65536)
    assert gb.table_limit() == T
    ref = O.primes(T)
    assert gb.table_count() == len(ref)
    assert np.array_equal(gb.table_read(), ref)


def test_base_primes_2_32(gb, O):
    table(gb, 2**32 - 1)
    ref = O.primes(2**32 - 1)
    assert gb.table_count() == len(ref) == 203280221
    got = gb.table_read()
    assert np.array_equal(got, ref)


# --- Phase-2 primality test ------------------------------------------------------

def test_device_miller_rabin(gb, O):
    import torch
    rng = random.Random(5)
    vals = list(range(0, 5000))
    vals += [561, 2047, 3215031751, 3825123056546413051, U64, U64 - 58, 4294967291,
             2**61 - 1, 2**32 + 15, (2**32 + 15) * (2**31 - 1), 2**63 + 1, 2**63 - 25]
    vals += [rng.getrandbits(64) | 1 for _ in range(4000)]
    vals += [rng.randrange(1 << 32, 1 << 34) | 1 for _ in range(2000)]
    vals += [U64 - 2 * i for i in range(3000)]
    q = torch.tensor(np.array(vals, dtype=np.uint64).view(np.int64), device="cuda")
    got = gb.is_prime_u64(q).cpu().numpy()
    exp = np.array([O.is_prime(v) for v in vals], dtype=np.uint8)
    assert np.array_equal(got, exp)


# --- the verification ---------------------------------------------------------

def test_small_config_full(gb, O):
    """[4, 10^7] with base primes <= 3163 and P_max = 65521."""
    r = check(gb, O, 4, 10**7, 65521, 3163)
    assert r["verified"] == 4999999 and r["n_unresolved"] == 0


def test_worked_values(gb, O):
    table(gb, 3163)
    r = gb.verify_range(4, 30, 65521)
    assert (r["verified"], r["checksum"], r["max_p"], r["max_p_n"]) == (14, 53, 7, 30)
    assert gb.verify_range(4, 4, 100)["checksum"] == 2
    assert gb.verify_range(6, 6, 100)["checksum"] == 3
    assert gb.verify_range(8, 8, 100)["checksum"] == 3


LAUNCH_SHAPES = [(lg, wg, win) for lg in (18, 19, 20) for wg in (256, 512, 1024)
                 for win in (0, 4096, 64)]


@pytest.mark.parametrize("shape", LAUNCH_SHAPES, ids=lambda s: "w%d_t%d_win%d" % s)
def test_launch_shapes_identical(gb, O, shape):
    lg, wg, win = shape
    saved = gb.get_params()
    try:
        gb.set_params(seg_log2=lg, wg_size=wg, window=win)
        # several segments at every shape plus a ragged tail
        check(gb, O, 4, 3_000_000 + 2 * 777, 65536, 10**6)
        check(gb, O, 10**11 + 2 * 12345, 10**11 + 2_400_000 + 2 * 31, 65536, 10**6)
    finally:
        gb.set_params(**saved)


@pytest.mark.parametrize("P_max", [2, 3, 7, 31, 100, 1000, 4096, 65521])
def test_tiny_and_mid_pmax(gb, O, P_max):
    check(gb, O, 4, 40000, P_max, 100000, cap=40000)


def test_unresolved_truncation_keeps_counts(gb, O):
    table(gb, 100000)
    r = gb.verify_range(4, 20000, 3, unresolved_cap=10)
    o = O.verify_range(4, 20000, 3, 100000, cap=20000)
    assert r["status"] == "GB_ETRUNC"
    assert r["n_unresolved"] == o["n_unresolved"] and r["unresolved"] == o["unresolved"][:10]
    assert r["checksum"] == o["checksum"] and r["verified"] == o["verified"]


@pytest.mark.parametrize("AB", [(0, 3), (0, 4), (1, 9), (5, 9), (100, 50), (4, 6), (10, 10),
                                (11, 11), (6, 5000), (7, 5001), (2**20 - 2, 2**20 + 2)])
def test_normalization_edges(gb, O, AB):
    check(gb, O, AB[0], AB[1], 65536, 3163)


def test_segment_boundaries(gb, O):
    """Ranges ending exactly at, one before and one after segment edges."""
    table(gb, 10**6)
    for lg in (18, 19):
        gb.set_params(seg_log2=lg, wg_size=256, window=4096)
        E = (1 << lg) - 2048
        for d in (-2, 0, 2):
            B = 4 + 2 * (E - 1) + d
            check(gb, O, 4, B, 65536, 10**6)
            check(gb, O, 10**10, 10**10 + 2 * (2 * E - 1) + d, 65536, 10**6)
    gb.set_params(seg_log2=18, wg_size=256, window=4096, wg_per_cu=0)


def test_near_2_64(gb, O):
    """Top of the u64 range: the overflow guards (Sec. 3.4)."""
    T = 2**32 - 1
    check(gb, O, U64 - 2 * 30000, U64, 65536, T, seg_evens=1 << 22)
    check(gb, O, U64 - 1, U64, 65536, T, seg_evens=1 << 22)
    check(gb, O, U64, U64, 65536, T)
    check(gb, O, U64 - 2 * 5000 - 1, U64 - 3, 7, T, cap=20000, seg_evens=1 << 22)


def test_table_too_small_is_erange(gb):
    table(gb, 3163)
    with pytest.raises(gb.GoldbachError) as e:
        gb.verify_range(4, 10**12, 65536)
    assert e.value.name == "GB_ERANGE"
    with pytest.raises(gb.GoldbachError) as e:
        gb.verify_range(4, 100, 70000)
    assert e.value.name == "GB_ERANGE"
    with pytest.raises(gb.GoldbachError) as e:
        gb.verify_range(4, 100, 1)
    assert e.value.name == "GB_EINVAL"


def test_batch_equals_single_calls_and_oracle(gb, O):
    table(gb, 2**32 - 1)
    ivs = [(4, 100000), (100, 50), (10**9, 10**9 + 300000), (U64 - 40000, U64),
           (10**12 + 2, 10**12 + 2), (5, 5), (10**15 + 1, 10**15 + 1 + 2 * 123457),
           (2**40, 2**40 + 2 * 70000), (4, 100000)]
    got = gb.verify_batch(ivs, 65536)
    for (A, B), g in zip(ivs, got):
        s = gb.verify_range(A, B, 65536)
        o = O.verify_range(A, B, 65536, 2**32 - 1, seg_evens=1 << 22)
        for f in FIELDS:
            assert g[f] == s[f] == o[f], (f, A, B)


def test_batch_with_tiny_pmax(gb, O):
    table(gb, 100000)
    ivs = [(4, 3000), (2000, 9000), (50000, 51000)]
    got = gb.verify_batch(ivs, 5, unresolved_cap=5000)
    for (A, B), g in zip(ivs, got):
        o = O.verify_range(A, B, 5, 100000, cap=5000)
        for f in FIELDS:
            assert g[f] == o[f], (f, A, B)


def test_repeat_runs_identical(gb):
    table(gb, 10**6)
    a = gb.verify_range(10**11, 10**11 + 4 * 10**6, 65536)
    for _ in range(3):
        assert gb.verify_range(10**11, 10**11 + 4 * 10**6, 65536) == a


def test_batch_graph_replays_identical(gb, O):
    """The batched form replays a captured graph: every replay, with eager work
    and synchronizations in between, must equal the first result and the oracle."""
    import torch
    table(gb, 10**6)
    ivs = [(10**9 + 2 * i * 100003, 10**9 + 2 * i * 100003 + 2 * 50000) for i in range(40)]
    first = gb.verify_batch(ivs, 65536)
    for (A, B), g in list(zip(ivs, first))[:6]:
        o = O.verify_range(A, B, 65536, 10**6)
        for f in FIELDS:
            assert g[f] == o[f], (f, A, B)
    for _ in range(4):
        gb.verify_range(4, 10**6, 65536)          # eager launches between replays
        torch.cuda.synchronize()
        assert gb.verify_batch(ivs, 65536) == first
    lat = gb.last_batch_latencies()
    assert len(lat) == len(ivs) and all(x > 0 for x in lat)
    # a different shape re-captures; the old one still replays correctly afterwards
    other = gb.verify_batch(ivs[:7], 65536)
    assert other == first[:7]
    assert gb.verify_batch(ivs, 65536) == first


BUCKET_CASES = [
    # (A, B, P_max, limit)
    (10**11 + 2 * 4567, 10**11 + 3_000_000, 65536, 10**6),
    (10**13 - 4 * 10**6, 10**13, 65536, 10**7),
    (10**15 + 2, 10**15 + 1_500_000, 65536, 2**32 - 1),
    ((1 << 64) - 2 * 200000, (1 << 64) - 1, 65536, 2**32 - 1),
    ((1 << 64) - 2 * 6000, (1 << 64) - 3, 7, 2**32 - 1),
]


@pytest.mark.parametrize("blog", [17, 19, 0])
@pytest.mark.parametrize("mib", [0, 1])
def test_strike_bitmaps_parity(gb, O, blog, mib):
    """Primes above the bucket bound cleared through strike bitmaps: identical to the
    oracle, with one or many rounds (a 1 MiB budget splits ranges into many
    chunks and rounds)."""
    saved = gb.get_params()
    try:
        gb.set_params(seg_log2=18, wg_size=256, window=4096, bucket_log2=blog, bucket_mib=mib)
        for A, B, P_max, limit in BUCKET_CASES:
            check(gb, O, A, B, P_max, limit, cap=20000, seg_evens=1 << 22)
    finally:
        gb.set_params(**saved)


def test_strike_bitmap_batch_equals_single(gb, O):
    table(gb, 2**32 - 1)
    saved = gb.get_params()
    try:
        gb.set_params(seg_log2=19, wg_size=512, window=4096, bucket_log2=18, bucket_mib=64)
        ivs = [(10**9, 10**9 + 200000), (U64 - 300000, U64), (10**18, 10**18 + 900000),
               (4, 50000), (2**50 + 2, 2**50 + 2 + 2 * 333333), (10**12, 10**12)]
        got = gb.verify_batch(ivs, 65536)
        for (A, B), g in zip(ivs, got):
            s = gb.verify_range(A, B, 65536)
            o = O.verify_range(A, B, 65536, 2**32 - 1, seg_evens=1 << 22)
            for f in FIELDS:
                assert g[f] == s[f] == o[f], (f, A, B)
    finally:
        gb.set_params(**saved)


def test_batch_autotuner_keeps_results(gb, O):
    """The batch autotuner only changes launch parameters: the batch verified
    under the parameters it picks equals the oracle."""
    table(gb, 2**32 - 1)
    saved = gb.get_params()
    try:
        ivs = [(10**9, 10**9 + 200000), (U64 - 300000, U64), (10**15, 10**15 + 2 * 77777),
               (4, 60000), (2**50 + 2, 2**50 + 2 + 2 * 150000)]
        p = gb.autotune_batch(ivs, 65536)
        assert p["seg_log2"] in (18, 19, 20) and p["wg_size"] in (256, 512, 1024)
        assert gb.get_params() == p
        got = gb.verify_batch(ivs, 65536)
        for (A, B), g in zip(ivs, got):
            o = O.verify_range(A, B, 65536, 2**32 - 1, seg_evens=1 << 22)
            for f in FIELDS:
                assert g[f] == o[f], (f, A, B)
        with pytest.raises(gb.GoldbachError) as e:
            gb.autotune_batch([], 65536)
        assert e.value.name == "GB_EINVAL"
    finally:
        gb.set_params(**saved)


@pytest.mark.parametrize("shape", [(18, 512), (19, 1024), (20, 256)])
@pytest.mark.parametrize("P_max", [600, 1000, 4096])
def test_two_pass_probe_and_queue_overflow(gb, O, shape, P_max):
    """Blocks handed to the probe's second pass, and (with small P_max, where many
    blocks stay open after the first pass) blocks that find the queue full and
    finish in the first pass, with spills to Phase 2: identical to the oracle."""
    saved = gb.get_params()
    try:
        gb.set_params(seg_log2=shape[0], wg_size=shape[1], window=4096)
        check(gb, O, 10**12, 10**12 + 2 * 3_000_000, P_max, 1_100_000, cap=1 << 20)
    finally:
        gb.set_params(**saved)


def test_range_autotuner_keeps_results(gb, O):
    """The range autotuner only changes launch parameters."""
    table(gb, 10**6)
    saved = gb.get_params()
    try:
        import time
        gb.autotune_cache_clear()
        p = gb.autotune(10**11, 10**11 + 2 * 4_000_000, 65536)
        assert p["seg_log2"] in (18, 19, 20) and p["wg_size"] in (256, 512, 1024)
        assert gb.get_params() == p
        check(gb, O, 10**11, 10**11 + 2 * 4_000_000, 65536, 10**6)
        # the choice is cached per device and size class: no timing again
        gb.set_params(**saved)
        t0 = time.perf_counter()
        assert gb.autotune(10**11 + 2 * 10, 10**11 + 2 * 4_000_010, 65536) == p
        assert time.perf_counter() - t0 < 0.05 and gb.get_params() == p
    finally:
        gb.set_params(**saved)


def same(g, o):
    for f in FIELDS:
        assert g[f] == o[f], (f, g[f], o[f])


@pytest.mark.gpu
def test_injected_failures_leave_the_library_usable(gb, O):
    """A call that fails before or after its kernels are enqueued (forced on
    the host through the test hook) reports GB_EHIP, and the next calls give
    the oracle's results (paper Sec. 3.4: errors are reported, not fatal)."""
    table(gb, 10 ** 6)
    gb.set_params(seg_log2=19, wg_size=1024, window=4096)
    A, B, P_max = 10 ** 9, 10 ** 9 + 4 * 10 ** 6, 65536
    want = O.verify_range(A, B, P_max, 10 ** 6)
    ivs = [(10 ** 9, 10 ** 9 + 10 ** 6), (4, 10 ** 6), (10 ** 10, 10 ** 10 + 2 * 10 ** 6)]
    want_b = [O.verify_range(a, b, P_max, 10 ** 6) for a, b in ivs]
    for where in (1, 2, 1, 2):
        print("[gpu] injected failure at point %d" % where, flush=True)
        gb.debug_fail_next(where)
        with pytest.raises(gb.GoldbachError) as e:
            gb.verify_range(A, B, P_max)
        assert e.value.name == "GB_EHIP" and "injected" in str(e.value)
        same(gb.verify_range(A, B, P_max), want)
        gb.debug_fail_next(where)
        with pytest.raises(gb.GoldbachError) as e:
            gb.verify_batch(ivs, P_max)
        assert e.value.name == "GB_EHIP"
        for g, o in zip(gb.verify_batch(ivs, P_max), want_b):
            same(g, o)
    gb.debug_fail_next(2)
    gb.debug_fail_next(0)
    same(gb.verify_range(A, B, P_max), want)


def _max_ties():
    import json
    with open(os.path.join(os.path.dirname(__file__), "golden", "max_ties.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("shape", LAUNCH_SHAPES, ids=lambda s: "w%d_t%d_win%d" % s)
def test_max_ties_smallest_n(gb, shape):
    """Windows whose largest p_min is attained by two or more n (oracle fixture):
    max_p_n is the smallest of them at every launch shape, alone and in a batch.
    A lane visits several blocks, not in ascending n, so a tie kept in visiting
    order instead of by n shows up here."""
    d = _max_ties()
    table(gb, d["limit"])
    lg, wg, win = shape
    saved = gb.get_params()
    try:
        gb.set_params(seg_log2=lg, wg_size=wg, window=win)
        wins = d["windows"]
        got_b = gb.verify_batch([(w["A"], w["B"]) for w in wins], d["P_max"])
        for w, gbat in zip(wins, got_b):
            g = gb.verify_range(w["A"], w["B"], d["P_max"])
            for f in ("verified", "checksum", "max_p", "max_p_n"):
                assert g[f] == gbat[f] == w[f], (f, w["A"], g[f], gbat[f], w[f])
    finally:
        gb.set_params(**saved)


def test_tiny_pmax_long_range(gb, O):
    """P_max = 3 over 10^7 evens: about 8.5 million evens go to Phase 2, and the
    ordered list is built by the bitmap-and-scan emission (the spill list
    overflows once and the call reruns once with room for every spill).
    Every field, the whole list included, equals the oracle's."""
    import concurrent.futures as cf
    import numpy as np
    table(gb, 10**6)
    A, B = 4, 2 * 10**7
    print("[gpu] verify_range(%d, %d, 3), long unresolved list" % (A, B), flush=True)
    g = gb.verify_range(A, B, 3, unresolved_cap=10**7, unresolved_array=True)
    # the oracle in 16 pieces on a thread pool, merged in order
    cuts = [A + 2 * (((B - A) // 2 + 1) * i // 16) for i in range(17)]
    with cf.ThreadPoolExecutor(16) as ex:
        parts = list(ex.map(lambda i: O.verify_range(cuts[i], cuts[i + 1] - 2, 3, 10**6,
                                                     cap=10**7, seg_evens=1 << 20,
                                                     unresolved_array=True), range(16)))
    assert g["verified"] == sum(p["verified"] for p in parts)
    assert g["n_unresolved"] == sum(p["n_unresolved"] for p in parts) > 8 * 10**6
    assert g["n_failed"] == sum(p["n_failed"] for p in parts)
    assert g["checksum"] == sum(p["checksum"] for p in parts) % (1 << 64)
    best = max(parts, key=lambda p: (p["max_p"], -p["max_p_n"]))
    assert (g["max_p"], g["max_p_n"]) == (best["max_p"], best["max_p_n"])
    assert np.array_equal(g["unresolved"], np.concatenate([p["unresolved"] for p in parts]))
    # the same emission in a batch beside other intervals, and a short list afterwards
    ivs = [(10**9, 10**9 + 2 * 19_999), (4, 100), (10**10, 10**10 + 2 * 50_000)]
    got = gb.verify_batch(ivs, 3, unresolved_cap=1 << 17)
    for (a, b), r in zip(ivs, got):
        ob = O.verify_range(a, b, 3, 10**6, cap=1 << 17)
        for f in FIELDS:
            assert r[f] == ob[f], (f, a, b)
    check(gb, O, 4, 40000, 7, 10**6, cap=40000)


def test_grown_spill_list_then_long_range(gb):
    """A spill list grown by a tiny-P_max call stays with the library; a later
    range too long for the ordered listing of that many entries (one bit per
    even: 7.5e10 evens would take 8.7 GiB) starts again from 2^16 entries and
    completes exactly (results equal to the same call after gb_release and a
    fresh table, which start from scratch)."""
    table(gb, 10**6)
    print("[gpu] tiny P_max to grow the spill list", flush=True)
    gb.verify_range(4, 2 * 10**6, 3)
    A, B = 4, 150 * 10**9
    print("[gpu] verify_range(%d, %d, 65536) after it" % (A, B), flush=True)
    g = gb.verify_range(A, B, 65536)
    assert g["verified"] == (B - A) // 2 + 1 and g["n_unresolved"] == 0 and g["n_failed"] == 0
    gb.release()
    _current["limit"] = None
    table(gb, 10**6)
    fresh = gb.verify_range(A, B, 65536)
    for f in FIELDS:
        assert g[f] == fresh[f], f
