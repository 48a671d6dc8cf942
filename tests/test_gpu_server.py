"""GPU tests of the served form: every request's result in a continuous-batching
mix is bit-identical to verifying it alone, and equal to the oracle where the
oracle can run it; admission respects slots and the HBM budget."""
import random
import time

import pytest

pytestmark = pytest.mark.gpu

FIELDS = ("A", "B", "P_max", "verified", "max_p", "max_p_n", "checksum", "n_unresolved",
          "n_failed", "unresolved")
U64 = (1 << 64) - 1


@pytest.fixture(scope="module")
def gb():
    import torch
    assert torch.cuda.is_available()
    import paper_2603_07850_amd as g
    g.base_primes(2**32 - 1)
    g.set_params(seg_log2=18, wg_size=512, window=4096)
    return g


def _mix(seed, n):
    rng = random.Random(seed)
    out = []
    for i in range(n):
        L = int(10 ** rng.uniform(3, 6.5))
        if i % 7 == 0:
            A = U64 - 2 * rng.randrange(0, 10**6) - 2 * L
        else:
            A = int(10 ** rng.uniform(6, 19.2))
        A = min(A, U64 - 2 * L - 1)
        A += A & 1
        out.append((A, A + 2 * (L - 1)))
    out += [(4, 10**6), (100, 50), (5, 5), (U64 - 1, U64)]
    return out


def test_served_equals_alone(gb):
    reqs = _mix(1, 60)
    alone = [gb.verify_range(a, b, 65536) for a, b in reqs]
    with gb.Server(65536, max_active=16, piece_segments=3) as srv:
        ids = {}
        for i, (a, b) in enumerate(reqs):
            ids[srv.submit(a, b)] = i
            if i % 5 == 0:
                time.sleep(0.002)          # arrivals while earlier requests are on the GPU
        got = {}
        while len(got) < len(reqs):
            r = srv.poll(wait_ms=20000)
            assert r is not None, "server stalled"
            rid, res, lat = r
            assert lat >= 0
            got[ids[rid]] = res
        st = srv.stats()
    for i in range(len(reqs)):
        for f in FIELDS:
            assert got[i][f] == alone[i][f], (f, reqs[i])
    assert st["completed"] == len(reqs) and st["ticks"] >= 2


def test_served_large_requests_equal_alone(gb):
    """The trace's large requests (L = 10^9 and 10^10 evens, starts near
    1.8e19, where every piece takes one remainder per large prime) served in a
    mix with small ones and with the server's default piece size: each result
    bit-identical to the request verified alone, and seeded 10^7-wide windows
    of the large requests against the oracle."""
    from oracle import oracle as O
    big = [(18 * 10**18 + 2 * 123456789, 18 * 10**18 + 2 * 123456789 + 2 * (10**9 - 1)),
           (17 * 10**18, 17 * 10**18 + 2 * (10**9 - 1)),
           (U64 - 1 - 2 * (10**10 - 1) - 2 * 777, U64 - 1 - 2 * 777)]
    reqs = big + _mix(5, 20)
    print("[gpu] served: %d requests, %d of them with 1e9+ evens" % (len(reqs), len(big)), flush=True)
    alone = [gb.verify_range(a, b, 65536) for a, b in reqs]
    with gb.Server(65536, max_active=16, piece_segments=256) as srv:
        ids = {}
        for i, (a, b) in enumerate(reqs):
            ids[srv.submit(a, b)] = i
        got = {}
        while len(got) < len(reqs):
            r = srv.poll(wait_ms=60000)
            assert r is not None, "server stalled"
            got[ids[r[0]]] = r[1]
    for i in range(len(reqs)):
        for f in FIELDS:
            assert got[i][f] == alone[i][f], (f, reqs[i])
    for a, b in big:
        assert alone[big.index((a, b))]["verified"] == (b - a) // 2 + 1
    import concurrent.futures as cf
    rng = random.Random(9)
    wins = []
    for a, b in big:
        s = a + 2 * rng.randrange(0, (b - a) // 2 - 10**7)
        wins.append((s, s + 2 * (5 * 10**6 - 1)))
    O.primes(2**32 - 1)
    with cf.ThreadPoolExecutor(len(wins)) as ex:
        ow = list(ex.map(lambda w: O.verify_range(w[0], w[1], 65536, 2**32 - 1,
                                                  seg_evens=1 << 23), wins))
    for w, o in zip(wins, ow):
        g = gb.verify_range(*w, 65536)
        for f in FIELDS:
            assert g[f] == o[f], (f, w)


def test_served_small_against_oracle(gb):
    from oracle import oracle as O
    reqs = [(4, 200000), (10**9, 10**9 + 123456), (U64 - 50000, U64), (10**15, 10**15 + 77776)]
    with gb.Server(65536, max_active=2, piece_segments=1) as srv:
        ids = {srv.submit(a, b): i for i, (a, b) in enumerate(reqs)}
        got = {}
        while len(got) < len(reqs):
            rid, res, _ = srv.poll(wait_ms=60000)
            got[ids[rid]] = res
    for i, (a, b) in enumerate(reqs):
        o = O.verify_range(a, b, 65536, 2**32 - 1, seg_evens=1 << 22)
        for f in FIELDS:
            assert got[i][f] == o[f], (f, a, b)


def test_served_tiny_pmax_unresolved_lists(gb):
    from oracle import oracle as O
    with gb.Server(5, max_active=4, piece_segments=1) as srv:
        reqs = [(4, 30000), (10**6, 10**6 + 20000)]
        ids = {srv.submit(a, b): i for i, (a, b) in enumerate(reqs)}
        got = {}
        while len(got) < len(reqs):
            rid, res, _ = srv.poll(wait_ms=60000, unresolved_cap=40000)
            got[ids[rid]] = res
    for i, (a, b) in enumerate(reqs):
        o = O.verify_range(a, b, 5, 2**32 - 1, cap=40000, seg_evens=1 << 22)
        for f in FIELDS:
            assert got[i][f] == o[f], (f, a, b)


def test_admission_budget_and_errors(gb):
    with gb.Server(65536, hbm_budget_bytes=8 << 20, max_active=8, piece_segments=512) as srv:
        with pytest.raises(gb.GoldbachError) as e:
            srv.submit(U64 - 2 * 10**9, U64)       # one piece's bitmaps need more than 8 MiB
        assert e.value.name == "GB_ENOMEM"
        a = srv.submit(10**12, 10**12 + 10**6)
        b = srv.submit(10**13, 10**13 + 10**6)
        seen = set()
        while len(seen) < 2:
            rid, res, _ = srv.poll(wait_ms=60000)
            seen.add(rid)
            assert res["verified"] == 500001
        assert seen == {a, b}
        assert srv.poll(wait_ms=0) is None
    with gb.Server(65536, max_active=1, piece_segments=1, max_pending=1) as srv:
        srv.submit(10**15, 10**15 + 4 * 10**6)
        busy = 0
        for _ in range(50):
            try:
                srv.submit(10**15, 10**15 + 10)
            except gb.GoldbachError as e:
                assert e.name == "GB_EBUSY"
                busy += 1
        assert busy > 0
