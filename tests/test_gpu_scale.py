"""GPU parity at the full workload sizes: [4, 10^10] with base primes up to
10^5, [4, 10^12] with base primes up to 10^6, and the seeded batch of 4096
uneven intervals reaching 2^64 - 2 with base primes up to 2^32.  The GPU runs
each workload whole, in the launch configurations the benchmark times; the
oracle checks what it can finish in seconds (the first 10^9, seeded 10^7-wide
windows, the short intervals of the batch), and properties that hold at any
size check the rest: every even is verified, nothing is left unresolved, the
result of a range is the merge of the results of any split of it, and the
launch shape changes nothing."""
import concurrent.futures as cf
import random
import time

import pytest

from paper_2603_07850_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("A", "B", "P_max", "verified", "max_p", "max_p_n", "checksum", "n_unresolved",
          "n_failed", "unresolved")
AGG = ("verified", "max_p", "max_p_n", "checksum", "n_unresolved", "n_failed")
THREADS = 16


@pytest.fixture(scope="module")
def gb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2603_07850_amd as g
    g.lib()
    saved = g.get_params()
    yield g
    g.set_params(**saved)


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    return oracle


def log(msg):
    print("[gpu-scale] " + msg, flush=True)


def golden(name):
    """Oracle aggregates written by tests/golden/make_full_ranges.py."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        return json.load(f)


def evens(A, B):
    return (B - A) // 2 + 1


def oracle_many(O, jobs):
    """Run oracle.verify_range over (A, B, P_max, limit, seg_evens) jobs on a
    thread pool (the C calls release the GIL); results in job order."""
    t = time.time()
    with cf.ThreadPoolExecutor(THREADS) as ex:
        out = list(ex.map(lambda j: O.verify_range(j[0], j[1], j[2], j[3], seg_evens=j[4]), jobs))
    log("oracle: %d jobs, %d evens, %.1f s" % (len(jobs), sum(evens(j[0], j[1]) for j in jobs),
                                               time.time() - t))
    return out


def oracle_split(O, A, B, P_max, limit, pieces=THREADS):
    """The oracle over [A, B], cut into even-aligned pieces run in parallel and merged."""
    cuts = [A + 2 * ((evens(A, B) * i) // pieces) for i in range(pieces + 1)]
    jobs = [(cuts[i], cuts[i + 1] - 2, P_max, limit, 1 << 16) for i in range(pieces)
            if cuts[i + 1] - 2 >= cuts[i]]
    parts = oracle_many(O, jobs)
    out = parts[0]
    for p in parts[1:]:
        out = O.merge(out, p)
    out["A"], out["B"] = A, B
    return out


def same(g, o, fields=FIELDS, what=""):
    for f in fields:
        assert g[f] == o[f], (what, f, g[f], o[f])


def merge_gpu(O, parts):
    out = dict(parts[0])
    for p in parts[1:]:
        out = O.merge(out, p)
    return out


_first_1e9 = {}


def oracle_first_1e9(O):
    if "r" not in _first_1e9:
        _first_1e9["r"] = oracle_split(O, 4, 10**9, 65536, 100000)
    return _first_1e9["r"]


SHAPES_C1 = [dict(seg_log2=18, wg_size=256, window=4096, bucket_log2=0),
             dict(seg_log2=19, wg_size=512, window=4096, bucket_log2=0),
             dict(seg_log2=20, wg_size=1024, window=4096, bucket_log2=0)]


def test_range_1e10_full_and_windows(gb, O):
    """Every even n in [4, 10^10], base primes up to 10^5, P_max = 2^16, at the
    three segment sizes: the whole range against the oracle's aggregates of it
    (tests/golden/full_1e10.json), the first 10^9 and the 64 seeded 10^7-wide
    windows of (10^9, 10^10] against the oracle live, and the merge of a split."""
    gb.base_primes(100000)
    o1 = oracle_first_1e9(O)
    wins = W.gpu_scale_windows()
    ow = oracle_many(O, [(a, b, 65536, 100000, 1 << 16) for a, b in wins])
    full = None
    for shape in SHAPES_C1:
        gb.set_params(**shape)
        log("[4,1e10] shape %s" % shape)
        same(gb.verify_range(4, 10**9, 65536), o1, what="[4,1e9] %s" % shape)
        for (a, b), o, g in zip(wins, ow, gb.verify_batch(wins, 65536)):
            same(g, o, what="window %d %s" % (a, shape))
        f = gb.verify_range(4, 10**10, 65536)
        same(f, golden("full_1e10.json")["result"], FIELDS, "[4,1e10] against the oracle's "
             "full-range aggregates %s" % shape)
        assert f["max_p"] >= max(o["max_p"] for o in ow + [o1])
        if full is None:
            full = f
            cut = 10**9 + 2 * 123456789
            parts = [gb.verify_range(4, 10**9, 65536), gb.verify_range(10**9 + 2, cut, 65536),
                     gb.verify_range(cut + 2, 10**10, 65536)]
            same(merge_gpu(O, parts), f, AGG, "split of [4,1e10]")
            # the oracle's first 10^9 is a prefix of the full range
            same(parts[0], o1, AGG, "prefix")
        else:
            same(f, full, FIELDS, "[4,1e10] shape %s" % shape)


def test_range_1e12_headline(gb, O):
    """Every even n in [4, 10^12], base primes up to 10^6, P_max = 2^16, in the
    benchmark's launch configurations: the whole range and its 100 slices of
    5e9 evens against the oracle's aggregates (tests/golden/full_1e12.json),
    the first 10^9 and the 256 seeded 10^7-wide windows against the oracle
    live, a three-way split, and identity across launch configurations."""
    gb.base_primes(10**6)
    g12 = golden("full_1e12.json")
    wins = W.headline_windows()
    ow = oracle_many(O, [(a, b, 65536, 10**6, 1 << 16) for a, b in wins])
    o1 = oracle_first_1e9(O)
    configs = [dict(seg_log2=18, wg_size=512, window=4096, bucket_log2=32),
               dict(seg_log2=18, wg_size=512, window=4096, bucket_log2=0),
               dict(seg_log2=19, wg_size=1024, window=4096, bucket_log2=0)]
    full = None
    for cfg in configs:
        gb.set_params(**cfg)
        log("[4,1e12] params %s" % cfg)
        same(gb.verify_range(4, 10**9, 65536), o1, what="[4,1e9] %s" % cfg)
        for (a, b), o, g in zip(wins, ow, gb.verify_batch(wins, 65536)):
            same(g, o, what="window %d %s" % (a, cfg))
        t = time.time()
        f = gb.verify_range(4, 10**12, 65536)
        log("[4,1e12] full range %.3f s: %s" % (time.time() - t, {k: f[k] for k in AGG}))
        same(f, g12["result"], FIELDS, "[4,1e12] against the oracle's full-range aggregates %s"
             % cfg)
        assert f["max_p"] >= max(o["max_p"] for o in ow + [o1])
        if full is None:
            full = f
            rng = random.Random(7)
            cut1 = 2 * rng.randrange(10**9, 2 * 10**11)
            cut2 = 2 * rng.randrange(2 * 10**11, 5 * 10**11)
            parts = [gb.verify_range(4, cut1, 65536), gb.verify_range(cut1 + 2, cut2, 65536),
                     gb.verify_range(cut2 + 2, 10**12, 65536)]
            same(merge_gpu(O, parts), f, AGG, "split of [4,1e12] at %d, %d" % (cut1, cut2))
            # the oracle's 100 slices of 5e9 evens, in one batched launch
            sl = g12["slices"]
            for o, g in zip(sl, gb.verify_batch([(x["A"], x["B"]) for x in sl], 65536)):
                same(g, o, FIELDS, "slice [%d, %d]" % (o["A"], o["B"]))
        else:
            same(f, full, FIELDS, "[4,1e12] %s" % cfg)


def golden_batch():
    """Per-interval oracle results of the 4096-interval batch
    (tests/golden/batch_4096.txt, written by make_full_ranges.py)."""
    import os
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", "batch_4096.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x) for x in line.split()]
            rows.append(dict(zip(("i", "A", "B", "verified", "checksum", "max_p", "max_p_n",
                                  "n_unresolved", "n_failed"), v)))
    return rows


def test_batch_4096_intervals(gb, O):
    """The seeded batch of 4096 uneven intervals (16 ending next to 2^64 - 2),
    base primes up to 2^32, in one batched launch with the automatic
    strike-bitmap policy: every interval bit-exact against the oracle's result
    for it (tests/golden/batch_4096.txt), the 16 edge intervals among them;
    and a seeded sample of the short intervals run through the oracle live,
    which pins the fixture to the oracle as it stands."""
    T = 2**32 - 1
    gb.base_primes(T)
    gb.set_params(seg_log2=18, wg_size=512, window=4096, bucket_log2=0)
    ivs = W.batch_intervals()
    want = golden_batch()
    assert len(want) == len(ivs) == 4096
    t = time.time()
    got = gb.verify_batch(ivs, 65536)
    log("batch of 4096 intervals %.3f s" % (time.time() - t))
    for (a, b), g, o in zip(ivs, got, want):
        assert (o["A"], o["B"]) == (a, b) == (g["A"], g["B"])
        for f in AGG:
            assert g[f] == o[f], ("interval", o["i"], a, b, f, g[f], o[f])
        assert g["unresolved"] == []
    edge = list(range(len(ivs) - 16, len(ivs)))
    assert all(ivs[i][1] >= (1 << 64) - 2 - 2 * 10**6 for i in edge)
    # a second launch configuration gives the same results
    gb.set_params(seg_log2=20, wg_size=1024, window=16384, bucket_log2=23)
    got2 = gb.verify_batch(ivs, 65536)
    assert got2 == got
    short = [i for i, (a, b) in enumerate(ivs) if evens(a, b) <= 1 << 20]
    pick = random.Random(11).sample(short, 16)
    log("batch live oracle sample: %d intervals" % len(pick))
    O.primes(T)   # build the oracle's table once, before the threads share it
    ow = oracle_many(O, [(ivs[i][0], ivs[i][1], 65536, T, 1 << 22) for i in pick])
    for i, o in zip(pick, ow):
        same(got[i], o, what="interval %d %s" % (i, ivs[i]))
