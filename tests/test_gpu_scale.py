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


def test_c1_full_range_and_windows(gb, O):
    """Every even n in [4, 10^10], base primes up to 10^5, P_max = 2^16: the
    first 10^9 against the oracle in full, the 64 seeded 10^7-wide windows of
    (10^9, 10^10] against the oracle, and the full range checked by counts and
    by the merge of a split, at the three segment sizes."""
    gb.base_primes(100000)
    o1 = oracle_first_1e9(O)
    wins = W.gpu_scale_windows()
    ow = oracle_many(O, [(a, b, 65536, 100000, 1 << 16) for a, b in wins])
    full = None
    for shape in SHAPES_C1:
        gb.set_params(**shape)
        log("c1 shape %s" % shape)
        same(gb.verify_range(4, 10**9, 65536), o1, what="[4,1e9] %s" % shape)
        for (a, b), o, g in zip(wins, ow, gb.verify_batch(wins, 65536)):
            same(g, o, what="window %d %s" % (a, shape))
        f = gb.verify_range(4, 10**10, 65536)
        assert f["verified"] == evens(4, 10**10)
        assert f["n_unresolved"] == 0 and f["n_failed"] == 0
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


def test_c2_headline_range(gb, O):
    """Every even n in [4, 10^12], base primes up to 10^6, P_max = 2^16, in the
    benchmark's launch configurations: the first 10^9 and the 256 seeded
    10^7-wide windows against the oracle, the full range by counts, by a
    three-way split, and across launch configurations."""
    gb.base_primes(10**6)
    wins = W.headline_windows()
    ow = oracle_many(O, [(a, b, 65536, 10**6, 1 << 16) for a, b in wins])
    o1 = oracle_first_1e9(O)
    configs = [dict(seg_log2=18, wg_size=512, window=4096, bucket_log2=32),
               dict(seg_log2=18, wg_size=512, window=4096, bucket_log2=0),
               dict(seg_log2=19, wg_size=1024, window=4096, bucket_log2=0)]
    full = None
    for cfg in configs:
        gb.set_params(**cfg)
        log("c2 params %s" % cfg)
        same(gb.verify_range(4, 10**9, 65536), o1, what="[4,1e9] %s" % cfg)
        for (a, b), o, g in zip(wins, ow, gb.verify_batch(wins, 65536)):
            same(g, o, what="window %d %s" % (a, cfg))
        t = time.time()
        f = gb.verify_range(4, 10**12, 65536)
        log("c2 full range %.3f s: %s" % (time.time() - t, {k: f[k] for k in AGG}))
        assert f["verified"] == evens(4, 10**12)
        assert f["n_unresolved"] == 0 and f["n_failed"] == 0
        assert f["max_p"] >= max(o["max_p"] for o in ow + [o1])
        if full is None:
            full = f
            rng = random.Random(7)
            c1 = 2 * rng.randrange(10**9, 2 * 10**11)
            c2 = 2 * rng.randrange(2 * 10**11, 5 * 10**11)
            parts = [gb.verify_range(4, c1, 65536), gb.verify_range(c1 + 2, c2, 65536),
                     gb.verify_range(c2 + 2, 10**12, 65536)]
            same(merge_gpu(O, parts), f, AGG, "split of [4,1e12] at %d, %d" % (c1, c2))
        else:
            same(f, full, FIELDS, "[4,1e12] %s" % cfg)


def test_c3_batch(gb, O):
    """The seeded batch of 4096 uneven intervals (16 ending next to 2^64 - 2),
    base primes up to 2^32, in one batched launch with the automatic
    strike-bitmap policy: every interval fully verified with its maximum inside
    it, and a seeded sample of the intervals short enough for the oracle
    (at most 2^21 evens, all edge intervals among them) bit-exact."""
    T = 2**32 - 1
    gb.base_primes(T)
    gb.set_params(seg_log2=18, wg_size=512, window=4096, bucket_log2=0)
    ivs = W.batch_intervals()
    t = time.time()
    got = gb.verify_batch(ivs, 65536)
    log("c3 batch %.3f s" % (time.time() - t))
    for (a, b), g in zip(ivs, got):
        assert g["A"] == a and g["B"] == b
        assert g["verified"] == evens(a, b), (a, b)
        assert g["n_unresolved"] == 0 and g["n_failed"] == 0, (a, b)
        assert a <= g["max_p_n"] <= b and 2 <= g["max_p"] <= 65536, (a, b)
    short = [i for i, (a, b) in enumerate(ivs) if evens(a, b) <= 1 << 21]
    edge = [i for i in short if i >= len(ivs) - 16]
    rest = sorted(set(short) - set(edge))
    pick = edge + random.Random(11).sample(rest, 24)
    log("c3 oracle sample: %d intervals (%d at the top of the range)" % (len(pick), len(edge)))
    O.primes(T)   # build the oracle's table once, before the threads share it
    ow = oracle_many(O, [(ivs[i][0], ivs[i][1], 65536, T, 1 << 22) for i in pick])
    for i, o in zip(pick, ow):
        same(got[i], o, what="interval %d %s" % (i, ivs[i]))
