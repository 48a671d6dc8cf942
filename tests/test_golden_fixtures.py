"""The stored oracle results (tests/golden/, written by the make_*.py scripts
there, which call only oracle/) agree with the oracle as it stands on the
entries that run in seconds, and are consistent with themselves: the full
[4, 10^12] aggregates are the merge of their slices, every batch interval is
fully verified, every tie window's maximum is attained at least twice."""
import json
import os
import random

from oracle import oracle as O
from paper_2603_07850_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
AGG = ("verified", "max_p", "max_p_n", "checksum", "n_unresolved", "n_failed")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_full_1e12_is_the_merge_of_its_slices():
    d = load("full_1e12.json")
    sl = d["slices"]
    assert sl[0]["A"] == 4 and sl[-1]["B"] == 10**12
    for a, b in zip(sl, sl[1:]):
        assert b["A"] == a["B"] + 2
    m = sl[0]
    for s in sl[1:]:
        m = O.merge(m, s)
    for f in AGG:
        assert m[f] == d["result"][f], f
    assert d["result"]["verified"] == (10**12 - 4) // 2 + 1


def test_full_ranges_first_slice_live():
    d = load("full_1e12.json")
    s = d["slices"][0]
    # the first 2e8 evens of the first slice, live, are a prefix of it
    r = O.verify_range(4, 4 + 2 * (2 * 10**8 - 1), 65536, 10**6, seg_evens=1 << 20)
    assert r["max_p"] <= s["max_p"] and r["verified"] == 2 * 10**8


def test_batch_golden_against_live_oracle():
    ivs = W.batch_intervals()
    rows = []
    with open(os.path.join(GOLDEN, "batch_4096.txt")) as f:
        for line in f:
            if line.startswith("#"):
                continue
            rows.append([int(x) for x in line.split()])
    assert len(rows) == 4096
    for (a, b), row in zip(ivs, rows):
        assert (row[1], row[2]) == (a, b)
        assert row[3] == (b - a) // 2 + 1 and row[7] == 0 and row[8] == 0
        assert a <= row[6] <= b
    rng = random.Random(3)
    short = [i for i, (a, b) in enumerate(ivs) if (b - a) // 2 + 1 <= 60000 and b < 10**15]
    for i in rng.sample(short, 6):
        a, b = ivs[i]
        r = O.verify_range(a, b, 65536, 2**26, seg_evens=1 << 20)
        assert [r[f] for f in ("verified", "checksum", "max_p", "max_p_n")] == \
            [rows[i][3], rows[i][4], rows[i][5], rows[i][6]], i


def test_tie_windows_live():
    d = load("max_ties.json")
    for w in d["windows"][:4]:
        r = O.verify_range(w["A"], w["B"], d["P_max"], d["limit"])
        assert (r["checksum"], r["max_p"], r["max_p_n"]) == (w["checksum"], w["max_p"], w["max_p_n"])
        assert len(w["n_at_max"]) >= 2 and w["n_at_max"][0] == w["max_p_n"]
        # every listed n has p_min = max_p: n - p prime for p = max_p and for no
        # smaller prime (checked with the oracle's Miller-Rabin, not its sieve)
        odd = [int(p) for p in O.primes(65536)[1:]]
        for n in w["n_at_max"]:
            first = next(p for p in odd if O.is_prime(n - p))
            assert first == w["max_p"], n
