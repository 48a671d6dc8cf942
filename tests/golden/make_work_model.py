"""Write tests/golden/work_model.json: the algorithmic work per even n of the
verification of [4, 10^12], counted with the CPU oracle on the geometry the
segment kernel uses.

What the method must do per segment of E evens (window of E + H odd bits,
H the probe halo, stored as the two classes of odd numbers mod 3 that are
not multiples of 3):
  * strikes: every odd multiple q >= p^2 of every prime 37 <= p <= sqrt(q_hi)
    inside the window, except the multiples of 3 (the class the window does
    not store) -- split into the primes up to E/512 (one wave per prime in the
    kernel) and the larger ones (one thread per prime);
  * first multiples: each sieving prime's first multiple in the window is
    located once per segment (split like the strikes);
  * presieve words: one 32-bit word per 32 bits of each stored class;
  * word-tests: evens of one residue class mod 6 go in blocks of 64 (a lane's
    two mask words); a block must test every entry of its candidate table (the
    candidates p <= window with n - p not a multiple of 3) up to the entry of
    its largest p_min, all entries when an even is left for Phase 2.
The p_min come from the oracle; the strike counts are exact counts of
multiples in each sampled window.  Sampled segments are spread uniformly over
the range (the range is uniform in n).

With --range-1e10 it adds (or replaces) the "range_1e10" section only: the same units for
every even n in [4, 10^10] with base primes <= 10^5 and probe window 16384,
per segment size.

With --batch it adds (or replaces) the "batch" section only: for the seeded
batch of 4096 intervals, the first-multiple computations the strike-bitmap
method must make, one per table prime p with bound < p <= isqrt(top) per
interval (an interval's prime must be located once; all its later multiples
follow by adding p), per even, for bitmap bounds 2^21 .. 2^25.

Run:  python tests/golden/make_work_model.py [--range-1e10 | --batch]
"""
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402

RANGE = (4, 10**12)
LIMIT = 10**6
WINDOW = 4096          # probe window of the benchmark's launch parameters
SAMPLES = 48
BLOCK = 64


def halo(window):
    cand = O.primes(65536)
    pc = int(cand[cand <= window][-1])
    return max(96, ((pc - 1) // 2 + 2 + 95) // 96 * 96)


def odd_multiples(p, lo, hi):
    """Number of odd multiples of p (array) in [lo, hi] (arrays, lo >= 1)."""
    f = lambda x: (x + 1) // 2
    return np.maximum(f(hi // p) - f((lo + p - 1) // p - 1), 0)


def segment_counts(n0, cnt, E, H, primes, cand, limit=LIMIT):
    """Strikes (wave tier, thread tier), presieve words and word-tests of one segment."""
    weff = cnt - 1 + H
    qlo = n0 - 1 - 2 * H
    qtop = qlo + 2 * (weff - 1)                  # last window bit the probe reads
    qhi = n0 + 2 * cnt - 5                       # largest q any n of the segment needs
    root = math.isqrt(qhi)
    p = primes[(primes >= 37) & (primes <= root)].astype(np.int64)
    lo = np.maximum(np.int64(max(qlo, 1)), p * p)
    hi = np.int64(qtop)
    s = odd_multiples(p, lo, hi) - odd_multiples(3 * p, lo, hi)
    s = np.where(lo <= hi, s, 0)
    wave = int(s[p <= E // 512].sum())
    thread = int(s[p > E // 512].sum())
    fm_wave = int(np.count_nonzero(p <= E // 512))
    fm_thread = int(np.count_nonzero(p > E // 512))
    words = 2 * ((weff + 95) // 96 + 1)
    # word-tests from the oracle's p_min
    r = O.verify_range(n0, n0 + 2 * (cnt - 1), 65536, limit, want_pmin=True)
    pm = np.asarray(r["pmin"], dtype=np.int64)
    n = n0 + 2 * np.arange(cnt, dtype=np.int64)
    tests = 0
    for cls in range(3):
        sel = np.arange(cls, cnt, 3)
        if len(sel) == 0:
            continue
        nm = int(n[sel[0]] % 3)                  # n mod 3 is the same across the class
        table = cand[(cand % 3) != nm]           # the class's candidate table
        idx = np.searchsorted(table, pm[sel], side="right")
        idx = np.where(pm[sel] > table[-1], len(table), idx)
        nb = (len(sel) + BLOCK - 1) // BLOCK
        pad = np.zeros(nb * BLOCK - len(sel), dtype=np.int64)
        tests += int(np.concatenate([idx, pad]).reshape(nb, BLOCK).max(axis=1).sum())
    return wave, thread, words, tests, fm_wave, fm_thread


def model(seg_log2, rng, rng_range=RANGE, limit=LIMIT, window=WINDOW):
    E = 1 << seg_log2
    H = halo(window)
    primes = O.primes(limit)
    cand = O.primes(65536)[1:].astype(np.int64)
    cand = cand[cand <= window]
    nseg = ((rng_range[1] - rng_range[0]) // 2 + 1 + E - 1) // E
    tot = np.zeros(6, dtype=np.float64)
    ev = 0
    for s in rng.choice(np.arange(1, nseg - 1), size=SAMPLES, replace=False):
        n0 = rng_range[0] + 2 * E * int(s)
        tot += segment_counts(n0, E, E, H, primes, cand, limit)
        ev += E
    w, t, wd, ts, fw, ft = tot / ev
    return {"seg_log2": seg_log2, "halo_bits": H, "window": window, "segments_sampled": SAMPLES,
            "evens_sampled": ev, "strikes_wave_per_even": w, "strikes_thread_per_even": t,
            "first_multiples_wave_per_even": fw, "first_multiples_thread_per_even": ft,
            "presieve_words_per_even": wd, "word_tests_per_even": ts}


def batch_section():
    from paper_2603_07850_amd import workloads as W
    P = O.primes(2**32 - 1)
    ivs = W.batch_intervals()
    evens = sum((b - a) // 2 + 1 for a, b in ivs)
    # the largest q an interval's sieve reads is below its B, so isqrt(B) bounds its primes
    roots = np.array([math.isqrt(b) for _, b in ivs], dtype=np.uint64)
    pi_root = np.searchsorted(P, roots, side="right").astype(np.int64)
    out = {"intervals": len(ivs), "evens": evens, "bounds": {}}
    for lg in range(21, 26):
        pb = int(np.searchsorted(P, np.uint64(1 << lg), side="right"))
        sel = roots > (1 << lg)
        items = int((pi_root[sel] - pb).sum())
        out["bounds"][str(lg)] = {"intervals_with_bitmaps": int(sel.sum()),
                                  "first_multiples": items,
                                  "first_multiples_per_even": items / evens}
    return out


def main():
    if "--range-1e10" in sys.argv:
        path = os.path.join(HERE, "work_model.json")
        with open(path) as f:
            out = json.load(f)
        rng = np.random.default_rng(1010)
        out["range_1e10"] = {"range": [4, 10**10], "base_prime_limit": 10**5,
                     "configs": {str(lg): model(lg, rng, (4, 10**10), 10**5, 16384)
                                 for lg in (18, 19, 20)}}
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
            f.write("\n")
        print(json.dumps(out["range_1e10"], indent=1))
        return
    if "--batch" in sys.argv:
        path = os.path.join(HERE, "work_model.json")
        with open(path) as f:
            out = json.load(f)
        out["batch"] = batch_section()
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
            f.write("\n")
        print(json.dumps(out["batch"], indent=1))
        return
    rng = np.random.default_rng(4242)
    out = {"source": "oracle p_min and exact multiple counts on sampled segments of [4, 1e12]",
           "range": list(RANGE), "base_prime_limit": LIMIT, "block_evens": BLOCK,
           "configs": {str(lg): model(lg, rng) for lg in (18, 19, 20)}}
    with open(os.path.join(HERE, "work_model.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
