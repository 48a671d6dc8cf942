"""Write tests/golden/work_model.json: the algorithmic work per even n of the
verification, measured with the CPU oracle only.

For the word-parallel probe a block of 32 consecutive evens must be tested
against every candidate up to the largest p_min of the block, so its word-test
count is max over the block of rank(p_min(n)), rank being the index of p_min
among the odd primes (3 -> 1, 5 -> 2, ...).  The sieve strikes each odd q once
per prime 37 <= p <= sqrt(q) dividing it, i.e. sum(1/p) strikes per odd on
average.  Both are sampled here on seeded windows of the benchmark's range
[4, 10^12] (uniform starts, as the range is uniform in n) and at a few fixed
magnitudes for reference.

Run:  python tests/golden/make_work_model.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2603_07850_amd import workloads as W  # noqa: E402

BLOCK = 32


def window_stats(A, n_evens, limit):
    r = O.verify_range(A, A + 2 * (n_evens - 1), 65536, limit, want_pmin=True)
    assert r["status"] == 0 and r["n_unresolved"] == 0, r["status"]
    pmin = np.asarray(r["pmin"], dtype=np.int64)
    odd = O.primes(65536)[1:].astype(np.int64)
    rank = np.searchsorted(odd, pmin) + 1          # 3 -> 1
    rank[pmin == 2] = 0
    nb = len(rank) // BLOCK
    blocks = rank[: nb * BLOCK].reshape(nb, BLOCK).max(axis=1)
    return float(rank.mean()), float(blocks.mean()), int(len(rank))


def strikes_per_odd(B, limit):
    p = O.primes(max(limit, 65536)).astype(np.float64)
    root = float(O.isqrt(B))
    sel = p[(p >= 37) & (p <= root)]
    return float((1.0 / sel).sum())


def main():
    out = {"block": BLOCK, "source": "oracle p_min on seeded windows", "headline": {}, "magnitudes": {}}
    # headline workload: all even n in [4, 1e12], base primes <= 1e6
    wins = W.windows(4242, 32, 4, 10**12, width=2 * (1 << 20))
    ranks, maxes, strikes, count = [], [], [], 0
    for a, b in wins:
        mr, mb, n = window_stats(a, 1 << 20, 10**6)
        ranks.append(mr)
        maxes.append(mb)
        strikes.append(strikes_per_odd(b, 10**6))
        count += n
    out["headline"] = {
        "range": [4, 10**12], "windows": len(wins), "evens_sampled": count,
        "mean_rank": float(np.mean(ranks)), "mean_block_max_rank": float(np.mean(maxes)),
        "strikes_per_odd": float(np.mean(strikes)),
    }
    for label, A, limit in (("1e7", 10**7, 10**5), ("1e9", 10**9, 10**5), ("1e10", 10**10, 2 * 10**5),
                            ("1e11", 10**11, 10**6), ("1e12", 10**12, 10**6),
                            ("1e15", 10**15, 10**8)):
        mr, mb, n = window_stats(A, 1 << 18, limit)
        out["magnitudes"][label] = {"A": A, "evens": n, "mean_rank": mr, "mean_block_max_rank": mb,
                                    "strikes_per_odd": strikes_per_odd(A + 2 * n, limit)}
    with open(os.path.join(HERE, "work_model.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
