"""Write tests/golden/max_ties.json: seeded windows of 10^5 evens in
[10^11, 10^12] whose largest p_min is attained by two or more n, with the
oracle's aggregates.

These windows pin the tie-break of the largest p_min (the smallest n attaining
it): an implementation that visits the evens out of order and keeps the first
n it sees, instead of the smallest, reports a wrong max_p_n on them.  Only the
CPU oracle computes anything here; the workloads module draws the starts.

Run:  python tests/golden/make_max_ties.py
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

WIDTH = 2 * 10**5       # 10^5 evens per window
WANT = 64
LIMIT = 10**6
P_MAX = 65536


def main():
    out = []
    tried = 0
    seed = 4001
    while len(out) < WANT:
        for A, B in W.windows(seed, 256, 10**11, 10**12, width=WIDTH):
            tried += 1
            r = O.verify_range(A, B, P_MAX, LIMIT, want_pmin=True)
            assert r["status"] == 0 and r["n_unresolved"] == 0
            pmin = np.asarray(r["pmin"])
            at = np.nonzero(pmin == r["max_p"])[0]
            if len(at) >= 2:
                ns = [int(A + 2 * i) for i in at]
                assert ns[0] == r["max_p_n"]
                out.append({"A": A, "B": B, "verified": r["verified"], "checksum": r["checksum"],
                            "max_p": r["max_p"], "max_p_n": r["max_p_n"], "n_at_max": ns})
                if len(out) == WANT:
                    break
        seed += 1
    with open(os.path.join(HERE, "max_ties.json"), "w") as f:
        json.dump({"what": "windows of 10^5 evens in [1e11, 1e12] whose largest p_min is "
                           "attained at least twice; prime table to 10^6; P_max = 2^16; "
                           "oracle aggregates; written by make_max_ties.py",
                   "limit": LIMIT, "P_max": P_MAX, "windows_scanned": tried,
                   "windows": out}, f, indent=1)
        f.write("\n")
    print("%d of %d windows have a tied maximum" % (len(out), tried))


if __name__ == "__main__":
    main()
