"""Write the oracle's aggregates of the full workloads to tests/golden/:

  full_1e10.json   every even n in [4, 10^10], table to 10^5, P_max = 2^16
  full_1e12.json   every even n in [4, 10^12], table to 10^6, P_max = 2^16,
                   with the aggregates of each 10^10-wide slice as well
  batch_4096.txt   each of the 4096 seeded batch intervals (workloads.batch_intervals,
                   seed 2001), table to 2^32 - 1, P_max = 2^16

Only the CPU oracle (oracle/) computes anything here; the workloads module
only draws the interval bounds.  Ranges are cut into pieces that run on a
thread pool (the oracle's C calls release the GIL) and merged with the
associative rules of the aggregates (sums mod 2^64, max with the smallest-n
tie, lists concatenated in ascending order).

Run:  python tests/golden/make_full_ranges.py [1e10] [1e12] [batch] [--threads N]
(about 25 min for 1e12 and 40 min for batch on 8 cores).
"""
import concurrent.futures as cf
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2603_07850_amd import workloads as W  # noqa: E402

AGG = ("A", "B", "P_max", "verified", "max_p", "max_p_n", "checksum", "n_unresolved",
       "n_failed")
P_MAX = 65536


def log(msg):
    print("[golden] %s" % msg, flush=True)


def evens(A, B):
    return (B - A) // 2 + 1


def pieces(A, B, n):
    """Cut [A, B] (even bounds) into n consecutive even-aligned pieces."""
    cuts = [A + 2 * ((evens(A, B) * i) // n) for i in range(n + 1)]
    return [(cuts[i], cuts[i + 1] - 2) for i in range(n) if cuts[i + 1] - 2 >= cuts[i]]


def run(jobs, threads):
    """jobs: (A, B, limit, seg_evens); results in job order."""
    done = [0]
    t0 = time.time()

    def one(j):
        r = O.verify_range(j[0], j[1], P_MAX, j[2], seg_evens=j[3])
        if r["status"] != 0:
            raise RuntimeError("oracle status %d on %s" % (r["status"], j))
        done[0] += 1
        if done[0] % max(1, len(jobs) // 20) == 0:
            log("%d / %d jobs, %.0f s" % (done[0], len(jobs), time.time() - t0))
        return r

    with cf.ThreadPoolExecutor(threads) as ex:
        return list(ex.map(one, jobs))


def merged(parts):
    out = dict(parts[0])
    for p in parts[1:]:
        out = O.merge(out, p)
    return {f: out[f] for f in AGG} | {"unresolved": out["unresolved"]}


def full_range(B, limit, slice_evens, piece_evens, threads):
    """Aggregates of [4, B], and of its slices of slice_evens evens."""
    O.primes(max(limit, 65536))
    slices = pieces(4, B, max(1, evens(4, B) // slice_evens))
    out_slices = []
    jobs, owner = [], []
    for si, (a, b) in enumerate(slices):
        for pa, pb in pieces(a, b, max(1, evens(a, b) // piece_evens)):
            jobs.append((pa, pb, limit, 1 << 20))
            owner.append(si)
    res = run(jobs, threads)
    for si in range(len(slices)):
        out_slices.append(merged([r for r, o in zip(res, owner) if o == si]))
    return merged(out_slices), out_slices


def write_json(name, obj):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(obj, f, indent=1)
        f.write("\n")
    log("wrote %s" % path)


def main():
    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    threads = 8
    if "--threads" in sys.argv:
        threads = int(sys.argv[sys.argv.index("--threads") + 1])
        args = [a for a in args if a != str(threads)]
    todo = args or ["1e10", "1e12", "batch"]
    if "1e10" in todo:
        t = time.time()
        total, _ = full_range(10**10, 10**5, 10**10, 10**8, threads)
        write_json("full_1e10.json", {
            "what": "oracle aggregates of every even n in [4, 10^10]; prime table to 10^5; "
                    "P_max = 2^16; written by make_full_ranges.py",
            "limit": 10**5, "result": total})
        log("[4, 1e10] %.0f s" % (time.time() - t))
    if "1e12" in todo:
        t = time.time()
        total, sl = full_range(10**12, 10**6, 10**10 // 2, 10**9 // 2, threads)
        write_json("full_1e12.json", {
            "what": "oracle aggregates of every even n in [4, 10^12]; prime table to 10^6; "
                    "P_max = 2^16; slices of 5e9 evens; written by make_full_ranges.py",
            "limit": 10**6, "result": total, "slices": sl})
        log("[4, 1e12] %.0f s" % (time.time() - t))
    if "batch" in todo:
        t = time.time()
        T = 2**32 - 1
        O.primes(T)
        ivs = W.batch_intervals()
        jobs, owner = [], []
        for i, (a, b) in enumerate(ivs):
            n = evens(a, b)
            # pieces of 2^24 evens amortize the per-piece cost of the large primes
            for pa, pb in pieces(a, b, max(1, -(-n // (1 << 24)))):
                jobs.append((pa, pb, T, 1 << 24))
                owner.append(i)
        # longest jobs first, so that the pool ends together
        order = sorted(range(len(jobs)), key=lambda j: -jobs[j][1])
        res_sorted = run([jobs[j] for j in order], threads)
        res = [None] * len(jobs)
        for j, r in zip(order, res_sorted):
            res[j] = r
        lines = ["# oracle result of each interval of workloads.batch_intervals() (seed 2001, "
                 "4096 intervals); prime table to 2^32 - 1; P_max = 2^16",
                 "# written by make_full_ranges.py; columns: index A B verified checksum "
                 "max_p max_p_n n_unresolved n_failed"]
        for i in range(len(ivs)):
            m = merged([r for r, o in zip(res, owner) if o == i])
            assert m["A"] == ivs[i][0] and m["B"] == ivs[i][1]
            lines.append("%d %d %d %d %d %d %d %d %d" % (
                i, m["A"], m["B"], m["verified"], m["checksum"], m["max_p"], m["max_p_n"],
                m["n_unresolved"], m["n_failed"]))
        path = os.path.join(HERE, "batch_4096.txt")
        with open(path, "w") as f:
            f.write("\n".join(lines) + "\n")
        log("wrote %s; batch %.0f s" % (path, time.time() - t))


if __name__ == "__main__":
    main()
