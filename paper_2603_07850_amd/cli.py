"""Command-line verifier: ``python -m paper_2603_07850_amd [OPTIONS] LIMIT``.

The deployment surface of the paper (Sec. "Deployment and CLI Interface"):
verify every even n in [START, LIMIT] on one GPU, with ``--start`` for
disjoint range partitioning across independent jobs and ``--progress`` for a
monitor thread that prints throughput and the estimated time to completion
without blocking the GPU work.  Resources are validated before any work
(Sec. 3.4): the library checks table limits and P_max before it enqueues
anything.

The range is verified in chunks of ``--chunk-evens`` evens, one
``gb_verify_range`` call each (``gb_verify_range_u128`` for a chunk that
reaches 2^64: past 2^64 primality of n - p is decided by Baillie-PSW, the
paper's future-work direction of Sec. 5; LIMIT may be up to 2^128 - 1), and
the chunk results are merged exactly: the
aggregates of a range are associative over any split into consecutive
sub-ranges (counts and the checksum add modulo 2^64, the largest minimal p
keeps the smallest n on ties, unresolved lists concatenate in ascending
order).  With ``--log FILE`` every finished chunk is appended to FILE as one
JSON line, and ``--resume`` continues a run from its log, so a job that is
stopped loses at most one chunk.

There is no CPU path: without the built HIP library the command fails.
"""
import argparse
import json
import math
import os
import sys
import threading
import time

U64 = (1 << 64) - 1
U128 = (1 << 128) - 1
WIDE_MAX_EVENS = 1 << 40      # evens past 2^64 per library call
FIELDS = ("verified", "checksum", "max_p", "max_p_n", "n_unresolved", "n_failed")


def normalize(A, B):
    """Even bounds [A', B'] of the evens n >= 4 in [A, B]; None if there is none."""
    A = max(4, A + (A & 1))
    B = min(B, U128 - 1)
    B -= B & 1
    return (A, B) if A <= B else None


def plan_chunks(A, B, chunk_evens):
    """Consecutive even sub-ranges of [A, B] (normalized) of chunk_evens evens each."""
    nb = normalize(A, B)
    if nb is None:
        return []
    A, B = nb
    step = 2 * max(int(chunk_evens), 1)
    out = []
    a = A
    while a <= B:
        b = min(B, a + step - 2)
        out.append((a, b))
        if b == B:
            break
        a = b + 2
    return out


def empty_result():
    r = {f: 0 for f in FIELDS}
    r["unresolved"] = []
    return r


def merge(acc, r, unresolved_cap):
    """Fold the result r of the next sub-range into acc (both dicts of FIELDS)."""
    out = dict(acc)
    out["verified"] = acc["verified"] + r["verified"]
    out["checksum"] = (acc["checksum"] + r["checksum"]) & U64
    out["n_unresolved"] = acc["n_unresolved"] + r["n_unresolved"]
    out["n_failed"] = acc["n_failed"] + r["n_failed"]
    if r["max_p"] > acc["max_p"] or (r["max_p"] == acc["max_p"] and r["max_p"] != 0
                                      and r["max_p_n"] < acc["max_p_n"]):
        out["max_p"], out["max_p_n"] = r["max_p"], r["max_p_n"]
    out["unresolved"] = (list(acc.get("unresolved", [])) +
                         list(r.get("unresolved", [])))[:unresolved_cap]
    return out


def read_log(path):
    """The chunk records of a log file, in order, and the length in bytes of
    the part that holds them: a line torn by a stopped job ends the log."""
    recs, good = [], 0
    if not os.path.exists(path):
        return recs, good
    with open(path, "rb") as f:
        data = f.read()
    pos = 0
    while pos < len(data):
        end = data.find(b"\n", pos)
        if end < 0:
            break                      # no newline: the write was cut short
        line = data[pos:end].strip()
        if line:
            try:
                recs.append(json.loads(line))
            except ValueError:
                break
        pos = end + 1
        good = pos
    return recs, good


def resume_point(recs, A, B, P_max):
    """Merged result of the logged chunks and the first even still to verify.

    The records must be consecutive sub-ranges starting at A, verified with the
    same P_max; anything else is an error (a log of another run).
    """
    nb = normalize(A, B)
    acc = empty_result()
    if nb is None:
        return acc, None
    nxt = nb[0]
    for r in recs:
        if r.get("P_max") != P_max or r.get("A") != nxt or r.get("B", 0) > nb[1]:
            raise ValueError("log record %r does not continue the range at %d with P_max %d"
                             % ({k: r.get(k) for k in ("A", "B", "P_max")}, nxt, P_max))
        acc = merge(acc, r, 1 << 62)
        nxt = r["B"] + 2
    return acc, (nxt if nxt <= nb[1] else None)


class Progress(threading.Thread):
    """Prints throughput and the estimated time to completion every interval."""

    def __init__(self, total_evens, interval, stream=sys.stderr):
        super().__init__(daemon=True)
        self.total = total_evens
        self.interval = interval
        self.stream = stream
        self.done = 0
        self.t0 = time.perf_counter()
        self.stop = threading.Event()
        self.lock = threading.Lock()

    def add(self, evens):
        with self.lock:
            self.done += evens

    def line(self):
        with self.lock:
            done = self.done
        dt = time.perf_counter() - self.t0
        rate = done / dt if dt > 0 else 0.0
        eta = (self.total - done) / rate if rate > 0 else float("inf")
        return "[goldbach] %d / %d evens (%.1f %%), %.3e evens/s, ETA %s" % (
            done, self.total, 100.0 * done / max(self.total, 1), rate,
            "%.1f s" % eta if math.isfinite(eta) else "-")

    def run(self):
        while not self.stop.wait(self.interval):
            print(self.line(), file=self.stream, flush=True)


def run(A, B, P_max, chunk_evens, verify, log=None, resume=False, unresolved_cap=1 << 16,
        progress=None, max_chunks=None):
    """Verify [A, B] chunk by chunk with verify(a, b, P_max) -> result dict.

    Returns (merged result, number of chunks verified by this call, complete).
    """
    acc, start = empty_result(), None
    nb = normalize(A, B)
    if nb is not None:
        start = nb[0]
    if resume and log:
        recs, good = read_log(log)
        acc, start = resume_point(recs, A, B, P_max)
        if os.path.exists(log) and os.path.getsize(log) > good:
            with open(log, "r+b") as f:   # drop a torn last line before appending
                f.truncate(good)
    chunks = plan_chunks(start, nb[1], chunk_evens) if (nb is not None and start is not None) else []
    if progress:
        progress.total = sum((b - a) // 2 + 1 for a, b in chunks)   # what this call verifies
    ran = 0
    fh = open(log, "a") if log else None
    try:
        for a, b in chunks:
            if max_chunks is not None and ran >= max_chunks:
                return acc, ran, False
            r = verify(a, b, P_max)
            rec = {"A": a, "B": b, "P_max": P_max}
            rec.update({f: int(r[f]) for f in FIELDS})
            rec["unresolved"] = [int(x) for x in r.get("unresolved", [])][:unresolved_cap]
            if fh:
                fh.write(json.dumps(rec) + "\n")
                fh.flush()
                os.fsync(fh.fileno())
            acc = merge(acc, rec, unresolved_cap)
            ran += 1
            if progress:
                progress.add((b - a) // 2 + 1)
    finally:
        if fh:
            fh.close()
    return acc, ran, True


def parse_args(argv):
    ap = argparse.ArgumentParser(
        prog="python -m paper_2603_07850_amd",
        description="Verify the Goldbach property for every even n in [START, LIMIT] on one "
                    "MI355X: each even's minimal prime p with n - p prime.")
    ap.add_argument("limit", type=int, metavar="LIMIT", help="last integer of the range")
    ap.add_argument("--start", type=int, default=4, help="first integer of the range (default 4)")
    ap.add_argument("--p-max", type=int, default=65536,
                    help="candidate bound of the sieve-and-probe phase (default 65536); evens "
                         "left open go to the Miller-Rabin fallback")
    ap.add_argument("--base-limit", type=int, default=0,
                    help="prime table bound (default: max(isqrt(LIMIT), P_max))")
    ap.add_argument("--seg-log2", type=int, default=0,
                    help="evens per segment as a power of two (18..20); 0 = autotune")
    ap.add_argument("--wg-size", type=int, default=1024, help="threads per workgroup")
    ap.add_argument("--window", type=int, default=4096, help="probe window (candidates in LDS)")
    ap.add_argument("--chunk-evens", type=int, default=10 ** 11,
                    help="evens per library call (progress and resume granularity)")
    ap.add_argument("--progress", action="store_true",
                    help="print throughput and the estimated time to completion")
    ap.add_argument("--progress-interval", type=float, default=5.0, help="seconds between lines")
    ap.add_argument("--log", default=None, help="append one JSON line per finished chunk")
    ap.add_argument("--resume", action="store_true", help="continue the run recorded in --log")
    ap.add_argument("--unresolved-cap", type=int, default=1 << 16,
                    help="unresolved evens kept in the output")
    ap.add_argument("--gpus", type=int, default=1, help="GPUs to use (the verifier drives one)")
    ap.add_argument("--max-chunks", type=int, default=None, help=argparse.SUPPRESS)
    a = ap.parse_args(argv)
    if a.gpus != 1:
        ap.error("--gpus=%d: the verifier runs on one GPU; partition the range across jobs "
                 "with --start instead" % a.gpus)
    if a.resume and not a.log:
        ap.error("--resume needs --log")
    if a.start < 0 or a.limit < 0 or a.limit > U128 or a.start > U128:
        ap.error("START and LIMIT must be in [0, 2^128 - 1]")
    if a.limit > U64 and a.chunk_evens > WIDE_MAX_EVENS:
        ap.error("--chunk-evens above 2^40 is not supported past 2^64")
    return a


def main(argv=None):
    """Exit status: 0 verified, 1 some even left unresolved by every test (a
    counterexample candidate), 2 an error (library, resources or log), 3 a run
    stopped before the end of the range."""
    a = parse_args(sys.argv[1:] if argv is None else argv)
    from . import _binding as gb   # loads the HIP library; raises if it is not built
    try:
        return _main(a, gb)
    except (gb.GoldbachError, ValueError, OSError) as e:
        print("goldbach: %s" % e, file=sys.stderr, flush=True)
        return 2


def _main(a, gb):
    nb = normalize(a.start, a.limit)
    # past 2^64 the table of primes to 2^32 - 1 serves both parts: the 64-bit
    # part below 2^64 needs it, and the sieve past 2^64 uses its primes to 2^28
    wide = nb is not None and nb[1] > U64
    base = a.base_limit or (U64 >> 32 if wide else
                            max(math.isqrt(nb[1]) if nb else 0, a.p_max))
    gb.base_primes(base)
    if a.seg_log2:
        gb.set_params(seg_log2=a.seg_log2, wg_size=a.wg_size, window=a.window)
    elif nb is not None and nb[0] <= U64:
        # tune on a slice of the 64-bit part's top end (its costliest part)
        top = min(nb[1], U64 - 1)
        span = min(top - nb[0], 2 * 10 ** 10)
        gb.autotune(top - span, top, a.p_max)

    total = (nb[1] - nb[0]) // 2 + 1 if nb else 0
    mon = None
    if a.progress:
        mon = Progress(total, a.progress_interval)
        mon.start()

    def verify(lo, hi, P_max):
        if hi > U64:
            return gb.verify_range_u128(lo, hi, P_max, unresolved_cap=a.unresolved_cap)
        return gb.verify_range(lo, hi, P_max, unresolved_cap=a.unresolved_cap)

    t0 = time.perf_counter()
    try:
        res, ran, complete = run(a.start, a.limit, a.p_max, a.chunk_evens, verify, log=a.log,
                                 resume=a.resume, unresolved_cap=a.unresolved_cap,
                                 progress=mon, max_chunks=a.max_chunks)
    finally:
        if mon:
            mon.stop.set()
    dt = time.perf_counter() - t0
    if mon:
        print(mon.line(), file=sys.stderr, flush=True)
    out = {"A": nb[0] if nb else None, "B": nb[1] if nb else None, "P_max": a.p_max,
           "complete": complete, "chunks_run": ran, "seconds": dt, "params": gb.get_params()}
    out.update({f: res[f] for f in FIELDS})
    out["unresolved"] = res["unresolved"]
    print(json.dumps(out))
    if res["n_failed"]:
        return 1
    return 0 if complete else 3
