"""The command-line verifier on the GPU: chunked, stopped-and-resumed and
range-partitioned runs give the aggregates of one library call over the whole
range, which the oracle checks in full.  Each run is a child process (the CLI
builds its own prime table)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CMP = ("verified", "checksum", "max_p", "max_p_n", "n_unresolved", "n_failed")


def cli(*args, timeout=600):
    cmd = [sys.executable, "-m", "paper_2603_07850_amd"] + [str(a) for a in args]
    print("[gpu] %s" % " ".join(cmd[2:]), flush=True)
    p = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=timeout)
    lines = [l for l in p.stdout.splitlines() if l.startswith("{")]
    assert lines, (p.returncode, p.stdout[-2000:], p.stderr[-2000:])
    return p.returncode, json.loads(lines[-1]), p.stderr


@pytest.fixture(scope="module", autouse=True)
def warm_torch():
    # the first import of torch on a fresh machine pages in its libraries
    # (a minute or more); do it here once, not inside a child's time limit
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"


@pytest.fixture(scope="module")
def whole():
    from oracle import oracle as O
    return O.verify_range(4, 10 ** 9, 65536, 65536)


@pytest.mark.gpu
def test_cli_chunked_run_matches_oracle(whole):
    rc, out, err = cli(10 ** 9, "--chunk-evens", 10 ** 8, "--seg-log2", 19, "--progress",
                       "--progress-interval", 0.05)
    assert rc == 0 and out["complete"] and out["chunks_run"] == 5
    for f in CMP:
        assert out[f] == whole[f], f
    assert "[goldbach]" in err and "ETA" in err


@pytest.mark.gpu
def test_cli_stop_and_resume(whole, tmp_path):
    log = str(tmp_path / "run.jsonl")
    rc1, out1, _ = cli(10 ** 9, "--chunk-evens", 7 * 10 ** 7, "--seg-log2", 18, "--wg-size", 512,
                       "--log", log, "--max-chunks", 3)
    assert rc1 == 3 and not out1["complete"] and out1["chunks_run"] == 3
    rc2, out2, _ = cli(10 ** 9, "--chunk-evens", 7 * 10 ** 7, "--seg-log2", 18, "--wg-size", 512,
                       "--log", log, "--resume")
    assert rc2 == 0 and out2["complete"] and out2["chunks_run"] == 8 - 3
    for f in CMP:
        assert out2[f] == whole[f], f


@pytest.mark.gpu
def test_cli_start_partitions_the_range(whole):
    from paper_2603_07850_amd.cli import empty_result, merge
    cut = 612345677                      # odd: the first job ends at cut - 1
    rc1, lo, _ = cli(cut, "--seg-log2", 20)
    rc2, hi, _ = cli(10 ** 9, "--start", cut, "--seg-log2", 20)
    assert rc1 == 0 and rc2 == 0 and lo["B"] + 2 == hi["A"]
    m = merge(merge(empty_result(), dict(lo, unresolved=[]), 16), dict(hi, unresolved=[]), 16)
    for f in CMP:
        assert m[f] == whole[f], f


@pytest.mark.gpu
def test_cli_reports_errors():
    # a prime table below isqrt(LIMIT) is refused before any work (exit status 2)
    cmd = [sys.executable, "-m", "paper_2603_07850_amd", str(10 ** 12), "--base-limit", "1000",
           "--seg-log2", "18", "--wg-size", "256"]
    print("[gpu] %s" % " ".join(cmd[2:]), flush=True)
    p = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert p.returncode == 2 and "GB_ERANGE" in p.stderr, (p.returncode, p.stderr[-2000:])


@pytest.mark.gpu
def test_cli_past_2_64_matches_wide_oracle():
    """A range across 2^64 in chunks of 1000 evens (one chunk across 2^64, the
    rest on either side): the 64-bit path below, Baillie-PSW above, merged;
    against the wide oracle over the whole range (every even resolves with
    p <= 2^16, so the oracle's smaller table gives the same result)."""
    from oracle import oracle as O
    A, B = 2**64 - 2 * 2500, 2**64 + 2 * 3500
    rc, out, _ = cli(B, "--start", A, "--chunk-evens", 1000, "--seg-log2", 18, "--wg-size", 256)
    assert rc == 0 and out["complete"] and out["chunks_run"] == 7
    o = O.verify_range_wide(A, B, 65536, 10 ** 7)
    for f in CMP:
        assert out[f] == o[f], f
    assert (out["A"], out["B"]) == (A, B)
