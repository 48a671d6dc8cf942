"""Host logic of the command-line verifier (no GPU).

The chunk plan must tile the normalized range, the merge of chunk results
must reproduce the aggregates of the whole range (checked against the oracle
run on the whole range and on each chunk), and a run stopped after some chunks
and resumed from its log must give the same result as one uninterrupted run.
The chunk verifier here is the oracle, handed to ``cli.run`` by the test; the
command itself only ever calls the HIP library.
"""
import json
import random

import pytest

from oracle import oracle as O
from paper_2603_07850_amd import cli

U64 = (1 << 64) - 1
U128 = (1 << 128) - 1
CMP = ("verified", "checksum", "max_p", "max_p_n", "n_unresolved", "n_failed", "unresolved")


def oracle_verify(limit):
    def verify(a, b, P_max):
        return O.verify_range(a, b, P_max, limit)
    return verify


def same(r, o):
    for f in CMP:
        assert r[f] == o[f], (f, r[f], o[f])


def test_plan_tiles_the_range():
    rng = random.Random(7)
    cases = [(4, 100, 7), (0, 3, 5), (5, 5, 1), (3, 1001, 1), (10, 8, 3), (4, 4, 100),
             (U64 - 100, U64, 7), (U64 - 1, U64, 1), (U64 - 100, U64 + 100, 13),
             (U128 - 100, U128, 7), (U128 - 1, U128, 1), (U128, U128, 1)]
    for _ in range(200):
        a = rng.randrange(0, 10 ** 6)
        cases.append((a, a + rng.randrange(0, 10 ** 4), rng.randrange(1, 3000)))
    for A, B, c in cases:
        chunks = cli.plan_chunks(A, B, c)
        nb = cli.normalize(A, B)
        if nb is None:
            assert chunks == []
            continue
        assert chunks[0][0] == nb[0] and chunks[-1][1] == nb[1]
        for (a, b), nxt in zip(chunks, chunks[1:] + [None]):
            assert a % 2 == 0 and b % 2 == 0 and a <= b
            assert (b - a) // 2 + 1 <= c
            if nxt:
                assert nxt[0] == b + 2
                assert (b - a) // 2 + 1 == c     # every chunk but the last is full


def test_normalize_edges():
    assert cli.normalize(0, 3) is None
    assert cli.normalize(4, 4) == (4, 4)
    assert cli.normalize(5, 7) == (6, 6)
    assert cli.normalize(U64, U64) is None
    assert cli.normalize(U64 - 3, U64) == (U64 - 3, U64 - 1)
    assert cli.normalize(U64, U64 + 1) == (U64 + 1, U64 + 1)
    assert cli.normalize(U128, U128) is None
    assert cli.normalize(U128 - 3, U128) == (U128 - 3, U128 - 1)


@pytest.mark.parametrize("A,B,P_max,chunk", [(4, 200000, 65536, 9000), (4, 60000, 7, 777),
                                              (1001, 90001, 64, 2500)])
def test_merged_chunks_equal_the_whole_range(A, B, P_max, chunk):
    limit = 1 << 17
    whole = O.verify_range(A, B, P_max, limit)
    res, ran, complete = cli.run(A, B, P_max, chunk, oracle_verify(limit))
    assert complete and ran == len(cli.plan_chunks(A, B, chunk))
    same(res, whole)


def test_merged_chunks_past_2_64():
    """Chunks on both sides of 2^64 and one across it, against the wide oracle
    over the whole range."""
    A, B, P_max, chunk = 2**64 - 2 * 300, 2**64 + 2 * 300, 65536, 137

    def verify(a, b, p):
        return O.verify_range_wide(a, b, p, 10**6)
    whole = verify(A, B, P_max)
    res, ran, complete = cli.run(A, B, P_max, chunk, verify)
    chunks = cli.plan_chunks(A, B, chunk)
    assert complete and ran == len(chunks)
    assert any(a < 2**64 <= b for a, b in chunks)
    same(res, whole)


def test_merge_keeps_smallest_n_on_ties():
    acc = cli.empty_result()
    r1 = dict(cli.empty_result(), verified=3, checksum=5, max_p=7, max_p_n=100)
    r2 = dict(cli.empty_result(), verified=2, checksum=U64, max_p=7, max_p_n=50)
    r3 = dict(cli.empty_result(), verified=1, checksum=2, max_p=5, max_p_n=10)
    m = cli.merge(cli.merge(cli.merge(acc, r1, 10), r2, 10), r3, 10)
    assert (m["verified"], m["checksum"], m["max_p"], m["max_p_n"]) == (6, 6, 7, 50)


def test_log_and_resume(tmp_path):
    limit = 1 << 17
    A, B, P_max, chunk = 4, 300000, 65536, 11111
    log = str(tmp_path / "run.jsonl")
    whole = O.verify_range(A, B, P_max, limit)
    r1, ran1, done1 = cli.run(A, B, P_max, chunk, oracle_verify(limit), log=log, max_chunks=4)
    assert (ran1, done1) == (4, False)
    recs, good = cli.read_log(log)
    assert len(recs) == 4 and recs[0]["A"] == 4 and recs[3]["B"] + 2 == cli.plan_chunks(A, B, chunk)[4][0]
    # a line torn by a stopped job ends the log, and the resumed run replaces it
    with open(log, "a") as f:
        f.write('{"A": 12')
    recs_t, good_t = cli.read_log(log)
    assert len(recs_t) == 4 and good_t == good
    r2, ran2, done2 = cli.run(A, B, P_max, chunk, oracle_verify(limit), log=log, resume=True)
    assert done2 and ran1 + ran2 == len(cli.plan_chunks(A, B, chunk))
    same(r2, whole)
    # resuming a finished log runs nothing and gives the same result
    r3, ran3, done3 = cli.run(A, B, P_max, chunk, oracle_verify(limit), log=log, resume=True)
    assert (ran3, done3) == (0, True)
    same(r3, whole)
    # every record holds the aggregates of its chunk
    recs, good = cli.read_log(log)
    with open(log, "rb") as f:
        assert len(f.read()) == good            # the torn line is gone
    for rec in recs:
        o = O.verify_range(rec["A"], rec["B"], P_max, limit)
        same(rec, o)


def test_resume_rejects_another_runs_log(tmp_path):
    limit = 1 << 17
    log = str(tmp_path / "run.jsonl")
    cli.run(4, 100000, 65536, 5000, oracle_verify(limit), log=log, max_chunks=2)
    with pytest.raises(ValueError):
        cli.run(4, 100000, 4096, 5000, oracle_verify(limit), log=log, resume=True)
    with pytest.raises(ValueError):
        cli.run(1000, 100000, 65536, 5000, oracle_verify(limit), log=log, resume=True)


def test_progress_line():
    p = cli.Progress(1000, 60.0)
    p.add(250)
    line = p.line()
    assert "250 / 1000" in line and "25.0 %" in line


def test_arguments():
    a = cli.parse_args(["1000000", "--start", "100", "--p-max", "4096"])
    assert (a.limit, a.start, a.p_max, a.gpus) == (1000000, 100, 4096, 1)
    with pytest.raises(SystemExit):
        cli.parse_args(["1000", "--gpus", "2"])
    with pytest.raises(SystemExit):
        cli.parse_args(["1000", "--resume"])
    a = cli.parse_args([str(1 << 64)])                 # past 2^64: Baillie-PSW
    assert a.limit == 1 << 64
    with pytest.raises(SystemExit):
        cli.parse_args([str(1 << 128)])
    with pytest.raises(SystemExit):
        cli.parse_args([str(1 << 70), "--chunk-evens", str((1 << 40) + 1)])
    # the output record is plain JSON
    assert json.loads(json.dumps(cli.empty_result())) == cli.empty_result()
