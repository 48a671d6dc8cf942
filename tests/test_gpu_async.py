"""gb_verify_range_async: the stream-ordered form of gb_verify_range.  Results
written by the stream into pinned memory equal the blocking call's and the
oracle's; calls on two streams back to back, with nothing waited for in
between, are ordered by the library and both exact; the call returns while
its work is still running; pageable memory is refused before any launch."""
import ctypes

import pytest

pytestmark = pytest.mark.gpu

FIELDS = ("A", "B", "P_max", "verified", "max_p", "max_p_n", "checksum", "n_unresolved",
          "n_failed", "unresolved")


@pytest.fixture(scope="module")
def gb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2603_07850_amd as g
    g.lib()
    print("[gpu-async] gb_base_primes(10^6)", flush=True)
    g.base_primes(10**6)
    return g


def same(a, b, what):
    for f in FIELDS:
        assert a[f] == b[f], (what, f, a[f], b[f])


def test_async_equals_blocking_and_oracle(gb):
    import torch
    from oracle import oracle as O
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    cases = [(10**11, 10**11 + 2 * 2_000_000, 65536), (4, 3_000_000, 65536), (4, 40_000, 7),
             (10**9 + 1, 10**9 + 2 * 99_999 + 1, 65536)]
    cap = 1 << 15     # holds every unresolved even of these cases
    want = [O.verify_range(a, b, p, 10**6, cap=cap) for a, b, p in cases]
    av = [gb.AsyncVerify(unresolved_cap=cap) for _ in cases]
    for i, ((a, b, p), v) in enumerate(zip(cases, av)):
        print("[gpu-async] launch %d on stream %d" % (i, 1 + i % 2), flush=True)
        v.launch(a, b, p, stream=s1 if i % 2 == 0 else s2)
    s1.synchronize()
    s2.synchronize()
    for (a, b, p), v, o in zip(cases, av, want):
        r = v.result()
        assert r["status"] == "GB_OK", r["status"]
        same(r, o, (a, b, p))
        same(gb.verify_range(a, b, p, unresolved_cap=cap), o, ("blocking", a, b, p))
    # a list longer than the buffer: status GB_ETRUNC, counts exact
    v = gb.AsyncVerify(unresolved_cap=100)
    v.launch(4, 40_000, 7, stream=s1)
    s1.synchronize()
    r = v.result()
    assert r["status"] == "GB_ETRUNC" and r["n_unresolved"] == want[2]["n_unresolved"]
    assert r["unresolved"] == want[2]["unresolved"][:100] and r["checksum"] == want[2]["checksum"]


def test_async_returns_before_the_work_ends(gb):
    import torch
    s = torch.cuda.Stream()
    v = gb.AsyncVerify()
    gb.verify_range(4, 10**9, 65536)     # workspaces at size
    torch.cuda.synchronize()
    print("[gpu-async] [4, 3e11] enqueued", flush=True)
    v.launch(4, 3 * 10**11, 65536, stream=s)
    pending = not s.query()
    s.synchronize()
    assert pending, "the stream had finished before the call returned"
    r = v.result()
    assert r["status"] == "GB_OK" and r["verified"] == (3 * 10**11 - 4) // 2 + 1
    same(r, gb.verify_range(4, 3 * 10**11, 65536), "[4, 3e11]")


def test_async_refuses_pageable_memory(gb):
    from paper_2603_07850_amd import _binding as b
    r = b.Result()
    status = ctypes.c_int32(-1)
    st = gb.lib().gb_verify_range_async(4, 1000, 65536, None, ctypes.byref(r),
                                        ctypes.byref(status))
    assert st == 1 and "pinned" in gb.lib().gb_last_error().decode()
    assert status.value == -1
