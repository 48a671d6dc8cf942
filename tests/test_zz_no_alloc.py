"""gb_verify_range_noalloc (for callers that cannot allocate device memory)
against gb_verify_range through the C ABI: every field identical, on two
calls in a row (the second on a smaller range, so stale scratch contents of
the first would show), with spills and an unresolved list, and the host-side
rejection of a range too long for the static scratch.  The free device memory
does not change across the calls."""
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
    return g


def same(a, b, what):
    for f in FIELDS:
        assert a[f] == b[f], (what, f, a[f], b[f])


def test_noalloc_equals_verify_range(gb):
    import torch
    print("[gpu] no-alloc: gb_base_primes(2*10^6)", flush=True)
    gb.base_primes(2 * 10**6)
    saved = gb.get_params()
    try:
        gb.set_params(seg_log2=18, wg_size=512, window=4096)
        cases = [
            (10**11 + 2 * 12345, 10**11 + 2 * 3_000_000 + 2 * 7, 65536),   # several segments
            (10**9, 10**9 + 2 * 40_000, 65536),                             # smaller, one segment
            (4, 60_000, 7),                                                 # spills, unresolved list
            (4, 30, 65536),
            (11, 11, 65536),                                                # empty range
        ]
        ref = []
        for A, B, P in cases:
            print("[gpu] no-alloc: verify_range(%d, %d, %d)" % (A, B, P), flush=True)
            ref.append(gb.verify_range(A, B, P, unresolved_cap=1 << 16))
        torch.cuda.synchronize()
        # warm-up call: the first launch of a kernel may load code
        gb.verify_range_noalloc(4, 1000, 65536)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for (A, B, P), r in zip(cases, ref):
            print("[gpu] no-alloc: verify_range_noalloc(%d, %d, %d)" % (A, B, P), flush=True)
            same(gb.verify_range_noalloc(A, B, P, unresolved_cap=1 << 16), r, (A, B, P))
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        # a range longer than the scratch holds (6e11 evens: 2.29 million
        # segments of 2^18) is refused before any launch
        with pytest.raises(gb.GoldbachError) as e:
            gb.verify_range_noalloc(4, 12 * 10**11, 65536)
        assert e.value.name == "GB_ENOMEM" and "no-alloc scratch" in str(e.value)
        # and the next call is exact again
        same(gb.verify_range_noalloc(*cases[1]), ref[1], "after refusal")
    finally:
        gb.set_params(**saved)
