"""gb_set_allocator: with PyTorch's caching allocator registered, every device
buffer of the library (the prime table, the probe tables, the workspaces of the
verify calls) comes from it, and the results equal the oracle's.  Setting the
default allocator back releases the library's buffers into torch's cache."""
import pytest

pytestmark = pytest.mark.gpu

FIELDS = ("A", "B", "P_max", "verified", "max_p", "max_p_n", "checksum", "n_unresolved",
          "n_failed", "unresolved")


def test_torch_caching_allocator(tmp_path):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2603_07850_amd as gb
    from oracle import oracle as O
    gb.lib()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    count = gb.use_torch_allocator()
    try:
        print("[gpu] allocator: gb_base_primes(10^7) through torch", flush=True)
        gb.base_primes(10**7)
        n = gb.table_count()
        assert count["alloc"] >= 3                      # table + two probe tables
        assert torch.cuda.memory_allocated() - before >= 4 * n
        cases = [(10**9, 10**9 + 2 * 1_000_000, 65536), (4, 50_000, 7),
                 (10**13 + 2, 10**13 + 2 * 600_000, 65536)]
        for A, B, P in cases:
            print("[gpu] allocator: verify_range(%d, %d, %d)" % (A, B, P), flush=True)
            g = gb.verify_range(A, B, P, unresolved_cap=1 << 16)
            o = O.verify_range(A, B, P, 10**7, cap=1 << 16)
            for f in FIELDS:
                assert g[f] == o[f], (f, A, B, g[f], o[f])
        got = gb.verify_batch([c[:2] for c in cases], 65536)
        for (A, B, _), g in zip(cases, got):
            o = O.verify_range(A, B, 65536, 10**7, cap=1 << 16)
            for f in FIELDS:
                assert g[f] == o[f], (f, A, B)
        held = count["bytes"]
        assert held > 0 and torch.cuda.memory_allocated() - before >= held
    finally:
        gb.set_allocator(None, None)            # everything goes back to torch's cache
    torch.cuda.synchronize()
    assert count["bytes"] == 0 and count["free"] == count["alloc"]
    assert torch.cuda.memory_allocated() == before
    assert gb.table_count() == 0
    # the default allocator works again afterwards
    gb.base_primes(10**6)
    g = gb.verify_range(10**9, 10**9 + 2 * 10_000, 65536)
    o = O.verify_range(10**9, 10**9 + 2 * 10_000, 65536, 10**6)
    for f in FIELDS:
        assert g[f] == o[f]
