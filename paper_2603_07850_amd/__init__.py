"""libgoldbach: device-resident segmented double-sieve Goldbach verification
on AMD Instinct MI355X (gfx950).

The compute runs in the HIP library ``libgoldbach.so`` built from ``csrc/``;
the ``_binding`` module only marshals arguments to its C ABI
(``include/goldbach.h``).  There is no CPU fallback: every call raises if the
library is missing.  Attributes are resolved lazily so that importing the
``workloads`` submodule does not touch the binding.
"""
_API = ("GoldbachError", "Params", "Server", "autotune", "autotune_batch", "autotune_cache_clear", "base_primes", "debug_fail_next", "get_params", "is_prime_u64", "lds_peak",
        "last_stats", "last_batch_latencies", "lib", "release", "set_params", "table_count", "table_limit", "table_read",
        "verify_batch", "verify_range", "verify_range_noalloc", "set_allocator",
        "verify_range_u128", "is_prime_u128", "AsyncVerify", "set_wide_chunk_log2",
        "get_wide_chunk_log2",
        "use_torch_allocator", "RESULT_FIELDS")


def __getattr__(name):
    if name in _API:
        from . import _binding
        return getattr(_binding, name)
    raise AttributeError(name)


__all__ = list(_API)
