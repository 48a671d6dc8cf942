"""ctypes binding of the libgoldbach C ABI (argument marshalling only).

Names follow the C entry points of ``include/goldbach.h``.  PyTorch, when
present, supplies the current HIP stream and device memory for
``is_prime_u64``; it is never used for any step of the computation.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgoldbach.so")

STATUS = {0: "GB_OK", 1: "GB_EINVAL", 2: "GB_ERANGE", 3: "GB_ENOMEM", 4: "GB_EHIP",
          5: "GB_ETRUNC", 6: "GB_ENOTABLE", 7: "GB_EBUSY"}


class GoldbachError(RuntimeError):
    def __init__(self, status, msg):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__("%s: %s" % (self.name, msg))


class Result(ctypes.Structure):
    _fields_ = [
        ("A", ctypes.c_uint64), ("B", ctypes.c_uint64), ("P_max", ctypes.c_uint64),
        ("verified", ctypes.c_uint64), ("max_p", ctypes.c_uint64), ("max_p_n", ctypes.c_uint64),
        ("checksum", ctypes.c_uint64), ("n_unresolved", ctypes.c_uint64),
        ("n_failed", ctypes.c_uint64),
        ("unresolved", ctypes.POINTER(ctypes.c_uint64)), ("unresolved_cap", ctypes.c_uint64),
    ]


class Result128(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in (
        "A_lo", "A_hi", "B_lo", "B_hi", "P_max", "verified", "max_p", "max_p_n_lo",
        "max_p_n_hi", "checksum", "n_unresolved", "n_failed")] + \
        [("unresolved", ctypes.POINTER(ctypes.c_uint64)), ("unresolved_cap", ctypes.c_uint64)]


class Params(ctypes.Structure):
    _fields_ = [("seg_log2", ctypes.c_uint32), ("wg_size", ctypes.c_uint32),
                ("window", ctypes.c_uint32), ("wg_per_cu", ctypes.c_uint32),
                ("bucket_log2", ctypes.c_uint32), ("bucket_mib", ctypes.c_uint32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [("probe_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("segments", ctypes.c_uint64), ("evens", ctypes.c_uint64),
                ("spills", ctypes.c_uint64), ("grid", ctypes.c_uint32),
                ("wg_size", ctypes.c_uint32), ("seg_log2", ctypes.c_uint32),
                ("halo_bits", ctypes.c_uint32), ("ncand", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("intervals", ctypes.c_uint64)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("P_max", ctypes.c_uint64),
                ("max_active", ctypes.c_uint32), ("piece_segments", ctypes.c_uint32),
                ("max_pending", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in ("submitted", "admitted", "completed",
                                               "completed_evens", "ticks", "active",
                                               "pending", "reserved_bytes")] + \
               [("busy_ms", ctypes.c_double), ("wall_ms", ctypes.c_double)]


# gb_alloc_fn / gb_free_fn of include/goldbach.h
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                           ctypes.c_void_p)

RESULT_FIELDS = ("A", "B", "P_max", "verified", "max_p", "max_p_n", "checksum",
                 "n_unresolved", "n_failed")

_lib = None


def lib():
    """Load libgoldbach.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgoldbach.so is not built (run python -m paper_2603_07850_amd.build);"
                          " there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    u64, vp, st = ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
    sig = {
        "gb_base_primes": (st, [u64]),
        "gb_table_limit": (u64, []),
        "gb_table_count": (u64, []),
        "gb_table_read": (st, [vp, u64, u64]),
        "gb_verify_range": (st, [u64, u64, u64, vp, ctypes.POINTER(Result)]),
        "gb_verify_batch": (st, [vp, u64, u64, vp, vp]),
        "gb_verify_range_noalloc": (st, [u64, u64, u64, vp, ctypes.POINTER(Result)]),
        "gb_verify_range_async": (st, [u64, u64, u64, vp, vp, vp]),
        "gb_verify_range_u128": (st, [u64, u64, u64, u64, u64, vp, ctypes.POINTER(Result128)]),
        "gb_is_prime_u128": (st, [vp, u64, vp, vp]),
        "gb_set_allocator": (st, [ALLOC_FN, FREE_FN, vp]),
        "gb_set_params": (st, [ctypes.POINTER(Params)]),
        "gb_get_params": (st, [ctypes.POINTER(Params)]),
        "gb_set_wide_chunk_log2": (st, [ctypes.c_uint32]),
        "gb_get_wide_chunk_log2": (st, [ctypes.POINTER(ctypes.c_uint32)]),
        "gb_autotune": (st, [u64, u64, u64, vp, ctypes.POINTER(Params)]),
        "gb_autotune_batch": (st, [ctypes.POINTER(ctypes.c_uint64), u64, u64, vp, ctypes.POINTER(Params)]),
        "gb_autotune_cache_clear": (st, []),
        "gb_is_prime_u64": (st, [vp, u64, vp, vp]),
        "gb_last_stats": (st, [ctypes.POINTER(Stats)]),
        "gb_debug_fail_next": (st, [ctypes.c_uint32]),
        "gb_lds_peak": (st, [ctypes.c_uint32, ctypes.POINTER(ctypes.c_double)]),
        "gb_last_latencies": (st, [vp, u64]),
        "gb_server_open": (st, [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]),
        "gb_server_submit": (st, [vp, u64, u64, ctypes.POINTER(u64)]),
        "gb_server_poll": (st, [vp, ctypes.c_int32, ctypes.POINTER(u64), ctypes.POINTER(Result),
                                ctypes.POINTER(ctypes.c_double)]),
        "gb_server_get_stats": (st, [vp, ctypes.POINTER(ServerStats)]),
        "gb_server_close": (st, [vp]),
        "gb_release": (st, []),
        "gb_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status, ok=(0,)):
    if status not in ok:
        raise GoldbachError(status, lib().gb_last_error().decode(errors="replace"))
    return status


def _stream(stream):
    """hipStream_t handle: an int/None, or a torch stream (default: torch's current one)."""
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except ImportError:
            pass
        return None
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


def base_primes(limit):
    _check(lib().gb_base_primes(int(limit)))


def table_limit():
    return int(lib().gb_table_limit())


def table_count():
    return int(lib().gb_table_count())


def table_read(first=0, count=None):
    import numpy as np
    n = table_count()
    if count is None:
        count = n - first
    out = np.empty(max(count, 1), dtype=np.uint32)
    _check(lib().gb_table_read(out.ctypes.data, int(first), int(count)))
    return out[:count]


def _to_dict(r, unres_buf, as_array=False):
    d = {f: int(getattr(r, f)) for f in RESULT_FIELDS}
    take = min(d["n_unresolved"], int(r.unresolved_cap))
    if as_array:
        import numpy as np
        d["unresolved"] = np.ctypeslib.as_array(unres_buf)[:take].copy()
    else:
        d["unresolved"] = [int(unres_buf[i]) for i in range(take)] if take else []
    return d


def verify_range(A, B, P_max, stream=None, unresolved_cap=1 << 16, allow_trunc=True,
                 unresolved_array=False):
    """Verify every even n in [A, B]; returns a dict of the gb_result fields
    (the unresolved list as a numpy array when unresolved_array)."""
    buf = (ctypes.c_uint64 * max(int(unresolved_cap), 1))()
    r = Result()
    r.unresolved = ctypes.cast(buf, ctypes.POINTER(ctypes.c_uint64))
    r.unresolved_cap = int(unresolved_cap)
    st = lib().gb_verify_range(int(A), int(B), int(P_max), _stream(stream), ctypes.byref(r))
    _check(st, ok=(0, 5) if allow_trunc else (0,))
    d = _to_dict(r, buf, unresolved_array)
    d["status"] = STATUS[st]
    return d


def verify_range_noalloc(A, B, P_max, stream=None, unresolved_cap=1 << 16, allow_trunc=True):
    """gb_verify_range_noalloc: as verify_range, with the call's scratch in the
    library's static device array (no device allocation)."""
    buf = (ctypes.c_uint64 * max(int(unresolved_cap), 1))()
    r = Result()
    r.unresolved = ctypes.cast(buf, ctypes.POINTER(ctypes.c_uint64))
    r.unresolved_cap = int(unresolved_cap)
    st = lib().gb_verify_range_noalloc(int(A), int(B), int(P_max), _stream(stream),
                                       ctypes.byref(r))
    _check(st, ok=(0, 5) if allow_trunc else (0,))
    d = _to_dict(r, buf)
    d["status"] = STATUS[st]
    return d


M64 = (1 << 64) - 1


def verify_range_u128(A, B, P_max, stream=None, unresolved_cap=1 << 12, allow_trunc=True):
    """gb_verify_range_u128: every even n in the u128 range [A, B]; past 2^64
    primality of n - p is decided by Baillie-PSW.  Python ints in and out."""
    A, B = int(A), int(B)
    buf = (ctypes.c_uint64 * (2 * max(int(unresolved_cap), 1)))()
    r = Result128()
    r.unresolved = ctypes.cast(buf, ctypes.POINTER(ctypes.c_uint64))
    r.unresolved_cap = int(unresolved_cap)
    st = lib().gb_verify_range_u128(A & M64, A >> 64, B & M64, B >> 64, int(P_max),
                                    _stream(stream), ctypes.byref(r))
    _check(st, ok=(0, 5) if allow_trunc else (0,))
    d = {"A": r.A_lo | (r.A_hi << 64), "B": r.B_lo | (r.B_hi << 64), "P_max": int(r.P_max),
         "verified": int(r.verified), "max_p": int(r.max_p),
         "max_p_n": r.max_p_n_lo | (r.max_p_n_hi << 64), "checksum": int(r.checksum),
         "n_unresolved": int(r.n_unresolved), "n_failed": int(r.n_failed)}
    take = min(d["n_unresolved"], int(unresolved_cap))
    d["unresolved"] = [int(buf[2 * i]) | (int(buf[2 * i + 1]) << 64) for i in range(take)]
    d["status"] = STATUS[st]
    return d


def is_prime_u128(values):
    """Device primality (Miller-Rabin below 2^64, Baillie-PSW above) of a list
    of Python ints below 2^128; returns a list of bools."""
    import numpy as np
    import torch
    v = np.array([[int(x) & M64, int(x) >> 64] for x in values], dtype=np.uint64).reshape(-1)
    q = torch.tensor(v.view(np.int64), device="cuda")
    out = torch.empty(len(values), dtype=torch.uint8, device="cuda")
    _check(lib().gb_is_prime_u128(q.data_ptr(), len(values), out.data_ptr(),
                                  torch.cuda.current_stream().cuda_stream))
    return [bool(x) for x in out.cpu().tolist()]


class AsyncVerify:
    """gb_verify_range_async with its pinned buffers (PyTorch pinned host
    tensors): launch() enqueues on a stream and returns at once; result()
    reads the record after the caller has synchronized that stream."""

    def __init__(self, unresolved_cap=1 << 12):
        import torch
        self.cap = int(unresolved_cap)
        self._rec = torch.zeros(ctypes.sizeof(Result), dtype=torch.uint8, pin_memory=True)
        self._status = torch.zeros(1, dtype=torch.int32, pin_memory=True)
        self._unres = torch.zeros(max(self.cap, 1), dtype=torch.int64, pin_memory=True)
        self.rec = Result.from_address(self._rec.data_ptr())

    def launch(self, A, B, P_max, stream=None):
        self.rec.unresolved = ctypes.cast(self._unres.data_ptr(), ctypes.POINTER(ctypes.c_uint64))
        self.rec.unresolved_cap = self.cap
        self._status[0] = -1
        _check(lib().gb_verify_range_async(int(A), int(B), int(P_max), _stream(stream),
                                           ctypes.addressof(self.rec), self._status.data_ptr()))

    def status(self):
        return STATUS.get(int(self._status[0]), int(self._status[0]))

    def result(self):
        d = {f: int(getattr(self.rec, f)) for f in RESULT_FIELDS}
        take = min(d["n_unresolved"], self.cap)
        d["unresolved"] = [int(x) & M64 for x in self._unres[:take].tolist()]
        d["status"] = self.status()
        return d


def verify_batch(intervals, P_max, stream=None, unresolved_cap=1024, allow_trunc=True):
    """Verify k intervals [(A, B), ...] in one persistent launch; list of dicts."""
    import numpy as np
    k = len(intervals)
    AB = (ctypes.c_uint64 * (2 * max(k, 1)))()
    AB[0:2 * k] = [int(x) for ab in intervals for x in ab]
    outs = (Result * max(k, 1))()
    cap = max(int(unresolved_cap), 1)
    pool = np.empty(cap * max(k, 1), dtype=np.uint64)   # one buffer, a slice per interval
    # the gb_result array seen as rows of 11 u64 (the pointer is the 10th)
    view = np.frombuffer(outs, dtype=np.uint64).reshape(max(k, 1), 11)
    view[:, 9] = pool.ctypes.data + np.arange(max(k, 1), dtype=np.uint64) * (cap * 8)
    view[:, 10] = int(unresolved_cap)
    st = lib().gb_verify_batch(AB, k, int(P_max), _stream(stream), outs)
    _check(st, ok=(0, 5) if allow_trunc else (0,))
    res = [dict(zip(RESULT_FIELDS, row)) for row in view[:k, :9].tolist()]
    for i, d in enumerate(res):
        n = min(d["n_unresolved"], int(unresolved_cap))
        d["unresolved"] = pool[i * cap:i * cap + n].tolist() if n else []
    return res


def set_params(seg_log2=18, wg_size=256, window=4096, wg_per_cu=0, bucket_log2=0, bucket_mib=0):
    p = Params(int(seg_log2), int(wg_size), int(window), int(wg_per_cu), int(bucket_log2),
               int(bucket_mib))
    _check(lib().gb_set_params(ctypes.byref(p)))


def get_params():
    p = Params()
    _check(lib().gb_get_params(ctypes.byref(p)))
    return p.as_dict()


def set_wide_chunk_log2(log2):
    """gb_set_wide_chunk_log2: evens per chunk (2^log2) of ranges past 2^64."""
    _check(lib().gb_set_wide_chunk_log2(int(log2)))


def get_wide_chunk_log2():
    v = ctypes.c_uint32()
    _check(lib().gb_get_wide_chunk_log2(ctypes.byref(v)))
    return int(v.value)


def autotune(A, B, P_max, stream=None):
    p = Params()
    _check(lib().gb_autotune(int(A), int(B), int(P_max), _stream(stream), ctypes.byref(p)))
    return p.as_dict()


def autotune_batch(intervals, P_max, stream=None):
    """Choose the launch parameters by timing gb_verify_batch on a sample batch."""
    k = len(intervals)
    AB = (ctypes.c_uint64 * (2 * max(k, 1)))()
    for i, (a, b) in enumerate(intervals):
        AB[2 * i] = int(a)
        AB[2 * i + 1] = int(b)
    p = Params()
    _check(lib().gb_autotune_batch(AB, k, int(P_max), _stream(stream), ctypes.byref(p)))
    return p.as_dict()


def autotune_cache_clear():
    """Forget the library's cached autotuner choices."""
    _check(lib().gb_autotune_cache_clear())


def is_prime_u64(q):
    """Device Miller-Rabin on a torch uint64/int64 CUDA tensor; returns a uint8 tensor."""
    import torch
    q = q.contiguous()
    out = torch.empty(q.numel(), dtype=torch.uint8, device=q.device)
    _check(lib().gb_is_prime_u64(q.data_ptr(), q.numel(), out.data_ptr(),
                                 torch.cuda.current_stream(q.device).cuda_stream))
    return out


def lds_peak(width=16):
    """gb_lds_peak: the device's measured LDS read bandwidth in bytes/s for
    `width`-byte reads per lane (16 or 4)."""
    out = ctypes.c_double(0)
    _check(lib().gb_lds_peak(int(width), ctypes.byref(out)))
    return out.value


def debug_fail_next(where):
    """Test hook: the next verify call fails with GB_EHIP at point `where`
    (1 before enqueue, 2 after the kernels are enqueued; 0 clears)."""
    _check(lib().gb_debug_fail_next(int(where)))


def last_stats():
    s = Stats()
    _check(lib().gb_last_stats(ctypes.byref(s)))
    return {f: (float(getattr(s, f)) if f.endswith("_ms") else int(getattr(s, f)))
            for f, _ in Stats._fields_ if f != "pad"}


def last_batch_latencies():
    """Per-interval device latency (seconds) of the last verify call."""
    k = last_stats()["intervals"]
    buf = (ctypes.c_double * max(k, 1))()
    _check(lib().gb_last_latencies(buf, k))
    return [buf[i] / 1e3 for i in range(k)]


def release():
    _check(lib().gb_release())


_allocator = {}   # the registered ctypes callbacks, kept alive while registered


def set_allocator(alloc=None, free=None):
    """gb_set_allocator with Python callables alloc(nbytes) -> int device
    pointer (0 for failure) and free(ptr, nbytes); None, None restores
    hipMalloc / hipFree.  Releases every table and buffer of the library."""
    if alloc is None and free is None:
        _check(lib().gb_set_allocator(ALLOC_FN(), FREE_FN(), None))
        _allocator.clear()
        return

    def _a(nbytes, stream, user):
        try:
            return int(alloc(int(nbytes))) or None
        except Exception:       # reported to the library as "no memory"
            return None

    def _f(ptr, nbytes, stream, user):
        try:
            free(int(ptr), int(nbytes))
        except Exception:
            pass

    cbs = (ALLOC_FN(_a), FREE_FN(_f))
    _check(lib().gb_set_allocator(cbs[0], cbs[1], None))
    _allocator["cbs"] = cbs


def use_torch_allocator(device=None):
    """Route every device allocation of the library through PyTorch's caching
    allocator (memory only; no computation runs in torch).  Returns the
    counters {'alloc': calls, 'free': calls, 'bytes': bytes held}."""
    import torch
    dev = torch.cuda.current_device() if device is None else int(device)
    count = {"alloc": 0, "free": 0, "bytes": 0}

    def alloc(nbytes):
        ptr = torch.cuda.caching_allocator_alloc(nbytes, dev)
        count["alloc"] += 1
        count["bytes"] += nbytes
        return ptr

    def free(ptr, nbytes):
        torch.cuda.caching_allocator_delete(ptr)
        count["free"] += 1
        count["bytes"] -= nbytes

    set_allocator(alloc, free)
    return count


class Server:
    """Served form: continuous batching of submitted ranges (gb_server_*)."""

    def __init__(self, P_max, hbm_budget_bytes=64 << 30, max_active=64, piece_segments=256,
                 max_pending=0):
        cfg = ServerConfig(int(hbm_budget_bytes), int(P_max), int(max_active),
                           int(piece_segments), int(max_pending), 0)
        self._h = ctypes.c_void_p()
        _check(lib().gb_server_open(ctypes.byref(cfg), ctypes.byref(self._h)))
        self.P_max = int(P_max)

    def submit(self, A, B):
        rid = ctypes.c_uint64()
        _check(lib().gb_server_submit(self._h, int(A), int(B), ctypes.byref(rid)))
        return int(rid.value)

    def poll(self, wait_ms=-1, unresolved_cap=1024):
        """(id, result dict, latency seconds), or None if nothing finished in time."""
        buf = (ctypes.c_uint64 * max(int(unresolved_cap), 1))()
        r = Result()
        r.unresolved = ctypes.cast(buf, ctypes.POINTER(ctypes.c_uint64))
        r.unresolved_cap = int(unresolved_cap)
        rid = ctypes.c_uint64()
        lat = ctypes.c_double()
        st = lib().gb_server_poll(self._h, int(wait_ms), ctypes.byref(rid), ctypes.byref(r),
                                  ctypes.byref(lat))
        if st == 7:
            return None
        _check(st, ok=(0, 5))
        return int(rid.value), _to_dict(r, buf), lat.value / 1e3

    def stats(self):
        s = ServerStats()
        _check(lib().gb_server_get_stats(self._h, ctypes.byref(s)))
        return {f: (float(getattr(s, f)) if f.endswith("_ms") else int(getattr(s, f)))
                for f, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            _check(lib().gb_server_close(self._h))
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
