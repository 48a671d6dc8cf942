"""ctypes wrapper around the plain C oracle (``gb_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.  Every function here is
argument marshalling; the arithmetic lives in ``gb_oracle.c`` and follows the
paper's definition of the verification (Sec. 1, Sec. 3.3, Sec. 3.4).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
_tables = {}


class OracleResult(ctypes.Structure):
    _fields_ = [
        ("A", ctypes.c_uint64), ("B", ctypes.c_uint64), ("P_max", ctypes.c_uint64),
        ("verified", ctypes.c_uint64), ("max_p", ctypes.c_uint64),
        ("max_p_n", ctypes.c_uint64), ("checksum", ctypes.c_uint64),
        ("n_unresolved", ctypes.c_uint64), ("n_failed", ctypes.c_uint64),
    ]


class OracleResultWide(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in (
        "A_lo", "A_hi", "B_lo", "B_hi", "P_max", "verified", "max_p", "max_p_n_lo",
        "max_p_n_hi", "checksum", "n_unresolved", "n_failed")]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.OUT):
            _build.build()
        L = ctypes.CDLL(_build.OUT)
        u64, p = ctypes.c_uint64, ctypes.c_void_p
        L.gbo_isqrt.argtypes = [u64]
        L.gbo_isqrt.restype = u64
        L.gbo_primes.argtypes = [u64, p, u64]
        L.gbo_primes.restype = ctypes.c_int64
        L.gbo_is_prime.argtypes = [u64]
        L.gbo_is_prime.restype = ctypes.c_int
        L.gbo_verify_range.argtypes = [u64, u64, u64, p, u64, u64, u64,
                                       ctypes.POINTER(OracleResult), p, u64, p]
        L.gbo_verify_range.restype = ctypes.c_int
        L.gbo_is_prime_window.argtypes = [u64, u64, p]
        L.gbo_is_prime_window.restype = None
        L.gbo_sieve_window.argtypes = [u64, u64, p, u64, u64, p]
        L.gbo_sieve_window.restype = ctypes.c_int
        L.gbo_bpsw.argtypes = [u64, u64]
        L.gbo_bpsw.restype = ctypes.c_int
        L.gbo_isqrt128.argtypes = [u64, u64]
        L.gbo_isqrt128.restype = u64
        L.gbo_verify_range_wide.argtypes = [u64, u64, u64, u64, u64, p, u64, u64,
                                            ctypes.POINTER(OracleResultWide), p, u64, p]
        L.gbo_verify_range_wide.restype = ctypes.c_int
        _lib = L
    return _lib


def isqrt(x):
    return int(lib().gbo_isqrt(int(x)))


def is_prime(q):
    return bool(lib().gbo_is_prime(int(q)))


def _pi_upper(limit):
    """An upper bound on pi(limit) for sizing (Rosser-Schoenfeld style)."""
    import math
    if limit < 100:
        return 30
    return int(1.26 * limit / math.log(limit)) + 64


def primes(limit):
    """All primes <= limit as a uint32 array (cached per limit)."""
    limit = int(limit)
    if limit in _tables:
        return _tables[limit]
    cap = _pi_upper(limit)
    out = np.empty(cap, dtype=np.uint32)
    n = lib().gbo_primes(limit, out.ctypes.data, cap)
    if n < 0:
        raise RuntimeError("gbo_primes failed: %d" % n)
    arr = out[:n].copy()
    _tables[limit] = arr
    return arr


def table_limit(limit):
    """The table the library builds for gb_base_primes(limit): primes <= max(limit, 65536)."""
    return max(int(limit), 65536)


def verify_range(A, B, P_max, limit, seg_evens=1 << 16, cap=1 << 16, want_pmin=False,
                 unresolved_array=False):
    """Aggregates (and optionally per-n p_min) for every even n in [A, B].

    ``limit`` is the base-prime limit handed to gb_base_primes; the oracle
    uses the same table, primes <= max(limit, 65536).
    """
    T = table_limit(limit)
    tab = primes(T)
    res = OracleResult()
    unres = np.zeros(max(cap, 1), dtype=np.uint64)
    pmin = None
    pmin_ptr = None
    An = A + (A & 1)
    Bn = B & ~1
    if want_pmin:
        if An < 4:
            An = 4
        n = (Bn - An) // 2 + 1 if Bn >= An else 0
        pmin = np.zeros(max(n, 1), dtype=np.uint32)
        pmin_ptr = pmin.ctypes.data
    st = lib().gbo_verify_range(int(A), int(B), int(P_max), tab.ctypes.data, len(tab), T,
                                int(seg_evens), ctypes.byref(res), unres.ctypes.data, cap,
                                pmin_ptr)
    out = {f: int(getattr(res, f)) for f, _ in OracleResult._fields_}
    out["status"] = int(st)
    k = min(out["n_unresolved"], cap)
    out["unresolved"] = unres[:k].copy() if unresolved_array else [int(x) for x in unres[:k]]
    if want_pmin:
        out["pmin"] = pmin[: (out["B"] - out["A"]) // 2 + 1] if out["B"] >= out["A"] else pmin[:0]
    return out


def is_prime_window(q0, count):
    out = np.zeros(count, dtype=np.uint8)
    lib().gbo_is_prime_window(int(q0), int(count), out.ctypes.data)
    return out


def sieve_window(q0, count, T):
    tab = primes(T)
    out = np.zeros(count, dtype=np.uint8)
    st = lib().gbo_sieve_window(int(q0), int(count), tab.ctypes.data, len(tab), int(T), out.ctypes.data)
    if st != 0:
        raise ValueError("gbo_sieve_window status %d" % st)
    return out


FIELDS = ("A", "B", "P_max", "verified", "max_p", "max_p_n", "checksum", "n_unresolved", "n_failed")


def merge(a, b):
    """Combine aggregates of two disjoint ranges (a below b)."""
    out = dict(a)
    out["B"] = b["B"]
    out["verified"] = a["verified"] + b["verified"]
    out["checksum"] = (a["checksum"] + b["checksum"]) % (1 << 64)
    out["n_unresolved"] = a["n_unresolved"] + b["n_unresolved"]
    out["n_failed"] = a["n_failed"] + b["n_failed"]
    out["unresolved"] = list(a.get("unresolved", [])) + list(b.get("unresolved", []))
    if (b["max_p"], -b["max_p_n"]) > (a["max_p"], -a["max_p_n"]):
        out["max_p"], out["max_p_n"] = b["max_p"], b["max_p_n"]
    return out


M64 = (1 << 64) - 1


def bpsw(q):
    """Baillie-PSW probable-primality of 0 <= q < 2^128 - 1 (gb_oracle_wide.c)."""
    q = int(q)
    return bool(lib().gbo_bpsw(q & M64, q >> 64))


def isqrt128(x):
    x = int(x)
    return int(lib().gbo_isqrt128(x & M64, x >> 64))


def verify_range_wide(A, B, P_max, limit, cap=1 << 12, want_pmin=False):
    """Aggregates of every even n in the u128 range [A, B] with primality of
    n - p decided by BPSW (gb_oracle_wide.c); unresolved n as Python ints."""
    T = table_limit(limit)
    tab = primes(T)
    res = OracleResultWide()
    unres = np.zeros(2 * max(cap, 1), dtype=np.uint64)
    A, B = int(A), int(B)
    pmin = None
    if want_pmin:
        a = max(4, A + (A & 1))
        n = (B - (B & 1) - a) // 2 + 1 if B - (B & 1) >= a else 0
        if n > 1 << 24:
            raise ValueError("want_pmin is for short ranges")
        pmin = np.zeros(max(n, 1), dtype=np.uint32)
    st = lib().gbo_verify_range_wide(A & M64, A >> 64, B & M64, B >> 64, int(P_max),
                                     tab.ctypes.data, len(tab), T, ctypes.byref(res),
                                     unres.ctypes.data, cap,
                                     pmin.ctypes.data if pmin is not None else None)
    out = {
        "A": res.A_lo | (res.A_hi << 64), "B": res.B_lo | (res.B_hi << 64),
        "P_max": int(res.P_max), "verified": int(res.verified), "max_p": int(res.max_p),
        "max_p_n": res.max_p_n_lo | (res.max_p_n_hi << 64), "checksum": int(res.checksum),
        "n_unresolved": int(res.n_unresolved), "n_failed": int(res.n_failed),
        "status": int(st),
    }
    k = min(out["n_unresolved"], cap)
    out["unresolved"] = [int(unres[2 * i]) | (int(unres[2 * i + 1]) << 64) for i in range(k)]
    if want_pmin:
        out["pmin"] = pmin[:(out["B"] - out["A"]) // 2 + 1] if out["B"] >= out["A"] else pmin[:0]
    return out
