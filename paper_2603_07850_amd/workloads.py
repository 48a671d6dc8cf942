"""Seeded synthetic workloads: the ranges, windows, batches and request traces
that the benchmark and the tests hand to both the GPU library and the oracle.

This module holds no arithmetic of the verification method; it only draws
integers.  The paper's workloads are the ranges [4, N] themselves (Sec. 4),
so the shapes here are: full ranges, seeded 10^7-wide windows of them, batches
of uneven intervals spread over the whole u64 range (log-uniform starts and
lengths, some forced to end next to 2^64 - 2), and Poisson request traces.
A "10^7-wide window" starting at even s is the range [s, s + 10^7 - 2].
"""
import math

import numpy as np

U64_MAX = (1 << 64) - 1
TOP_EVEN = U64_MAX - 1          # 2^64 - 2, the largest even u64


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def _even_in(rng, lo, hi):
    """Uniform even integer in [lo, hi] (bounds may exceed 2^63)."""
    lo2 = (lo + 1) // 2
    hi2 = hi // 2
    r = (int(rng.integers(0, 1 << 62)) << 62) | int(rng.integers(0, 1 << 62))
    return 2 * (lo2 + r % (hi2 - lo2 + 1))


def _log_uniform(rng, lo, hi):
    """Integer log-uniform in [lo, hi]."""
    x = math.exp(rng.uniform(math.log(lo), math.log(hi)))
    return max(lo, min(hi, int(x)))


def windows(seed, count, lo, hi, width=10**7):
    """`count` windows [s, s + width - 2] with s even and uniform in [lo, hi - width]."""
    rng = _rng(seed)
    out = []
    for _ in range(count):
        s = _even_in(rng, lo, hi - width)
        out.append((s, s + width - 2))
    return out


def gpu_scale_windows(seed=1001):
    """64 windows of 10^7 in (10^9, 10^10]: the spot checks of [4, 10^10]."""
    return windows(seed, 64, 10**9 + 2, 10**10)


def headline_windows(seed=1002):
    """256 windows of 10^7 with uniform starts in [4, 10^12]."""
    return windows(seed, 256, 4, 10**12)


def batch_intervals(seed=2001, k=4096, n_edge=16, lmin=10**4, lmax=10**8, amin=10**9):
    """k uneven intervals [A, B]: L (number of evens) log-uniform in [lmin, lmax],
    A even and log-uniform in [amin, 2^64 - 2 - 2L]; the last `n_edge` of them
    end within 10^6 of 2^64 - 2."""
    rng = _rng(seed)
    out = []
    for i in range(k):
        L = _log_uniform(rng, lmin, lmax)
        if i >= k - n_edge:
            B = TOP_EVEN - 2 * int(rng.integers(0, 500000))
            A = B - 2 * (L - 1)
        else:
            A = _log_uniform(rng, amin, TOP_EVEN - 2 * L)
            A += A & 1
            B = A + 2 * (L - 1)
        out.append((A, B))
    return out


def request_trace(seed=3001, n=2000, rate_per_s=100.0, lmin=10**4, lmax=10**8,
                  amin=10**6, amax=18 * 10**18):
    """Served-form requests: Poisson arrivals (exponential gaps at `rate_per_s`),
    90 % with L log-uniform in [lmin, lmax], 9 % with L = 10^9 and 1 % with
    L = 10^10 evens; starts log-uniform in [amin, amax].  Returns a list of
    (arrival_s, A, B)."""
    rng = _rng(seed)
    t = 0.0
    out = []
    for _ in range(n):
        t += float(rng.exponential(1.0 / rate_per_s))
        u = float(rng.uniform())
        if u < 0.90:
            L = _log_uniform(rng, lmin, lmax)
        elif u < 0.99:
            L = 10**9
        else:
            L = 10**10
        A = _log_uniform(rng, amin, min(amax, TOP_EVEN - 2 * L))
        A += A & 1
        out.append((t, A, A + 2 * (L - 1)))
    return out
