"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke
check.  Holds none of the transform's arithmetic.

Generator: splitmix64 evaluated at counters seed, seed+1, ... (counter-based,
so any prefix is reproducible), as published by Steele, Lea and Flood
("Fast splittable pseudorandom number generators", 2014).

- residues: uniform in [0, p) by rejection on the low bitlen(p) bits;
- signed24: uniform in [-2^23, 2^23) from the top 24 bits;
- log-uniform lengths: floor(lo (hi/lo)^U), U uniform in [0, 1), clamped;
- Poisson arrivals: exponential gaps -mean ln(1 - U).
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)

# workload primes (p, g) and seeds
P998 = (998244353, 3)
GOLDILOCKS = (2**64 - 2**32 + 1, 7)
CRT_PRIMES = [(2013265921, 31), (469762049, 3), (1811939329, 13)]


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs number start..start+count-1 of the splitmix64 stream for seed."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & (2**64 - 1)) + i * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        return z ^ (z >> np.uint64(31))


def residues(p: int, n: int, seed: int) -> np.ndarray:
    """n residues uniform in [0, p) (uint64)."""
    bits = p.bit_length()
    mask = np.uint64((1 << bits) - 1) if bits < 64 else np.uint64(2**64 - 1)
    out = np.empty(n, dtype=np.uint64)
    got, pos = 0, 0
    while got < n:
        need = n - got
        chunk = splitmix64(seed, pos, need + need // 4 + 64)
        pos += len(chunk)
        v = chunk & mask
        v = v[v < np.uint64(p)]
        take = min(len(v), need)
        out[got:got + take] = v[:take]
        got += take
    return out


def residues_u32(p: int, n: int, seed: int) -> np.ndarray:
    assert p < 2**32
    return residues(p, n, seed).astype(np.uint32)


def signed24(n: int, seed: int) -> np.ndarray:
    """n integers uniform in [-2^23, 2^23) (int64)."""
    return (splitmix64(seed, 0, n) >> np.uint64(40)).astype(np.int64) - (1 << 23)


def uniform01(n: int, seed: int) -> np.ndarray:
    return (splitmix64(seed, 0, n) >> np.uint64(11)).astype(np.float64) * (1.0 / 2**53)


def log_uniform_lengths(lo: int, hi: int, n: int, seed: int) -> np.ndarray:
    u = uniform01(n, seed)
    v = np.floor(lo * (hi / lo) ** u).astype(np.int64)
    return np.clip(v, lo, hi)


def poisson_arrivals(rate_per_s: float, duration_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream on [0, duration)."""
    expect = int(rate_per_s * duration_s * 1.2 + 100)
    gaps = -np.log1p(-uniform01(expect, seed)) / rate_per_s
    t = np.cumsum(gaps)
    while t[-1] < duration_s:
        more = -np.log1p(-uniform01(expect, seed + 7919 * len(t))) / rate_per_s
        t = np.concatenate([t, t[-1] + np.cumsum(more)])
    return t[t < duration_s]
