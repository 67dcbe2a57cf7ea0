"""Seeded synthetic inputs for the kernel-actor pipelines.

This module only draws numbers; it holds none of the pipelines' arithmetic (no
sorting, scanning, compaction or encoding).  Both the GPU path and the CPU
oracle are fed the exact bytes produced here.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014).  Its i-th output is a fixed 64-bit mixing
function of ``seed + (i + 1) * 0x9E3779B97F4A7C15``, so it is counter based and
vectorises directly in numpy.  Independent streams inside one workload use
derived seeds (``derive``).

Workload shapes follow the paper's indexing use case (Sec. 4: uint32 values,
each tagged with its input position) and its overhead experiments (Sec. 5.2,
5.3, and the empty-stage probe of Sec. 3.6); the paper's index data are not
described, so every distribution below is synthetic.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1


def _mix64_scalar(z: int) -> int:
    z &= _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def derive(seed: int, stream: int) -> int:
    """Seed of an independent sub-stream ``stream`` of base seed ``seed``."""
    return _mix64_scalar(_mix64_scalar(seed) ^ ((stream + 1) * 0xD1B54A32D192ED03))


def splitmix64(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Outputs ``start .. start+n-1`` of the SplitMix64 sequence for ``seed``."""
    i = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _MASK64) + i * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def u32(seed: int, n: int) -> np.ndarray:
    """n uniform uint32 values (upper halves of the 64-bit outputs)."""
    return (splitmix64(seed, n) >> np.uint64(32)).astype(np.uint32)


def uniform_values(seed: int, n: int, bound: int) -> np.ndarray:
    """n uint32 values uniform in [0, bound).  Unbiased when bound divides 2^32."""
    return (u32(seed, n) % np.uint32(bound)).astype(np.uint32)


def unit_doubles(seed: int, n: int) -> np.ndarray:
    """n doubles in [0, 1) with 53 random bits each."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def zipf_values(seed: int, n: int, s: float = 1.1, nvals: int = 1 << 16) -> np.ndarray:
    """n values ``rank - 1`` with P(rank = r) proportional to r^-s, r in 1..nvals.

    Inverse-CDF sampling over a double-precision cumulative table."""
    w = np.arange(1, nvals + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = unit_doubles(seed, n)
    r = np.searchsorted(cdf, u, side="right")
    return np.minimum(r, nvals - 1).astype(np.uint32)


def affine_params(seed: int, stages: int = 8):
    """Per-stage (a_i, b_i) of the affine chain: a_i odd, b_i any uint32."""
    r = u32(seed, 2 * stages)
    a = (r[0::2] | np.uint32(1)).astype(np.uint32)
    b = r[1::2].astype(np.uint32)
    return a, b


def log_uniform_sizes(seed: int, count: int, lo_log2: float, hi_log2: float) -> np.ndarray:
    """count sizes floor(2^(lo + (hi - lo) u)), u uniform in [0, 1)."""
    u = unit_doubles(seed, count)
    return np.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)


def poisson_arrivals(seed: int, count: int, rate_per_s: float) -> np.ndarray:
    """Arrival times in seconds of a Poisson process (exponential gaps)."""
    u = unit_doubles(seed, count)
    gaps = -np.log1p(-u) / rate_per_s
    return np.cumsum(gaps)


# --- the benchmark configurations -------------------------------------------------

def plain_request(seed: int = 1, n: int = 1 << 16, bound: int = 1024) -> np.ndarray:
    """One index request: n values uniform in [0, bound)."""
    return uniform_values(derive(seed, 0), n, bound)


def large_request(seed: int = 3, n: int = 1 << 26, s: float = 1.1, nvals: int = 1 << 16) -> np.ndarray:
    """One large index request: n Zipf(s) values over nvals distinct values."""
    return zipf_values(derive(seed, 0), n, s, nvals)


def chain_input(seed: int = 2, m: int = 1 << 20) -> np.ndarray:
    return u32(derive(seed, 1), m)


def chain_params(seed: int = 2, stages: int = 8):
    return affine_params(derive(seed, 0), stages)


def batched_requests(seed: int = 4, count: int = 4096, lo_log2: float = 10, hi_log2: float = 20,
                     bound: int = 1 << 12, max_total: int | None = None):
    """count index requests of log-uniform sizes, values uniform in [0, bound).

    Returns (offsets int64[count+1], values uint32[total]); request j is
    values[offsets[j]:offsets[j+1]]."""
    sizes = log_uniform_sizes(derive(seed, 0), count, lo_log2, hi_log2)
    if max_total is not None:
        keep = np.cumsum(sizes) <= max_total
        sizes = sizes[keep]
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    values = uniform_values(derive(seed, 1), int(offsets[-1]), bound)
    return offsets, values


KIND_WAH, KIND_SCAN, KIND_CHAIN = 0, 1, 2


def served_requests(seed: int = 5, count: int = 20000, rate_per_s: float = 10000.0,
                    lo_log2: float = 8, hi_log2: float = 22):
    """The served mix: arrival times, sizes, kinds (40% WAH / 30% scan / 30% chain)
    and one data seed per request."""
    t = poisson_arrivals(derive(seed, 0), count, rate_per_s)
    sizes = log_uniform_sizes(derive(seed, 1), count, lo_log2, hi_log2)
    u = unit_doubles(derive(seed, 2), count)
    kinds = np.where(u < 0.4, KIND_WAH, np.where(u < 0.7, KIND_SCAN, KIND_CHAIN)).astype(np.int32)
    data_seeds = splitmix64(derive(seed, 3), count)
    return t, sizes, kinds, data_seeds


def served_payload(kind: int, size: int, data_seed: int) -> np.ndarray:
    """The input array of one served request."""
    if kind == KIND_WAH:
        return uniform_values(int(data_seed), size, 1 << 12)
    return u32(int(data_seed), size)


# --- structured inputs for edge-case tests ----------------------------------------

def structured(kind: str, n: int, seed: int = 0) -> np.ndarray:
    """Adversarial value layouts used by parity tests."""
    if kind == "uniform1024":
        return uniform_values(seed, n, 1024)
    if kind == "uniform4096":
        return uniform_values(seed, n, 4096)
    if kind == "u32":
        return u32(seed, n)
    if kind == "all_equal":
        return np.full(n, 7, dtype=np.uint32)
    if kind == "all_zero":
        return np.zeros(n, dtype=np.uint32)
    if kind == "all_max":
        return np.full(n, 0xFFFFFFFF, dtype=np.uint32)
    if kind == "distinct":
        return np.arange(n, dtype=np.uint32)
    if kind == "reverse":
        return np.arange(n, 0, -1, dtype=np.uint64).astype(np.uint32)
    if kind == "presorted":
        return np.sort(uniform_values(seed, n, 1024))
    if kind == "zipf":
        return zipf_values(seed, n, 1.1, 1 << 16)
    if kind == "alternating_chunks":
        return ((np.arange(n, dtype=np.int64) // 31) % 2).astype(np.uint32)
    if kind == "sparse_hot":
        v = u32(seed, n)
        hot = uniform_values(derive(seed, 9), n, 8) != 0
        v[hot] = 5
        return v
    if kind == "high_bits":
        return (u32(seed, n) | np.uint32(0x80000000)).astype(np.uint32)
    raise ValueError(kind)


STRUCTURED_KINDS = ("uniform1024", "uniform4096", "u32", "all_equal", "all_zero", "all_max",
                    "distinct", "reverse", "presorted", "zipf", "alternating_chunks",
                    "sparse_hot", "high_bits")
