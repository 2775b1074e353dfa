"""Seeded synthetic inputs shaped like the paper's benchmark inputs.

This module only produces inputs.  It holds none of the sorting method's
arithmetic, and both the product path and the oracle receive the arrays it
builds.  Random draws use the SplitMix64 generator (Steele, Lea and Flood,
OOPSLA 2014), implemented here from its published definition with numpy's
wrapping uint64 arithmetic.

Distributions follow the paper's experimental-setup section (ten input
distributions, six data types); where the paper's one-line definitions leave
freedom, the choices are stated on each function.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
MASTER_SEED = 0x0002009135690000
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

DISTRIBUTIONS = ("uniform", "exponential", "rootdup", "twodup", "eightdup",
                 "almostsorted", "sorted", "reversesorted", "zero", "zipf")


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied to a state array (in place safe)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64_scalar(state: int) -> tuple[int, int]:
    """One SplitMix64 step on a Python int: returns (new_state, output)."""
    state = (state + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    return state, z ^ (z >> 31)


def seed_for(config: int, array: int = 0) -> int:
    """Seed of array `array` of benchmark configuration `config`."""
    _, out = splitmix64_scalar(MASTER_SEED ^ (config << 32) ^ array)
    return out


def stream(seed: int, n: int, start: int = 0, chunk: int = 1 << 24) -> np.ndarray:
    """Outputs start .. start+n-1 of the SplitMix64 generator seeded with `seed`.

    Output i is mix(seed + (i+1)*golden), so any slice can be produced
    independently of the others.
    """
    out = np.empty(n, dtype=np.uint64)
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        idx = np.arange(start + c0 + 1, start + c1 + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            out[c0:c1] = _mix(s + idx * GOLDEN)
    return out


def _mulhi(x: np.ndarray, m: int) -> np.ndarray:
    """floor(x * m / 2**64) for uint64 x and 0 <= m < 2**32, exactly."""
    x = np.asarray(x, dtype=np.uint64)
    m = np.uint64(m)
    lo = x & np.uint64(0xFFFFFFFF)
    hi = x >> np.uint64(32)
    with np.errstate(over="ignore"):
        return (hi * m + ((lo * m) >> np.uint64(32))) >> np.uint64(32)


def _isqrt(n: int) -> int:
    import math
    return math.isqrt(n)


def gen_u64(dist: str, n: int, seed: int) -> np.ndarray:
    """uint64 keys of distribution `dist` (see module docstring)."""
    i = np.arange(n, dtype=np.uint64)
    if dist == "uniform":
        return stream(seed, n)
    if dist == "exponential":
        # A number drawn uniformly from [2^e, 2^(e+1)) with e uniform in
        # 0..floor(log2 n); two draws per element.
        lg = max(n, 1).bit_length() - 1
        x = stream(seed, 2 * n)
        e = _mulhi(x[0::2], lg + 1)
        y = x[1::2]
        base = np.left_shift(np.uint64(1), e)
        sh = np.uint64(64) - e
        frac = np.where(e == 0, np.uint64(0), y >> np.minimum(sh, np.uint64(63)))
        return base + frac
    if dist == "rootdup":
        return i % np.uint64(max(1, _isqrt(n)))
    if dist == "twodup":
        nn = np.uint64(max(n, 1))
        if n >= (1 << 32):
            raise ValueError("twodup needs n < 2^32 for exact arithmetic")
        with np.errstate(over="ignore"):
            return (i * i % nn + np.uint64(n // 2)) % nn
    if dist == "eightdup":
        nn = np.uint64(max(n, 1))
        if n >= (1 << 32):
            raise ValueError("eightdup needs n < 2^32 for exact arithmetic")
        with np.errstate(over="ignore"):
            i2 = i * i % nn
            i4 = i2 * i2 % nn
            i8 = i4 * i4 % nn
            return (i8 + np.uint64(n // 2)) % nn
    if dist == "almostsorted":
        a = np.arange(n, dtype=np.uint64)
        if n >= 2:
            sw = _isqrt(n)
            pos = _mulhi(stream(seed, sw), n - 1).astype(np.int64)
            for p in pos.tolist():          # sequential adjacent swaps
                a[p], a[p + 1] = a[p + 1], a[p]
        return a
    if dist == "sorted":
        return np.sort(stream(seed, n))
    if dist == "reversesorted":
        return np.sort(stream(seed, n))[::-1].copy()
    if dist == "zero":
        return np.zeros(n, dtype=np.uint64)
    if dist == "zipf":
        return zipf_values(n, seed)
    raise ValueError(f"unknown distribution {dist!r}")


_ZIPF_CDF = None


def zipf_values(n: int, seed: int, nvals: int = 1 << 20) -> np.ndarray:
    """Zipf with exponent 1 over 1..nvals by inverse-CDF table lookup."""
    global _ZIPF_CDF
    if _ZIPF_CDF is None or _ZIPF_CDF.size != nvals:
        w = 1.0 / np.arange(1, nvals + 1, dtype=np.float64)
        c = np.cumsum(w)
        _ZIPF_CDF = c / c[-1]
    u = (stream(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    v = np.searchsorted(_ZIPF_CDF, u, side="right")
    return (np.minimum(v, nvals - 1) + 1).astype(np.uint64)


def gen_u32(dist: str, n: int, seed: int) -> np.ndarray:
    if dist == "uniform":
        return (stream(seed, n) >> np.uint64(32)).astype(np.uint32)
    if dist in ("sorted", "reversesorted"):
        a = np.sort((stream(seed, n) >> np.uint64(32)).astype(np.uint32))
        return a if dist == "sorted" else a[::-1].copy()
    v = gen_u64(dist, n, seed)
    if v.size and int(v.max()) >= (1 << 32):
        raise ValueError(f"{dist} at n={n} does not fit uint32")
    return v.astype(np.uint32)


def gen_f64(dist: str, n: int, seed: int) -> np.ndarray:
    """IEEE doubles: uniform in [0,1), exponential with rate 1, sorted or
    reverse-sorted uniform doubles, or the integer distribution `dist`
    converted to double (exact: its values are below 2^53)."""
    if dist in ("uniform", "exponential", "sorted", "reversesorted"):
        u = (stream(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        if dist == "exponential":
            return -np.log1p(-u)
        if dist == "sorted":
            return np.sort(u)
        if dist == "reversesorted":
            return np.sort(u)[::-1].copy()
        return u
    v = gen_u64(dist, n, seed)
    if v.size and int(v.max()) >= (1 << 53):
        raise ValueError(f"{dist} at n={n} is not exact in double")
    return v.astype(np.float64)


def gen_pair(dist: str, n: int, seed: int) -> np.ndarray:
    """(n, 2) uint64: column 0 the key, column 1 the original index."""
    out = np.empty((n, 2), dtype=np.uint64)
    out[:, 0] = gen_u64(dist, n, seed)
    out[:, 1] = np.arange(n, dtype=np.uint64)
    return out


def gen_rec100(dist: str, n: int, seed: int) -> np.ndarray:
    """(n, 100) uint8 records: 10-byte key, then the index (8 bytes, little
    endian) and 82 random payload bytes."""
    rnd = stream(seed, 12 * n).view(np.uint8).reshape(n, 96)
    out = np.empty((n, 100), dtype=np.uint8)
    if dist == "uniform":
        out[:, 0:10] = rnd[:, 0:10]
    elif dist == "rootdup":
        k = (np.arange(n, dtype=np.uint64) % np.uint64(4096)).astype(">u8")
        out[:, 0:2] = 0
        out[:, 2:10] = k.view(np.uint8).reshape(n, 8)
    else:
        raise ValueError(dist)
    out[:, 10:18] = np.arange(n, dtype="<u8").view(np.uint8).reshape(n, 8)
    out[:, 18:100] = rnd[:, 10:92]
    return out


def gen_quartet(dist: str, n: int, seed: int) -> np.ndarray:
    """(n, 4) uint64: key words a, b, c and the original index.  Uniform:
    three independent uniform words.  Other distributions: a from the
    integer distribution and b, c derived from a (b = a >> 1, c = a ^
    0x5555...), so that equal a means an equal key and the distribution's
    duplicates reach the comparison of all three words."""
    out = np.empty((n, 4), dtype=np.uint64)
    if dist == "uniform":
        x = stream(seed, 3 * n)
        out[:, 0], out[:, 1], out[:, 2] = x[0::3], x[1::3], x[2::3]
    else:
        a = gen_u64(dist, n, seed)
        out[:, 0] = a
        out[:, 1] = a >> np.uint64(1)
        out[:, 2] = a ^ np.uint64(0x5555555555555555)
    out[:, 3] = np.arange(n, dtype=np.uint64)
    return out


def generate(kind: str, dist: str, n: int, seed: int) -> np.ndarray:
    """kind in {u32, u64, f64, pair, rec100, quartet}."""
    if kind == "u64":
        return gen_u64(dist, n, seed)
    if kind == "u32":
        return gen_u32(dist, n, seed)
    if kind == "f64":
        return gen_f64(dist, n, seed)
    if kind == "pair":
        return gen_pair(dist, n, seed)
    if kind == "rec100":
        return gen_rec100(dist, n, seed)
    if kind == "quartet":
        return gen_quartet(dist, n, seed)
    raise ValueError(kind)


def batch_layout(count: int, lo_log2: float, hi_log2: float, seed: int,
                 dists=("uniform", "twodup", "almostsorted")) -> tuple[np.ndarray, list]:
    """Sizes and distributions of a batch of `count` arrays: size i is
    floor(2^(lo + u_i (hi - lo))) (log-uniform) and distribution i is drawn
    uniformly from `dists`, both from the SplitMix64 stream of `seed`."""
    x = stream(seed, 2 * count)
    u = (x[0::2] >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    sizes = np.floor(2.0 ** (lo_log2 + u * (hi_log2 - lo_log2))).astype(np.int64)
    pick = (x[1::2] % np.uint64(len(dists))).astype(np.int64)
    return sizes, [dists[int(p)] for p in pick]


def generate_batch(kind: str, sizes, dists, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Concatenation of arrays generate(kind, dists[i], sizes[i], seed_i),
    seed_i = SplitMix64 output i+1 of `seed`; returns (data, offsets)."""
    sizes = np.asarray(sizes, dtype=np.int64)
    offs = np.zeros(len(sizes), dtype=np.int64)
    if len(sizes):
        offs[1:] = np.cumsum(sizes)[:-1]
    total = int(sizes.sum())
    seeds = stream(seed, len(sizes))
    first = generate(kind, dists[0] if len(sizes) else "uniform", 0, 0)
    out = np.empty((total,) + first.shape[1:], dtype=first.dtype)
    for i, (o, n) in enumerate(zip(offs, sizes)):
        out[o:o + n] = generate(kind, dists[i], int(n), int(seeds[i]))
    return out, offs


def poisson_arrivals(count: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of the given rate:
    cumulative sums of exponential gaps -log1p(-u)/rate."""
    u = (stream(seed, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return np.cumsum(-np.log1p(-u) / rate_per_s)
