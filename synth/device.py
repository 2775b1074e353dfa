"""The generators of `synth` evaluated on a GPU with torch, for workloads
too large to build on the host (batched arrays, serving traces).

Integer outputs are identical to `synth.generate` for the same arguments
(SplitMix64 in wrapping int64 arithmetic with logical shifts); the f64
exponential distribution may differ from the host's in the last bit
(device log1p).  Input generation only: none of the sorting method's
arithmetic is here.
"""
from __future__ import annotations

import math

import numpy as np
import torch

import synth

_MASK64 = (1 << 64) - 1


def _s64(v: int) -> int:
    v &= _MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


_G = _s64(0x9E3779B97F4A7C15)
_M1 = _s64(0xBF58476D1CE4E5B9)
_M2 = _s64(0x94D049BB133111EB)
_SIGN = -(1 << 63)


def _lsr(z: torch.Tensor, s: int) -> torch.Tensor:
    return (z >> s) & ((1 << (64 - s)) - 1)


def _mix(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _lsr(z, 30)) * _M1
    z = (z ^ _lsr(z, 27)) * _M2
    return z ^ _lsr(z, 31)


def stream(seed: int, n: int, device, start: int = 0) -> torch.Tensor:
    """synth.stream as int64 bit patterns on `device`."""
    idx = torch.arange(start + 1, start + n + 1, dtype=torch.int64, device=device)
    return _mix(idx * _G + _s64(seed))


def _mulhi(x: torch.Tensor, m: int) -> torch.Tensor:
    """floor(x * m / 2^64) for x as uint64 bit patterns and 0 <= m < 2^32."""
    lo = x & 0xFFFFFFFF
    hi = _lsr(x, 32)
    return _lsr(hi * m + _lsr(lo * m, 32), 32)


def _usort(x: torch.Tensor) -> torch.Tensor:
    """Sort int64 bit patterns in unsigned order."""
    return torch.sort(x ^ _SIGN).values ^ _SIGN


def gen_u64(dist: str, n: int, seed: int, device) -> torch.Tensor:
    """synth.gen_u64 on the device (int64 tensor holding the uint64 bits)."""
    if dist == "uniform":
        return stream(seed, n, device)
    i = torch.arange(n, dtype=torch.int64, device=device)
    if dist == "exponential":
        lg = max(n, 1).bit_length() - 1
        x = stream(seed, 2 * n, device)
        e = _mulhi(x[0::2], lg + 1)
        y = x[1::2]
        sh = (64 - e).clamp(max=63)
        frac = (y >> sh) & ((torch.ones_like(sh) << (64 - sh)) - 1)
        frac = torch.where(e == 0, torch.zeros_like(frac), frac)
        return (torch.ones_like(e) << e) + frac
    if dist == "rootdup":
        return i % max(1, math.isqrt(n))
    if dist in ("twodup", "eightdup"):
        if n >= (1 << 31):
            raise ValueError(f"{dist} needs n < 2^31 on the device")
        nn = max(n, 1)
        v = i * i % nn
        if dist == "eightdup":
            v = v * v % nn
            v = v * v % nn
        return (v + n // 2) % nn
    if dist == "almostsorted":
        a = i.clone()
        if n >= 2:
            sw = math.isqrt(n)
            pos = synth._mulhi(synth.stream(seed, sw), n - 1).astype(np.int64).tolist()
            cur = {}
            for p in pos:                      # sequential adjacent swaps, on the host
                vp, vq = cur.get(p, p), cur.get(p + 1, p + 1)
                cur[p], cur[p + 1] = vq, vp
            if cur:
                k = torch.tensor(list(cur.keys()), dtype=torch.int64, device=device)
                v = torch.tensor(list(cur.values()), dtype=torch.int64, device=device)
                a[k] = v
        return a
    if dist == "sorted":
        return _usort(stream(seed, n, device))
    if dist == "reversesorted":
        return _usort(stream(seed, n, device)).flip(0)
    if dist == "zero":
        return torch.zeros(n, dtype=torch.int64, device=device)
    if dist == "zipf":
        synth.zipf_values(0, 0)                 # builds the host CDF table
        cdf = torch.from_numpy(synth._ZIPF_CDF).to(device)
        u = _lsr(stream(seed, n, device), 11).to(torch.float64) * (2.0 ** -53)
        v = torch.searchsorted(cdf, u, right=True)
        return torch.clamp(v, max=cdf.numel() - 1) + 1
    raise ValueError(f"unknown distribution {dist!r}")


def _u32_bits(v: torch.Tensor) -> torch.Tensor:
    return torch.where(v >= (1 << 31), v - (1 << 32), v).to(torch.int32)


def generate(kind: str, dist: str, n: int, seed: int, device) -> torch.Tensor:
    """synth.generate(kind, dist, n, seed) for kind in {u32, u64, f64, pair}
    as a device tensor (int32 / int64 bit patterns, float64, (n, 2) int64)."""
    if kind == "u64":
        return gen_u64(dist, n, seed, device)
    if kind == "u32":
        if dist == "uniform":
            return _u32_bits(_lsr(stream(seed, n, device), 32))
        if dist in ("sorted", "reversesorted"):
            a = torch.sort(_lsr(stream(seed, n, device), 32)).values
            return _u32_bits(a if dist == "sorted" else a.flip(0))
        v = gen_u64(dist, n, seed, device)
        return _u32_bits(v)
    if kind == "f64":
        if dist in ("uniform", "exponential", "sorted", "reversesorted"):
            u = _lsr(stream(seed, n, device), 11).to(torch.float64) * (2.0 ** -53)
            if dist == "exponential":
                return -torch.log1p(-u)
            if dist == "sorted":
                return torch.sort(u).values
            if dist == "reversesorted":
                return torch.sort(u).values.flip(0)
            return u
        return gen_u64(dist, n, seed, device).to(torch.float64)
    if kind == "pair":
        out = torch.empty((n, 2), dtype=torch.int64, device=device)
        out[:, 0] = gen_u64(dist, n, seed, device)
        out[:, 1] = torch.arange(n, dtype=torch.int64, device=device)
        return out
    raise ValueError(kind)
