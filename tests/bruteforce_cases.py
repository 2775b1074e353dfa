"""Inputs of the brute-force checks: for every element type, every
permutation of n <= 8 distinct keys and every sequence of n <= 8 keys over
three values.  Input construction only (no sorting arithmetic); the CPU
pins check the oracle on these inputs and the GPU tests the HIP library.

The key values are chosen so that the order of their bit patterns matters:
u32/u64 keys straddle the sign bit, f64 keys include both zeros, both
infinities, a subnormal and NaNs of both signs (IEEE 754 totalOrder), and
100-byte record keys differ in different byte positions with bytes above
0x7F (unsigned byte order)."""
from __future__ import annotations

import itertools

import numpy as np

NMAX = 8

# Eight distinct keys per type, listed in increasing key order.
_U32 = [0, 1, 0x7FFFFFFF, 0x80000000, 0x9E3779B9, 0xC0000000, 0xFFFFFFFE, 0xFFFFFFFF]
_U64 = [0, 1, 0x7FFFFFFFFFFFFFFF, 0x8000000000000000, 0x9E3779B97F4A7C15, 0xC000000000000000,
        0xFFFFFFFFFFFFFFFE, 0xFFFFFFFFFFFFFFFF]
# totalOrder: -NaN < -inf < -1.5 < -0.0 < +0.0 < smallest subnormal < +inf < +NaN
_F64 = [0xFFF8000000000000, 0xFFF0000000000000, 0xBFF8000000000000, 0x8000000000000000,
        0x0000000000000000, 0x0000000000000001, 0x7FF0000000000000, 0x7FF8000000000000]
# three values per type for the 3^n sequences
_TRI = {"u32": [0, 0x80000000, 0xFFFFFFFF],
        "u64": [0, 0x8000000000000000, 0xFFFFFFFFFFFFFFFF],
        "f64": [0x8000000000000000, 0x0000000000000000, 0x7FF8000000000000],   # -0.0, +0.0, NaN
        "pair": [0, 0x8000000000000000, 0xFFFFFFFFFFFFFFFF]}


def _rec_key(i: int) -> bytes:
    """Ten-byte key number i of eight, increasing in unsigned byte order:
    key i differs from key i-1 at a different byte position each time."""
    table = [bytes([0x00] * 10), bytes([0x00] * 9 + [0x01]), bytes([0x00] * 9 + [0xFF]),
             bytes([0x00] * 5 + [0x80] + [0x00] * 4), bytes([0x00, 0x7F] + [0xFF] * 8),
             bytes([0x00, 0x80] + [0x00] * 8), bytes([0x80] + [0x00] * 9), bytes([0xFF] * 10)]
    return table[i]


_REC_TRI = [bytes([0x00] * 10), bytes([0x7F] + [0xFF] * 9), bytes([0x80] + [0x00] * 9)]

# Quartet keys (a, b, c), increasing lexicographically, each differing from
# the one before in a different word (Algorithm 3).
_M = 0xFFFFFFFFFFFFFFFF
_QUARTET = [(0, 0, 0), (0, 0, 1), (0, 0, 1 << 63), (0, 1, 0), (0, 1 << 63, 0), (1, 0, 0), (1 << 63, 0, 0),
            (_M, _M, _M)]
_QUARTET_TRI = [(0, 0, _M), (0, 1, 0), (1, 0, 0)]


def key_values(kind: str) -> list:
    if kind == "quartet":
        return _QUARTET
    return {"u32": _U32, "u64": _U64, "f64": _F64, "pair": _U64}.get(kind) or [_rec_key(i) for i in range(8)]


def tri_values(kind: str) -> list:
    if kind == "quartet":
        return _QUARTET_TRI
    return _TRI.get(kind) or _REC_TRI


def build(kind: str, keyseqs: list[list], base_index: int = 0) -> np.ndarray:
    """One array per key sequence, concatenated: keys given as integers
    (bit patterns for f64), 10-byte strings (records) or (a, b, c) triples
    (Quartet).  Pair and Quartet values and record payloads (bytes 10..17,
    little endian) hold the element's position in the concatenation plus
    base_index; the rest of a record's payload is a fixed pattern."""
    flat = [k for s in keyseqs for k in s]
    n = len(flat)
    if kind == "u32":
        return np.array(flat, dtype=np.uint32)
    if kind == "u64":
        return np.array(flat, dtype=np.uint64)
    if kind == "f64":
        return np.array(flat, dtype=np.uint64).view(np.float64)
    idx = np.arange(base_index, base_index + n, dtype=np.uint64)
    if kind == "quartet":
        out = np.empty((n, 4), dtype=np.uint64)
        if n:
            out[:, :3] = np.array(flat, dtype=np.uint64).reshape(n, 3)
        out[:, 3] = idx
        return out
    if kind == "pair":
        out = np.empty((n, 2), dtype=np.uint64)
        out[:, 0] = np.array(flat, dtype=np.uint64)
        out[:, 1] = idx
        return out
    out = np.zeros((n, 100), dtype=np.uint8)
    if n:
        out[:, 0:10] = np.frombuffer(b"".join(flat), dtype=np.uint8).reshape(n, 10)
        out[:, 10:18] = idx.astype("<u8").view(np.uint8).reshape(n, 8)
        out[:, 18:] = (np.arange(82, dtype=np.uint16) * 37 % 251).astype(np.uint8)
    return out


def permutation_seqs(kind: str, n: int) -> list[list]:
    """Every permutation of the first n distinct keys of the type."""
    vals = key_values(kind)[:n]
    return [[vals[i] for i in p] for p in itertools.permutations(range(n))]


def ternary_seqs(kind: str, n: int) -> list[list]:
    """Every sequence of n keys over the type's three values."""
    vals = tri_values(kind)
    return [[vals[i] for i in s] for s in itertools.product(range(3), repeat=n)]
