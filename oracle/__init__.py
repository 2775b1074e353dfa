"""Test infrastructure: ctypes wrapper around the plain C oracle.

Only the test suite, ``__graft_entry__.smoke`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does.
Functions follow arXiv 2009.13569 as cited in ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

TYPES = {"u32": 1, "u64": 2, "f64": 3, "pair": 4, "rec100": 5, "quartet": 6}
ELEM_BYTES = {"u32": 4, "u64": 8, "f64": 8, "pair": 16, "rec100": 100, "quartet": 32}
_DT = {"u32": np.uint32, "u64": np.uint64, "f64": np.float64,
       "pair": np.uint64, "rec100": np.uint8, "quartet": np.uint64}

_lib = None


def build() -> str:
    """Compile liboracle.so with gcc (always recompiles)."""
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-Wall", "-o", tmp, SRC])
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        L.oracle_elem_bytes.argtypes = [i32]; L.oracle_elem_bytes.restype = ctypes.c_size_t
        L.oracle_splitmix64_next.argtypes = [ctypes.POINTER(u64)]; L.oracle_splitmix64_next.restype = u64
        L.oracle_mulhi64.argtypes = [u64, u64]; L.oracle_mulhi64.restype = u64
        L.oracle_key_less.argtypes = [i32, vp, vp]; L.oracle_key_less.restype = i32
        L.oracle_sort.argtypes = [vp, u64, i32]; L.oracle_sort.restype = i32
        L.oracle_alpha.argtypes = [u64]; L.oracle_alpha.restype = u32
        L.oracle_adaptive_k.argtypes = [u64, u32, u32]; L.oracle_adaptive_k.restype = u32
        L.oracle_task_seed.argtypes = [u64, u64, u32]; L.oracle_task_seed.restype = u64
        L.oracle_sample_step.argtypes = [vp, u64, u64, i32, u32, u32, u64, u32, i32, vp, vp, vp]
        L.oracle_sample_step.restype = i32
        L.oracle_classify.argtypes = [i32, vp, vp, u32, i32]; L.oracle_classify.restype = u32
        L.oracle_histogram.argtypes = [vp, u64, i32, vp, u32, i32, vp]; L.oracle_histogram.restype = i32
        L.oracle_radix_digit_info.argtypes = [vp, u64, i32, vp]; L.oracle_radix_digit_info.restype = i32
        L.oracle_radix_histogram.argtypes = [vp, u64, i32, u32, u32, vp]; L.oracle_radix_histogram.restype = i32
        L.oracle_check_partition.argtypes = [vp, u64, i32, vp, u32, i32, vp, vp]
        L.oracle_check_partition.restype = i32
        L.oracle_count_less.argtypes = [vp, u64, i32, vp, i32]; L.oracle_count_less.restype = u64
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _n(a: np.ndarray, kind: str) -> int:
    return a.shape[0]


def _check(a: np.ndarray, kind: str) -> np.ndarray:
    a = np.ascontiguousarray(a)
    if a.dtype != _DT[kind]:
        raise TypeError(f"{kind} needs dtype {_DT[kind]}, got {a.dtype}")
    if kind == "pair" and (a.ndim != 2 or a.shape[1] != 2):
        raise TypeError("pair arrays are (n, 2)")
    if kind == "rec100" and (a.ndim != 2 or a.shape[1] != 100):
        raise TypeError("rec100 arrays are (n, 100)")
    if kind == "quartet" and (a.ndim != 2 or a.shape[1] != 4):
        raise TypeError("quartet arrays are (n, 4)")
    return a


def splitmix64(state: int, count: int) -> list[int]:
    st = ctypes.c_uint64(state)
    return [int(lib().oracle_splitmix64_next(ctypes.byref(st))) for _ in range(count)]


def mulhi64(a: int, b: int) -> int:
    return int(lib().oracle_mulhi64(a, b))


def key_less(kind: str, a: np.ndarray, b: np.ndarray) -> bool:
    a = _check(a.reshape((1,) + a.shape) if kind in ("pair", "rec100", "quartet") and a.ndim == 1
               else np.atleast_1d(a), kind)
    b = _check(b.reshape((1,) + b.shape) if kind in ("pair", "rec100", "quartet") and b.ndim == 1
               else np.atleast_1d(b), kind)
    return bool(lib().oracle_key_less(TYPES[kind], _ptr(a), _ptr(b)))


def sort(a: np.ndarray, kind: str) -> np.ndarray:
    """Sorted copy of `a` (stable bottom-up merge sort, see oracle.c)."""
    out = _check(a, kind).copy()
    rc = lib().oracle_sort(_ptr(out), _n(out, kind), TYPES[kind])
    if rc:
        raise RuntimeError(f"oracle_sort failed: {rc}")
    return out


def alpha(n: int) -> int:
    return int(lib().oracle_alpha(n))


def adaptive_k(n: int, k: int = 256, n0: int = 16) -> int:
    return int(lib().oracle_adaptive_k(n, k, n0))


def task_seed(seed: int, l: int, level: int) -> int:
    return int(lib().oracle_task_seed(seed, l, level))


def sample_step(a: np.ndarray, kind: str, l: int = 0, n: int | None = None, k: int = 256,
                n0: int = 16, seed: int = 0, level: int = 0, eq_mode: int = -1) -> dict:
    a = _check(a, kind)
    if n is None:
        n = a.shape[0] - l
    info = np.zeros(7, dtype=np.uint32)
    kp = adaptive_k(n, k, n0)
    spl = np.zeros((kp + 1,) + a.shape[1:], dtype=a.dtype)
    m = alpha(n) * kp
    smp = np.zeros((m,) + a.shape[1:], dtype=a.dtype)
    rc = lib().oracle_sample_step(_ptr(a), l, n, TYPES[kind], k, n0, seed, level, eq_mode,
                                  _ptr(info), _ptr(spl), _ptr(smp))
    if rc:
        raise RuntimeError(f"oracle_sample_step failed: {rc}")
    K = int(info[4])
    return {"alpha": int(info[0]), "k_prime": int(info[1]), "m": int(info[2]), "u": int(info[3]),
            "K": K, "eq": bool(info[5]), "nb": int(info[6]), "splitters": spl[:K].copy(),
            "sample": smp}


def classify(e: np.ndarray, kind: str, splitters: np.ndarray, K: int, eq: bool) -> int:
    e = _check(e.reshape((1,) + e.shape) if kind in ("pair", "rec100", "quartet") and e.ndim == 1
               else np.atleast_1d(e), kind)
    s = _check(splitters, kind)
    return int(lib().oracle_classify(TYPES[kind], _ptr(e), _ptr(s), K, int(eq)))


def histogram(a: np.ndarray, kind: str, splitters: np.ndarray, K: int, eq: bool) -> np.ndarray:
    a = _check(a, kind)
    s = _check(splitters, kind)
    out = np.zeros(2 * K if eq else K, dtype=np.uint64)
    rc = lib().oracle_histogram(_ptr(a), _n(a, kind), TYPES[kind], _ptr(s), K, int(eq), _ptr(out))
    if rc:
        raise RuntimeError("oracle_histogram failed")
    return out


def radix_digit_info(a: np.ndarray, kind: str) -> dict:
    a = _check(a, kind)
    info = np.zeros(3, dtype=np.uint32)
    rc = lib().oracle_radix_digit_info(_ptr(a), _n(a, kind), TYPES[kind], _ptr(info))
    if rc:
        raise RuntimeError("oracle_radix_digit_info failed")
    return {"shift": int(info[0]), "width": int(info[1]), "all_equal": bool(info[2])}


def radix_histogram(a: np.ndarray, kind: str, shift: int, width: int) -> np.ndarray:
    a = _check(a, kind)
    out = np.zeros(1 << width, dtype=np.uint64)
    rc = lib().oracle_radix_histogram(_ptr(a), _n(a, kind), TYPES[kind], shift, width, _ptr(out))
    if rc:
        raise RuntimeError("oracle_radix_histogram failed")
    return out


def check_partition(a: np.ndarray, kind: str, splitters: np.ndarray, K: int, eq: bool,
                    bucket_start: np.ndarray) -> int | None:
    """None if every element lies in its bucket's range, else the first bad index."""
    a = _check(a, kind)
    s = _check(splitters, kind)
    bs = np.ascontiguousarray(bucket_start, dtype=np.uint64)
    bad = np.zeros(1, dtype=np.uint64)
    rc = lib().oracle_check_partition(_ptr(a), _n(a, kind), TYPES[kind], _ptr(s), K, int(eq),
                                      _ptr(bs), _ptr(bad))
    return None if rc == 0 else int(bad[0])


def count_less(a: np.ndarray, kind: str, v: np.ndarray, or_equal: bool = False) -> int:
    a = _check(a, kind)
    v = _check(v.reshape((1,) + v.shape) if kind in ("pair", "rec100", "quartet") and v.ndim == 1
               else np.atleast_1d(v), kind)
    return int(lib().oracle_count_less(_ptr(a), _n(a, kind), TYPES[kind], _ptr(v), int(or_equal)))
