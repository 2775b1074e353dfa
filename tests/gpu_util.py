"""Helpers of the GPU parity tests: move numpy arrays through the HIP sort
(via the C ABI binding) and compare with the oracle."""
from __future__ import annotations

import sys
from collections import Counter

import numpy as np

import oracle
import synth


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_sort(sorter, a: np.ndarray, kind: str, algo: str = "samplesort", params=None) -> np.ndarray:
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    sorter.sort_(t, algo=algo, params=params, kind=kind)
    torch.cuda.synchronize()
    return t.cpu().numpy()


def keys_of(a: np.ndarray, kind: str) -> np.ndarray:
    if kind in ("u32", "u64", "f64"):
        return a.view(np.uint32 if kind == "u32" else np.uint64)
    if kind == "pair":
        return a[:, 0]
    if kind == "quartet":
        return a[:, :3]
    return a[:, :10]


def assert_parity(out: np.ndarray, inp: np.ndarray, kind: str, ref: np.ndarray | None = None) -> None:
    """Keys bit-identical to the oracle's; for records, equal multisets and
    (pairs) every value still names an input index with that key."""
    if ref is None:
        ref = oracle.sort(inp, kind)
    ko, kr = keys_of(out, kind), keys_of(ref, kind)
    if not np.array_equal(ko, kr):
        bad = np.nonzero((ko != kr).reshape(ko.shape[0], -1).any(axis=1))[0]
        raise AssertionError(f"{kind}: {bad.size} keys differ, first at {bad[:5].tolist()}")
    if kind in ("pair", "rec100", "quartet"):
        rows_o = np.ascontiguousarray(out).view(np.dtype((np.void, out.shape[1] * out.itemsize))).ravel()
        rows_i = np.ascontiguousarray(inp).view(np.dtype((np.void, inp.shape[1] * inp.itemsize))).ravel()
        assert np.array_equal(np.sort(rows_o), np.sort(rows_i)), "record multiset changed"
    vc = {"pair": 1, "quartet": 3}.get(kind)
    if vc is not None and np.array_equal(inp[:, vc], np.arange(inp.shape[0], dtype=np.uint64)):
        # inputs whose values are the original indices: each output value
        # must name an input row with the same key
        v = out[:, vc].astype(np.int64)
        assert np.array_equal(np.sort(v), np.arange(inp.shape[0])), "values are not a permutation"
        assert np.array_equal(inp[v, :vc], out[:, :vc]), "value does not match its key"


def generate(kind: str, dist: str, n: int, seed: int) -> np.ndarray:
    if kind == "f64":
        return synth.gen_f64(dist, n, seed)
    if kind == "rec100":
        return synth.gen_rec100(dist if dist in ("uniform", "rootdup") else "uniform", n, seed)
    return synth.generate(kind, dist, n, seed)   # u32, u64, pair, quartet
