"""Brute force on the GPU: every permutation of n <= 8 distinct keys and every
sequence of n <= 8 keys over three values, for every element type and both
algorithms, each as one batched call (ips_sort_segments) with one segment
per input.  The LDS tier is off (lds_task_max = 1) and blocks hold one or
two elements, so every segment of two or more elements goes through
partitioning steps (sampling, classification, block permutation, cleanup)
with k = 2 or 4 buckets and every equality-bucket mode.  Each segment's
output is compared with the oracle's sort of the same segment."""
import numpy as np
import pytest

import bruteforce_cases as bc
import oracle
import paper_2009_13569_amd as ips
from gpu_util import keys_of, log

pytestmark = pytest.mark.gpu

KINDS = ["u32", "u64", "f64", "pair", "rec100", "quartet"]


@pytest.fixture(scope="module")
def sorter():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return ips.Sorter(0, tuning=None)


_CACHE = {}


def _inputs(kind):
    """(input, oracle output, offsets, sizes) of all segments of a type."""
    if kind not in _CACHE:
        seqs, sizes = [], []
        for n in range(1, bc.NMAX + 1):
            for s in bc.permutation_seqs(kind, n) + bc.ternary_seqs(kind, n):
                seqs.append(s)
                sizes.append(n)
        inp = bc.build(kind, seqs)
        offs = np.zeros(len(sizes), dtype=np.int64)
        offs[1:] = np.cumsum(sizes)[:-1]
        ref = inp.copy()
        for o, n in zip(offs.tolist(), sizes):
            ref[o:o + n] = oracle.sort(inp[o:o + n], kind)
        _CACHE[kind] = (inp, ref, offs, np.asarray(sizes, dtype=np.int64))
    return _CACHE[kind]


def _check(out, inp, ref, offs, kind, what):
    ko, kr = keys_of(out, kind), keys_of(ref, kind)
    if not np.array_equal(ko, kr):
        bad = np.nonzero((ko != kr).reshape(ko.shape[0], -1).any(axis=1))[0]
        seg = np.searchsorted(offs, bad[0], side="right") - 1
        raise AssertionError(f"{what}: {bad.size} keys differ, first at element {bad[0]} (segment {seg})")
    if kind in ("pair", "rec100", "quartet"):
        if kind == "rec100":
            ix = out[:, 10:18].copy().view("<u8")[:, 0].astype(np.int64)
        else:
            ix = out[:, {"pair": 1, "quartet": 3}[kind]].astype(np.int64)
        assert np.array_equal(np.sort(ix), np.arange(inp.shape[0])), f"{what}: payload indices not a permutation"
        assert np.array_equal(out, inp[ix]), f"{what}: a record changed"
        seg_of = np.repeat(np.arange(offs.size), np.diff(np.append(offs, inp.shape[0])))
        assert np.array_equal(seg_of[ix], seg_of), f"{what}: a record left its segment"


def _run(sorter, kind, algo, params, what):
    import torch
    inp, ref, offs, sizes = _inputs(kind)
    log(f"brute {what}: {offs.size} segments, {inp.shape[0]} elements")
    t = torch.from_numpy(inp.copy()).cuda()
    sorter.sort_segments_(t, offs.tolist(), sizes.tolist(), algo=algo, params=params, kind=kind)
    torch.cuda.synchronize()
    _check(t.cpu().numpy(), inp, ref, offs, kind, what)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("k,bmul", [(2, 1), (4, 2)])
@pytest.mark.parametrize("eq", ["auto", "on", "off"])
def test_brute_force_samplesort(sorter, kind, k, bmul, eq):
    flags = ips.FLAG_NO_SORTED_CHECK | {"auto": 0, "on": ips.FLAG_EQ_ON, "off": ips.FLAG_EQ_OFF}[eq]
    p = ips.make_params(k=k, block_bytes=bmul * ips.ELEM_BYTES[kind], n0=1, lds_task_max=1, flags=flags)
    _run(sorter, kind, "samplesort", p, f"{kind} samplesort k={k} b={bmul} eq={eq}")


@pytest.mark.parametrize("kind", ["u32", "u64", "f64", "pair"])
@pytest.mark.parametrize("bmul", [1, 2])
def test_brute_force_radix(sorter, kind, bmul):
    p = ips.make_params(block_bytes=bmul * ips.ELEM_BYTES[kind], lds_task_max=1, flags=ips.FLAG_NO_SORTED_CHECK)
    _run(sorter, kind, "radix", p, f"{kind} radix b={bmul}")


@pytest.mark.parametrize("kind", KINDS)
def test_brute_force_graph_and_sorted_check(sorter, kind):
    """The same inputs with the sorted / reverse-sorted detection on (sorted
    and reversed segments are recognised, the rest partitioned), and as
    replays of a captured graph of device-planned steps."""
    import torch
    p = ips.make_params(k=4, block_bytes=ips.ELEM_BYTES[kind], n0=1, lds_task_max=1)
    _run(sorter, kind, "samplesort", p, f"{kind} samplesort sorted-check")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        pg = ips.make_params(k=2, block_bytes=ips.ELEM_BYTES[kind], n0=1, lds_task_max=1,
                             flags=ips.FLAG_GRAPH | ips.FLAG_NO_SORTED_CHECK)
        _run(sorter, kind, "samplesort", pg, f"{kind} samplesort graph")
        if kind not in ("rec100", "quartet"):
            pr = ips.make_params(lds_task_max=1, flags=ips.FLAG_GRAPH)
            _run(sorter, kind, "radix", pr, f"{kind} radix graph")
    stream.synchronize()
