"""Parity of the batched entry point (ips_sort_segments) with the oracle.

Every segment must come out bit-identical (keys) to the oracle's sort of
that segment alone, elements between segments must stay untouched, and a
segment sorted in a batch must equal the same segment sorted alone.
"""
import numpy as np
import pytest

import oracle
import paper_2009_13569_amd as ips
import synth
from gpu_util import assert_parity, generate, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sorter():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return ips.Sorter(0)


def _run_segments(sorter, data, offs, sizes, kind, algo="samplesort", params=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(data)).cuda()
    sorter.sort_segments_(t, offs, sizes, algo=algo, params=params, kind=kind)
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _layout(sizes, gap=0):
    offs, o = [], 0
    for n in sizes:
        offs.append(o)
        o += n + gap
    return offs, o


def _check(out, data, offs, sizes, kind):
    covered = np.zeros(data.shape[0], dtype=bool)
    for o, n in zip(offs, sizes):
        assert_parity(out[o:o + n], data[o:o + n], kind)
        covered[o:o + n] = True
    assert np.array_equal(out[~covered], data[~covered]), "elements outside the segments changed"


MIXED = [0, 1, 2, 17, 1000, 16384, 16385, 40_000, 3, 150_001, 9000, 70_000]


@pytest.mark.parametrize("kind", ["u32", "u64", "f64", "pair", "rec100", "quartet"])
def test_segments_mixed_sizes(sorter, kind):
    sizes = [s for s in MIXED if kind not in ("rec100", "quartet") or s <= 40_000]
    offs, total = _layout(sizes, gap=5)
    data = generate(kind, "uniform", total, 31)
    log(f"segments {kind} samplesort sizes={sizes}")
    out = _run_segments(sorter, data, offs, sizes, kind)
    _check(out, data, offs, sizes, kind)


@pytest.mark.parametrize("kind", ["u32", "u64", "f64", "pair"])
def test_segments_radix(sorter, kind):
    offs, total = _layout(MIXED, gap=3)
    data = generate(kind, "uniform", total, 32)
    log(f"segments {kind} radix")
    out = _run_segments(sorter, data, offs, MIXED, kind, algo="radix")
    _check(out, data, offs, MIXED, kind)


@pytest.mark.parametrize("dist", ["twodup", "rootdup", "zero", "almostsorted", "exponential"])
def test_segments_distributions(sorter, dist):
    sizes = [100_000, 20_000, 300, 65_537]
    offs, total = _layout(sizes)
    data = np.concatenate([generate("u64", dist, n, 40 + i) for i, n in enumerate(sizes)])
    for algo in ("samplesort", "radix"):
        log(f"segments u64 {dist} {algo}")
        out = _run_segments(sorter, data, offs, sizes, "u64", algo=algo)
        _check(out, data, offs, sizes, "u64")


def test_segments_forced_partitioning(sorter):
    # Every segment of two or more elements goes through partitioning steps,
    # many tasks per batch.
    sizes = [int(s) for s in np.random.default_rng(3).integers(0, 3000, size=300)]
    offs, total = _layout(sizes)
    data = generate("u64", "uniform", total, 44)
    p = ips.make_params(lds_task_max=64, k=16)
    log("segments forced partitioning")
    out = _run_segments(sorter, data, offs, sizes, "u64", params=p)
    _check(out, data, offs, sizes, "u64")


def test_segment_alone_equals_in_batch(sorter):
    import torch
    sizes = [200_000, 50_000, 123_457]
    offs, total = _layout(sizes)
    data = generate("pair", "rootdup", total, 45)
    out = _run_segments(sorter, data, offs, sizes, "pair")
    for o, n in zip(offs, sizes):
        t = torch.from_numpy(np.ascontiguousarray(data[o:o + n])).cuda()
        sorter.sort_(t, kind="pair")
        alone = t.cpu().numpy()
        assert np.array_equal(alone[:, 0], out[o:o + n, 0])
        assert_parity(out[o:o + n], data[o:o + n], "pair", ref=oracle.sort(data[o:o + n], "pair"))


def test_batch_workload_scaled(sorter):
    # The batched workload's shape (log-uniform sizes, three distributions)
    # at a size the oracle checks in seconds.
    sizes, dists = synth.batch_layout(256, 8, 18, synth.seed_for(4, 1))
    data, offs = synth.generate_batch("u64", sizes, dists, synth.seed_for(4, 2))
    log(f"batch workload scaled: {len(sizes)} arrays, {int(sizes.sum())} keys")
    out = _run_segments(sorter, data, offs, sizes, "u64")
    _check(out, data, offs, sizes, "u64")


@pytest.mark.parametrize("kind", ["u32", "u64", "f64", "pair"])
def test_segments_all_distributions(sorter, kind):
    # One segment per distribution of the paper, sizes above the LDS tier.
    sizes = [70_000 + 1000 * i for i in range(len(synth.DISTRIBUTIONS))]
    offs, total = _layout(sizes, gap=1)
    data = np.zeros((total,) + generate(kind, "uniform", 1, 0).shape[1:],
                    dtype=generate(kind, "uniform", 1, 0).dtype)
    for i, (dist, o, n) in enumerate(zip(synth.DISTRIBUTIONS, offs, sizes)):
        data[o:o + n] = generate(kind, dist, n, 50 + i)
    for algo in ("samplesort", "radix"):
        log(f"segments all distributions {kind} {algo}")
        out = _run_segments(sorter, data, offs, sizes, kind, algo=algo)
        _check(out, data, offs, sizes, kind)


@pytest.mark.parametrize("kind", ["u32", "u64", "pair"])
def test_segments_one_bucket_many_pieces(sorter, kind):
    # All-equal keys in large segments: the single equality bucket spans
    # every stripe, so its placement pieces far outnumber one mask word.
    sizes = [4_000_037, 1_500_000, 20_000]
    offs, total = _layout(sizes, gap=2)
    data = generate(kind, "uniform", total, 70)
    for o, n in zip(offs[:2], sizes[:2]):
        data[o:o + n] = generate(kind, "zero", n, 71)
    log(f"segments one bucket many pieces {kind}")
    out = _run_segments(sorter, data, offs, sizes, kind)
    _check(out, data, offs, sizes, kind)


@pytest.mark.parametrize("kind", ["u32", "f64", "pair", "rec100"])
def test_segments_sorted_detection(sorter, kind):
    # Sorted segments stay, reverse-sorted ones are reversed, ties allowed;
    # with the detection off the same segments are partitioned.
    n = 30_000 if kind == "rec100" else 100_003
    parts = []
    for i, dist in enumerate(["sorted", "reversesorted", "zero", "uniform"]):
        a = generate(kind, dist if kind != "rec100" else "uniform", n, 75 + i)
        if kind == "rec100" and dist in ("sorted", "reversesorted"):
            a = oracle.sort(a, kind)
            if dist == "reversesorted":
                a = a[::-1].copy()
        parts.append(a)
    sizes = [n] * 4
    offs, total = _layout(sizes, gap=3)
    data = np.zeros((total,) + parts[0].shape[1:], dtype=parts[0].dtype)
    for o, a in zip(offs, parts):
        data[o:o + n] = a
    for flags in (0, ips.FLAG_NO_SORTED_CHECK):
        log(f"segments sorted detection {kind} flags={flags}")
        out = _run_segments(sorter, data, offs, sizes, kind, params=ips.make_params(flags=flags))
        _check(out, data, offs, sizes, kind)


@pytest.mark.parametrize("kind", ["u64", "pair"])
def test_segments_order_check_late_descent(sorter, kind):
    """The per-segment order check stops a chunk early once it has seen a
    descent and an ascent; a segment whose only descent (or ascent) lies far
    into a later chunk must still be found unsorted and be sorted."""
    n = 200_003
    base = oracle.sort(generate(kind, "uniform", n, 91), kind)
    parts = []
    for pos in (n - 2, 65536 + 1000, 3 * 65536 + 7):      # one adjacent swap late in the segment
        a = base.copy()
        a[[pos, pos + 1]] = a[[pos + 1, pos]]
        parts.append(a)
    rev = base[::-1].copy()
    rev[[n - 2, n - 1]] = rev[[n - 1, n - 2]]              # reverse sorted but for its last pair
    parts.append(rev)
    parts.append(base.copy())                               # sorted: stays as it is
    sizes = [n] * len(parts)
    offs, total = _layout(sizes, gap=5)
    data = np.zeros((total,) + base.shape[1:], dtype=base.dtype)
    for o, a in zip(offs, parts):
        data[o:o + n] = a
    log(f"segments late descent {kind}")
    out = _run_segments(sorter, data, offs, sizes, kind)
    _check(out, data, offs, sizes, kind)
