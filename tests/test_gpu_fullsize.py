"""Bit-exact parity at the full benchmark sizes: 2^28 u64 and u32 keys of all
ten generators (samplesort and IPS2Ra), 2^27 doubles, Pair records and
Quartets, 2^24 100-byte records.  The sort runs through the C ABI with the parameters the
benchmark uses; the digest of its sorted key sequence must equal the digest
of the oracle's sorted keys of the same input (tests/golden/fullsize.py
writes those from the oracle alone).  Records must also keep their multiset:
Pair values, Quartet word 3 and record payload bytes 10..17 hold each
element's input index, so the output values must be a permutation of 0..n-1 and every
output record must equal the input record its index names.

The small configuration (2^20 u64 Uniform keys, k = 256, 2 KiB blocks,
alpha = 4, n0 = 16) is compared with the oracle element by element."""
import json
import os

import numpy as np
import pytest

import oracle
import paper_2009_13569_amd as ips
from golden import fullsize as fs
from gpu_util import assert_parity, log

pytestmark = pytest.mark.gpu

with open(fs.OUT) as _f:
    GOLD = json.load(_f)["cases"]


@pytest.fixture(scope="module")
def sorter():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return ips.Sorter(0)


def _device_input(c, dev):
    """The case's input as a device tensor (integer kinds as signed bit
    patterns of the same width; the library is told the kind)."""
    import torch
    import synth
    import synth.device as sd
    n = 1 << c["log2n"]
    kind, dist = c["kind"], c["dist"]
    if kind in ("u32", "u64", "pair") or (kind == "f64" and dist == "uniform"):
        return sd.generate(kind, dist, n, synth.seed_for(c["config"], c["array"]), dev)
    return torch.from_numpy(fs.generate(c)).to(dev)   # f64 Exponential (host log1p), records


def _key_digest(t, kind):
    """fs.digest of the key bytes of a sorted device array."""
    k = {"pair": lambda: t[:, 0], "rec100": lambda: t[:, :10], "quartet": lambda: t[:, :3]}.get(kind, lambda: t)()
    host = np.ascontiguousarray(k.contiguous().cpu().numpy())
    return fs.digest(memoryview(host).cast("B"), threads=16)


def _check_records(out, inp, kind):
    """Output indices form a permutation and each output record is the
    input record its index names (exact multiset equality)."""
    import torch
    n = out.shape[0]
    if kind in ("pair", "quartet"):
        ix = out[:, 1 if kind == "pair" else 3].view(torch.int64)
    else:
        ix = out[:, 10:18].contiguous().view(torch.int64).reshape(n)
    assert int(ix.min()) >= 0 and int(ix.max()) < n, "index out of range"
    seen = torch.zeros(n, dtype=torch.int32, device=out.device)
    seen.index_add_(0, ix, torch.ones(n, dtype=torch.int32, device=out.device))
    assert bool((seen == 1).all()), "payload indices are not a permutation"
    assert bool((inp.index_select(0, ix) == out).all()), "a record changed"


CASES = [(name, algo) for name, c in sorted(GOLD.items())
         for algo in (("samplesort", "radix") if c["kind"] not in ("rec100", "quartet") else ("samplesort",))]


@pytest.mark.parametrize("name,algo", CASES, ids=[f"{n}-{a}" for n, a in CASES])
def test_fullsize_digest(sorter, name, algo):
    import torch
    c = GOLD[name]
    kind = c["kind"]
    dev = torch.device("cuda:0")
    log(f"fullsize {name} {algo}: generating")
    src = _device_input(c, dev)
    work = src.clone()
    log(f"fullsize {name} {algo}: sorting {work.shape[0]} elements")
    sorter.sort_(work, algo=algo, kind=kind)
    torch.cuda.synchronize()
    log(f"fullsize {name} {algo}: digest")
    assert _key_digest(work, kind) == c["digest"], f"{name} {algo}: sorted keys differ from the oracle's"
    if kind in ("pair", "rec100", "quartet"):
        _check_records(work, src, kind)
    del src, work
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def untuned():
    """Without the tuning table: the configuration's parameters exactly."""
    return ips.Sorter(0, tuning=None)


def test_small_config_elementwise(untuned):
    """2^20 u64 Uniform keys with k = 256, 2 KiB blocks (buffer blocks in the
    workspace), n0 = 16 and the root's alpha = 4, element by element."""
    import synth
    a = synth.generate("u64", "uniform", 1 << 20, synth.seed_for(1, 0))
    import torch
    p1 = ips.make_params(k=256, block_bytes=2048, n0=16,
                         flags=ips.FLAG_GLOBAL_BUFFERS | ips.FLAG_LEVEL1_ONLY | ips.FLAG_PAPER_ROOT_ALPHA)
    t = torch.from_numpy(a).cuda()
    untuned.sort_(t, params=p1)              # the root step alone: its parameters
    torch.cuda.synchronize()
    ri = untuned.root_info()
    assert (ri.valid, ri.alpha, ri.k_prime, ri.m, ri.block_elems) == (1, 4, 256, 1024, 256)
    p = ips.make_params(k=256, block_bytes=2048, n0=16, flags=ips.FLAG_GLOBAL_BUFFERS | ips.FLAG_PAPER_ROOT_ALPHA)
    t = torch.from_numpy(a).cuda()
    untuned.sort_(t, params=p)
    torch.cuda.synchronize()
    assert_parity(t.cpu().numpy(), a, "u64", ref=oracle.sort(a, "u64"))


def test_small_config_insertion_base_case(untuned):
    """The same configuration with the paper's base case: buckets of at most
    2 n0 = 32 elements, and every bucket of a task of at most k n0 = 4096
    elements, sorted by insertion sort; everything larger partitioned again
    (IPS_FLAG_INSERTION_BASE).  Element by element against the oracle, also
    for records and for inputs with many equal keys."""
    import synth
    import torch
    flags = ips.FLAG_GLOBAL_BUFFERS | ips.FLAG_INSERTION_BASE | ips.FLAG_PAPER_ROOT_ALPHA
    p = ips.make_params(k=256, block_bytes=2048, n0=16, flags=flags)
    a = synth.generate("u64", "uniform", 1 << 20, synth.seed_for(1, 0))
    t = torch.from_numpy(a).cuda()
    log("config 1 with insertion-sort base cases")
    untuned.sort_(t, params=p)
    torch.cuda.synchronize()
    assert_parity(t.cpu().numpy(), a, "u64", ref=oracle.sort(a, "u64"))
    st = untuned.stats()
    assert st.levels >= 3, st.levels   # 2^20 -> 2^12 -> 16: three partitioning levels (k' adapts below)
    from gpu_util import generate
    for kind, dist, n in (("u32", "twodup", 300_001), ("pair", "rootdup", 100_003), ("rec100", "uniform", 20_011),
                          ("quartet", "eightdup", 50_001), ("f64", "exponential", 100_003)):
        a = generate(kind, dist, n, 31)
        log(f"insertion base case {kind} {dist} n={n}")
        q = ips.make_params(n0=16, flags=ips.FLAG_INSERTION_BASE | ips.FLAG_NO_SORTED_CHECK)
        t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
        untuned.sort_(t, params=q, kind=kind)
        torch.cuda.synchronize()
        assert_parity(t.cpu().numpy(), a, kind)


with open(fs.OUT) as _f:
    GOLD_BATCH = json.load(_f).get("batch")


@pytest.mark.skipif(GOLD_BATCH is None, reason="no oracle digest of the batched workload")
@pytest.mark.parametrize("graph", [True, False])
def test_batch_workload_digest(sorter, graph):
    """The batched workload at full size (4096 u64 arrays of 2^8 to 2^22
    keys, 1.79 G keys), as one ips_sort_segments call, and as replays of a
    captured graph of device-planned steps: the concatenation of the sorted
    arrays must equal the oracle's (digest)."""
    import torch
    import synth.device as sd
    sizes, dists, seeds = fs.batch_inputs()
    offs = np.zeros(len(sizes), dtype=np.int64)
    offs[1:] = np.cumsum(sizes)[:-1]
    total = int(sizes.sum())
    assert total == GOLD_BATCH["keys"]
    log(f"batch workload digest graph={graph}: generating {total} keys")
    t = torch.empty(total, dtype=torch.int64, device="cuda")
    for o, n, d, s in zip(offs.tolist(), sizes.tolist(), dists, seeds.tolist()):
        t[o:o + n] = sd.gen_u64(d, n, int(s), "cuda")
    stream = torch.cuda.Stream()
    p = ips.make_params(flags=ips.FLAG_GRAPH if graph else 0)
    log(f"batch workload digest graph={graph}: sorting")
    with torch.cuda.stream(stream):
        sorter.sort_segments_(t, offs.tolist(), sizes.tolist(), params=p, kind="u64", stream=stream)
    stream.synchronize()
    host = np.ascontiguousarray(t.cpu().numpy())
    del t
    torch.cuda.empty_cache()
    assert fs.digest(memoryview(host).cast("B"), threads=16) == GOLD_BATCH["digest"]
