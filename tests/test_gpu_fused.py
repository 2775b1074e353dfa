"""The radix step with exact bucket sizes and classification fused into the
block permutation (IPS_FLAG_FUSED): every element type with a radix key,
every generator, sizes spanning tiles and ragged tails, forced recursion
with tiny blocks and small LDS tasks (deferred swap reads, many claims per
bucket), batched segments and graph replay, brute force over n <= 8, and the
full-size inputs against the oracle's digests."""
import json

import numpy as np
import pytest

import bruteforce_cases as bc
import oracle
import paper_2009_13569_amd as ips
from golden import fullsize as fs
from gpu_util import assert_parity, generate, gpu_sort, log

pytestmark = pytest.mark.gpu

KINDS = ["u32", "u64", "f64", "pair"]
DISTS = ["uniform", "exponential", "rootdup", "twodup", "eightdup", "almostsorted", "zipf", "zero"]
F = ips.FLAG_FUSED


@pytest.fixture(scope="module")
def sorter():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return ips.Sorter(0, tuning=None)


@pytest.mark.parametrize("kind", KINDS)
def test_fused_matches_oracle(sorter, kind):
    for dist in DISTS if kind in ("u32", "u64") else ["uniform", "exponential", "rootdup"]:
        for n in (20_011, 300_001, 2_000_003):
            a = generate(kind, dist, n, 17 + n)
            log(f"fused {kind} {dist} n={n}")
            p = ips.make_params(flags=F | ips.FLAG_NO_SORTED_CHECK)
            assert_parity(gpu_sort(sorter, a, kind, algo="radix", params=p), a, kind)


@pytest.mark.parametrize("kind", ["u64", "pair"])
def test_fused_forced_recursion(sorter, kind):
    """Blocks of one to four elements and LDS tasks of at most 64: many
    levels, many claims and reservations per bucket, swap reads that exceed a
    tile and go through the deferral stack."""
    D = ips.ELEM_BYTES[kind]
    for bmul in (1, 4):
        for n in (65, 1000, 20_011, 150_001):
            for dist in ("uniform", "twodup"):
                a = generate(kind, dist, n, 900 + n)
                log(f"fused forced {kind} b={bmul} {dist} n={n}")
                p = ips.make_params(block_bytes=bmul * D, lds_task_max=64, flags=F | ips.FLAG_NO_SORTED_CHECK)
                assert_parity(gpu_sort(sorter, a, kind, algo="radix", params=p), a, kind)


def test_fused_segments_and_graph(sorter):
    import torch
    sizes = [0, 1, 2, 17, 1000, 16384, 16385, 40_000, 3, 150_001, 9000, 70_000, 1_000_003]
    offs = np.zeros(len(sizes), dtype=np.int64)
    offs[1:] = np.cumsum(sizes)[:-1]
    total = int(sum(sizes))
    data = generate("u64", "uniform", total, 55)
    for name, fl in (("device", 0), ("graph", ips.FLAG_GRAPH)):
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            t = torch.from_numpy(data.copy()).cuda()
            p = ips.make_params(flags=F | fl)
            log(f"fused segments {name}")
            sorter.sort_segments_(t, offs.tolist(), sizes, algo="radix", params=p, kind="u64")
        stream.synchronize()
        out = t.cpu().numpy()
        for o, n in zip(offs.tolist(), sizes):
            assert np.array_equal(out[o:o + n], oracle.sort(data[o:o + n], "u64")), (name, o, n)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("bmul", [1, 2])
def test_fused_brute_force(sorter, kind, bmul):
    """Every permutation of n <= 8 distinct keys and every sequence over
    three values, one segment each, through fused partitioning steps."""
    import torch
    seqs, sizes = [], []
    for n in range(1, bc.NMAX + 1):
        for sq in bc.permutation_seqs(kind, n) + bc.ternary_seqs(kind, n):
            seqs.append(sq)
            sizes.append(n)
    inp = bc.build(kind, seqs)
    offs = np.zeros(len(sizes), dtype=np.int64)
    offs[1:] = np.cumsum(sizes)[:-1]
    p = ips.make_params(block_bytes=bmul * ips.ELEM_BYTES[kind], lds_task_max=1,
                        flags=F | ips.FLAG_NO_SORTED_CHECK)
    log(f"fused brute {kind} b={bmul}: {len(sizes)} segments")
    t = torch.from_numpy(inp.copy()).cuda()
    sorter.sort_segments_(t, offs.tolist(), sizes, algo="radix", params=p, kind=kind)
    torch.cuda.synchronize()
    out = t.cpu().numpy()
    for o, n in zip(offs.tolist(), sizes):
        assert_parity(out[o:o + n], inp[o:o + n], kind)


with open(fs.OUT) as _f:
    GOLD = json.load(_f)["cases"]
FULL = sorted(name for name, c in GOLD.items() if c["kind"] in KINDS)


@pytest.mark.parametrize("name", FULL)
def test_fused_fullsize_digest(sorter, name):
    import torch
    import synth
    import synth.device as sd
    c = GOLD[name]
    kind, n = c["kind"], 1 << c["log2n"]
    seed = synth.seed_for(c["config"], c["array"])
    if kind == "f64" and c["dist"] != "uniform":
        t = torch.from_numpy(fs.generate(c)).cuda()
    else:
        t = sd.generate(kind, c["dist"], n, seed, "cuda")
    log(f"fused fullsize {name}")
    sorter.sort_(t, algo="radix", params=ips.make_params(flags=F), kind=kind)
    torch.cuda.synchronize()
    k = t[:, 0] if kind == "pair" else t
    host = np.ascontiguousarray(k.contiguous().cpu().numpy())
    assert fs.digest(memoryview(host).cast("B"), threads=16) == c["digest"], name
