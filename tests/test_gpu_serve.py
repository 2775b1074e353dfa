"""Batched sorting of separate buffers (ips_sort_batch) and the serving
scheduler (ips_serve_trace): every request's result must equal the
oracle's sort of that request alone."""
import numpy as np
import pytest

import paper_2009_13569_amd as ips
import synth
from gpu_util import assert_parity, generate, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sorter():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return ips.Sorter(0)


def _to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(t, kind):
    a = t.cpu().numpy()
    if kind == "u32":
        return a.view(np.uint32)
    if kind in ("u64", "pair"):
        return a.view(np.uint64)
    return a


@pytest.mark.parametrize("kind", ["u32", "u64", "f64", "pair", "rec100"])
def test_sort_batch_separate_buffers(sorter, kind):
    import torch
    sizes = [0, 1, 5, 3000, 20_000, 70_001, 150_000, 16_385]
    if kind == "rec100":
        sizes = [0, 1, 5, 3000, 20_000, 1025]
    inputs = [generate(kind, "uniform", n, 60 + i) for i, n in enumerate(sizes)]
    tens = [_to_dev(a) for a in inputs]
    algos = ["samplesort"] + (["radix"] if kind != "rec100" else [])
    for algo in algos:
        ts = [t.clone() for t in tens]
        log(f"sort_batch {kind} {algo}")
        sorter.sort_batch_(ts, algo=algo, kind=kind)
        torch.cuda.synchronize()
        for a, t in zip(inputs, ts):
            assert_parity(t.cpu().numpy(), a, kind)


def _trace(count, seed, lo=10, hi=18, kinds=("u32", "u64", "f64", "pair")):
    x = synth.stream(seed, 3 * count)
    u = (x[0::3] >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    sizes = np.floor(2.0 ** (lo + u * (hi - lo))).astype(np.int64)
    kind = [kinds[int(v % np.uint64(len(kinds)))] for v in x[1::3]]
    dist = [synth.DISTRIBUTIONS[int(v % np.uint64(len(synth.DISTRIBUTIONS)))] for v in x[2::3]]
    return sizes, kind, dist


@pytest.mark.parametrize("policy", [ips.SERVE_BATCH, ips.SERVE_FIFO])
def test_serve_trace_results_equal_alone(sorter, policy):
    import torch
    sizes, kinds, dists = _trace(48, 71)
    inputs = [generate(k, d, int(n), 80 + i) for i, (k, d, n) in enumerate(zip(kinds, dists, sizes))]
    tens = [_to_dev(a) for a in inputs]
    arrivals = synth.poisson_arrivals(len(tens), 2000.0, 72)
    arrivals -= arrivals[0]
    algos = ["radix" if i % 3 == 0 else "samplesort" for i in range(len(tens))]
    budget = 64 << 20      # forces several rounds
    torch.cuda.synchronize()
    log(f"serve policy={policy} requests={len(tens)} keys={int(sizes.sum())}")
    res, rc = sorter.serve_trace(tens, arrivals, algos=algos, hbm_budget=budget, policy=policy)
    torch.cuda.synchronize()
    assert rc == 0, rc
    for i, (a, t, r) in enumerate(zip(inputs, tens, res)):
        assert r["status"] == 0
        assert r["done_s"] >= r["start_s"] >= arrivals[i] - 1e-9
        assert_parity(t.cpu().numpy(), a, kinds[i])
    nb = len({r["batch"] for r in res})
    if policy == ips.SERVE_FIFO:
        assert nb == len(tens)
        starts = [res[i]["start_s"] for i in np.argsort(arrivals, kind="stable")]
        assert starts == sorted(starts)
    else:
        # continuous batching: some request was admitted while another one
        # (possibly of another element type) was still being sorted
        iv = sorted((r["start_s"], r["done_s"]) for r in res)
        assert any(iv[j][0] < iv[i][1] for i in range(len(iv)) for j in range(i + 1, len(iv))), iv[:5]
    lat = np.array([r["done_s"] - arrivals[i] for i, r in enumerate(res)])
    log(f"  batches={nb} p50={np.percentile(lat, 50) * 1e3:.2f} ms p99={np.percentile(lat, 99) * 1e3:.2f} ms")


def test_serve_rejects_request_over_budget(sorter):
    import torch
    small = [generate("u64", "uniform", 5000, 90 + i) for i in range(3)]
    big = generate("u64", "uniform", 1 << 20, 93)
    inputs = small[:2] + [big] + small[2:]
    tens = [_to_dev(a) for a in inputs]
    res, rc = sorter.serve_trace(tens, [0.0, 0.0, 0.0, 0.0], hbm_budget=4 << 20)
    torch.cuda.synchronize()
    assert rc == -3
    assert [r["status"] for r in res] == [0, 0, -3, 0]
    assert np.array_equal(tens[2].cpu().numpy().view(np.uint64), big)     # untouched
    for i in (0, 1, 3):
        assert_parity(tens[i].cpu().numpy(), inputs[i], "u64")


def test_serve_requests_arriving_mid_flight_equal_alone(sorter):
    """Large requests keep the queues busy while small and large requests of
    every type keep arriving: each result must still equal the oracle's sort
    of that request alone, and later arrivals must be admitted before the
    first large requests finish."""
    import torch
    kinds = ["u64", "u32", "f64", "pair"]
    # the first four need more than one round of steps (two partitioning levels)
    specs = [(kinds[i % 4], 1 << 23 if i < 4 else int(3000 + 977 * i), ("uniform", "twodup", "zipf")[i % 3])
             for i in range(24)]
    inputs = [generate(k, d, n, 300 + i) for i, (k, n, d) in enumerate(specs)]
    tens = [_to_dev(a) for a in inputs]
    arrivals = [0.0] * 4 + [0.0001 * (i + 1) for i in range(20)]
    torch.cuda.synchronize()
    res, rc = sorter.serve_trace(tens, arrivals, hbm_budget=1 << 30, policy=ips.SERVE_BATCH)
    torch.cuda.synchronize()
    assert rc == 0, rc
    for i, (a, t, r) in enumerate(zip(inputs, tens, res)):
        assert r["status"] == 0, (i, r)
        assert_parity(t.cpu().numpy(), a, specs[i][0])
    first_done = min(res[i]["done_s"] for i in range(4))
    assert any(res[i]["start_s"] < first_done for i in range(4, 24)), "no request admitted mid-flight"
