"""The out-of-place ablation (ips_sort_oop: super scalar samplesort's
partitioning step with the in-place path's sampling, tree and LDS-tier base
case) against the oracle, for every element type, one and several levels
(the result returning from the second array after an odd number of levels),
equality buckets (two-byte oracle entries), forced deep recursion, and the
2^28 u64 Uniform input against the oracle's digest."""
import json

import numpy as np
import pytest

import paper_2009_13569_amd as ips
from golden import fullsize as fs
from gpu_util import assert_parity, generate, log

pytestmark = pytest.mark.gpu

KINDS = ["u32", "u64", "f64", "pair", "rec100"]


@pytest.fixture(scope="module")
def sorter():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return ips.Sorter(0, tuning=None)


def _oop(sorter, a, kind, params=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    sorter.sort_oop_(t, params=params, kind=kind)
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("kind", KINDS)
def test_oop_matches_oracle(sorter, kind):
    cap = ips.LDS_CAP[kind]
    for n in (0, 1, 2, 1000, cap, cap + 1, 3 * cap + 17, 70_001, 1_000_003 if kind != "rec100" else 200_003):
        for dist in ("uniform", "rootdup", "twodup", "zero"):
            a = generate(kind, dist, n, 500 + n)
            log(f"oop {kind} {dist} n={n}")
            assert_parity(_oop(sorter, a, kind), a, kind)
            st = sorter.stats()
            if n > cap and dist == "uniform":
                assert st.levels >= 1


@pytest.mark.parametrize("kind", ["u64", "pair"])
def test_oop_forced_recursion(sorter, kind):
    """Small LDS tier and few buckets: many levels, both parities."""
    p = ips.make_params(k=4, lds_task_max=64)
    for n in (65, 1000, 20_011):
        for dist in ("uniform", "eightdup"):
            a = generate(kind, dist, n, 700 + n)
            log(f"oop forced {kind} {dist} n={n}")
            assert_parity(_oop(sorter, a, kind, p), a, kind)
            if n > 20_000 and dist == "uniform":   # 4 buckets per step: several levels of both parities
                assert sorter.stats().levels >= 3


def test_oop_fullsize_digest(sorter):
    import torch
    import synth
    import synth.device as sd
    with open(fs.OUT) as f:
        gold = json.load(f)["cases"]["u64-uniform-2p28"]
    t = sd.generate("u64", "uniform", 1 << 28, synth.seed_for(gold["config"], gold["array"]), "cuda")
    log("oop u64 uniform 2^28")
    sorter.sort_oop_(t, kind="u64")
    torch.cuda.synchronize()
    host = np.ascontiguousarray(t.cpu().numpy())
    assert fs.digest(memoryview(host).cast("B"), threads=16) == gold["digest"]
