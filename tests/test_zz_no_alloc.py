"""The allocation-free entry point (ips_sort_keys_noalloc, static per-GPU
scratch) against ips_sort_keys (caller workspace) on the same inputs: bit
identical outputs on two calls in a row, the second smaller than the first,
for every key type and both algorithms; oversized calls and flags that
would create HIP objects are rejected and leave the keys untouched."""
import numpy as np
import pytest

import paper_2009_13569_amd as ips
from gpu_util import generate, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sorter():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return ips.Sorter(0)


def _pair_of_sorts(sorter, a, kind, algo):
    import torch
    t_ref = torch.from_numpy(a).cuda()
    t_na = t_ref.clone()
    sorter.sort_(t_ref, algo=algo, kind=kind)
    sorter.sort_noalloc_(t_na, algo=algo, kind=kind)
    torch.cuda.synchronize()
    return t_ref.cpu().numpy(), t_na.cpu().numpy()


@pytest.mark.parametrize("kind,algo,n1,n2", [
    ("u64", "samplesort", 3_000_017, 70_001),
    ("u64", "radix", 2_000_003, 65_537),
    ("u32", "samplesort", 5_000_011, 1_001),
    ("u32", "radix", 4_000_037, 300_007),
    ("f64", "samplesort", 2_500_009, 16_385),
])
def test_noalloc_matches_workspace_entry_point(sorter, kind, algo, n1, n2):
    for i, (n, dist) in enumerate(((n1, "uniform"), (n2, "twodup"))):
        a = generate(kind, dist if kind != "f64" else "uniform", n, 900 + i)
        log(f"noalloc {kind} {algo} call {i + 1}: n={n}")
        ref, got = _pair_of_sorts(sorter, a, kind, algo)
        assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), (kind, algo, n)
        assert np.array_equal(ref.view(np.uint8), np.sort(a).view(np.uint8)) or kind == "f64"


def test_noalloc_rejects_oversized_and_object_creating_calls(sorter):
    import torch
    n = 1 << 25                                     # workspace above the 64 MiB scratch
    assert ips.workspace_bytes(n, "u64") > 64 << 20
    t = torch.arange(n, 0, -1, dtype=torch.int64, device="cuda")
    before = t.clone()
    with pytest.raises(ips.IpsError) as e:
        sorter.sort_noalloc_(t, kind="u64")
    assert e.value.code == -9
    with pytest.raises(ips.IpsError) as e:
        sorter.sort_noalloc_(t[:1000], kind="u64", params=ips.make_params(flags=ips.FLAG_PROFILE))
    assert e.value.code == -1
    torch.cuda.synchronize()
    assert torch.equal(t, before)
