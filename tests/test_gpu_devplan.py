"""Device-planned execution (the task queue and per-step planning on the
GPU), its graph-captured form, and the host-planned form give the same,
oracle-exact results."""
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


def _sort(sorter, a, kind, algo, flags, stream=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    torch.cuda.synchronize()
    p = ips.make_params(flags=flags)
    if stream is not None:
        with torch.cuda.stream(stream):
            sorter.sort_(t, algo=algo, params=p, kind=kind, stream=stream)
        stream.synchronize()
    else:
        sorter.sort_(t, algo=algo, params=p, kind=kind)
    torch.cuda.synchronize()
    return t.cpu().numpy()


MODES = [("device", 0), ("host", ips.FLAG_HOST_PLAN), ("graph", ips.FLAG_GRAPH)]


@pytest.mark.parametrize("kind", ["u32", "u64", "f64", "pair", "rec100", "quartet"])
def test_plan_modes_agree(sorter, kind):
    import torch
    stream = torch.cuda.Stream()
    n = {"rec100": 60_000, "quartet": 200_003}.get(kind, 700_001)
    for dist in ("uniform", "twodup", "zero") if kind != "rec100" else ("uniform", "rootdup"):
        a = generate(kind, dist, n, 13)
        algos = ["samplesort"] + (["radix"] if kind not in ("rec100", "quartet") else [])
        for algo in algos:
            for name, fl in MODES:
                log(f"plan mode {name} {kind} {dist} {algo}")
                out = _sort(sorter, a, kind, algo, fl | ips.FLAG_NO_SORTED_CHECK,
                            stream if name == "graph" else None)
                assert_parity(out, a, kind)


def test_graph_replays_repeatedly(sorter):
    # The same call several times in a row on one stream, with eager work in
    # between; every result must be exact.
    import torch
    stream = torch.cuda.Stream()
    a = synth.gen_u64("uniform", 1 << 21, 17)
    ref = np.sort(a)
    for rep in range(3):
        log(f"graph replay {rep}")
        out = _sort(sorter, a, "u64", "samplesort", ips.FLAG_GRAPH, stream)
        assert np.array_equal(out, ref)
        x = torch.arange(1000, device="cuda").sum()       # unrelated eager work
        assert int(x) == 499500


def test_devplan_small_tasks_many_steps(sorter):
    # A tiny LDS tier and few buckets force many partitioning steps, so that
    # the queue is refilled over several rounds of steps.
    a = synth.gen_u64("uniform", 200_003, 19)
    p = ips.make_params(lds_task_max=64, k=4, flags=ips.FLAG_NO_SORTED_CHECK)
    import torch
    t = torch.from_numpy(a).cuda()
    sorter.sort_(t, params=p, kind="u64")
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), np.sort(a))
    st = sorter.stats()
    log(f"steps={st.steps} batches={st.batches} levels={st.levels}")
    assert st.levels >= 8 and st.batches >= 8
