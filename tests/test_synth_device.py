"""The torch generators of synth.device reproduce synth's numpy generators
(run on the CPU device here; the same code runs on the GPU in the batched
and serving workloads)."""
import numpy as np
import pytest
import torch

import synth
import synth.device as sd


@pytest.mark.parametrize("kind", ["u32", "u64", "f64", "pair"])
def test_device_generators_match_host(kind):
    for dist in synth.DISTRIBUTIONS:
        for n in (0, 1, 7, 1000, 65537):
            ref = synth.generate(kind, dist, n, 12345)
            got = sd.generate(kind, dist, n, 12345, "cpu").numpy()
            if kind == "u32":
                got = got.view(np.uint32)
            elif kind in ("u64", "pair"):
                got = got.view(np.uint64)
            if kind == "f64" and dist == "exponential":
                assert np.allclose(got, ref, rtol=1e-15, atol=0)
            else:
                assert np.array_equal(got, ref), (kind, dist, n)


def test_batch_layout_shape():
    sizes, dists = synth.batch_layout(4096, 8, 22, synth.seed_for(4, 0))
    assert sizes.min() >= 256 and sizes.max() < (1 << 22)
    assert set(dists) == {"uniform", "twodup", "almostsorted"}
    # log-uniform: the median size is near 2^15
    assert 2 ** 14 < np.median(sizes) < 2 ** 16


def test_poisson_arrivals_rate():
    t = synth.poisson_arrivals(20000, 100.0, 5)
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] / 20000 - 0.01) < 0.0005
    assert torch.is_tensor(sd.stream(1, 3, "cpu"))
