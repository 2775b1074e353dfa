"""Memory-system probes (include/ips_probe.h) on the GPU: each moves what it
states (a copy equals its source, the block probe writes a permutation of
the source's blocks, the chain probe makes the stated number of atomic
updates), so the bandwidth figures derived from them count real bytes."""
import pytest
import torch

import paper_2009_13569_amd as ips

pytestmark = pytest.mark.gpu


def _src(nbytes):
    g = torch.Generator(device="cuda").manual_seed(5)
    return torch.randint(-2**62, 2**62, (nbytes // 8,), generator=g, device="cuda", dtype=torch.int64)


def test_copy_read_write():
    src = _src(1 << 22)
    dst = torch.zeros_like(src)
    assert ips.probe_memory("copy", src, dst, reps=2) > 0
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    assert ips.probe_memory("read", src, dst, reps=2) > 0
    assert ips.probe_memory("write", src, dst, reps=2) > 0


@pytest.mark.parametrize("bb", [256, 512, 1024, 2048])
def test_blocks_move_a_permutation_of_blocks(bb):
    nbytes = 1 << 22
    src = _src(nbytes)
    dst = torch.zeros_like(src)
    assert ips.probe_memory("blocks", src, dst, block_bytes=bb, reps=1) > 0
    torch.cuda.synchronize()
    per = bb // 8
    a = src.view(-1, per)
    b = dst.view(-1, per)
    # every destination block is some source block, each source block used once
    ka = torch.sort(a[:, 0] ^ (a[:, -1] * 3)).values
    kb = torch.sort(b[:, 0] ^ (b[:, -1] * 3)).values
    assert torch.equal(ka, kb)
    assert torch.equal(torch.sort(a.sum(1)).values, torch.sort(b.sum(1)).values)


@pytest.mark.parametrize("bb,groups", [(512, 1024), (1024, 300)])
def test_chain_counts_its_atomics(bb, groups):
    nbytes = 1 << 22
    src = _src(nbytes)
    dst = torch.zeros_like(src)
    table = torch.zeros(4096, dtype=torch.int64, device="cuda")
    reps = 3
    assert ips.probe_memory("chain", src, dst, block_bytes=bb, table=table, groups=groups, reps=reps) > 0
    torch.cuda.synchronize()
    iters = nbytes // (groups * bb)
    assert int(table.sum()) == (reps + 1) * groups * iters
