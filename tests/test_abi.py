"""C-ABI checks that need no GPU: the library loads, exports every function
the headers in include/ declare, and rejects bad arguments before any HIP call."""
import ctypes
import glob
import os
import re

import pytest

import paper_2009_13569_amd as ips

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(ips_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert "ips_sort_keys" in names and "ips_sort_pairs" in names
    for name in names:
        assert hasattr(ips.lib(), name), name
    assert set(names) == set(ips.EXPORTS)


def test_abi_version_and_status_strings():
    assert ips.lib().ips_abi_version() == 2
    for code in range(-9, 1):
        assert ips.lib().ips_status_string(code).decode().startswith("IPS_")


def _ws(n, t, algo, params=None):
    out = ctypes.c_size_t(0)
    rc = ips.lib().ips_workspace_bytes(n, t, algo, ctypes.byref(params) if params else None,
                                       ctypes.byref(out))
    return rc, out.value


def test_workspace_validation():
    assert _ws(1 << 20, 2, 0)[0] == 0
    assert _ws(1 << 20, 9, 0)[0] == -1                 # bad element type
    assert _ws(1 << 20, 2, 7)[0] == -1                 # bad algorithm
    assert _ws(1 << 20, 5, 1)[0] == -2                 # radix on 100-byte records
    assert _ws(1, 2, 0) == (0, 0)
    assert _ws(0, 2, 0) == (0, 0)
    assert _ws(1 << 20, 2, 0, ips.make_params(k=3))[0] == -1      # k not a power of two
    assert _ws(1 << 20, 2, 0, ips.make_params(k=512))[0] == -1
    assert _ws(1 << 20, 2, 0, ips.make_params(block_bytes=4096))[0] == -1
    assert _ws(1 << 20, 2, 0, ips.make_params(flags=ips.FLAG_EQ_ON | ips.FLAG_EQ_OFF))[0] == -1
    assert _ws(1 << 20, 2, 0, ips.make_params(lds_task_max=1 << 20))[0] == -1
    assert _ws(1 << 20, 2, 0, ips.make_params(flags=1 << 11))[0] == -1
    rc = ips.lib().ips_workspace_bytes(1 << 20, 2, 0, None, None)
    assert rc == -1


# LDS-tier capacities (elements) of the element types: every queued
# partitioning task holds more than this many elements.
_CAP = {"u32": 16384, "u64": 16384, "f64": 16384, "pair": 8192, "rec100": 1024, "quartet": 2048}


def _ws_bound(n, kind, gbuf=False):
    """The in-place workspace bound (Section 5.1: O(k b) extra memory per
    thread), with the step's budgets of at most 2048 workgroups and 512
    tasks: per workgroup one buffer block per bucket (k b D: the 128 KiB LDS
    budget, or k = 512 buckets of 2 KiB blocks with the buffers in the
    workspace) plus O(k) counters; per task one spill area of the same size,
    the step record (splitters, tree, start table) and O(k) bucket, piece and
    child entries.  Two terms grow with n, both by well under 0.1 % of the
    data: the task queue (32 bytes per cap elements: every queued task holds
    more than cap) and the permutation's pointer pieces (52 bytes per 1024
    blocks of at least 256 bytes)."""
    D = ips.ELEM_BYTES[kind]
    kbd = 512 * 2048 if gbuf else 128 << 10
    per_wg = kbd + 512 * 24 + 16
    per_task = kbd + 24 * 1024 + 512 * 400
    return (2048 * per_wg + 512 * per_task + 40 * (n // _CAP[kind] + 512) + 64 * (n * D // (256 << 10))
            + (1 << 20))


@pytest.mark.parametrize("kind", ["u32", "u64", "f64", "pair", "rec100", "quartet"])
def test_workspace_in_place_bound(kind):
    D = ips.ELEM_BYTES[kind]
    top = {"rec100": 31, "quartet": 33}.get(kind, 34)          # n below 2^31 blocks
    for lg in range(10, top + 1):
        n = 1 << lg
        for algo in ("samplesort", "radix"):
            if algo == "radix" and kind in ("rec100", "quartet"):
                continue
            ws = ips.workspace_bytes(n, kind, algo)
            assert ws <= _ws_bound(n, kind), (kind, algo, lg, ws)
            # below the data itself from 2^16 elements (samplesort) and 2^20
            # (radix: 256 buckets per step whatever the task size)
            if lg >= (16 if algo == "samplesort" else 20):
                assert ws < n * D, (kind, algo, lg, ws / (n * D))
        gb = ips.workspace_bytes(n, kind, params=ips.make_params(flags=ips.FLAG_GLOBAL_BUFFERS))
        assert gb <= _ws_bound(n, kind, gbuf=True), (kind, lg, gb)
    # beyond the budgets only the two small terms grow (and the list of next
    # tasks of one step, up to 32 bytes x 512 tasks x 512 buckets)
    w28 = ips.workspace_bytes(1 << 28, kind)
    w34 = ips.workspace_bytes(1 << top, kind)
    dn = (1 << top) - (1 << 28)
    assert w34 - w28 <= 40 * (dn // _CAP[kind]) + 64 * (dn * D // (256 << 10)) + 32 * 512 * 512, (w28, w34)


def test_sort_rejects_bad_arguments_before_hip():
    L = ips.lib()
    fake = ctypes.c_void_p(0x1000)
    # null context
    assert L.ips_sort_keys(None, fake, 10, 2, 0, fake, 1 << 20, None, None) == -1
    # wrong type codes for each entry point
    assert L.ips_sort_keys(None, fake, 10, 4, 0, fake, 1 << 20, None, None) == -1
    assert L.ips_sort_pairs(None, fake, 10, 2, 0, fake, 1 << 20, None, None) == -1
    assert L.ips_sort_keys_noalloc(None, fake, 10, 2, 0, None, None) == -1


def test_ctx_create_null_out():
    assert ips.lib().ips_ctx_create(None, 0) == -1
    assert ips.lib().ips_ctx_destroy(None) == 0


def _segws(n_total, offs, sizes, t=2, algo=0):
    segs, nseg = ips.segment_array(offs, sizes)
    out = ctypes.c_size_t(0)
    rc = ips.lib().ips_segments_workspace_bytes(n_total, segs, nseg, t, algo, None, ctypes.byref(out))
    return rc, out.value


def test_segments_validation():
    n = 1 << 20
    rc, ws = _segws(n, [0, 1000, 500000], [1000, 400000, 524288])
    base = _ws(1000 + 400000 + 524288, 2, 0)[1]       # planned for the elements sorted
    assert rc == 0 and base <= ws <= base + 16384     # plus the per-segment order flags
    assert _segws(n, [0, 999], [1000, 10])[0] == -1            # overlap
    assert _segws(n, [n - 10], [11])[0] == -1                  # past the end
    assert _segws(n, [1 << 63], [1 << 63])[0] == -1            # offset + n overflows
    assert _segws(n, [5, 5], [0, 10])[0] == 0                  # empty segments never overlap
    assert _segws(n, [0], [n], t=5, algo=1)[0] == -2           # radix on 100-byte records
    # the radix path needs room for the key ranges of the partitioned segments
    assert _segws(n, [0], [n], algo=1)[1] > _ws(n, 2, 1)[1]
    # level-1-only mode is meaningless for many arrays: rejected before any HIP call
    L = ips.lib()
    segs, nseg = ips.segment_array([0], [100])
    p = ips.make_params(flags=ips.FLAG_LEVEL1_ONLY)
    fake = ctypes.c_void_p(0x1000)
    assert L.ips_sort_segments(ctypes.c_void_p(0x10), fake, 100, 2, 0, segs, nseg, fake, 1 << 20,
                               ctypes.byref(p), None) == -1
    assert L.ips_sort_segments(None, fake, 100, 2, 0, segs, nseg, fake, 1 << 20, None, None) == -1


def test_exported_symbols_are_exactly_the_declared_ones():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", ips.LIB_PATH], capture_output=True, text=True).stdout
    exported = sorted({ln.split()[-1] for ln in out.splitlines() if " T ips_" in ln})
    assert exported == _declared()


def _batchws(ptrs, ns, t=2, algo=0):
    cnt = len(ptrs)
    P = (ctypes.c_void_p * max(1, cnt))(*ptrs)
    N = (ctypes.c_uint64 * max(1, cnt))(*ns)
    out = ctypes.c_size_t(0)
    rc = ips.lib().ips_batch_workspace_bytes(P, N, cnt, t, algo, None, ctypes.byref(out))
    return rc, out.value


def test_batch_validation():
    base = 1 << 40
    rc, ws = _batchws([base, base + 8 * 5000, base + (1 << 30)], [5000, 100000, 20000])
    assert rc == 0 and ws > 0
    assert _batchws([base, base + 8 * 4999], [5000, 10])[0] == -1        # overlap
    assert _batchws([base + 4], [100])[0] == -4                            # u64 misaligned
    assert _batchws([0], [100])[0] == -1                                   # null with n > 0
    assert _batchws([0, base], [0, 100])[0] == 0                           # empty entries are ignored
    assert _batchws([base + 4], [100], t=1)[0] == 0                        # u32 needs 4 bytes
    assert _batchws([base], [100], t=5, algo=1)[0] == -2                   # radix on records
    # records at addresses that differ by a non-multiple of 100 bytes form
    # separate groups: each is planned on its own
    r1 = _batchws([base, base + 2_000_064], [20000, 20000], t=5)
    assert r1[0] == 0 and r1[1] > 0
    assert _batchws([base, base + 1_999_964], [20000, 20000], t=5)[0] == -1   # overlap across groups


def _requests(specs):
    arr = (ips.Request * max(1, len(specs)))()
    for i, (ptr, n, t, algo, at) in enumerate(specs):
        arr[i].d_data, arr[i].n, arr[i].elem_type, arr[i].algo, arr[i].arrival_s = ptr, n, t, algo, at
    return arr


def test_serve_validation_and_rejection_without_device():
    L = ips.lib()
    base = 1 << 40
    cfg = ips.ServeConfig(1 << 20, ips.SERVE_BATCH, 0)
    reqs = _requests([(base, 1 << 20, 2, 0, 0.0), (base + (1 << 24), 1 << 21, 1, 0, 0.001)])
    out = ctypes.c_size_t(0)
    assert L.ips_serve_workspace_bytes(reqs, 2, ctypes.byref(cfg), None, ctypes.byref(out)) == 0
    assert out.value > 0
    bad = ips.ServeConfig(1 << 20, 7, 0)
    fake_ctx = ctypes.c_void_p(0x10)
    assert L.ips_serve_trace(fake_ctx, reqs, 2, ctypes.byref(bad), None, 0, None, None) == -1
    assert L.ips_serve_trace(None, reqs, 2, ctypes.byref(cfg), None, 0, None, None) == -1
    neg = _requests([(base, 10, 2, 0, -1.0)])
    assert L.ips_serve_trace(fake_ctx, neg, 1, ctypes.byref(cfg), None, 0, None, None) == -1
    # Both requests exceed the 1 MiB budget alone: the admission step rejects
    # them without ever calling a sort (so no device is touched).
    rc = L.ips_serve_trace(fake_ctx, reqs, 2, ctypes.byref(cfg), ctypes.c_void_p(0x1000), 1 << 30, None, None)
    assert rc == -3
    assert [reqs[i].status for i in range(2)] == [-3, -3]
    assert reqs[1].done_s >= 0.001                  # rejected only once it had arrived


def test_tuned_params_lookup():
    table, cnt = ips.tune_table([
        {"kind": "u64", "log2n_min": 16, "log2n_max": 19, "k": 64, "block_bytes": 512},
        {"kind": "u64", "log2n_min": 20, "log2n_max": 40, "k": 128, "piece_blocks": 2048},
        {"kind": "u64", "log2n_min": 20, "log2n_max": 40, "k": 32},                       # shadowed
        {"kind": "u64", "log2n_min": 0, "log2n_max": 40, "batched": 1, "perm_groups": 65536},
        {"kind": "u32", "algo": "radix", "log2n_min": 0, "log2n_max": 40, "n0": 4096},
    ])
    L = ips.lib()
    out = ips.Params()
    # first matching entry; untouched fields stay zero
    p = ips.tuned_params(table, cnt, (1 << 20) + 5, "u64")
    assert (p.k, p.block_bytes, p.piece_blocks, p.perm_groups) == (128, 0, 2048, 0)
    p = ips.tuned_params(table, cnt, 1 << 17, "u64")
    assert (p.k, p.block_bytes) == (64, 512)
    # no entry below 2^16 for single calls
    assert L.ips_tuned_params(table, cnt, 1000, 2, 0, 0, None, ctypes.byref(out)) == 0
    assert out.k == 0
    # caller's fields and flags are kept
    base = ips.make_params(k=16, flags=ips.FLAG_NO_SORTED_CHECK, seed=7)
    p = ips.tuned_params(table, cnt, 1 << 24, "u64", base=base)
    assert (p.k, p.piece_blocks, p.flags, p.seed) == (16, 2048, ips.FLAG_NO_SORTED_CHECK, 7)
    # batched calls and other algorithms have entries of their own
    p = ips.tuned_params(table, cnt, 1 << 24, "u64", batched=True)
    assert (p.k, p.perm_groups) == (0, 65536)
    p = ips.tuned_params(table, cnt, 1 << 24, "u32", "radix")
    assert p.n0 == 4096
    assert ips.tuned_params(table, cnt, 1 << 24, "u32").n0 == 0
    # errors
    assert L.ips_tuned_params(table, cnt, 1 << 20, 2, 0, 0, None, None) == -1
    assert L.ips_tuned_params(None, 1, 1 << 20, 2, 0, 0, None, ctypes.byref(out)) == -1
    bad, bc = ips.tune_table([{"kind": "u64", "log2n_min": 30, "log2n_max": 20}])
    assert L.ips_tuned_params(bad, bc, 1 << 20, 2, 0, 0, None, ctypes.byref(out)) == -1
    # an empty table matches nothing
    assert L.ips_tuned_params(None, 0, 1 << 20, 2, 0, 0, None, ctypes.byref(out)) == 0


def test_tuning_file_entries_are_valid():
    """The committed tuning table (if any) only names valid kinds and fields,
    and every entry's parameters are accepted by the library."""
    entries = ips.load_tuning()
    table, cnt = ips.tune_table(entries)
    for e in entries:
        assert set(e) <= {"kind", "algo", "log2n_min", "log2n_max", "batched", *ips.TUNE_FIELDS}
        n = 1 << max(int(e["log2n_min"]), 1)
        p = ips.tuned_params(table, cnt, n, e["kind"], e.get("algo", "samplesort"), bool(e.get("batched", 0)))
        assert ips.workspace_bytes(n, e["kind"], e.get("algo", "samplesort"), p) > 0


def test_fused_flag_validation():
    """IPS_FLAG_FUSED is a radix option of device-planned steps: rejected
    with samplesort, host planning, the root-step-only mode and global
    buffers, and for more elements than its 31-bit positions hold."""
    F = ips.FLAG_FUSED
    assert ips.workspace_bytes(1 << 20, "u64", "radix", ips.make_params(flags=F)) > 0
    assert ips.workspace_bytes(1 << 20, "pair", "radix", ips.make_params(flags=F)) > 0
    for kind, algo, extra in (("u64", "samplesort", 0), ("u64", "radix", ips.FLAG_HOST_PLAN),
                              ("u64", "radix", ips.FLAG_LEVEL1_ONLY), ("u64", "radix", ips.FLAG_GLOBAL_BUFFERS),
                              ("rec100", "radix", 0)):
        with pytest.raises(ips.IpsError) as e:
            ips.workspace_bytes(1 << 20, kind, algo, ips.make_params(flags=F | extra))
        assert e.value.code == -2, (kind, algo, extra)
    with pytest.raises(ips.IpsError) as e:
        ips.workspace_bytes((1 << 31) - (1 << 16) + 1, "u32", "radix", ips.make_params(flags=F))
    assert e.value.code == -5
    with pytest.raises(ips.IpsError) as e:
        ips.workspace_bytes(1000, "u64", "radix", ips.make_params(flags=0x800))
    assert e.value.code == -1


def test_insertion_base_validation():
    I = ips.FLAG_INSERTION_BASE
    assert ips.workspace_bytes(1 << 20, "u64", params=ips.make_params(n0=16, flags=I)) > 0
    with pytest.raises(ips.IpsError) as e:
        ips.workspace_bytes(1 << 20, "u64", params=ips.make_params(flags=I))     # n0 = 0
    assert e.value.code == -1
    with pytest.raises(ips.IpsError) as e:
        ips.workspace_bytes(1 << 20, "u64", "radix", ips.make_params(n0=16, flags=I))
    assert e.value.code == -2


def test_probe_rejects_bad_arguments_before_any_hip_call():
    f = ips.lib().ips_probe_memory
    ms = ctypes.c_float(0.0)
    a, b, t = 0x10000, 0x20000, 0x30000   # never dereferenced: every case fails validation
    bad = [
        (7, a, b, 1 << 20, 0, None, 0, 0, 1),          # mode
        (0, None, b, 1 << 20, 0, None, 0, 0, 1),       # null src
        (0, a, b, 1 << 20 | 8, 0, None, 0, 0, 1),      # bytes not a multiple of 16
        (0, a + 8, b, 1 << 20, 0, None, 0, 0, 1),      # misaligned
        (0, a, b, 1 << 20, 0, None, 0, 0, 0),          # reps
        (3, a, b, 1 << 20, 384, None, 0, 0, 1),        # block size
        (3, a, b, 3 << 20, 512, None, 0, 0, 1),        # block count not a power of two
        (4, a, b, 1 << 20, 512, None, 4096, 64, 1),    # no table
        (4, a, b, 1 << 20, 512, t, 3000, 64, 1),       # table size
        (4, a, b, 1 << 20, 512, t, 4096, 0, 1),        # groups
        (4, a, b, 1 << 20, 512, t, 4096, 4096, 1),     # fewer blocks than groups
    ]
    for mode, s, d, nbytes, bb, tab, tw, g, reps in bad:
        assert f(mode, s, d, nbytes, bb, tab, tw, g, reps, None, ctypes.byref(ms)) == -1, (mode, nbytes, bb, tw, g)
    assert f(0, a, b, 1 << 20, 0, None, 0, 0, 1, None, None) == -1   # null result
