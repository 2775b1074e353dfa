"""C-ABI checks that need no GPU: the library loads, exports every function
include/ips.h declares, and rejects bad arguments before any HIP call."""
import ctypes
import os
import re

import pytest

import paper_2009_13569_amd as ips

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ips.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ips_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert "ips_sort_keys" in names and "ips_sort_pairs" in names
    for name in names:
        assert hasattr(ips.lib(), name), name
    assert set(names) == set(ips.EXPORTS)


def test_abi_version_and_status_strings():
    assert ips.lib().ips_abi_version() == 1
    for code in range(-8, 1):
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
    assert _ws(1 << 20, 2, 0, ips.make_params(flags=1 << 10))[0] == -1
    rc = ips.lib().ips_workspace_bytes(1 << 20, 2, 0, None, None)
    assert rc == -1


@pytest.mark.parametrize("kind", ["u32", "u64", "f64", "pair", "rec100"])
def test_workspace_is_small_relative_to_data(kind):
    # O(k b) per workgroup of a batch: well below the data for large arrays.
    for n, frac in ((1 << 24, 1.0), (1 << 28, 0.35)):
        ws = ips.workspace_bytes(n, kind)
        assert ws < n * ips.ELEM_BYTES[kind] * frac, (n, ws)
    n = 1 << 24
    gb = ips.workspace_bytes(n, kind, params=ips.make_params(flags=ips.FLAG_GLOBAL_BUFFERS))
    assert gb > 0


def test_sort_rejects_bad_arguments_before_hip():
    L = ips.lib()
    fake = ctypes.c_void_p(0x1000)
    # null context
    assert L.ips_sort_keys(None, fake, 10, 2, 0, fake, 1 << 20, None, None) == -1
    # wrong type codes for each entry point
    assert L.ips_sort_keys(None, fake, 10, 4, 0, fake, 1 << 20, None, None) == -1
    assert L.ips_sort_pairs(None, fake, 10, 2, 0, fake, 1 << 20, None, None) == -1


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
    assert rc == 0 and ws >= _ws(n, 2, 0)[1]
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
