"""The build's check of the device assembly: a 64-bit VALU shift whose amount
is in the last VGPR of an 8-register granule (v7, v15, ..., v127) must not
appear in any kernel.  Such a shift was seen to take its amount from the
register after it, outside the wavefront's allocation, which corrupted the
LDS tier's bin numbers for one wavefront at a time."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build_mod():
    spec = importlib.util.spec_from_file_location("ips_build", os.path.join(ROOT, "paper_2009_13569_amd", "build.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_scanner_flags_granule_end_amounts_only():
    b = _build_mod()
    asm = "\n".join([
        "_ZN3ips4k_one:",
        "\tv_lshrrev_b64 v[42:43], v127, v[42:43]",      # flagged: v127 = 8*15 + 7
        "\tv_lshlrev_b64 v[4:5], v15, v[4:5]",           # flagged
        "\tv_ashrrev_i64 v[4:5], v63, v[4:5]",           # flagged
        "_ZN3ips4k_two:",
        "\tv_lshrrev_b64 v[42:43], v126, v[42:43]",      # other registers are fine
        "\tv_lshlrev_b64 v[34:35], 2, v[10:11]",         # constant amount
        "\tv_lshrrev_b64 v[2:3], s4, v[2:3]",            # scalar amount
        "\tv_alignbit_b32 v1, v2, v3, v127",             # 32-bit funnel shift
    ])
    hits = b.shift64_hazards(asm)
    assert [(fn, ins.split()[2].rstrip(",")) for fn, _, ins in hits] == [
        ("_ZN3ips4k_one", "v127"), ("_ZN3ips4k_one", "v15"), ("_ZN3ips4k_one", "v63")]


def test_last_build_has_no_hazard():
    b = _build_mod()
    if not os.path.isdir(b.BUILD):
        pytest.skip("no build directory: build() has not run here")
    files = b.check_device_asm(b.BUILD)   # raises on a hazard
    if not files:
        pytest.skip("no device assembly kept by the last build")
    assert len(files) == len(b.SOURCES)


def test_counter_build_needs_its_own_output():
    """A build with counter macros never replaces the package's library."""
    build = _build_mod()
    with pytest.raises(ValueError):
        build.build(defines=("IPS_PERM_STATS",))
    assert set(build.COUNTER_DEFINES) == {"IPS_PERM_STATS", "IPS_FUSED_STATS", "IPS_LDS_STATS"}
