"""Builds libips.so (the gfx950 HIP library behind include/ips.h) in-tree.

Every HIP translation unit is compiled with hipcc for gfx950 and linked
into paper_2009_13569_amd/libips.so.  Packed FP32 instructions are disabled
for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libips.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["ips_host.hip", "ips_serve.hip", "ips_kern_common.hip", "ips_kern_u32.hip", "ips_kern_u64.hip",
           "ips_kern_f64.hip", "ips_kern_pair.hip", "ips_kern_rec100.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-mcode-object-version=5", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def _hip_stub() -> str:
    """An empty shared object whose soname is plain `libamdhip64.so`.

    Linking against it records the HIP runtime dependency under that name,
    so a process that already holds a HIP runtime under this name (PyTorch's
    bundled one) shares it with libips.so instead of loading a second
    runtime; elsewhere the name resolves to /opt/rocm/lib through the rpath.
    """
    d = os.path.join(BUILD, "stub")
    os.makedirs(d, exist_ok=True)
    src = os.path.join(d, "stub.c")
    with open(src, "w") as f:
        f.write("/* placeholder: symbols come from the HIP runtime at load time */\n")
    lib = os.path.join(d, "libamdhip64.so")
    subprocess.check_call(["gcc", "-shared", "-fPIC", "-Wl,-soname,libamdhip64.so", "-o", lib, src])
    return d


def build(verbose: bool = False) -> str:
    """Compile all sources and link libips.so; always rebuilds."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    stub = _hip_stub()
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", f"-L{stub}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
