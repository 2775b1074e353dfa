"""Oracle digests of the full-size benchmark inputs.

The configurations measured at full size (2^28 u64 and u32 keys of every
generator, 2^27 doubles and Pair records, 2^24 100-byte records) are far too
large to store sorted outputs for.  This module defines those inputs (the
generator, size and seed of each; also 2^27 Quartets), a digest of a sorted key sequence, and a
writer that sorts every input with the CPU oracle and stores the digests in
``fullsize_digests.json`` next to this file.  The GPU tests generate the same
inputs, sort them with the HIP library and compare digests, so every stored
value comes from the oracle alone.

Writer (CPU only, about 15 minutes on 8 cores):

    python tests/golden/fullsize.py --jobs 4

The digest is SHA-256 (FIPS 180-4) over the concatenation of the byte count
(8 bytes, little endian) and the SHA-256 of each consecutive 64 MiB chunk of
the key bytes; the chunks are hashed in parallel threads.  Key bytes are the
array itself for u32, u64 and f64 (f64 by its bit pattern), column 0 (the
u64 key) for Pair, bytes 0..9 of every record for 100-byte records, and the
key words a, b, c (columns 0..2) of every Quartet.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "fullsize_digests.json")
CHUNK = 64 << 20

DISTS = ("uniform", "exponential", "rootdup", "twodup", "eightdup", "almostsorted", "sorted",
         "reversesorted", "zero", "zipf")


def cases() -> list[dict]:
    """Every full-size input: (kind, dist, log2n, config, array index).  The
    seed of a case is synth.seed_for(config, array) with array = the
    generator's index in DISTS, as the sweep benchmark uses."""
    out = [dict(kind=k, dist=d, log2n=28, config=2, array=DISTS.index(d))
           for k in ("u64", "u32") for d in DISTS]
    out += [dict(kind="f64", dist=d, log2n=27, config=3, array=DISTS.index(d)) for d in ("uniform", "exponential")]
    out += [dict(kind="pair", dist=d, log2n=27, config=3, array=DISTS.index(d)) for d in ("uniform", "rootdup")]
    out += [dict(kind="rec100", dist=d, log2n=24, config=3, array=DISTS.index(d)) for d in ("uniform", "rootdup")]
    out += [dict(kind="quartet", dist="uniform", log2n=27, config=3, array=DISTS.index("uniform"))]
    return out


def case_name(c: dict) -> str:
    return f"{c['kind']}-{c['dist']}-2p{c['log2n']}"


def generate(c: dict) -> np.ndarray:
    """The case's input on the host (numpy)."""
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import synth
    n = 1 << c["log2n"]
    seed = synth.seed_for(c["config"], c["array"])
    return synth.generate(c["kind"], c["dist"], n, seed)


def key_bytes(a: np.ndarray, kind: str) -> memoryview:
    """The key bytes of a (sorted) array, as described in the module doc."""
    if kind in ("u32", "u64", "f64"):
        return memoryview(np.ascontiguousarray(a)).cast("B")
    if kind == "pair":
        return memoryview(np.ascontiguousarray(a[:, 0])).cast("B")
    if kind == "rec100":
        return memoryview(np.ascontiguousarray(a[:, :10])).cast("B")
    if kind == "quartet":
        return memoryview(np.ascontiguousarray(a[:, :3])).cast("B")
    raise ValueError(kind)


def digest(buf: memoryview, threads: int = 8) -> str:
    mv = memoryview(buf).cast("B")
    n = mv.nbytes
    parts = [mv[o:o + CHUNK] for o in range(0, n, CHUNK)]
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        hs = list(ex.map(lambda p: hashlib.sha256(p).digest(), parts))
    h = hashlib.sha256()
    h.update(n.to_bytes(8, "little"))
    for x in hs:
        h.update(x)
    return h.hexdigest()


def _oracle_digest(c: dict) -> tuple[str, dict]:
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import oracle
    t0 = time.time()
    a = generate(c)
    t1 = time.time()
    s = oracle.sort(a, c["kind"])
    t2 = time.time()
    d = digest(key_bytes(s, c["kind"]), threads=2)
    return case_name(c), {**c, "digest": d, "gen_s": round(t1 - t0, 1), "oracle_s": round(t2 - t1, 1)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("--only", default=None, help="comma-separated case names")
    args = ap.parse_args()
    sel = cases()
    if args.only:
        want = set(args.only.split(","))
        sel = [c for c in sel if case_name(c) in want]
    old = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            old = json.load(f).get("cases", {})
    res = dict(old)
    # largest first so that the pool's tail is short
    sel.sort(key=lambda c: -(c["log2n"] + (1 if c["kind"] in ("u64", "pair", "f64") else 0)))
    with cf.ProcessPoolExecutor(max_workers=args.jobs) as ex:
        for name, row in ex.map(_oracle_digest, sel):
            res[name] = row
            print(f"{name}: {row['digest'][:16]}... oracle {row['oracle_s']} s", flush=True)
            with open(OUT + ".tmp", "w") as f:
                json.dump({"writer": "python tests/golden/fullsize.py --jobs 4",
                           "digest": "sha256(le64(bytes) || sha256(chunk_0) || ... ), 64 MiB chunks of the "
                                     "sorted key bytes",
                           "cases": dict(sorted(res.items()))}, f, indent=1)
            os.replace(OUT + ".tmp", OUT)
    return 0


if __name__ == "__main__":
    sys.exit(main())
