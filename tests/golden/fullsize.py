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
    python tests/golden/fullsize.py --batch

The second command adds the batched workload (4096 u64 arrays of 2^8 to
2^22 keys, the batch benchmark's input): the digest of the concatenation
of every array sorted by the oracle.

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


BATCH = dict(name="batch-4096-u64", arrays=4096, lo_log2=8, hi_log2=22, layout_seed=(4, 0), data_seed=(4, 1))


def batch_inputs():
    """The batched workload: sizes and generators of its 4096 u64 arrays and
    the seed of each (synth.batch_layout and synth.generate_batch's seeds)."""
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import synth
    sizes, dists = synth.batch_layout(BATCH["arrays"], BATCH["lo_log2"], BATCH["hi_log2"],
                                      synth.seed_for(*BATCH["layout_seed"]))
    seeds = synth.stream(synth.seed_for(*BATCH["data_seed"]), len(sizes))
    return sizes, dists, seeds


def _oracle_batch_digest() -> dict:
    """Every array of the batched workload sorted by the oracle, the digest
    of their concatenation (u64 keys)."""
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import oracle
    import synth
    sizes, dists, seeds = batch_inputs()
    out = np.empty(int(sizes.sum()), dtype=np.uint64)
    o = 0
    t0 = time.time()
    for n, d, sd in zip(sizes.tolist(), dists, seeds.tolist()):
        out[o:o + n] = oracle.sort(synth.gen_u64(d, n, int(sd)), "u64")
        o += n
    t1 = time.time()
    return {**BATCH, "keys": int(sizes.sum()), "digest": digest(memoryview(out).cast("B"), threads=8),
            "oracle_s": round(t1 - t0, 1)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("--only", default=None, help="comma-separated case names")
    ap.add_argument("--batch", action="store_true", help="only the batched workload's digest")
    args = ap.parse_args()
    if args.batch:
        row = _oracle_batch_digest()
        with open(OUT) as f:
            doc = json.load(f)
        doc["batch"] = row
        with open(OUT + ".tmp", "w") as f:
            json.dump(doc, f, indent=1)
        os.replace(OUT + ".tmp", OUT)
        print(f"{row['name']}: {row['digest'][:16]}... oracle {row['oracle_s']} s", flush=True)
        return 0
    sel = cases()
    if args.only:
        want = set(args.only.split(","))
        sel = [c for c in sel if case_name(c) in want]
    old, batch = {}, None
    if os.path.exists(OUT):
        with open(OUT) as f:
            prev = json.load(f)
        old, batch = prev.get("cases", {}), prev.get("batch")
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
                           "cases": dict(sorted(res.items())), **({"batch": batch} if batch else {})}, f,
                          indent=1)
            os.replace(OUT + ".tmp", OUT)
    return 0


if __name__ == "__main__":
    sys.exit(main())
