"""Autotuner: measures the sort under candidate parameters on the GPU and
writes the tuning table (TUNING_PATH) that Sorter applies to every call.

    python -m paper_2009_13569_amd.tune [--kinds u32 u64 f64 pair rec100 quartet]
                                        [--algos samplesort radix] [--classes 16 18 20 22 24 26 28]
                                        [--batch] [--reps 5] [--out PATH] [--update]

For each element kind, algorithm and size class 2^c it sorts a Uniform
array of 2^c elements (restored before every run, untimed) and times each
run with HIP events on the sort's stream (median of `reps`).  Size classes
beyond a kind's largest benchmark size (2^27 for f64, Pair and Quartet, 2^24
for 100-byte records) are skipped, and that size is a class of its own, so the
table's last entry of a kind is measured at its benchmark size rather than
carried over from a smaller class; radix is not tuned for the kinds it does
not sort (records, Quartets).
Starting from the library defaults it tunes one parameter at a time over a
small candidate list, keeping a change only when it is at least 1% faster,
for two rounds over the list (coordinate descent).  The paper tunes k, the
block size and the base case per machine (Section 6); the parameters here
are the same three plus the pieces and groups of the block permutation.
Workgroup sizes: the block permutation is compiled for 128, 256 and 512
threads (perm_wg), and the LDS-tier threshold (lds_task_max) selects which
of the tier's compiled workgroup shapes take the small tasks.

--batch tunes the batched call on 4096 arrays with log-uniform sizes in
[2^8, 2^22] (one entry for batched calls).  Every run's output is checked
on the device (sorted, same key sum); a failing candidate stops the tuner.

--update keeps the entries of the existing table for the (kind, algorithm,
batched) combinations this run does not tune, so that the table can be
built over several shorter runs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


CANDIDATES = {
    "k": [32, 64, 128, 256],
    "block_bytes": [0, 128, 256, 512, 1024],
    "lds_task_max": [0, "cap/2", "cap/4"],
    "n0": [0, 1024, 4096],
    "piece_blocks": [256, 512, 1024, 2048],
    "perm_groups": [32768, 65536, 131072, 262144],
    "perm_wg": [128, 256, 512],
    "k_root": [64, 128],
}
RADIX_CANDIDATES = {f: v for f, v in CANDIDATES.items() if f not in ("k", "n0", "k_root")}   # radix: 8-bit digits
MAX_LOG2 = {"u32": 28, "u64": 28, "f64": 27, "pair": 27, "rec100": 24, "quartet": 27}
CAP = {"u32": 16384, "u64": 16384, "f64": 16384, "pair": 8192, "rec100": 1024, "quartet": 2048}
NO_RADIX = ("rec100", "quartet")


def _resolve(field, v, kind):
    if isinstance(v, str):
        return CAP[kind] // int(v.split("/")[1])
    return v


def _descend(measure, kind, cands_all=None):
    """Coordinate descent from the defaults; returns (best dict, best ms,
    ms of the defaults)."""
    cands_all = cands_all or CANDIDATES
    cur = {f: 0 for f in cands_all}
    best = measure(cur)
    base = best
    _log(f"    defaults: {best:.3f} ms")
    for rnd in range(2):
        changed = False
        for f, cands in cands_all.items():
            for v in cands:
                v = _resolve(f, v, kind)
                if v == cur[f]:
                    continue
                trial = dict(cur)
                trial[f] = v
                try:
                    ms = measure(trial)
                except ValueError as e:   # rejected by the library: not a candidate
                    _log(f"    {f}={v}: rejected ({e})")
                    continue
                if ms < best * 0.99:
                    _log(f"    {f}={v}: {ms:.3f} ms (was {best:.3f})")
                    cur, best, changed = trial, ms, True
        if not changed:
            break
    return cur, best, base


def _source(kind: str, n: int, seed: int, dev):
    import torch

    import synth
    from synth import device as sd
    if kind == "rec100":
        return torch.from_numpy(synth.gen_rec100("uniform", n, seed)).to(dev)
    if kind == "quartet":
        return torch.from_numpy(synth.gen_quartet("uniform", n, seed)).to(dev)
    return sd.generate(kind, "uniform", n, seed, dev)


def _digest(t, kind):
    """(sorted in key order, sum of the bit patterns) on the device."""
    import torch
    if kind == "rec100":
        b = t[:, :10].to(torch.int64)
        hi = torch.zeros(t.shape[0], dtype=torch.int64, device=t.device)
        for i in range(8):
            hi = hi | (b[:, i] << (56 - 8 * i))
        hi = hi ^ (-(1 << 63))
        lo = (b[:, 8] << 8) | b[:, 9]
        ok = (hi[1:] > hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] >= lo[:-1]))
        return bool(ok.all()), int(t.view(torch.int32).to(torch.int64).sum())
    if kind == "quartet":     # (a, b, c) lexicographic, as signed images of the unsigned words
        t = t.view(torch.int64)
        a, b, c = (t[:, i] ^ (-(1 << 63)) for i in range(3))
        ok = (a[1:] > a[:-1]) | ((a[1:] == a[:-1]) & ((b[1:] > b[:-1]) | ((b[1:] == b[:-1]) & (c[1:] >= c[:-1]))))
        return bool(ok.all()), int(t.sum())
    if kind == "u32":
        v = t.to(torch.int64) & 0xFFFFFFFF
        return bool((v[1:] >= v[:-1]).all()), int(v.sum())
    if kind == "f64":
        return bool((t[1:] >= t[:-1]).all()), int(t.view(torch.int64).sum())
    k = t[:, 0] if kind == "pair" else t
    v = k.view(torch.int64) ^ (-(1 << 63))
    return bool((v[1:] >= v[:-1]).all()), int(t.view(torch.int64).sum())


def tune_single(kind: str, algo: str, log2n: int, reps: int):
    import torch

    import paper_2009_13569_amd as ips

    n = 1 << log2n
    dev = torch.device("cuda:0")
    src = _source(kind, n, 1000 + log2n, dev)
    work = torch.empty_like(src)
    sorter = ips.Sorter(0, tuning=None)
    ref_sum = _digest(src, kind)[1]

    def measure(cfg):
        p = ips.make_params(flags=ips.FLAG_NO_SORTED_CHECK, **{f: int(v) for f, v in cfg.items()})
        try:
            need = ips.workspace_bytes(n, kind, algo, p)
        except ips.IpsError as e:
            raise ValueError(str(e))
        ws = sorter.workspace(need)
        times = []
        for r in range(reps + 1):
            work.copy_(src)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            sorter.sort_(work, algo=algo, params=p, kind=kind, ws=ws)
            e1.record()
            torch.cuda.synchronize()
            if r:
                times.append(e0.elapsed_time(e1))
        ok, s = _digest(work, kind)
        if not ok or s != ref_sum:
            raise RuntimeError("tuner run produced a wrong result")
        times.sort()
        return times[len(times) // 2]

    _log(f"  {kind} {algo} 2^{log2n}")
    return _descend(measure, kind, CANDIDATES if algo == "samplesort" else RADIX_CANDIDATES)


def tune_batch(reps: int, arrays: int = 4096):
    import numpy as np
    import torch

    import paper_2009_13569_amd as ips
    import synth
    import synth.device as sd

    dev = torch.device("cuda:0")
    sizes, dists = synth.batch_layout(arrays, 8, 22, synth.seed_for(4, 0))
    offs = np.zeros(len(sizes), dtype=np.int64)
    offs[1:] = np.cumsum(sizes)[:-1]
    total = int(sizes.sum())
    seeds = synth.stream(synth.seed_for(4, 1), len(sizes))
    src = torch.empty(total, dtype=torch.int64, device=dev)
    for i, (o, m) in enumerate(zip(offs.tolist(), sizes.tolist())):
        src[o:o + m] = sd.gen_u64(dists[i], m, int(seeds[i]), dev)
    ref_sum = int(src.sum())
    work = torch.empty_like(src)
    sorter = ips.Sorter(0, tuning=None)
    offl, szl = offs.tolist(), sizes.tolist()
    segs, nseg = ips.segment_array(offl, szl)
    sign = torch.tensor(-(1 << 63), dtype=torch.int64, device=dev)
    ends = torch.tensor((offs + sizes - 1).tolist(), device=dev)

    def measure(cfg):
        p = ips.make_params(**{f: int(v) for f, v in cfg.items()})
        try:
            need = ips.segments_workspace_bytes(total, segs, nseg, "u64", "samplesort", p)
        except ips.IpsError as e:
            raise ValueError(str(e))
        ws = sorter.workspace(need)
        times = []
        for r in range(reps + 1):
            work.copy_(src)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            sorter.sort_segments_(work, offl, szl, params=p, kind="u64", ws=ws)
            e1.record()
            torch.cuda.synchronize()
            if r:
                times.append(e0.elapsed_time(e1))
        v = work ^ sign
        bad = (v[1:] < v[:-1])
        bad[ends[:-1]] = False   # array boundaries
        if bool(bad.any()) or int(work.sum()) != ref_sum:
            raise RuntimeError("tuner run produced a wrong result")
        times.sort()
        return times[len(times) // 2]

    _log(f"  batch: {arrays} u64 arrays, {total} keys")
    cfg, ms, ms0 = _descend(measure, "u64")
    return cfg, ms, ms0, total


def summary(path: str) -> int:
    """Markdown table of a tuning table's measurements: per element type,
    algorithm and size class (and the batched call) the median time with the
    library defaults and with the tuned parameters."""
    with open(path) as f:
        doc = json.load(f)
    skip = ("kind", "algo", "log2n_min", "log2n_max", "batched")
    print("| kind | algo | n | defaults ms | tuned ms | speedup | tuned parameters |")
    print("|---|---|---|---|---|---|---|")
    for m in doc["measurements"]:
        n = f"2^{m['log2n']}" if "log2n" in m else f"batch of {m.get('batch_keys')} keys"
        d0 = m.get("defaults_ms")
        sp = f"{d0 / m['ms']:.2f}" if d0 else "-"
        params = ", ".join(f"{k}={v}" for k, v in m["params"].items() if k not in skip) or "(defaults)"
        print(f"| {m['kind']} | {m.get('algo', 'samplesort')} | {n} | {d0 if d0 is not None else '-'} | "
              f"{m['ms']} | {sp} | {params} |")
    return 0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--kinds", nargs="+", default=["u32", "u64", "f64", "pair", "rec100", "quartet"])
    ap.add_argument("--algos", nargs="+", default=["samplesort", "radix"])
    ap.add_argument("--classes", nargs="+", type=int, default=[16, 18, 20, 22, 24, 26, 28])
    ap.add_argument("--batch", action="store_true", help="also tune batched calls (4096 arrays)")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=None)
    ap.add_argument("--update", action="store_true", help="keep the existing table's other entries")
    ap.add_argument("--summary", metavar="TABLE", help="print a tuning table's measurements as markdown and exit")
    args = ap.parse_args(argv)
    if args.summary:
        return summary(args.summary)
    sys.path.insert(0, ROOT)
    import torch

    import paper_2009_13569_amd as ips

    out = args.out or ips.TUNING_PATH
    entries, notes = [], []
    t0 = time.time()
    classes = sorted(args.classes)
    for kind in args.kinds:
        for algo in args.algos:
            if algo == "radix" and kind in NO_RADIX:
                continue
            ks = [c for c in classes if c <= MAX_LOG2[kind]]
            if ks and MAX_LOG2[kind] > ks[-1] and MAX_LOG2[kind] <= classes[-1]:
                ks.append(MAX_LOG2[kind])   # the kind's largest benchmark size is measured, not extrapolated
            for i, c in enumerate(ks):
                cfg, ms, ms0 = tune_single(kind, algo, c, args.reps)
                hi = ks[i + 1] - 1 if i + 1 < len(ks) else 40
                e = {"kind": kind, "algo": algo, "log2n_min": c, "log2n_max": hi, "batched": 0}
                e.update({f: int(v) for f, v in cfg.items() if v})
                entries.append(e)
                notes.append({"kind": kind, "algo": algo, "log2n": c, "ms": round(ms, 4),
                              "defaults_ms": round(ms0, 4), "params": e})
                torch.cuda.empty_cache()
    if args.batch:
        cfg, ms, ms0, total = tune_batch(args.reps)
        e = {"kind": "u64", "algo": "samplesort", "log2n_min": 0, "log2n_max": 40, "batched": 1}
        e.update({f: int(v) for f, v in cfg.items() if v})
        entries.append(e)
        notes.append({"kind": "u64", "batch_keys": total, "ms": round(ms, 4), "defaults_ms": round(ms0, 4),
                      "params": e})
    if args.update and os.path.exists(out):
        with open(out) as f:
            old = json.load(f)
        done = {(e["kind"], e["algo"], e["batched"]) for e in entries}
        entries = [e for e in old.get("entries", []) if (e["kind"], e["algo"], e["batched"]) not in done] + entries
        notes = [m for m in old.get("measurements", [])
                 if (m["params"]["kind"], m["params"]["algo"], m["params"]["batched"]) not in done] + notes
    doc = {"device": torch.cuda.get_device_name(0), "seconds": round(time.time() - t0, 1),
           "method": "coordinate descent from the defaults, median of reps HIP-event timings per candidate",
           "entries": entries, "measurements": notes}
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    _log(f"wrote {out} ({len(entries)} entries) in {time.time() - t0:.0f}s")
    print(json.dumps(doc))
    return 0


if __name__ == "__main__":
    sys.exit(main())
