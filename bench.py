#!/usr/bin/env python3
"""Throughput of the in-place samplesort (IPS4o) hot path on one MI355X.

One step sorts n = 2^28 uint64 keys drawn uniformly from [0, 2^64) (the
paper's Uniform distribution, synthetic, SplitMix64-seeded) in place in HBM.
K pristine copies of the input are made before the timed region, so the
timed region is exactly K back-to-back sorts bracketed by device
synchronizations.  Every launch is timed with HIP events on the sort's
stream (library profiling flag) to give per-level and per-kernel HBM
rates; the dominant kernel's rate is reported against the 8 TB/s peak.
The CPU baseline is the oracle's single-threaded merge sort on a 2^24-key
sample of the same distribution.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--kind", default="u64", choices=["u32", "u64"])
    ap.add_argument("--dist", default="uniform")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--no-radix", action="store_true", help="skip the radix-path measurement")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the sort runs on a single "
              f"MI355X and has no multi-GPU path.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2009_13569_amd as ips
    import synth

    n = 1 << args.log2n
    kind = args.kind
    D = ips.ELEM_BYTES[kind]
    log(f"generating {kind} {args.dist} n=2^{args.log2n}")
    t0 = time.time()
    host = synth.generate(kind, args.dist, n, synth.seed_for(2, 0))
    log(f"  {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    pristine = torch.from_numpy(host).to(dev)
    copies = [pristine.clone() for _ in range(args.steps)]
    torch.cuda.synchronize()
    sorter = ips.Sorter(0)
    prof_flags = ips.FLAG_PROFILE
    params = ips.make_params(flags=prof_flags)
    ws = sorter.workspace(ips.workspace_bytes(n, kind, "samplesort", params))
    log(f"workspace {ws.numel() / 2**20:.1f} MiB for {n * D / 2**30:.2f} GiB of data")

    for w in range(args.warmup):
        x = pristine.clone()
        sorter.sort_(x, params=params, ws=ws)
        del x
    torch.cuda.synchronize()

    # Timed region: exactly `steps` sorts.
    prof_sum: dict = {}
    step_ms = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for c in copies:
        s0 = time.perf_counter()
        sorter.sort_(c, params=params, ws=ws)
        step_ms.append((time.perf_counter() - s0) * 1e3)
        for row, phases in sorter.profile().items():
            for ph, (ms, el, la) in phases.items():
                a = prof_sum.setdefault(row, {}).setdefault(ph, [0.0, 0, 0])
                a[0] += ms; a[1] += el; a[2] += la
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    value = n * args.steps / elapsed / 1e9
    log(f"samplesort: {elapsed / args.steps * 1e3:.2f} ms/step, {value:.2f} Gkeys/s")

    # Output check on the device: every copy sorted, multiset kept (sum, xor).
    sign = torch.tensor(-(1 << 63), dtype=torch.int64, device=dev)
    ref_sum = pristine.view(torch.int64).sum()
    for c in copies:
        v = c.view(torch.int64) ^ sign if kind == "u64" else c.view(torch.int32).to(torch.int64) ^ (1 << 31)
        assert bool((v[1:] >= v[:-1]).all()), "output not sorted"
        assert int(c.view(torch.int64).sum() if kind == "u64" else c.view(torch.int32).to(torch.int64).sum()) == \
            int(ref_sum if kind == "u64" else pristine.view(torch.int32).to(torch.int64).sum()), "multiset changed"

    # Per level: algorithmic bytes 4 D n' (classification and permutation
    # each read and write every element once), LDS tier 2 D n'.
    steps = args.steps
    levels = []
    for row in sorted(k for k in prof_sum if k != "outside"):
        ph = prof_sum[row]
        part = ["sample", "classify", "boundaries", "flags", "permute", "cleanup_a", "cleanup_b"]
        ms = sum(ph[p][0] for p in part if p in ph) / steps
        el = ph.get("classify", [0, 0, 0])[1] / steps
        rec = {"level": row, "elems": int(el), "ms": round(ms, 4)}
        if el and ms:
            gbs = 4 * D * el / (ms * 1e-3) / 1e9
            rec.update({"GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)})
        if "lds_sort" in ph:
            lms = ph["lds_sort"][0] / steps
            lel = ph["lds_sort"][1] / steps
            rec["lds_ms"] = round(lms, 4)
            rec["lds_elems"] = int(lel)
            if lms:
                rec["lds_GBps"] = round(2 * D * lel / (lms * 1e-3) / 1e9, 1)
        rec["kernels_ms"] = {p: round(v[0] / steps, 4) for p, v in ph.items()}
        levels.append(rec)
    # Dominant kernel over the whole sort.
    tot = {}
    for row, ph in prof_sum.items():
        for p, (ms, el, la) in ph.items():
            a = tot.setdefault(p, [0.0, 0, 0])
            a[0] += ms; a[1] += el; a[2] += la
    dom = max(tot, key=lambda p: tot[p][0])
    dms, delems, dla = tot[dom]
    bytes_per_elem = {"classify": 2 * D, "permute": 2 * D, "lds_sort": 2 * D, "sorted_check": D,
                      "minmax": D, "reverse": 2 * D}.get(dom, 2 * D)
    achieved = bytes_per_elem * delems / dla / (dms / dla * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_launch_ms": round(dms / dla, 4), "bytes_per_launch": int(bytes_per_elem * delems / dla)}
    log(f"dominant kernel {dom}: {dms / steps:.3f} ms/step, {achieved:.0f} GB/s")

    radix = None
    if not args.no_radix:
        for c in copies:
            c.copy_(pristine)
        x = pristine.clone()
        sorter.sort_(x, algo="radix", params=params, ws=None)
        torch.cuda.synchronize()
        r0 = time.perf_counter()
        for c in copies:
            sorter.sort_(c, algo="radix", params=params)
        torch.cuda.synchronize()
        rel = time.perf_counter() - r0
        radix = {"value": round(n * steps / rel / 1e9, 3), "ms_per_step": round(rel / steps * 1e3, 3)}
        log(f"radix: {rel / steps * 1e3:.2f} ms/step, {radix['value']:.2f} Gkeys/s")
        v = copies[0].view(torch.int64) ^ sign if kind == "u64" else None
        if v is not None:
            assert bool((v[1:] >= v[:-1]).all()), "radix output not sorted"

    cpu = None
    if not args.no_cpu:
        import numpy as np

        import oracle
        ns = 1 << 24
        sample = synth.generate(kind, args.dist, ns, synth.seed_for(2, 0))
        times = []
        for r in range(4):
            t0 = time.perf_counter()
            oracle.sort(sample, kind)
            times.append(time.perf_counter() - t0)
        med = float(np.median(times[1:]))
        cpu = {"value": round(ns / med / 1e9, 5), "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
               "sample": f"2^24 {kind} {args.dist} keys, single-threaded merge sort, 4 runs, first dropped, "
                         f"median {med:.2f} s"}
        log(f"cpu oracle: {cpu['value']} Gkeys/s")

    out = {
        "metric": f"Gkeys/s, {kind} {args.dist.capitalize()} n=2^{args.log2n} in-place samplesort",
        "value": round(value, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": kind,
        "data": "synthetic: SplitMix64-seeded keys, resident in HBM before the timed region",
        "config": {"workload": f"{kind} {args.dist} n=2^{args.log2n}, IPS4o samplesort (k=256, n0=16)",
                   "n": n, "kind": kind, "algo": "samplesort", "dist": args.dist,
                   "workspace_bytes": int(ws.numel())},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "levels": levels,
        "radix": radix,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
