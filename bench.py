#!/usr/bin/env python3
"""PHOBIC build + bulk query on one MI355X.

Workload (the 100M-key configuration): 100,000,000 distinct uniform uint64 keys (seed 1), P = 2500,
lambda = 7, alpha = 1, interleaved Rice coding; then 100,000,000 lookups drawn uniformly with
replacement from the key set (seed 2), queried in batches of 1,000,000. One step = one full build
(hash, partition, bucket, order, search, encode) plus the 100 query batches. Keys and query keys are
resident in HBM before timing starts.

Prints one JSON line. ``value`` is build ns/key + query ns/query (lower is better); the breakdown,
bits/key, the roofline of the dominant kernel and the CPU-oracle baseline ride along.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T int32 lane-ops/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--lam", type=float, default=7.0)
    ap.add_argument("--coding", default="rice", choices=["rice", "compact"])
    ap.add_argument("--batch", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000)
    return ap.parse_args()


def cpu_baseline(args):
    """The oracle as it stands, on a bounded sample of the same workload (1M keys of the same
    distribution, same parameters): build ns/key + query ns/query on the host cores."""
    import oracle
    from paper_2404_18497_amd import synth

    threads = max(1, min(16, os.cpu_count() or 1))
    keys = synth.u64_keys(args.cpu_sample, 1)
    q = keys[synth.query_indices(keys.size, keys.size, 2)]
    prm = oracle.params(lam=args.lam, coding=args.coding)
    t0 = time.perf_counter()
    h = oracle.build_u64(keys, prm, threads=threads)
    t1 = time.perf_counter()
    h.query_u64(q)
    t2 = time.perf_counter()
    b = (t1 - t0) * 1e9 / keys.size
    qn = (t2 - t1) * 1e9 / q.size
    return {"value": round(b + qn, 2), "unit": "ns/key (build + query)", "cores": threads, "kind": "oracle",
            "sample": f"{keys.size} keys of the same distribution (seed 1), lambda {args.lam}, {args.coding}; "
                      f"build {b:.1f} ns/key on {threads} threads, query {qn:.1f} ns/query on 1 thread",
            "build_ns_per_key": round(b, 2), "query_ns_per_query": round(qn, 2)}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU: this library has no multi-GPU path (how it would shard is described "
              "in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2404_18497_amd import binding, synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    binding.lib()
    n, batch = args.n, args.batch
    print(f"[bench] generating {n} keys", file=sys.stderr, flush=True)
    keys = synth.u64_keys(n, 1)
    qidx = synth.query_indices(n, n, 2)
    dk = torch.from_numpy(keys.view(np.int64)).to(dev)
    dq = dk[torch.from_numpy(qidx).to(dev)]
    dp = torch.empty(n, dtype=torch.int64, device=dev)
    del qidx
    prm = binding.params(lam=args.lam, coding=args.coding)
    stream = torch.cuda.current_stream()

    def step(record=None):
        # events on the build/query stream: [0] before the build, [1] after it, [2] after the queries
        if record is not None:
            record[0].record(stream)
        h = binding.build_u64(dk, prm)
        if record is not None:
            record[1].record(stream)
        for b in range(0, n, batch):
            h.query_u64(dq[b:b + batch], out=dp[b:b + batch])
        if record is not None:
            record[2].record(stream)
        return h

    print("[bench] warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step().close()
    torch.cuda.synchronize()

    handles, events = [], []
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ev = tuple(torch.cuda.Event(enable_timing=True) for _ in range(3))
        handles.append(step(ev))
        events.append(ev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    infos = [h.build_info() for h in handles]
    build_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in events]))
    query_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in events]))
    phase = {k: float(np.mean([i[k] for i in infos])) for k in
             ["hash_count_ms", "scan_ms", "scatter_ms", "bucket_sort_ms", "search_ms", "encode_ms"]}
    bits = handles[0].size_bits() / n
    nlaunch = (n + batch - 1) // batch

    # kernels with their algorithmic traffic per launch
    kern = {
        "k_query_u64": {"ms": query_ms / nlaunch, "bytes": 16.0 * min(batch, n), "bound": "hbm"},
        "k_search": {"ms": phase["search_ms"], "bytes": 16.0 * n + 4.0 * n / args.lam * 2, "bound": "hbm"},
        "k_scatter_u64": {"ms": phase["scatter_ms"], "bytes": 24.0 * n, "bound": "hbm"},
        "k_hash_count_u64": {"ms": phase["hash_count_ms"], "bytes": 8.0 * n, "bound": "hbm"},
        "k_bucket_sort": {"ms": phase["bucket_sort_ms"], "bytes": 32.0 * n, "bound": "hbm"},
    }
    total_per_kernel = {k: v["ms"] * (nlaunch if k == "k_query_u64" else 1) for k, v in kern.items()}
    dom = max(total_per_kernel, key=total_per_kernel.get)
    d = kern[dom]
    achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
    roofline = {"kernel": dom, "bound": d["bound"], "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "per_launch_ms": round(d["ms"], 4), "launches_per_step": nlaunch if dom == "k_query_u64" else 1,
                "algorithmic_bytes_per_launch": d["bytes"]}

    out = {
        "metric": "build ns/key + query ns/key @100M keys, bits/key",
        "value": round(ms_per_step * 1e6 / n, 4),
        "unit": "ns/key",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"{n} distinct uniform u64 keys (seed 1), P 2500, lambda {args.lam:g}, alpha 1, "
                               f"interleaved {args.coding}; {n} uniform lookups (seed 2) in batches of {batch}",
                   "n_keys": n, "lambda": args.lam, "partition_size": 2500, "coding": args.coding,
                   "query_batch": batch},
        "build_ns_per_key": round(build_ms * 1e6 / n, 4),
        "query_ns_per_key": round(query_ms * 1e6 / n, 4),
        "bits_per_key": round(bits, 4),
        "phases_ms": {k: round(v, 4) for k, v in phase.items()} | {"build_ms": round(build_ms, 4),
                                                                   "query_all_batches_ms": round(query_ms, 4)},
        "roofline": roofline,
    }
    for h in handles:
        h.close()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
