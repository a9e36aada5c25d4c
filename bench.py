#!/usr/bin/env python3
"""PHOBIC on one MI355X: build + bulk query (default), batched builds, and serving.

--workload build_query (default; the 100M-key configuration): 100,000,000 distinct uniform uint64 keys
    (seed 1), P = 2500, lambda = 7, alpha = 1, interleaved Rice coding; then 100,000,000 lookups drawn
    uniformly with replacement from the key set (seed 2), queried in batches of 1,000,000 issued
    round-robin on two streams (the batches are independent, so one launch's tail overlaps the next
    launch's start). One step =
    one full build (hash, partition, bucket, order, search, encode) plus the 100 query batches. Keys
    and query keys are resident in HBM before timing starts. ``value`` = build ns/key + query
    ns/query (lower is better). The same line then carries the rest of the metric, each after the
    timed region: lambda 5 and 9 on the same keys and lookups; the mixed-coding curve (query ns/key
    and bits/key for several counts of leading Compact encoders); 100M random strings (lengths 10-50,
    [a-z0-9]) at alpha 1 and 0.99 with 100M lookups; a short serving trace at 0.5, 0.8 and 0.95 of the
    plain capacity (``--loads``; p50/p99 per request kind, throughput and mean batch, plain vs served); the bucket assignment functions compared in Sec. 3.1 (beta_*, PTHash's skewed,
    CHD's uniform) on the same keys; and the oracle on the host cores (``cpu_baseline``).
    ``--no-extras`` skips all but the last.
--workload batch: 4096 MPHFs, key counts lognormal(median 50K, sigma 1.5) clipped to [1K, 10M]
    (seed 5), uniform uint64 keys (set t from seed 100 + t), P 2500, lambda 7; one batched build with
    an autotuned search shape versus 4096 sequential plain builds. ``value`` = batched ns/key.
--workload serve: Poisson arrivals of build requests (10%, lognormal sizes median 5e5, sigma 1.5,
    clipped to [10K, 50M]) and query requests (90%, 1K-1M lookups, log-uniform, against resident
    MPHFs) under a 200 GB HBM budget; the library's server with continuous batching versus plain
    per-request FIFO execution, at the same arrival trace, for each load in ``--loads`` (fractions of
    the measured plain capacity). ``value`` = p99 query latency (ms) at the first load.

--workload psweep: the 100M-key build at lambda 7 for several partition sizes P (1K to 200K): build ns/key,
    search time, bits/key, and the pilot payload in interleaved versus mono Rice coding.

--workload copy: a plain 1 GiB device-to-device copy, repeated; the reference kernel whose HBM counter
    readings (FETCH_SIZE, WRITE_SIZE) calibrate the traffic figures of the other kernels, and a
    measured copy bandwidth next to the 8 TB/s peak.

Each mode prints one JSON line.
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

HBM_PEAK_GBS = 8000.0                                # MI355X HBM3E, 8 TB/s
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12           # 39.3 T int32 lane-ops/s (256 CU x 4 SIMD16 x 2.4 GHz)
HASH_OPS = 30          # int32 ops of one position-hash evaluation (one 64-bit mixer, xor, multiply-high)
PROBE_OPS = 1.0 / 16   # a funnel shift and an AND test 32 displacements: 2 ops per 32 slot probes


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="build_query", choices=["build_query", "batch", "serve", "copy", "psweep"])
    ap.add_argument("--psizes", default="1000,2500,10000,50000,200000", help="psweep: partition sizes")
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--lam", type=float, default=7.0)
    ap.add_argument("--coding", default="rice", choices=["rice", "compact"])
    ap.add_argument("--n-compact", type=int, default=0, help="leading Compact encoders (mixed coding)")
    ap.add_argument("--batch", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000)
    ap.add_argument("--mphfs", type=int, default=4096)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--requests", type=int, default=1500)
    ap.add_argument("--load", type=float, default=0.8, help="arrival rate as a fraction of plain capacity")
    ap.add_argument("--loads", default="", help="serve workload: comma-separated load fractions")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only: no lambda 5/9 lines, mixed-coding curve, strings or serving trace")
    ap.add_argument("--mixed", default="16,64,128,-1",
                    help="mixed-coding curve: leading Compact encoders per point (-1 = Compact coding)")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args):
    """The oracle as it stands, on a bounded sample of the same workload: the first args.cpu_sample
    keys' worth of the same distribution (same seed, P, lambda, coding). Per-key build and query cost do
    not depend on n at fixed P (every partition holds about P keys and is searched alone), so the
    sample's ns/key stands for the 100M-key workload; its 100M-key equivalent is ns/key x 1e8.
    The build is timed on one thread and on every host core; the query on one thread."""
    import oracle
    from paper_2404_18497_amd import synth

    cores = os.cpu_count() or 1
    keys = synth.u64_keys(args.cpu_sample, 1)
    q = keys[synth.query_indices(keys.size, keys.size, 2)]
    prm = oracle.params(lam=args.lam, coding=args.coding)
    t0 = time.perf_counter()
    oracle.build_u64(keys, prm, threads=1)
    t1 = time.perf_counter()
    h = oracle.build_u64(keys, prm, threads=cores)
    t2 = time.perf_counter()
    h.query_u64(q)
    t3 = time.perf_counter()
    b1 = (t1 - t0) * 1e9 / keys.size
    bn = (t2 - t1) * 1e9 / keys.size
    qn = (t3 - t2) * 1e9 / q.size
    return {"value": round(bn + qn, 2), "unit": "ns/key (build + query)", "cores": cores, "kind": "oracle",
            "sample": f"{keys.size} keys of the same distribution (seed 1), lambda {args.lam:g}, {args.coding}, "
                      f"{keys.size} lookups (seed 2); build {bn:.1f} ns/key on {cores} threads and {b1:.1f} ns/key "
                      f"on 1 thread, query {qn:.1f} ns/query on 1 thread; per-key cost is independent of n at "
                      f"fixed P, so x 1e8 gives the 100M-key equivalent",
            "cpu_model": cpu_model(), "build_ns_per_key": round(bn, 2), "build_ns_per_key_1thread": round(b1, 2),
            "query_ns_per_query": round(qn, 2),
            "equivalent_100m_s": {"build_all_cores": round(bn * 0.1, 2), "build_1thread": round(b1 * 0.1, 2),
                                  "query_1thread": round(qn * 0.1, 2)}}


def search_work(n, lam):
    """The oracle's exact search counters for the 100M-key workload (tests/golden), else None."""
    path = os.path.join(ROOT, "tests", "golden", "search_work_100m.json")
    if n != 100_000_000 or not os.path.exists(path):
        return None
    return json.load(open(path))["counters"].get(f"{lam:g}")


def measured_traffic(kernel: str, n: int, lam: float):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE / WRITE_SIZE summary of this
    workload (copy-calibrated), or None if there is none or the kernel's source changed since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"traffic_build_query_{n // 1_000_000}m_lambda{lam:g}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))["kernels"].get(kernel)
    if not rec or not rec.get("source"):
        return None
    src = os.path.join(ROOT, "paper_2404_18497_amd", "csrc", rec["source"])
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    return rec["read_bytes"] + rec["write_bytes"]


def _timed(torch, build, queries, steps, warmup):
    """Runs `warmup` untimed and `steps` timed steps of build() followed by queries(handle); returns
    (ms per step by the host clock around the synchronized timed region, mean build ms and mean query
    ms from events on the build stream, build infos, bits per key source handle)."""
    stream = torch.cuda.current_stream()

    def step(record=None):
        if record is not None:
            record[0].record(stream)
        h = build()  # returns once the image is complete
        if record is not None:
            record[1].record(stream)
        queries(h)
        if record is not None:
            record[2].record(stream)
        return h

    for _ in range(warmup):
        step().close()
    torch.cuda.synchronize()
    handles, events = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        ev = tuple(torch.cuda.Event(enable_timing=True) for _ in range(3))
        handles.append(step(ev))
        events.append(ev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    infos = [h.build_info() for h in handles]
    build_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in events]))
    query_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in events]))
    bits = handles[0].size_bits()
    for h in handles:
        h.close()
    return (t1 - t0) * 1e3 / steps, build_ms, query_ms, infos, bits


def _phases(infos):
    return {k: float(np.mean([i[k] for i in infos])) for k in
            ["hash_count_ms", "scan_ms", "scatter_ms", "bucket_sort_ms", "search_ms", "encode_ms"]}


def _batched_queries(torch, n, batch, qstreams, launch):
    """Issues the lookups in batches of `batch`, round-robin on qstreams, then joins them into the
    current stream. launch(lo, hi, stream) queries lookups [lo, hi)."""
    stream = torch.cuda.current_stream()
    for i, b in enumerate(range(0, n, batch)):
        launch(b, min(n, b + batch), qstreams[i % len(qstreams)])
    for qs in qstreams[1:]:
        stream.wait_stream(qs)


def headline(args):
    import torch

    from paper_2404_18497_amd import binding, synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    binding.lib()
    n, batch = args.n, args.batch
    log(f"generating {n} keys")
    keys = synth.u64_keys(n, 1)
    qidx = synth.query_indices(n, n, 2)
    dk = torch.from_numpy(keys.view(np.int64)).to(dev)
    dq = dk[torch.from_numpy(qidx).to(dev)]
    dp = torch.empty(n, dtype=torch.int64, device=dev)
    del qidx
    # The query batches are independent: they go round-robin to two streams (default priority), so
    # the next batch's wavefronts fill the device while the previous launch drains.
    qstreams = [torch.cuda.current_stream(), torch.cuda.Stream()]

    def u64_run(prm, steps, warmup):
        def queries(h):
            _batched_queries(torch, n, batch, qstreams,
                             lambda lo, hi, st: h.query_u64(dq[lo:hi], out=dp[lo:hi], stream=st))
        return _timed(torch, lambda: binding.build_u64(dk, prm), queries, steps, warmup)

    log(f"timing {args.steps} steps")
    ms_per_step, build_ms, query_ms, infos, bits = u64_run(
        binding.params(lam=args.lam, coding=args.coding, n_compact=args.n_compact), args.steps, args.warmup)
    phase = _phases(infos)
    bits /= n
    nlaunch = (n + batch - 1) // batch

    # dominant kernel and its roofline (per launch; durations from HIP events on the launch stream)
    cfg = binding.get_search_config()
    # tables of P 2500 partitions stay below 4096 slots: the one-pass scan instance
    search_kernel = (f"k_search_persistent<{cfg['waves_per_group']}, false>" if cfg["groups_per_cu"]
                     else f"k_search<{cfg['waves_per_group']}, false>")
    per_step = {"k_search": phase["search_ms"], "k_query_u64": query_ms}
    dom = max(per_step, key=per_step.get)
    if dom == "k_search":
        w = search_work(n, args.lam)
        ops = HASH_OPS * w["hash_evals"] + PROBE_OPS * w["slot_probes"] if w else None
        achieved = ops / (phase["search_ms"] * 1e-3) / 1e12 if ops else None
        roofline = {"kernel": search_kernel, "bound": "alu", "achieved": None if achieved is None else round(achieved, 3),
                    "peak": round(ALU_PEAK_TOPS, 1), "unit": "TOP/s",
                    "frac": None if achieved is None else round(achieved / ALU_PEAK_TOPS, 4),
                    "traffic": measured_traffic(search_kernel, n, args.lam),
                    "per_launch_ms": round(phase["search_ms"], 4), "launches_per_step": 1,
                    "algorithmic_ops_per_launch": ops,
                    "work": None if not w else {"hash_evals": w["hash_evals"], "slot_probes": w["slot_probes"]}}
    else:
        per = query_ms / nlaunch
        achieved = 16.0 * min(batch, n) / (per * 1e-3) / 1e9
        # the query instance that stages the bucket table and encoder words in LDS (B <= 1024)
        qkernel = "k_query_u64<true, unsigned int>"
        roofline = {"kernel": qkernel, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(qkernel, n, args.lam),
                    "per_launch_ms": round(per, 4), "launches_per_step": nlaunch,
                    "algorithmic_bytes_per_launch": 16.0 * min(batch, n)}
    q_per = query_ms / nlaunch
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
                               f"interleaved {args.coding}"
                               + (f" with the first {args.n_compact} encoders Compact" if args.n_compact else "")
                               + f"; {n} uniform lookups (seed 2) in batches of {batch} on {len(qstreams)} streams",
                   "n_keys": n, "lambda": args.lam, "partition_size": 2500, "coding": args.coding,
                   "n_compact": args.n_compact, "query_batch": batch},
        "build_ns_per_key": round(build_ms * 1e6 / n, 4),
        "query_ns_per_key": round(query_ms * 1e6 / n, 4),
        "bits_per_key": round(bits, 4),
        "phases_ms": {k: round(v, 4) for k, v in phase.items()} | {"build_ms": round(build_ms, 4),
                                                                   "query_all_batches_ms": round(query_ms, 4)},
        "roofline": roofline,
        "query_kernel": {"ms_per_batch": round(q_per, 4), "streams": len(qstreams),
                         "hbm_GBps": round(16.0 * min(batch, n) / (q_per * 1e-3) / 1e9, 1)},
    }
    if not args.no_extras:
        # the rest of the metric, each on the same keys and lookups, one warm-up and two timed steps
        lam_rows = {}
        for lam in (5.0, 9.0):
            log(f"lambda {lam:g}")
            ms, b_ms, q_ms, inf, bt = u64_run(binding.params(lam=lam), 2, 1)
            lam_rows[f"{lam:g}"] = {"ms_per_step": round(ms, 3), "build_ns_per_key": round(b_ms * 1e6 / n, 4),
                                    "query_ns_per_key": round(q_ms * 1e6 / n, 4), "bits_per_key": round(bt / n, 4),
                                    "search_ms": round(_phases(inf)["search_ms"], 4)}
        out["lambda_sweep"] = lam_rows
        curve = []
        for c in args.mixed:
            log(f"mixed coding, {c} Compact encoders")
            coding = "compact" if c < 0 else "rice"
            ms, b_ms, q_ms, inf, bt = u64_run(binding.params(lam=args.lam, coding=coding, n_compact=max(c, 0)), 2, 1)
            curve.append({"n_compact": "all (Compact coding)" if c < 0 else c, "bits_per_key": round(bt / n, 4),
                          "query_ns_per_key": round(q_ms * 1e6 / n, 4), "build_ns_per_key": round(b_ms * 1e6 / n, 4)})
        out["mixed_coding_curve"] = curve
        # the bucket assignment functions of the comparison in Sec. 3.1, same keys, lambda and coding
        fns = {"optimized (beta_eps)": {"build_ns_per_key": out["build_ns_per_key"], "bits_per_key": out["bits_per_key"],
                                        "search_ms": out["phases_ms"]["search_ms"]}}
        for fn in ("beta_star", "skew", "uniform"):
            log(f"bucket function {fn}")
            ms, b_ms, q_ms, inf, bt = u64_run(binding.params(lam=args.lam, coding=args.coding, bucket_fn=fn), 1, 1)
            fns[fn] = {"build_ns_per_key": round(b_ms * 1e6 / n, 4), "bits_per_key": round(bt / n, 4),
                       "search_ms": round(_phases(inf)["search_ms"], 4), "query_ns_per_key": round(q_ms * 1e6 / n, 4)}
        out["bucket_functions"] = fns
    del dk, dq, dp
    torch.cuda.empty_cache()
    if not args.no_extras:
        out["strings"] = strings_rows(args, qstreams)
        log("serving (short trace)")
        loads = [float(x) for x in args.loads.split(",")] if args.loads else [0.5, 0.8, 0.95]
        out["serving"] = serve_run(args.requests, loads)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


def strings_rows(args, qstreams):
    """100M random strings (seed 3; lengths 10-50, [a-z0-9]) at lambda 7, alpha 1 and 0.99: build and
    100M lookups drawn uniformly with replacement (seed 4), in batches of 1M on two streams."""
    import torch

    from paper_2404_18497_amd import binding, synth

    dev = torch.device("cuda", 0)
    n, batch = args.n, args.batch
    log(f"generating {n} strings")
    buf, offs = synth.ascii_strings(n, 3)
    db = torch.from_numpy(buf).to(dev)
    do = torch.from_numpy(offs.view(np.int64)).to(dev)
    del buf, offs
    # the lookups' strings gathered once into their own contiguous buffer (before timing)
    qi = torch.from_numpy(synth.query_indices(n, n, 4)).to(dev)
    ql = (do[1:] - do[:-1])[qi]
    qo = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    torch.cumsum(ql, 0, out=qo[1:])
    qb = torch.empty(int(qo[-1]), dtype=torch.uint8, device=dev)
    for c0 in range(0, n, 1_000_000):
        c1 = min(n, c0 + 1_000_000)
        L = ql[c0:c1]
        base = qo[c0]
        rel = torch.arange(int(qo[c1] - base), device=dev) - torch.repeat_interleave(qo[c0:c1] - base, L)
        qb[int(base):int(qo[c1])] = db[torch.repeat_interleave(do[qi[c0:c1]], L) + rel]
    del qi, ql
    dp = torch.empty(n, dtype=torch.int64, device=dev)
    rows = {}
    for alpha in [(1, 1), (99, 100)]:
        log(f"strings, alpha {alpha[0]}/{alpha[1]}")
        prm = binding.params(lam=7.0, alpha=alpha)

        def queries(h):
            # offsets are absolute positions in qb, so a slice of them is a batch
            _batched_queries(torch, n, batch, qstreams,
                             lambda lo, hi, st: h.query_str(qb, qo[lo:hi + 1], out=dp[lo:hi], stream=st))
        ms, b_ms, q_ms, inf, bt = _timed(torch, lambda: binding.build_str(db, do, prm), queries, 2, 1)
        rows[f"alpha_{alpha[0]}/{alpha[1]}"] = {
            "ms_per_step": round(ms, 3), "build_ns_per_key": round(b_ms * 1e6 / n, 4),
            "query_ns_per_key": round(q_ms * 1e6 / n, 4), "bits_per_key": round(bt / n, 4),
            "phases_ms": {k: round(v, 4) for k, v in _phases(inf).items()}}
    rows["workload"] = (f"{n} random strings (seed 3), lengths 10-50, [a-z0-9], P 2500, lambda 7, interleaved "
                        f"Rice; {n} uniform lookups (seed 4) in batches of {batch} on {len(qstreams)} streams")
    del db, do, qb, qo, dp
    torch.cuda.empty_cache()
    return rows


def batch_mode(args):
    import torch

    from paper_2404_18497_amd import autotune, binding, synth

    torch.cuda.set_device(0)
    binding.lib()
    sizes = synth.lognormal_sizes(args.mphfs, 50_000, 1.5, 1_000, 10_000_000, 5)
    log(f"generating {args.mphfs} key sets, {int(sizes.sum())} keys")
    sets = synth.u64_key_sets(sizes, 100)
    dev = [torch.from_numpy(s.view(np.int64)).cuda() for s in sets]
    del sets
    prm = binding.params(lam=7.0)
    total = int(sizes.sum())
    tuned, table = None, None
    if not args.no_tune:
        # on the whole batch: a sample of 512 key sets (a eighth of the partitions) favoured one wavefront
        # per partition, while the whole batch runs faster on a persistent grid
        log("autotuning the search shape on the whole batch")
        tuned, table = autotune.tune_batch(binding.BatchKeys(dev), prm, repeats=1, log=log)
    cfg = binding.get_search_config()
    log("batched build")
    bkeys = binding.BatchKeys(dev)  # the key sets' pointer arrays, checked once like the resident keys
    binding.build_batch_u64(bkeys, prm)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hs = binding.build_batch_u64(bkeys, prm)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    info = hs[0].build_info()
    bits = sum(h.size_bits() for h in hs) / total
    del hs
    log("sequential plain builds")
    binding.build_u64(dev[0], prm).close()
    t0 = time.perf_counter()
    for d in dev:
        binding.build_u64(d, prm).close()
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    out = {
        "metric": "batched build ns/key (4096 MPHFs in one launch) vs sequential plain builds",
        "value": round(t_batch * 1e9 / total, 4), "unit": "ns/key", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(t_batch * 1e3, 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"{args.mphfs} MPHFs, sizes lognormal(median 50K, sigma 1.5) clipped [1K, 10M] "
                               f"(seed 5), uniform u64 keys (set t seed 100+t), P 2500, lambda 7",
                   "total_keys": total},
        "batched_ms": round(t_batch * 1e3, 3), "sequential_ms": round(t_seq * 1e3, 3),
        "speedup_vs_sequential": round(t_seq / t_batch, 2), "bits_per_key": round(bits, 4),
        "batched_phases_ms": {k: round(info[k], 3) for k in ["bucket_sort_ms", "search_ms", "encode_ms", "total_ms"]},
        "search_config": cfg, "tuned": tuned,
        "tuning_table": None if table is None else [[c, round(ms, 3)] for c, ms in table],
    }
    print(json.dumps(out), flush=True)


def serve_run(R, loads):
    """C5: R requests, 10% builds (lognormal median 5e5, sigma 1.5, clipped to [10K, 50M]) and 90%
    queries (1K-1M lookups, log-uniform) against 16 resident MPHFs, 200 GB HBM budget. The plain
    capacity is measured with every request queued at once and run one at a time (FIFO); then for each
    load factor the same Poisson trace at load x capacity runs plain and served (continuous batching)."""
    import torch

    from paper_2404_18497_amd import binding, synth

    torch.cuda.set_device(0)
    binding.lib()
    rng = np.random.default_rng(6)
    kinds = rng.random(R) < 0.1  # True = build
    nb = int(kinds.sum())
    bsizes = synth.lognormal_sizes(nb + 16, 500_000, 1.5, 10_000, 50_000_000, 7)
    qsizes = synth.log_uniform_sizes(R - nb, 1_000, 1_000_000, 8)
    log(f"{R} requests: {nb} builds ({int(bsizes[16:].sum())} keys), {R - nb} queries; 16 resident MPHFs")
    keysets = synth.u64_key_sets(bsizes, 500)
    dkeys = [torch.from_numpy(k.view(np.int64)).cuda() for k in keysets]
    targets = rng.integers(0, 16, R - nb)
    qkeys = [dkeys[t][torch.from_numpy(rng.integers(0, keysets[t].size, int(m))).cuda()]
             for t, m in zip(targets, qsizes)]
    outs = [torch.empty(int(m), dtype=torch.int64, device="cuda") for m in qsizes]
    del keysets
    prm = binding.params(lam=7.0)
    budget = 200 << 30

    def run(server_kw, arrivals):
        srv = binding.Server(prm, budget_bytes=budget, **server_kw)
        ids0 = [srv.submit_build(dkeys[t]) for t in range(16)]
        done = {}
        while len(done) < 16:
            for r in srv.poll(wait_ms=100):
                done[r["request_id"]] = r
        srv.poll()
        t_start = srv.now()
        results, bi, qi = {}, 16, 0
        for i in range(R):
            if arrivals is not None:
                while srv.now() - t_start < arrivals[i]:
                    for r in srv.poll():
                        results[r["request_id"]] = r
                    time.sleep(0.0002)
            if kinds[i]:
                srv.submit_build(dkeys[bi])
                bi += 1
            else:
                srv.submit_query(ids0[targets[qi]], qkeys[qi], outs[qi])
                qi += 1
        while len(results) < R:
            for r in srv.poll(wait_ms=100):
                results[r["request_id"]] = r
        t_end = max(r["done_s"] for r in results.values())
        st = srv.stats()
        srv.close()
        lat = {k: np.array([r["done_s"] - r["submit_s"] for r in results.values() if r["kind"] == k]) * 1e3
               for k in ("build", "query")}
        batches = {k: [r["batch"] for r in results.values() if r["kind"] == k] for k in ("build", "query")}
        r3 = lambda v: round(float(v), 3)  # noqa: E731
        return {"ok": all(r["status"] == 0 for r in results.values()),
                "throughput_rps": round(R / (t_end - t_start), 2), "makespan_s": round(t_end - t_start, 3),
                "p50_ms": {k: r3(np.percentile(v, 50)) for k, v in lat.items() if v.size},
                "p99_ms": {k: r3(np.percentile(v, 99)) for k, v in lat.items() if v.size},
                "mean_batch": {k: r3(np.mean(v)) for k, v in batches.items() if v},
                "query_launches": st["query_launches"], "build_launches": st["build_launches"],
                "peak_bytes": st["peak_bytes"]}

    plain_kw = dict(workers=1, max_query_batch=1, max_build_batch=1)
    served_kw = dict(workers=4, max_query_batch=64, max_build_batch=8, query_workers=1)
    log("plain capacity (all requests at once, FIFO, one at a time)")
    cap = run(plain_kw, None)
    out = {"requests": R, "plain_capacity_rps": cap["throughput_rps"], "loads": {}}
    for load in loads:
        rate = load * cap["throughput_rps"]
        arrivals = synth.poisson_arrivals(R, rate, 9)
        log(f"open loop at {load:g} x capacity ({rate:.1f} requests/s): plain")
        plain = run(plain_kw, arrivals)
        log("open loop: served (continuous batching)")
        served = run(served_kw, arrivals)
        out["loads"][f"{load:g}"] = {"offered_rps": round(rate, 2), "plain": plain, "served": served}
    out["workload"] = (f"{R} requests, 10% builds (lognormal median 5e5, sigma 1.5, [10K, 50M]), 90% queries "
                       f"(log-uniform 1K-1M) on 16 resident MPHFs, Poisson arrivals (seed 9) at the given fractions "
                       f"of plain capacity, 200 GB budget; served = 4 workers (1 query-only), up to 64 queries per "
                       f"launch and 8 builds per batched build; plain = one at a time, FIFO")
    return out


def serve_mode(args):
    loads = [float(x) for x in args.loads.split(",")] if args.loads else [args.load]
    res = serve_run(args.requests, loads)
    main_load = res["loads"][f"{loads[0]:g}"]
    out = {
        "metric": "serving p99 query latency (ms), Poisson arrivals, 200 GB HBM budget",
        "value": main_load["served"]["p99_ms"]["query"], "unit": "ms", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(main_load["served"]["makespan_s"] * 1e3, 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": res["workload"], "load": loads[0]},
        "serving": res,
    }
    print(json.dumps(out), flush=True)


def rice_width(total: int, count: int) -> int:
    """Golomb-Rice parameter of a geometric source of the given mean (Kiely's rule, as the library
    uses it); reporting only."""
    import math

    if total == 0 or count == 0:
        return 0
    mu = total / count
    b = 1 + math.floor(math.log2(math.log((math.sqrt(5) - 1) / 2) / math.log(mu / (mu + 1))))
    return max(0, min(32, b))


def rice_payload_bits(v: np.ndarray) -> int:
    """Bits of one Golomb-Rice code over the values v: b + 1 + (v >> b) each, b by Kiely's rule."""
    v = v.astype(np.uint64, copy=False)
    b = rice_width(int(v.sum()), v.size)
    return int(v.size) * (b + 1) + int((v >> np.uint64(b)).sum())


def psweep_mode(args):
    """Partition-size sweep (the paper's partition-size experiments): for each P, the 100M-key workload
    at lambda 7 (Rice): build ns/key and search time, bits/key of the whole structure, and the pilot
    payload under interleaved Rice coding (one Rice code per bucket index, Sec. 4.1) against one Rice
    code for all pilots (mono)."""
    import torch

    from paper_2404_18497_amd import binding, synth

    torch.cuda.set_device(0)
    binding.lib()
    n = args.n
    log(f"generating {n} keys")
    keys = synth.u64_keys(n, 1)
    dk = torch.from_numpy(keys.view(np.int64)).cuda()
    del keys
    rows = []
    for P in [int(x) for x in args.psizes.split(",")]:
        prm = binding.params(partition_size=P, lam=args.lam, keep_pilots=True)
        log(f"P = {P}")
        h = binding.build_u64(dk, prm)  # warm-up
        h.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = binding.build_u64(dk, prm)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        info = h.build_info()
        pil = h.pilots()  # K x B
        ic = sum(rice_payload_bits(pil[:, i]) for i in range(pil.shape[1]))
        mono = rice_payload_bits(pil.reshape(-1))
        rows.append({"P": P, "K": h.K, "B": h.B, "build_ms": round(ms, 3), "build_ns_per_key": round(ms * 1e6 / n, 4),
                     "search_ms": round(info["search_ms"], 3), "partition_path": info["partition_path"],
                     "max_partition_keys": info["max_partition_keys"], "bits_per_key": round(h.size_bits() / n, 4),
                     "pilot_bits_per_key_ic_rice": round(ic / n, 4), "pilot_bits_per_key_mono_rice": round(mono / n, 4),
                     "phases_ms": {k: round(v, 3) for k, v in _phases([info]).items()}})
        log(json.dumps(rows[-1]))
        h.close()
    out = {"metric": "partition-size sweep: build ns/key, bits/key, interleaved vs mono Rice pilot bits/key",
           "value": rows[0]["build_ns_per_key"], "unit": "ns/key", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": rows[0]["build_ms"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "u64", "data": "synthetic",
           "config": {"workload": f"{n} distinct uniform u64 keys (seed 1), lambda {args.lam:g}, alpha 1, interleaved "
                                  f"Rice, P in {args.psizes}"},
           "rows": rows}
    print(json.dumps(out), flush=True)


def copy_mode(args):
    import torch

    torch.cuda.set_device(0)
    nbytes = 1 << 30
    src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(args.steps):
        dst.copy_(src)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / args.steps
    gbs = 2.0 * nbytes / (ms * 1e-3) / 1e9
    out = {"metric": "device copy GB/s (read + write)", "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
           "config": {"workload": "1 GiB device-to-device copy", "bytes_read": nbytes, "bytes_written": nbytes},
           "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    args.mixed = [int(x) for x in args.mixed.split(",") if x.strip()] if isinstance(args.mixed, str) else args.mixed
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU: this library has no multi-GPU path; partitions are independent, so a "
              "multi-GPU build would give each GPU a range of partitions", file=sys.stderr)
        sys.exit(2)
    {"build_query": headline, "batch": batch_mode, "serve": serve_mode, "copy": copy_mode,
     "psweep": psweep_mode}[args.workload](args)


if __name__ == "__main__":
    main()
