"""Writes search_work_100m.json: the oracle's exact work counters for the 100M-key benchmark
workload (100,000,000 distinct uniform u64 keys, seed 1, P 2500, alpha 1) at lambda 5, 7 and 9.

Calls only the oracle. The counters are the nested-loop search's work measures: hash evaluations
h(x, s), slot probes (the key checks of the loop over displacements, the paper's work measure in
Sec. 3), seeds tried, and buckets placed. The benchmark divides them by the measured search time.
It also records the SHA-256 of the oracle's whole interleaved-Rice image and of its pilot array
(partition-major u32, the same for either coding), which the full-size GPU parity test compares
against the device build.

Run: python tests/golden/make_search_work.py   (about 5 minutes on 8 cores)
"""

import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2404_18497_amd import synth  # noqa: E402


def main():
    n = 100_000_000
    keys = synth.u64_keys(n, 1)
    out = {"workload": "100000000 distinct uniform u64 keys (seed 1), P 2500, alpha 1, hash seed 0x5EED",
           "counters": {}}
    for lam in (5.0, 7.0, 9.0):
        t = time.time()
        h = oracle.build_u64(keys, oracle.params(lam=lam), threads=os.cpu_count() or 1)
        c = h.counters()
        c["bits_per_key_rice"] = h.size_bits() / n
        c["image_sha256_rice"] = hashlib.sha256(h.image().tobytes()).hexdigest()
        c["pilots_sha256"] = hashlib.sha256(np.ascontiguousarray(h.pilots(), dtype=np.uint32).tobytes()).hexdigest()
        out["counters"][f"{lam:g}"] = c
        print(lam, c, f"{time.time() - t:.1f}s", flush=True)
        del h
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "search_work_100m.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
