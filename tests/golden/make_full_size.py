"""Writes full_size_images.json: SHA-256 of the oracle's whole image and pilot array for the
full-size parity cases the GPU tests compare against.

Calls only the oracle (and the seeded input generators, which hold none of the method's
arithmetic). Cases, each named on the command line or all by default:

  u64_100m_l7_compact   100M distinct uniform u64 keys (seed 1), lambda 7, interleaved Compact
  u64_100m_l7_mixed64   the same keys, interleaved Rice with the first 64 encoders Compact
                        (mixed interleaved coding, Sec. 4.1)
  u64_150m_l7_rice      150M distinct uniform u64 keys (seed 1), lambda 7, interleaved Rice: more
                        partitions than the coarse-bin partitioner takes, so the device build runs
                        its general (per-key atomics) partitioner
  str_100m_l7_a1        100M random strings (seed 3; lengths 10-50, [a-z0-9]), lambda 7, alpha 1
  str_100m_l7_a099      the same strings, alpha 0.99 with remapping (App. B)
  u64_10m_l13_rice      10M distinct uniform u64 keys (seed 1), lambda 13, interleaved Rice

All use P 2500 and hash seed 0x5EED. A case's entry holds the image hash, the pilot-array hash
(partition-major u32) and bits/key.

Run: python tests/golden/make_full_size.py [case ...]   (tens of minutes on 8 cores; lambda 13 alone
takes about a quarter of an hour)
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

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size_images.json")

CASES = {
    "u64_100m_l7_compact": dict(kind="u64", n=100_000_000, seed=1, lam=7.0, coding="compact"),
    "u64_100m_l7_mixed64": dict(kind="u64", n=100_000_000, seed=1, lam=7.0, coding="rice", n_compact=64),
    "u64_150m_l7_rice": dict(kind="u64", n=150_000_000, seed=1, lam=7.0, coding="rice"),
    "str_100m_l7_a1": dict(kind="str", n=100_000_000, seed=3, lam=7.0, coding="rice", alpha=(1, 1)),
    "str_100m_l7_a099": dict(kind="str", n=100_000_000, seed=3, lam=7.0, coding="rice", alpha=(99, 100)),
    "u64_10m_l13_rice": dict(kind="u64", n=10_000_000, seed=1, lam=13.0, coding="rice"),
}


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def run(name, spec, threads):
    prm = oracle.params(lam=spec["lam"], coding=spec["coding"], alpha=spec.get("alpha", (1, 1)),
                        n_compact=spec.get("n_compact", 0))
    if spec["kind"] == "u64":
        keys = synth.u64_keys(spec["n"], spec["seed"])
        h = oracle.build_u64(keys, prm, threads=threads)
    else:
        buf, offs = synth.ascii_strings(spec["n"], spec["seed"])
        h = oracle.build_str(buf, offs, prm, threads=threads)
    entry = {k: (list(v) if isinstance(v, tuple) else v) for k, v in spec.items()}
    entry.update(image_sha256=sha(h.image()), pilots_sha256=sha(np.asarray(h.pilots(), dtype=np.uint32)),
                 bits_per_key=h.size_bits() / spec["n"])
    return entry


def main():
    names = sys.argv[1:] or list(CASES)
    out = json.load(open(PATH)) if os.path.exists(PATH) else {}
    threads = os.cpu_count() or 1
    for name in names:
        t = time.time()
        out[name] = run(name, CASES[name], threads)
        print(name, out[name], f"{time.time() - t:.1f}s", flush=True)
        with open(PATH, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
