"""Summaries of rocprofv3 output for the benchmark workloads.

    python -m paper_2404_18497_amd.profile_summary kernels --stats DIR/run_kernel_stats.csv \\
        --steps S --title T --command C --out profiles/NAME.md
    python -m paper_2404_18497_amd.profile_summary traffic --fetch F.csv --write W.csv \\
        --copy-fetch CF.csv --copy-write CW.csv --copy-bytes 1073741824 --title T --commands C1 C2 C3 C4 \\
        --out profiles/NAME.md --json profiles/NAME.json
    python -m paper_2404_18497_amd.profile_summary counters --csv DIR/run_counter_collection.csv \\
        --kernel k_search --title T --command C --out profiles/NAME.md

`traffic` scales each kernel's FETCH_SIZE and WRITE_SIZE (KiB per dispatch) by the ratio between the
bytes a plain device copy of known size moves and what the same counter reads for it, and writes a
JSON record per kernel with the SHA-256 of the source file that defines it, so that a reader can
tell whether the kernel has changed since the counters were taken.
"""

from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2404_18497_amd", "csrc")


def short_name(name: str) -> str:
    m = re.search(r"(k_[A-Za-z0-9_]+)(<[^>(]*>)?", name)
    if m:
        return m.group(1) + (m.group(2) or "")
    return name.split("(")[0][:60]


def source_of(kernel: str):
    """The csrc file that defines the kernel, or None."""
    base = kernel.split("<")[0]
    for f in sorted(os.listdir(CSRC)):
        if f.endswith(".hip"):
            with open(os.path.join(CSRC, f)) as fh:
                if re.search(r"void\s+" + re.escape(base) + r"\s*\(", fh.read()):
                    return f
    return None


def source_sha(fname: str) -> str:
    with open(os.path.join(CSRC, fname), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def per_dispatch(csv_path: str, counter: str):
    """kernel -> list of counter values (one per dispatch)."""
    out = collections.defaultdict(list)
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] == counter:
            out[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return out


def cmd_kernels(a):
    rows = list(csv.DictReader(open(a.stats)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# {a.title}", "", "Command (from the repository root on the GPU host, `$R` = repository root):", "",
             "```", a.command, "```", "", f"Per step = total / {a.steps} timed+warm-up steps profiled.", ""]
    if a.note:
        lines += [a.note, ""]
    lines += ["| Kernel | Calls | Total ms | Avg us | % of summed kernel time |", "|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| {short_name(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {100 * float(r['TotalDurationNs']) / total:.2f} |")
    open(a.out, "w").write("\n".join(lines) + "\n")


def cmd_traffic(a):
    fetch = per_dispatch(a.fetch, "FETCH_SIZE")
    write = per_dispatch(a.write, "WRITE_SIZE")
    cf = per_dispatch(a.copy_fetch, "FETCH_SIZE")
    cw = per_dispatch(a.copy_write, "WRITE_SIZE")
    copy_kib = a.copy_bytes / 1024.0

    def copy_factor(d):
        vals = [v for k, vs in d.items() for v in vs if v > copy_kib / 4]  # the 1 GiB copy dispatches
        return copy_kib / (sum(vals) / len(vals))

    ff, fw = copy_factor(cf), copy_factor(cw)
    lines = [f"# {a.title}", "", "Commands (from the repository root on the GPU host, `$R` = repository root):", "",
             "```"] + list(a.commands) + ["```", "",
             f"Calibration: a {a.copy_bytes} B device copy reads {copy_kib / ff:.1f} KiB on FETCH_SIZE and writes "
             f"{copy_kib / fw:.1f} KiB on WRITE_SIZE, so HBM bytes = FETCH_SIZE x {ff:.3f} KiB and WRITE_SIZE x "
             f"{fw:.3f} KiB.", "",
             "| Kernel | Dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM read MB | HBM write MB |",
             "|---|---|---|---|---|---|"]
    rec = {"calibration": {"copy_bytes": a.copy_bytes, "fetch_factor": ff, "write_factor": fw}, "kernels": {}}
    for k in sorted(set(fetch) | set(write)):
        f = sum(fetch.get(k, [0])) / max(1, len(fetch.get(k, [0])))
        w = sum(write.get(k, [0])) / max(1, len(write.get(k, [0])))
        rd, wr = f * ff * 1024, w * fw * 1024
        lines.append(f"| {k} | {len(fetch.get(k, []))} | {f:.1f} | {w:.1f} | {rd / 1e6:.1f} | {wr / 1e6:.1f} |")
        src = source_of(k)
        rec["kernels"][k] = {"fetch_kib": f, "write_kib": w, "read_bytes": rd, "write_bytes": wr,
                             "source": src, "source_sha256": source_sha(src) if src else None}
    open(a.out, "w").write("\n".join(lines) + "\n")
    json.dump(rec, open(a.json, "w"), indent=1, sort_keys=True)


def cmd_counters(a):
    vals = collections.defaultdict(list)
    for r in csv.DictReader(open(a.csv)):
        if a.kernel in r["Kernel_Name"]:
            vals[r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = [f"# {a.title}", "", "Command (from the repository root on the GPU host, `$R` = repository root):", "",
             "```", a.command, "```", "", f"Per dispatch of {a.kernel} (mean over {max(map(len, vals.values()))} "
             "dispatches).", "", "| Counter | Value |", "|---|---|"]
    for k in sorted(vals):
        lines.append(f"| {k} | {sum(vals[k]) / len(vals[k]):.4e} |")
    open(a.out, "w").write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("--stats", required=True)
    k.add_argument("--steps", type=int, default=1)
    k.add_argument("--title", required=True)
    k.add_argument("--command", required=True)
    k.add_argument("--out", required=True)
    k.add_argument("--note", default="", help="a paragraph printed above the table")
    t = sub.add_parser("traffic")
    for x in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--title", "--out", "--json"):
        t.add_argument(x, required=True)
    t.add_argument("--copy-bytes", type=int, default=1 << 30)
    t.add_argument("--commands", nargs="+", required=True)
    c = sub.add_parser("counters")
    for x in ("--csv", "--kernel", "--title", "--command", "--out"):
        c.add_argument(x, required=True)
    a = ap.parse_args()
    {"kernels": cmd_kernels, "traffic": cmd_traffic, "counters": cmd_counters}[a.what](a)


if __name__ == "__main__":
    main()
