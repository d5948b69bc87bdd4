"""Summaries of rocprofv3 runs of bench.py, written under profiles/.

    python -m paper_2507_18413_amd.profiling summarize \
        --stats DIR/c2_kernel_stats.csv \
        --fetch DIRF/c2_counter_collection.csv --write DIRW/c2_counter_collection.csv \
        --copy-bytes N --command "..." --out profiles/propagate_large_table.md

The kernel-trace statistics give the chosen kernel's (--kernel, a regular
expression; default the propagate kernel) average duration.
The two counter runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) are
scaled by what the same counter reads for a plain copy kernel of known size
(the runtime's device-to-device copyBuffer kernel of `--copy-bytes` bytes,
run by `bench.py --calibration-copy`)
and give HBM bytes per launch.  The summary ends with a JSON line that
bench.py reads back, keyed by the SHA-256 of the kernel source, so the
traffic figure is dropped as soon as the kernel changes.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRCS = [os.path.join(HERE, "csrc", "ct_kernels.hip"), os.path.join(HERE, "csrc", "ct_engine.hip")]
KERNEL = "propagate_kernel"
DEFAULT_TITLE = "propagate_kernel, one 200,000-tuple table"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def counter_by_kernel(path, counter, largest=False):
    """Mean (or largest) counter value per dispatch, per kernel name."""
    vals = {}
    for r in _rows(path):
        name = r.get("Kernel_Name", "")
        if r.get("Counter_Name", counter) != counter:
            continue
        v = float(r.get("Counter_Value", "nan"))
        vals.setdefault(name, {}).setdefault(r.get("Dispatch_Id", len(vals)), 0.0)
        vals[name][r.get("Dispatch_Id")] += v
    agg = max if largest else statistics.mean
    return {k: (agg(d.values()), len(d)) for k, d in vals.items()}


def pick(d, pattern):
    for k, v in d.items():
        if re.search(pattern, k):
            return k, v
    return None, None


def summarize(args):
    kernel = args.kernel
    stats = _rows(args.stats)
    prop = [r for r in stats if re.search(kernel, r["Name"])][0]
    avg_ns = float(prop["AverageNs"])
    out = {"kernel": prop["Name"], "calls": int(prop["Calls"]), "avg_us": round(avg_ns / 1e3, 3),
           "min_us": round(float(prop["MinNs"]) / 1e3, 3), "max_us": round(float(prop["MaxNs"]) / 1e3, 3),
           "kernel_source_sha256": kernel_source_hash()}
    if args.calls_traced:
        # a resident kernel serves many calls per dispatch: its dispatches'
        # whole lifetimes over the calls they served
        out["calls_traced"] = args.calls_traced
        out["dispatch_us_per_call"] = round(avg_ns * int(prop["Calls"]) / 1e3 / args.calls_traced, 3)
    lines = [f"# {args.title}", "", f"Command (from the repository root): `{args.command}`", "",
             "Kernel-trace statistics (rocprofv3 --kernel-trace --stats):", "",
             "| kernel | calls | avg µs | min µs | max µs | share |", "|---|---|---|---|---|---|"]
    for r in stats[:6]:
        lines.append(f"| {r['Name'][:60]} | {r['Calls']} | {float(r['AverageNs'])/1e3:.3f} | "
                     f"{float(r['MinNs'])/1e3:.3f} | {float(r['MaxNs'])/1e3:.3f} | {float(r['Percentage']):.2f} % |")
    if args.calls_traced:
        lines += ["", f"* {prop['Name'][:60]}: {out['calls']} dispatches served the {args.calls_traced} calls of the "
                      f"traced run: {out['dispatch_us_per_call']:.3f} µs of dispatch lifetime per call"]
    if args.fetch and args.write and args.copy_bytes:
        f = counter_by_kernel(args.fetch, "FETCH_SIZE")
        w = counter_by_kernel(args.write, "WRITE_SIZE")
        _, (kf, nf) = pick(f, kernel)
        _, (kw, nw) = pick(w, kernel)
        # the calibration copy is the largest copyBuffer dispatch of the run
        cname, (cf, _) = pick(counter_by_kernel(args.fetch, "FETCH_SIZE", largest=True), r"copyBuffer")
        _, (cw, _) = pick(counter_by_kernel(args.write, "WRITE_SIZE", largest=True), r"copyBuffer")
        kib = args.copy_bytes / 1024.0
        ffac, wfac = cf / kib, cw / kib
        traffic = kf / ffac * 1024 + kw / wfac * 1024
        out.update({"fetch_kib_per_launch": round(kf, 2), "write_kib_per_launch": round(kw, 2),
                    "copy_kernel": cname, "copy_fetch_factor": round(ffac, 4),
                    "copy_write_factor": round(wfac, 4), "hbm_bytes_per_launch": round(traffic, 1),
                    "dispatches_fetch": nf, "dispatches_write": nw})
        if args.calls:
            # a resident kernel serves many calls per dispatch: all its
            # dispatches' bytes over all the calls of the counted runs
            per_call = (kf * nf / ffac + kw * nw / wfac) * 1024 / args.calls
            out["hbm_bytes_per_call"] = round(per_call, 1)
            out["calls_counted"] = args.calls
        lines += ["", "HBM traffic (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE; KiB per dispatch):", "",
                  f"* {prop['Name'][:60]}: FETCH {kf:.2f} KiB, WRITE {kw:.2f} KiB per launch "
                  f"({nf} / {nw} dispatches)",
                  f"* calibration copy of {args.copy_bytes} bytes ({cname[:50]}): FETCH reads {cf:.1f} KiB "
                  f"(factor {ffac:.3f}), WRITE reads {cw:.1f} KiB (factor {wfac:.3f})",
                  f"* scaled HBM bytes per launch of that kernel: {traffic:.0f}"]
    if "hbm_bytes_per_call" in out:
        lines += [f"* over all {out['dispatches_fetch']} dispatches and the {args.calls} calls they served "
                  f"(counter runs): {out['hbm_bytes_per_call']:.0f} HBM bytes per call"]
    lines += ["", "Machine-readable (read by bench.py while the kernel source hash matches):", "",
              "```json", json.dumps(out), "```", ""]
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


def read_summary(path):
    """The JSON block of a summary, or None if absent / the kernel changed."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return d


def main():
    p = argparse.ArgumentParser()
    sub = p.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("summarize")
    s.add_argument("--stats", required=True)
    s.add_argument("--fetch")
    s.add_argument("--write")
    s.add_argument("--copy-bytes", type=int, default=0)
    s.add_argument("--command", required=True)
    s.add_argument("--kernel", default=KERNEL, help="regular expression naming the kernel")
    s.add_argument("--calls", type=int, default=0,
                   help="calls served by the kernel's dispatches in each counter run (resident kernels)")
    s.add_argument("--calls-traced", type=int, default=0,
                   help="calls served by the kernel's dispatches in the kernel-trace run (resident kernels)")
    s.add_argument("--title", default=DEFAULT_TITLE)
    s.add_argument("--out", required=True)
    a = p.parse_args()
    if a.cmd == "summarize":
        summarize(a)


if __name__ == "__main__":
    main()
