#!/usr/bin/env python3
"""Compact-Table propagation benchmark on one MI355X.

Workload (one large table): arity 5, every domain of size 50, 200,000
distinct uniform tuples (3,125 uint64 words per support row), driven by a
simulated search of 1,000 propagate calls; each call removes 5 % of the
remaining values (rounded up) of 1-3 random variables, a level is pushed
before every call and every 10th call pops U{1..depth} levels (one level
after a failure).  The call script is drawn once, untimed, from the
library's own results; one timed step replays the whole script from the root
state through the C ABI (push, propagate, pop), so every propagate is a
synchronous host call with its domain bitmaps crossing the boundary.

Printed: one JSON line with propagations/s (`value`), p50/p99 call latency,
the propagate kernel's HIP-event duration against the HBM roofline, and the
CPU oracle timed on a bounded sample of the same script.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--seed", type=int, default=None)
    p.add_argument("--calls", type=int, default=1000)
    p.add_argument("--cpu-seconds", type=float, default=10.0)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--nodes", type=int, default=4096)
    p.add_argument("--no-nodes", action="store_true")
    return p.parse_args()


class GpuSut:
    def __init__(self, table):
        self.t = table

    def propagate(self, dom_in):
        st, dom_out = self.t.propagate(dom_in)
        return st, dom_out

    def push(self):
        assert self.t.push() == 0

    def pop(self):
        assert self.t.pop() == 0

    def domains(self):
        return self.t.domains()


def replay(table, script, lat=None):
    """Run the recorded operations; returns the number of propagate calls."""
    import numpy as np
    n = 0
    for kind, payload in script:
        if kind == "push":
            table.push()
        elif kind == "pop":
            table.pop()
        else:
            if lat is not None:
                t0 = time.perf_counter()
                table.propagate(payload)
                lat.append(time.perf_counter() - t0)
            else:
                table.propagate(payload)
            n += 1
    return n


def algorithmic_bytes(d_stats, D, calls):
    """Bytes the method must move for the counted work:
    every active granule reads its k support-row segments and its currTable
    words and writes the words back; each trailed granule saves 64 words and
    a header; each residue check reads two words; each scanned granule reads
    64 currTable and 64 support words; domain words cross in and out."""
    g = 512
    return (g * d_stats["granule_rows"] + 2 * g * d_stats["granules_in"] + 520 * d_stats["trail_granules"]
            + 16 * d_stats["residue_checks"] + 2 * g * d_stats["scan_granules"] + 16 * D * calls)


def cpu_baseline(spec, script, seconds):
    from oracle import oracle as O
    o = O.OracleTable(spec.tuples, spec.lo, spec.dsizes)
    props = 0
    passes = 0
    t0 = time.perf_counter()
    while True:
        for kind, payload in script:
            if kind == "push":
                o.push()
            elif kind == "pop":
                o.pop()
            else:
                o.propagate(payload)
                props += 1
        passes += 1
        el = time.perf_counter() - t0
        if el >= seconds or passes >= 50:
            break
    while o.depth > 0:
        o.pop()
    return props / el, props, el, passes


def nodes_leg(seed, n_nodes, reps, warmup, schedule=0):
    """Batched CT across search nodes: one arity-6 table with 1,000,000 Zipf
    tuples, n_nodes independent domain states (each removes a random 0-60 %
    of every variable's values), all propagated from the root state in one
    launch with per-node currTable copies in HBM."""
    import numpy as np
    import torch
    from paper_2507_18413_amd import ct
    from paper_2507_18413_amd import workloads as W
    spec = W.config4_table(seed)
    lay = spec.layout()
    table = ct.Table(spec.tuples, spec.lo, spec.dsizes, max_depth=0, schedule=schedule)
    root = table.domains()
    nodes = W.config4_nodes(lay, root, n_nodes, seed)
    first = table.slots_alloc(n_nodes, max_depth=0)
    din = torch.from_numpy(nodes.view(np.int64)).cuda()
    dout = torch.zeros_like(din)
    status = torch.zeros(n_nodes, dtype=torch.int32, device="cuda")
    jobs = [dict(table=table, slot=first + k, flags=ct.JOB_PROPAGATE | ct.JOB_FROM_ROOT,
                 dom_in=din[k], dom_out=dout[k]) for k in range(n_nodes)]
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        ct.propagate_batch(jobs, status, stream)
    torch.cuda.synchronize()
    s0 = [table.stats(first + k) for k in (0,)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(reps):
        ct.propagate_batch(jobs, status, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ct.batch_status(stream)
    gpu_ms = e0.elapsed_time(e1) / reps
    st = status.cpu().numpy()
    # algorithmic bytes of one batch: compulsory traffic = supports once +
    # root currTable once + per node currTable write + domains
    W_words = table.W
    comp = 8 * table.rows * W_words + 8 * W_words + n_nodes * (8 * W_words + 16 * lay.D)
    return {
        "nodes": n_nodes, "tuples": spec.t, "ms_per_batch": round(gpu_ms, 3),
        "node_props_per_s": round(n_nodes / (gpu_ms / 1e3), 1),
        "wall_ms_per_batch": round(wall / reps * 1e3, 3),
        "status_counts": {int(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))},
        "compulsory_bytes": comp,
        "compulsory_GBps": round(comp / (gpu_ms / 1e3) / 1e9, 1),
        "frac_of_hbm_peak": round(comp / (gpu_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the library runs "
              f"on a single MI355X; see DESIGN.md for how the path would shard)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2507_18413_amd import ct
    from paper_2507_18413_amd import workloads as W

    seed = W.DEFAULT_SEED if args.seed is None else args.seed
    torch.cuda.set_device(0)
    spec = W.config2_table(seed)
    lay = spec.layout()
    table = ct.Table(spec.tuples, spec.lo, spec.dsizes)
    # record the call script from the library's own answers (untimed)
    script = W.run_plain_script(GpuSut(table), lay, args.calls, seed, 2, W.pick_fraction_removal)
    depth = sum(1 if k == "push" else -1 if k == "pop" else 0 for k, _ in script)
    for _ in range(depth):
        script.append(("pop", None))
        table.pop()
    n_calls = sum(1 for k, _ in script if k == "prop")

    for _ in range(args.warmup):
        replay(table, script)
    torch.cuda.synchronize()
    s0 = table.stats()
    table.set_timing(True)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    props = 0
    for _ in range(args.steps):
        props += replay(table, script, lat)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernel_ms, launches = table.timing()
    table.set_timing(False)
    s1 = table.stats()
    d = {k: s1[k] - s0[k] for k in s1}
    elapsed = t1 - t0
    value = props / elapsed
    lat_us = np.array(lat) * 1e6
    bytes_total = algorithmic_bytes(d, lay.D, props)
    per_launch_bytes = bytes_total / max(launches, 1)
    avg_kernel_s = kernel_ms / 1e3 / max(launches, 1)
    achieved = per_launch_bytes / avg_kernel_s / 1e9 if avg_kernel_s > 0 else 0.0

    out = {
        "metric": "CT propagations/sec (plain calls, one large table)",
        "value": round(value, 1),
        "unit": "propagations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "plain CT, one table: arity 5, |dom| 50, 200000 distinct uniform tuples, "
                        "3125 words per support row; 1000 propagate calls removing 5% of the values "
                        "of 1-3 variables, push before every call, pop U{1..depth} every 10 calls",
            "tuples": spec.t, "arity": spec.n, "dom_size": 50, "calls_per_step": n_calls, "seed": seed,
        },
        "latency_us": {"p50": round(float(np.percentile(lat_us, 50)), 2),
                       "p99": round(float(np.percentile(lat_us, 99)), 2),
                       "mean": round(float(lat_us.mean()), 2)},
        "kernel": {"name": "ctk::propagate_kernel", "launches": launches,
                   "avg_us": round(avg_kernel_s * 1e6, 3),
                   "support_words_per_s": round(d["granule_rows"] * 64 / elapsed, 1)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                     "bytes_per_launch": round(per_launch_bytes, 1)},
    }
    if not args.no_nodes:
        out["batched_nodes"] = nodes_leg(seed, args.nodes, max(1, args.steps), 1)
    if not args.no_cpu_baseline:
        cps, cprops, cel, passes = cpu_baseline(spec, script, args.cpu_seconds)
        out["cpu_baseline"] = {"value": round(cps, 1), "unit": "propagations/s", "cores": 1, "kind": "oracle",
                               "sample": f"{passes} replays of the same {n_calls}-call script "
                                         f"({cprops} propagations, {cel:.1f} s, 1 thread)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
