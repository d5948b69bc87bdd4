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
the propagate kernel's device-clock duration against the HBM roofline, the
batched legs (4,096 search nodes in one launch; a 2,000-table model solved to
a fixpoint per search step, batched vs one launch per table vs the CPU
oracle), and the CPU oracle timed on a bounded sample of the same script.
"""
import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
LDS_PEAK_GBS = 256 * 128 * 2.4  # 256 CUs x 128 B/clock x 2.4 GHz
MAX_DEPTH_SERVE = 64  # push levels per serving slot


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--seed", type=int, default=None)
    p.add_argument("--calls", type=int, default=1000)
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--nodes", type=int, default=4096)
    p.add_argument("--no-nodes", action="store_true")
    p.add_argument("--model-steps", type=int, default=100)
    p.add_argument("--no-serve", action="store_true")
    p.add_argument("--serve-requests", type=int, default=200_000)
    p.add_argument("--serve-rate", type=float, default=20_000.0)
    p.add_argument("--serve-budget", type=int, default=0)
    p.add_argument("--calibration-copy", type=int, default=0,
                   help="MiB copied once by torch before the timed run (counter calibration)")
    p.add_argument("--no-model", action="store_true")
    p.add_argument("--no-wide", action="store_true")
    p.add_argument("--no-split", action="store_true")
    p.add_argument("--wide-only", action="store_true",
                   help="only the wide-scope leg, without its split propagators (profiling)")
    p.add_argument("--no-driver", action="store_true")
    p.add_argument("--no-tiny", action="store_true", help="skip the tiny-table leg (profiling the plain leg)")
    p.add_argument("--no-probe", action="store_true", help="skip the device copy probe")
    p.add_argument("--no-paper-shape", action="store_true")
    p.add_argument("--nodes-only", action="store_true",
                   help="only the search-node batches (4,096 nodes, 1,000,000-tuple Zipf table; profiling)")
    p.add_argument("--root-batch-only", action="store_true",
                   help="only the batched root recomputation of the 2,000-table model (profiling)")
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


def oracle_bytes(st, D):
    """Algorithmic bytes of one call from the oracle's own counts (the
    word-level form: support words read by updateTable, currTable words read
    and written, a support word per residue check and per scanned word, the
    domain words in and out)."""
    return (8 * st["update_words"] + 16 * st["nonzero_words_in"] + 8 * (st["residue_checks"] + st["scan_words"])
            + 16 * D)


def cpu_baseline(spec, script, seconds, fast=True):
    """The oracle replaying the script on one host thread: (props/s, props,
    seconds, passes, support words read per call, algorithmic bytes per call)."""
    from oracle import oracle as O
    o = O.OracleTable(spec.tuples, spec.lo, spec.dsizes, fast=fast)
    D = spec.layout().D
    props = 0
    passes = 0
    words = byts = 0
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
                if passes == 0:
                    st = o.last_stats()
                    words += st["update_words"] + st["scan_words"] + st["residue_checks"]
                    byts += oracle_bytes(st, D)
        passes += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    while o.depth > 0:
        o.pop()
    n1 = sum(1 for k, _ in script if k == "prop")
    return props / el, props, el, passes, words / max(n1, 1), byts / max(n1, 1)


def nodes_oracle_threads(spec, nodes, threads, seconds):
    """Oracle (fast mode) propagations of the node states on `threads` host
    threads (the oracle's calls release the interpreter lock), each thread
    with its own oracle table; a bounded prefix of the nodes.  Returns
    (nodes done, seconds, threads)."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    tabs = [O.OracleTable(spec.tuples, spec.lo, spec.dsizes, fast=True) for _ in range(threads)]
    n = len(nodes)

    def work(k, stop):
        o = tabs[k]
        done = 0
        for i in range(k, n, threads):
            if time.perf_counter() > stop:
                break
            o.push()
            o.propagate(nodes[i])
            o.pop()
            done += 1
        return done

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        done = sum(ex.map(lambda k: work(k, t0 + seconds), range(threads)))
    return done, time.perf_counter() - t0, threads


def nodes_leg(seed, n_nodes, reps, warmup, schedule=0, plain=True, cpu=False):
    """Batched CT across search nodes: one arity-6 table with 1,000,000 Zipf
    tuples, n_nodes independent domain states (each removes a random 0-60 %
    of every variable's values), all propagated from the root state in one
    launch with per-node currTable copies in HBM."""
    import numpy as np
    import torch
    from paper_2507_18413_amd import ct
    from paper_2507_18413_amd import workloads as W
    spec = W.zipf_table(seed)
    lay = spec.layout()
    table = ct.Table(spec.tuples, spec.lo, spec.dsizes, max_depth=0, schedule=schedule)
    root = table.domains()
    nodes = W.node_states(lay, root, n_nodes, seed)
    first = table.slots_alloc(n_nodes, max_depth=0)
    din = torch.from_numpy(nodes.view(np.int64)).cuda()
    dout = torch.zeros_like(din)
    status = torch.zeros(n_nodes, dtype=torch.int32, device="cuda")
    jobs = ct.Batch([dict(table=table, slot=first + k, flags=ct.JOB_PROPAGATE | ct.JOB_FROM_ROOT,
                          dom_in=din[k], dom_out=dout[k]) for k in range(n_nodes)])
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        ct.propagate_batch(jobs, status, stream)
    torch.cuda.synchronize()
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
    # the update kernel reads one 512-byte granule of a support row from LDS
    # per (node, selected row, active granule); the slots are fresh, so their
    # counters cover exactly the warmup and timed batches
    lds_bytes = 512 * sum(table.stats(first + k)["granule_rows"] for k in range(n_nodes)) / (warmup + reps)
    st = status.cpu().numpy()
    # algorithmic bytes of one batch: compulsory traffic = supports once +
    # root currTable once + per node currTable write + domains
    W_words = table.W
    comp = 8 * table.rows * W_words + 8 * W_words + n_nodes * (8 * W_words + 16 * lay.D)
    from paper_2507_18413_amd import profiling
    prof = profiling.read_summary(os.path.join(ROOT, "profiles", "nodes_update_4096_nodes.md"))
    extra = {}
    if plain:
        # the same node states, one launch per node (a one-job batch on the
        # same table: updateTable split over workgroups, then filterDomains)
        singles = [ct.Batch([dict(table=table, slot=first + k, flags=ct.JOB_PROPAGATE | ct.JOB_FROM_ROOT,
                                  dom_in=din[k], dom_out=dout[k])]) for k in range(n_nodes)]
        for b in singles[:8]:
            b.run(status[:1], stream)
        torch.cuda.synchronize()
        e0.record(stream)
        p0 = time.perf_counter()
        for k, b in enumerate(singles):
            b.run(status[k:k + 1], stream)
        e1.record(stream)
        torch.cuda.synchronize()
        pwall = time.perf_counter() - p0
        ct.batch_status(stream)
        pms = e0.elapsed_time(e1)
        same = bool((status.cpu().numpy() == st).all())
        extra["plain_one_launch_per_node"] = {
            "ms_total": round(pms, 3), "node_props_per_s": round(n_nodes / (pms / 1e3), 1),
            "wall_ms_total": round(pwall * 1e3, 3), "same_statuses_as_batch": same,
            "batched_speedup": round(pms / gpu_ms, 1)}
    if cpu:
        hi = host_info()
        thr = max(1, min(16, hi["usable_cores"] or 1))
        done, sec, thr = nodes_oracle_threads(spec, nodes, thr, 8.0)
        extra["oracle_all_cores"] = {"node_props_per_s": round(done / sec, 1), "threads": thr,
                                     "sample": f"{done} of the {n_nodes} node states in {sec:.1f} s, "
                                               "fast mode, one oracle table per thread"}
    return {**extra, 
        "nodes": n_nodes, "tuples": spec.t, "ms_per_batch": round(gpu_ms, 3),
        "node_props_per_s": round(n_nodes / (gpu_ms / 1e3), 1),
        "wall_ms_per_batch": round(wall / reps * 1e3, 3),
        "status_counts": {int(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))},
        "compulsory_bytes": comp,
        "compulsory_GBps": round(comp / (gpu_ms / 1e3) / 1e9, 1),
        "frac_of_hbm_peak": round(comp / (gpu_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "update_kernel_hbm_bytes": prof.get("hbm_bytes_per_launch") if prof else None,
        "update_kernel_avg_us_profiled": prof.get("avg_us") if prof else None,
        "update_kernel_lds_bytes": lds_bytes,
        "update_kernel_lds_roofline": None if not prof else {
            "bound": "lds", "achieved": round(lds_bytes / prof["avg_us"] / 1e3, 1), "peak": LDS_PEAK_GBS,
            "unit": "GB/s", "frac": round(lds_bytes / prof["avg_us"] / 1e3 / LDS_PEAK_GBS, 4)},
    }


class PlainModel:
    """AC-3 over the tables on the host, one synchronous GPU call per table
    propagation (the one-constraint-per-launch baseline)."""

    def __init__(self, tables, scopes, lay):
        import numpy as np
        self.t, self.sc, self.lay = tables, scopes, lay
        self.last = [t.domains() for t in tables]
        self.stack = []
        self.nbr = {}
        for c, sc in enumerate(scopes):
            for v in sc:
                self.nbr.setdefault(int(v), []).append(c)

    def push(self):
        for t in self.t:
            t.push()
        self.stack.append([x.copy() for x in self.last])

    def pop(self):
        for t in self.t:
            t.pop()
        self.last = self.stack.pop()

    def fixpoint(self, pool, seed=None):
        """AC-3 from `pool`; seed: the tables to start from (default all; a
        step after a fixpoint needs only the tables touching a changed
        variable, the rule the batched model's first round follows)."""
        import numpy as np
        from collections import deque
        lay = self.lay
        pool = pool.copy()
        start = range(len(self.t)) if seed is None else seed
        q = deque(start)
        inq = [False] * len(self.t)
        for c in start:
            inq[c] = True
        props = 0
        while q:
            c = q.popleft()
            inq[c] = False
            tb, sc, last = self.t[c], self.sc[c], self.last[c]
            din = np.concatenate([pool[lay.off[v]: lay.off[v] + lay.words[v]] for v in sc]) & last
            st, dout = tb.propagate(din)
            props += 1
            if st != 0:
                return st, pool, props
            self.last[c] = dout
            o = 0
            for v in sc:
                nw = int(lay.words[v])
                seg = dout[o: o + nw]
                if (pool[lay.off[v]: lay.off[v] + nw] != seg).any():
                    pool[lay.off[v]: lay.off[v] + nw] = seg
                    for c2 in self.nbr[int(v)]:
                        if c2 != c and not inq[c2]:
                            q.append(c2)
                            inq[c2] = True
                o += nw
        return 0, pool, props


def wide_leg(seed, n_calls, cpu, split=True, paper_shape=False):
    """Plain calls on a wide-scope table, where filterDomains dominates: 100
    variables, domains 64-160, 10,000 tuples (the shape of the paper's
    linear instances), or with paper_shape 150 variables, domains up to
    2,000, 15,000 tuples (the size of its Gecode comparison set)."""
    import numpy as np
    from paper_2507_18413_amd import ct
    from paper_2507_18413_amd import workloads as W
    spec = W.paper_shape_table(seed) if paper_shape else W.wide_table(seed)
    lay = spec.layout()
    # the recorder runs the schedule the timed table gets, so a profile of
    # the leg averages one kind of launch
    rec = ct.Table(spec.tuples, spec.lo, spec.dsizes, schedule=ct.SCHED_SPLIT)
    script = W.run_plain_script(GpuSut(rec), lay, n_calls, seed, 6, W.pick_fraction_removal)
    rec.close()
    depth = sum(1 if k == "push" else -1 if k == "pop" else 0 for k, _ in script)
    script += [("pop", None)] * depth
    table = ct.Table(spec.tuples, spec.lo, spec.dsizes)
    replay(table, script)
    s0 = table.stats()
    table.set_timing(True)
    t0 = time.perf_counter()
    props = replay(table, script)
    el = time.perf_counter() - t0
    kernel_ms, launches = table.timing()
    life_ms, dispatches = table.dispatch_timing() if table.resident_split else (None, None)
    table.set_timing(False)
    s1 = table.stats()
    d = {k: s1[k] - s0[k] for k in s1}
    byts = algorithmic_bytes(d, lay.D, props)
    lat = []  # latencies from one more replay, outside the timed one
    replay(table, script, lat)
    lat_us = np.array(lat) * 1e6
    from paper_2507_18413_amd import profiling
    prof = profiling.read_summary(os.path.join(ROOT, "profiles", "split_engine_wide_scope.md" if table.resident_split
                                               else "propagate_wide_scope.md"))
    split_out = split_leg(table, script, 1) if split else None
    shape = ("arity 150, domains U{2..2000}, 15,000 distinct uniform tuples" if paper_shape else
             "arity 100, domains U{64..160}, 10,000 distinct uniform tuples")
    out = {"workload": f"{shape} ({table.rows} support rows of {table.W} words, {table.D} domain words); "
                       f"{n_calls} calls as in the plain leg",
           "props_per_s": round(props / el, 1),
           "latency_us": {"p50": round(float(np.percentile(lat_us, 50)), 2),
                          "p99": round(float(np.percentile(lat_us, 99)), 2)},
           "kernel": {"name": "ctk::engine_kernel" if table.resident else
                      "ctk::split_engine_kernel" if table.resident_split else "ctk::propagate_kernel",
                      "calls_timed": launches,
                      # the resident split schedule: workgroup 0's time per
                      # call (receipt to the hand-over to the filters); the
                      # launched one: each launch's first start to last end
                      "device_us_per_call" if not table.resident_split else "update_us_per_call":
                          round(kernel_ms * 1e3 / max(launches, 1), 3),
                      "algorithmic_bytes_per_call": round(byts / max(props, 1), 1),
                      "algorithmic_GBps": round(byts / ((life_ms if table.resident_split else kernel_ms) / 1e3)
                                                / 1e9, 2) if kernel_ms > 0 else None,
                      "profiled_hbm_bytes_per_launch" if not table.resident_split else "profiled_hbm_bytes_per_call":
                          (prof.get("hbm_bytes_per_call") if table.resident_split else
                           prof.get("hbm_bytes_per_launch")) if prof else None,
                      "profiled_avg_us": prof.get("avg_us") if prof else None,
                      "counters_per_call": {k: round(v / max(props, 1), 1) for k, v in d.items()}},
           "schedule": "resident split" if table.resident_split else "resident engine" if table.resident
           else "launched",
           "split_propagators": split_out}
    if table.resident_split:
        # launch lifetimes over the calls they served (the waits for the
        # host's next call included)
        out["kernel"]["launches"] = dispatches
        out["kernel"]["launch_us_per_call"] = round(life_ms * 1e3 / max(launches, 1), 3)
    if cpu:
        from oracle import oracle as O
        for fast in (True, False):
            o = O.OracleTable(spec.tuples, spec.lo, spec.dsizes, fast=fast)

            class OracleSut:
                def propagate(self, d):
                    return o.propagate(d)

                def push(self):
                    o.push()

                def pop(self):
                    o.pop()

            t0 = time.perf_counter()
            oprops = replay(OracleSut(), script)
            out["oracle_fast_props_per_s" if fast else "oracle_plain_props_per_s"] = \
                round(oprops / (time.perf_counter() - t0), 1)
    table.close()
    return out


def tiny_leg(seed, reps, cpu):
    """Plain calls on the tiny table (arity 3, domains {0..7}, 200 distinct
    tuples; one currTable granule): 100 calls removing 1-2 values each, with
    push / pop every 10 calls -- launch-latency bound: latency p50 / p99 and
    calls/s (a roofline fraction means nothing at 768 bytes per call)."""
    import numpy as np
    from paper_2507_18413_amd import ct
    from paper_2507_18413_amd import workloads as W
    spec = W.tiny_table(seed)
    lay = spec.layout()
    rec = ct.Table(spec.tuples, spec.lo, spec.dsizes, schedule=ct.SCHED_SOLO)
    script = W.run_plain_script(GpuSut(rec), lay, 100, seed, 1, W.pick_small_removal)
    rec.close()
    depth = sum(1 if k == "push" else -1 if k == "pop" else 0 for k, _ in script)
    script += [("pop", None)] * depth
    table = ct.Table(spec.tuples, spec.lo, spec.dsizes)
    for _ in range(3):
        replay(table, script)
    t0 = time.perf_counter()
    props = sum(replay(table, script) for _ in range(reps))
    el = time.perf_counter() - t0
    lat = []  # latencies from as many more replays, outside the timed ones
    for _ in range(reps):
        replay(table, script, lat)
    lat_us = np.array(lat) * 1e6
    out = {"workload": "arity 3, domains {0..7}, 200 distinct tuples, 100 calls removing 1-2 values, "
                       "push before every call, pop U{1..depth} every 10 calls",
           "calls": props, "props_per_s": round(props / el, 1),
           "latency_us": {"p50": round(float(np.percentile(lat_us, 50)), 2),
                          "p99": round(float(np.percentile(lat_us, 99)), 2)},
           "schedule": "resident engine" if table.resident else "resident split" if table.resident_split
           else "launched"}
    if cpu:
        from oracle import oracle as O
        o = O.OracleTable(spec.tuples, spec.lo, spec.dsizes, fast=True)

        class OracleSut:
            def propagate(self, d):
                return o.propagate(d)

            def push(self):
                o.push()

            def pop(self):
                o.pop()

        t0 = time.perf_counter()
        oprops = sum(replay(OracleSut(), script) for _ in range(reps))
        out["oracle_fast_props_per_s"] = round(oprops / (time.perf_counter() - t0), 1)
    table.close()
    return out


def split_leg(table, script, passes):
    """The same call script through the two split propagators of the table
    (updateTable or filterDomains on the device, the other procedure on the
    host; one copy in per call, results written by the device into pinned
    host memory)."""
    import numpy as np
    from paper_2507_18413_amd import ct
    out = {}
    for name, mode in (("update_on_device", ct.SPLIT_UPDATE), ("filter_on_device", ct.SPLIT_FILTER)):
        sp = ct.SplitPropagator(table, mode)
        bad = []

        class Counted:
            """Counts error statuses (a propagator that went wrong answers
            every later call with an error, quickly)."""

            def propagate(self, d):
                st = sp.propagate(d)[0]
                if st < 0:
                    bad.append(st)

            def push(self):
                sp.push()

            def pop(self):
                sp.pop()

        replay(Counted(), script)
        lat = []
        t0 = time.perf_counter()
        props = sum(replay(Counted(), script, lat) for _ in range(passes))
        el = time.perf_counter() - t0
        lat_us = np.array(lat) * 1e6
        out[name] = {"props_per_s": round(props / el, 1),
                     "latency_us": {"p50": round(float(np.percentile(lat_us, 50)), 2),
                                    "p99": round(float(np.percentile(lat_us, 99)), 2)},
                     "error_statuses": len(bad)}
        sp.close()
    return out


def solver_leg(seed, cpu, n=100, dom=(2, 160), t=10_000):
    """A complete search of an instance in the form of the paper's first test
    set (Sec. 5.1): one table constraint over all n item-count variables of a
    bounded knapsack (t distinct configurations) and one linear equation
    over all of them (the form of the Gecode comparison set, Sec. 5.3),
    input order and largest value first, all solutions.  The table is one
    ct.Table on the GPU (synchronous calls); the equation is propagated on
    the host.  The same search with the oracle's table (fast mode) beside it
    must explore the same tree."""
    from paper_2507_18413_amd import ct
    from paper_2507_18413_amd import solver as S
    from paper_2507_18413_amd import workloads as W
    spec, E, w, c = W.lin_instance(seed, n=n, dom=dom, t=t, eq_frac=1.0)
    lay = spec.layout()
    table = ct.Table(spec.tuples, spec.lo, spec.dsizes, max_depth=max(256, n + 8))
    prop = S.OneTable(table)
    g = S.Search(lay, prop, S.LinearEQ(lay, E, w, c), var_order="input", val_order="max")
    t0 = time.perf_counter()
    g.run(lay.full(), 10 ** 7, 10 ** 7)
    el = time.perf_counter() - t0
    out = {"instance": f"{n} variables, domains U{{{dom[0]}..{dom[1]}}} ({int(spec.dsizes.sum())} support rows, "
                       f"{lay.D} domain words), {t} distinct tuples, sum w_i x_i = C over all variables "
                       f"(w_i in 1..20); input order, largest value first, all solutions",
           "nodes": g.nodes, "fails": g.fails, "solutions": len(g.solutions),
           "table_propagations": prop.props, "solve_seconds": round(el, 3),
           "table_seconds": round(prop.seconds, 3),
           "table_props_per_s": round(prop.props / prop.seconds, 1) if prop.seconds > 0 else None,
           "nodes_per_s": round(g.nodes / el, 1), "table_schedule": "resident engine" if table.resident
           else "resident split" if table.resident_split else "launched"}
    table.close()
    if cpu:
        from oracle import oracle as O
        o = O.OracleTable(spec.tuples, spec.lo, spec.dsizes, fast=True)
        oprop = S.OneTable(o)
        s2 = S.Search(lay, oprop, S.LinearEQ(lay, E, w, c), var_order="input", val_order="max")
        t0 = time.perf_counter()
        s2.run(lay.full(), 10 ** 7, 10 ** 7)
        oel = time.perf_counter() - t0
        out["oracle_solve_seconds"] = round(oel, 3)
        out["oracle_table_seconds"] = round(oprop.seconds, 3)
        out["oracle_table_props_per_s"] = round(oprop.props / oprop.seconds, 1) if oprop.seconds > 0 else None
        out["same_tree_as_oracle"] = bool((s2.nodes, s2.fails, s2.solutions) == (g.nodes, g.fails, g.solutions))
    return out


def root_batch_leg(tabs, specs, reps, per_table=True):
    """Every table's root recomputed from scratch (ROOT jobs: all tuples,
    every variable on the reset branch) in one batched launch: each support
    row is streamed once, the HBM-bound form of updateTable.  Compared with
    one launch per table, and checked against each table's own root."""
    import numpy as np
    import torch
    from paper_2507_18413_amd import ct
    from paper_2507_18413_amd import workloads as W
    n = len(tabs)
    fulls = [W.DomLayout(sp.dsizes, sp.lo).full() for sp in specs]
    offs = np.cumsum([0] + [len(f) for f in fulls])
    din = torch.from_numpy(np.concatenate(fulls).view(np.int64)).cuda()
    dout = torch.zeros_like(din)
    status = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    jobs = []
    for k, t in enumerate(tabs):
        slot = t.slots_alloc(1, max_depth=0)
        jobs.append(dict(table=t, slot=slot, flags=ct.JOB_PROPAGATE | ct.JOB_ROOT,
                         dom_in=din[offs[k]:offs[k + 1]], dom_out=dout[offs[k]:offs[k + 1]]))
    batch = ct.Batch(jobs)
    batch.run(status)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    got = dout.cpu().numpy().view(np.uint64)
    same = all(int(st[k]) == (ct.FAIL if t.root_failed else ct.OK) and
               (t.root_failed or (got[offs[k]:offs[k + 1]] == t.domains(0)).all())
               for k, t in enumerate(tabs))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    h0 = time.perf_counter()
    for _ in range(reps):
        batch.run(status)
    host_ms = (time.perf_counter() - h0) * 1e3 / reps
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    rows_w = sum(int(t.rows) * int(t.W) for t in tabs)
    # compulsory bytes: every support row once, currTable written once, the
    # domains read and written
    byts = 8 * rows_w + 8 * sum(int(t.W) for t in tabs) + 16 * int(offs[-1])
    out = {"jobs": n, "matches_table_roots": bool(same), "ms_per_batch": round(ms, 4),
           "compulsory_bytes": byts, "compulsory_GBps": round(byts / ms / 1e6, 1),
           "frac_of_hbm_peak": round(byts / ms / 1e6 / HBM_PEAK_GBS, 4),
           "host_issue_ms_per_batch": round(host_ms, 4),
           "timing": "HIP events around the batches on the launch stream"}
    # the streaming kernel alone, from the committed rocprofv3 summary
    from paper_2507_18413_amd import profiling
    prof = profiling.read_summary(os.path.join(ROOT, "profiles", "root_stream_2000_tables.md"))
    stream_bytes = 8 * rows_w + 8 * sum(int(t.W) for t in tabs)
    out["stream_kernel"] = {"name": "ctk::root_stream_kernel", "algorithmic_bytes": stream_bytes}
    if prof:
        us = prof["avg_us"]
        out["stream_kernel"].update({
            "avg_us_profiled": us, "hbm_bytes_profiled": prof.get("hbm_bytes_per_launch"),
            "roofline": {"bound": "hbm", "achieved": round(stream_bytes / us / 1e3, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(stream_bytes / us / 1e3 / HBM_PEAK_GBS, 4)}})
    if per_table:
        singles = [ct.Batch([j]) for j in jobs]
        torch.cuda.synchronize()
        e0.record()
        for b in singles:
            b.run(status)
        e1.record()
        torch.cuda.synchronize()
        ms1 = e0.elapsed_time(e1)
        out["one_launch_per_table_ms"] = round(ms1, 3)
        out["batched_speedup"] = round(ms1 / ms, 2)
    return out


def model_leg(seed, steps, cpu):
    """Batched CT across constraints: 2,000 tables over a pool of 5,000
    variables, root fixpoint then `steps` search steps (push, remove 5 % of
    the values of 1-3 pool variables, fixpoint; every 10 steps pop
    U{1..depth}, one level after a failure)."""
    import numpy as np
    import torch
    from paper_2507_18413_amd import ct
    from paper_2507_18413_amd import workloads as W
    t0 = time.perf_counter()
    spec = W.multi_table_model(seed)
    lay = spec.pool_layout()
    gen_s = time.perf_counter() - t0
    tabs = [ct.Table(tb.tuples, tb.lo, tb.dsizes) for tb in spec.tables]
    M = ct.Model(np.zeros(lay.n, np.int32), spec.pool_dsizes)
    for tb, sc in zip(tabs, spec.scopes):
        M.add(tb, sc)
    build_s = time.perf_counter() - t0 - gen_s
    root_batch = root_batch_leg(tabs, spec.tables, 20)
    full = lay.full()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()
    pin, pout = dev(full), dev(full)
    def timed_root_fixpoint(reps=3):
        # the root fixpoint between a push and a pop: a first, untimed one
        # builds the model's device state and captures its graphs, then the
        # median of `reps`
        M.push()
        M.fixpoint(pin, pout)
        M.pop()
        ts = []
        for _ in range(reps):
            M.push()
            torch.cuda.synchronize()
            r0 = time.perf_counter()
            M.fixpoint(pin, pout)
            ts.append(time.perf_counter() - r0)
            M.pop()
        return sorted(ts)[len(ts) // 2]

    # root fixpoint (phase 1), with the default schedule, then autotuned
    root_s = timed_root_fixpoint()
    cache = os.environ.get("CT_TUNE_CACHE") or os.path.join(ROOT, "gpurun_out", "ct_tune_cache.json")
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    from_cache, timed = M.autotune(pin, cache)
    classes = {}
    for c, tb in enumerate(tabs):
        cls = f"g{log4_bucket(tb.granules)} r{log4_bucket(tb.rows)}"
        classes.setdefault(cls, M.choice(c))
    best = {"from_cache": from_cache, "candidates_timed": timed,
            "classes": {k: {"solo": v[0], "tile": v[1]} for k, v in sorted(classes.items())}}
    root_tuned_s = timed_root_fixpoint()
    st, props, rounds = M.fixpoint(pin, pout)
    root = pout.cpu().numpy().view(np.uint64).copy()
    supports_bytes = sum(8 * int(tb.dsizes.sum()) * ((tb.t + 63) // 64) for tb in spec.tables)
    # the search script, drawn from the batched results (untimed), then timed
    rng = W.rng_for(seed, 3, 99)
    bt = W.Backtracker(rng)
    stack, pool, script = [], root.copy(), []
    var_tabs = {}
    for c, sc in enumerate(spec.scopes):
        for v in sc:
            var_tabs.setdefault(int(v), []).append(c)
    seeds = []
    for k in range(steps):
        new = W.pick_fraction_removal(rng, lay, pool)
        # tables whose scope holds a variable the step changes
        touched = set()
        for v in range(lay.n):
            o_, w_ = int(lay.off[v]), int(lay.words[v])
            if (new[o_:o_ + w_] != pool[o_:o_ + w_]).any():
                touched.update(var_tabs.get(v, []))
        seeds.append(sorted(touched))
        M.push()
        stack.append(pool)
        out = dev(new)
        st2, p2, r2 = M.fixpoint(dev(new), out)
        script.append(("step", new))
        pool = out.cpu().numpy().view(np.uint64).copy() if st2 == 0 else pool
        for _ in range(bt.pops_after(st2 != 0, len(stack))):
            M.pop()
            pool = stack.pop()
            script.append(("pop", None))
    while stack:
        M.pop()
        stack.pop()
        script.append(("pop", None))
    ins = [dev(x) if k == "step" else None for k, x in script]
    torch.cuda.synchronize()
    b0 = time.perf_counter()
    bprops = 0
    for (kind, _), din in zip(script, ins):
        if kind == "step":
            M.push()
            stt, p2, _ = M.fixpoint(din, pout)
            bprops += p2
        else:
            M.pop()
    torch.cuda.synchronize()
    batched_s = time.perf_counter() - b0
    out = {"tables": len(spec.tables), "pool_vars": lay.n, "tuples": int(sum(tb.t for tb in spec.tables)),
           "support_bytes": supports_bytes, "generate_s": round(gen_s, 1), "build_s": round(build_s, 1),
           "root_fixpoint_ms": round(root_s * 1e3, 3), "root_fixpoint_tuned_ms": round(root_tuned_s * 1e3, 3),
           "autotune": best, "root_props": props, "root_rounds": rounds,
           "steps": steps, "batched_props": bprops, "batched_step_props_per_s": round(bprops / batched_s, 1),
           "batched_ms_per_step": round(batched_s / steps * 1e3, 3), "root_gac_batch": root_batch}
    # plain GPU baseline: AC-3 on the host, one synchronous launch per table
    # propagation, seeded like the batched model's first round with the
    # tables the step touches; the same steps as the batched run
    pm = PlainModel(tabs, spec.scopes, lay)
    pm.push()
    p0 = time.perf_counter()
    _, _, rprops = pm.fixpoint(full)
    out["plain_root_ms"] = round((time.perf_counter() - p0) * 1e3, 3)
    pm.pop()
    pcnt, pstep, si = 0, 0, 0
    p0 = time.perf_counter()
    for kind, x in script:
        if kind == "step":
            pm.push()
            st3, _, pp = pm.fixpoint(x, seed=seeds[si])
            si += 1
            pcnt += pp
            pstep += 1
        else:
            pm.pop()
    plain_s = time.perf_counter() - p0
    while pm.stack:
        pm.pop()
    out["plain_steps"] = pstep
    out["plain_props"] = pcnt
    out["plain_step_props_per_s"] = round(pcnt / plain_s, 1)
    out["plain_ms_per_step"] = round(plain_s / max(pstep, 1) * 1e3, 3)
    # both reach the same closure from the same input every step; per-step
    # time is the like-for-like figure (the two count slightly different
    # propagations: the plain queue also runs a touched table whose own
    # domains lost nothing)
    out["batched_speedup_per_step"] = round(out["plain_ms_per_step"] / out["batched_ms_per_step"], 2)
    out["batched_wins"] = bool(out["batched_ms_per_step"] < out["plain_ms_per_step"])
    if cpu:
        from oracle import oracle as O
        ots = [O.OracleTable(tb.tuples, tb.lo, tb.dsizes, fast=True) for tb in spec.tables]
        c0 = time.perf_counter()
        for o in ots:
            o.push()
        ost, opool, oprops = O.fixpoint(ots, spec.scopes, lay, full)
        out["oracle_root_ms"] = round((time.perf_counter() - c0) * 1e3, 3)
        out["root_matches_oracle"] = bool(ost == st and (ost != 0 or (opool == root).all()))
        for o in ots:
            o.pop()
        ocnt, ostep, si = 0, 0, 0
        c0 = time.perf_counter()
        for kind, x in script:
            if kind == "step":
                for o in ots:
                    o.push()
                _, _, pp = O.fixpoint(ots, spec.scopes, lay, x, seed=seeds[si])
                si += 1
                ocnt += pp
                ostep += 1
            else:
                for o in ots:
                    o.pop()
        oel = time.perf_counter() - c0
        out["oracle_steps"] = ostep
        out["oracle_props"] = ocnt
        out["oracle_step_props_per_s"] = round(ocnt / oel, 1)
        out["oracle_ms_per_step"] = round(oel / max(ostep, 1) * 1e3, 3)
        out["oracle_note"] = ("fast mode, 1 thread, seeded FIFO AC-3; every push / pop visits all "
                              "2,000 tables")
    return out


def serve_leg(tables_spec, seed, rate, n_requests, n_searches, budget, sample_check, tabs=None):
    """Serving loop: Poisson arrivals at `rate` requests/s (rate <= 0: every
    request arrives at once, a saturation run), each given to a random idle
    search among `n_searches` simulated DFS searches bound to uniformly drawn
    tables of the 300-table mix; latency = completion time - arrival time
    (arrivals wait while no search is idle)."""
    import collections
    import numpy as np
    import torch
    from paper_2507_18413_amd import ct
    from paper_2507_18413_amd import workloads as W
    t0 = time.perf_counter()
    if tabs is None:
        tabs = [ct.Table(sp.tuples, sp.lo, sp.dsizes, max_depth=MAX_DEPTH_SERVE) for sp in tables_spec]
    build_s = time.perf_counter() - t0
    rng = W.rng_for(seed, 5, 777)
    # per-table pools of deltas: U{1..4} variables, ceil(5 %) of each one's
    # initial values (values already gone make no difference)
    pools = []
    for sp in tables_spec:
        lay = sp.layout()
        pool = np.zeros((256, lay.D), np.uint64)
        for k in range(256):
            for v in rng.choice(lay.n, size=min(lay.n, int(rng.integers(1, 5))), replace=False):
                d = int(lay.dsizes[v])
                for a in rng.choice(d, size=int(np.ceil(0.05 * d)), replace=False):
                    pool[k, lay.off[v] + a // 64] |= np.uint64(1 << (int(a) % 64))
        pools.append(pool)
    srv = ct.Server(mem_budget=budget, max_batch=1024, streams=2)
    search_tab = rng.integers(0, len(tabs), size=n_searches)
    sids = [srv.add_search(tabs[int(c)], max_depth=MAX_DEPTH_SERVE) for c in search_tab]
    depth = np.zeros(n_searches, np.int64)
    count = np.zeros(n_searches, np.int64)
    length = rng.integers(50, 201, size=n_searches)
    failed = np.zeros(n_searches, bool)
    arrivals = W.poisson_arrivals(rng, rate, n_requests) if rate > 0 else np.zeros(n_requests)
    idle = list(range(n_searches))
    waiting = collections.deque()
    t_arr, t_launch, t_done, sreq = {}, [], [], {}
    sample = set(range(min(sample_check, n_searches)))
    logs = {s: [] for s in sample}
    outs = {}
    issued = completed = 0
    start = srv.now() + 0.05
    arrivals = arrivals + start
    nxt = 0
    drained = set()   # tags of the drain requests (not measured)
    last_note = time.perf_counter()
    while completed < n_requests:
        now = srv.now()
        while nxt < n_requests and arrivals[nxt] <= now:
            waiting.append(arrivals[nxt])
            nxt += 1
        if time.perf_counter() - last_note > 5.0:
            note(f"serving: {completed} of {n_requests} requests done")
            last_note = time.perf_counter()
        if nxt == n_requests and not waiting:
            # every request is issued: a search keeps its slot between its
            # requests, so under a memory budget the searches still waiting
            # for a slot need the slot holders to finish; each idle search in
            # the middle of its life gets one more request, its last (not
            # measured)
            for s in [s for s in idle if count[s] > 0]:
                idle.remove(s)
                n_pop = 1 if failed[s] and depth[s] > 0 else 0
                srv.submit(sids[s], remove=None, n_pop=n_pop, push=0, finish=True, dom_out=None, tag=issued)
                sreq[issued] = (s, True)
                drained.add(issued)
                count[s] = 0
                issued += 1
        while waiting and idle:
            ta = waiting.popleft()
            j = int(rng.integers(0, len(idle)))
            s = idle[j]
            idle[j] = idle[-1]
            idle.pop()
            c = int(search_tab[s])
            if count[s] == 0:
                n_pop, push = 0, 0
            else:
                n_pop = 1 if failed[s] else (int(rng.integers(1, depth[s] + 1)) if count[s] % 10 == 0 and depth[s] else 0)
                push = 1
                # the slots hold max_depth levels: a search that would pass
                # it backtracks to half of it first
                if depth[s] - n_pop + push > MAX_DEPTH_SERVE:
                    n_pop = depth[s] - MAX_DEPTH_SERVE // 2
            depth[s] += push - n_pop
            failed[s] = False
            rem = pools[c][int(rng.integers(0, 256))]
            count[s] += 1
            finish = count[s] >= length[s]
            out = np.empty(tabs[c].D, np.uint64) if s in sample else None
            srv.submit(sids[s], remove=rem, n_pop=n_pop, push=push, finish=finish, dom_out=out, tag=issued)
            t_arr[issued] = ta
            sreq[issued] = (s, finish)
            if s in sample:
                logs[s].append((n_pop, push, rem, out))
            issued += 1
        res = srv.poll(wait_us=50 if not waiting else 0)
        for (tg, sid, status, ts, tl, td) in res:
            s, finish = sreq.pop(tg)
            if tg in drained:
                # a finishing request releases the slot whatever its status
                drained.discard(tg)
                depth[s] = 0
                failed[s] = False
                idle.append(s)
                continue
            t_done.append(td - t_arr.pop(tg))
            t_launch.append(tl)
            if status == 1:
                failed[s] = True
            elif status != 0:
                raise RuntimeError(f"serving status {status}")
            if finish:
                count[s] = 0
                depth[s] = 0
                failed[s] = False
            if s in sample:
                logs[s][-1] = logs[s][-1] + (status,) if len(logs[s][-1]) == 4 else logs[s][-1]
            idle.append(s)
            completed += 1
    wall = srv.now() - start
    st = srv.stats()
    srv.close()
    lat = np.array(t_done) * 1e6
    out = {"tables": len(tabs), "searches": n_searches, "requests": n_requests, "offered_rate": rate,
           "build_s": round(build_s, 1), "throughput_req_per_s": round(n_requests / wall, 1),
           "latency_us": {"p50": round(float(np.percentile(lat, 50)), 1),
                          "p99": round(float(np.percentile(lat, 99)), 1),
                          "mean": round(float(lat.mean()), 1)},
           "launches": st["launches"], "mean_batch": round(n_requests / max(st["launches"], 1), 2),
           "max_batch": st["max_batch"], "multi_request_launches": st["multi_request_launches"],
           "multi_table_launches": st["multi_table_launches"],
           "admission_waits": st["admission_waits"], "peak_slot_bytes": st["peak_slot_bytes"],
           "slots_allocated": st["slots_allocated"], "mem_budget": budget}
    # the sampled searches replayed alone on the oracle must give the same results
    if sample_check:
        from oracle import oracle as O
        ok = True
        for s in sample:
            sp = tables_spec[int(search_tab[s])]
            o = None
            dom, stack = None, []
            for (n_pop, push, rem, outv, *stl) in logs[s]:
                if o is None or (n_pop == 0 and push == 0):
                    o = O.OracleTable(sp.tuples, sp.lo, sp.dsizes)
                    dom, stack = o.domains(), []
                for _ in range(n_pop):
                    o.pop()
                    dom = stack.pop()
                if push:
                    o.push()
                    stack.append(dom.copy())
                sto, od = o.propagate(dom & ~rem)
                if stl and sto != stl[0]:
                    ok = False
                if sto == 0:
                    if not (od == outv).all():
                        ok = False
                    dom = od
        out["sampled_searches_equal_alone"] = ok
    return out


def log4_bucket(x):
    """floor(log4(x)) for x >= 1 (the autotuner's class buckets)."""
    b = 0
    while x >= 4:
        x //= 4
        b += 1
    return b


def host_info():
    """Cores and CPU model of the machine the run is on."""
    model = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable, "under_profiler": under_profiler()}


def copy_probe(mib=2048, reps=10):
    """Device-to-device copy of `mib` MiB by the runtime: HBM bytes moved
    (read + write) per second, the measured ceiling beside the 8 TB/s peak."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes": 2 * mib * (1 << 20), "ms": round(ms, 4),
            "GBps": round(2 * mib * (1 << 20) / ms / 1e6, 1), "what": f"torch copy_ of {mib} MiB (read + write)"}


def calibration_copy(mib):
    """One device-to-device copy of `mib` MiB by the runtime (the reference
    dispatch that scales the HBM byte counters)."""
    if not mib:
        return
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def under_profiler(env=None):
    """True when a profiler's preload library is in the process (rocprofv3
    loads its tool library before the program starts, and that library has
    already initialised the GPU)."""
    env = os.environ if env is None else env
    pre = env.get("LD_PRELOAD", "")
    return "rocprof" in pre or any(k.startswith("ROCPROF") for k in env)


def serving_workers(env=None):
    """Worker threads for generating the serving mix (threads, never
    processes: under a profiler the GPU is initialised before main() runs,
    and such a process must not start fresh interpreters)."""
    return min(16, os.cpu_count() or 1)


def note(msg):
    """Progress on stderr (the JSON result line is the only stdout output)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    # the cyclic garbage collector runs between the legs only: a full
    # collection inside a timed loop (tens of ms once the run holds many
    # Python objects) would be charged to the library
    gc.disable()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the library runs "
              f"on a single MI355X; sharding over several GPUs is a design, not a build)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2507_18413_amd import ct
    from paper_2507_18413_amd import workloads as W

    seed = W.DEFAULT_SEED if args.seed is None else args.seed
    if args.root_batch_only:
        note("generating the 2,000-table model")
        mspec = W.multi_table_model(seed)
        torch.cuda.set_device(0)
        calibration_copy(args.calibration_copy)
        tabs = [ct.Table(tb.tuples, tb.lo, tb.dsizes) for tb in mspec.tables]
        note("batched root recomputation")
        print(json.dumps({"root_gac_batch": root_batch_leg(tabs, mspec.tables, max(1, args.steps),
                                                           per_table=False)}), flush=True)
        return
    if args.nodes_only:
        torch.cuda.set_device(0)
        calibration_copy(args.calibration_copy)
        note("search-node leg")
        print(json.dumps({"batched_nodes": nodes_leg(seed, args.nodes, max(1, args.steps), max(0, args.warmup),
                                                     plain=False)}), flush=True)
        return
    if args.wide_only:
        torch.cuda.set_device(0)
        calibration_copy(args.calibration_copy)
        note("wide-scope leg")
        print(json.dumps({"wide_scope": wide_leg(seed, 300, False, split=False)}), flush=True)
        return
    serve_spec = None
    if not args.no_serve:
        workers = serving_workers()
        note(f"generating the serving mix (300 tables, {workers} threads)")
        serve_spec = W.serving_tables(seed, workers=workers)
    note("plain leg: building the 200,000-tuple table")
    torch.cuda.set_device(0)
    calibration_copy(args.calibration_copy)
    spec = W.large_table(seed)
    lay = spec.layout()
    # the table under test (synchronous calls go to the resident engine when
    # its state fits one workgroup's LDS) and a twin on launched kernels that
    # records the call script from the library's own answers (untimed; it
    # reads domains back after every call, which would stop the engine)
    table = ct.Table(spec.tuples, spec.lo, spec.dsizes)
    rec = ct.Table(spec.tuples, spec.lo, spec.dsizes, schedule=ct.SCHED_SOLO)
    script = W.run_plain_script(GpuSut(rec), lay, args.calls, seed, 2, W.pick_fraction_removal)
    depth = sum(1 if k == "push" else -1 if k == "pop" else 0 for k, _ in script)
    for _ in range(depth):
        script.append(("pop", None))
    rec.close()
    n_calls = sum(1 for k, _ in script if k == "prop")

    for _ in range(args.warmup):
        replay(table, script)
    torch.cuda.synchronize()
    s0 = table.stats()
    # the warmup's engine launch ends here, so that the timed calls are
    # served by launches whose whole lifetime is measured
    ct.quiesce()
    table.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    props = 0
    for _ in range(args.steps):
        props += replay(table, script)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernel_ms, launches = table.timing()
    disp_ms, dispatches = table.dispatch_timing()
    table.set_timing(False)
    s1 = table.stats()
    d = {k: s1[k] - s0[k] for k in s1}
    elapsed = t1 - t0
    value = props / elapsed
    # per-call latencies from as many more replays (outside the timed
    # steps: the timers around every call would be charged to them)
    lat = []
    for _ in range(args.steps):
        replay(table, script, lat)
    lat_us = np.array(lat) * 1e6
    bytes_total = algorithmic_bytes(d, lay.D, props)
    bytes_per_call = bytes_total / max(props, 1)
    # roofline of the dominant kernel: the algorithmic bytes of the calls a
    # launch served over the launch's lifetime (device clock, every launch
    # of the timed region); for the resident engine a launch serves many
    # calls and its lifetime includes the waits for the next call
    achieved = bytes_total / (disp_ms / 1e3) / 1e9 if disp_ms > 0 else 0.0
    busy_s = kernel_ms / 1e3

    from paper_2507_18413_amd import profiling
    kname = "ctk::engine_kernel" if table.resident else "ctk::propagate_kernel"
    prof = profiling.read_summary(os.path.join(
        ROOT, "profiles", "engine_large_table.md" if table.resident else "propagate_large_table.md"))
    calls_per_launch = props / max(dispatches, 1)
    # HBM bytes per launch of the timed region: the profiled bytes per call
    # (the engine's dispatches serve many calls each) times the calls a
    # timed launch served
    traffic = None
    if prof:
        per_call = prof.get("hbm_bytes_per_call") if table.resident else prof.get("hbm_bytes_per_launch")
        traffic = None if per_call is None else round(per_call * calls_per_launch, 1)
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
        "kernel": {"name": kname, "calls": props, "launches": dispatches,
                   "calls_per_launch": round(calls_per_launch, 1),
                   "launch_us_avg": round(disp_ms * 1e3 / max(dispatches, 1), 3),
                   "launch_us_per_call": round(disp_ms * 1e3 / max(props, 1), 3),
                   "busy_us_per_call": round(busy_s * 1e6 / max(launches, 1), 3),
                   "timing": "device clock: launch lifetimes (from the launch's start to its exit, the "
                             "engine's waits for calls included) and, per call, the time from command "
                             "receipt to publication" if table.resident else
                             "device clock: launch lifetimes (earliest workgroup start to latest end)",
                   "support_words_per_s": round(d["granule_rows"] * 64 / elapsed, 1),
                   "achieved_GBps_busy": round(bytes_total / busy_s / 1e9, 2) if busy_s > 0 else None,
                   "profiled_launch_us_per_call": prof.get("dispatch_us_per_call") if prof else None},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": traffic,
                     "bytes_per_launch": round(bytes_total / max(dispatches, 1), 1),
                     "bytes_per_call": round(bytes_per_call, 1)},
        "host": host_info(),
    }
    note(f"plain leg done: {value:.0f} propagations/s")
    if not args.no_tiny:
        note("tiny-table leg")
        out["tiny_table"] = tiny_leg(seed, 50, not args.no_cpu_baseline)
    if not args.no_probe:
        note("copy probe")
        out["copy_probe"] = copy_probe()
    if not args.no_split:
        note("split propagators on the plain script")
        out["split_propagators"] = split_leg(table, script, max(1, args.steps))
    if serve_spec is not None:
        # first of the other legs: its tables (gigabytes of host arrays) are
        # released before the batched legs time their host-side issue
        note("serving leg")
        stabs = [ct.Table(sp.tuples, sp.lo, sp.dsizes, max_depth=MAX_DEPTH_SERVE) for sp in serve_spec]
        out["serving"] = serve_leg(serve_spec, seed, args.serve_rate, args.serve_requests, 512,
                                   args.serve_budget, 0 if args.no_cpu_baseline else 8, tabs=stabs)
        note("serving leg: saturation")
        sat = serve_leg(serve_spec, seed + 1, 0.0, args.serve_requests // 4, 512, 0, 0, tabs=stabs)
        note("serving leg: a memory budget of a quarter of the peak slot bytes")
        peak = out["serving"]["peak_slot_bytes"]
        bud = serve_leg(serve_spec, seed + 2, 0.0, args.serve_requests // 8, 512, max(1, peak // 4),
                        0 if args.no_cpu_baseline else 4, tabs=stabs)
        out["serving"]["saturation"] = {k: sat[k] for k in ("requests", "throughput_req_per_s", "latency_us",
                                                          "launches", "mean_batch", "max_batch",
                                                          "multi_table_launches")}
        out["serving"]["budget_quarter_of_peak"] = {
            k: bud[k] for k in ("requests", "mem_budget", "throughput_req_per_s", "latency_us", "mean_batch",
                                "admission_waits", "peak_slot_bytes", "sampled_searches_equal_alone")
            if k in bud}
        del stabs
        serve_spec = None
        gc.collect()
    if not args.no_wide:
        gc.collect()
        note("wide-scope leg")
        out["wide_scope"] = wide_leg(seed, 300, not args.no_cpu_baseline)
        if not args.no_paper_shape:
            gc.collect()
            note("paper-shape leg")
            out["paper_shape"] = wide_leg(seed, 200, not args.no_cpu_baseline, split=False, paper_shape=True)
    if not args.no_driver:
        gc.collect()
        note("search driver leg")
        out["search_driver"] = solver_leg(seed, not args.no_cpu_baseline)
    if not args.no_nodes:
        gc.collect()
        note("search-node leg")
        out["batched_nodes"] = nodes_leg(seed, args.nodes, max(20, args.steps), 1,
                                         cpu=not args.no_cpu_baseline)
    if not args.no_model:
        gc.collect()
        note("multi-table model leg")
        out["batched_model"] = model_leg(seed, args.model_steps, not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        note("oracle on the host cores")
        cps, cprops, cel, passes, wpc, bpc = cpu_baseline(spec, script, args.cpu_seconds)
        pps, pprops, pel, ppasses, _, _ = cpu_baseline(spec, script, max(1.0, args.cpu_seconds / 4), fast=False)
        hi = host_info()
        out["cpu_baseline"] = {"value": round(cps, 1), "unit": "propagations/s", "cores": 1, "kind": "oracle",
                               "sample": f"{passes} replays of the same {n_calls}-call script "
                                         f"({cprops} propagations, {cel:.1f} s, 1 thread; the oracle's "
                                         f"fast mode: sparse word list, residues, word trail)",
                               "mode": "fast", "cpu_model": hi["cpu_model"], "nproc": hi["nproc"],
                               "usable_cores": hi["usable_cores"],
                               "support_words_per_call": round(wpc, 1),
                               "support_words_per_s": round(wpc * cps, 1),
                               "algorithmic_bytes_per_call": round(bpc, 1),
                               "plain_mode": {"value": round(pps, 1), "sample": f"{ppasses} replays, {pel:.1f} s, "
                                                                               "1 thread (dense Alg. 1-3)"},
                               "why_one_core": "the calls of one search depend on each other: each is the "
                                               "next call's input"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
