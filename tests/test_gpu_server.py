"""Serving loop: results of every request in a mixed, continuously batched
run equal those of the same search replayed alone on the oracle, also when a
tiny memory budget makes searches wait for slots."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_18413_amd import ct
from paper_2507_18413_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def small_tables(seed, n):
    rng = W.rng_for(seed, 500, 0)
    out = []
    for c in range(n):
        k = int(rng.integers(3, 6))
        ds = rng.integers(8, 40, size=k)
        t = min(int(rng.integers(500, 30_000)), int(np.prod(ds)) // 2)
        tup = (W.distinct_uniform_tuples(rng, ds, t) if c % 2 == 0
               else W._distinct_zipf_mixed(rng, ds.astype(np.int64), 1.1, t))
        out.append(W.TableSpec(tup, np.zeros(k, np.int32), ds.astype(np.int32)))
    return out


def run_mixed(specs, tables, n_searches, length, budget, seed):
    srv = ct.Server(mem_budget=budget, max_batch=64, streams=2)
    rng = W.rng_for(seed, 501, 0)
    searches, sids = [], []
    for s in range(n_searches):
        c = int(rng.integers(0, len(tables)))
        sids.append(srv.add_search(tables[c], max_depth=64))
        lay = specs[c].layout()
        root = tables[c].domains()
        searches.append((c, W.SimSearch(lay, root, W.rng_for(seed, 502, s), length)))
    results = {s: [] for s in range(n_searches)}
    outs = {}
    tag = 0
    inflight = set()
    # keep every search busy: submit its next request as soon as the previous completes
    for s, (c, sim) in enumerate(searches):
        n_pop, push, remove, finish = sim.next_request()
        buf = np.zeros(tables[c].D, np.uint64)
        outs[tag] = (s, buf)
        srv.submit(sids[s], remove=remove, n_pop=n_pop, push=push, finish=finish, dom_out=buf, tag=tag)
        inflight.add(tag)
        tag += 1
    while inflight:
        for (tg, sid, status, ts, tl, td) in srv.poll(wait_us=20000):
            inflight.discard(tg)
            s, buf = outs.pop(tg)
            c, sim = searches[s]
            results[s].append((status, buf.copy()))
            sim.on_result(status, buf)
            if not sim.done():
                n_pop, push, remove, finish = sim.next_request()
                nb = np.zeros(tables[c].D, np.uint64)
                outs[tag] = (s, nb)
                srv.submit(sids[s], remove=remove, n_pop=n_pop, push=push, finish=finish, dom_out=nb, tag=tag)
                inflight.add(tag)
                tag += 1
    stats = srv.stats()
    srv.close()
    return searches, results, stats


def check_alone(specs, searches, results):
    for s, (c, sim) in enumerate(searches):
        sp = specs[c]
        o = O.OracleTable(sp.tuples, sp.lo, sp.dsizes)
        dom = o.domains()
        stack = []
        for (n_pop, push, remove), (status, out) in zip(sim.log, results[s]):
            for _ in range(n_pop):
                assert o.pop() == O.OK
                dom = stack.pop()
            if push:
                assert o.push() == O.OK
                stack.append(dom.copy())
            st, od = o.propagate(dom & ~remove)
            assert st == status, (s, st, status)
            if st == O.OK:
                assert (od == out).all(), s
                dom = od


@pytest.mark.parametrize("budget", [0, 1])
def test_mixed_equals_alone(budget):
    specs = small_tables(3, 6)
    say("server: 6 tables, 24 searches of 30 requests, budget", budget)
    tables = [ct.Table(sp.tuples, sp.lo, sp.dsizes) for sp in specs]
    # budget 1 byte per slot beyond the first: one search holds a slot at a time
    searches, results, stats = run_mixed(specs, tables, 24, 30, budget, 7)
    assert stats["done"] == 24 * 30
    if budget:
        assert stats["admission_waits"] > 0
    else:
        # continuous batching really mixed the searches: fewer launches than
        # requests, some launch carried several searches, some of them on
        # different tables
        assert stats["launches"] < stats["done"], stats
        assert stats["multi_request_launches"] > 0, stats
        assert stats["multi_table_launches"] > 0, stats
        assert stats["max_batch"] >= 2, stats
    check_alone(specs, searches, results)
