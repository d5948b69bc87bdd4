"""Parity at the full sizes of the batched and served workloads, in the
launch configurations the benchmark times.

* 2,000 tables over a pool of 5,000 variables (tuple counts log-uniform from
  100 to 500,000): the root fixpoint and search steps (push, removals,
  fixpoint, backtracking) against the oracle's seeded FIFO fixpoint;
* 4,096 search nodes on the 1,000,000-tuple Zipf table in one batch (the
  search-node schedule): every node's status and domains, and a sample of
  node currTables, against the oracle;
* the 300-table serving mix with 512 searches at saturation: sampled
  searches replayed alone on the oracle give the same statuses and domains.
"""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2507_18413_amd import ct
from paper_2507_18413_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def host(t):
    return t.cpu().numpy().view(np.uint64)


def test_full_model_root_fixpoint_and_search_steps():
    say("full model: generating 2,000 tables")
    spec = W.multi_table_model(W.DEFAULT_SEED)
    lay = spec.pool_layout()
    M = ct.Model(np.zeros(lay.n, np.int32), spec.pool_dsizes)
    gts = []
    for tb, sc in zip(spec.tables, spec.scopes):
        g = ct.Table(tb.tuples, tb.lo, tb.dsizes)
        M.add(g, sc)
        gts.append(g)
    ots = [O.OracleTable(tb.tuples, tb.lo, tb.dsizes, fast=True) for tb in spec.tables]
    for g, o in zip(gts, ots):
        assert g.create_status == o.create_status
    say("full model: root fixpoint")
    full = lay.full()
    pout = dev(np.zeros(lay.D, np.uint64))
    st, props, rounds = M.fixpoint(dev(full), pout)
    ost, opool, oprops = O.fixpoint(ots, spec.scopes, lay, full)
    assert st == ost == 0
    pool = host(pout).copy()
    assert (pool == opool).all()
    var_tabs = {}
    for c, sc in enumerate(spec.scopes):
        for v in sc:
            var_tabs.setdefault(int(v), []).append(c)
    rng = W.rng_for(W.DEFAULT_SEED, 3, 4242)
    bt = W.Backtracker(rng, every=4)
    stack = []
    fails = oks = 0
    for step in range(16):
        new = W.pick_fraction_removal(rng, lay, pool, frac=0.3, nvars=(2, 6))
        touched = sorted({c for v in range(lay.n) if (new[lay.off[v]:lay.off[v] + lay.words[v]] !=
                                                      pool[lay.off[v]:lay.off[v] + lay.words[v]]).any()
                          for c in var_tabs.get(v, [])})
        say("full model: step", step, "tables touched", len(touched))
        M.push()
        for o in ots:
            o.push()
        stack.append(pool)
        st, props, rounds = M.fixpoint(dev(new), pout)
        ost, opool, oprops = O.fixpoint(ots, spec.scopes, lay, new, seed=touched)
        assert st == ost, step
        if st == 0:
            oks += 1
            pool = host(pout).copy()
            assert (pool == opool).all(), step
        else:
            fails += 1
        for _ in range(bt.pops_after(st != 0, len(stack))):
            M.pop()
            for o in ots:
                o.pop()
            pool = stack.pop()
    assert oks > 0
    # the tables' slot-0 states equal the oracle tables' after the search
    while stack:
        M.pop()
        for o in ots:
            o.pop()
        pool = stack.pop()
    for c in range(0, len(gts), 97):
        gd, gc = gts[c].state()
        od, oc, of = ots[c].state()
        assert (gd == od).all() and (of or (gc == oc).all()), c


def test_full_nodes_batch():
    say("full nodes: 1,000,000-tuple Zipf table, 4,096 nodes")
    spec = W.zipf_table(W.DEFAULT_SEED)
    lay = spec.layout()
    g = ct.Table(spec.tuples, spec.lo, spec.dsizes, max_depth=0)
    root = g.domains()
    n = 4096
    nodes = W.node_states(lay, root, n, W.DEFAULT_SEED)
    first = g.slots_alloc(n, max_depth=0)
    din = dev(nodes)
    dout = torch.zeros_like(din)
    sample = list(range(0, n, 64))
    cts = {k: torch.zeros(g.W, dtype=torch.int64, device="cuda") for k in sample}
    status = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    jobs = [dict(table=g, slot=first + k, flags=ct.JOB_PROPAGATE | ct.JOB_FROM_ROOT, dom_in=din[k],
                 dom_out=dout[k], ct_out=cts.get(k)) for k in range(n)]
    ct.propagate_batch(jobs, status)
    ct.batch_status()
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    got = host(dout)
    ct_host = {k: host(v) for k, v in cts.items()}
    say("full nodes: oracle on host threads")

    def check(part):
        o = O.OracleTable(spec.tuples, spec.lo, spec.dsizes, fast=True)
        bad = []
        for k in range(part, n, 16):
            o.push()
            want_ct = k in cts
            r = o.propagate(nodes[k], want_ct=want_ct)
            if r[0] != st[k] or (r[0] == O.OK and not (r[1] == got[k]).all()):
                bad.append(k)
            elif want_ct and r[0] == O.OK and not (r[2] == ct_host[k]).all():
                bad.append(k)
            o.pop()
        return bad

    with ThreadPoolExecutor(16) as ex:
        bad = sum(ex.map(check, range(16)), [])
    assert not bad, bad[:10]
    assert (st == ct.OK).sum() > n // 2


def test_full_serving_mix_sampled_searches():
    say("full serving mix: generating 300 tables (threads)")
    specs = W.serving_tables(W.DEFAULT_SEED, workers=16)
    tabs = [ct.Table(sp.tuples, sp.lo, sp.dsizes, max_depth=64) for sp in specs]
    srv = ct.Server(mem_budget=0, max_batch=1024, streams=2)
    rng = W.rng_for(W.DEFAULT_SEED, 5, 4243)
    n_searches = 512
    search_tab = rng.integers(0, len(tabs), size=n_searches)
    sims, sids = [], []
    for s in range(n_searches):
        c = int(search_tab[s])
        sids.append(srv.add_search(tabs[c], max_depth=64))
        sims.append(W.SimSearch(specs[c].layout(), tabs[c].domains(), W.rng_for(W.DEFAULT_SEED, 502, s), 40))
    sample = set(range(0, n_searches, 32))
    results = {s: [] for s in sample}
    outs, inflight, tag = {}, set(), 0
    say("full serving mix: 512 searches x 40 requests at saturation")

    def submit(s):
        nonlocal tag
        c = int(search_tab[s])
        n_pop, push, remove, finish = sims[s].next_request()
        buf = np.zeros(tabs[c].D, np.uint64)
        outs[tag] = (s, buf)
        srv.submit(sids[s], remove=remove, n_pop=n_pop, push=push, finish=finish, dom_out=buf, tag=tag)
        inflight.add(tag)
        tag += 1

    for s in range(n_searches):
        submit(s)
    while inflight:
        for (tg, sid, status, ts, tl, td) in srv.poll(wait_us=20000):
            inflight.discard(tg)
            s, buf = outs.pop(tg)
            if s in sample:
                results[s].append((status, buf.copy()))
            sims[s].on_result(status, buf)
            if not sims[s].done():
                submit(s)
    stats = srv.stats()
    srv.close()
    assert stats["done"] == n_searches * 40
    assert stats["multi_table_launches"] > 0 and stats["launches"] < stats["done"]
    say("full serving mix: replaying", len(sample), "searches alone on the oracle")
    for s in sorted(sample):
        sp = specs[int(search_tab[s])]
        o = O.OracleTable(sp.tuples, sp.lo, sp.dsizes, fast=True)
        dom, stack = o.domains(), []
        for (n_pop, push, remove), (status, out) in zip(sims[s].log, results[s]):
            for _ in range(n_pop):
                assert o.pop() == O.OK
                dom = stack.pop()
            if push:
                assert o.push() == O.OK
                stack.append(dom.copy())
            st, od = o.propagate(dom & ~remove)
            assert st == status, s
            if st == O.OK:
                assert (od == out).all(), s
                dom = od
