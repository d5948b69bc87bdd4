"""ct_propagate_batch_noalloc, the batch entry point that allocates nothing,
against ct_propagate_batch on the same jobs: every status, output domain,
currTable and slot state is equal (bit-exact), on two calls in a row, the
second with fewer jobs, for each schedule a batch can take (search nodes,
the work queue with pops and pushes, roots recomputed from scratch); both
are also checked against the oracle."""
import sys

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


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def from_dev(t):
    return t.cpu().numpy().view(np.uint64)


def test_noalloc_search_nodes_equal_batch():
    spec = W.zipf_table(t=60_000)
    lay = spec.layout()
    ga = ct.Table(spec.tuples, spec.lo, spec.dsizes)
    gb = ct.Table(spec.tuples, spec.lo, spec.dsizes)
    ot = O.OracleTable(spec.tuples, spec.lo, spec.dsizes)
    nodes = W.node_states(lay, ot.domains(), 256)
    fa = ga.slots_alloc(256, max_depth=0)
    fb = gb.slots_alloc(256, max_depth=0)
    for n in (256, 70):
        say("noalloc: search nodes, Zipf table 60k tuples,", n, "nodes")
        din = to_dev(nodes[:n])
        res = {}
        for g, first, noalloc in ((ga, fa, False), (gb, fb, True)):
            dout = torch.zeros_like(din)
            cts = torch.zeros((n, g.W), dtype=torch.int64, device="cuda")
            status = torch.full((n,), 99, dtype=torch.int32, device="cuda")
            jobs = [dict(table=g, slot=first + k, flags=ct.JOB_PROPAGATE | ct.JOB_FROM_ROOT,
                         dom_in=din[k], dom_out=dout[k], ct_out=cts[k]) for k in range(n)]
            ct.propagate_batch(jobs, status, noalloc=noalloc)
            torch.cuda.synchronize()
            res[noalloc] = (status.cpu().numpy(), from_dev(dout), from_dev(cts))
        ct.batch_status()
        (sa, da, ca), (sb, db, cb) = res[False], res[True]
        assert (sa == sb).all()
        ok = sa == ct.OK
        assert (da[ok] == db[ok]).all() and (ca[ok] == cb[ok]).all()
        for k in range(n):
            ot.push()
            os_, od, oc = ot.propagate(nodes[k], want_ct=True)
            ot.pop()
            assert sb[k] == os_, k
            if os_ == O.OK:
                assert (db[k] == od).all() and (cb[k] == oc).all(), k
            sta, stb = ga.state(fa + k), gb.state(fb + k)
            assert (sta[0] == stb[0]).all() and (sta[1] == stb[1]).all(), k


def test_noalloc_work_queue_with_backtracking_equal_batch():
    spec = W.large_table(t=30_000, d=20, n=4)
    lay = spec.layout()
    ga = ct.Table(spec.tuples, spec.lo, spec.dsizes)
    gb = ct.Table(spec.tuples, spec.lo, spec.dsizes)
    nsl = 32
    fa, fb = ga.slots_alloc(nsl), gb.slots_alloc(nsl)
    rng = W.rng_for(1, 207, 0)
    depth = np.zeros(nsl, int)
    for rnd, n in enumerate((32, 32, 32, 11)):
        say("noalloc: work queue,", n, "slots with pops and pushes, round", rnd)
        specs = []
        for k in range(n):
            n_pop = int(rng.integers(0, depth[k] + 1)) if rng.random() < 0.3 else 0
            n_push = int(rng.integers(0, 2))
            specs.append((n_pop, n_push))
        # the domains after the pops: the batched table's own (read before
        # the batch), then a random subset of them
        doms = []
        for k, (n_pop, n_push) in enumerate(specs):
            for _ in range(n_pop):
                assert ga.pop(fa + k) == ct.OK and gb.pop(fb + k) == ct.OK
            for _ in range(n_push):
                assert ga.push(fa + k) == ct.OK and gb.push(fb + k) == ct.OK
            depth[k] += n_push - n_pop
            cur = ga.domains(fa + k)
            assert (cur == gb.domains(fb + k)).all()
            keep = np.zeros_like(cur)
            for v in range(lay.n):
                for w in range(lay.off[v], lay.off[v] + lay.words[v]):
                    word = int(cur[w])
                    bits = [b for b in range(64) if (word >> b) & 1]
                    kept = [b for b in bits if rng.random() < 0.9] or bits[:1]
                    keep[w] = np.uint64(sum(1 << b for b in kept))
            doms.append(keep)
        din = to_dev(np.stack(doms))
        res = {}
        for g, first, noalloc in ((ga, fa, False), (gb, fb, True)):
            dout = torch.zeros_like(din)
            status = torch.full((n,), 99, dtype=torch.int32, device="cuda")
            jobs = [dict(table=g, slot=first + k, flags=ct.JOB_PROPAGATE, dom_in=din[k], dom_out=dout[k])
                    for k in range(n)]
            ct.propagate_batch(jobs, status, noalloc=noalloc)
            torch.cuda.synchronize()
            res[noalloc] = (status.cpu().numpy(), from_dev(dout))
        ct.batch_status()
        (sa, da), (sb, db) = res[False], res[True]
        assert (sa == sb).all(), (rnd, sa, sb)
        ok = sa == ct.OK
        assert (da[ok] == db[ok]).all()
        for k in range(n):
            sta, stb = ga.state(fa + k), gb.state(fb + k)
            if sa[k] == ct.OK:
                assert (sta[0] == stb[0]).all() and (sta[1] == stb[1]).all(), (rnd, k)
            if sa[k] == ct.FAIL and depth[k] > 0:
                assert ga.pop(fa + k) == ct.OK and gb.pop(fb + k) == ct.OK
                depth[k] -= 1


def test_noalloc_roots_from_scratch_equal_batch():
    rng = W.rng_for(1, 209, 0)
    specs = [W.large_table(t=int(t), d=int(d), n=int(n), seed=100 + k)
             for k, (t, d, n) in enumerate([(1_000, 12, 3), (40_000, 20, 4), (700, 8, 5), (10_000, 30, 3)])]
    tabs = {False: [ct.Table(s.tuples, s.lo, s.dsizes) for s in specs],
            True: [ct.Table(s.tuples, s.lo, s.dsizes) for s in specs]}
    for n in (4, 2):
        say("noalloc: roots recomputed from scratch,", n, "tables")
        doms = []
        for s in specs[:n]:
            lay = s.layout()
            doms.append(W.pick_fraction_removal(rng, lay, lay.full(), frac=0.3, nvars=(1, 3)))
        res = {}
        for noalloc in (False, True):
            status = torch.full((n,), 99, dtype=torch.int32, device="cuda")
            dins = [to_dev(d) for d in doms]
            douts = [torch.zeros_like(d) for d in dins]
            cts = [torch.zeros(t.W, dtype=torch.int64, device="cuda") for t in tabs[noalloc][:n]]
            jobs = [dict(table=tabs[noalloc][k], slot=0, flags=ct.JOB_PROPAGATE | ct.JOB_ROOT, dom_in=dins[k],
                         dom_out=douts[k], ct_out=cts[k]) for k in range(n)]
            ct.propagate_batch(jobs, status, noalloc=noalloc)
            torch.cuda.synchronize()
            res[noalloc] = (status.cpu().numpy(), [from_dev(d) for d in douts], [from_dev(c) for c in cts])
        ct.batch_status()
        (sa, da, ca), (sb, db, cb) = res[False], res[True]
        assert (sa == sb).all()
        for k in range(n):
            o = O.OracleTable(specs[k].tuples, specs[k].lo, specs[k].dsizes, init_dom=doms[k])
            assert sb[k] == o.create_status, k
            if sa[k] == ct.OK:
                od, oc, _ = o.state()
                assert (da[k] == db[k]).all() and (ca[k] == cb[k]).all(), k
                assert (db[k] == od).all() and (cb[k] == oc).all(), k


def test_noalloc_refuses_oversized_batch():
    spec = W.tiny_table()
    g = ct.Table(spec.tuples, spec.lo, spec.dsizes)
    lay = spec.layout()
    din = to_dev(lay.full())
    dout = torch.zeros_like(din)
    status = torch.zeros(8193, dtype=torch.int32, device="cuda")
    jobs = [dict(table=g, slot=0, flags=ct.JOB_PROPAGATE, dom_in=din, dom_out=dout)] * 8193
    with pytest.raises(ct.CTError) as e:
        ct.propagate_batch(jobs, status, noalloc=True)
    assert e.value.code == ct.E_INVALID
    assert "8192" in str(e.value)
    # the table is untouched and a batch within the limit still runs
    ct.propagate_batch(jobs[:1], status[:1], noalloc=True)
    torch.cuda.synchronize()
    assert int(status[0].item()) == ct.OK
    assert (g.domains(0) == from_dev(dout)).all()
