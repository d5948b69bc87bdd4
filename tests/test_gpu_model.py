"""Multi-table fixpoint on the GPU against the oracle's FIFO fixpoint and the
enumeration closure: pool domains must match bit for bit after every step."""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_18413_amd import ct
from paper_2507_18413_amd import workloads as W
from tests.bruteforce import closure

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def host(t):
    return t.cpu().numpy().view(np.uint64)


def build(spec, schedule=None):
    lay = spec.pool_layout()
    M = ct.Model(np.zeros(lay.n, np.int32), spec.pool_dsizes)
    gts, ots = [], []
    for tb, sc in zip(spec.tables, spec.scopes):
        g = ct.Table(tb.tuples, tb.lo, tb.dsizes)
        M.add(g, sc)
        gts.append(g)
        ots.append(O.OracleTable(tb.tuples, tb.lo, tb.dsizes))
    if schedule is not None:
        M.set_schedule(*schedule)
    return lay, M, gts, ots


def random_model(seed, n_pool, n_tables, dom, arity, tup):
    rng = W.rng_for(seed, 300, 0)
    pool = rng.integers(dom[0], dom[1] + 1, size=n_pool).astype(np.int32)
    tables, scopes = [], []
    for c in range(n_tables):
        k = int(rng.integers(arity[0], min(arity[1], n_pool) + 1))
        scope = rng.choice(n_pool, size=k, replace=False).astype(np.int32)
        ds = pool[scope]
        t = int(rng.integers(tup[0], tup[1] + 1))
        tp = np.stack([rng.integers(0, ds[i], size=t) for i in range(k)], 1).astype(np.int32)
        tables.append(W.TableSpec(tp, np.zeros(k, np.int32), ds.astype(np.int32)))
        scopes.append(scope)
    return W.ModelSpec(pool, tables, scopes)


@pytest.mark.parametrize("schedule", [(0, 1), (1000, 8), (4, 3)])
@pytest.mark.parametrize("seed", range(3))
def test_small_models_vs_oracle_and_closure(seed, schedule):
    import torch
    spec = random_model(seed, 8, 6, (2, 5), (1, 3), (1, 14))
    say("small model", seed, schedule)
    lay, M, gts, ots = build(spec, schedule)
    rng = W.rng_for(seed, 301, 0)
    for trial in range(4):
        start = lay.full()
        for i in range(lay.n):
            for a in lay.values(start, i):
                if rng.random() < 0.15:
                    lay.clear(start, i, int(a))
        M.push()
        for o in ots:
            o.push()
        pin, pout = dev(start), dev(np.zeros(lay.D, np.uint64))
        st, props, rounds = M.fixpoint(pin, pout)
        ost, opool, _ = O.fixpoint(ots, spec.scopes, lay, start)
        failed, want = closure([(t.tuples, t.lo) for t in spec.tables], spec.scopes, lay.to_sets(start))
        assert (st == ct.FAIL) == (ost == O.FAIL) == failed
        if st == ct.OK:
            got = host(pout)
            assert (got == opool).all()
            assert lay.to_sets(got) == want
        M.pop()
        for o in ots:
            o.pop()


@pytest.mark.parametrize("schedule", [(0, 8), (1000, 8)])
def test_search_steps_vs_oracle(schedule):
    import torch
    spec = random_model(7, 40, 30, (3, 70), (2, 4), (20, 3000))
    say("search steps", schedule)
    lay, M, gts, ots = build(spec, schedule)
    rng = W.rng_for(7, 302, 0)
    pool = lay.full()
    st, _, _ = M.fixpoint(dev(pool), out := dev(pool))
    ost, opool, _ = O.fixpoint(ots, spec.scopes, lay, pool)
    assert st == ost
    pool = host(out)
    assert (pool == opool).all()
    stack = []
    for step in range(30):
        M.push()
        for o in ots:
            o.push()
        stack.append(pool.copy())
        new = W.pick_fraction_removal(rng, lay, pool)
        out = dev(new)
        st, props, rounds = M.fixpoint(dev(new), out)
        ost, opool, _ = O.fixpoint(ots, spec.scopes, lay, new)
        assert st == ost, step
        if st == ct.OK:
            pool = host(out)
            assert (pool == opool).all(), step
        if st == ct.FAIL or (step % 7 == 6):
            k = 1 if st == ct.FAIL else int(rng.integers(1, len(stack) + 1))
            for _ in range(k):
                M.pop()
                for o in ots:
                    o.pop()
                pool = stack.pop()


def test_scaled_multi_table_root_and_steps(tmp_path):
    import torch
    say("multi-table model scaled: 150 tables over 400 variables")
    spec = W.multi_table_model(n_pool=400, n_tables=150, tuples=(100, 20_000))
    lay, M, gts, ots = build(spec)
    full = lay.full()
    out = dev(full)
    st, props, rounds = M.fixpoint(dev(full), out)
    ost, opool, oprops = O.fixpoint(ots, spec.scopes, lay, full)
    assert st == ost
    pool = host(out)
    if st == ct.OK:
        assert (pool == opool).all()
    assert props >= len(spec.tables) and rounds >= 1
    cache = os.path.join(str(tmp_path), "tune.json")
    from_cache, timed = M.autotune(dev(pool), cache)
    assert not from_cache and timed >= 4
    choices = [M.choice(c) for c in range(len(gts))]
    assert all(t in (2, 4, 8) for _, t in choices)
    text = open(cache).read()
    assert text.startswith("{") and '": [' in text
    # a second tuning of the same model (or any model whose classes the
    # cache holds) reuses the cached choices without timing
    from_cache, timed = M.autotune(dev(pool), cache)
    assert from_cache and timed == 0
    assert [M.choice(c) for c in range(len(gts))] == choices
    rng = W.rng_for(3, 303, 0)
    for step in range(10):
        M.push()
        for o in ots:
            o.push()
        new = W.pick_fraction_removal(rng, lay, pool)
        out = dev(new)
        st, _, _ = M.fixpoint(dev(new), out)
        ost, opool, _ = O.fixpoint(ots, spec.scopes, lay, new)
        assert st == ost
        if st == ct.OK:
            assert (host(out) == opool).all()
        M.pop()
        for o in ots:
            o.pop()


def test_queued_push_pop_seen_by_direct_table_use():
    """The model's push and pop are queued on its stream without waiting; a
    direct call on one of its tables right after must see them done."""
    spec = random_model(9, 30, 20, (8, 40), (2, 4), (500, 4000))
    say("model push / pop queued, then direct table use")
    lay, M, gts, ots = build(spec)
    pool = lay.full()
    st, _, _ = M.fixpoint(dev(pool), out := dev(pool))
    assert st == ct.OK
    before = [g.state(0) for g in gts]
    rng = W.rng_for(9, 303, 0)
    for trial in range(10):
        M.push()
        new = W.pick_fraction_removal(rng, lay, host(out).copy(), 0.3, (3, 6))
        st, _, _ = M.fixpoint(dev(new), dev(new))
        M.pop()  # queued: the table calls below must wait for it
        for g, (d0, c0) in zip(gts, before):
            d, c = g.state(0)
            assert (d == d0).all() and (c == c0).all(), trial
    # a direct propagate right after a queued push lands on the pushed level
    M.push()
    g = gts[0]
    sub = g.domains(0).copy()
    s2, d2 = g.propagate(sub)
    assert s2 == ct.OK
    assert g.pop(0) == ct.OK
    d, c = g.state(0)
    assert (d == before[0][0]).all() and (c == before[0][1]).all()
