"""The resident engine of synchronous calls (CT_SCHED_RESIDENT, the default
for tables whose state fits one workgroup's LDS) against the oracle: long
runs of calls without state reads in between (the engine keeps its state in
LDS throughout), idle exits and restarts, hand-over between tables, and
other operations on the same table that must first stop the engine."""
import sys
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_18413_amd import ct
from paper_2507_18413_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def pair(spec, schedule=ct.SCHED_RESIDENT, policy=ct.BRANCH_AUTO):
    g = ct.Table(spec.tuples, spec.lo, spec.dsizes, schedule=schedule, branch_policy=policy)
    o = O.OracleTable(spec.tuples, spec.lo, spec.dsizes)
    return g, o


def step(G, Ot, rng, lay, frac=0.08):
    """push, propagate the same removal on both, compare outputs."""
    dom_in = W.pick_fraction_removal(rng, lay, Ot.domains(), frac)
    assert G.push() == ct.OK and Ot.push() == O.OK
    gs, gd, gc = G.propagate(dom_in, want_ct=True)
    os_, od, oc = Ot.propagate(dom_in, want_ct=True)
    assert gs == os_
    if os_ == O.OK:
        assert (gd == od).all() and (gc == oc).all()
    return os_


def unwind(G, Ot, rng, status):
    k = 1 if status == O.FAIL else (int(rng.integers(1, Ot.depth + 1)) if rng.random() < 0.15 else 0)
    for _ in range(k):
        assert G.pop() == ct.OK and Ot.pop() == O.OK


@pytest.mark.parametrize("policy", [ct.BRANCH_AUTO, ct.BRANCH_RESET, ct.BRANCH_INCREMENTAL])
def test_long_run_without_state_reads(policy):
    spec = W.large_table(t=40_000, d=24, n=5)
    say("engine: 400 calls, policy", policy)
    G, Ot = pair(spec, policy=policy)
    lay = spec.layout()
    rng = W.rng_for(2, 600, policy)
    for call in range(400):
        st = step(G, Ot, rng, lay)
        unwind(G, Ot, rng, st)
    gd, gc = G.state()
    od, oc, of = Ot.state()
    assert (gd == od).all()
    if not of:
        assert (gc == oc).all()


def test_deep_levels_past_the_lds_rings():
    """Pops that reach levels and trail entries older than what the engine
    mirrors in LDS (64 levels; trail headers up to 4,096 entries, about 83
    levels of this 49-granule table) take them from HBM: 100 levels pushed,
    each removing one value, then pops of 37, 41 and 15 levels with calls in
    between (the second pop reaches a level record older than the ring, the
    third trail entries older than it too), every output and the final state
    equal to the oracle's."""
    spec = W.large_table(t=200_000, d=50, n=5)
    say("engine: 100 levels, pops across the LDS rings")
    G, Ot = pair(spec)
    assert G.resident
    lay = spec.layout()
    rng = W.rng_for(4, 602, 0)

    def call(want_ct):
        dom_in = Ot.domains().copy()
        cand = [i for i in range(lay.n) if lay.count(dom_in, i) > 1]
        i = cand[int(rng.integers(0, len(cand)))]
        vals = lay.values(dom_in, i)
        lay.clear(dom_in, i, int(vals[int(rng.integers(0, vals.shape[0]))]))
        if want_ct:
            gs, gd, gc = G.propagate(dom_in, want_ct=True)
            os_, od, oc = Ot.propagate(dom_in, want_ct=True)
        else:
            gs, gd = G.propagate(dom_in)
            os_, od = Ot.propagate(dom_in)
            gc = oc = None
        assert gs == os_
        if os_ == O.OK:
            assert (gd == od).all()
            if gc is not None:
                assert (gc == oc).all()
        return os_

    for level in range(100):
        assert G.push() == ct.OK and Ot.push() == O.OK
        assert call(level % 16 == 0) == O.OK, level
    for k in (37, 41, 15):
        for _ in range(k):
            assert G.pop() == ct.OK and Ot.pop() == O.OK
        for j in range(3):
            assert G.push() == ct.OK and Ot.push() == O.OK
            call(j == 2)
        for _ in range(3):
            assert G.pop() == ct.OK and Ot.pop() == O.OK
    gd, gc = G.state()
    od, oc, of = Ot.state()
    assert (gd == od).all() and (gc == oc).all()


def test_idle_exit_and_restart():
    spec = W.large_table(t=20_000, d=20, n=4)
    say("engine: idle exits between calls")
    G, Ot = pair(spec)
    lay = spec.layout()
    rng = W.rng_for(3, 601, 0)
    for call in range(40):
        st = step(G, Ot, rng, lay)
        unwind(G, Ot, rng, st)
        if call % 5 == 4:
            time.sleep(0.01)  # longer than the engine's idle limit: it exits
    gd, _ = G.state()
    assert (gd == Ot.domains()).all()


def test_tables_take_turns():
    a = W.large_table(t=15_000, d=16, n=4)
    b = W.TableSpec(W.distinct_uniform_tuples(W.rng_for(4, 602, 0), [9, 9, 9], 300),
                    np.zeros(3, np.int32), np.full(3, 9, np.int32))
    say("engine: two tables alternate (one engine per process)")
    Ga, Oa = pair(a)
    Gb, Ob = pair(b)
    rng = W.rng_for(4, 603, 0)
    la, lb = a.layout(), b.layout()
    for call in range(60):
        G, Ot, lay = (Ga, Oa, la) if call % 2 == 0 else (Gb, Ob, lb)
        st = step(G, Ot, rng, lay, frac=0.2)
        unwind(G, Ot, rng, st)
    for G, Ot in ((Ga, Oa), (Gb, Ob)):
        gd, _ = G.state()
        assert (gd == Ot.domains()).all()


def test_other_slots_batches_and_stats_interleaved():
    import torch
    spec = W.large_table(t=30_000, d=20, n=5)
    say("engine: slot 0 calls interleaved with batches on other slots, stats")
    G, Ot = pair(spec)
    lay = spec.layout()
    root = Ot.domains()
    first = G.slots_alloc(8, max_depth=0)
    nodes = W.node_states(lay, root, 8, max_frac=0.3)
    din = torch.from_numpy(nodes.view(np.int64)).cuda()
    dout = torch.zeros_like(din)
    status = torch.zeros(8, dtype=torch.int32, device="cuda")
    jobs = ct.Batch([dict(table=G, slot=first + k, flags=ct.JOB_PROPAGATE | ct.JOB_FROM_ROOT,
                          dom_in=din[k], dom_out=dout[k]) for k in range(8)])
    R = ct.Table(spec.tuples, spec.lo, spec.dsizes, schedule=ct.SCHED_SOLO)  # launched reference
    O0 = O.OracleTable(spec.tuples, spec.lo, spec.dsizes)                    # stays at the root
    rng = W.rng_for(5, 604, 0)
    for call in range(30):
        dom_in = W.pick_fraction_removal(rng, lay, Ot.domains(), 0.08)
        assert G.push() == ct.OK and Ot.push() == O.OK and R.push() == ct.OK
        gs, gd, gstats = G.propagate(dom_in, want_stats=True)
        rs, rd, rstats = R.propagate(dom_in, want_stats=True)
        os_, od = Ot.propagate(dom_in)
        assert gs == os_ == rs
        if os_ == O.OK:
            assert (gd == od).all()
        for k in ("jobs", "granules_in", "rows_or", "granule_rows", "trail_granules"):
            assert gstats[k] == rstats[k], (call, k)
        if call % 6 == 5:
            jobs.run(status)
            torch.cuda.synchronize()
            ct.batch_status(None)
            for k in range(8):
                O0.push()
                s2, d2 = O0.propagate(nodes[k])
                O0.pop()
                assert int(status[k]) == s2
                if s2 == O.OK:
                    assert (dout[k].cpu().numpy().view(np.uint64) == d2).all()
        if os_ == O.FAIL:
            assert G.pop() == ct.OK and Ot.pop() == O.OK and R.pop() == ct.OK
    assert ct.lib().ct_quiesce() == ct.OK
    gd, _ = G.state()
    assert (gd == Ot.domains()).all()
