"""Short and negative tables on the GPU against the oracle, call by call.

Short tables (cells that stand for every value of their column) and
negative tables (tuples that list the forbidden combinations) are the table
kinds of the paper's footnote on Sec. 2.  Statuses, domains and currTable
must equal the oracle's after every call, push and pop, under the
schedules each kind runs on, in single calls and in batches."""
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


def short_spec(seed, n, dom, t, star_p):
    rng = W.rng_for(seed, 700, 0)
    ds = rng.integers(dom[0], dom[1] + 1, size=n)
    tup = np.stack([rng.integers(0, ds[i] + 1, size=t) for i in range(n)], axis=1).astype(np.int32)
    tup[rng.random(tup.shape) < star_p] = ct.STAR
    return tup, np.zeros(n, np.int32), ds.astype(np.int32)


def negative_spec(seed, n, dom, t):
    rng = W.rng_for(seed, 701, 0)
    ds = rng.integers(dom[0], dom[1] + 1, size=n)
    tup = W.distinct_uniform_tuples(rng, ds, t)
    return tup, np.zeros(n, np.int32), ds.astype(np.int32)


def run_sequence(g, o, lay, seed, calls, frac):
    rng = W.rng_for(seed, 702, 1)
    depth = 0
    for k in range(calls):
        din = W.pick_fraction_removal(rng, lay, o.domains(), frac=frac, nvars=(1, 3))
        assert g.push() == o.push() == 0
        depth += 1
        gs, gd, gc = g.propagate(din, want_ct=True)
        os_, od, oc = o.propagate(din, want_ct=True)
        assert gs == os_, k
        if os_ == O.OK:
            assert (gd == od).all(), k
            assert (gc == oc).all(), k
        if os_ != O.OK or k % 4 == 3:
            pops = 1 if os_ != O.OK else int(rng.integers(1, depth + 1))
            for _ in range(pops):
                assert g.pop() == o.pop() == 0
            depth -= pops
            gd, gc = g.state()
            od, oc, of = o.state()
            assert (gd == od).all() and (gc == oc).all(), k


@pytest.mark.parametrize("schedule", [ct.SCHED_AUTO, ct.SCHED_SOLO, ct.SCHED_SPLIT])
@pytest.mark.parametrize("shape", [(4, (3, 9), 300, 0.3), (6, (5, 20), 9000, 0.15), (30, (4, 40), 2000, 0.5)])
def test_short_tables(schedule, shape):
    n, dom, t, p = shape
    tup, lo, ds = short_spec(3 + n, n, dom, t, p)
    say("short table", shape, "schedule", schedule)
    g = ct.Table(tup, lo, ds, schedule=schedule)
    o = O.OracleTable(tup, lo, ds)
    assert g.kind == ct.KIND_SHORT
    assert (g.supports() == np.stack([o.support_row(r) for r in range(g.rows)])).all()
    assert g.create_status == o.create_status
    gd, gc = g.state()
    od, oc, _ = o.state()
    assert (gd == od).all() and (gc == oc).all()
    run_sequence(g, o, DomLayout_of(ds), 5, 60, 0.2)


def DomLayout_of(ds):
    return W.DomLayout(ds, np.zeros(len(ds), np.int64))


@pytest.mark.parametrize("shape", [(2, (4, 6), 10), (3, (6, 8), 150), (5, (7, 9), 12000), (12, (2, 5), 3000)])
def test_negative_tables(shape):
    n, dom, t = shape
    tup, lo, ds = negative_spec(11 + n, n, dom, t)
    say("negative table", shape)
    g = ct.Table(tup, lo, ds, kind=ct.KIND_NEGATIVE)
    o = O.OracleTable(tup, lo, ds, kind=O.KIND_NEGATIVE)
    assert g.kind == ct.KIND_NEGATIVE and not g.resident
    assert g.create_status == o.create_status
    if o.create_status != O.OK:
        return
    gd, gc = g.state()
    od, oc, _ = o.state()
    assert (gd == od).all() and (gc == oc).all()
    run_sequence(g, o, DomLayout_of(ds), 7, 80, 0.3)


def test_negative_and_short_batches():
    """FROM_ROOT node batches and stateful batches of both kinds mixed in one
    launch, each job against the oracle."""
    specs = [("neg", *negative_spec(21, 4, (4, 9), 1500)), ("short", *short_spec(22, 5, (4, 12), 4000, 0.2)),
             ("neg", *negative_spec(23, 3, (5, 7), 100))]
    say("mixed batch of short and negative tables")
    tabs, ors, lays = [], [], []
    for kind, tup, lo, ds in specs:
        k = ct.KIND_NEGATIVE if kind == "neg" else ct.KIND_POSITIVE
        tabs.append(ct.Table(tup, lo, ds, kind=k, max_depth=4))
        ors.append((tup, lo, ds, O.KIND_NEGATIVE if kind == "neg" else O.KIND_POSITIVE))
        lays.append(DomLayout_of(ds))
    rng = W.rng_for(24, 703, 0)
    n_per = 40
    firsts = [t.slots_alloc(n_per, max_depth=0) for t in tabs]
    jobs, dins, douts, plan = [], [], [], []
    for c, t in enumerate(tabs):
        root = t.domains()
        for k in range(n_per):
            din = W.pick_fraction_removal(rng, lays[c], root, frac=0.4, nvars=(1, 3))
            d = torch.from_numpy(din.view(np.int64)).cuda()
            e = torch.zeros_like(d)
            dins.append(d)
            douts.append(e)
            jobs.append(dict(table=t, slot=firsts[c] + k, flags=ct.JOB_PROPAGATE | ct.JOB_FROM_ROOT,
                             dom_in=d, dom_out=e))
            plan.append((c, din))
    status = torch.full((len(jobs),), 99, dtype=torch.int32, device="cuda")
    ct.propagate_batch(jobs, status)
    ct.batch_status()
    st = status.cpu().numpy()
    for j, (c, din) in enumerate(plan):
        tup, lo, ds, kind = ors[c]
        o = O.OracleTable(tup, lo, ds, kind=kind)
        os_, od = o.propagate(din)
        assert st[j] == os_, (j, c)
        if os_ == O.OK:
            assert (douts[j].cpu().numpy().view(np.uint64) == od).all(), (j, c)


def test_kind_errors():
    say("kind errors")
    with pytest.raises(ct.CTError):
        ct.Table(np.array([[0, 1], [0, 1]], np.int32), [0, 0], [2, 2], kind=ct.KIND_NEGATIVE)
    with pytest.raises(ct.CTError):
        ct.Table(np.array([[0, ct.STAR]], np.int32), [0, 0], [2, 2], kind=ct.KIND_NEGATIVE)
    with pytest.raises(ct.CTError):
        ct.Table(np.array([[0, ct.STAR]], np.int32), [0, 0], [2, 2], branch_policy=ct.BRANCH_INCREMENTAL)
    g = ct.Table(np.array([[0, 1]], np.int32), [0, 0], [2, 2], kind=ct.KIND_NEGATIVE)
    with pytest.raises(ct.CTError):
        ct.SplitPropagator(g, ct.SPLIT_FILTER)
