"""Parity of the HIP library with the CPU oracle, call by call, bit-exact.

Every case drives the GPU (through the C ABI) and the oracle with the same
seeded inputs and compares statuses, domains and currTable after every
operation.  The work is exact integer bit manipulation, so the tolerance is
zero.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_18413_amd import ct
from paper_2507_18413_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1.json")


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def bits_of(words, t):
    return [int((int(words[j // 64]) >> (j % 64)) & 1) for j in range(t)]


def pair(tup, lo, ds, init=None, policy=ct.BRANCH_AUTO, max_depth=256, schedule=ct.SCHED_AUTO):
    say("create", f"t={len(tup)}", f"n={len(ds)}", f"policy={policy}", f"schedule={schedule}")
    g = ct.Table(tup, lo, ds, init_dom=init, branch_policy=policy, max_depth=max_depth, schedule=schedule)
    o = O.OracleTable(tup, lo, ds, init_dom=init)
    return g, o


def same_state(g, o, slot=0, where=""):
    gd, gc = g.state(slot)
    od, oc, of = o.state()
    assert (gd == od).all(), f"domains differ {where}"
    if not of:
        assert (gc == oc).all(), f"currTable differs {where}"


def random_subset(rng, lay, dom, p_keep):
    out = dom.copy()
    for i in range(lay.n):
        for a in lay.values(dom, i):
            if rng.random() > p_keep:
                lay.clear(out, i, int(a))
    return out


# --------------------------------------------------------------------------
def test_table1_on_gpu():
    g = json.load(open(GOLDEN))
    tup = np.array(g["tuples"], np.int32)
    G, Ot = pair(tup, g["lo"], g["dsizes"])
    S = G.supports()
    for name, want in g["printed_support_rows"].items():
        if name == "comment":
            continue
        i = {"x1": 0, "x2": 1, "x3": 2}[name.split("=")[0]]
        row = 4 * i + int(name.split("=")[1]) - 1
        assert bits_of(S[row], 5) == want, name
    same_state(G, Ot, where="root")
    lay = W.DomLayout(g["dsizes"], g["lo"])
    dom_in = lay.from_sets([[v - 1 for v in s] for s in g["derived"]["dom_giving_printed_currtable"]])
    st, dom_out, c = G.propagate(dom_in, want_ct=True)
    assert st == ct.OK
    assert bits_of(c, 5) == g["printed_currtable"]


@pytest.mark.parametrize("seed", range(4))
def test_support_builder_bit_exact(seed):
    rng = W.rng_for(seed, 200, 0)
    n = int(rng.integers(1, 6))
    ds = rng.integers(1, 140, size=n).astype(np.int32)
    lo = rng.integers(-50, 50, size=n).astype(np.int32)
    t = int(rng.integers(1, 64 * 64 * 3 + 50))
    tup = np.stack([rng.integers(lo[i] - 2, lo[i] + ds[i] + 2, size=t) for i in range(n)], 1).astype(np.int32)
    G, Ot = pair(tup, lo, ds)
    S = G.supports()
    for r in range(G.rows):
        assert (S[r] == Ot.support_row(r)).all(), r
    same_state(G, Ot, where="root")


def random_case(rng):
    n = int(rng.integers(1, 6))
    ds = rng.integers(1, 12, size=n).astype(np.int32)
    lo = rng.integers(-3, 4, size=n).astype(np.int32)
    t = int(rng.choice([0, 1, 5, 63, 64, 65, 300, 4096, 4097, 9000]))
    tup = np.stack([rng.integers(lo[i] - 1, lo[i] + ds[i] + 1, size=t) for i in range(n)], 1).astype(np.int32) \
        if t else np.zeros((0, n), np.int32)
    if t and rng.random() < 0.3:
        tup = np.concatenate([tup, tup[: max(1, t // 3)]])
    return tup, lo, ds


@pytest.mark.parametrize("chunk", range(6))
def test_random_sequences_vs_oracle(chunk):
    rng = W.rng_for(chunk, 201, 0)
    for case in range(12):
        tup, lo, ds = random_case(rng)
        lay = W.DomLayout(ds, lo)
        init = random_subset(rng, lay, lay.full(), 0.8) if rng.random() < 0.3 else None
        policy = int(rng.integers(0, 3))
        schedule = (ct.SCHED_SOLO, ct.SCHED_SPLIT, ct.SCHED_RESIDENT)[case % 3]
        say(f"chunk={chunk} case={case}")
        G, Ot = pair(tup, lo, ds, init=init, policy=policy, schedule=schedule)
        assert (G.create_status == ct.FAIL) == (Ot.create_status == O.FAIL)
        if Ot.create_status == O.FAIL:
            st, _ = G.propagate(lay.full() if init is None else init)
            assert st == ct.E_STATE
            continue
        same_state(G, Ot, where="root")
        for step in range(25):
            r = rng.random()
            if r < 0.25 and Ot.depth > 0:
                assert G.pop() == O.OK and Ot.pop() == O.OK
                same_state(G, Ot, where=f"pop step {step}")
                continue
            if r < 0.6:
                a, b = G.push(), Ot.push()
                assert a == b, (a, b)
            dom = Ot.domains()
            dom_in = random_subset(rng, lay, dom, float(rng.uniform(0.5, 1.0)))
            if rng.random() < 0.05:         # a value that is not present any more
                dom_in = lay.full()
            gs, gd, gc = G.propagate(dom_in, want_ct=True)
            os_, od, oc = Ot.propagate(dom_in, want_ct=True)
            assert gs == os_, (step, gs, os_)
            if os_ == O.OK:
                assert (gd == od).all(), step
                assert (gc == oc).all(), step
            if os_ == O.FAIL:
                assert not gc.any()
                if Ot.depth > 0:
                    assert G.pop() == O.OK and Ot.pop() == O.OK
                else:
                    assert G.push() == ct.E_STATE and Ot.push() == O.E_STATE
                    break
            same_state(G, Ot, where=f"step {step}")


def run_plain(spec, n_calls, picker, family, check_every=1, schedule=ct.SCHED_AUTO, ct_every=2,
              state_after_pops=True):
    G, Ot = pair(spec.tuples, spec.lo, spec.dsizes, schedule=schedule)
    lay = spec.layout()
    same_state(G, Ot, where="root")
    rng = W.rng_for(W.DEFAULT_SEED, family, 9)
    bt = W.Backtracker(rng)
    depth = 0
    for call in range(n_calls):
        dom_in = picker(rng, lay, Ot.domains())
        assert G.push() == ct.OK and Ot.push() == O.OK
        depth += 1
        # every ct_every-th call (0: none) with a currTable copy: the others
        # answer through flagged result slots (launched, or the resident
        # schedules), these through the fenced, counted status
        want_ct = ct_every > 0 and call % ct_every == 0
        if want_ct:
            gs, gd, gc = G.propagate(dom_in, want_ct=True)
            os_, od, oc = Ot.propagate(dom_in, want_ct=True)
        else:
            gs, gd = G.propagate(dom_in)
            os_, od = Ot.propagate(dom_in)
        assert gs == os_, (call, gs, os_)
        if os_ == O.OK and call % check_every == 0:
            assert (gd == od).all(), call
            if want_ct:
                assert (gc == oc).all(), call
        for _ in range(bt.pops_after(os_ == O.FAIL, depth)):
            assert G.pop() == ct.OK and Ot.pop() == O.OK
            depth -= 1
            if state_after_pops and call % check_every == 0:
                same_state(G, Ot, where=f"after pop at call {call}")
    return G, Ot


def test_tiny_table_full():
    say("tiny table: arity 3, d=8, 200 tuples, 100 calls")
    run_plain(W.tiny_table(), 100, W.pick_small_removal, 1)


@pytest.mark.parametrize("schedule", [ct.SCHED_SOLO, ct.SCHED_SPLIT])
def test_large_table_scaled(schedule):
    say("large table scaled: arity 5, d=50, 20,000 tuples, 300 calls, schedule", schedule)
    spec = W.large_table(t=20_000)
    run_plain(spec, 300, W.pick_fraction_removal, 2, schedule=schedule)


@pytest.mark.parametrize("schedule", [ct.SCHED_AUTO, ct.SCHED_SPLIT])
def test_large_table_full(schedule):
    say("large table: arity 5, d=50, 200,000 tuples, 1,000 calls, schedule", schedule)
    spec = W.large_table()
    G, Ot = run_plain(spec, 1000, W.pick_fraction_removal, 2, schedule=schedule)
    assert G.W == 3125


@pytest.mark.parametrize("schedule", [ct.SCHED_AUTO, ct.SCHED_SPLIT, ct.SCHED_SOLO, ct.SCHED_RESIDENT])
def test_wide_scope_vs_oracle(schedule):
    """A wide-scope table (100 variables, domains 64-160, 10,000 tuples:
    11,072 support rows of 157 words, 227 domain words; filterDomains
    dominates): 200 calls with backtracking, every call checked."""
    say("wide scope: arity 100, d in [64,160], 10,000 tuples, 200 calls, schedule", schedule)
    spec = W.wide_table()
    G, Ot = run_plain(spec, 200, W.pick_fraction_removal, 6, schedule=schedule)
    assert G.D == 227 and G.rows == 11072 and G.W == 157
    # the resident engine takes the 227-word table when asked (its wide
    # prologue and flat filter); AUTO gives its plain calls to the resident
    # split schedule and the calls that want currTable to the launched one
    assert G.resident == (schedule == ct.SCHED_RESIDENT)
    assert G.resident_split == (schedule == ct.SCHED_AUTO)


def test_wide_scope_resident_split_vs_oracle():
    """The resident split schedule on its own: 300 plain calls in a row on the
    wide-scope table (no call stops the persistent launch), backtracking
    included; every call's status and domains against the oracle, and the
    slot's state at the end."""
    say("wide scope: resident split schedule, 300 plain calls")
    spec = W.wide_table()
    # (no state reads inside the run: a read ends the persistent launch)
    G, Ot = run_plain(spec, 300, W.pick_fraction_removal, 7, ct_every=0, state_after_pops=False)
    assert G.resident_split and not G.resident
    same_state(G, Ot, where="end")


def test_wide_scope_nodes_batch_vs_oracle():
    """Search nodes on the wide-scope table (too many rows for the node
    schedule: the work queue runs them), each node against the oracle."""
    import torch
    say("wide scope: 96 search nodes in one batch")
    spec = W.wide_table()
    lay = spec.layout()
    G, Ot = pair(spec.tuples, spec.lo, spec.dsizes)
    root = Ot.domains()
    n = 96
    nodes = W.node_states(lay, root, n, max_frac=0.3)
    first = G.slots_alloc(n, max_depth=0)
    din = to_dev(nodes)
    dout = torch.zeros_like(din)
    cts = torch.zeros((n, G.W), dtype=torch.int64, device="cuda")
    status = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    jobs = [dict(table=G, slot=first + k, flags=ct.JOB_PROPAGATE | ct.JOB_FROM_ROOT,
                 dom_in=din[k], dom_out=dout[k], ct_out=cts[k]) for k in range(n)]
    ct.propagate_batch(jobs, status)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    got_dom, got_ct = from_dev(dout), from_dev(cts)
    for k in range(n):
        Ot.push()
        os_, od, oc = Ot.propagate(nodes[k], want_ct=True)
        Ot.pop()
        assert st[k] == os_, k
        if os_ == O.OK:
            assert (got_dom[k] == od).all(), k
            assert (got_ct[k] == oc).all(), k


def test_errors_match_oracle():
    g = json.load(open(GOLDEN))
    tup = np.array(g["tuples"], np.int32)
    G, Ot = pair(tup, g["lo"], g["dsizes"])
    lay = W.DomLayout(g["dsizes"], g["lo"])
    root = Ot.domains()
    stray = root.copy()
    stray[0] |= np.uint64(1 << 5)
    assert G.propagate(stray)[0] == ct.E_INVALID
    grow = root.copy()
    grow[2] |= np.uint64(1 << 1)
    assert G.propagate(grow)[0] == ct.E_NOT_SUBSET
    assert G.pop() == ct.E_STATE
    same_state(G, Ot, where="after errors")
    assert G.push() == ct.OK
    empty = lay.from_sets([[], [0, 1, 2, 3], [0, 2]])
    assert G.propagate(empty)[0] == ct.FAIL
    assert G.propagate(root)[0] == ct.E_STATE
    assert G.push() == ct.E_STATE
    assert G.pop() == ct.OK
    same_state(G, Ot, where="after fail + pop")


def test_depth_limit():
    spec = W.tiny_table()
    G = ct.Table(spec.tuples, spec.lo, spec.dsizes, max_depth=3)
    for _ in range(3):
        assert G.push() == ct.OK
    assert G.push() == ct.E_NOMEM
    for _ in range(3):
        assert G.pop() == ct.OK
    assert G.pop() == ct.E_STATE


def test_multiword_domains_and_ragged_tail():
    rng = W.rng_for(5, 202, 0)
    ds = np.array([130, 3, 65, 1], np.int32)
    lo = np.array([-7, 0, 100, 5], np.int32)
    t = 64 * 64 * 2 + 17
    tup = np.stack([rng.integers(lo[i], lo[i] + ds[i], size=t) for i in range(4)], 1).astype(np.int32)
    G, Ot = pair(tup, lo, ds)
    lay = W.DomLayout(ds, lo)
    same_state(G, Ot, where="root")
    for step in range(40):
        G.push(); Ot.push()
        dom_in = random_subset(rng, lay, Ot.domains(), 0.93)
        gs, gd, gc = G.propagate(dom_in, want_ct=True)
        os_, od, oc = Ot.propagate(dom_in, want_ct=True)
        assert gs == os_
        if os_ == O.OK:
            assert (gd == od).all() and (gc == oc).all()
        if os_ == O.FAIL or rng.random() < 0.2:
            G.pop(); Ot.pop()
            same_state(G, Ot, where=f"pop {step}")


# --------------------------------------------------------------------------
# batched jobs
# --------------------------------------------------------------------------
def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def from_dev(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("schedule", [ct.SCHED_AUTO, ct.SCHED_SPLIT, ct.SCHED_NODES])
def test_batch_from_root_nodes_vs_oracle(schedule):
    import torch
    say("batch: FROM_ROOT search nodes, Zipf table 60k tuples, 256 nodes, schedule", schedule)
    spec = W.zipf_table(t=60_000)
    lay = spec.layout()
    G, Ot = pair(spec.tuples, spec.lo, spec.dsizes, schedule=schedule)
    root = Ot.domains()
    nodes = W.node_states(lay, root, 256)
    first = G.slots_alloc(256, max_depth=0)
    din = to_dev(nodes)
    dout = torch.zeros_like(din)
    cts = torch.zeros((256, G.W), dtype=torch.int64, device="cuda")
    status = torch.full((256,), 99, dtype=torch.int32, device="cuda")
    jobs = [dict(table=G, slot=first + k, flags=ct.JOB_PROPAGATE | ct.JOB_FROM_ROOT,
                 dom_in=din[k], dom_out=dout[k], ct_out=cts[k]) for k in range(256)]
    ct.propagate_batch(jobs, status)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    got_dom = from_dev(dout)
    got_ct = from_dev(cts)
    for k in range(256):
        Ot.push()
        os_, od, oc = Ot.propagate(nodes[k], want_ct=True)
        Ot.pop()
        assert st[k] == os_, k
        if os_ == O.OK:
            assert (got_dom[k] == od).all(), k
            assert (got_ct[k] == oc).all(), k
            gd, gc = G.state(first + k)
            assert (gd == od).all() and (gc == oc).all(), k
    # a second batch reuses the slots from the root again
    ct.propagate_batch(jobs[:64], status[:64])
    torch.cuda.synchronize()
    assert (from_dev(dout[:64]) == got_dom[:64]).all()


@pytest.mark.parametrize("n_nodes,rows", [(1, 239), (100, 239), (200, 239), (1, 94), (150, 94)])
def test_batch_nodes_schedule_edge_cases(n_nodes, rows):
    """Granule-major node schedule on a table with multi-word domains, a
    ragged last word (an odd word count) and a granule count that is not a
    multiple of 8, with nodes that fail (an empty domain, no surviving tuple),
    nodes equal to the root, and rejected inputs (stray bits, values outside
    the root domains).  239 support rows take one-granule tiles (10
    granules); 94 rows take two-granule tiles (9 granules: the last tile half
    past the table's end)."""
    import torch
    say("batch nodes schedule: edge cases,", n_nodes, "nodes,", rows, "rows")
    rng = W.rng_for(11, 204, n_nodes + rows)
    if rows == 239:
        ds = np.array([130, 3, 65, 1, 40], np.int32)
    else:
        ds = np.array([40, 3, 20, 1, 30], np.int32)
    assert int(ds.sum()) == rows
    lo = np.array([-7, 0, 100, 5, 0], np.int32)
    t = 64 * 64 * 9 + 37 if rows == 239 else 64 * 64 * 8 + 37   # 577 or 513 words
    hi = ds.copy()
    hi[0] -= 10                               # the last 10 values of x0 have no support
    tup = np.stack([rng.integers(lo[i], lo[i] + hi[i], size=t) for i in range(5)], 1).astype(np.int32)
    G, Ot = pair(tup, lo, ds, schedule=ct.SCHED_NODES)
    lay = W.DomLayout(ds, lo)
    root = Ot.domains()
    nodes = np.empty((n_nodes, lay.D), np.uint64)
    for k in range(n_nodes):
        kind = k % 10
        if kind == 0:
            nodes[k] = root
        elif kind == 1:
            d = root.copy()
            for a in lay.values(root, 3):
                lay.clear(d, 3, int(a))      # empty domain
            nodes[k] = d
        elif kind == 2:
            d = root.copy()
            d[lay.D - 1] |= np.uint64(1) << np.uint64(63)  # stray bit past the last value
            nodes[k] = d
        elif kind == 3:
            d = lay.full()                    # values the root pruned
            nodes[k] = d
        else:
            nodes[k] = random_subset(rng, lay, root, float(rng.uniform(0.05, 0.97)))
    first = G.slots_alloc(n_nodes, max_depth=0)
    din = to_dev(nodes)
    dout = torch.zeros_like(din)
    cts = torch.zeros((n_nodes, G.W), dtype=torch.int64, device="cuda")
    status = torch.full((n_nodes,), 99, dtype=torch.int32, device="cuda")
    jobs = [dict(table=G, slot=first + k, flags=ct.JOB_PROPAGATE | ct.JOB_FROM_ROOT,
                 dom_in=din[k], dom_out=dout[k], ct_out=cts[k]) for k in range(n_nodes)]
    for rep in range(2):
        ct.propagate_batch(jobs, status)
        torch.cuda.synchronize()
        st = status.cpu().numpy()
        got_dom, got_ct = from_dev(dout), from_dev(cts)
        for k in range(n_nodes):
            Ot.push()
            os_, od, oc = Ot.propagate(nodes[k], want_ct=True)
            Ot.pop()
            assert st[k] == os_, (rep, k)
            if os_ == O.OK:
                assert (got_dom[k] == od).all(), (rep, k)
                assert (got_ct[k] == oc).all(), (rep, k)
                gd, gc = G.state(first + k)
                assert (gd == od).all() and (gc == oc).all(), (rep, k)
            elif os_ == O.FAIL:
                assert not got_ct[k].any(), (rep, k)
            else:
                # rejected input: the slot still holds the root
                gd, _ = G.state(first + k)
                assert (gd == root).all(), (rep, k)
        if n_nodes > 3:
            assert {int(x) for x in st} >= {ct.OK, ct.FAIL, ct.E_INVALID, ct.E_NOT_SUBSET}


@pytest.mark.parametrize("schedule", [ct.SCHED_SOLO, ct.SCHED_SPLIT])
def test_batch_with_backtracking_equals_sequential(schedule):
    import torch
    say("batch: 32 slots with pops/pushes vs single calls, schedule", schedule)
    spec = W.large_table(t=30_000, d=20, n=4)
    lay = spec.layout()
    Gb = ct.Table(spec.tuples, spec.lo, spec.dsizes, schedule=schedule)   # batched
    Gs = ct.Table(spec.tuples, spec.lo, spec.dsizes,             # single calls, other schedule
                  schedule=ct.SCHED_SPLIT if schedule == ct.SCHED_SOLO else ct.SCHED_SOLO)
    nsl = 32
    fb = Gb.slots_alloc(nsl)
    fs = Gs.slots_alloc(nsl)
    rng = W.rng_for(1, 203, 0)
    depth = np.zeros(nsl, int)
    for rnd in range(12):
        jobs, doms = [], []
        for k in range(nsl):
            n_pop = int(rng.integers(0, depth[k] + 1)) if rng.random() < 0.3 else 0
            for _ in range(n_pop):
                assert Gs.pop(fs + k) == ct.OK
            n_push = int(rng.integers(0, 2))
            for _ in range(n_push):
                assert Gs.push(fs + k) == ct.OK
            depth[k] += n_push - n_pop
            dom_in = random_subset(rng, lay, Gs.domains(fs + k), 0.9)
            doms.append(dom_in)
            jobs.append(dict(slot=fb + k, n_pop=n_pop, n_push=n_push))
        din = to_dev(np.stack(doms))
        dout = torch.zeros_like(din)
        status = torch.full((nsl,), 99, dtype=torch.int32, device="cuda")
        bj = [dict(table=Gb, slot=j["slot"], flags=ct.JOB_PROPAGATE, n_pop=j["n_pop"],
                   n_push=j["n_push"], dom_in=din[k], dom_out=dout[k]) for k, j in enumerate(jobs)]
        ct.propagate_batch(bj, status)
        torch.cuda.synchronize()
        st = status.cpu().numpy()
        gd = from_dev(dout)
        for k in range(nsl):
            ss, sd, sc = Gs.propagate(doms[k], slot=fs + k, want_ct=True)
            assert st[k] == ss, (rnd, k, st[k], ss)
            if ss == ct.OK:
                assert (gd[k] == sd).all()
                bd, bc = Gb.state(fb + k)
                assert (bd == sd).all() and (bc == sc).all()
            if ss == ct.FAIL:
                # both pop one level so the slot is usable again
                if depth[k] > 0:
                    Gs.pop(fs + k)
                    Gb.pop(fb + k)
                    depth[k] -= 1


@pytest.mark.parametrize("schedule,mixed", [(ct.SCHED_AUTO, False), (ct.SCHED_AUTO, True),
                                            (ct.SCHED_SOLO, False), (ct.SCHED_SPLIT, False)])
def test_batch_root_from_scratch_vs_oracle(schedule, mixed):
    """ROOT jobs recompute a table's root state from all tuples (Alg. 1, every
    variable on the reset branch) for any input domains: the result must be
    the GAC closure that an oracle table created with those initial domains
    reaches, and the slot must then carry on like that oracle table.  A batch
    of ROOT jobs alone runs on the streaming root kernels; mixed with an
    ordinary job, or under the SOLO / SPLIT schedules, on the work queue."""
    import torch
    say("batch ROOT jobs from scratch, schedule", schedule, "mixed" if mixed else "")
    rng = W.rng_for(12, 205, schedule)
    cases = []
    # a one-granule table, and one of 21 granules with multi-word domains and a
    # ragged last word (solo below 17 granules, split above under AUTO)
    for t, ds, lo in [(300, [5, 7, 3], [0, -2, 1]),
                      (64 * 64 * 20 + 37, [130, 3, 65, 1, 40], [-7, 0, 100, 5, 0])]:
        ds = np.array(ds, np.int32)
        lo = np.array(lo, np.int32)
        hi = ds.copy()
        hi[0] = max(1, hi[0] - 2)              # the last values of x0 have no support
        tup = np.stack([rng.integers(lo[i], lo[i] + hi[i], size=t) for i in range(len(ds))],
                       1).astype(np.int32)
        cases.append((tup, lo, ds))
    tabs, jobs_spec = [], []
    for ci, (tup, lo, ds) in enumerate(cases):
        lay = W.DomLayout(ds, lo)
        init = random_subset(rng, lay, lay.full(), 0.9)   # the table's own initial domains
        G = ct.Table(tup, lo, ds, init_dom=init, schedule=schedule)
        G.init_dom = init
        tabs.append(G)
        nj = 10
        first = G.slots_alloc(nj, max_depth=4)
        for k in range(nj):
            kind = k % 5
            if kind == 0:
                d = init.copy()                  # recomputes the table's own root
            elif kind == 1:
                d = lay.full()                   # values the table's root pruned
            elif kind == 2:
                d = lay.full()
                for a in lay.values(d, 1):
                    lay.clear(d, 1, int(a))      # an empty domain
            elif kind == 3:
                d = lay.full()
                d[lay.D - 1] |= np.uint64(1) << np.uint64(63)   # a stray bit
            else:
                d = random_subset(rng, lay, lay.full(), float(rng.uniform(0.1, 0.95)))
            jobs_spec.append((ci, G, first + k, d, kind))
    # one batch mixes both tables; ordinary jobs first move every slot off the root
    status = torch.full((len(jobs_spec),), 99, dtype=torch.int32, device="cuda")
    pre = []
    for ci, G, slot, d, kind in jobs_spec:
        assert G.push(slot) == ct.OK
        sub = random_subset(rng, W.DomLayout(cases[ci][2], cases[ci][1]), G.domains(slot), 0.7)
        G.propagate(sub, slot=slot)
        pre.append(G.state(slot))
    dins = [to_dev(d) for _, _, _, d, _ in jobs_spec]
    douts = [torch.zeros_like(x) for x in dins]
    cts = [torch.zeros((G.W,), dtype=torch.int64, device="cuda") for _, G, _, _, _ in jobs_spec]
    jobs = [dict(table=G, slot=slot, flags=ct.JOB_PROPAGATE | ct.JOB_ROOT,
                 dom_in=dins[j], dom_out=douts[j], ct_out=cts[j])
            for j, (_, G, slot, _, _) in enumerate(jobs_spec)]
    if mixed:
        # an ordinary job on slot 0 of the first table, checked against a
        # single call on a twin table
        tup, lo, ds = cases[0]
        G0 = tabs[0]
        twin = ct.Table(tup, lo, ds, init_dom=G0.domains(0))
        sub = random_subset(rng, W.DomLayout(ds, lo), G0.domains(0), 0.6)
        xin, xout = to_dev(sub), to_dev(np.zeros_like(sub))
        jobs.append(dict(table=G0, slot=0, flags=ct.JOB_PROPAGATE, dom_in=xin, dom_out=xout))
        status = torch.full((len(jobs),), 99, dtype=torch.int32, device="cuda")
    ct.propagate_batch(jobs, status)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    if mixed:
        ts, td = twin.propagate(sub)
        assert st[-1] == ts
        if ts == ct.OK:
            assert (from_dev(xout) == td).all()
    for j, (ci, G, slot, d, kind) in enumerate(jobs_spec):
        tup, lo, ds = cases[ci]
        if kind == 3:
            assert st[j] == ct.E_INVALID, j
            # a rejected job still resets the slot: it holds the table's root at depth 0
            gd, gc = G.state(slot)
            od, oc, _ = O.OracleTable(tup, lo, ds, init_dom=G.init_dom).state()
            assert (gd == od).all() and (gc == oc).all(), j
            assert G.pop(slot) != ct.OK, j
            continue
        Ox = O.OracleTable(tup, lo, ds, init_dom=d)
        od, oc, of = Ox.state()
        if of:
            assert st[j] == ct.FAIL, (j, st[j])
            assert not from_dev(cts[j]).any(), j
            continue
        assert st[j] == ct.OK, (j, st[j])
        assert (from_dev(douts[j]) == od).all(), j
        assert (from_dev(cts[j]) == oc).all(), j
        gd, gc = G.state(slot)
        assert (gd == od).all() and (gc == oc).all(), j
        if kind == 0 and not mixed:
            rd, rc = G.state(0)
            assert (gd == rd).all() and (gc == rc).all(), j
        # the slot is at depth 0 and continues like the oracle table
        lay = W.DomLayout(ds, lo)
        assert G.pop(slot) != ct.OK, j
        assert G.push(slot) == ct.OK and Ox.push() == O.OK
        sub = random_subset(rng, lay, od, 0.6)
        gs_, gdd = G.propagate(sub, slot=slot)
        os_, odd = Ox.propagate(sub)
        assert gs_ == os_, j
        if os_ == O.OK:
            assert (gdd == odd).all(), j
        assert G.pop(slot) == ct.OK and Ox.pop() == O.OK
        same_state(G, Ox, slot, f"job {j} after pop")
