"""Parity at the size of the paper's instances (Sec. 5.1 Table 2 and
Sec. 5.3: 100-200 variables, domains up to 2,000 values, 10,000-15,000
tuples): about 150,000 support rows and 2,400 domain words, so row lists are
staged through LDS in chunks and domain words beyond the LDS copy are read
from memory.  Every call's status, domains and currTable against the
oracle, under the automatic and solo schedules, in a batch of search nodes
and as roots recomputed from scratch."""
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


@pytest.fixture(scope="module")
def spec():
    return W.paper_shape_table(W.DEFAULT_SEED)


@pytest.mark.parametrize("schedule,calls", [(ct.SCHED_AUTO, 60), (ct.SCHED_SOLO, 25)])
def test_paper_shape_calls(spec, schedule, calls):
    say("paper shape: 150 variables, domains up to 2,000, 15,000 tuples; schedule", schedule)
    g = ct.Table(spec.tuples, spec.lo, spec.dsizes, schedule=schedule)
    o = O.OracleTable(spec.tuples, spec.lo, spec.dsizes, fast=True)
    assert g.rows > 100_000 and g.D > 2000 and not g.resident
    # support rows of the first, a middle and the last variable
    for r0 in (0, g.rows // 2, g.rows - 300):
        got = g.supports(r0, 300)
        want = np.stack([o.support_row(r) for r in range(r0, r0 + 300)])
        assert (got == want).all(), r0
    gd, gc = g.state()
    od, oc, _ = o.state()
    assert (gd == od).all() and (gc == oc).all()
    lay = spec.layout()
    rng = W.rng_for(5, 800, schedule)
    depth = 0
    for k in range(calls):
        # removals of 5 % of 1-3 variables, and now and then a large cut
        frac = 0.6 if k % 7 == 3 else 0.05
        din = W.pick_fraction_removal(rng, lay, o.domains(), frac=frac, nvars=(1, 3))
        assert g.push() == o.push() == 0
        depth += 1
        gs, gdom, gct = g.propagate(din, want_ct=True)
        os_, odom, oct_ = o.propagate(din, want_ct=True)
        assert gs == os_, k
        if os_ == O.OK:
            assert (gdom == odom).all(), k
            assert (gct == oct_).all(), k
        if os_ != O.OK or k % 5 == 4:
            pops = 1 if os_ != O.OK else int(rng.integers(1, depth + 1))
            for _ in range(pops):
                assert g.pop() == o.pop() == 0
            depth -= pops
    gd, gc = g.state()
    od, oc, _ = o.state()
    assert (gd == od).all() and (gc == oc).all()


def test_paper_shape_batches(spec):
    say("paper shape: a batch of 48 search nodes and 8 roots from scratch")
    g = ct.Table(spec.tuples, spec.lo, spec.dsizes, max_depth=0)
    lay = spec.layout()
    root = g.domains()
    n = 48
    nodes = W.node_states(lay, root, n, 7, max_frac=0.3)
    first = g.slots_alloc(n + 8, max_depth=0)
    din = torch.from_numpy(nodes.view(np.int64)).cuda()
    dout = torch.zeros_like(din)
    status = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    ct.propagate_batch([dict(table=g, slot=first + k, flags=ct.JOB_PROPAGATE | ct.JOB_FROM_ROOT,
                             dom_in=din[k], dom_out=dout[k]) for k in range(n)], status)
    ct.batch_status()
    st = status.cpu().numpy()
    got = dout.cpu().numpy().view(np.uint64)
    o = O.OracleTable(spec.tuples, spec.lo, spec.dsizes, fast=True)
    for k in range(n):
        o.push()
        os_, od = o.propagate(nodes[k])
        assert st[k] == os_, k
        if os_ == O.OK:
            assert (got[k] == od).all(), k
        o.pop()
    # roots recomputed from scratch for arbitrary input domains (all tuples,
    # every variable on the reset branch) equal an oracle table created with
    # those domains
    full = lay.full()
    ins = np.stack([W.pick_fraction_removal(W.rng_for(9, 801, k), lay, full, frac=0.3, nvars=(5, 40))
                    for k in range(8)])
    rin = torch.from_numpy(ins.view(np.int64)).cuda()
    rout = torch.zeros_like(rin)
    rst = torch.full((8,), 99, dtype=torch.int32, device="cuda")
    ct.propagate_batch([dict(table=g, slot=first + n + k, flags=ct.JOB_PROPAGATE | ct.JOB_ROOT,
                             dom_in=rin[k], dom_out=rout[k]) for k in range(8)], rst)
    ct.batch_status()
    rs = rst.cpu().numpy()
    rg = rout.cpu().numpy().view(np.uint64)
    for k in range(8):
        ok = O.OracleTable(spec.tuples, spec.lo, spec.dsizes, init_dom=ins[k])
        assert rs[k] == ok.create_status, k
        if ok.create_status == O.OK:
            assert (rg[k] == ok.domains()).all(), k
