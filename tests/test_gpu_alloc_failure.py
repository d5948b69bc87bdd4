"""Allocation failures, injected through the library's test hook
(ct_debug_fail_alloc): every allocation point of table creation, slot
allocation and batch staging returns CT_E_NOMEM, releases what it took and
leaves existing state untouched, and the library works normally after."""
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


def test_injected_allocation_failures():
    L = ct.lib()
    spec = W.large_table(3, t=5000, d=10, n=4)
    say("alloc failure: every allocation of ct_create in turn")
    created = None
    fired = 0
    for k in range(1, 64):
        L.ct_debug_fail_alloc(k)
        try:
            created = ct.Table(spec.tuples, spec.lo, spec.dsizes, max_depth=8)
        except ct.CTError as e:
            assert e.code == ct.E_NOMEM and "injected" in str(e), (k, str(e))
            fired += 1
            continue
        finally:
            left = L.ct_debug_fail_alloc(0)
        # the k-th allocation lies beyond those of ct_create
        assert left > 0
        break
    assert created is not None and fired >= 5
    g = created
    o = O.OracleTable(spec.tuples, spec.lo, spec.dsizes)
    say("alloc failure: slots")
    n0 = g.n_slots
    L.ct_debug_fail_alloc(1)
    with pytest.raises(ct.CTError) as e:
        g.slots_alloc(4, max_depth=8)
    L.ct_debug_fail_alloc(0)
    assert e.value.code == ct.E_NOMEM and g.n_slots == n0
    first = g.slots_alloc(4, max_depth=8)
    say("alloc failure: batch staging on a new stream")
    lay = spec.layout()
    rng = W.rng_for(3, 990, 0)
    din_h = [W.pick_fraction_removal(rng, lay, g.domains(), frac=0.2) for _ in range(4)]
    din = torch.from_numpy(np.stack(din_h).view(np.int64)).cuda()
    dout = torch.zeros_like(din)
    status = torch.full((4,), 99, dtype=torch.int32, device="cuda")
    jobs = [dict(table=g, slot=first + k, flags=ct.JOB_PROPAGATE, n_push=1, dom_in=din[k], dom_out=dout[k])
            for k in range(4)]
    stream = torch.cuda.Stream()
    for k in (1, 2, 3):
        L.ct_debug_fail_alloc(k)
        try:
            ct.propagate_batch(jobs, status, stream)
        except ct.CTError as err:
            assert err.code == ct.E_NOMEM
        finally:
            L.ct_debug_fail_alloc(0)
        torch.cuda.synchronize()
        # whether or not the batch ran, the slots are consistent: reset them
        for s in range(first, first + 4):
            while g.pop(s) == ct.OK:
                pass
    ct.propagate_batch(jobs, status, stream)
    ct.batch_status(stream)
    st = status.cpu().numpy()
    got = dout.cpu().numpy().view(np.uint64)
    for k in range(4):
        o.push()
        os_, od = o.propagate(din_h[k])
        assert st[k] == os_
        if os_ == O.OK:
            assert (got[k] == od).all()
        o.pop()
    # the table's own slot still propagates like the oracle (a level is
    # popped after every failure and every second call: the depth stays
    # within the table's 8 levels)
    for k in range(10):
        d = W.pick_fraction_removal(rng, lay, o.domains())
        assert g.push() == o.push() == 0
        gs, gd = g.propagate(d)
        os_, od = o.propagate(d)
        assert gs == os_
        if os_ == O.OK:
            assert (gd == od).all()
        if os_ != O.OK or k % 2 == 1:
            assert g.pop() == o.pop() == 0
