"""Slot lifetime through the C ABI: ct_slots_alloc / ct_slots_free.

A released slot answers every call with CT_E_INVALID; ct_slots_alloc hands
released slots out again (same ids), reset to the root state, and a reused
slot then propagates exactly like the oracle from the root."""
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


def test_free_then_alloc_reuses_and_resets():
    spec = W.large_table(11, t=20_000, d=20, n=4)
    say("slots: alloc/free/alloc on a 20,000-tuple table")
    g = ct.Table(spec.tuples, spec.lo, spec.dsizes, max_depth=8)
    lay = spec.layout()
    root = g.domains()
    first = g.slots_alloc(4, max_depth=8)
    assert first == 1
    rng = W.rng_for(11, 900, 0)
    # dirty slots 2 and 3: push and propagate
    for s in (2, 3):
        assert g.push(s) == ct.OK
        st, _ = g.propagate(W.pick_fraction_removal(rng, lay, root, frac=0.3), slot=s)
        assert st in (ct.OK, ct.FAIL)
    g.slots_free(2, 2)
    # every call on a freed slot is rejected
    assert g.push(2) == ct.E_INVALID
    assert g.pop(3) == ct.E_INVALID
    assert g.propagate(root, slot=2)[0] == ct.E_INVALID
    with pytest.raises(ct.CTError):
        g.state(3)
    with pytest.raises(ct.CTError):
        g.stats(2)
    din = torch.from_numpy(root.view(np.int64)).cuda()
    dout = torch.zeros_like(din)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(ct.CTError):
        ct.propagate_batch([dict(table=g, slot=3, flags=ct.JOB_PROPAGATE, dom_in=din, dom_out=dout)], status)
    # double free, slot 0, out of range
    with pytest.raises(ct.CTError):
        g.slots_free(2, 1)
    with pytest.raises(ct.CTError):
        g.slots_free(0, 1)
    with pytest.raises(ct.CTError):
        g.slots_free(4, 2)
    n_before = g.n_slots
    # a run of two freed slots is reused, both reset to the root state
    again = g.slots_alloc(2, max_depth=8)
    assert again == 2 and g.n_slots == n_before
    o = O.OracleTable(spec.tuples, spec.lo, spec.dsizes)
    od, oc, _ = o.state()
    for s in (2, 3):
        gd, gc = g.state(s)
        assert (gd == od).all() and (gc == oc).all(), s
        assert g.pop(s) == ct.E_STATE  # depth 0 after reuse
    # the reused slot propagates like the oracle (a level is popped after
    # every failure and every second call: at most 7 of its 8 levels)
    for k in range(14):
        din_k = W.pick_fraction_removal(rng, lay, o.domains())
        assert g.push(2) == o.push() == ct.OK
        gs, gdom, gct = g.propagate(din_k, slot=2, want_ct=True)
        os_, odom, oct_ = o.propagate(din_k, want_ct=True)
        assert gs == os_, k
        if os_ == O.OK:
            assert (gdom == odom).all() and (gct == oct_).all(), k
        if os_ != O.OK or k % 2 == 1:
            assert g.pop(2) == o.pop() == ct.OK
    # a larger depth than the freed slots hold takes new slots
    g.slots_free(1, 1)
    deeper = g.slots_alloc(1, max_depth=16)
    assert deeper == n_before
    # the freed shallow slot is reused by a request that fits it
    assert g.slots_alloc(1, max_depth=4) == 1
    g.close()
