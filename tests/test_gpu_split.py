"""Parity of the split propagators (updateTable or filterDomains on the
device, the other procedure on the host; Sec. 4.1 and 4.2) with the CPU
oracle, call by call, bit-exact: statuses, domains and currTable after
every operation, through the C ABI."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_18413_amd import ct
from paper_2507_18413_amd import workloads as W

from .test_gpu_parity import GOLDEN, random_case, random_subset, say

pytestmark = pytest.mark.gpu
MODES = [ct.SPLIT_UPDATE, ct.SPLIT_FILTER]


def split_pair(tup, lo, ds, mode, init=None, policy=ct.BRANCH_AUTO):
    say("split create", f"t={len(tup)}", f"n={len(ds)}", f"mode={mode}", f"policy={policy}")
    G = ct.Table(tup, lo, ds, init_dom=init, branch_policy=policy)
    S = ct.SplitPropagator(G, mode)
    Ot = O.OracleTable(tup, lo, ds, init_dom=init)
    return G, S, Ot


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("chunk", range(3))
def test_split_random_sequences_vs_oracle(mode, chunk):
    """Random small tables (empty, one tuple, ragged word tails, duplicate
    tuples, restricted initial domains, every branch policy) and random
    sequences of removals, pushes and pops."""
    rng = W.rng_for(chunk, 205, mode)
    for case in range(10):
        tup, lo, ds = random_case(rng)
        lay = W.DomLayout(ds, lo)
        init = random_subset(rng, lay, lay.full(), 0.8) if rng.random() < 0.3 else None
        policy = int(rng.integers(0, 3))
        say(f"mode={mode} chunk={chunk} case={case}")
        G, S, Ot = split_pair(tup, lo, ds, mode, init=init, policy=policy)
        root = Ot.domains()
        if Ot.create_status == O.FAIL:
            assert S.propagate(root)[0] == ct.E_STATE
            continue
        for step in range(25):
            r = rng.random()
            if r < 0.25 and Ot.depth > 0:
                assert S.pop() == ct.OK and Ot.pop() == O.OK
                continue
            if r < 0.6:
                assert S.push() == Ot.push()
            dom = Ot.domains()
            dom_in = random_subset(rng, lay, dom, float(rng.uniform(0.5, 1.0)))
            if rng.random() < 0.05:
                dom_in = lay.full()
            gs, gd, gc = S.propagate(dom_in, want_ct=True)
            os_, od, oc = Ot.propagate(dom_in, want_ct=True)
            assert gs == os_, (step, gs, os_)
            if os_ == O.OK:
                assert (gd == od).all(), step
                assert (gc == oc).all(), step
            if os_ == O.FAIL:
                assert not gc.any()
                if Ot.depth > 0:
                    assert S.pop() == ct.OK and Ot.pop() == O.OK
                else:
                    assert S.push() == ct.E_STATE and Ot.push() == O.E_STATE
                    break
        S.close()


def run_split_plain(spec, mode, n_calls, picker, family):
    G, S, Ot = split_pair(spec.tuples, spec.lo, spec.dsizes, mode)
    lay = spec.layout()
    rng = W.rng_for(W.DEFAULT_SEED, family, 9)
    bt = W.Backtracker(rng)
    depth = 0
    for call in range(n_calls):
        dom_in = picker(rng, lay, Ot.domains())
        assert S.push() == ct.OK and Ot.push() == O.OK
        depth += 1
        gs, gd, gc = S.propagate(dom_in, want_ct=True)
        os_, od, oc = Ot.propagate(dom_in, want_ct=True)
        assert gs == os_, (call, gs, os_)
        if os_ == O.OK:
            assert (gd == od).all(), call
            assert (gc == oc).all(), call
        for _ in range(bt.pops_after(os_ == O.FAIL, depth)):
            assert S.pop() == ct.OK and Ot.pop() == O.OK
            depth -= 1
    return G, S, Ot


@pytest.mark.parametrize("mode", MODES)
def test_split_tiny_table(mode):
    say("split tiny table: arity 3, d=8, 200 tuples, 100 calls, mode", mode)
    run_split_plain(W.tiny_table(), mode, 100, W.pick_small_removal, 1)


@pytest.mark.parametrize("mode", MODES)
def test_split_large_table(mode):
    say("split large table: arity 5, d=50, 200,000 tuples, 1,000 calls, mode", mode)
    G, S, Ot = run_split_plain(W.large_table(), mode, 1000, W.pick_fraction_removal, 2)
    assert G.W == 3125


@pytest.mark.parametrize("mode", MODES)
def test_split_wide_scope(mode):
    """227 domain words (one filter wave each) and 11,072 support rows."""
    say("split wide scope: arity 100, d in [64,160], 10,000 tuples, 200 calls, mode", mode)
    G, S, Ot = run_split_plain(W.wide_table(), mode, 200, W.pick_fraction_removal, 6)
    assert G.D == 227 and G.rows == 11072


@pytest.mark.parametrize("mode", MODES)
def test_split_errors_and_table_untouched(mode):
    g = json.load(open(GOLDEN))
    tup = np.array(g["tuples"], np.int32)
    G, S, Ot = split_pair(tup, g["lo"], g["dsizes"], mode)
    lay = W.DomLayout(g["dsizes"], g["lo"])
    root = Ot.domains()
    stray = root.copy()
    stray[0] |= np.uint64(1 << 5)
    assert S.propagate(stray)[0] == ct.E_INVALID
    grow = root.copy()
    grow[2] |= np.uint64(1 << 1)
    assert S.propagate(grow)[0] == ct.E_NOT_SUBSET
    assert S.pop() == ct.E_STATE
    st, d, c = S.propagate(root, want_ct=True)
    os_, od, oc = Ot.propagate(root, want_ct=True)
    assert st == os_ == ct.OK and (d == od).all() and (c == oc).all()
    assert S.push() == ct.OK
    empty = lay.from_sets([[], [0, 1, 2, 3], [0, 2]])
    assert S.propagate(empty)[0] == ct.FAIL
    assert S.propagate(root)[0] == ct.E_STATE
    assert S.push() == ct.E_STATE
    assert S.pop() == ct.OK
    st, d, c = S.propagate(root, want_ct=True)
    assert st == ct.OK and (d == od).all() and (c == oc).all()
    # the table's own slot never moved
    gd, gc = G.state(0)
    assert (gd == root).all()
    with pytest.raises(ct.CTError):
        ct.SplitPropagator(G, 7)
    S.close()


@pytest.mark.parametrize("mode", MODES)
def test_split_created_right_after_engine_calls(mode):
    """A split propagator created on a table whose resident engine has just
    served calls (still alive, holding slot 0 in LDS) starts from the root
    and matches the oracle from its first call: its host copies of the
    supports and of the root state have landed before the first call."""
    spec = W.large_table(t=20_000)
    lay = spec.layout()
    G = ct.Table(spec.tuples, spec.lo, spec.dsizes)
    Ot = O.OracleTable(spec.tuples, spec.lo, spec.dsizes)
    rng = W.rng_for(W.DEFAULT_SEED, 206, mode)
    root = Ot.domains()
    for _ in range(20):  # engine calls on slot 0, each from the root and popped
        assert G.push() == ct.OK
        G.propagate(W.pick_fraction_removal(rng, lay, root))
        assert G.pop() == ct.OK
    say("split created after engine calls, mode", mode, "resident", G.resident)
    S = ct.SplitPropagator(G, mode)
    for call in range(50):
        dom_in = W.pick_fraction_removal(rng, lay, Ot.domains())
        gs, gd, gc = S.propagate(dom_in, want_ct=True)
        os_, od, oc = Ot.propagate(dom_in, want_ct=True)
        assert gs == os_, call
        if os_ != O.OK:
            break
        assert (gd == od).all() and (gc == oc).all(), call
    S.close()
