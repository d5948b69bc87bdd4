"""Pins of the CPU oracle against things other than itself: the paper's
Table 1, brute-force GAC by enumeration, and exact invariants."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_18413_amd.workloads import DomLayout, rng_for
from tests.bruteforce import closure, gac

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1.json")


def bits_of(words, t):
    return [int((int(words[j // 64]) >> (j % 64)) & 1) for j in range(t)]


def table1():
    g = json.load(open(GOLDEN))
    tup = np.array(g["tuples"], np.int32)
    return g, O.OracleTable(tup, g["lo"], g["dsizes"])


# --------------------------------------------------------------------------
# Table 1 of the paper
# --------------------------------------------------------------------------
def test_table1_printed_support_rows():
    g, T = table1()
    names = {"x1": 0, "x2": 1, "x3": 2}
    for name, want in g["printed_support_rows"].items():
        if name == "comment":
            continue
        var, val = name.split("=")
        i = names[var]
        row = 4 * i + int(val) - g["lo"][i]          # prefix sums of |dom0| = 0, 4, 8
        assert bits_of(T.support_row(row), 5) == want, name


def test_table1_printed_currtable():
    g, T = table1()
    lay = DomLayout(g["dsizes"], g["lo"])
    d = g["derived"]
    dom_in = lay.from_sets([[v - 1 for v in s] for s in d["dom_giving_printed_currtable"]])
    st, dom_out, ct = T.propagate(dom_in, want_ct=True)
    assert st == O.OK
    assert bits_of(ct, 5) == g["printed_currtable"]
    assert lay.to_sets(dom_out) == [set(v - 1 for v in s) for s in d["gac_after_x1_eq_1"]]


def test_table1_root():
    g, T = table1()
    lay = DomLayout(g["dsizes"], g["lo"])
    dom, ct, failed = T.state()
    assert not failed and T.create_status == O.OK
    assert lay.to_sets(dom) == [set(v - 1 for v in s) for s in g["derived"]["root_gac"]]
    assert bits_of(ct, 5) == g["derived"]["root_currtable"]


# --------------------------------------------------------------------------
# brute force on tiny random tables
# --------------------------------------------------------------------------
def random_tiny(rng):
    n = int(rng.integers(1, 5))
    ds = rng.integers(1, 7, size=n)
    lo = rng.integers(-3, 4, size=n)
    t = int(rng.integers(0, 41))
    # values may fall one below / above the initial interval (never valid)
    tup = np.stack([rng.integers(lo[i] - 1, lo[i] + ds[i] + 1, size=t) for i in range(n)], axis=1) \
        if t else np.zeros((0, n), np.int64)
    if t and rng.random() < 0.3:                          # duplicates
        tup = np.concatenate([tup, tup[: max(1, t // 4)]])
    return n, ds.astype(np.int32), lo.astype(np.int32), tup.astype(np.int32)


def random_subset(rng, lay, dom, p_keep):
    out = dom.copy()
    for i in range(lay.n):
        for a in lay.values(dom, i):
            if rng.random() > p_keep:
                lay.clear(out, i, int(a))
    return out


@pytest.mark.parametrize("chunk", range(8))
def test_bruteforce_sequences(chunk):
    rng = rng_for(11, 100, chunk)
    cases = 0
    for _ in range(120):
        n, ds, lo, tup = random_tiny(rng)
        lay = DomLayout(ds, lo)
        init = None
        if rng.random() < 0.3:
            init = random_subset(rng, lay, lay.full(), 0.8)
        T = O.OracleTable(tup, lo, ds, init_dom=init)
        start = lay.full() if init is None else init
        failed, want, valid = gac(tup, lo, lay.to_sets(start))
        dom, ct, f = T.state()
        assert f == failed
        if failed:
            assert T.create_status == O.FAIL
            continue
        assert lay.to_sets(dom) == want
        assert [j for j in range(T.t) if bits_of(ct, T.t)[j]] == valid
        for step in range(6):
            dom_prev, _, _ = T.state()
            dom_in = random_subset(rng, lay, dom_prev, float(rng.uniform(0.4, 1.0)))
            mode = int(rng.integers(0, 3))
            T.push()
            st, dom_out, ct = T.propagate(dom_in, mode=mode, want_ct=True)
            failed, want, valid = gac(tup, lo, lay.to_sets(dom_in))
            cases += 1
            if failed:
                assert st == O.FAIL
                assert not ct.any()
                assert T.pop() == O.OK
                continue
            assert st == O.OK
            assert lay.to_sets(dom_out) == want
            assert [j for j in range(T.t) if bits_of(ct, T.t)[j]] == valid
            if rng.random() < 0.3:
                T.pop()
    assert cases > 200


def test_invalid_inputs():
    g, T = table1()
    lay = DomLayout(g["dsizes"], g["lo"])
    root = T.domains()
    stray = root.copy()
    stray[0] |= np.uint64(1 << 5)                 # bit beyond d = 4
    assert T.propagate(stray)[0] == O.E_INVALID
    grow = root.copy()
    grow[2] |= np.uint64(1 << 1)                  # x3 = 2 was pruned at the root
    assert T.propagate(grow)[0] == O.E_NOT_SUBSET
    assert T.pop() == O.E_STATE                   # depth 0
    # no state change after the errors
    dom, ct, f = T.state()
    assert (dom == root).all() and not f
    # failure, then only pop is accepted
    assert T.push() == O.OK
    empty = lay.from_sets([[], [0, 1, 2, 3], [0, 2]])
    assert T.propagate(empty)[0] == O.FAIL
    assert T.propagate(root)[0] == O.E_STATE
    assert T.push() == O.E_STATE
    assert T.pop() == O.OK
    dom, ct, f = T.state()
    assert (dom == root).all() and not f and bits_of(ct, 5) == [1] * 5


# --------------------------------------------------------------------------
# invariants on a medium table
# --------------------------------------------------------------------------
def medium(seed=3, n=4, d=9, t=900):
    from paper_2507_18413_amd.workloads import distinct_uniform_tuples
    rng = rng_for(seed, 101, 0)
    tup = distinct_uniform_tuples(rng, [d] * n, t)
    return tup, np.zeros(n, np.int32), np.full(n, d, np.int32)


def valid_mask(tup, lo, lay, dom):
    sets = lay.to_sets(dom)
    ok = np.ones(tup.shape[0], bool)
    for i in range(lay.n):
        ok &= np.isin(tup[:, i] - lo[i], list(sets[i]) or [-10**9])
    return ok


def test_invariants_and_modes():
    tup, lo, ds = medium()
    lay = DomLayout(ds, lo)
    Ts = [O.OracleTable(tup, lo, ds) for _ in range(3)]
    rng = rng_for(5, 102, 0)
    t = tup.shape[0]
    for step in range(60):
        dom = Ts[0].domains()
        dom_in = random_subset(rng, lay, dom, 0.85)
        ct_before = Ts[0].state()[1]
        res = []
        for m, T in enumerate(Ts):
            T.push()
            res.append(T.propagate(dom_in, mode=m, want_ct=True))
        st, dom_out, ct = res[0]
        for st2, d2, c2 in res[1:]:          # reset, incremental and auto agree
            assert st2 == st
            if st == O.OK:
                assert (d2 == dom_out).all() and (c2 == ct).all()
        want_valid = valid_mask(tup, lo, lay, dom_in)
        got_valid = np.array(bits_of(ct, t), bool)
        assert (got_valid == want_valid).all()          # currTable = valid tuples
        assert not (ct & ~ct_before).any()              # only shrinks
        if st == O.FAIL:
            assert not want_valid.any()
            for T in Ts:
                T.pop()
            continue
        assert not (dom_out & ~dom_in).any()            # dom_out subset of dom_in
        # each valid tuple has one value per column
        for i in range(lay.n):
            total = 0
            for a in lay.values(dom_out, i):
                row = Ts[0].support_row(int(lay.off[i] * 0 + sum(ds[:i]) + a))
                total += int(sum(bin(int(x)).count("1") for x in (row & ct)))
            assert total == int(got_valid.sum())
        # idempotence
        for T in Ts:
            T.push()
        st2, d2, c2 = Ts[0].propagate(dom_out, want_ct=True)
        assert st2 == O.OK and (d2 == dom_out).all() and (c2 == ct).all()
        for T in Ts[1:]:
            T.propagate(dom_out)
        for T in Ts:
            T.pop()
        if rng.random() < 0.25:
            snap = [T.state() for T in Ts]
            for T in Ts:
                T.pop()
                T.push()
                T.pop()


def test_push_pop_restores_exactly():
    tup, lo, ds = medium(seed=9)
    lay = DomLayout(ds, lo)
    T = O.OracleTable(tup, lo, ds)
    rng = rng_for(6, 103, 0)
    stack = []
    for step in range(80):
        if stack and rng.random() < 0.3:
            want = stack.pop()
            assert T.pop() == O.OK
            got = T.state()
            assert (got[0] == want[0]).all() and (got[1] == want[1]).all() and got[2] == want[2]
            continue
        stack.append(T.state())
        T.push()
        dom = T.domains()
        st, _ = T.propagate(random_subset(rng, lay, dom, 0.8))
        if st == O.FAIL:
            want = stack.pop()
            T.pop()
            got = T.state()
            assert (got[0] == want[0]).all() and (got[1] == want[1]).all()
    assert T.depth == len(stack)


# --------------------------------------------------------------------------
# multi-table fixpoint
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(6))
def test_fixpoint_against_naive_closure(seed):
    rng = rng_for(seed, 104, 0)
    n_pool = int(rng.integers(3, 7))
    pool_ds = rng.integers(2, 5, size=n_pool).astype(np.int32)
    lay = DomLayout(pool_ds, np.zeros(n_pool, np.int32))
    tables, scopes, oracles = [], [], []
    for c in range(int(rng.integers(2, 6))):
        k = int(rng.integers(1, min(4, n_pool) + 1))
        scope = rng.choice(n_pool, size=k, replace=False).astype(np.int32)
        ds = pool_ds[scope]
        t = int(rng.integers(1, 12))
        tup = np.stack([rng.integers(0, ds[i], size=t) for i in range(k)], axis=1).astype(np.int32)
        tables.append((tup, np.zeros(k, np.int32)))
        scopes.append(scope)
    for trial in range(4):
        oracles = [O.OracleTable(tp, lo, pool_ds[s]) for (tp, lo), s in zip(tables, scopes)]
        start = random_subset(rng, lay, lay.full(), 0.9)
        failed, want = closure(tables, scopes, lay.to_sets(start))
        order = rng.permutation(len(tables)).astype(np.int32)
        st, pool_out, props = O.fixpoint(oracles, scopes, lay, start, order=order)
        if any(o.create_status == O.FAIL for o in oracles):
            assert failed
            continue
        assert (st == O.FAIL) == failed
        if not failed:
            assert lay.to_sets(pool_out) == want


@pytest.mark.parametrize("seed", range(6))
def test_seeded_fixpoint_after_a_fixpoint_equals_the_closure(seed):
    """After a fixpoint, a search step that removes values of some pool
    variables needs only the tables whose scope holds one of them: the
    fixpoint seeded with those tables equals the enumeration closure (and the
    fixpoint seeded with every table)."""
    rng = rng_for(seed, 105, 0)
    n_pool = int(rng.integers(4, 8))
    pool_ds = rng.integers(2, 5, size=n_pool).astype(np.int32)
    lay = DomLayout(pool_ds, np.zeros(n_pool, np.int32))
    tables, scopes = [], []
    for c in range(int(rng.integers(3, 7))):
        k = int(rng.integers(1, min(4, n_pool) + 1))
        scope = rng.choice(n_pool, size=k, replace=False).astype(np.int32)
        ds = pool_ds[scope]
        t = int(rng.integers(2, 20))
        tup = np.stack([rng.integers(0, ds[i], size=t) for i in range(k)], axis=1).astype(np.int32)
        tables.append((tup, np.zeros(k, np.int32)))
        scopes.append(scope)
    checked = 0
    for trial in range(6):
        seeded = [O.OracleTable(tp, lo, pool_ds[s]) for (tp, lo), s in zip(tables, scopes)]
        full = [O.OracleTable(tp, lo, pool_ds[s]) for (tp, lo), s in zip(tables, scopes)]
        if any(o.create_status == O.FAIL for o in seeded):
            break
        st, root, _ = O.fixpoint(seeded, scopes, lay, lay.full())
        O.fixpoint(full, scopes, lay, lay.full())
        if st != O.OK:
            break
        pool = root
        for step in range(4):
            new = random_subset(rng, lay, pool, 0.8)
            changed = [v for v in range(n_pool) if lay.to_sets(new)[v] != lay.to_sets(pool)[v]]
            touch = [c for c, sc in enumerate(scopes) if set(int(v) for v in sc) & set(changed)]
            for o in seeded + full:
                o.push()
            st_s, out_s, props_s = O.fixpoint(seeded, scopes, lay, new, seed=touch)
            st_f, out_f, _ = O.fixpoint(full, scopes, lay, new)
            failed, want = closure(tables, scopes, lay.to_sets(new))
            assert (st_s == O.FAIL) == (st_f == O.FAIL) == failed
            assert props_s <= len(tables) * 64
            checked += 1
            if failed:
                for o in seeded + full:
                    o.pop()
                continue
            assert lay.to_sets(out_s) == want == lay.to_sets(out_f)
            pool = out_s
    assert checked > 0
