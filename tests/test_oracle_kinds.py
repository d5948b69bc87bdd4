"""Pins of the oracle's short and negative tables (the table kinds the
paper's footnote on Sec. 2 names: cells that stand for several values, and
tables that list the forbidden combinations).

* short tables (a STAR cell stands for every value of its column): results
  equal brute-force GAC by enumeration under every branch policy, including
  a forced incremental branch on an emptied domain;
* negative tables: results equal the enumeration of the product of the
  domains minus the listed tuples; currTable holds exactly the listed tuples
  whose values are all in the output domains; duplicates and stars are
  refused."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_18413_amd.workloads import DomLayout, rng_for
from tests.bruteforce import STAR, gac_negative, gac_short


def bits_of(words, t):
    return [int((int(words[j // 64]) >> (j % 64)) & 1) for j in range(t)]


def random_subset(rng, lay, dom, p_keep):
    out = dom.copy()
    for i in range(lay.n):
        for a in lay.values(dom, i):
            if rng.random() > p_keep:
                lay.clear(out, i, int(a))
    return out


def short_table(rng):
    n = int(rng.integers(1, 5))
    ds = rng.integers(1, 6, size=n)
    lo = rng.integers(-2, 3, size=n)
    t = int(rng.integers(0, 30))
    tup = np.stack([rng.integers(lo[i] - 1, lo[i] + ds[i] + 1, size=t) for i in range(n)], axis=1) \
        if t else np.zeros((0, n), np.int64)
    tup = tup.astype(np.int64)
    if t:
        tup[rng.random(tup.shape) < 0.25] = STAR
    return n, ds.astype(np.int32), lo.astype(np.int32), tup.astype(np.int32)


def test_short_table_star_rows():
    """A star cell is in every support row of its column (short tables:
    supports[x, a] holds the tuples naming a or a star)."""
    tup = np.array([[0, STAR], [1, 2], [STAR, STAR]], np.int32)
    T = O.OracleTable(tup, [0, 0], [3, 3])
    assert bits_of(T.support_row(0), 3) == [1, 0, 1]   # x0 = 0
    assert bits_of(T.support_row(1), 3) == [0, 1, 1]   # x0 = 1
    assert bits_of(T.support_row(2), 3) == [0, 0, 1]   # x0 = 2
    assert bits_of(T.support_row(3), 3) == [1, 0, 1]   # x1 = 0
    assert bits_of(T.support_row(5), 3) == [1, 1, 1]   # x1 = 2
    lay = DomLayout([3, 3], [0, 0])
    # x0 = {2}: only the all-star tuple is valid, every x1 value stays
    st, dom, ct = T.propagate(lay.from_sets([{2}, {0, 1, 2}]), mode=O.MODE_INCREMENTAL, want_ct=True)
    assert st == O.OK and bits_of(ct, 3) == [0, 0, 1] and lay.to_sets(dom) == [{2}, {0, 1, 2}]


@pytest.mark.parametrize("chunk", range(5))
def test_short_tables_bruteforce(chunk):
    rng = rng_for(21, 120, chunk)
    cases = 0
    for _ in range(120):
        n, ds, lo, tup = short_table(rng)
        lay = DomLayout(ds, lo)
        T = O.OracleTable(tup, lo, ds)
        F = O.OracleTable(tup, lo, ds, fast=True)
        failed, want, valid = gac_short(tup, lo, lay.to_sets(lay.full()))
        assert (T.create_status == O.FAIL) == failed == (F.create_status == O.FAIL)
        if failed:
            continue
        assert lay.to_sets(T.domains()) == want
        for step in range(6):
            dom_in = random_subset(rng, lay, T.domains(), float(rng.uniform(0.2, 1.0)))
            mode = int(rng.integers(0, 3))
            T.push(), F.push()
            st, dom_out, ct = T.propagate(dom_in, mode=mode, want_ct=True)
            sf, df, cf = F.propagate(dom_in, mode=mode, want_ct=True)
            failed, want, valid = gac_short(tup, lo, lay.to_sets(dom_in))
            cases += 1
            assert st == sf == (O.FAIL if failed else O.OK)
            if failed:
                T.pop(), F.pop()
                continue
            assert lay.to_sets(dom_out) == want and (df == dom_out).all()
            assert [j for j in range(T.t) if bits_of(ct, T.t)[j]] == valid and (cf == ct).all()
            if rng.random() < 0.3:
                T.pop(), F.pop()
    assert cases > 200


def negative_table(rng):
    n = int(rng.integers(1, 4))
    ds = rng.integers(1, 5, size=n)
    lo = rng.integers(-2, 3, size=n)
    space = int(np.prod(ds))
    t = int(rng.integers(0, space + 1))
    codes = rng.permutation(space)[:t]
    tup = np.zeros((t, n), np.int64)
    c = codes.copy()
    for i in range(n - 1, -1, -1):
        tup[:, i] = c % ds[i] + lo[i]
        c //= ds[i]
    if t and rng.random() < 0.2:  # a value outside the initial domain: never valid
        tup[0, 0] = lo[0] + ds[0] + 1
    return n, ds.astype(np.int32), lo.astype(np.int32), tup.astype(np.int32)


@pytest.mark.parametrize("chunk", range(5))
def test_negative_tables_bruteforce(chunk):
    rng = rng_for(22, 121, chunk)
    cases = 0
    for _ in range(120):
        n, ds, lo, tup = negative_table(rng)
        lay = DomLayout(ds, lo)
        init = random_subset(rng, lay, lay.full(), 0.85) if rng.random() < 0.3 else None
        T = O.OracleTable(tup, lo, ds, init_dom=init, kind=O.KIND_NEGATIVE)
        start = lay.full() if init is None else init
        failed, want, valid = gac_negative(tup, lo, lay.to_sets(start))
        assert (T.create_status == O.FAIL) == failed
        if failed:
            continue
        dom, ct, _ = T.state()
        assert lay.to_sets(dom) == want
        assert [j for j in range(T.t) if bits_of(ct, T.t)[j]] == valid
        for step in range(6):
            dom_in = random_subset(rng, lay, T.domains(), float(rng.uniform(0.3, 1.0)))
            mode = int(rng.integers(0, 3))
            T.push()
            st, dom_out, ct = T.propagate(dom_in, mode=mode, want_ct=True)
            failed, want, valid = gac_negative(tup, lo, lay.to_sets(dom_in))
            cases += 1
            assert st == (O.FAIL if failed else O.OK)
            if failed:
                assert T.pop() == O.OK
                continue
            assert lay.to_sets(dom_out) == want
            assert [j for j in range(T.t) if bits_of(ct, T.t)[j]] == valid
            if rng.random() < 0.3:
                T.pop()
    assert cases > 150


def test_negative_table_worked_example():
    """x, y in {0, 1, 2}; forbidden: every pair with x = 0, and (1, 1).
    Root: x = 0 has no allowed pair -> x in {1, 2}; y keeps {0, 1, 2}.
    Then y = {1}: (1, 1) is forbidden, so x = {2}."""
    tup = np.array([[0, 0], [0, 1], [0, 2], [1, 1]], np.int32)
    lay = DomLayout([3, 3], [0, 0])
    T = O.OracleTable(tup, [0, 0], [3, 3], kind=O.KIND_NEGATIVE)
    dom, ct, f = T.state()
    assert T.create_status == O.OK and lay.to_sets(dom) == [{1, 2}, {0, 1, 2}]
    assert bits_of(ct, 4) == [0, 0, 0, 1]      # only (1, 1) is still within the domains
    st, dom, ct = T.propagate(lay.from_sets([{1, 2}, {1}]), want_ct=True)
    assert st == O.OK and lay.to_sets(dom) == [{2}, {1}] and bits_of(ct, 4) == [0, 0, 0, 0]
    assert T.propagate(lay.from_sets([{2}, set()]))[0] == O.FAIL


def test_negative_table_refuses_duplicates_and_stars():
    with pytest.raises(ValueError):
        O.OracleTable(np.array([[0, 1], [0, 1]], np.int32), [0, 0], [2, 2], kind=O.KIND_NEGATIVE)
    with pytest.raises(ValueError):
        O.OracleTable(np.array([[0, STAR]], np.int32), [0, 0], [2, 2], kind=O.KIND_NEGATIVE)
