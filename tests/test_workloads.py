"""Seeded generators: determinism and the shapes the workloads promise."""
import numpy as np
import pytest

from paper_2507_18413_amd import workloads as W


def test_same_seed_same_bytes():
    a = W.tiny_table(7)
    b = W.tiny_table(7)
    c = W.tiny_table(8)
    assert a.tuples.tobytes() == b.tuples.tobytes()
    assert a.tuples.tobytes() != c.tuples.tobytes()


def test_tiny_table_shape_distinct():
    s = W.tiny_table()
    assert s.tuples.shape == (200, 3)
    assert s.tuples.min() >= 0 and s.tuples.max() <= 7
    assert len({tuple(r) for r in s.tuples.tolist()}) == 200


def test_distinct_uniform_small_space():
    rng = W.rng_for(1, 99, 0)
    t = W.distinct_uniform_tuples(rng, [3, 4], 12)          # whole space
    assert len({tuple(r) for r in t.tolist()}) == 12


def test_zipf_skew_and_distinct():
    rng = W.rng_for(1, 98, 0)
    t = W.distinct_zipf_tuples(rng, 3, 20, 1.1, 4000)
    assert len({tuple(r) for r in t.tolist()}) == 4000
    counts = np.bincount(t[:, 0], minlength=20)
    assert counts[0] > counts[19]                           # rank 1 most frequent


def test_layout_roundtrip():
    lay = W.DomLayout([3, 64, 65, 130], [0, 5, -2, 0])
    assert list(lay.words) == [1, 1, 2, 3] and lay.D == 7
    full = lay.full()
    assert [lay.count(full, i) for i in range(4)] == [3, 64, 65, 130]
    sets = [{0, 2}, {63}, {64, 1}, {129, 0, 77}]
    assert lay.to_sets(lay.from_sets(sets)) == sets


def test_removal_pickers_only_remove():
    lay = W.DomLayout([50] * 5, [0] * 5)
    rng = W.rng_for(3, 97, 0)
    dom = lay.full()
    for _ in range(20):
        new = W.pick_fraction_removal(rng, lay, dom)
        assert not (new & ~dom).any()
        removed = sum(lay.count(dom, i) - lay.count(new, i) for i in range(5))
        assert 1 <= removed <= 3 * 3
        dom = new
    lay1 = W.DomLayout([8] * 3, [0] * 3)
    d1 = lay1.full()
    new = W.pick_small_removal(rng, lay1, d1)
    removed = sum(lay1.count(d1, i) - lay1.count(new, i) for i in range(3))
    assert removed in (1, 2)


def test_distinct_generators_reject_more_tuples_than_the_space():
    rng = W.rng_for(1, 900, 0)
    with pytest.raises(ValueError):
        W.distinct_uniform_tuples(rng, [3, 4], 13)
    with pytest.raises(ValueError):
        W.distinct_zipf_tuples(rng, 2, 3, 1.1, 10)
    with pytest.raises(ValueError):
        W._distinct_zipf_mixed(rng, np.array([27, 14, 8], np.int64), 1.1, 3025)
    assert W._distinct_zipf_mixed(rng, np.array([3, 4], np.int64), 1.1, 12).shape == (12, 2)


def test_wide_table_shape_and_determinism():
    a = W.wide_table()
    b = W.wide_table()
    assert a.n == 100 and a.t == 10_000
    assert (a.tuples == b.tuples).all() and (a.dsizes == b.dsizes).all()
    assert a.dsizes.min() >= 64 and a.dsizes.max() <= 160
    assert (a.tuples >= 0).all() and (a.tuples < a.dsizes[None, :]).all()
    assert np.unique(a.tuples, axis=0).shape[0] == a.t
