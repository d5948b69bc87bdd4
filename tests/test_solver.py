"""The search driver (paper_2507_18413_amd/solver.py) on the CPU: with the
oracle's tables as the table propagator it must find exactly the solutions
that enumerating the Cartesian product finds, on tiny generated models."""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_18413_amd import solver as S
from paper_2507_18413_amd.workloads import DomLayout


class OracleTables:
    def __init__(self, dsz, tables):
        self.scopes = [sc for _, sc in tables]
        self.ots = [O.OracleTable(t, np.zeros(len(sc), np.int32), dsz[sc]) for t, sc in tables]
        self.lay = DomLayout(dsz, np.zeros_like(dsz))
        self.props = 0

    def fixpoint(self, pool):
        st, out, props = O.fixpoint(self.ots, self.scopes, self.lay, pool)
        self.props += props
        return st != O.OK, (out if st == O.OK else pool)

    def push(self):
        for o in self.ots:
            o.push()

    def pop(self):
        for o in self.ots:
            o.pop()


def brute_force(dsz, tables, w, cap):
    sols = []
    rels = [(set(map(tuple, t.tolist())), list(sc)) for t, sc in tables]
    for x in itertools.product(*[range(int(d)) for d in dsz]):
        if sum(int(a) * b for a, b in zip(w, x)) > cap:
            continue
        if all(tuple(x[i] for i in sc) in rel for rel, sc in rels):
            sols.append(x)
    return sols


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_search_finds_exactly_the_solutions(seed):
    dsz, tables, w, cap = S.lin_model(seed, n_vars=6, d=4, n_tables=3, arity=3, density=(0.3, 0.7))
    lay = DomLayout(dsz, np.zeros_like(dsz))
    s = S.Search(lay, OracleTables(dsz, tables), S.LinearLE(lay, range(lay.n), w, cap))
    s.run(lay.full(), 10 ** 6, 10 ** 6)
    got = sorted(tuple(int(min(v)) for v in sol) for sol in s.solutions)
    assert got == sorted(brute_force(dsz, tables, w, cap))
    assert s.nodes >= len(got)


def test_linear_bounds_reasoning():
    lay = DomLayout(np.array([5, 5], np.int32), np.zeros(2, np.int32))
    lin = S.LinearLE(lay, [0, 1], [2, 3], 9)
    failed, out = lin.propagate(lay.full())
    assert not failed
    # x0 <= (9 - 0) // 2 = 4, x1 <= 9 // 3 = 3
    assert lay.to_sets(out) == [{0, 1, 2, 3, 4}, {0, 1, 2, 3}]
    pool = lay.from_sets([[4], [0, 1, 2, 3, 4]])
    failed, out = lin.propagate(pool)
    assert lay.to_sets(out) == [{4}, {0}]
    failed, _ = lin.propagate(lay.from_sets([[4], [2, 3]]))
    assert failed


# --------------------------------------------------------------------------
# the paper's instance form: one table over every variable and one linear
# equation over some of them, searched with input order / largest value
# first (Sec. 5.1)
# --------------------------------------------------------------------------
def brute_force_eq(tup, E, w, c):
    return sorted(tuple(int(v) for v in row) for row in tup
                  if int(sum(int(a) * int(b) for a, b in zip(w, row[E]))) == c)


def test_linear_equation_bounds_reasoning():
    lay = DomLayout(np.array([5, 5, 4], np.int32), np.zeros(3, np.int32))
    eq = S.LinearEQ(lay, [0, 1], [2, 3], 8)
    failed, out = eq.propagate(lay.full())
    # 2 x0 + 3 x1 = 8 with x0, x1 in {0..4}: x1 <= 8 // 3 = 2 and x0 >= (8 - 6) // 2 = 1;
    # then x0 <= (8 - 0) // 2 = 4 and nothing else by bounds; x2 is untouched
    assert not failed
    assert lay.to_sets(out) == [{1, 2, 3, 4}, {0, 1, 2}, {0, 1, 2, 3}]
    failed, out = eq.propagate(lay.from_sets([[4], [0, 1, 2, 3, 4], [0]]))
    assert not failed and lay.to_sets(out)[1] == {0}
    failed, _ = eq.propagate(lay.from_sets([[4], [1, 2], [0]]))
    assert failed
    failed, _ = eq.propagate(lay.from_sets([[0], [0], [0]]))
    assert failed


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_lin_instance_first_solution_is_the_lexicographic_maximum(seed):
    """input_order + indomain_max, complete: the first solution is the
    lexicographically largest solution, and all-solutions search finds
    exactly the table rows that satisfy the equation."""
    from paper_2507_18413_amd import workloads as W
    spec, E, w, c = W.lin_instance(seed, n=7, dom=(2, 6), t=300, eq_frac=0.6, weights=(1, 5))
    lay = spec.layout()
    want = brute_force_eq(spec.tuples, E, w, c)
    assert want  # the planted configuration
    for sols in (1, 10 ** 6):
        o = O.OracleTable(spec.tuples, spec.lo, spec.dsizes, fast=True)
        s = S.Search(lay, S.OneTable(o), S.LinearEQ(lay, E, w, c), var_order="input", val_order="max")
        s.run(lay.full(), 10 ** 6, sols)
        got = [tuple(int(min(v)) for v in sol) for sol in s.solutions]
        if sols == 1:
            assert got == [max(want)]
        else:
            assert sorted(got) == want
