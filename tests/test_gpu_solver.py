"""The search driver with the library's tables on the GPU explores the same
tree as with the oracle's tables: same nodes, failures and solutions."""
import sys

import numpy as np
import pytest

from paper_2507_18413_amd import solver as S
from paper_2507_18413_amd.workloads import DomLayout

from .test_solver import OracleTables

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed,kw", [
    (5, dict(n_vars=16, d=6, n_tables=5, arity=4, density=(0.1, 0.3))),
    (6, dict(n_vars=24, d=10, n_tables=8, arity=6, density=(0.002, 0.01))),
])
def test_search_tree_equals_oracle(seed, kw):
    print("[gpu-case] solver", seed, kw, flush=True)
    sys.stdout.flush()
    dsz, tables, w, cap = S.lin_model(seed, **kw)
    lay = DomLayout(dsz, np.zeros_like(dsz))
    M, tabs = S.build_gpu(dsz, tables)
    g = S.Search(lay, S.GpuTables(M, lay.D), S.LinearLE(lay, range(lay.n), w, cap))
    g.run(lay.full(), 300, 50)
    o = S.Search(lay, OracleTables(dsz, tables), S.LinearLE(lay, range(lay.n), w, cap))
    o.run(lay.full(), 300, 50)
    assert (g.nodes, g.fails) == (o.nodes, o.fails)
    assert g.solutions == o.solutions
    assert g.nodes > 10


def test_lin_instance_search_tree_equals_oracle():
    """One table over every variable and one linear equation (the paper's
    first test set, Sec. 5.1), input order and largest value first, all
    solutions: the GPU table gives the oracle table's tree."""
    from oracle import oracle as O
    from paper_2507_18413_amd import ct
    from paper_2507_18413_amd import workloads as W
    print("[gpu-case] lin instance search", flush=True)
    spec, E, w, c = W.lin_instance(11, n=50, dom=(2, 60), t=2500, eq_frac=1.0)
    lay = spec.layout()
    g = S.Search(lay, S.OneTable(ct.Table(spec.tuples, spec.lo, spec.dsizes)), S.LinearEQ(lay, E, w, c),
                 var_order="input", val_order="max")
    g.run(lay.full(), 10 ** 6, 10 ** 6)
    o = S.Search(lay, S.OneTable(O.OracleTable(spec.tuples, spec.lo, spec.dsizes, fast=True)),
                 S.LinearEQ(lay, E, w, c), var_order="input", val_order="max")
    o.run(lay.full(), 10 ** 6, 10 ** 6)
    assert (g.nodes, g.fails) == (o.nodes, o.fails)
    assert g.solutions == o.solutions and len(g.solutions) >= 1
    assert g.nodes > 50
