"""The GPU's work counters against the oracle's, call by call.

The roofline figures of the benchmark are built from the library's own
counters (support rows OR-ed per call, active granules at entry, granule x
row loads, values checked by filterDomains).  Here each per-call difference
of those counters must equal what the oracle counts for the same call from
the paper's definitions: the rows Alg. 2's branch rule selects over s_val
(sum of |Delta_i| or |dom(x_i)|), and the 64-word groups of currTable that
hold a valid tuple at entry.  The oracle's counters are pinned by hand counts
on Table 1 (tests/test_oracle_fast.py)."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_18413_amd import ct
from paper_2507_18413_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def oracle_script(spec, n_calls, family):
    """The plain-call script drawn from the fast oracle's own answers, with
    its per-call counters."""
    lay = spec.layout()
    o = O.OracleTable(spec.tuples, spec.lo, spec.dsizes, fast=True)
    counts = []

    class Sut:
        def domains(self):
            return o.domains()

        def push(self):
            o.push()

        def pop(self):
            o.pop()

        def propagate(self, d):
            st, dom = o.propagate(d)
            counts.append((st, o.last_stats()))
            return st, dom

    script = W.run_plain_script(Sut(), lay, n_calls, W.DEFAULT_SEED, family, W.pick_fraction_removal)
    return script, counts


@pytest.mark.parametrize("schedule", [ct.SCHED_AUTO, ct.SCHED_SOLO, ct.SCHED_SPLIT])
def test_counters_equal_oracle_counts_on_the_large_table_script(schedule):
    spec = W.large_table(W.DEFAULT_SEED)
    say("counters: large-table script (1,000 calls), schedule", schedule)
    script, counts = oracle_script(spec, 1000, 2)
    g = ct.Table(spec.tuples, spec.lo, spec.dsizes, schedule=schedule)
    prev = g.stats()
    k = 0
    for kind, payload in script:
        if kind == "push":
            assert g.push() == ct.OK
        elif kind == "pop":
            assert g.pop() == ct.OK
        else:
            st, _, now = g.propagate(payload, want_stats=True)
            ost, oc = counts[k]
            assert st == ost, k
            d = {key: now[key] - prev[key] for key in now}
            assert d["jobs"] == 1, (k, d)
            assert d["rows_or"] == oc["rows_selected"], (k, d, oc)
            assert d["granules_in"] == oc["nonzero_granules_in"], (k, d, oc)
            # every active granule reads every selected row (a call that
            # changes no domain reads nothing)
            want_gr = d["granules_in"] * d["rows_or"] if oc["sval"] else 0
            assert d["granule_rows"] == want_gr, (k, d, oc)
            if st == ct.OK and oc["sval"]:
                # every present value of a variable with two or more values
                # is checked once (s_sup of Alg. 1)
                assert d["residue_checks"] == oc["residue_checks"], (k, d, oc)
            prev = now
            k += 1
    assert k == 1000
    g.close()


@pytest.mark.parametrize("schedule", [ct.SCHED_AUTO, ct.SCHED_RESIDENT])
def test_counters_on_the_wide_scope_table(schedule):
    spec = W.wide_table(W.DEFAULT_SEED)
    say("counters: wide-scope script (200 calls), schedule", schedule)
    script, counts = oracle_script(spec, 200, 6)
    g = ct.Table(spec.tuples, spec.lo, spec.dsizes, schedule=schedule)
    prev = g.stats()
    k = 0
    for kind, payload in script:
        if kind == "push":
            assert g.push() == ct.OK
        elif kind == "pop":
            assert g.pop() == ct.OK
        else:
            st, _, now = g.propagate(payload, want_stats=True)
            ost, oc = counts[k]
            assert st == ost, k
            d = {key: now[key] - prev[key] for key in now}
            assert d["rows_or"] == oc["rows_selected"], (k, d, oc)
            assert d["granules_in"] == oc["nonzero_granules_in"], (k, d, oc)
            if st == ct.OK and oc["sval"]:
                assert d["residue_checks"] == oc["residue_checks"], (k, d, oc)
            prev = now
            k += 1
    g.close()
