"""A small depth-first search driven through the library.

The paper measures CT inside a constraint solver (Sec. 5: search with the
table propagator next to the solver's other propagators).  This driver does
the same on a generated model: pool variables with bitmap domains, table
constraints propagated to their GAC closure by a table propagator object (the
GPU one wraps ``ct.Model``), and one linear inequality sum_i w_i x_i <= cap
propagated on the host by bounds reasoning.  Branching: the variable with the
smallest domain of more than one value (lowest index first), its values in
increasing order; each branch pushes a level, fixes the variable and
propagates until neither the tables nor the inequality change anything.

A table propagator exposes ``fixpoint(pool) -> (failed, pool_out)``, ``push()``
and ``pop()``; ``GpuTables`` is the library's.  Two propagators that compute
the same closure give the same search tree.
"""
from __future__ import annotations

import time

import numpy as np

from . import ct
from .workloads import DomLayout, distinct_uniform_tuples, rng_for


class GpuTables:
    """The tables of a ``ct.Model``, the pool in device memory."""

    def __init__(self, model: "ct.Model", n_words: int):
        import torch
        self.torch = torch
        self.m = model
        self.din = torch.zeros(n_words, dtype=torch.int64, device="cuda")
        self.dout = torch.zeros_like(self.din)
        self.props = 0

    def fixpoint(self, pool: np.ndarray):
        self.din.copy_(self.torch.from_numpy(pool.view(np.int64)))
        st, props, _ = self.m.fixpoint(self.din, self.dout)
        self.props += props
        if st != ct.OK:
            return True, pool
        return False, self.dout.cpu().numpy().view(np.uint64).copy()

    def push(self):
        self.m.push()

    def pop(self):
        self.m.pop()


class LinearLE:
    """sum_i w_i * x_i <= cap over pool variables (w_i > 0, values lo_i + k),
    bounds reasoning: with S = sum of the weighted minima, a value v of x_i
    stays only if S - w_i * min_i + w_i * v <= cap."""

    def __init__(self, layout: DomLayout, vars_, weights, cap: int):
        self.lay = layout
        self.vars = [int(v) for v in vars_]
        self.w = [int(x) for x in weights]
        self.cap = int(cap)

    def propagate(self, pool: np.ndarray):
        lay = self.lay
        mins = []
        for v in self.vars:
            vals = lay.values(pool, v)
            if vals.size == 0:
                return True, pool
            mins.append(int(vals[0]))
        s = sum(w * m for w, m in zip(self.w, mins))
        if s > self.cap:
            return True, pool
        out = pool.copy()
        for v, w, m in zip(self.vars, self.w, mins):
            top = m + (self.cap - s) // w  # largest value that still fits
            for a in lay.values(pool, v):
                if int(a) > top:
                    lay.clear(out, v, int(a))
        return False, out


class LinearEQ:
    """sum_i w_i * x_i = c over pool variables (w_i > 0, lo_i = 0), bounds
    reasoning repeated until the bounds settle: with Smin / Smax the sums of
    the weighted minima / maxima, x_i <= min_i + (c - Smin) // w_i and
    x_i >= max_i - (Smax - c) // w_i; fails when c lies outside
    [Smin, Smax] or a domain empties."""

    def __init__(self, layout: DomLayout, vars_, weights, c: int):
        self.lay = layout
        self.vars = [int(v) for v in vars_]
        self.w = [int(x) for x in weights]
        self.c = int(c)

    def propagate(self, pool: np.ndarray):
        lay = self.lay
        vals = [lay.values(pool, v) for v in self.vars]
        if any(v.size == 0 for v in vals):
            return True, pool
        lo = [int(v[0]) for v in vals]
        hi = [int(v[-1]) for v in vals]
        smin = sum(w * a for w, a in zip(self.w, lo))
        smax = sum(w * b for w, b in zip(self.w, hi))
        changed = False
        while True:
            if self.c < smin or self.c > smax:
                return True, pool
            moved = False
            for k, w in enumerate(self.w):
                nhi = min(hi[k], lo[k] + (self.c - smin) // w)
                nlo = max(lo[k], hi[k] - (smax - self.c) // w)
                if nhi != hi[k] or nlo != lo[k]:
                    v = vals[k]
                    v = v[(v >= nlo) & (v <= nhi)]
                    if v.size == 0:
                        return True, pool
                    vals[k] = v
                    a, b = int(v[0]), int(v[-1])
                    smin += w * (a - lo[k])
                    smax += w * (b - hi[k])
                    lo[k], hi[k] = a, b
                    moved = changed = True
                    if self.c < smin or self.c > smax:
                        return True, pool
            if not moved:
                break
        if not changed:
            return False, pool
        out = pool.copy()
        for v, k in zip(self.vars, range(len(self.vars))):
            for a in lay.values(pool, v):
                if int(a) < lo[k] or int(a) > hi[k]:
                    lay.clear(out, v, int(a))
        return False, out


class OneTable:
    """One table constraint over all the pool variables, in column order, as
    a table propagator: a single propagate call reaches its GAC (a table is
    idempotent after its own call).  ``t`` is a ``ct.Table`` or any object
    with the same propagate / push / pop (the oracle's table in the tests)."""

    def __init__(self, t):
        self.t = t
        self.props = 0
        self.seconds = 0.0  # host time spent inside the table's propagate calls

    def fixpoint(self, pool: np.ndarray):
        t0 = time.perf_counter()
        st, out = self.t.propagate(pool)[:2]
        self.seconds += time.perf_counter() - t0
        self.props += 1
        if st != 0:
            return True, pool
        return False, np.asarray(out, dtype=np.uint64).copy()

    def push(self):
        self.t.push()

    def pop(self):
        self.t.pop()


class Search:
    """Depth-first search.  var_order: "min_dom" (smallest domain of more
    than one value, lowest index first) or "input" (the first variable with
    more than one value, MiniZinc's input_order); val_order: "min"
    (increasing values) or "max" (decreasing, indomain_max)."""

    def __init__(self, layout: DomLayout, tables, linear, var_order: str = "min_dom",
                 val_order: str = "min"):
        self.lay = layout
        self.tables = tables
        self.lin = linear
        self.var_order = var_order
        self.val_order = val_order
        self.nodes = 0
        self.fails = 0
        self.solutions = []

    def _propagate(self, pool):
        while True:
            failed, pool = self.tables.fixpoint(pool)
            if failed:
                return True, pool
            failed, nxt = self.lin.propagate(pool)
            if failed:
                return True, pool
            if (nxt == pool).all():
                return False, pool
            pool = nxt

    def _branch_var(self, pool):
        best, size = -1, 0
        for i in range(self.lay.n):
            k = self.lay.values(pool, i).size
            if k > 1 and self.var_order == "input":
                return i
            if k > 1 and (best < 0 or k < size):
                best, size = i, k
        return best

    def _values(self, pool, var):
        v = list(self.lay.values(pool, var))
        return v[::-1] if self.val_order == "max" else v

    def run(self, pool: np.ndarray, max_nodes: int, max_solutions: int):
        """Depth-first search from ``pool``; stops after ``max_nodes`` nodes or
        ``max_solutions`` solutions.  Returns the number of nodes visited."""
        self.tables.push()
        failed, pool = self._propagate(pool)
        self.nodes += 1
        if failed:
            self.fails += 1
            self.tables.pop()
            return self.nodes
        # frames: (pool at the frame, variable, values left to try)
        stack = []
        var = self._branch_var(pool)
        if var < 0:
            self.solutions.append(self.lay.to_sets(pool))
            self.tables.pop()
            return self.nodes
        stack.append((pool, var, self._values(pool, var)))
        while stack and self.nodes < max_nodes and len(self.solutions) < max_solutions:
            base, var, left = stack[-1]
            if not left:
                stack.pop()
                self.tables.pop()  # the level pushed when this frame's node was entered
                continue
            a = int(left.pop(0))
            child = base.copy()
            for b in self.lay.values(base, var):
                if int(b) != a:
                    self.lay.clear(child, var, int(b))
            self.tables.push()
            self.nodes += 1
            failed, child = self._propagate(child)
            if failed:
                self.fails += 1
                self.tables.pop()
                continue
            nv = self._branch_var(child)
            if nv < 0:
                self.solutions.append(self.lay.to_sets(child))
                self.tables.pop()
                continue
            stack.append((child, nv, self._values(child, nv)))
        while stack:
            stack.pop()
            self.tables.pop()
        return self.nodes


def lin_model(seed: int, n_vars: int = 24, d: int = 10, n_tables: int = 6, arity: int = 6,
              density=(0.05, 0.3)):
    """A knapsack-like model in the spirit of the paper's linear instances:
    ``n_vars`` variables over {0..d-1}; ``n_tables`` tables of the given arity
    over random distinct variables, each allowing a random fraction (in
    ``density``) of the value combinations; one inequality
    sum_i w_i x_i <= cap with w_i ~ U{1..9} and cap = a third of the largest
    sum.  Returns (pool dsizes, [(tuples, scope)], weights, cap)."""
    rng = rng_for(seed, 8, 0)
    dsz = np.full(n_vars, d, np.int32)
    tables = []
    for _ in range(n_tables):
        scope = rng.choice(n_vars, size=arity, replace=False).astype(np.int32)
        frac = float(rng.uniform(*density))
        t = max(1, int(frac * d ** arity))
        tables.append((distinct_uniform_tuples(rng, dsz[scope], t), scope))
    w = rng.integers(1, 10, size=n_vars)
    cap = int(w.sum() * (d - 1) // 3)
    return dsz, tables, w, cap


def build_gpu(dsz, tables):
    """ct.Model over the pool with one ct.Table per table; returns (model, tables)."""
    M = ct.Model(np.zeros(dsz.shape[0], np.int32), dsz)
    tabs = []
    for tup, scope in tables:
        T = ct.Table(tup, np.zeros(len(scope), np.int32), dsz[scope])
        M.add(T, scope)
        tabs.append(T)
    return M, tabs


def solve_gpu(seed: int, max_nodes: int, max_solutions: int, **kw):
    """The generated model searched with the GPU tables; returns a summary."""
    dsz, tables, w, cap = lin_model(seed, **kw)
    lay = DomLayout(dsz, np.zeros_like(dsz))
    M, tabs = build_gpu(dsz, tables)
    prop = GpuTables(M, lay.D)
    s = Search(lay, prop, LinearLE(lay, range(lay.n), w, cap))
    t0 = time.perf_counter()
    s.run(lay.full(), max_nodes, max_solutions)
    el = time.perf_counter() - t0
    return {"nodes": s.nodes, "fails": s.fails, "solutions": len(s.solutions), "seconds": el,
            "table_propagations": prop.props, "search": s, "keep": (M, tabs)}
