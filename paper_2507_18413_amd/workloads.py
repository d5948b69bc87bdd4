"""Seeded synthetic inputs for Compact-Table propagation.

This module is shared by the CPU oracle tests and the HIP path: it draws
tables (tuples + initial domains) and chooses which domain values a simulated
search removes.  It holds none of the propagation arithmetic (no support
bitsets, no currTable, no filtering): the only bit operations here read and
clear single domain bits chosen at random.

Domain bitmap layout (the boundary's layout, used by both sides): variable i
with initial domain ``[lo_i, lo_i + d_i)`` owns ``ceil(d_i / 64)`` consecutive
uint64 words starting at ``dom_off[i]``; value ``v`` is bit ``(v - lo_i) % 64``
of word ``dom_off[i] + (v - lo_i) // 64``, LSB first; bits at or beyond ``d_i``
are zero.

The workloads stand in for the paper's MiniZinc instance suites (LIN_B,
LIN_EB, orienteering, the Gecode comparison set, Sec. 5.1), which are not
available: every table here is drawn from a seeded generator with the stated
shape.  Seeds follow ``SeedSequence([base, family, stream])``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DEFAULT_SEED = 20250724


def rng_for(base: int, family: int, stream: int = 0) -> np.random.Generator:
    """Independent PCG64 stream for (base seed, workload family number, stream id)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([base, family, stream])))


# ---------------------------------------------------------------------------
# domain layout helpers (bookkeeping only)
# ---------------------------------------------------------------------------
@dataclass
class DomLayout:
    dsizes: np.ndarray                 # int64 [n]
    lo: np.ndarray                     # int64 [n]
    words: np.ndarray = field(init=False)
    off: np.ndarray = field(init=False)
    D: int = field(init=False)

    def __post_init__(self):
        self.dsizes = np.asarray(self.dsizes, dtype=np.int64)
        self.lo = np.asarray(self.lo, dtype=np.int64)
        self.words = (self.dsizes + 63) // 64
        self.off = np.concatenate([[0], np.cumsum(self.words)[:-1]]).astype(np.int64)
        self.D = int(self.words.sum())

    @property
    def n(self) -> int:
        return int(self.dsizes.shape[0])

    def full(self) -> np.ndarray:
        """Bitmap with every initial value present."""
        out = np.zeros(self.D, dtype=np.uint64)
        for i in range(self.n):
            d = int(self.dsizes[i])
            for k in range(int(self.words[i])):
                nb = min(64, d - 64 * k)
                out[self.off[i] + k] = np.uint64((1 << nb) - 1) if nb < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
        return out

    def values(self, dom: np.ndarray, i: int) -> np.ndarray:
        """Offsets (v - lo_i) present in variable i, ascending."""
        seg = dom[self.off[i]: self.off[i] + self.words[i]]
        bits = np.unpackbits(seg.view(np.uint8), bitorder="little")
        return np.nonzero(bits[: int(self.dsizes[i])])[0]

    def count(self, dom: np.ndarray, i: int) -> int:
        return int(self.values(dom, i).shape[0])

    def from_sets(self, sets) -> np.ndarray:
        """Bitmap from per-variable iterables of value offsets."""
        out = np.zeros(self.D, dtype=np.uint64)
        for i, s in enumerate(sets):
            for a in s:
                a = int(a)
                assert 0 <= a < self.dsizes[i]
                out[self.off[i] + a // 64] |= np.uint64(1 << (a % 64))
        return out

    def to_sets(self, dom: np.ndarray):
        return [set(int(a) for a in self.values(dom, i)) for i in range(self.n)]

    def clear(self, dom: np.ndarray, i: int, a: int) -> None:
        dom[self.off[i] + a // 64] &= ~np.uint64(1 << (a % 64))


# ---------------------------------------------------------------------------
# tuple generators
# ---------------------------------------------------------------------------
def _codes_to_tuples(codes: np.ndarray, dsizes: np.ndarray) -> np.ndarray:
    n = dsizes.shape[0]
    out = np.empty((codes.shape[0], n), dtype=np.int32)
    c = codes.copy()
    for i in range(n - 1, -1, -1):
        out[:, i] = (c % dsizes[i]).astype(np.int32)
        c //= dsizes[i]
    return out


def _first_occurrence_distinct(codes: np.ndarray, t: int) -> np.ndarray:
    """The first ``t`` distinct codes in draw order (deterministic, unsorted)."""
    _, first = np.unique(codes, return_index=True)
    first.sort()
    return codes[first[:t]]


_CODE_LIMIT = 1 << 62


def _row_hash(tup: np.ndarray) -> np.ndarray:
    """64-bit hash of each row (equal rows, equal hashes)."""
    h = np.zeros(tup.shape[0], dtype=np.uint64)
    with np.errstate(over="ignore"):
        for i in range(tup.shape[1]):
            h = (h ^ tup[:, i].astype(np.uint64)) * np.uint64(0x9E3779B97F4A7C15)
            h ^= h >> np.uint64(29)
    return h


def _distinct_rows(draw_rows, t: int, n: int) -> np.ndarray:
    """First ``t`` distinct rows of the stream ``draw_rows(m)`` (int64 [m, n]),
    in draw order.  Rows whose hashes coincide count as one, so the kept rows
    are always distinct (a collision only costs an extra draw)."""
    rows = np.zeros((0, n), dtype=np.int64)
    want, rate = t, 1.0
    while True:
        m = int(want / max(rate, 0.02) * 1.15) + 64
        new = draw_rows(m)
        before = rows.shape[0]
        rows = np.concatenate([rows, new])
        _, first = np.unique(_row_hash(rows), return_index=True)
        first.sort()
        if first.shape[0] >= t:
            return rows[first[:t]].astype(np.int32)
        rows = rows[first]
        rate = max((rows.shape[0] - before) / m, 1e-3)
        want = t - rows.shape[0]


def distinct_uniform_tuples(rng: np.random.Generator, dsizes, t: int) -> np.ndarray:
    """``t`` distinct tuples, each column uniform over ``[0, d_i)``, in draw order."""
    dsizes = np.asarray(dsizes, dtype=np.int64)
    space = int(np.prod([int(x) for x in dsizes], dtype=object))
    if t > space:
        raise ValueError("more distinct tuples requested than the domain product holds")
    if t == 0:
        return np.zeros((0, dsizes.shape[0]), dtype=np.int32)
    if space >= _CODE_LIMIT:
        n = dsizes.shape[0]
        return _distinct_rows(lambda m: np.stack([rng.integers(0, d, size=m) for d in dsizes], 1), t, n)
    if 2 * t >= space:
        codes = rng.permutation(space)[:t].astype(np.int64)
        return _codes_to_tuples(codes, dsizes)
    draw = int(t * 1.2) + 64
    got = np.zeros(0, dtype=np.int64)
    while True:
        new = rng.integers(0, space, size=draw, dtype=np.int64)
        got = np.concatenate([got, new])
        dist = _first_occurrence_distinct(got, t)
        if dist.shape[0] >= t:
            return _codes_to_tuples(dist, dsizes)
        draw = max(64, int((t - dist.shape[0]) * 1.5))


def zipf_probs(d: int, s: float) -> np.ndarray:
    """Truncated Zipf over ranks 1..d: p(r) proportional to r^-s; rank r is value r-1."""
    w = np.arange(1, d + 1, dtype=np.float64) ** (-s)
    return w / w.sum()


def distinct_zipf_tuples(rng: np.random.Generator, n: int, d: int, s: float, t: int) -> np.ndarray:
    """``t`` distinct tuples whose columns are i.i.d. truncated Zipf(s) over ``[0, d)``.

    Distinctness by rejection: draws continue until ``t`` distinct codes exist;
    draw order is kept.
    """
    space = d ** n
    if t > space:
        raise ValueError("more distinct tuples requested than the domain product holds")
    p = zipf_probs(d, s)
    cdf = np.cumsum(p)
    cdf[-1] = 1.0
    dsizes = np.full(n, d, dtype=np.int64)
    got = np.zeros(0, dtype=np.int64)
    draw = int(t * 1.9) + 64
    while True:
        vals = np.searchsorted(cdf, rng.random((draw, n)), side="right").astype(np.int64)
        vals = np.minimum(vals, d - 1)
        codes = np.zeros(draw, dtype=np.int64)
        for i in range(n):
            codes = codes * d + vals[:, i]
        got = np.concatenate([got, codes])
        dist = _first_occurrence_distinct(got, t)
        if dist.shape[0] >= t:
            return _codes_to_tuples(dist, dsizes)
        draw = max(1024, int((t - dist.shape[0]) * 3))


@dataclass
class TableSpec:
    tuples: np.ndarray            # int32 [t, n], values already offset by lo (absolute)
    lo: np.ndarray                # int32 [n]
    dsizes: np.ndarray            # int32 [n]

    @property
    def n(self):
        return int(self.dsizes.shape[0])

    @property
    def t(self):
        return int(self.tuples.shape[0])

    def layout(self) -> DomLayout:
        return DomLayout(self.dsizes, self.lo)


def tiny_table(seed: int = DEFAULT_SEED) -> TableSpec:
    """Arity 3, every domain {0..7}, 200 distinct tuples out of the 512 codes."""
    rng = rng_for(seed, 1, 0)
    tup = distinct_uniform_tuples(rng, [8, 8, 8], 200)
    return TableSpec(tup, np.zeros(3, np.int32), np.full(3, 8, np.int32))


def large_table(seed: int = DEFAULT_SEED, t: int = 200_000, d: int = 50, n: int = 5) -> TableSpec:
    """Arity 5, domain size 50, 200,000 distinct uniform tuples (3,125 words per row)."""
    rng = rng_for(seed, 2, 0)
    tup = distinct_uniform_tuples(rng, [d] * n, t)
    return TableSpec(tup, np.zeros(n, np.int32), np.full(n, d, np.int32))


def wide_table(seed: int = DEFAULT_SEED, n: int = 100, dom=(64, 160), t: int = 10_000) -> TableSpec:
    """A wide-scope table in the shape of the paper's linear-constraint
    instances (Sec. 5.1, Table 2: tens to hundreds of variables, large
    domains, a few thousand tuples): arity n, domain sizes uniform in
    [dom[0], dom[1]], t distinct uniform tuples.  Support rows are many and
    short (about 11,000 rows of 157 words at the defaults), so a call is
    dominated by filterDomains."""
    rng = rng_for(seed, 6, 0)
    ds = rng.integers(dom[0], dom[1] + 1, size=n).astype(np.int32)
    tup = distinct_uniform_tuples(rng, ds, t)
    return TableSpec(tup, np.zeros(n, np.int32), ds)


def paper_shape_table(seed: int = DEFAULT_SEED, n: int = 150, dom=(2, 2000), t: int = 15_000) -> TableSpec:
    """A table of the size of the paper's Gecode comparison set (Sec. 5.3:
    100-150 variables, domains up to 2,000 values, 10,000-15,000 tuples):
    arity n, domain sizes uniform in [dom[0], dom[1]], t distinct uniform
    tuples.  About 150,000 support rows of 235 words and 2,400 domain words
    at the defaults: a call is dominated by filterDomains."""
    rng = rng_for(seed, 10, 0)
    ds = rng.integers(dom[0], dom[1] + 1, size=n).astype(np.int32)
    tup = distinct_uniform_tuples(rng, ds, t)
    return TableSpec(tup, np.zeros(n, np.int32), ds)


def zipf_table(seed: int = DEFAULT_SEED, t: int = 1_000_000, d: int = 20, n: int = 6,
                  s: float = 1.1) -> TableSpec:
    """Arity 6, domain size 20, distinct tuples with Zipf(1.1) columns."""
    rng = rng_for(seed, 4, 0)
    tup = distinct_zipf_tuples(rng, n, d, s, t)
    return TableSpec(tup, np.zeros(n, np.int32), np.full(n, d, np.int32))


def node_states(layout: DomLayout, root_dom: np.ndarray, n_nodes: int,
                  seed: int = DEFAULT_SEED, max_frac: float = 0.6) -> np.ndarray:
    """Search-node domain states: per node and variable draw f ~ U[0, max_frac]
    and remove floor(f * |root domain|) values chosen uniformly from the root
    domain.  Returns uint64 [n_nodes, D]."""
    rng = rng_for(seed, 4, 1)
    out = np.empty((n_nodes, layout.D), dtype=np.uint64)
    present = [layout.values(root_dom, i) for i in range(layout.n)]
    for k in range(n_nodes):
        dom = root_dom.copy()
        for i in range(layout.n):
            vals = present[i]
            f = rng.random() * max_frac
            m = int(math.floor(f * vals.shape[0]))
            if m:
                for a in rng.choice(vals, size=m, replace=False):
                    layout.clear(dom, i, int(a))
        out[k] = dom
    return out


@dataclass
class ModelSpec:
    """Many tables over a shared pool of variables (lo = 0 everywhere)."""
    pool_dsizes: np.ndarray       # int32 [n_pool]
    tables: list                  # list[TableSpec]
    scopes: list                  # list[np.ndarray int32], pool var ids per table column

    def pool_layout(self) -> DomLayout:
        return DomLayout(self.pool_dsizes, np.zeros_like(self.pool_dsizes))


def multi_table_model(seed: int = DEFAULT_SEED, n_pool: int = 5000, n_tables: int = 2000,
                  arity=(2, 8), dom=(4, 64), tuples=(100, 500_000), plant: bool = True) -> ModelSpec:
    """Pool of variables with d ~ U{dom}, tables of arity ~ U{arity} over distinct
    pool variables, tuple counts log-uniform in ``tuples`` capped at half the
    domain product, distinct uniform tuples.  With ``plant`` a hidden
    assignment of every pool variable is drawn and each table holds its
    projection (replacing the first tuple when absent), so the model has a
    solution and the root fixpoint never fails."""
    rng = rng_for(seed, 3, 0)
    pool = rng.integers(dom[0], dom[1] + 1, size=n_pool).astype(np.int32)
    hidden = (rng.random(n_pool) * pool).astype(np.int64)
    tables, scopes = [], []
    for c in range(n_tables):
        n = int(rng.integers(arity[0], arity[1] + 1))
        scope = rng.choice(n_pool, size=n, replace=False).astype(np.int32)
        ds = pool[scope].astype(np.int64)
        t = int(round(math.exp(rng.uniform(math.log(tuples[0]), math.log(tuples[1])))))
        space = int(np.prod([int(x) for x in ds], dtype=object))
        t = max(1, min(t, space // 2))
        trng = rng_for(seed, 3, 1 + c)
        tup = distinct_uniform_tuples(trng, ds, t)
        if plant:
            sol = hidden[scope].astype(np.int32)
            if not (tup == sol).all(axis=1).any():
                tup[0] = sol
        tables.append(TableSpec(tup, np.zeros(n, np.int32), ds.astype(np.int32)))
        scopes.append(scope)
    return ModelSpec(pool, tables, scopes)


def _serving_one(args):
    seed, c, ds, t, s = args
    trng = rng_for(seed, 5, 1 + c)
    if c % 2 == 0:
        tup = distinct_uniform_tuples(trng, ds, t)
    else:
        tup = _distinct_zipf_mixed(trng, ds, s, t)
    return TableSpec(tup, np.zeros(ds.shape[0], np.int32), ds.astype(np.int32))


def serving_tables(seed: int = DEFAULT_SEED, n_tables: int = 300, arity=(3, 10), dom=(8, 128),
                   tuples=(1_000, 2_000_000), s: float = 1.1, workers: int = 0):
    """Serving mix: even-index tables uniform, odd-index Zipf(s) columns.

    Each table's tuples come from its own stream, so the result does not
    depend on ``workers`` (> 1: a pool of threads; numpy's sorting and
    drawing release the interpreter lock, and no process is started, so the
    call is safe in a process that already uses the GPU)."""
    rng = rng_for(seed, 5, 0)
    jobs = []
    for c in range(n_tables):
        n = int(rng.integers(arity[0], arity[1] + 1))
        ds = rng.integers(dom[0], dom[1] + 1, size=n).astype(np.int64)
        t = int(round(math.exp(rng.uniform(math.log(tuples[0]), math.log(tuples[1])))))
        space = int(np.prod([int(x) for x in ds], dtype=object))
        t = max(1, min(t, space // 2))
        jobs.append((seed, c, ds, t, s))
    if workers and workers > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(workers) as ex:
            return list(ex.map(_serving_one, jobs))
    return [_serving_one(j) for j in jobs]


def _distinct_zipf_mixed(rng, dsizes, s, t):
    n = dsizes.shape[0]
    cdfs = []
    for d in dsizes:
        c = np.cumsum(zipf_probs(int(d), s))
        c[-1] = 1.0
        cdfs.append(c)
    space = int(np.prod([int(x) for x in dsizes], dtype=object))
    if t > space:
        raise ValueError("more distinct tuples requested than the domain product holds")
    if space >= _CODE_LIMIT:
        def draw(m):
            u = rng.random((m, n))
            return np.stack([np.minimum(np.searchsorted(cdfs[i], u[:, i], side="right"), dsizes[i] - 1)
                             for i in range(n)], 1).astype(np.int64)
        return _distinct_rows(draw, t, n)
    got = np.zeros(0, dtype=np.int64)
    draw, rate = int(t * 1.9) + 64, 1.0
    while True:
        codes = np.zeros(draw, dtype=np.int64)
        u = rng.random((draw, n))
        for i in range(n):
            v = np.minimum(np.searchsorted(cdfs[i], u[:, i], side="right"), dsizes[i] - 1)
            codes = codes * dsizes[i] + v
        before = got.shape[0]
        got = _first_occurrence_distinct(np.concatenate([got, codes]), 1 << 62)
        if got.shape[0] >= t:
            return _codes_to_tuples(got[:t], dsizes)
        # keep only distinct codes; size the next round from the distinct rate
        rate = max((got.shape[0] - before) / draw, 1e-3)
        draw = int((t - got.shape[0]) / rate * 1.15) + 1024


def lin_instance(seed: int = DEFAULT_SEED, n: int = 100, dom=(2, 160), t: int = 10_000,
                 eq_frac: float = 0.5, weights=(1, 20)):
    """A bounded-knapsack instance in the shape of the paper's first test set
    (Sec. 5.1: one table constraint over all the item-count variables plus one
    linear equation over some of them; Table 2 gives 80-200 variables and
    5,000-15,000 tuples).  Variable i counts the copies of item i, domain
    {0..d_i - 1} with d_i ~ U{dom}; the table lists t distinct knapsack
    configurations drawn uniformly; the equation sum_{i in E} w_i x_i = C
    with w_i ~ U{weights} over a random subset E of ``eq_frac`` of the
    variables, and C the weighted sum of one configuration of the table (so
    the instance has a solution).  Returns (TableSpec, E, w, C)."""
    rng = rng_for(seed, 9, 0)
    ds = rng.integers(dom[0], dom[1] + 1, size=n).astype(np.int64)
    tup = distinct_uniform_tuples(rng, ds, t)
    k = max(1, int(round(eq_frac * n)))
    E = np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
    w = rng.integers(weights[0], weights[1] + 1, size=k).astype(np.int64)
    planted = tup[int(rng.integers(0, t))]
    C = int((w * planted[E].astype(np.int64)).sum())
    return TableSpec(tup, np.zeros(n, np.int32), ds.astype(np.int32)), E, w, C


# ---------------------------------------------------------------------------
# search simulation: which values a step removes
# ---------------------------------------------------------------------------
def pick_small_removal(rng, layout: DomLayout, dom: np.ndarray) -> np.ndarray:
    """Remove 1 or 2 values: each time a variable is chosen uniformly among those
    with a non-empty domain and a present value uniformly within it."""
    out = dom.copy()
    k = int(rng.integers(1, 3))
    for _ in range(k):
        cand = [i for i in range(layout.n) if layout.count(out, i) > 0]
        if not cand:
            break
        i = cand[int(rng.integers(0, len(cand)))]
        vals = layout.values(out, i)
        layout.clear(out, i, int(vals[int(rng.integers(0, vals.shape[0]))]))
    return out


def pick_fraction_removal(rng, layout: DomLayout, dom: np.ndarray, frac: float = 0.05,
                          nvars=(1, 3), var_ids=None) -> np.ndarray:
    """Remove ceil(frac * |dom_i|) present values from each of U{nvars} distinct
    variables chosen uniformly (among ``var_ids`` if given)."""
    out = dom.copy()
    ids = np.arange(layout.n) if var_ids is None else np.asarray(var_ids)
    k = int(rng.integers(nvars[0], nvars[1] + 1))
    k = min(k, ids.shape[0])
    for i in rng.choice(ids, size=k, replace=False):
        vals = layout.values(out, int(i))
        if vals.shape[0] == 0:
            continue
        m = int(math.ceil(frac * vals.shape[0]))
        for a in rng.choice(vals, size=m, replace=False):
            layout.clear(out, int(i), int(a))
    return out


class Backtracker:
    """Push/pop schedule of the plain-call workloads: a push before every
    propagate, after every ``every``-th call a pop of U{1..depth} levels, and a
    pop of one level after a failed call."""

    def __init__(self, rng, every: int = 10):
        self.rng = rng
        self.every = every
        self.calls = 0

    def pops_after(self, status_failed: bool, depth: int) -> int:
        self.calls += 1
        if status_failed:
            return 1 if depth > 0 else 0
        if self.calls % self.every == 0 and depth > 0:
            return int(self.rng.integers(1, depth + 1))
        return 0


def run_plain_script(sut, layout: DomLayout, n_calls: int, seed: int, family: int,
                     picker, on_step=None):
    """Drive one table through a simulated search.

    ``sut`` exposes ``propagate(dom_in) -> (status, dom_out)``, ``push()``,
    ``pop()`` and ``domains() -> bitmap``; status 0 = OK, 1 = FAIL.  Choices
    are drawn from the domains the system under test returns, so two systems
    that agree on every call see the same script.  ``on_step(kind, info)`` is
    called after each operation (kind in {"prop", "pop"}).  Returns the list
    of operations as (kind, payload) for replay.
    """
    rng = rng_for(seed, family, 7)
    bt = Backtracker(rng)
    depth = 0
    script = []
    for _ in range(n_calls):
        dom = sut.domains()
        dom_in = picker(rng, layout, dom)
        sut.push()
        depth += 1
        script.append(("push", None))
        status, dom_out = sut.propagate(dom_in)
        script.append(("prop", dom_in))
        if on_step:
            on_step("prop", (dom_in, status, dom_out))
        k = bt.pops_after(status == 1, depth)
        for _ in range(k):
            sut.pop()
            depth -= 1
            script.append(("pop", None))
            if on_step:
                on_step("pop", None)
    return script


class SimSearch:
    """A simulated depth-first search over one table, as a stream of requests.

    Request k: pops (one after a failure; U{1..depth} every ``every``-th
    request), a push (except the first request), then the values to remove:
    ceil(``frac`` x |dom|) present values of U{nvars} distinct variables.  The
    search keeps the domains it was given back, so the choices follow the
    results; ``log`` records (n_pop, push, remove) for replay.
    """

    def __init__(self, layout: DomLayout, root: np.ndarray, rng, length: int, every: int = 10,
                 frac: float = 0.05, nvars=(1, 4)):
        self.lay, self.rng, self.length = layout, rng, length
        self.every, self.frac, self.nvars = every, frac, nvars
        self.dom = root.copy()
        self.stack = []
        self.failed = False
        self.k = 0
        self.log = []

    def done(self) -> bool:
        return self.k >= self.length

    def next_request(self):
        """(n_pop, push, remove, finish) of the next request."""
        n_pop = 0
        if self.k > 0:
            if self.failed:
                n_pop = 1
            elif self.k % self.every == 0 and self.stack:
                n_pop = int(self.rng.integers(1, len(self.stack) + 1))
        for _ in range(n_pop):
            self.dom = self.stack.pop()
        self.failed = False
        push = 1 if self.k > 0 else 0
        if push:
            self.stack.append(self.dom.copy())
        new = pick_fraction_removal(self.rng, self.lay, self.dom, self.frac, self.nvars)
        remove = self.dom & ~new
        self.pending = new
        self.k += 1
        finish = self.k >= self.length
        self.log.append((n_pop, push, remove))
        return n_pop, push, remove, finish

    def on_result(self, status: int, dom_out):
        if status == 0:
            self.dom = np.asarray(dom_out, dtype=np.uint64).copy()
        elif status == 1:
            self.failed = True
        else:
            raise RuntimeError(f"unexpected status {status}")


def poisson_arrivals(rng, rate: float, n: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
