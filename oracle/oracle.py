"""ctypes front end of the plain-C oracle (test infrastructure only).

The oracle follows the paper's definitions and Algorithms 1-3 (see the header
of ct_oracle.c).  Only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libct_oracle.so")
# the mutation test points this at a deliberately broken build of the oracle
LIB_PATH = os.environ.get("CT_ORACLE_LIB", LIB_PATH)

OK, FAIL, E_INVALID, E_NOT_SUBSET, E_STATE, E_NOMEM = 0, 1, -1, -2, -3, -4
KIND_POSITIVE, KIND_NEGATIVE = 0, 1
STAR = -(1 << 31)  # a cell of a short table: any value of the column
MODE_AUTO, MODE_RESET, MODE_INCREMENTAL = 0, 1, 2

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.cto_create.argtypes = [P, C.c_int64, C.c_int32, P, P, P, C.POINTER(P)]
        L.cto_create.restype = C.c_int
        L.cto_create_fast.argtypes = [P, C.c_int64, C.c_int32, P, P, P, C.POINTER(P)]
        L.cto_create_fast.restype = C.c_int
        L.cto_create_kind.argtypes = [P, C.c_int64, C.c_int32, P, P, P, C.c_int32, C.POINTER(P)]
        L.cto_create_kind.restype = C.c_int
        L.cto_destroy.argtypes = [P]
        L.cto_layout.argtypes = [P, P, P, P, P]
        L.cto_get_state.argtypes = [P, P, P, P]
        L.cto_support_row.argtypes = [P, C.c_int32, P]
        L.cto_propagate.argtypes = [P, P, P, P, C.c_int32]
        L.cto_push.argtypes = [P]
        L.cto_pop.argtypes = [P]
        L.cto_last_stats.argtypes = [P, P, C.c_int32]
        L.cto_last_stats.restype = C.c_int
        L.cto_fixpoint.argtypes = [C.c_int32, P, P, P, C.c_int32, P, P, C.c_int32, P, P, C.c_int32, P]
        L.cto_fixpoint.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class OracleTable:
    """One table constraint with its reversible propagator state."""

    def __init__(self, tuples, lo, dsizes, init_dom=None, fast=False, kind=KIND_POSITIVE):
        """fast: CT's sparse word list, residues and a word trail (same
        results as the plain mode, which follows Alg. 1-3 densely; positive
        tables only).  kind: KIND_POSITIVE (cells may hold STAR: a short
        table) or KIND_NEGATIVE (the tuples are the forbidden combinations)."""
        L = lib()
        self.fast = bool(fast)
        self.kind = int(kind)
        if fast and kind != KIND_POSITIVE:
            raise ValueError("the fast mode takes positive tables")
        tuples = np.ascontiguousarray(tuples, dtype=np.int32)
        self.n = int(len(dsizes))
        self.lo = np.ascontiguousarray(lo, dtype=np.int32)
        self.dsizes = np.ascontiguousarray(dsizes, dtype=np.int32)
        t = int(tuples.shape[0]) if tuples.ndim == 2 else 0
        if init_dom is not None:
            init_dom = np.ascontiguousarray(init_dom, dtype=np.uint64)
        h = C.c_void_p()
        if kind != KIND_POSITIVE:
            st = L.cto_create_kind(_p(tuples) if t else None, t, self.n, _p(self.lo), _p(self.dsizes),
                                   _p(init_dom), int(kind), C.byref(h))
        else:
            create = L.cto_create_fast if fast else L.cto_create
            st = create(_p(tuples) if t else None, t, self.n, _p(self.lo), _p(self.dsizes),
                        _p(init_dom), C.byref(h))
        self.create_status = st
        if h.value is None:
            raise ValueError(f"cto_create failed with status {st}")
        self.h = h
        D, W, rows, depth = C.c_int32(), C.c_int64(), C.c_int32(), C.c_int32()
        L.cto_layout(h, C.byref(D), C.byref(W), C.byref(rows), C.byref(depth))
        self.D, self.W, self.rows, self.t = D.value, W.value, rows.value, t

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value is not None:
            lib().cto_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def depth(self):
        d = C.c_int32()
        lib().cto_layout(self.h, None, None, None, C.byref(d))
        return d.value

    def state(self):
        dom = np.zeros(self.D, np.uint64)
        ct = np.zeros(max(self.W, 1), np.uint64)
        f = C.c_int32()
        lib().cto_get_state(self.h, _p(dom), _p(ct), C.byref(f))
        return dom, ct[: self.W], bool(f.value)

    def domains(self):
        return self.state()[0]

    def support_row(self, row):
        out = np.zeros(max(self.W, 1), np.uint64)
        st = lib().cto_support_row(self.h, int(row), _p(out))
        assert st == OK
        return out[: self.W]

    def propagate(self, dom_in, mode=MODE_AUTO, want_ct=False):
        dom_in = np.ascontiguousarray(dom_in, dtype=np.uint64)
        dom_out = np.zeros(self.D, np.uint64)
        ct = np.zeros(max(self.W, 1), np.uint64) if want_ct else None
        st = lib().cto_propagate(self.h, _p(dom_in), _p(dom_out), _p(ct), int(mode))
        if want_ct:
            return st, dom_out, ct[: self.W]
        return st, dom_out

    STAT_NAMES = ("nonzero_words_in", "update_rows", "sval", "ssup", "nonzero_granules_in",
                  "rows_selected", "residue_checks", "residue_misses", "scan_words", "update_words")

    def last_stats(self):
        """Work counters of the last propagate call (see cto_last_stats):
        non-zero currTable words and 64-word granules at entry, rows OR-ed
        (up to Alg. 2's break) and rows selected over all of s_val, |s_val|,
        |s_sup|, support words read by updateTable, and in the fast mode the
        residue checks, misses and words scanned by filterDomains."""
        out = np.zeros(len(self.STAT_NAMES), np.int64)
        n = lib().cto_last_stats(self.h, _p(out), len(self.STAT_NAMES))
        assert n == len(self.STAT_NAMES)
        return {k: int(v) for k, v in zip(self.STAT_NAMES, out)}

    def push(self):
        return lib().cto_push(self.h)

    def pop(self):
        return lib().cto_pop(self.h)


def fixpoint(tables, scopes, pool_layout, pool_in, order=None, seed=None):
    """GAC closure over tables sharing pool variables (FIFO queue of tables).

    order: the initial queue (default: every table in index order); seed: the
    tables to start from instead (a fixpoint whose previous state was a
    fixpoint needs only the tables touching a changed variable).
    Returns (status, pool_out, n_propagations)."""
    L = lib()
    n = len(tables)
    arr = (C.c_void_p * n)(*[t.h.value for t in tables])
    scope_off = np.zeros(n + 1, np.int32)
    for c, s in enumerate(scopes):
        scope_off[c + 1] = scope_off[c] + len(s)
    flat = np.ascontiguousarray(np.concatenate([np.asarray(s, np.int32) for s in scopes])
                                if n else np.zeros(0, np.int32), dtype=np.int32)
    pool_off = np.ascontiguousarray(pool_layout.off, dtype=np.int32)
    pool_in = np.ascontiguousarray(pool_in, dtype=np.uint64)
    pool_out = np.zeros_like(pool_in)
    n_init = -1
    if seed is not None:
        order = np.asarray(seed, dtype=np.int32)
        n_init = int(order.shape[0])
    ordr = None if order is None else np.ascontiguousarray(order, dtype=np.int32)
    props = C.c_int64()
    st = L.cto_fixpoint(n, C.cast(arr, C.c_void_p), _p(scope_off), _p(flat), pool_layout.n,
                        _p(pool_off), _p(pool_in), int(pool_in.shape[0]), _p(pool_out), _p(ordr),
                        n_init, C.byref(props))
    return st, pool_out, props.value
