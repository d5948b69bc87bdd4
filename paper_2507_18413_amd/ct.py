"""Thin Python binding of libct.so (argument marshalling only).

Every step of propagation runs in the library's HIP kernels; this module only
converts numpy arrays / torch tensors to pointers and back.  If the library
is missing it raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "libct.so")
HEADER = os.path.join(ROOT, "include", "ct.h")

OK, FAIL = 0, 1
E_INVALID, E_NOT_SUBSET, E_STATE, E_NOMEM, E_DEVICE = -1, -2, -3, -4, -5
BRANCH_AUTO, BRANCH_RESET, BRANCH_INCREMENTAL = 0, 1, 2
SCHED_AUTO, SCHED_SOLO, SCHED_SPLIT, SCHED_NODES, SCHED_RESIDENT = 0, 1, 2, 3, 4
JOB_PROPAGATE, JOB_FROM_ROOT, JOB_ROOT = 1, 2, 4
SPLIT_UPDATE, SPLIT_FILTER = 1, 2
KIND_POSITIVE, KIND_NEGATIVE, KIND_SHORT = 0, 1, 2
STAR = -(1 << 31)  # a cell of a short table: every value of its column


try:  # CPython binding of the per-call entry points (built with libct.so)
    from . import _ctfast as _F
except ImportError:  # the ctypes path below marshals the same calls
    _F = None


class CTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"CT error {code}: {msg}")
        self.code = code


class ct_config(C.Structure):
    _fields_ = [("branch_policy", C.c_int32), ("max_depth", C.c_int32), ("schedule", C.c_int32)]


class ct_layout_info(C.Structure):
    _fields_ = [("n_vars", C.c_int32), ("D", C.c_int32), ("W", C.c_int64), ("n_tuples", C.c_int64),
                ("rows", C.c_int32), ("n_slots", C.c_int32), ("granules", C.c_int32),
                ("root_failed", C.c_int32), ("resident", C.c_int32), ("kind", C.c_int32)]


class ct_stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("jobs", "granules_in", "rows_or", "granule_rows",
                                         "trail_granules", "residue_checks", "residue_misses",
                                         "scan_granules")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class ct_job(C.Structure):
    _fields_ = [("table", C.c_void_p), ("slot", C.c_int32), ("flags", C.c_uint32),
                ("n_pop", C.c_int32), ("n_push", C.c_int32), ("dom_in", C.c_void_p),
                ("dom_out", C.c_void_p), ("ct_out", C.c_void_p)]


class ct_server_cfg(C.Structure):
    _fields_ = [("mem_budget", C.c_int64), ("max_batch", C.c_int32), ("streams", C.c_int32)]


class ct_request(C.Structure):
    _fields_ = [("search", C.c_int32), ("flags", C.c_uint32), ("n_pop", C.c_int32), ("push", C.c_int32),
                ("remove", C.c_void_p), ("dom_out", C.c_void_p), ("tag", C.c_uint64)]


class ct_completion(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("search", C.c_int32), ("status", C.c_int32),
                ("t_submit", C.c_double), ("t_launch", C.c_double), ("t_done", C.c_double)]


REQ_FINISH = 1

_lib = None


def exported_names():
    """Function names declared in include/ct.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|void|const char \*)\s*(ct_\w+)\s*\(", text, re.M)))


def _preload_shared_hip_runtime():
    """Load the HIP runtime PyTorch ships before libct.so, so that the
    library, torch's streams and torch's allocations share one runtime
    (the library's libamdhip64.so.7 dependency resolves to the loaded copy,
    and a later `import torch` maps the same file again)."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.origin:
        return
    path = os.path.join(os.path.dirname(spec.origin), "lib", "libamdhip64.so")
    if os.path.exists(path):
        C.CDLL(path, mode=C.RTLD_GLOBAL)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        _preload_shared_hip_runtime()
        L = C.CDLL(LIB_PATH)
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "ct_create": ([P, I64, I32, P, P, P, P, C.POINTER(P)], C.c_int),
            "ct_create_table": ([P, I64, I32, P, P, P, P, I32, C.POINTER(P)], C.c_int),
            "ct_destroy": ([P], None),
            "ct_layout": ([P, C.POINTER(ct_layout_info), P], C.c_int),
            "ct_get_supports": ([P, I32, I32, P], C.c_int),
            "ct_propagate": ([P, P, P, P, P], C.c_int),
            "ct_propagate_slot": ([P, I32, P, P, P, P], C.c_int),
            "ct_push": ([P], C.c_int),
            "ct_pop": ([P], C.c_int),
            "ct_push_slot": ([P, I32], C.c_int),
            "ct_pop_slot": ([P, I32], C.c_int),
            "ct_get_state": ([P, I32, P, P], C.c_int),
            "ct_slots_alloc": ([P, I32, I32, C.POINTER(I32)], C.c_int),
            "ct_slots_free": ([P, I32, I32], C.c_int),
            "ct_slot_stats": ([P, I32, C.POINTER(ct_stats)], C.c_int),
            "ct_propagate_batch": ([P, I32, P, P], C.c_int),
            "ct_propagate_batch_noalloc": ([P, I32, P, P], C.c_int),
            "ct_batch_status": ([P], C.c_int),
            "ct_set_timing": ([P, I32], C.c_int),
            "ct_get_timing": ([P, C.POINTER(C.c_double), C.POINTER(I64)], C.c_int),
            "ct_get_dispatch_timing": ([P, C.POINTER(C.c_double), C.POINTER(I64)], C.c_int),
            "ct_model_create": ([I32, P, P, C.POINTER(P)], C.c_int),
            "ct_model_destroy": ([P], None),
            "ct_model_add": ([P, P, P, C.POINTER(I32)], C.c_int),
            "ct_model_layout": ([P, P, C.POINTER(I32)], C.c_int),
            "ct_model_fixpoint": ([P, P, P, P, C.POINTER(I64), C.POINTER(I64)], C.c_int),
            "ct_model_push": ([P], C.c_int),
            "ct_model_pop": ([P], C.c_int),
            "ct_model_set_schedule": ([P, I32, I32], C.c_int),
            "ct_model_autotune": ([P, P, C.c_char_p, C.POINTER(I32), C.POINTER(I32)], C.c_int),
            "ct_model_get_choice": ([P, I32, C.POINTER(I32), C.POINTER(I32)], C.c_int),
            "ct_server_create": ([C.POINTER(ct_server_cfg), C.POINTER(P)], C.c_int),
            "ct_server_destroy": ([P], None),
            "ct_server_add_search": ([P, P, I32, C.POINTER(I32)], C.c_int),
            "ct_server_submit": ([P, C.POINTER(ct_request)], C.c_int),
            "ct_server_poll": ([P, P, I32, I32], C.c_int),
            "ct_server_stats": ([P, P, I32], C.c_int),
            "ct_server_now": ([], C.c_double),
            "ct_split_create": ([P, I32, C.POINTER(P)], C.c_int),
            "ct_split_propagate": ([P, P, P, P], C.c_int),
            "ct_split_push": ([P], C.c_int),
            "ct_split_pop": ([P], C.c_int),
            "ct_split_destroy": ([P], None),
            "ct_last_error": ([], C.c_char_p),
            "ct_debug_fail_alloc": ([I32], C.c_int),
            "ct_quiesce": ([], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
        if _F is not None:
            addr = lambda f: C.cast(f, C.c_void_p).value  # noqa: E731
            _F.bind(addr(L.ct_propagate_slot), addr(L.ct_push_slot), addr(L.ct_pop_slot))
        # a resident engine writes its state back and ends before exit
        import atexit
        atexit.register(L.ct_quiesce)
    return _lib


def last_error() -> str:
    return lib().ct_last_error().decode()


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _ptr(x):
    """Device pointer of a torch tensor, or an int address."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


class Table:
    """One table constraint on the GPU with its slots (reversible states)."""

    def __init__(self, tuples, lo, dsizes, init_dom=None, branch_policy=BRANCH_AUTO, max_depth=256,
                 schedule=SCHED_AUTO, kind=KIND_POSITIVE):
        L = lib()
        tuples = np.ascontiguousarray(tuples, dtype=np.int32)
        lo = np.ascontiguousarray(lo, dtype=np.int32)
        ds = np.ascontiguousarray(dsizes, dtype=np.int32)
        t = int(tuples.shape[0]) if tuples.ndim == 2 and tuples.size else 0
        if init_dom is not None:
            init_dom = np.ascontiguousarray(init_dom, dtype=np.uint64)
        cfg = ct_config(int(branch_policy), int(max_depth), int(schedule))
        h = C.c_void_p()
        st = L.ct_create_table(_p(tuples) if t else None, t, int(ds.shape[0]), _p(lo), _p(ds), _p(init_dom),
                               C.byref(cfg), int(kind), C.byref(h))
        if st < 0:
            raise CTError(st, last_error())
        self.h = h
        self.create_status = st
        info = ct_layout_info()
        off = np.zeros(ds.shape[0], np.int32)
        L.ct_layout(h, C.byref(info), _p(off))
        self.n, self.D, self.W, self.t = info.n_vars, info.D, info.W, info.n_tuples
        self.rows, self.granules, self.root_failed = info.rows, info.granules, bool(info.root_failed)
        # synchronous calls on slot 0: the resident engine (one workgroup, its
        # state in LDS) or the resident split schedule (persistent update and
        # filter workgroups)
        self.resident = info.resident == 1
        self.resident_split = info.resident == 2
        self.kind = int(info.kind)
        self.dom_off = off
        # marshalling buffers of the synchronous calls: fixed addresses, so a
        # call converts no pointer (numpy's ctypes pointers cost microseconds)
        self._din = np.zeros(max(self.D, 1), np.uint64)
        self._dout = np.zeros(max(self.D, 1), np.uint64)
        self._din_p = self._din.__array_interface__["data"][0]
        self._dout_p = self._dout.__array_interface__["data"][0]
        self._prop = L.ct_propagate_slot
        self._push = L.ct_push_slot
        self._pop = L.ct_pop_slot
        self._hv = h.value  # the handle as an int, for the CPython binding

    @property
    def n_slots(self):
        info = ct_layout_info()
        lib().ct_layout(self.h, C.byref(info), None)
        return info.n_slots

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value is not None:
            lib().ct_destroy(self.h)
            self.h = None
            self._hv = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def propagate(self, dom_in, slot=0, want_ct=False, want_stats=False):
        if len(dom_in) != self.D:
            raise ValueError(f"dom_in has {len(dom_in)} words, the table {self.D}")
        D = self.D
        if not (want_ct or want_stats):
            if _F is not None:
                # uint64 arrays go straight to the library; None: marshal below
                out = np.empty(D, np.uint64)
                st = _F.propagate(self._hv, slot, dom_in, out, D)
                if st is not None:
                    if st == E_DEVICE:
                        raise CTError(st, last_error())
                    if st != OK:  # dom_out is written only on OK
                        out[:] = dom_in
                    return st, out
            # the common call: one copy in, one out
            self._din[:D] = dom_in
            st = self._prop(self.h, slot, self._din_p, self._dout_p, None, None)
            if st == E_DEVICE:
                raise CTError(st, last_error())
            # dom_out is written only on OK (the input is returned otherwise)
            return st, (self._dout if st == OK else self._din)[:D].copy()
        self._din[:D] = dom_in
        self._dout[:D] = self._din[:D]
        ct = np.zeros(max(self.W, 1), np.uint64) if want_ct else None
        stats = ct_stats() if want_stats else None
        st = self._prop(self.h, int(slot), self._din_p, self._dout_p, _p(ct),
                        C.byref(stats) if stats is not None else None)
        if st == E_DEVICE:
            raise CTError(st, last_error())
        out = [st, self._dout[: self.D].copy()]
        if want_ct:
            out.append(ct[: self.W])
        if want_stats:
            out.append(stats.as_dict())
        return tuple(out)

    def push(self, slot=0):
        if _F is not None:
            return _F.push(self._hv, slot)
        return self._push(self.h, int(slot))

    def pop(self, slot=0):
        if _F is not None:
            return _F.pop(self._hv, slot)
        return self._pop(self.h, int(slot))

    def state(self, slot=0):
        dom = np.zeros(self.D, np.uint64)
        ct = np.zeros(max(self.W, 1), np.uint64)
        st = lib().ct_get_state(self.h, int(slot), _p(dom), _p(ct))
        if st < 0:
            raise CTError(st, last_error())
        return dom, ct[: self.W]

    def domains(self, slot=0):
        return self.state(slot)[0]

    def supports(self, row_begin=0, n_rows=None):
        n_rows = self.rows - row_begin if n_rows is None else n_rows
        out = np.zeros((n_rows, max(self.W, 1)), np.uint64)
        st = lib().ct_get_supports(self.h, int(row_begin), int(n_rows), _p(out))
        if st < 0:
            raise CTError(st, last_error())
        return out[:, : self.W]

    def slots_alloc(self, n, max_depth=-1):
        first = C.c_int32()
        st = lib().ct_slots_alloc(self.h, int(n), int(max_depth), C.byref(first))
        if st < 0:
            raise CTError(st, last_error())
        return first.value

    def slots_free(self, first, n=1):
        st = lib().ct_slots_free(self.h, int(first), int(n))
        if st < 0:
            raise CTError(st, last_error())

    def set_timing(self, on=True):
        st = lib().ct_set_timing(self.h, 1 if on else 0)
        if st < 0:
            raise CTError(st, last_error())

    def timing(self):
        """(cumulative kernel milliseconds, launches) since set_timing(True)."""
        ms, n = C.c_double(), C.c_int64()
        lib().ct_get_timing(self.h, C.byref(ms), C.byref(n))
        return ms.value, n.value

    def dispatch_timing(self):
        """(cumulative launch lifetimes in ms, launches) since set_timing(True);
        for the resident engine, whole launch lifetimes (ends the engine)."""
        ms, n = C.c_double(), C.c_int64()
        st = lib().ct_get_dispatch_timing(self.h, C.byref(ms), C.byref(n))
        if st < 0:
            raise CTError(st, last_error())
        return ms.value, n.value

    def stats(self, slot=0):
        s = ct_stats()
        st = lib().ct_slot_stats(self.h, int(slot), C.byref(s))
        if st < 0:
            raise CTError(st, last_error())
        return s.as_dict()


def quiesce():
    """End the resident engine of any table (it writes its state back)."""
    st = lib().ct_quiesce()
    if st < 0:
        raise CTError(st, last_error())


def batch_status(stream=None):
    """Synchronize `stream`; raise if a batch on it hit a device-side error."""
    s = None if stream is None else (stream if isinstance(stream, int) else stream.cuda_stream)
    st = lib().ct_batch_status(s)
    if st < 0:
        raise CTError(st, last_error())


class SplitPropagator:
    """One of the two split propagators over a table (updateTable or
    filterDomains on the device, the other procedure on the host); same
    calls and results as ``Table.propagate`` / ``push`` / ``pop``."""

    def __init__(self, table: Table, mode: int):
        L = lib()
        h = C.c_void_p()
        st = L.ct_split_create(table.h, int(mode), C.byref(h))
        if st < 0:
            raise CTError(st, last_error())
        self.h = h
        self.table = table  # the supports stay on the table's device buffers
        self.D, self.W = table.D, table.W
        self._din = np.zeros(max(self.D, 1), np.uint64)
        self._dout = np.zeros(max(self.D, 1), np.uint64)
        self._din_p = self._din.__array_interface__["data"][0]
        self._dout_p = self._dout.__array_interface__["data"][0]
        self._prop = L.ct_split_propagate

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value is not None:
            lib().ct_split_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def propagate(self, dom_in, want_ct=False):
        if len(dom_in) != self.D:
            raise ValueError(f"dom_in has {len(dom_in)} words, the table {self.D}")
        D = self.D
        self._din[:D] = dom_in
        ct = np.zeros(max(self.W, 1), np.uint64) if want_ct else None
        st = self._prop(self.h, self._din_p, self._dout_p, _p(ct))
        if st == E_DEVICE:
            raise CTError(st, last_error())
        dom = (self._dout if st == OK else self._din)[:D].copy()
        return (st, dom, ct[: self.W]) if want_ct else (st, dom)

    def push(self):
        return lib().ct_split_push(self.h)

    def pop(self):
        return lib().ct_split_pop(self.h)


class Batch:
    """A job list marshalled once into the ct_job array, for batches that are
    launched repeatedly with the same jobs (the buffers stay the caller's)."""

    def __init__(self, jobs):
        jobs = list(jobs)
        self.n = len(jobs)
        self.arr = (ct_job * max(1, self.n))()
        for k, j in enumerate(jobs):
            a = self.arr[k]
            a.table = j["table"].h.value
            a.slot = int(j.get("slot", 0))
            a.flags = int(j.get("flags", JOB_PROPAGATE))
            a.n_pop = int(j.get("n_pop", 0))
            a.n_push = int(j.get("n_push", 0))
            a.dom_in = _ptr(j.get("dom_in"))
            a.dom_out = _ptr(j.get("dom_out"))
            a.ct_out = _ptr(j.get("ct_out"))
        self._refs = jobs  # keep tensors alive

    def run(self, status_dev, stream=None, noalloc=False):
        s = None if stream is None else (stream if isinstance(stream, int) else stream.cuda_stream)
        fn = lib().ct_propagate_batch_noalloc if noalloc else lib().ct_propagate_batch
        st = fn(C.cast(self.arr, C.c_void_p), self.n, s, _ptr(status_dev))
        if st < 0:
            raise CTError(st, last_error())
        return st


def propagate_batch(jobs, status_dev, stream=None, noalloc=False):
    """jobs: a Batch, or an iterable of dicts with keys table, slot, flags,
    n_pop, n_push, dom_in, dom_out, ct_out (torch tensors or device
    addresses).  status_dev: int32 device tensor (or address) with one entry
    per job.  noalloc: call ct_propagate_batch_noalloc (no allocation; the
    library's static device scratch)."""
    b = jobs if isinstance(jobs, Batch) else Batch(jobs)
    return b.run(status_dev, stream, noalloc)


class Model:
    """Tables sharing a pool of variables; fixpoint propagation on the GPU."""

    def __init__(self, lo, dsizes):
        L = lib()
        lo = np.ascontiguousarray(lo, dtype=np.int32)
        ds = np.ascontiguousarray(dsizes, dtype=np.int32)
        h = C.c_void_p()
        st = L.ct_model_create(int(ds.shape[0]), _p(lo), _p(ds), C.byref(h))
        if st < 0:
            raise CTError(st, last_error())
        self.h = h
        self.n = int(ds.shape[0])
        self.tables = []
        off = np.zeros(self.n, np.int32)
        w = C.c_int32()
        L.ct_model_layout(h, _p(off), C.byref(w))
        self.pool_off, self.pool_words = off, w.value

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value is not None:
            lib().ct_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, table, scope):
        scope = np.ascontiguousarray(scope, dtype=np.int32)
        idx = C.c_int32()
        st = lib().ct_model_add(self.h, table.h, _p(scope), C.byref(idx))
        if st < 0:
            raise CTError(st, last_error())
        self.tables.append(table)
        return idx.value

    def fixpoint(self, pool_in, pool_out, stream=None):
        """pool_in / pool_out: device tensors of pool_words int64 (bit patterns).
        Returns (status, propagations, rounds)."""
        s = None if stream is None else (stream if isinstance(stream, int) else stream.cuda_stream)
        props, rounds = C.c_int64(), C.c_int64()
        st = lib().ct_model_fixpoint(self.h, _ptr(pool_in), _ptr(pool_out), s, C.byref(props),
                                     C.byref(rounds))
        if st < 0:
            raise CTError(st, last_error())
        return st, props.value, rounds.value

    def push(self):
        st = lib().ct_model_push(self.h)
        if st < 0:
            raise CTError(st, last_error())

    def pop(self):
        st = lib().ct_model_pop(self.h)
        if st < 0:
            raise CTError(st, last_error())

    def set_schedule(self, solo_max_granules, rounds_per_graph=8):
        st = lib().ct_model_set_schedule(self.h, int(solo_max_granules), int(rounds_per_graph))
        if st < 0:
            raise CTError(st, last_error())

    def autotune(self, pool_in, cache_path=None):
        """Tune the per-class schedule (solo / split, tile); returns
        (from_cache, candidates timed)."""
        fc, timed = C.c_int32(), C.c_int32()
        path = None if cache_path is None else os.fsencode(cache_path)
        st = lib().ct_model_autotune(self.h, _ptr(pool_in), path, C.byref(fc), C.byref(timed))
        if st < 0:
            raise CTError(st, last_error())
        return bool(fc.value), timed.value

    def choice(self, table_index):
        """(solo, tile) of a table's round job."""
        solo, tile = C.c_int32(), C.c_int32()
        st = lib().ct_model_get_choice(self.h, int(table_index), C.byref(solo), C.byref(tile))
        if st < 0:
            raise CTError(st, last_error())
        return bool(solo.value), tile.value


class Server:
    """Continuous-batching serving loop over many searches (one thread in the
    library).  Requests name values to remove; completions carry status and
    timestamps; dom_out is written into the caller's buffer."""

    def __init__(self, mem_budget=0, max_batch=1024, streams=2):
        cfg = ct_server_cfg(int(mem_budget), int(max_batch), int(streams))
        h = C.c_void_p()
        st = lib().ct_server_create(C.byref(cfg), C.byref(h))
        if st < 0:
            raise CTError(st, last_error())
        self.h = h
        self._keep = {}

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value is not None:
            lib().ct_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_search(self, table, max_depth=64):
        sid = C.c_int32()
        st = lib().ct_server_add_search(self.h, table.h, int(max_depth), C.byref(sid))
        if st < 0:
            raise CTError(st, last_error())
        return sid.value

    def submit(self, search, remove=None, n_pop=0, push=0, finish=False, dom_out=None, tag=0):
        """remove / dom_out: numpy uint64 arrays (dom_out must stay alive until
        the completion is polled)."""
        r = ct_request(int(search), REQ_FINISH if finish else 0, int(n_pop), int(push),
                       _p(remove), _p(dom_out), int(tag))
        if dom_out is not None:
            self._keep[int(tag)] = dom_out
        st = lib().ct_server_submit(self.h, C.byref(r))
        if st < 0:
            raise CTError(st, last_error())

    def poll(self, max_n=4096, wait_us=1000):
        arr = (ct_completion * max_n)()
        n = lib().ct_server_poll(self.h, C.cast(arr, C.c_void_p), int(max_n), int(wait_us))
        if n < 0:
            raise CTError(n, last_error())
        out = []
        for k in range(n):
            c = arr[k]
            self._keep.pop(int(c.tag), None)
            out.append((int(c.tag), int(c.search), int(c.status), c.t_submit, c.t_launch, c.t_done))
        return out

    def stats(self):
        a = np.zeros(9, np.int64)
        lib().ct_server_stats(self.h, _p(a), 9)
        return dict(done=int(a[0]), launches=int(a[1]), admission_waits=int(a[2]),
                    slot_bytes_in_use=int(a[3]), peak_slot_bytes=int(a[4]), slots_allocated=int(a[5]),
                    multi_request_launches=int(a[6]), multi_table_launches=int(a[7]),
                    max_batch=int(a[8]))

    @staticmethod
    def now():
        return lib().ct_server_now()
