"""Python binding of libcoremaint (batched core maintenance on MI355X).

Argument marshalling only: every step of the maintenance path runs in the HIP
kernels of ``libcoremaint.so``; this module passes pointers and sizes through
the C ABI declared in ``include/coremaint.h``.  Arrays may be torch tensors
(device tensors are passed as device pointers, CPU tensors as host pointers)
or numpy arrays (host).  PyTorch is used only for device memory and streams.

The library must have been built (``python -m paper_1612_09368_amd.build`` or
``__graft_entry__.build()``); importing the binding without it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcoremaint.so")

OK = 0
E_ARG, E_RANGE, E_SELF_LOOP, E_DUP, E_EXISTS, E_MISSING, E_DEAD = -1, -2, -3, -4, -5, -6, -7
E_NOMEM, E_CAPACITY, E_STATE, E_DEVICE, E_INTERNAL, E_BUSY, E_IO = -8, -9, -10, -11, -12, -13, -14
MODE_PLAIN, MODE_PERSISTENT = 0, 1
BATCH_INSERT, BATCH_DELETE = 0, 1

EXPORTED = [
    "cm_config_default", "cm_create", "cm_destroy", "cm_strerror", "cm_last_error",
    "cm_load_graph", "cm_core_decompose", "cm_insert_edges", "cm_delete_edges",
    "cm_insert_vertices", "cm_delete_vertices", "cm_get_cores", "cm_num_vertices",
    "cm_num_edges", "cm_export_edges", "cm_get_superior_degrees", "cm_run_batches", "cm_phase_times",
    "cm_serve_config_default", "cm_serve_start", "cm_serve_submit_edges", "cm_serve_submit_insert_vertices",
    "cm_serve_submit_delete_vertices", "cm_serve_poll", "cm_serve_result", "cm_serve_stop",
    "cm_snapshot", "cm_restore", "cm_debug_log", "cm_update_edges_noalloc",
]
REQ_INSERT_EDGES, REQ_DELETE_EDGES, REQ_INSERT_VERTICES, REQ_DELETE_VERTICES = 0, 1, 2, 3


class Config(ctypes.Structure):
    _fields_ = [
        ("vertex_capacity", ctypes.c_int32),
        ("edge_capacity_hint", ctypes.c_int64),
        ("strict", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("partition_rounds", ctypes.c_int32),
        ("blocks_per_cu", ctypes.c_int32),
        ("small_degree", ctypes.c_int32),
        ("large_degree", ctypes.c_int32),
        ("chunk", ctypes.c_int32),
        ("local_edges", ctypes.c_int32),
        ("local_items", ctypes.c_int32),
        ("local_work", ctypes.c_int32),
        ("timing", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("async_steps", ctypes.c_int32),
        ("single_edge", ctypes.c_int32),
        ("debug", ctypes.c_int32),
        ("expand_mode", ctypes.c_int32),
        ("stamp_limit", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
    ]


class ServeConfig(ctypes.Structure):
    _fields_ = [
        ("ring_requests", ctypes.c_int32),
        ("idle_ms", ctypes.c_int32),
        ("ring_items", ctypes.c_int64),
        ("max_items", ctypes.c_int64),
        ("budget_bytes", ctypes.c_int64),
        ("vertex_headroom", ctypes.c_int32),
        ("fuse", ctypes.c_int32),
    ]


class BatchStats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iterations", ctypes.c_int32),
        ("first_bad", ctypes.c_int64),
        ("applied", ctypes.c_int64),
        ("dropped", ctypes.c_int64),
        ("remaining_sum", ctypes.c_int64),
        ("candidates", ctypes.c_int64),
        ("evicted", ctypes.c_int64),
        ("changed", ctypes.c_int64),
        ("scanned", ctypes.c_int64),
        ("alg_bytes", ctypes.c_int64),
        ("rounds", ctypes.c_int64),
        ("cand_degree", ctypes.c_int64),
        ("evicted_degree", ctypes.c_int64),
        ("changed_degree", ctypes.c_int64),
        ("grid_steps", ctypes.c_int64),
        ("local_steps", ctypes.c_int64),
        ("launches", ctypes.c_int32),
        ("graph_launch", ctypes.c_int32),
        ("group", ctypes.c_int32),
        ("first_stamp", ctypes.c_int32),
        ("kernel_ms", ctypes.c_double),
        ("ms_total", ctypes.c_double),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class CoreMaintError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


_lib = None


def library():
    """Load libcoremaint.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1612_09368_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "cm_config_default": (None, [P]),
        "cm_create": (ctypes.c_int, [P, P]),
        "cm_destroy": (None, [P]),
        "cm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "cm_last_error": (ctypes.c_char_p, [P]),
        "cm_load_graph": (ctypes.c_int, [P, I32, I64, P, P, ctypes.c_int]),
        "cm_core_decompose": (ctypes.c_int, [P, P]),
        "cm_insert_edges": (ctypes.c_int, [P, I64, P, P, ctypes.c_int, P]),
        "cm_delete_edges": (ctypes.c_int, [P, I64, P, P, ctypes.c_int, P]),
        "cm_insert_vertices": (ctypes.c_int, [P, I32, P, P, ctypes.c_int, P, P]),
        "cm_delete_vertices": (ctypes.c_int, [P, I32, P, ctypes.c_int, P]),
        "cm_get_cores": (ctypes.c_int, [P, P, I32, ctypes.c_int]),
        "cm_num_vertices": (ctypes.c_int, [P, P, P]),
        "cm_num_edges": (ctypes.c_int, [P, P]),
        "cm_export_edges": (ctypes.c_int, [P, P, P, I64, P, ctypes.c_int]),
        "cm_get_superior_degrees": (ctypes.c_int, [P, P, I32, ctypes.c_int]),
        "cm_run_batches": (ctypes.c_int, [P, I32, P, P, P, P, P, I32, ctypes.c_int, P, P]),
        "cm_phase_times": (ctypes.c_int, [P, P, P, I32, ctypes.c_int]),
        "cm_serve_config_default": (None, [P]),
        "cm_serve_start": (ctypes.c_int, [P, P]),
        "cm_serve_submit_edges": (ctypes.c_int, [P, I32, I32, I64, P, P, P]),
        "cm_serve_submit_insert_vertices": (ctypes.c_int, [P, I32, P, P, P, P]),
        "cm_serve_submit_delete_vertices": (ctypes.c_int, [P, I32, P, P]),
        "cm_serve_poll": (ctypes.c_int, [P, P]),
        "cm_serve_result": (ctypes.c_int, [P, I64, P]),
        "cm_serve_stop": (ctypes.c_int, [P]),
        "cm_update_edges_noalloc": (ctypes.c_int, [P, I32, I64, P, P, P]),
        "cm_snapshot": (ctypes.c_int, [P, ctypes.c_char_p]),
        "cm_restore": (ctypes.c_int, [P, ctypes.c_char_p, P]),
        "cm_debug_log": (ctypes.c_int, [P, P, P, I64, P, P, I64]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _torch():
    import torch
    return torch


def _ptr(x, dtype):
    """(pointer, on_device, keepalive, length) for a torch tensor or array."""
    if x is None:
        return None, 0, None, 0
    mod = type(x).__module__
    if mod.startswith("torch"):
        torch = _torch()
        want = {np.int32: torch.int32, np.int64: torch.int64}[dtype]
        if x.dtype != want:
            x = x.to(want)
        x = x.contiguous()
        return ctypes.c_void_p(x.data_ptr()), int(x.is_cuda), x, x.numel()
    a = np.ascontiguousarray(x, dtype=dtype)
    return ctypes.c_void_p(a.ctypes.data), 0, a, a.size


def default_stream():
    try:
        torch = _torch()
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return ctypes.c_void_p(0)


class Graph:
    """A dynamic graph held on the GPU with exact core numbers."""

    def __init__(self, mode=MODE_PLAIN, strict=True, vertex_capacity=0, edge_capacity_hint=0,
                 partition_rounds=0, blocks_per_cu=0, small_degree=0, large_degree=0, chunk=0,
                 local_edges=0, local_items=0, local_work=0, timing=False, use_graph=False, async_steps=False,
                 single_edge=False, debug=0, expand_mode=0, stamp_limit=0, stream=None, _restore_from=None):
        lib = library()
        cfg = Config()
        lib.cm_config_default(ctypes.byref(cfg))
        cfg.mode = mode
        cfg.strict = 1 if strict else 0
        cfg.vertex_capacity = vertex_capacity
        cfg.edge_capacity_hint = edge_capacity_hint
        cfg.partition_rounds = partition_rounds
        cfg.blocks_per_cu = blocks_per_cu
        cfg.small_degree = small_degree
        cfg.large_degree = large_degree
        cfg.chunk = chunk
        cfg.local_edges = local_edges
        cfg.local_items = local_items
        cfg.local_work = local_work
        cfg.timing = 1 if timing else 0
        cfg.use_graph = 1 if use_graph else 0
        cfg.async_steps = 1 if async_steps else 0
        cfg.single_edge = 1 if single_edge else 0
        cfg.debug = int(debug)
        cfg.expand_mode = int(expand_mode)
        cfg.stamp_limit = int(stamp_limit)
        cfg.stream = stream if stream is not None else default_stream()
        h = ctypes.c_void_p()
        if _restore_from is None:
            st = lib.cm_create(ctypes.byref(cfg), ctypes.byref(h))
            what = "cm_create"
        else:
            st = lib.cm_restore(ctypes.byref(cfg), os.fsencode(_restore_from), ctypes.byref(h))
            what = "cm_restore"
        if st != OK:
            raise CoreMaintError(st, f"{what}: " + lib.cm_strerror(st).decode())
        self._lib = lib
        self._h = h
        self.config = cfg
        self.last_stats = None

    @classmethod
    def restore(cls, path, **cfg):
        """A new handle holding the state cm_snapshot wrote to `path`."""
        return cls(_restore_from=path, **cfg)

    def snapshot(self, path):
        """Write the graph's state (ids, cores, SD, edges) to `path`."""
        self._check(self._lib.cm_snapshot(self._h, os.fsencode(path)), "cm_snapshot")

    def debug_log(self):
        """Iteration log of the last update call (debug mode): (sel, chg),
        int32 arrays of shape (k, 3): (iteration stamp, u, v) per selected
        edge and (iteration stamp, v, new core) per core change."""
        ns, nc = ctypes.c_int64(), ctypes.c_int64()
        st = self._lib.cm_debug_log(self._h, ctypes.byref(ns), None, 0, ctypes.byref(nc), None, 0)
        self._check(st, "cm_debug_log")
        sel = np.empty((max(ns.value, 1), 3), dtype=np.int32)
        chg = np.empty((max(nc.value, 1), 3), dtype=np.int32)
        st = self._lib.cm_debug_log(self._h, ctypes.byref(ns), ctypes.c_void_p(sel.ctypes.data), ns.value,
                                    ctypes.byref(nc), ctypes.c_void_p(chg.ctypes.data), nc.value)
        self._check(st, "cm_debug_log")
        return sel[:ns.value], chg[:nc.value]

    def close(self):
        if getattr(self, "_h", None):
            self._lib.cm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- helpers --------------------------------------------------------
    def _check(self, st, what):
        if st != OK:
            msg = self._lib.cm_last_error(self._h).decode() or self._lib.cm_strerror(st).decode()
            raise CoreMaintError(st, f"{what}: {msg}")

    def _call_stats(self, fn, *args, check=True, what=""):
        stats = BatchStats()
        st = fn(self._h, *args, ctypes.byref(stats))
        self.last_stats = stats
        if check:
            self._check(st, what)
        return st, stats

    # -- API ------------------------------------------------------------
    def load(self, n, src, dst):
        ps, ds, ks, m = _ptr(src, np.int32)
        pd, dd, kd, m2 = _ptr(dst, np.int32)
        if m != m2 or ds != dd:
            raise ValueError("src and dst must have the same length and location")
        self._check(self._lib.cm_load_graph(self._h, int(n), m, ps, pd, ds), "cm_load_graph")

    def decompose(self):
        return self._call_stats(self._lib.cm_core_decompose, what="cm_core_decompose")[1]

    def _edges(self, fn, src, dst, check, what):
        ps, ds, ks, m = _ptr(src, np.int32)
        pd, dd, kd, m2 = _ptr(dst, np.int32)
        if m != m2 or ds != dd:
            raise ValueError("src and dst must have the same length and location")
        st, stats = self._call_stats(fn, m, ps, pd, ds, check=check, what=what)
        return stats if check else (st, stats)

    def insert_edges(self, src, dst, check=True):
        return self._edges(self._lib.cm_insert_edges, src, dst, check, "cm_insert_edges")

    def delete_edges(self, src, dst, check=True):
        return self._edges(self._lib.cm_delete_edges, src, dst, check, "cm_delete_edges")

    def update_edges_noalloc(self, kind, src, dst, check=True):
        """cm_update_edges_noalloc: insert (kind BATCH_INSERT) or delete
        (BATCH_DELETE) device-resident edges without allocating."""
        ps, ds, ks, m = _ptr(src, np.int32)
        pd, dd, kd, m2 = _ptr(dst, np.int32)
        if m != m2 or not ds or not dd:
            raise ValueError("src and dst must be device arrays of the same length")
        st, stats = self._call_stats(self._lib.cm_update_edges_noalloc, int(kind), m, ps, pd, check=check,
                                     what="cm_update_edges_noalloc")
        return stats if check else (st, stats)

    def insert_vertices(self, off, nbrs, check=True):
        po, do, ko, c1 = _ptr(off, np.int64)
        pn, dn, kn, _ = _ptr(nbrs, np.int32)
        first = ctypes.c_int32(-1)
        st, stats = self._call_stats(self._lib.cm_insert_vertices, c1 - 1, po, pn, do,
                                     ctypes.byref(first), check=check, what="cm_insert_vertices")
        return (first.value, stats) if check else (st, first.value, stats)

    def delete_vertices(self, ids, check=True):
        pi, di, ki, c = _ptr(ids, np.int32)
        st, stats = self._call_stats(self._lib.cm_delete_vertices, c, pi, di, check=check,
                                     what="cm_delete_vertices")
        return stats if check else (st, stats)

    def run_batches(self, kinds, offsets, src, dst, sub=None, nsub=0):
        """Run a sequence of edge batches (see cm_run_batches).  kinds / offsets
        are host sequences; src, dst (and sub) may live on the device.
        Returns (list of BatchStats, sub-batch statuses or None)."""
        kinds = np.ascontiguousarray(kinds, dtype=np.int32)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        nb = kinds.size
        ps, ds, ks, m = _ptr(src, np.int32)
        pd, dd, kd, m2 = _ptr(dst, np.int32)
        if m != m2 or ds != dd or offsets.size != nb + 1 or (nb and offsets[-1] != m):
            raise ValueError("inconsistent batch arrays")
        psub, dsub, ksub = None, ds, None
        if sub is not None:
            psub, dsub, ksub, m3 = _ptr(sub, np.int32)
            if m3 != m or dsub != ds:
                raise ValueError("sub must match src")
        res = (BatchStats * max(nb, 1))()
        sst = np.zeros(max(nsub, 1), dtype=np.int32)
        st = self._lib.cm_run_batches(self._h, nb, ctypes.c_void_p(kinds.ctypes.data),
                                      ctypes.c_void_p(offsets.ctypes.data), ps, pd, psub, int(nsub), ds,
                                      ctypes.cast(res, ctypes.c_void_p),
                                      ctypes.c_void_p(sst.ctypes.data) if sub is not None else None)
        self._check(st, "cm_run_batches")
        return [res[j] for j in range(nb)], (sst[:nsub] if sub is not None else None)

    def num_vertices(self):
        n = ctypes.c_int32()
        a = ctypes.c_int32()
        self._check(self._lib.cm_num_vertices(self._h, ctypes.byref(n), ctypes.byref(a)), "cm_num_vertices")
        return n.value, a.value

    def num_edges(self):
        m = ctypes.c_int64()
        self._check(self._lib.cm_num_edges(self._h, ctypes.byref(m)), "cm_num_edges")
        return m.value

    def cores(self, out=None):
        """Core numbers of every id (dead ids -1).  Returns a numpy array,
        or fills `out` (a torch int32 tensor, device or host) and returns it."""
        n, _ = self.num_vertices()
        if out is None:
            arr = np.empty(n, dtype=np.int32)
            self._check(self._lib.cm_get_cores(self._h, ctypes.c_void_p(arr.ctypes.data), n, 0),
                        "cm_get_cores")
            return arr
        p, dev, keep, cnt = _ptr(out, np.int32)
        self._check(self._lib.cm_get_cores(self._h, p, min(n, cnt), dev), "cm_get_cores")
        return out

    PHASES = ("claim", "select", "apply", "expand", "evict", "peel", "core", "sd",
              "local", "validate", "reserve", "compact")

    def phase_times(self, reset=False):
        """{phase: (ms, count)} of the device phase clock (see cm_phase_times)."""
        k = len(self.PHASES)
        ms = np.zeros(k, dtype=np.float64)
        cnt = np.zeros(k, dtype=np.int64)
        self._check(self._lib.cm_phase_times(self._h, ctypes.c_void_p(ms.ctypes.data),
                                             ctypes.c_void_p(cnt.ctypes.data), k, 1 if reset else 0),
                    "cm_phase_times")
        return {p: (float(ms[i]), int(cnt[i])) for i, p in enumerate(self.PHASES)}

    def superior_degrees(self):
        n, _ = self.num_vertices()
        arr = np.empty(n, dtype=np.int32)
        self._check(self._lib.cm_get_superior_degrees(self._h, ctypes.c_void_p(arr.ctypes.data), n, 0),
                    "cm_get_superior_degrees")
        return arr

    def export_edges(self):
        m = self.num_edges()
        s = np.empty(max(m, 1), dtype=np.int32)
        d = np.empty(max(m, 1), dtype=np.int32)
        got = ctypes.c_int64()
        self._check(self._lib.cm_export_edges(self._h, ctypes.c_void_p(s.ctypes.data),
                                              ctypes.c_void_p(d.ctypes.data), m, ctypes.byref(got), 0),
                    "cm_export_edges")
        return s[:got.value], d[:got.value]


def union_edges(graphs):
    """Disjoint union of [(n, src, dst), ...]: (base int64[len+1], src, dst)
    with graph i's ids offset by base[i]."""
    base = np.concatenate([[0], np.cumsum([int(n) for n, _, _ in graphs])]).astype(np.int64)
    if not graphs:
        return base, np.empty(0, np.int32), np.empty(0, np.int32)
    src = np.concatenate([np.asarray(s, np.int64) + b for (_, s, _), b in zip(graphs, base)])
    dst = np.concatenate([np.asarray(d, np.int64) + b for (_, _, d), b in zip(graphs, base)])
    return base, src.astype(np.int32), dst.astype(np.int32)


def pack_batches(base, batches):
    """Group per-graph batches into union batches with sub-batch ids.

    batches: list of (graph_id, kind, src, dst) in submission order (ids
    local to the graph).  The t-th batch of every graph forms stage t; each
    stage becomes one insertion batch and one deletion batch of the union
    (in that order; a graph's own order is kept because its t-th batch is
    in stage t).  Returns (kinds, offsets, src, dst, sub, nsub, order), where
    order[k] is the sub-batch id of submission k."""
    per_graph = {}
    stage_of = []
    for gid, kind, s, d in batches:
        t = per_graph.get(gid, 0)
        per_graph[gid] = t + 1
        stage_of.append(t)
    nstages = max(stage_of) + 1 if batches else 0
    kinds, offs, srcs, dsts, subs = [], [0], [], [], []
    order = np.full(len(batches), -1, dtype=np.int64)
    nsub = 0
    for t in range(nstages):
        for kind in (BATCH_INSERT, BATCH_DELETE):
            members = [k for k in range(len(batches)) if stage_of[k] == t and batches[k][1] == kind]
            if not members:
                continue
            for k in members:
                gid, _, s, d = batches[k]
                b = base[gid]
                srcs.append(np.asarray(s, np.int64) + b)
                dsts.append(np.asarray(d, np.int64) + b)
                subs.append(np.full(len(s), nsub, np.int32))
                order[k] = nsub
                nsub += 1
            kinds.append(kind)
            offs.append(offs[-1] + sum(len(batches[k][2]) for k in members))
    cat = (lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.empty(0, dt))
    return (np.asarray(kinds, np.int32), np.asarray(offs, np.int64), cat(srcs, np.int32),
            cat(dsts, np.int32), cat(subs, np.int32), nsub, order)


class GraphPool:
    """Many independent graphs updated together.

    The graphs are packed as one disjoint union (graph i's ids are offset by
    the sizes of the graphs before it); a disjoint union has no edge between
    two members, so its core numbers are exactly the members' core numbers.
    Per-graph batches are grouped into stages (see pack_batches) so that one
    ``cm_run_batches`` call (one persistent launch, optionally a hipGraph
    replay) updates every graph; an invalid member batch is dropped alone.
    """

    def __init__(self, graphs, **cfg):
        self.base, src, dst = union_edges(graphs)
        self.sizes = np.diff(self.base).tolist()
        self.graph = Graph(**cfg)
        self.graph.load(int(self.base[-1]), src, dst)
        self.graph.decompose()

    def pack(self, batches):
        return pack_batches(self.base, batches)

    def run(self, batches, device=None):
        """Apply the per-graph batches; returns (one status per submission, stats)."""
        kinds, offs, s, d, sub, nsub, order = self.pack(batches)
        if device is not None:
            torch = _torch()
            s, d, sub = (torch.from_numpy(x).to(device) for x in (s, d, sub))
        stats, sst = self.graph.run_batches(kinds, offs, s, d, sub=sub, nsub=nsub)
        return [int(sst[order[k]]) for k in range(len(batches))], stats

    def cores(self, gid):
        c = self.graph.cores()
        return c[self.base[gid]:self.base[gid + 1]]

    def close(self):
        self.graph.close()
