"""CPU oracle for batched core maintenance -- TEST INFRASTRUCTURE ONLY.

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  The GPU library never imports, links or calls it,
and it imports nothing from the GPU path (inputs come from ``graphgen``).

What the oracle computes.  Core maintenance must reach exactly the core
numbers of the updated graph (problem statement, Section III: incremental and
decremental core maintenance; core number definition).  That result is a graph
invariant with a plain definition, so the oracle *is* the definition: apply
the batch to the oracle's own host copy of the edge set, then recompute every
core number from scratch.

Functions
---------
``bz_cores``       Batagelj-Zaversnik O(m) bucket decomposition (the paper's
                   cited linear-time static algorithm, Introduction), in C
                   (``bz.c``), on a symmetric CSR built by the oracle itself.
``peel_cores``     Threshold peeling: for k = 1, 2, ... repeatedly delete
                   vertices of degree < k; core(v) is the last k at which v
                   survives (the k-core definition, Section III, written out).
``brute_cores``    Definitional brute force for tiny graphs: core(v) is the
                   largest min-degree of an induced subgraph containing v
                   (core number definition, Section III).
``DynamicGraph``   Host edge-set model with the batch validation convention of
                   the C library boundary, recomputing cores after each batch.
``method``         (submodule) the paper's iterative algorithms (Algorithms
                   1-7, Sections V-VI) in plain Python for tiny graphs; used to
                   pin the paper's lemmas and the readings taken of it.

Pins (tests/test_oracle.py): brute force == peeling == BZ == networkx on all
labelled graphs with n <= 5 and random graphs up to n = 2000; closed forms
(complete, cycle, tree, complete bipartite, Petersen, wheel, grid, empty).
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

# Status codes of the C boundary convention, mirrored for expected values.
OK = 0
E_ARG = -1
E_RANGE = -2
E_SELF_LOOP = -3
E_DUP = -4
E_EXISTS = -5
E_MISSING = -6
E_DEAD = -7


def build(force: bool = True) -> str:
    """Compile bz.c with gcc into liboracle.so (host code, no GPU)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp,
                               os.path.join(_HERE, "bz.c")])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        lib.oracle_bz_cores.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_bz_cores.restype = ctypes.c_int
        lib.oracle_build_csr.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_build_csr.restype = ctypes.c_int64
        _lib = lib
    return _lib


def csr(n: int, src, dst):
    """Symmetric CSR (off int64[n+1], adj int32[2m]) of an undirected edge list."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    off = np.zeros(n + 1, dtype=np.int64)
    adj = np.empty(max(2 * src.size, 1), dtype=np.int32)
    got = lib.oracle_build_csr(n, src.size, src.ctypes.data, dst.ctypes.data,
                               off.ctypes.data, adj.ctypes.data)
    if got < 0:
        raise MemoryError("oracle_build_csr")
    return off, adj


def bz_cores(n: int, src, dst, alive=None) -> np.ndarray:
    """Core numbers of the simple graph (n, edges) by the BZ bucket algorithm.
    Ids with alive[v] == 0 report -1 (they must have no edges)."""
    lib = _load()
    core = np.empty(max(n, 1), dtype=np.int32)
    if n == 0:
        return core[:0]
    off, adj = csr(n, src, dst)
    al = None
    if alive is not None:
        al = np.ascontiguousarray(alive, dtype=np.uint8)
    rc = lib.oracle_bz_cores(n, off.ctypes.data, adj.ctypes.data,
                             al.ctypes.data if al is not None else None, core.ctypes.data)
    if rc != 0:
        raise MemoryError("oracle_bz_cores")
    return core[:n]


def peel_cores(n: int, src, dst) -> np.ndarray:
    """Threshold peeling, written from the k-core definition: the k-core is
    what remains after repeatedly removing vertices of degree < k; a vertex's
    core number is the largest k whose k-core still contains it."""
    nbrs = [set() for _ in range(n)]
    for a, b in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()):
        nbrs[a].add(b)
        nbrs[b].add(a)
    core = np.zeros(n, dtype=np.int32)
    alive = set(range(n))
    k = 0
    while alive:
        k += 1
        deg = {v: sum(1 for w in nbrs[v] if w in alive) for v in alive}
        changed = True
        while changed:
            changed = False
            for v in list(alive):
                if deg[v] < k:
                    alive.discard(v)
                    for w in nbrs[v]:
                        if w in alive:
                            deg[w] -= 1
                    changed = True
        for v in alive:
            core[v] = k
    return core


def brute_cores(n: int, src, dst) -> np.ndarray:
    """Definitional brute force (n <= 16): core(v) = max over vertex subsets S
    containing v of the minimum degree of the induced subgraph G[S]."""
    if n > 16:
        raise ValueError("brute force is for tiny graphs")
    adjmask = [0] * n
    for a, b in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()):
        adjmask[a] |= 1 << b
        adjmask[b] |= 1 << a
    best = [0] * n
    for s in range(1, 1 << n):
        members = [v for v in range(n) if s >> v & 1]
        mindeg = min(bin(adjmask[v] & s).count("1") for v in members)
        for v in members:
            if mindeg > best[v]:
                best[v] = mindeg
    return np.asarray(best, dtype=np.int32)


def keys_of(a, b):
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    return (np.minimum(a, b) << 32) | np.maximum(a, b)


class DynamicGraph:
    """Host model of the dynamic graph: the canonical edge keys plus an alive
    mask of vertex ids.  Each batch method validates the batch with the C
    boundary's convention, applies it (or not, in strict mode) and the caller
    recomputes cores with ``cores()`` (BZ from scratch).

    Storage: the keys of the initial graph stay in one sorted array with a
    presence mask; keys inserted later live in a sorted side array.  A batch
    therefore costs a search per item instead of a re-sort of the whole set,
    which keeps streams of 10^7 updates on 6.4 x 10^7 edges checkable.  The
    edge set it represents is the plain set union / difference of the batches.

    Validation convention (boundary rule, not from the paper): in a batch of
    edges, item i is invalid if an endpoint is out of [0, n_ids) (E_RANGE),
    an endpoint is a dead id (E_DEAD), it is a self-loop (E_SELF_LOOP), its
    unordered pair appeared at an earlier index of the batch (E_DUP), or,
    for insertion, the edge exists (E_EXISTS) / for deletion, it does not
    (E_MISSING).  Checks apply in that order.  Strict mode rejects the whole
    batch and reports the smallest invalid index; filter mode drops invalid
    items.
    """

    def __init__(self, n: int, src, dst):
        self.n = int(n)
        self.alive = np.ones(self.n, dtype=np.uint8)
        self._base = np.unique(keys_of(src, dst))
        self._present = np.ones(self._base.size, dtype=bool)
        self._added = np.empty(0, dtype=np.int64)
        self._m = int(self._base.size)

    # -- queries --------------------------------------------------------
    @property
    def keys(self) -> np.ndarray:
        """Sorted canonical keys (min << 32 | max) of the current edges."""
        return np.sort(np.concatenate([self._base[self._present], self._added]))

    def edges(self):
        k = np.concatenate([self._base[self._present], self._added])
        return (k >> 32).astype(np.int32), (k & 0xFFFFFFFF).astype(np.int32)

    def num_edges(self):
        return self._m

    def cores(self) -> np.ndarray:
        s, d = self.edges()
        return bz_cores(self.n, s, d, self.alive)

    def _base_pos(self, keys):
        if self._base.size == 0:
            return np.zeros(keys.shape, dtype=np.int64), np.zeros(keys.shape, dtype=bool)
        p = np.minimum(np.searchsorted(self._base, keys), self._base.size - 1)
        return p, self._base[p] == keys

    def _added_pos(self, keys):
        if self._added.size == 0:
            return np.zeros(keys.shape, dtype=np.int64), np.zeros(keys.shape, dtype=bool)
        p = np.minimum(np.searchsorted(self._added, keys), self._added.size - 1)
        return p, self._added[p] == keys

    def has(self, keys):
        keys = np.asarray(keys, dtype=np.int64)
        p, hit = self._base_pos(keys)
        out = hit & self._present[p] if self._base.size else hit
        return out | self._added_pos(keys)[1]

    def _add_keys(self, keys):
        """Add distinct keys that are not edges."""
        p, hit = self._base_pos(keys)
        self._present[p[hit]] = True
        new = np.sort(keys[~hit])
        self._added = np.insert(self._added, np.searchsorted(self._added, new), new)
        self._m += int(keys.size)

    def _remove_keys(self, keys):
        """Remove distinct keys that are edges."""
        p, hit = self._base_pos(keys)
        hit &= self._present[p] if self._base.size else hit
        self._present[p[hit]] = False
        rest = keys[~hit]
        if rest.size:
            q, ok = self._added_pos(rest)
            assert ok.all()
            self._added = np.delete(self._added, q)
        self._m -= int(keys.size)

    # -- validation ----------------------------------------------------------
    def validate(self, src, dst, inserting: bool):
        """Per-item error code array (0 = valid) under the convention above."""
        src = np.asarray(src, dtype=np.int64)
        dst = np.asarray(dst, dtype=np.int64)
        err = np.zeros(src.size, dtype=np.int32)
        rng_bad = (src < 0) | (src >= self.n) | (dst < 0) | (dst >= self.n)
        err[rng_bad] = E_RANGE
        ok = err == 0
        dead = np.zeros(src.size, dtype=bool)
        dead[ok] = (self.alive[src[ok]] == 0) | (self.alive[dst[ok]] == 0)
        err[(err == 0) & dead] = E_DEAD
        err[(err == 0) & (src == dst)] = E_SELF_LOOP
        k = keys_of(src, dst)
        ok = err == 0
        idx = np.nonzero(ok)[0]
        _, first = np.unique(k[idx], return_index=True)
        is_first = np.zeros(src.size, dtype=bool)
        is_first[idx[first]] = True
        err[ok & ~is_first] = E_DUP
        ok = err == 0
        present = np.zeros(src.size, dtype=bool)
        present[ok] = self.has(k[ok])
        if inserting:
            err[ok & present] = E_EXISTS
        else:
            err[ok & ~present] = E_MISSING
        return err

    def _result(self, err, strict):
        bad = np.nonzero(err)[0]
        if strict and bad.size:
            return int(err[bad[0]]), int(bad[0])
        return OK, (int(bad[0]) if bad.size else -1)

    # -- updates -------------------------------------------------------------
    def insert_edges(self, src, dst, strict=True):
        """Returns (status, first_bad, applied)."""
        err = self.validate(src, dst, True)
        st, fb = self._result(err, strict)
        if st != OK:
            return st, fb, 0
        ok = err == 0
        self._add_keys(keys_of(np.asarray(src)[ok], np.asarray(dst)[ok]))
        return OK, fb, int(ok.sum())

    def delete_edges(self, src, dst, strict=True):
        err = self.validate(src, dst, False)
        st, fb = self._result(err, strict)
        if st != OK:
            return st, fb, 0
        ok = err == 0
        self._remove_keys(keys_of(np.asarray(src)[ok], np.asarray(dst)[ok]))
        return OK, fb, int(ok.sum())

    def insert_vertices(self, off, nbrs, strict=True, keep_failed_ids=False):
        """New ids n..n+c-1 (core 0), then the edges (new id, nbr) of each
        neighbour list.  Returns (status, first_bad, first_new_id).

        A rejected request frees its ids again, except with keep_failed_ids
        (the serving convention: ids are handed out at submission, so a
        rejected request's ids stay allocated as dead ids)."""
        off = np.asarray(off, dtype=np.int64)
        nbrs = np.asarray(nbrs, dtype=np.int64)
        c = off.size - 1
        first = self.n
        own = np.repeat(np.arange(first, first + c, dtype=np.int64), np.diff(off))
        saved = (self.n, self.alive)
        self.n = first + c
        self.alive = np.concatenate([self.alive, np.ones(c, dtype=np.uint8)])
        st, fb, _ = self.insert_edges(own, nbrs, strict)
        if st != OK:
            if keep_failed_ids:
                self.alive[first:first + c] = 0
                return st, fb, first
            self.n, self.alive = saved
            return st, fb, -1
        return OK, fb, first

    def delete_vertices(self, ids, strict=True):
        """Delete every edge incident to the ids, then mark them dead.
        Invalid items: out of range (E_RANGE), dead (E_DEAD), repeated (E_DUP).
        Returns (status, first_bad)."""
        ids = np.asarray(ids, dtype=np.int64)
        err = np.zeros(ids.size, dtype=np.int32)
        err[(ids < 0) | (ids >= self.n)] = E_RANGE
        ok = err == 0
        err[ok & (self.alive[np.where(ok, ids, 0)] == 0)] = E_DEAD
        ok = err == 0
        idx = np.nonzero(ok)[0]
        _, first = np.unique(ids[idx], return_index=True)
        is_first = np.zeros(ids.size, dtype=bool)
        is_first[idx[first]] = True
        err[ok & ~is_first] = E_DUP
        st, fb = self._result(err, strict)
        if st != OK:
            return st, fb
        dead = np.unique(ids[err == 0])
        if dead.size:
            self._remove_keys(self._incident_keys(dead))
            self.alive[dead] = 0
        return OK, fb

    def _incident_keys(self, dead):
        """Keys of the current edges with an endpoint in the sorted id array
        `dead`: (lo, hi) keys are sorted by lo, so the edges whose lo is a dead
        id are contiguous runs; for the hi side the initial keys keep an index
        sorted by hi (built once, the initial keys never change) and the later
        keys are few enough to test directly."""
        dead = np.asarray(dead, dtype=np.int64)
        mask = 0xFFFFFFFF

        def runs(sorted_vals, lo_vals, hi_vals):
            a = np.searchsorted(sorted_vals, lo_vals)
            b = np.searchsorted(sorted_vals, hi_vals)
            lens = b - a
            if lens.sum() == 0:
                return np.empty(0, dtype=np.int64)
            start = np.repeat(a - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
            return start + np.arange(lens.sum())

        parts = []
        if self._base.size:
            i = runs(self._base, dead << 32, (dead + 1) << 32)
            parts.append(self._base[i[self._present[i]]])
            if getattr(self, "_hi_order", None) is None:
                self._hi_order = np.argsort(self._base & mask, kind="stable")
                self._hi_sorted = (self._base & mask)[self._hi_order]
            j = self._hi_order[runs(self._hi_sorted, dead, dead + 1)]
            parts.append(self._base[j[self._present[j]]])
        if self._added.size:
            i = runs(self._added, dead << 32, (dead + 1) << 32)
            parts.append(self._added[i])
            parts.append(self._added[np.isin(self._added & mask, dead)])
        return np.unique(np.concatenate(parts)) if parts else np.empty(0, dtype=np.int64)


def all_graphs(n: int):
    """Every labelled simple graph on n vertices, as (src, dst) lists."""
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        s = [p[0] for i, p in enumerate(pairs) if mask >> i & 1]
        d = [p[1] for i, p in enumerate(pairs) if mask >> i & 1]
        yield np.asarray(s, dtype=np.int32), np.asarray(d, dtype=np.int32)
