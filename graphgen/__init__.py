"""Seeded synthetic graphs and update streams.

This module only draws random inputs: it holds none of the core-maintenance
arithmetic, and both the CPU oracle's tests and the GPU path consume what it
produces.  Every generator takes a ``numpy.random.Generator`` (PCG64) so that a
caller controls seeding; ``rng_for(tag)`` derives one child stream per named
workload from ``SeedSequence(0)``.

Edges are returned as two int32 arrays ``(src, dst)`` in canonical form
(``src < dst``), simple (no loops, no duplicates).  A graph on ``n`` vertices
uses ids ``0 .. n-1``.

The paper evaluates on SNAP datasets and on ER, BA and R-MAT graphs generated
by SNAP (Section VII, "Datasets"); none of those are available here, so these
generators stand in for them with the shapes the workloads name.
"""
from __future__ import annotations

import math
import zlib

import numpy as np

__all__ = [
    "rng_for", "keys_of", "split_keys", "er_graph", "chung_lu_graph",
    "rmat_graph", "ba_graph", "uniform_non_edges", "weighted_non_edges",
    "rmat_non_edges", "existing_edges", "log_uniform_sizes", "EdgeSet",
    "vertex_insert_payload", "power_law_degrees",
]


def rng_for(tag: str, seed: int = 0) -> np.random.Generator:
    """Child generator for a named workload: SeedSequence(seed) spawned by tag."""
    ss = np.random.SeedSequence([seed, zlib.crc32(tag.encode())])
    return np.random.Generator(np.random.PCG64(ss))


def keys_of(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Canonical int64 key (min << 32 | max) of each unordered pair."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    return (lo << 32) | hi


def split_keys(k: np.ndarray):
    k = np.asarray(k, dtype=np.int64)
    return (k >> 32).astype(np.int32), (k & 0xFFFFFFFF).astype(np.int32)


def _simple_keys(a, b):
    """Canonical keys of the pairs with loops removed, deduplicated (sorted)."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    keep = a != b
    return np.unique(keys_of(a[keep], b[keep]))


def er_graph(n: int, m: int, rng: np.random.Generator):
    """Erdos-Renyi G(n, m): m distinct unordered non-loop pairs, uniform."""
    if m > n * (n - 1) // 2:
        raise ValueError("m exceeds the number of pairs")
    keys = np.empty(0, dtype=np.int64)
    while keys.size < m:
        need = m - keys.size
        draw = int(need * 1.1) + 16
        a = rng.integers(0, n, draw)
        b = rng.integers(0, n, draw)
        new = _simple_keys(a, b)
        new = new[~np.isin(new, keys, assume_unique=True)]
        if new.size > need:
            new = rng.choice(new, need, replace=False)
        keys = np.union1d(keys, new)
    return split_keys(keys)


def _cl_weights(n: int, avg_deg: float, gamma: float, w_max: float):
    """Chung-Lu weights w_i = w_max (1 + i/i0)^(-1/(gamma-1)), i0 set so that
    sum(w) = n * avg_deg (found by bisection on i0)."""
    target = n * avg_deg
    i = np.arange(n, dtype=np.float64)
    expo = -1.0 / (gamma - 1.0)

    def total(i0):
        return float(np.sum(w_max * (1.0 + i / i0) ** expo))

    lo, hi = 1e-9, 1e12
    if total(hi) < target:  # even flat weights cannot reach the target
        return np.full(n, min(w_max, avg_deg))
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if total(mid) < target:
            lo = mid
        else:
            hi = mid
    return w_max * (1.0 + i / hi) ** expo


def chung_lu_graph(n: int, m: int, gamma: float, w_max: float,
                   rng: np.random.Generator):
    """Chung-Lu power-law graph with exactly m edges.

    Endpoint pairs are drawn with probability proportional to the weights;
    loops and duplicate pairs are dropped and the deficit is redrawn until m
    distinct edges exist.  Vertex ids are then relabelled by a random
    permutation so that id order carries no degree information.
    """
    w = _cl_weights(n, 2.0 * m / n, gamma, w_max)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    keys = np.empty(0, dtype=np.int64)
    while keys.size < m:
        need = m - keys.size
        draw = int(need * 1.15) + 64
        a = np.searchsorted(cdf, rng.random(draw), side="right")
        b = np.searchsorted(cdf, rng.random(draw), side="right")
        a = np.minimum(a, n - 1)
        b = np.minimum(b, n - 1)
        new = _simple_keys(a, b)
        new = new[~np.isin(new, keys, assume_unique=True)]
        if new.size > need:
            new = rng.choice(new, need, replace=False)
        keys = np.union1d(keys, new)
    s, d = split_keys(keys)
    perm = rng.permutation(n).astype(np.int64)
    return split_keys(np.unique(keys_of(perm[s], perm[d])))


def rmat_graph(scale: int, edge_factor: int, rng: np.random.Generator,
               a=0.57, b=0.19, c=0.19, relabel=True, chunk=1 << 24):
    """R-MAT: edge_factor * 2^scale pairs, each bit chosen with quadrant
    probabilities (a, b, c, d = 1-a-b-c); then canonicalised, deduplicated,
    loops dropped and (by default) relabelled by a random permutation."""
    n = 1 << scale
    total = edge_factor * n
    t1 = int(round(a * 65536))
    t2 = int(round((a + b) * 65536))
    t3 = int(round((a + b + c) * 65536))
    parts = []
    done = 0
    while done < total:
        cnt = min(chunk, total - done)
        u = np.zeros(cnt, dtype=np.int64)
        v = np.zeros(cnt, dtype=np.int64)
        for lvl in range(scale):
            r = rng.integers(0, 65536, cnt, dtype=np.int32)
            bit = np.int64(1) << lvl
            ub = r >= t2                      # quadrants c, d: row bit set
            vb = ((r >= t1) & (r < t2)) | (r >= t3)  # quadrants b, d: col bit set
            u |= ub.astype(np.int64) * bit
            v |= vb.astype(np.int64) * bit
        parts.append(_simple_keys(u, v))
        done += cnt
    keys = np.unique(np.concatenate(parts)) if len(parts) > 1 else parts[0]
    s, d = split_keys(keys)
    if relabel:
        perm = rng.permutation(n).astype(np.int64)
        keys = np.unique(keys_of(perm[s], perm[d]))
        s, d = split_keys(keys)
    return n, s, d


def ba_graph(n: int, k: int, rng: np.random.Generator):
    """Barabasi-Albert preferential attachment: each new vertex attaches k
    edges to distinct existing vertices chosen proportionally to degree
    (seeded by a (k+1)-clique)."""
    src, dst = [], []
    for i in range(k + 1):
        for j in range(i + 1, k + 1):
            src.append(i)
            dst.append(j)
    targets = list(src) + list(dst)  # endpoint multiset: degree-proportional
    for v in range(k + 1, n):
        chosen = set()
        while len(chosen) < k:
            chosen.add(targets[int(rng.integers(0, len(targets)))])
        for u in chosen:
            src.append(u)
            dst.append(v)
            targets.append(u)
            targets.append(v)
    return split_keys(np.unique(keys_of(np.array(src), np.array(dst))))


class EdgeSet:
    """Sorted canonical keys of a simple graph, for sampling updates that are
    valid against the current edge set (no method arithmetic)."""

    def __init__(self, src, dst):
        self.keys = np.unique(keys_of(src, dst))

    def __len__(self):
        return int(self.keys.size)

    def contains(self, keys):
        keys = np.asarray(keys, dtype=np.int64)
        if self.keys.size == 0:
            return np.zeros(keys.shape, dtype=bool)
        pos = np.searchsorted(self.keys, keys)
        pos = np.minimum(pos, self.keys.size - 1)
        return self.keys[pos] == keys

    def insert(self, src, dst):
        self.keys = np.union1d(self.keys, keys_of(src, dst))

    def delete(self, src, dst):
        self.keys = np.setdiff1d(self.keys, keys_of(src, dst), assume_unique=True)

    def edges(self):
        return split_keys(self.keys)


def _fresh_pairs(draw_fn, count, es: EdgeSet, rng):
    """Distinct non-loop pairs not in es, drawn by draw_fn(k) -> (a, b)."""
    got = np.empty(0, dtype=np.int64)
    stale = 0
    while got.size < count:
        need = count - got.size
        a, b = draw_fn(int(need * 1.2) + 16)
        new = _simple_keys(a, b)
        new = new[~es.contains(new)]
        new = new[~np.isin(new, got, assume_unique=True)]
        if new.size == 0:
            stale += 1
            if stale > 64:
                raise ValueError(f"could not draw {count} fresh pairs (got {got.size})")
            continue
        stale = 0
        if new.size > need:
            new = rng.choice(new, need, replace=False)
        got = np.union1d(got, new)
    got = rng.permutation(got)
    return split_keys(got)


def uniform_non_edges(n: int, count: int, es: EdgeSet, rng, lo: int = 0):
    """count distinct non-edges with both endpoints uniform on [lo, n)."""
    return _fresh_pairs(lambda k: (rng.integers(lo, n, k), rng.integers(lo, n, k)),
                        count, es, rng)


def weighted_non_edges(count: int, es: EdgeSet, rng):
    """count distinct non-edges whose endpoints are each the endpoint of a
    uniformly drawn existing edge (so endpoints are degree-weighted)."""
    s, d = es.edges()
    ends = np.concatenate([s, d])

    def draw(k):
        return ends[rng.integers(0, ends.size, k)], ends[rng.integers(0, ends.size, k)]
    return _fresh_pairs(draw, count, es, rng)


def rmat_non_edges(scale: int, count: int, es: EdgeSet, rng, perm=None,
                   a=0.57, b=0.19, c=0.19):
    """count distinct non-edges sampled from the R-MAT distribution (mapped
    through the same vertex relabelling as the graph when perm is given)."""
    t1 = int(round(a * 65536))
    t2 = int(round((a + b) * 65536))
    t3 = int(round((a + b + c) * 65536))

    def draw(k):
        u = np.zeros(k, dtype=np.int64)
        v = np.zeros(k, dtype=np.int64)
        for lvl in range(scale):
            r = rng.integers(0, 65536, k, dtype=np.int32)
            bit = np.int64(1) << lvl
            u |= (r >= t2).astype(np.int64) * bit
            v |= (((r >= t1) & (r < t2)) | (r >= t3)).astype(np.int64) * bit
        if perm is not None:
            u, v = perm[u], perm[v]
        return u, v
    return _fresh_pairs(draw, count, es, rng)


def existing_edges(count: int, es: EdgeSet, rng):
    """count distinct existing edges, uniform without replacement; each is
    returned in a random orientation."""
    count = min(count, len(es))
    idx = rng.choice(len(es), count, replace=False)
    s, d = split_keys(es.keys[idx])
    flip = rng.random(count) < 0.5
    return np.where(flip, d, s).astype(np.int32), np.where(flip, s, d).astype(np.int32)


def log_uniform_sizes(count: int, lo: float, hi: float, rng):
    """Sizes round(exp(U[ln lo, ln hi]))."""
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), count))).astype(np.int64)


def power_law_degrees(count: int, lo: int, hi: int, exponent: float, rng):
    """Discrete power law P(d) ~ d^-exponent on [lo, hi]."""
    d = np.arange(lo, hi + 1, dtype=np.float64)
    p = d ** (-exponent)
    p /= p.sum()
    return rng.choice(np.arange(lo, hi + 1), count, p=p).astype(np.int64)


def vertex_insert_payload(first_new: int, count: int, degrees, es: EdgeSet, rng):
    """Neighbour lists for `count` new vertices with ids first_new.. (CSR
    offsets int64[count+1], nbrs int32).  Neighbours are degree-weighted
    existing vertices, distinct per new vertex."""
    s, d = es.edges()
    ends = np.concatenate([s, d])
    offs = [0]
    nbrs = []
    for i in range(count):
        want = int(degrees[i])
        picked = np.unique(ends[rng.integers(0, ends.size, want * 2 + 4)])[:want] \
            if ends.size else np.empty(0, dtype=np.int32)
        nbrs.append(picked.astype(np.int32))
        offs.append(offs[-1] + picked.size)
    return np.asarray(offs, dtype=np.int64), (np.concatenate(nbrs) if nbrs else
                                               np.empty(0, dtype=np.int32))
