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
    "rmat_non_edges", "existing_edges", "log_uniform_sizes", "EdgeSet", "DynamicEdgeSet",
    "vertex_insert_payload", "power_law_degrees", "rmat_stream", "chung_lu_pool", "StreamEdgeSet", "serve_stream", "ba_graph_blocks",
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


def _rmat_chunk(args):
    """Canonical unique keys of `cnt` R-MAT pairs drawn from a child seed."""
    seed, cnt, scale, t1, t2, t3 = args
    rng = np.random.Generator(np.random.PCG64(seed))
    u = np.zeros(cnt, dtype=np.int64)
    v = np.zeros(cnt, dtype=np.int64)
    for lvl in range(scale):
        r = rng.integers(0, 65536, cnt, dtype=np.int32)
        bit = np.int64(1) << lvl
        ub = r >= t2                      # quadrants c, d: row bit set
        vb = ((r >= t1) & (r < t2)) | (r >= t3)  # quadrants b, d: col bit set
        u |= ub.astype(np.int64) * bit
        v |= vb.astype(np.int64) * bit
    return np.unique(_simple_keys(u, v))


def rmat_graph(scale: int, edge_factor: int, rng: np.random.Generator,
               a=0.57, b=0.19, c=0.19, relabel=True, chunk=1 << 22, workers=1):
    """R-MAT: edge_factor * 2^scale pairs, each bit chosen with quadrant
    probabilities (a, b, c, d = 1-a-b-c); then canonicalised, deduplicated,
    loops dropped and (by default) relabelled by a random permutation.

    The pairs are drawn in chunks, each from its own child seed taken from
    `rng`, so the graph does not depend on `workers` (processes used to draw
    the chunks)."""
    n = 1 << scale
    total = edge_factor * n
    t1 = int(round(a * 65536))
    t2 = int(round((a + b) * 65536))
    t3 = int(round((a + b + c) * 65536))
    nchunks = (total + chunk - 1) // chunk
    seeds = rng.integers(0, 2 ** 63 - 1, nchunks, dtype=np.int64)
    jobs = [(int(seeds[i]), min(chunk, total - i * chunk), scale, t1, t2, t3) for i in range(nchunks)]
    if workers > 1 and nchunks > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=workers) as ex:
            parts = list(ex.map(_rmat_chunk, jobs))
    else:
        parts = [_rmat_chunk(j) for j in jobs]
    keys = np.unique(np.concatenate(parts))
    del parts
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


class DynamicEdgeSet:
    """Edge set for long update streams on large graphs: the initial keys stay
    in one sorted array with an alive mask; keys inserted later live in a
    small sorted side array.  Same queries as EdgeSet, without re-sorting
    the whole set on every batch."""

    def __init__(self, src, dst):
        self.base = np.unique(keys_of(src, dst))
        self.alive = np.ones(self.base.size, dtype=bool)
        self.n_alive = int(self.base.size)
        self.added = np.empty(0, dtype=np.int64)

    def __len__(self):
        return self.n_alive + int(self.added.size)

    def _base_pos(self, keys):
        pos = np.minimum(np.searchsorted(self.base, keys), max(self.base.size - 1, 0))
        hit = self.base[pos] == keys if self.base.size else np.zeros(keys.shape, dtype=bool)
        return pos, hit

    def contains(self, keys):
        keys = np.asarray(keys, dtype=np.int64)
        pos, hit = self._base_pos(keys)
        out = hit & self.alive[pos] if self.base.size else hit
        if self.added.size:
            p2 = np.minimum(np.searchsorted(self.added, keys), self.added.size - 1)
            out |= self.added[p2] == keys
        return out

    def insert(self, src, dst):
        keys = keys_of(src, dst)
        pos, hit = self._base_pos(keys)
        revive = pos[hit]
        self.n_alive += int((~self.alive[revive]).sum())
        self.alive[revive] = True
        self.added = np.union1d(self.added, keys[~hit])

    def delete(self, src, dst):
        keys = keys_of(src, dst)
        pos, hit = self._base_pos(keys)
        kill = pos[hit]
        self.n_alive -= int(self.alive[kill].sum())
        self.alive[kill] = False
        self.added = np.setdiff1d(self.added, keys[~hit], assume_unique=True)

    def edges(self):
        return split_keys(np.concatenate([self.base[self.alive], self.added]))

    def sample_keys(self, count, rng):
        """count distinct present keys, uniform without replacement."""
        count = min(count, len(self))
        idx = rng.choice(len(self), count, replace=False)
        live = np.flatnonzero(self.alive)
        in_base = idx < live.size
        out = np.empty(count, dtype=np.int64)
        out[in_base] = self.base[live[idx[in_base]]]
        out[~in_base] = self.added[idx[~in_base] - live.size]
        return out


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
    if isinstance(es, DynamicEdgeSet):
        s, d = split_keys(es.sample_keys(count, rng))
    else:
        idx = rng.choice(len(es), count, replace=False)
        s, d = split_keys(es.keys[idx])
    flip = rng.random(count) < 0.5
    return np.where(flip, d, s).astype(np.int32), np.where(flip, s, d).astype(np.int32)


def edge_levels(s, d, cores):
    """Core number of each edge: the smaller core number of its endpoints
    (`cores` is an input here, computed by whoever calls)."""
    cores = np.asarray(cores)
    return np.minimum(cores[s], cores[d])


def typical_levels(s, d, cores, count=5):
    """Up to `count` distinct edge core numbers in increasing order, taken
    at the quantiles (i + 1/2) / count of the edge core distribution, so
    that each stands for an equal share of the edges."""
    ec = edge_levels(s, d, cores)
    if ec.size == 0:
        return []
    q = (np.arange(count) + 0.5) / count
    return sorted({int(x) for x in np.quantile(ec, q, method="lower")})


def edges_at_level(s, d, cores, level, frac, rng):
    """A uniform random share `frac` (rounded, at least one when any exist)
    of the edges whose core number equals `level`, without replacement."""
    idx = np.flatnonzero(edge_levels(s, d, cores) == level)
    if idx.size == 0:
        return s[:0].copy(), d[:0].copy()
    cnt = max(1, int(round(frac * idx.size)))
    pick = np.sort(rng.choice(idx, cnt, replace=False))
    return s[pick].astype(np.int32), d[pick].astype(np.int32)


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


# ---------------------------------------------------------------------------
# Workload recipes (graph + update stream), shared by the benchmark and the
# scaled-down parity tests.
# ---------------------------------------------------------------------------

def rmat_stream(scale: int, nbatches: int, lo: int, hi: int, rng, edge_factor=16, workers=1,
                progress=None):
    """R-MAT graph plus a stream of `nbatches` batches, sizes log-uniform in
    [lo, hi], half insertions (R-MAT-sampled non-edges) and half deletions
    (uniform existing edges at that moment), in shuffled order.

    Returns (n, src, dst, kinds int32[nb] (0 insert, 1 delete),
    offsets int64[nb+1], xs int32[total], ys int32[total])."""
    n, s, d = rmat_graph(scale, edge_factor, rng, workers=workers)
    if progress:
        progress(f"r-mat scale {scale}: {s.size} edges")
    perm_rng = rng
    # the relabel permutation is not kept by rmat_graph: inserts are drawn
    # from the same R-MAT distribution under a fresh random relabel
    perm = perm_rng.permutation(n).astype(np.int64)
    es = DynamicEdgeSet(s, d)
    sizes = log_uniform_sizes(nbatches, lo, hi, rng)
    kinds = rng.permutation(np.arange(nbatches) % 2).astype(np.int32)
    xs, ys = [], []
    for j in range(nbatches):
        if kinds[j] == 0:
            a, b = rmat_non_edges(scale, int(sizes[j]), es, rng, perm=perm)
            es.insert(a, b)
        else:
            a, b = existing_edges(int(sizes[j]), es, rng)
            es.delete(a, b)
        xs.append(np.asarray(a, np.int32))
        ys.append(np.asarray(b, np.int32))
        if progress and (j + 1) % 16 == 0:
            progress(f"stream: {j + 1}/{nbatches} batches")
    offs = np.concatenate([[0], np.cumsum([x.size for x in xs])]).astype(np.int64)
    return n, s, d, kinds, offs, np.concatenate(xs), np.concatenate(ys)


def _pool_member(args):
    seed, nlo, nhi, dlo, dhi, gamma, wratio, frac = args
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(np.rint(np.exp(rng.uniform(math.log(nlo), math.log(nhi)))))
    deg = rng.uniform(dlo, dhi)
    m = int(round(n * deg / 2))
    s, d = chung_lu_graph(n, m, gamma, wratio * n, rng)
    es = EdgeSet(s, d)
    k = max(1, int(round(frac * m)))
    a, b = weighted_non_edges(k, es, rng)
    es.insert(a, b)
    x, y = existing_edges(k, es, rng)
    return n, s, d, (a, b), (x, y)


def chung_lu_pool(count: int, rng, nlo=1000, nhi=200_000, dlo=4.0, dhi=32.0, gamma=2.3,
                  wratio=0.05, frac=0.05, workers=1):
    """`count` independent Chung-Lu graphs: n log-uniform in [nlo, nhi], mean
    degree uniform in [dlo, dhi], largest weight wratio * n; each with one
    insertion batch (frac * m degree-weighted non-edges) and then one deletion
    batch (frac * m uniform existing edges).  Each member is drawn from its
    own child seed, so the result does not depend on `workers`.

    Returns a list of (n, src, dst, (ins_src, ins_dst), (del_src, del_dst))."""
    seeds = rng.integers(0, 2 ** 63 - 1, count, dtype=np.int64)
    jobs = [(int(sd), nlo, nhi, dlo, dhi, gamma, wratio, frac) for sd in seeds]
    if workers > 1 and count > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=workers) as ex:
            return list(ex.map(_pool_member, jobs, chunksize=4))
    return [_pool_member(j) for j in jobs]


class StreamEdgeSet:
    """Edge and vertex state for long mixed request streams on large graphs.

    Edges: the initial keys (sorted, with an alive mask) plus two sorted
    levels of inserted keys (a small recent level merged into a larger one
    when it grows), each with a validity mask, so that an insertion or
    deletion costs O(batch log m) and only the occasional merge touches the
    whole inserted level.  Vertices: an alive mask over the ids handed out;
    a deleted vertex's edges are not removed eagerly -- they are skipped
    (and dropped) when sampled, and their endpoints are never drawn again."""

    def __init__(self, n, src, dst):
        self.n = int(n)
        self.valive = np.ones(self.n, dtype=bool)
        self.base = np.unique(keys_of(src, dst))
        self.base_ok = np.ones(self.base.size, dtype=bool)
        self.lv = [np.empty(0, np.int64), np.empty(0, np.int64)]   # big, recent
        self.lv_ok = [np.empty(0, bool), np.empty(0, bool)]

    @staticmethod
    def _find(arr, keys):
        if arr.size == 0:
            return np.zeros(keys.size, np.int64), np.zeros(keys.size, bool)
        # sorted needles keep the binary searches cache-friendly on large arrays
        order = np.argsort(keys, kind="stable")
        pos = np.empty(keys.size, np.int64)
        pos[order] = np.searchsorted(arr, keys[order])
        pos = np.minimum(pos, arr.size - 1)
        return pos, arr[pos] == keys

    def contains(self, keys):
        keys = np.asarray(keys, dtype=np.int64)
        pos, hit = self._find(self.base, keys)
        out = hit & self.base_ok[pos]
        for a, ok in zip(self.lv, self.lv_ok):
            p, h = self._find(a, keys)
            if a.size:
                out |= h & ok[p]
        return out

    def _merge(self):
        a = np.concatenate([self.lv[0][self.lv_ok[0]], self.lv[1][self.lv_ok[1]]])
        a.sort()
        self.lv = [a, np.empty(0, np.int64)]
        self.lv_ok = [np.ones(a.size, bool), np.empty(0, bool)]

    def insert_keys(self, keys):
        keys = np.asarray(keys, dtype=np.int64)
        pos, hit = self._find(self.base, keys)
        self.base_ok[pos[hit]] = True
        rest = keys[~hit]
        for i in (0, 1):
            p, h = self._find(self.lv[i], rest)
            if self.lv[i].size:
                self.lv_ok[i][p[h]] = True
                rest = rest[~h]
        if rest.size:
            rest = np.unique(rest)
            at = np.searchsorted(self.lv[1], rest)
            self.lv[1] = np.insert(self.lv[1], at, rest)
            self.lv_ok[1] = np.insert(self.lv_ok[1], at, True)
        if self.lv[1].size > max(1 << 20, self.lv[0].size // 8):
            self._merge()

    def delete_keys(self, keys):
        keys = np.asarray(keys, dtype=np.int64)
        pos, hit = self._find(self.base, keys)
        self.base_ok[pos[hit]] = False
        for i in (0, 1):
            p, h = self._find(self.lv[i], keys)
            if self.lv[i].size:
                self.lv_ok[i][p[h]] = False

    def new_vertices(self, c):
        first = self.n
        self.n += int(c)
        self.valive = np.concatenate([self.valive, np.ones(int(c), dtype=bool)])
        return first

    def delete_vertices(self, ids):
        self.valive[np.asarray(ids, dtype=np.int64)] = False

    def sample_edges(self, count, rng):
        """Up to `count` distinct present edges between live vertices, uniform
        (rejection over all stored keys); fewer only if too few remain."""
        sizes = [self.base.size, self.lv[0].size, self.lv[1].size]
        total = sum(sizes)
        got = np.empty(0, np.int64)
        tries = 0
        acc = getattr(self, "_acc", 1.0)   # acceptance seen by the last draw
        while got.size < count and total > 0 and tries < 64:
            tries += 1
            k = int((count - got.size) * 1.3 / max(acc, 0.02)) + 16
            idx = rng.integers(0, total, k)
            keys = np.empty(k, np.int64)
            ok = np.empty(k, bool)
            lo = 0
            for arr, okm in zip([self.base] + self.lv, [self.base_ok] + self.lv_ok):
                sel = (idx >= lo) & (idx < lo + arr.size)
                keys[sel] = arr[idx[sel] - lo]
                ok[sel] = okm[idx[sel] - lo]
                lo += arr.size
            u, v = keys >> 32, keys & 0xFFFFFFFF
            dead_end = ~(self.valive[u] & self.valive[v])
            stale = ok & dead_end
            if stale.any():   # edges of deleted vertices are gone: drop them now
                self.delete_keys(keys[stale])
            keys = keys[ok & ~dead_end]
            acc = max(keys.size / k, 0.02)
            self._acc = acc
            keys = np.setdiff1d(np.unique(keys), got, assume_unique=True)
            if keys.size > count - got.size:
                keys = rng.choice(keys, count - got.size, replace=False)
            got = np.concatenate([got, keys])
        return got

    def sample_vertices(self, count, rng):
        """Up to `count` distinct live ids, uniform."""
        got = np.empty(0, np.int64)
        tries = 0
        live = max(float(self.valive.mean()), 0.02) if self.n else 1.0
        while got.size < count and tries < 64:
            tries += 1
            k = int((count - got.size) * 1.3 / live) + 16
            ids = rng.integers(0, self.n, k)
            ids = np.setdiff1d(np.unique(ids[self.valive[ids]]), got, assume_unique=True)
            if ids.size > count - got.size:
                ids = rng.choice(ids, count - got.size, replace=False)
            got = np.concatenate([got, ids])
        return got


def serve_stream(scale, nreq, rng, edge_factor=16, max_size=100_000, mix=(0.4, 0.4, 0.1, 0.1),
                 deg_lo=1, deg_hi=1000, deg_exp=2.1, workers=1, graph=None, progress=None):
    # graph=(n, src, dst) serves a given graph instead of an R-MAT one; its
    # insertions then draw uniform pairs of live ids
    """R-MAT graph plus a stream of `nreq` serving requests, sizes
    round(exp U[0, ln max_size]): edge insertions (R-MAT-sampled non-edges
    between live vertices), edge deletions (uniform present edges), vertex
    insertions (s new vertices, degrees from a discrete power law on
    [deg_lo, deg_hi], degree-weighted live neighbours, distinct per vertex)
    and vertex deletions (s uniform live vertices), chosen by `mix`.

    Returns (n, src, dst, requests) with requests as ("ins", src, dst),
    ("del", src, dst), ("vins", off int64[c+1], nbrs) or ("vdel", ids); every
    request is valid against the state the earlier ones leave (ids of
    vertex insertions are assigned in request order from n)."""
    if graph is None:
        n, s, d = rmat_graph(scale, edge_factor, rng, workers=workers)
    else:
        n, s, d = graph
    if progress:
        progress(f"graph: n={n} m={s.size}")
    st = StreamEdgeSet(n, s, d)
    perm = rng.permutation(n).astype(np.int64)
    t1, t2, t3 = int(round(0.57 * 65536)), int(round(0.76 * 65536)), int(round(0.95 * 65536))
    sizes = np.maximum(1, np.rint(np.exp(rng.uniform(0.0, math.log(max_size), nreq)))).astype(np.int64)
    kinds = rng.choice(4, nreq, p=np.asarray(mix) / np.sum(mix))
    reqs = []
    ins_acc = 1.0

    def rmat_pairs(k):
        if graph is not None:
            return rng.integers(0, st.n, k), rng.integers(0, st.n, k)
        u = np.zeros(k, np.int64)
        v = np.zeros(k, np.int64)
        for lvl in range(scale):
            r = rng.integers(0, 65536, k, dtype=np.int32)
            bit = np.int64(1) << lvl
            u |= (r >= t2).astype(np.int64) * bit
            v |= (((r >= t1) & (r < t2)) | (r >= t3)).astype(np.int64) * bit
        return perm[u], perm[v]

    for j in range(nreq):
        k, size = int(kinds[j]), int(sizes[j])
        if k == 0:
            got = np.empty(0, np.int64)
            for _ in range(64):
                if got.size >= size:
                    break
                draw = int((size - got.size) * 1.3 / ins_acc) + 16
                a, b = rmat_pairs(draw)
                keep = (a != b) & st.valive[a] & st.valive[b]
                keys = np.unique(keys_of(a[keep], b[keep]))
                keys = keys[~st.contains(keys)]
                ins_acc = max(keys.size / draw, 0.02)
                keys = np.setdiff1d(keys, got, assume_unique=True)
                if keys.size > size - got.size:
                    keys = rng.choice(keys, size - got.size, replace=False)
                got = np.concatenate([got, keys])
            got = rng.permutation(got)
            st.insert_keys(got)
            a, b = split_keys(got)
            reqs.append(("ins", a, b))
        elif k == 1:
            keys = st.sample_edges(size, rng)
            st.delete_keys(keys)
            a, b = split_keys(keys)
            flip = rng.random(keys.size) < 0.5
            reqs.append(("del", np.where(flip, b, a).astype(np.int32), np.where(flip, a, b).astype(np.int32)))
        elif k == 2:
            degs = power_law_degrees(size, deg_lo, deg_hi, deg_exp, rng)
            first = st.new_vertices(size)
            ends = st.sample_edges(int(degs.sum() * 1.5) + 16, rng)
            pool = np.concatenate([ends >> 32, ends & 0xFFFFFFFF])
            if pool.size == 0:
                pool = np.flatnonzero(st.valive[:first])
            if pool.size == 0:   # nothing left to attach to: isolated new vertices
                degs = np.zeros(size, np.int64)
                pool = np.zeros(1, np.int64)
            own = np.repeat(np.arange(size, dtype=np.int64), degs)
            nb = pool[rng.integers(0, pool.size, own.size)]
            pair = np.unique(own * (1 << 32) + nb)   # distinct per new vertex
            own, nb = pair >> 32, pair & 0xFFFFFFFF
            off = np.zeros(size + 1, np.int64)
            np.add.at(off, own + 1, 1)
            off = np.cumsum(off)
            st.insert_keys(keys_of(own + first, nb))
            reqs.append(("vins", off, nb.astype(np.int32)))
        else:
            ids = st.sample_vertices(size, rng)
            st.delete_vertices(ids)
            reqs.append(("vdel", rng.permutation(ids).astype(np.int32)))
        if progress and (j + 1) % 1000 == 0:
            progress(f"requests: {j + 1}/{nreq}")
    return n, s, d, reqs


def ba_graph_blocks(n: int, k: int, rng, block: int = 4096):
    """Preferential attachment (Barabasi-Albert) for large n, drawn in blocks:
    every vertex of a block attaches up to k edges to distinct earlier
    vertices, each chosen with probability proportional to its degree in the
    graph as it stood before the block (a block is never larger than the
    graph before it; the seed is a (k+1)-clique).  A vertex whose 3k degree-
    weighted draws hold fewer than k distinct targets keeps fewer edges."""
    k0 = k + 1
    cs, cd = np.triu_indices(k0, 1)
    ends = np.empty(2 * (cs.size + k * max(n - k0, 0)), dtype=np.int64)
    ends[: 2 * cs.size] = np.concatenate([cs, cd])
    ne = 2 * cs.size
    srcs, dsts = [cs.astype(np.int64)], [cd.astype(np.int64)]
    v0 = k0
    while v0 < n:
        b = min(block, n - v0, v0)
        cand = ends[rng.integers(0, ne, (b, 3 * k))]
        cand.sort(axis=1)
        dup = np.zeros_like(cand, dtype=bool)
        dup[:, 1:] = cand[:, 1:] == cand[:, :-1]
        # first k distinct targets per row, in a random order of the row
        keyed = np.where(dup, np.iinfo(np.int64).max, rng.integers(0, 1 << 40, cand.shape))
        order = np.argsort(keyed, axis=1)[:, :k]
        pick = np.take_along_axis(cand, order, axis=1)
        ok = ~np.take_along_axis(dup, order, axis=1)
        own = np.repeat(np.arange(v0, v0 + b, dtype=np.int64), k).reshape(b, k)
        s_new, d_new = pick[ok], own[ok]
        srcs.append(s_new)
        dsts.append(d_new)
        cnt = s_new.size
        ends[ne:ne + cnt] = s_new
        ends[ne + cnt:ne + 2 * cnt] = d_new
        ne += 2 * cnt
        v0 += b
    return split_keys(np.unique(keys_of(np.concatenate(srcs), np.concatenate(dsts))))
