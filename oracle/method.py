"""The paper's iterative core-maintenance algorithms, sequential and plain --
TEST INFRASTRUCTURE ONLY (part of the oracle; shares nothing with the GPU path).

Written from the paper's description of the method (Section IV definitions,
Section V incremental, Section VI decremental), in the paper's notation, for
tiny graphs stored as ``dict[int, set[int]]``.  Its purpose is to pin the
paper's lemmas and the readings this project takes where the text is silent or
inconsistent; the final core numbers it produces must equal a from-scratch
decomposition (``oracle.bz_cores``) after every batch.

Readings taken (each is also listed in the design notes):

* Superior-edge-set selection.  Definition of the k-superior edge set forbids
  two of its edges from sharing an endpoint whose core is k.  The
  per-vertex selection of ComputeSuperiorEdgeSet (Algorithm 2) can break that
  rule when an edge joins two core-k vertices (each may pick a different edge
  through the other).  Read: an edge is selected only if every endpoint whose
  core equals the edge's core number is still free at that level; the scan
  order is the order of the remaining batch.
* The level set C is recomputed in every iteration (the decremental driver
  says so explicitly; the incremental driver is read the same way).
* In the incremental per-level routine the root's counter is set with
  cd += CSD in both branches (an unvisited counter is always <= 0).
* Decremental eviction test is "cd < k" (Algorithms 6 and 7), not the
  "SD <= k" of the lemma on superior degree: with "<=", a vertex that keeps
  exactly k supporters would be dropped wrongly (theta-graph pin).
* SD and CSD are evaluated on the graph with the current superior edge set
  already applied (inserted / deleted), with the pre-iteration core numbers.
"""
from __future__ import annotations

from typing import Dict, List, Set, Tuple

Graph = Dict[int, Set[int]]


def sd(G: Graph, core: Dict[int, int], u: int) -> int:
    """Superior degree: neighbours w with core(w) >= core(u)."""
    return sum(1 for w in G[u] if core[w] >= core[u])


def csd(G: Graph, core: Dict[int, int], u: int) -> int:
    """Constraint superior degree: neighbours w with core(w) > core(u), or
    core(w) == core(u) and SD(w) > core(u)."""
    k = core[u]
    return sum(1 for w in G[u]
               if core[w] > k or (core[w] == k and sd(G, core, w) > k))


def superior_edge_set(edges: List[Tuple[int, int]], core: Dict[int, int]):
    """Split the remaining edges into (selected superior edge set, rest).

    An edge <u, v> has core number k = min(core u, core v); it is superior for
    every endpoint whose core is k.  At most one selected edge may touch a
    core-k endpoint at level k (Definition of the k-superior edge set (ii));
    edges of different levels may share vertices (union of k-sets).
    """
    used: Set[int] = set()  # vertices already holding a selected edge at their level
    chosen, rest = [], []
    for (u, v) in edges:
        k = min(core[u], core[v])
        ends = [x for x in (u, v) if core[x] == k]
        if all(x not in used for x in ends):
            used.update(ends)
            chosen.append((u, v))
        else:
            rest.append((u, v))
    return chosen, rest


def _insert_level(G: Graph, Ek, core, k):
    """K-SuperiorInsert for one level: positive DFS from the roots over core-k
    vertices with SD > k, negative DFS (InsertRemove) evicting vertices whose
    counter falls to k.  Returns the vertices that rise to k+1."""
    visited: Set[int] = set()
    removed: Set[int] = set()
    cd: Dict[int, int] = {}

    def insert_remove(r):
        stack = [r]
        removed.add(r)
        while stack:
            v = stack.pop()
            for w in G[v]:
                if core[w] == k:
                    cd[w] = cd.get(w, 0) - 1
                    if cd[w] == k and w not in removed:
                        stack.append(w)
                        removed.add(w)

    for (u, v) in Ek:
        r = u if core[u] == k else v
        if r in visited or r in removed:
            continue
        cd[r] = cd.get(r, 0) + csd(G, core, r)
        stack = [r]
        visited.add(r)
        while stack:
            x = stack.pop()
            if cd[x] > k:
                for w in G[x]:
                    if core[w] == k and w not in visited and sd(G, core, w) > k:
                        stack.append(w)
                        visited.add(w)
                        cd[w] = cd.get(w, 0) + csd(G, core, w)
            elif x not in removed:
                insert_remove(x)
    return {x for x in visited if x not in removed}


def _delete_level(G: Graph, Ek, core, k, le=False):
    """K-SuperiorDelete for one level: counters start at SD on the graph
    without the deleted edges; a vertex whose counter is below k is peeled
    (DeleteRemove) and lowers its core-k neighbours' counters in cascade.
    Returns the vertices that fall to k-1."""
    visited: Set[int] = set()
    removed: Set[int] = set()
    cd: Dict[int, int] = {}

    def below(c):
        return c <= k if le else c < k

    def delete_remove(r):
        stack = [r]
        removed.add(r)
        while stack:
            v = stack.pop()
            for w in G[v]:
                if core[w] != k:
                    continue
                if w not in visited:
                    visited.add(w)
                    cd[w] = cd.get(w, 0) + sd(G, core, w)
                cd[w] -= 1
                if below(cd[w]) and w not in removed:
                    stack.append(w)
                    removed.add(w)

    def check_root(r):
        if r not in visited:
            visited.add(r)
            cd[r] = sd(G, core, r)
        if r not in removed and below(cd[r]):
            delete_remove(r)

    for (u, v) in Ek:
        if core[u] != core[v]:
            check_root(u if core[u] < core[v] else v)
        else:
            check_root(u)
            check_root(v)
    return {x for x in removed if x in visited}


def insert_edges(G: Graph, core: Dict[int, int], edges, trace=None):
    """SuperiorEdgeInsert: repeat {select a superior edge set; insert it;
    find the rising vertices of every level; +1} until no edge remains.
    Mutates G and core.  Returns the number of iterations."""
    rest = list(edges)
    it = 0
    while rest:
        chosen, rest = superior_edge_set(rest, core)
        for (u, v) in chosen:
            G[u].add(v)
            G[v].add(u)
        levels: Dict[int, list] = {}
        for (u, v) in chosen:
            levels.setdefault(min(core[u], core[v]), []).append((u, v))
        rise = set()
        for k, Ek in levels.items():  # independent per level
            rise |= _insert_level(G, Ek, core, k)
        for x in rise:
            core[x] += 1
        it += 1
        if trace is not None:
            trace.append((list(chosen), dict(core)))
    return it


def delete_edges(G: Graph, core: Dict[int, int], edges, threshold_le=False, trace=None):
    """SuperiorEdgeDelete: same loop with deletion and -1.  threshold_le=True
    swaps the eviction test to the lemma's "SD <= k" (used only to show that
    reading is wrong)."""
    rest = list(edges)
    it = 0
    while rest:
        chosen, rest = superior_edge_set(rest, core)
        for (u, v) in chosen:
            G[u].discard(v)
            G[v].discard(u)
        levels: Dict[int, list] = {}
        for (u, v) in chosen:
            levels.setdefault(min(core[u], core[v]), []).append((u, v))
        fall = set()
        for k, Ek in levels.items():
            fall |= _delete_level(G, Ek, core, k, le=threshold_le)
        for x in fall:
            core[x] -= 1
        it += 1
        if trace is not None:
            trace.append((list(chosen), dict(core)))
    return it


def graph_from_edges(n, src, dst) -> Graph:
    G: Graph = {v: set() for v in range(n)}
    for a, b in zip(list(src), list(dst)):
        G[int(a)].add(int(b))
        G[int(b)].add(int(a))
    return G
