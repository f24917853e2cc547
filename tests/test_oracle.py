"""Pins of the CPU oracle against facts fixed outside it: the definition
(brute force), an independent library (networkx), closed forms, and
hand-derived fixtures.  CPU only."""
import itertools

import numpy as np
import pytest

import graphgen
from tests.golden import cases as golden


def _nx_cores(n, s, d):
    nx = pytest.importorskip("networkx")
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from(zip(s.tolist(), d.tolist()))
    c = nx.core_number(G)
    return np.asarray([c[v] for v in range(n)], dtype=np.int32)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_all_labelled_graphs_small(oracle_mod, n):
    for s, d in oracle_mod.all_graphs(n):
        b = oracle_mod.brute_cores(n, s, d)
        z = oracle_mod.bz_cores(n, s, d)
        p = oracle_mod.peel_cores(n, s, d)
        assert np.array_equal(b, z), (s, d, b, z)
        assert np.array_equal(b, p), (s, d, b, p)


def test_random_tiny_graphs_brute(oracle_mod):
    rng = np.random.default_rng(1)
    for _ in range(40):
        n = int(rng.integers(6, 13))
        pairs = list(itertools.combinations(range(n), 2))
        keep = rng.random(len(pairs)) < rng.uniform(0.1, 0.7)
        s = np.asarray([p[0] for p, k in zip(pairs, keep) if k], dtype=np.int32)
        d = np.asarray([p[1] for p, k in zip(pairs, keep) if k], dtype=np.int32)
        assert np.array_equal(oracle_mod.brute_cores(n, s, d), oracle_mod.bz_cores(n, s, d))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bz_vs_networkx(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    n = 2000
    for gen in ("er", "cl"):
        if gen == "er":
            s, d = graphgen.er_graph(n, 8000, rng)
        else:
            s, d = graphgen.chung_lu_graph(n, 10000, 2.1, 300.0, rng)
        assert np.array_equal(_nx_cores(n, s, d), oracle_mod.bz_cores(n, s, d))
        assert np.array_equal(oracle_mod.peel_cores(n, s, d), oracle_mod.bz_cores(n, s, d))


def _edges(pairs):
    return (np.asarray([a for a, _ in pairs], dtype=np.int32),
            np.asarray([b for _, b in pairs], dtype=np.int32))


def test_closed_forms(oracle_mod):
    bz = oracle_mod.bz_cores
    # complete graph K_n -> n-1
    for n in (2, 3, 7, 20):
        s, d = _edges(list(itertools.combinations(range(n), 2)))
        assert (bz(n, s, d) == n - 1).all()
    # cycle C_n -> 2
    for n in (3, 10, 101):
        s, d = _edges([(i, (i + 1) % n) for i in range(n)])
        assert (bz(n, s, d) == 2).all()
    # random tree (plus isolated vertices) -> 1 (isolated -> 0)
    rng = np.random.default_rng(3)
    n = 500
    s, d = _edges([(int(rng.integers(0, i)), i) for i in range(1, 400)])
    c = bz(n, s, d)
    assert (c[:400] == 1).all() and (c[400:] == 0).all()
    # complete bipartite K_{a,b} -> min(a, b)
    for a, b in ((1, 5), (3, 4), (6, 6), (2, 9)):
        s, d = _edges([(i, a + j) for i in range(a) for j in range(b)])
        assert (bz(a + b, s, d) == min(a, b)).all()
    # Petersen graph (3-regular) -> 3
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    s, d = _edges(outer + spokes + inner)
    assert (bz(10, s, d) == 3).all()
    # wheel with r >= 4 rim vertices -> 3
    for r in (4, 5, 12):
        s, d = _edges([(0, i) for i in range(1, r + 1)] +
                      [(i, i % r + 1) for i in range(1, r + 1)])
        assert (bz(r + 1, s, d) == 3).all()
    # grid P_a x P_b -> 2
    a, b = 7, 9
    pairs = []
    for i in range(a):
        for j in range(b):
            v = i * b + j
            if j + 1 < b:
                pairs.append((v, v + 1))
            if i + 1 < a:
                pairs.append((v, v + b))
    s, d = _edges(pairs)
    assert (bz(a * b, s, d) == 2).all()
    # empty graph -> 0 ; dead ids -> -1
    e = np.empty(0, dtype=np.int32)
    assert (bz(9, e, e) == 0).all()
    alive = np.ones(9, dtype=np.uint8)
    alive[[2, 5]] = 0
    c = bz(9, e, e, alive)
    assert c[2] == -1 and c[5] == -1 and c[0] == 0


@pytest.mark.parametrize("name", golden.all_cases())
def test_golden_fixtures_oracle(oracle_mod, name):
    case = golden.load(name)
    g = oracle_mod.DynamicGraph(case["n"], *case["edges"])
    assert np.array_equal(g.cores(), case["cores"])
    for kind, s, d, want in case["steps"]:
        st = (g.insert_edges if kind == "insert" else g.delete_edges)(s, d)[0]
        assert st == oracle_mod.OK
        assert np.array_equal(g.cores(), want), (name, kind)


def test_theta_threshold_reading(oracle_mod):
    """The paper's algorithms (method model) with the cd < k test reproduce the
    hand-derived theta fixture; the lemma's "SD <= k" reading does not."""
    from oracle import method
    case = golden.load("theta_delete.txt")
    kind, s, d, want = case["steps"][0]
    for le, ok in ((False, True), (True, False)):
        G = method.graph_from_edges(case["n"], *case["edges"])
        core = {v: int(c) for v, c in enumerate(case["cores"])}
        method.delete_edges(G, core, list(zip(s.tolist(), d.tolist())), threshold_le=le)
        got = np.asarray([core[v] for v in range(case["n"])], dtype=np.int32)
        assert np.array_equal(got, want) == ok


def _random_graph(rng, n, p):
    pairs = [pq for pq in itertools.combinations(range(n), 2) if rng.random() < p]
    return pairs


@pytest.mark.parametrize("seed", range(6))
def test_method_model_matches_definition(oracle_mod, seed):
    """The paper's iterative method (Algorithms 1-7, with the readings in
    oracle.method) ends at the from-scratch core numbers after every batch;
    after every iteration each core moved by at most one (Section IV-A lemmas
    on superior edge sets) and equals the decomposition of the graph so far."""
    from oracle import method
    rng = np.random.default_rng(100 + seed)
    for _ in range(25):
        n = int(rng.integers(5, 16))
        pairs = _random_graph(rng, n, rng.uniform(0.1, 0.5))
        all_pairs = list(itertools.combinations(range(n), 2))
        absent = [p for p in all_pairs if p not in set(pairs)]
        rng.shuffle(absent)
        ins = absent[: int(rng.integers(0, len(absent) + 1))]
        s, d = _edges(pairs) if pairs else (np.empty(0, np.int32), np.empty(0, np.int32))
        G = method.graph_from_edges(n, s, d)
        core = {v: int(c) for v, c in enumerate(oracle_mod.bz_cores(n, s, d))}
        trace = []
        prev = dict(core)
        method.insert_edges(G, core, ins, trace=trace)
        cur_pairs = set(pairs)
        for chosen, snap in trace:
            cur_pairs |= set(chosen)
            cs, cd_ = _edges(sorted(cur_pairs))
            ref = oracle_mod.bz_cores(n, cs, cd_)
            assert all(snap[v] == ref[v] for v in range(n))
            assert all(0 <= snap[v] - prev[v] <= 1 for v in range(n))
            prev = snap
        # delete a random subset of the current edges
        cur = sorted(cur_pairs)
        rng.shuffle(cur)
        dels = cur[: int(rng.integers(0, len(cur) + 1))]
        trace = []
        prev = dict(core)
        method.delete_edges(G, core, dels, trace=trace)
        for chosen, snap in trace:
            cur_pairs -= set(chosen)
            cs, cd_ = _edges(sorted(cur_pairs)) if cur_pairs else (np.empty(0, np.int32),) * 2
            ref = oracle_mod.bz_cores(n, cs, cd_)
            assert all(snap[v] == ref[v] for v in range(n))
            assert all(0 <= prev[v] - snap[v] <= 1 for v in range(n))
            prev = snap


def test_superior_set_definition_and_literal_alg2(oracle_mod):
    """Every selected set satisfies the k-superior edge set definition; the
    literal per-vertex pick of Algorithm 2 can violate it (two edges at one
    core-k vertex), which is why the selection reading is needed."""
    from oracle import method
    core = {0: 2, 1: 2, 2: 2, 3: 5}
    edges = [(0, 1), (1, 2), (2, 3)]
    chosen, rest = method.superior_edge_set(edges, core)
    for (u, v) in chosen:
        k = min(core[u], core[v])
        for (a, b) in chosen:
            if (a, b) == (u, v):
                continue
            shared = {u, v} & {a, b}
            assert all(core[x] > k for x in shared)
    # literal Algorithm 2: vertex 0 picks <0,1>, vertex 1 picks <1,2>:
    # vertex 1 (core 2) then holds two edges of core number 2.
    literal = [(0, 1), (1, 2)]
    shared = {0, 1} & {1, 2}
    assert any(core[x] == 2 for x in shared) and len(literal) == 2


def test_dynamic_graph_validation(oracle_mod):
    g = oracle_mod.DynamicGraph(5, np.array([0, 1], np.int32), np.array([1, 2], np.int32))
    E = oracle_mod
    err = g.validate(np.array([0, 9, 3, 2, 3, 1, 4]), np.array([1, 0, 3, 3, 2, 0, 0]), True)
    assert err.tolist() == [E.E_EXISTS, E.E_RANGE, E.E_SELF_LOOP, 0, E.E_DUP, E.E_DUP, 0]
    err = g.validate(np.array([0, 2, 3]), np.array([1, 1, 4]), False)
    assert err.tolist() == [0, 0, E.E_MISSING]
    st, fb, applied = g.insert_edges(np.array([3, 3]), np.array([4, 3]), strict=True)
    assert (st, fb, applied) == (E.E_SELF_LOOP, 1, 0) and g.num_edges() == 2
    st, fb, applied = g.insert_edges(np.array([3, 3]), np.array([4, 3]), strict=False)
    assert (st, applied) == (E.OK, 1) and g.num_edges() == 3
    st, fb = g.delete_vertices(np.array([1, 1]))
    assert st == E.E_DUP and fb == 1
    st, fb = g.delete_vertices(np.array([1]))
    assert st == E.OK and g.cores()[1] == -1 and g.num_edges() == 1
    st, fb, first = g.insert_vertices(np.array([0, 2]), np.array([3, 4]))
    assert st == E.OK and first == 5 and g.cores()[5] == 2


def _hindex(vals):
    vals = sorted(vals, reverse=True)
    h = 0
    for i, x in enumerate(vals):
        if x >= i + 1:
            h = i + 1
    return h


@pytest.mark.parametrize("seed", range(6))
def test_vertex_star_bounds(oracle_mod, seed):
    """The vertex-star step used for one-pass vertex operations, checked
    against Batagelj-Zaversnik on random graphs: (a) new vertices inserted
    with all their edges, several per step, such that every existing vertex
    is constrained (core <= hK of the star) by at most one of them: every
    existing vertex ends at its old core or one more, every star at hK or
    hK + 1, where hK is the h-index of the neighbours' old cores; (b) deleted
    vertices removed with all their edges, pairwise non-adjacent, every other
    vertex constrained (core <= the star's core) by at most one of them:
    every other vertex ends at its old core or one less."""
    rng = np.random.default_rng(1000 + seed)
    for trial in range(40):
        n = int(rng.integers(8, 40))
        m = int(rng.integers(n, 4 * n))
        s, d = graphgen.er_graph(n, min(m, n * (n - 1) // 2), rng)
        K = oracle_mod.bz_cores(n, s, d)
        # (a) insertion stars, greedily admitted under the one-constraint rule
        c = int(rng.integers(1, 6))
        taken = set()
        stars = []
        for i in range(c):
            nb = sorted(set(rng.integers(0, n, int(rng.integers(1, n))).tolist()))
            hk = _hindex([K[w] for w in nb])
            cons = {w for w in nb if K[w] <= hk}
            if cons & taken:
                continue
            taken |= cons
            stars.append((nb, hk))
        ss, dd = list(s), list(d)
        for j, (nb, _) in enumerate(stars):
            for w in nb:
                ss.append(w)
                dd.append(n + j)
        C = oracle_mod.bz_cores(n + len(stars), np.array(ss), np.array(dd))
        assert all(K[u] <= C[u] <= K[u] + 1 for u in range(n)), (seed, trial)
        for j, (nb, hk) in enumerate(stars):
            assert hk <= C[n + j] <= hk + 1, (seed, trial, j)
        # (b) deletion stars
        order = rng.permutation(n)
        adj = [set() for _ in range(n)]
        for a, b in zip(s, d):
            adj[a].add(b)
            adj[b].add(a)
        chosen, used = [], set()
        for x in order[: int(rng.integers(1, 6))]:
            x = int(x)
            if any(y in adj[x] for y in chosen):
                continue
            cons = {w for w in adj[x] if K[w] <= K[x]}
            if cons & used:
                continue
            used |= cons
            chosen.append(x)
        dead = set(chosen)
        keep = [(a, b) for a, b in zip(s, d) if a not in dead and b not in dead]
        ks = np.array([a for a, _ in keep], dtype=np.int64)
        kd = np.array([b for _, b in keep], dtype=np.int64)
        C2 = oracle_mod.bz_cores(n, ks, kd)
        for u in range(n):
            if u not in dead:
                assert K[u] - 1 <= C2[u] <= K[u], (seed, trial, u)


def _definitional_cores_all(n):
    """Core numbers of every labelled graph on n vertices at once, straight
    from the definition (core(v) = the largest minimum degree of an induced
    subgraph containing v): graphs are rows of neighbour bitmasks, and every
    vertex subset S is tried for every graph in one vectorised pass."""
    pairs = list(itertools.combinations(range(n), 2))
    masks = np.arange(1 << len(pairs), dtype=np.int64)
    adj = np.zeros((masks.size, n), dtype=np.int64)
    for i, (a, b) in enumerate(pairs):
        on = (masks >> i) & 1
        adj[:, a] |= on << b
        adj[:, b] |= on << a
    best = np.zeros((masks.size, n), dtype=np.int64)
    popcount = np.vectorize(lambda x: bin(int(x)).count("1"))
    table = popcount(np.arange(1 << n))
    for S in range(1, 1 << n):
        members = [v for v in range(n) if S >> v & 1]
        mindeg = np.min(np.stack([table[adj[:, v] & S] for v in members]), axis=0)
        for v in members:
            np.maximum(best[:, v], mindeg, out=best[:, v])
    return pairs, masks, best


def test_all_labelled_graphs_n6(oracle_mod):
    """Every one of the 2^15 labelled graphs on 6 vertices: definition ==
    BZ == threshold peeling."""
    n = 6
    pairs, masks, best = _definitional_cores_all(n)
    for g in range(masks.size):
        sel = [p for i, p in enumerate(pairs) if g >> i & 1]
        s = np.asarray([p[0] for p in sel], dtype=np.int32)
        d = np.asarray([p[1] for p in sel], dtype=np.int32)
        z = oracle_mod.bz_cores(n, s, d)
        assert np.array_equal(z, best[g]), (sel, z, best[g])
        if g % 7 == 0:  # peeling is slower: every seventh graph
            assert np.array_equal(oracle_mod.peel_cores(n, s, d), best[g]), sel


def test_method_model_fuzz(oracle_mod):
    """10^4 random tiny cases of the paper's iterative method (Algorithms 1-7
    with the readings in oracle.method): after every iteration the cores
    equal BZ of the graph so far, every core moved by at most one in the
    batch's direction and only at a level of an edge of the iteration's set
    (lemmas and theorems on superior edge set insertion and deletion,
    Section IV-A).  Sets holding edges of adjacent levels k and k + 1 -- the
    case whose proof is informal -- must occur often."""
    from oracle import method
    rng = np.random.default_rng(2024)
    adjacent = 0
    iterations = 0
    for case in range(10_000):
        n = int(rng.integers(4, 12))
        pairs = _random_graph(rng, n, rng.uniform(0.15, 0.7))
        all_pairs = list(itertools.combinations(range(n), 2))
        present = set(pairs)
        absent = [p for p in all_pairs if p not in present]
        rng.shuffle(absent)
        ins = absent[: int(rng.integers(0, len(absent) + 1))]
        s, d = _edges(pairs) if pairs else (np.empty(0, np.int32), np.empty(0, np.int32))
        G = method.graph_from_edges(n, s, d)
        core = {v: int(c) for v, c in enumerate(oracle_mod.bz_cores(n, s, d))}
        cur = set(pairs)
        for inserting in (True, False):
            if inserting:
                batch = ins
            else:
                batch = sorted(cur)
                rng.shuffle(batch)
                batch = batch[: int(rng.integers(0, len(batch) + 1))]
            trace = []
            prev = dict(core)
            (method.insert_edges if inserting else method.delete_edges)(G, core, batch, trace=trace)
            for chosen, snap in trace:
                iterations += 1
                levels = {min(prev[u], prev[v]) for u, v in chosen}
                adjacent += any(k + 1 in levels for k in levels)
                cur = cur | set(chosen) if inserting else cur - set(chosen)
                cs, cd_ = _edges(sorted(cur)) if cur else (np.empty(0, np.int32),) * 2
                ref = oracle_mod.bz_cores(n, cs, cd_)
                for v in range(n):
                    delta = snap[v] - prev[v]
                    assert snap[v] == ref[v], (case, inserting, v)
                    assert delta in ((0, 1) if inserting else (0, -1)), (case, v, delta)
                    assert delta == 0 or prev[v] in levels, (case, v, prev[v], levels)
                prev = snap
    assert iterations > 20_000
    assert adjacent > 1_000, adjacent


def test_insert_vertices_keep_failed_ids(oracle_mod):
    """The serving convention: ids of a vertex insertion are handed out when
    it is submitted, so a rejected request keeps them as dead ids (core -1)
    and the next request's ids come after them; a valid request's new
    vertices join with their edges."""
    E = oracle_mod
    g = E.DynamicGraph(4, np.array([0, 1, 2], np.int32), np.array([1, 2, 0], np.int32))
    # rejected: neighbour 9 is out of range
    st, fb, first = g.insert_vertices(np.array([0, 2, 3]), np.array([0, 9, 1]), keep_failed_ids=True)
    assert (st, fb, first) == (E.E_RANGE, 1, 4)
    assert g.n == 6 and g.cores().tolist() == [2, 2, 2, 0, -1, -1] and g.num_edges() == 3
    # edges to the dead ids are now invalid
    assert g.insert_edges(np.array([0]), np.array([4]))[0] == E.E_DEAD
    # the next insertion gets ids 6, 7: vertex 6 joins the triangle, 7 hangs off 6
    st, fb, first = g.insert_vertices(np.array([0, 3, 4]), np.array([0, 1, 2, 6]), keep_failed_ids=True)
    assert (st, first) == (E.OK, 6)
    assert g.cores().tolist() == [3, 3, 3, 0, -1, -1, 3, 1] and g.num_edges() == 7
    # the one-call convention frees the ids of a rejected request instead
    h = E.DynamicGraph(3, np.array([0], np.int32), np.array([1], np.int32))
    st, fb, first = h.insert_vertices(np.array([0, 1]), np.array([7]))
    assert (st, first) == (E.E_RANGE, -1) and h.n == 3


def test_dynamic_graph_matches_a_plain_edge_set(oracle_mod):
    """The oracle's edge storage (initial keys with a presence mask, later
    keys in a side array) against a Python set on a random stream of
    insertions, deletions, re-insertions of deleted initial edges and vertex
    deletions."""
    rng = np.random.default_rng(7)
    n = 60
    s, d = graphgen.er_graph(n, 300, rng)
    g = oracle_mod.DynamicGraph(n, s, d)
    model = set(zip(np.minimum(s, d).tolist(), np.maximum(s, d).tolist()))
    for step in range(400):
        op = rng.integers(0, 3)
        if op == 0:
            cand = [(a, b) for a, b in itertools.combinations(range(n), 2)
                    if (a, b) not in model and g.alive[a] and g.alive[b]]
            if not cand:
                continue
            k = min(len(cand), int(rng.integers(1, 8)))
            pick = [cand[i] for i in rng.choice(len(cand), k, replace=False)]
            a, b = _edges(pick)
            assert g.insert_edges(b, a)[0] == oracle_mod.OK  # either orientation
            model |= set(pick)
        elif op == 1 and model:
            cur = sorted(model)
            k = min(len(cur), int(rng.integers(1, 8)))
            pick = [cur[i] for i in rng.choice(len(cur), k, replace=False)]
            a, b = _edges(pick)
            assert g.delete_edges(a, b)[0] == oracle_mod.OK
            model -= set(pick)
        elif op == 2 and step % 50 == 0:
            live = np.nonzero(g.alive)[0]
            x = int(rng.choice(live))
            assert g.delete_vertices(np.array([x]))[0] == oracle_mod.OK
            model = {(a, b) for a, b in model if x not in (a, b)}
        assert g.num_edges() == len(model)
        assert g.keys.tolist() == sorted((a << 32) | b for a, b in model)
        assert g.has(np.array([(a << 32) | b for a, b in list(model)[:5]], np.int64)).all()
