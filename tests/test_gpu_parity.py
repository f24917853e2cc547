"""Parity of the HIP path (through the C ABI) with the CPU oracle: core numbers
bit-exact after the initial decomposition and after every batch; the
maintained superior degree SD equals its definition on the oracle's cores."""
import itertools

import numpy as np
import pytest

import graphgen
from tests.golden import cases as golden

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    import torch
    assert torch.cuda.is_available()
    import paper_1612_09368_amd as cm
    cm.library()
    return cm


@pytest.fixture(scope="module")
def dev():
    import torch
    return torch.device("cuda:0")


def _t(x, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def sd_definition(n, s, d, core):
    """SD(v) = #{w in N(v) : core(w) >= core(v)} (superior degree, Section IV-B)."""
    sd = np.zeros(n, dtype=np.int64)
    s = s.astype(np.int64)
    d = d.astype(np.int64)
    np.add.at(sd, s, (core[d] >= core[s]).astype(np.int64))
    np.add.at(sd, d, (core[s] >= core[d]).astype(np.int64))
    sd[core < 0] = 0
    return sd.astype(np.int32)


def check_state(g, ref, tag=""):
    got = g.cores()
    want = ref.cores()
    assert got.shape == want.shape, tag
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{tag}: {bad.size} cores differ, first {bad[:5]} got {got[bad[:5]]} want {want[bad[:5]]}"
    s, d = ref.edges()
    sd = g.superior_degrees()
    want_sd = sd_definition(ref.n, s, d, want)
    badsd = np.nonzero(sd != want_sd)[0]
    assert badsd.size == 0, f"{tag}: SD differs at {badsd[:5]} got {sd[badsd[:5]]} want {want_sd[badsd[:5]]}"
    assert g.num_edges() == ref.num_edges(), tag


FORMS = {
    "rounds": {},
    "async": {"async_steps": True},
    "pruned": {"expand_mode": 1},
    "fullscan": {"expand_mode": 2},
    "sublists": {"expand_mode": 3},
}
FORM = {}


@pytest.fixture(autouse=True, params=list(FORMS))
def _cascade_form(request):
    """Every parity test runs with round-synchronous cascades (default
    expansion: supporter runs for the eviction and up-lists of long lists),
    with asynchronous (work-queue) cascades, with Algorithm 3's pruned
    two-pass expansion, with the one-pass expansion alone, and with
    supporter runs but no up-lists."""
    global FORM
    FORM = FORMS[request.param]
    yield
    FORM = {}


def new_graph(cm, n, s, d, dev, **kw):
    for key, val in FORM.items():
        kw.setdefault(key, val)
    g = cm.Graph(**kw)
    g.load(n, _t(s, dev), _t(d, dev))
    g.decompose()
    return g


@pytest.mark.parametrize("name", golden.all_cases())
@pytest.mark.parametrize("mode", [0, 1])
def test_golden_fixtures(cm, dev, name, mode):
    case = golden.load(name)
    with new_graph(cm, case["n"], *case["edges"], dev, mode=mode) as g:
        assert np.array_equal(g.cores(), case["cores"])
        for kind, s, d, want in case["steps"]:
            (g.insert_edges if kind == "insert" else g.delete_edges)(_t(s, dev), _t(d, dev))
            assert np.array_equal(g.cores(), want), (name, kind, g.cores(), want)


def test_decompose_closed_forms(cm, dev, oracle_mod):
    graphs = []
    for n in (2, 7, 40):
        graphs.append((n, list(itertools.combinations(range(n), 2))))
    graphs.append((101, [(i, (i + 1) % 101) for i in range(101)]))
    graphs.append((12, [(i, 4 + j) for i in range(4) for j in range(8)]))
    r = 9
    graphs.append((r + 1, [(0, i) for i in range(1, r + 1)] + [(i, i % r + 1) for i in range(1, r + 1)]))
    graphs.append((50, []))
    for n, pairs in graphs:
        s = np.asarray([p[0] for p in pairs], dtype=np.int32)
        d = np.asarray([p[1] for p in pairs], dtype=np.int32)
        with new_graph(cm, n, s, d, dev) as g:
            assert np.array_equal(g.cores(), oracle_mod.brute_cores(n, s, d) if n <= 12
                                  else oracle_mod.bz_cores(n, s, d))


@pytest.mark.parametrize("kind", ["er", "cl", "rmat"])
def test_decompose_random(cm, dev, oracle_mod, kind):
    rng = graphgen.rng_for("dec-" + kind)
    if kind == "er":
        n = 30_000
        s, d = graphgen.er_graph(n, 150_000, rng)
    elif kind == "cl":
        n = 50_000
        s, d = graphgen.chung_lu_graph(n, 400_000, 2.1, 8000.0, rng)
    else:
        n, s, d = graphgen.rmat_graph(15, 16, rng)
    ref = oracle_mod.DynamicGraph(n, s, d)
    with new_graph(cm, n, s, d, dev) as g:
        check_state(g, ref, kind)


def _batches(ref, rng, n, count, size):
    """Alternating insert / delete batches valid against the current graph
    (sizes capped by the non-edges / edges available)."""
    es = graphgen.EdgeSet(*ref.edges())
    out = []
    for b in range(count):
        if b % 2 == 0:
            free = n * (n - 1) // 2 - len(es)
            if min(size, free) == 0:
                continue
            s, d = graphgen.uniform_non_edges(n, min(size, free), es, rng)
            es.insert(s, d)
            out.append(("insert", s, d))
        else:
            if len(es) == 0:
                continue
            s, d = graphgen.existing_edges(size, es, rng)
            es.delete(s, d)
            out.append(("delete", s, d))
    return out


@pytest.mark.parametrize("mode", [0, 1])
def test_er_config_parity(cm, dev, oracle_mod, mode):
    """G(10,000, 50,000), seed 0: insert 1,000 non-edges, then delete 1,000
    existing edges; cores compared after each batch."""
    rng = graphgen.rng_for("er-10k")
    n = 10_000
    s, d = graphgen.er_graph(n, 50_000, np.random.default_rng(0))
    ref = oracle_mod.DynamicGraph(n, s, d)
    es = graphgen.EdgeSet(s, d)
    with new_graph(cm, n, s, d, dev, mode=mode) as g:
        check_state(g, ref, "initial")
        a, b = graphgen.uniform_non_edges(n, 1000, es, rng)
        st = g.insert_edges(_t(a, dev), _t(b, dev))
        ref.insert_edges(a, b)
        es.insert(a, b)
        assert st.applied == 1000 and st.iterations >= 1
        check_state(g, ref, "after insert")
        a, b = graphgen.existing_edges(1000, es, rng)
        st = g.delete_edges(_t(a, dev), _t(b, dev))
        ref.delete_edges(a, b)
        assert st.applied == 1000
        check_state(g, ref, "after delete")


@pytest.mark.parametrize("seed", range(4))
def test_fuzz_small_graphs(cm, dev, oracle_mod, seed):
    rng = np.random.default_rng(1000 + seed)
    for trial in range(12):
        n = int(rng.integers(5, 60))
        maxm = n * (n - 1) // 2
        m = int(rng.integers(0, min(maxm, 4 * n) + 1))
        s, d = graphgen.er_graph(n, m, rng)
        ref = oracle_mod.DynamicGraph(n, s, d)
        mode = int(rng.integers(0, 2))
        rounds = int(rng.integers(1, 4))
        print(f"fuzz seed {seed} trial {trial}: n={n} m={m} mode={mode} rounds={rounds}", flush=True)
        with new_graph(cm, n, s, d, dev, mode=mode, partition_rounds=rounds,
                       small_degree=int(rng.choice([1, 4, 16])), large_degree=int(rng.choice([8, 32, 4096])),
                       chunk=int(rng.choice([8, 64, 2048]))) as g:
            check_state(g, ref, f"seed {seed} trial {trial} initial")
            for kind, a, b in _batches(ref, rng, n, 6, int(rng.integers(1, max(2, n)))):
                if a.size == 0:
                    continue
                (g.insert_edges if kind == "insert" else g.delete_edges)(_t(a, dev), _t(b, dev))
                (ref.insert_edges if kind == "insert" else ref.delete_edges)(a, b)
                check_state(g, ref, f"seed {seed} trial {trial} {kind}")


@pytest.mark.parametrize("kind", ["cl", "rmat"])
def test_skewed_batches(cm, dev, oracle_mod, kind):
    """Degree-weighted updates on skewed graphs: hubs collect many updates, so
    batches need many superior edge sets; long lists take the chunked path."""
    rng = graphgen.rng_for("skew-" + kind)
    if kind == "cl":
        n = 40_000
        s, d = graphgen.chung_lu_graph(n, 300_000, 2.1, 6000.0, rng)
    else:
        n, s, d = graphgen.rmat_graph(14, 16, rng)
    ref = oracle_mod.DynamicGraph(n, s, d)
    es = graphgen.EdgeSet(s, d)
    for mode in (0, 1):
        with new_graph(cm, n, s, d, dev, mode=mode, large_degree=512, chunk=256) as g:
            r2 = oracle_mod.DynamicGraph(n, s, d)
            e2 = graphgen.EdgeSet(s, d)
            for step in range(2):
                a, b = graphgen.weighted_non_edges(5000, e2, rng)
                st = g.insert_edges(_t(a, dev), _t(b, dev))
                r2.insert_edges(a, b)
                e2.insert(a, b)
                check_state(g, r2, f"{kind} mode {mode} insert {step}")
                assert st.iterations > 1
                a, b = graphgen.existing_edges(5000, e2, rng)
                g.delete_edges(_t(a, dev), _t(b, dev))
                r2.delete_edges(a, b)
                e2.delete(a, b)
                check_state(g, r2, f"{kind} mode {mode} delete {step}")
    del ref, es


@pytest.mark.parametrize("mode", [0, 1])
def test_locate_scan_long_lists(cm, dev, oracle_mod, mode):
    """Validation of edges between long lists (the locate scan reads whole
    lists, several wave steps per item, and a ragged last item): deletions
    whose partners sit anywhere in a hub's list, a missing edge and an
    existing edge between two long lists, in strict and in filter mode."""
    rng = np.random.default_rng(1612)
    n = 4000
    h0, h1, h2 = 0, 1, 2
    # h0: 1037 neighbours besides h1 (four full items of 256 slots and a
    # ragged one); h1: 600 besides h0; h2: 300, none of them h0
    p0 = rng.choice(np.arange(3, n), 1037, replace=False)
    p1 = rng.choice(np.arange(3, n), 600, replace=False)
    p2 = rng.choice(np.arange(3, n), 300, replace=False)
    rest = rng.integers(3, n, size=(6000, 2))
    rest = rest[rest[:, 0] != rest[:, 1]]
    s = np.concatenate([np.full(1037, h0), np.full(600, h1), [h0], np.full(300, h2), rest[:, 0]])
    d = np.concatenate([p0, p1, [h1], p2, rest[:, 1]])
    s, d = graphgen.EdgeSet(s.astype(np.int32), d.astype(np.int32)).edges()
    s, d = s.astype(np.int32), d.astype(np.int32)
    ref = oracle_mod.DynamicGraph(n, s, d)
    with new_graph(cm, n, s, d, dev, mode=mode) as g:
        check_state(g, ref, "load")
        # an edge missing between two long lists fails the whole batch
        a = np.array([h0, h2], np.int32)
        b = np.array([p0[5], h0], np.int32)
        st, stats = g.delete_edges(_t(a, dev), _t(b, dev), check=False)
        assert st == cm.E_MISSING and stats.first_bad == 1, (st, stats.first_bad)
        assert int(ref.validate(a, b, False)[1]) == cm.E_MISSING
        # an existing edge between two long lists
        a = np.array([p2[0], h1], np.int32)
        b = np.array([h2 if p2[0] not in p0 else p1[0], h0], np.int32)
        err = ref.validate(a, b, True)
        assert int(err[1]) == cm.E_EXISTS
        st, stats = g.insert_edges(_t(a, dev), _t(b, dev), check=False)
        first = int(np.nonzero(err)[0][0])
        assert st == int(err[first]) and stats.first_bad == first, (st, stats.first_bad, err)
        check_state(g, ref, "after rejected batches")
        # deletions spread over every item of h0's list and over h1's
        a = np.concatenate([np.full(97, h0), np.full(41, h1), [h0]]).astype(np.int32)
        b = np.concatenate([rng.choice(p0, 97, replace=False), rng.choice(p1, 41, replace=False),
                            [h1]]).astype(np.int32)
        g.delete_edges(_t(b, dev), _t(a, dev))
        ref.delete_edges(b, a)
        check_state(g, ref, "spread deletions")
        s2, d2 = ref.edges()
        s2, d2 = s2.astype(np.int32), d2.astype(np.int32)
    # filter mode: invalid items between long lists are dropped, the rest applied
    ref2 = oracle_mod.DynamicGraph(n, s2, d2)
    with new_graph(cm, n, s2, d2, dev, mode=mode, strict=False) as g:
        live0 = d2[s2 == h0]
        a = np.array([h0, h0, h2, h0, h1], np.int32)
        b = np.array([h1, live0[-1], h0, live0[0], p1[0]], np.int32)
        st = g.delete_edges(_t(a, dev), _t(b, dev))
        ref2.delete_edges(a, b, strict=False)
        ok = int((oracle_mod.DynamicGraph(n, s2, d2).validate(a, b, False) == 0).sum())
        assert st.applied == ok and st.dropped == a.size - ok, (st.applied, st.dropped, ok)
        check_state(g, ref2, "filtered deletions")


@pytest.mark.parametrize("mode", [0, 1])
def test_hub_lists_cross_levels(cm, dev, oracle_mod, mode):
    """Vertices with long lists (257, 513, 700 and 1025 entries: several
    chunks with ragged ends) change core in both directions: a 24-clique
    holds four hubs padded with leaves, and deleting or re-inserting clique
    edges moves every member between cores 23 and 22 (and lower), so the
    peel, the SD recount and the expansion walk the hubs chunk by chunk."""
    q = 24
    hubs_len = [257, 513, 700, 1025]
    clique = np.arange(q)
    s, d = [], []
    for i in range(q):
        for j in range(i + 1, q):
            s.append(i)
            d.append(j)
    nxt = q
    for h, L in enumerate(hubs_len):
        for _ in range(L - (q - 1)):
            s.append(h)
            d.append(nxt)
            nxt += 1
    # a ring through the leaves of hubs 2 and 3 gives them degree 2
    ring = np.arange(q + hubs_len[0] + hubs_len[1] - 2 * (q - 1), nxt)
    s.extend(ring[:-1].tolist())
    d.extend(ring[1:].tolist())
    n = nxt + 8
    s = np.array(s, np.int32)
    d = np.array(d, np.int32)
    ref = oracle_mod.DynamicGraph(n, s, d)
    steps = [
        ("delete", [5], [6]),                      # one clique edge: every member 23 -> 22
        ("insert", [5], [6]),                      # back to 23
        ("delete", [0, 7, 9], [1, 8, 10]),         # a hub-hub edge and two more
        ("delete", [2, 11], [3, 12]),
        ("insert", [0, 2, 7], [1, 3, 8]),
        ("insert", [9, 11], [10, 12]),
        ("delete", [3, 3, 3], [20, 21, 22]),       # the longest hub loses three clique edges
        ("insert", [3, 3, 3], [20, 21, 22]),
    ]
    with new_graph(cm, n, s, d, dev, mode=mode) as g:
        check_state(g, ref, "load")
        assert int(g.cores()[clique].min()) == q - 1
        for i, (kind, a, b) in enumerate(steps):
            a = np.array(a, np.int32)
            b = np.array(b, np.int32)
            (g.insert_edges if kind == "insert" else g.delete_edges)(_t(a, dev), _t(b, dev))
            (ref.insert_edges if kind == "insert" else ref.delete_edges)(a, b)
            check_state(g, ref, f"step {i} {kind}")
        assert int(g.cores()[clique].min()) == q - 1


def test_insert_then_delete_restores(cm, dev, oracle_mod):
    rng = graphgen.rng_for("restore")
    n = 5000
    s, d = graphgen.chung_lu_graph(n, 30_000, 2.3, 500.0, rng)
    es = graphgen.EdgeSet(s, d)
    a, b = graphgen.weighted_non_edges(3000, es, rng)
    with new_graph(cm, n, s, d, dev) as g:
        before = g.cores().copy()
        sd0 = g.superior_degrees().copy()
        g.insert_edges(_t(a, dev), _t(b, dev))
        after = g.cores()
        assert (after >= before).all()
        g.delete_edges(_t(b, dev), _t(a, dev))
        assert np.array_equal(g.cores(), before)
        assert np.array_equal(g.superior_degrees(), sd0)


def test_strict_errors_leave_graph_unchanged(cm, dev, oracle_mod):
    n = 6
    s = np.array([0, 1, 2, 3], dtype=np.int32)
    d = np.array([1, 2, 3, 4], dtype=np.int32)
    with new_graph(cm, n, s, d, dev) as g:
        before = g.cores().copy()
        cases = [
            ("insert", [0, 9], [5, 1], cm.E_RANGE, 1),
            ("insert", [5, 2], [0, 2], cm.E_SELF_LOOP, 1),
            ("insert", [0, 5, 2], [5, 0, 5], cm.E_DUP, 1),
            ("insert", [0, 2], [5, 1], cm.E_EXISTS, 1),
            ("delete", [0, 0], [1, 5], cm.E_MISSING, 1),
            ("delete", [1, 0], [0, 1], cm.E_DUP, 1),
        ]
        ref = oracle_mod.DynamicGraph(n, s, d)
        for kind, a, b, code, idx in cases:
            a = np.array(a, dtype=np.int32)
            b = np.array(b, dtype=np.int32)
            fn = g.insert_edges if kind == "insert" else g.delete_edges
            st, stats = fn(_t(a, dev), _t(b, dev), check=False)
            assert st == code and stats.first_bad == idx, (kind, a, b, st, stats.first_bad)
            err = ref.validate(a, b, kind == "insert")
            assert int(err[np.nonzero(err)[0][0]]) == code
            assert np.array_equal(g.cores(), before) and g.num_edges() == 4
        # host inputs take the same path
        st, stats = g.insert_edges(np.array([0, 4], np.int32), np.array([1, 4], np.int32), check=False)
        assert st == cm.E_EXISTS and stats.first_bad == 0


def test_filter_mode_drops_invalid(cm, dev, oracle_mod):
    n = 8
    s = np.array([0, 1, 2], dtype=np.int32)
    d = np.array([1, 2, 0], dtype=np.int32)
    with new_graph(cm, n, s, d, dev, strict=False) as g:
        a = np.array([0, 3, 3, 7, 0, 4, 4], dtype=np.int32)
        b = np.array([1, 4, 4, 7, 3, 5, 3], dtype=np.int32)
        st = g.insert_edges(_t(a, dev), _t(b, dev))
        ref = oracle_mod.DynamicGraph(n, s, d)
        ref.insert_edges(a, b, strict=False)
        assert st.applied == 3 and st.dropped == 4 and st.first_bad == 0
        check_state(g, ref, "filter insert")


@pytest.mark.parametrize("mode", [0, 1])
def test_vertex_ops(cm, dev, oracle_mod, mode):
    # mode 0: the Introduction's reduction (edges through superior edge sets);
    # mode 1: one persistent launch, vertices entering / leaving as stars
    rng = graphgen.rng_for("vops")
    n = 3000
    s, d = graphgen.chung_lu_graph(n, 15_000, 2.2, 300.0, rng)
    ref = oracle_mod.DynamicGraph(n, s, d)
    es = graphgen.EdgeSet(s, d)
    with new_graph(cm, n, s, d, dev, vertex_capacity=0, mode=mode) as g:
        # insert 200 vertices with power-law degrees, neighbours degree-weighted
        degs = graphgen.power_law_degrees(200, 1, 60, 2.1, rng)
        off, nb = graphgen.vertex_insert_payload(n, 200, degs, es, rng)
        first, st = g.insert_vertices(_t(off, dev), _t(nb, dev))
        st2, _, first2 = ref.insert_vertices(off, nb)
        assert first == first2 == n
        check_state(g, ref, "vertex insert")
        # a new vertex joined to an earlier new vertex and existing ones
        off2 = np.array([0, 3], dtype=np.int64)
        nb2 = np.array([n, n + 1, 5], dtype=np.int32)
        first, _ = g.insert_vertices(off2, nb2)
        ref.insert_vertices(off2, nb2)
        check_state(g, ref, "vertex insert 2")
        # delete 300 live vertices (old and new)
        ids = rng.choice(n + 201, 300, replace=False).astype(np.int32)
        g.delete_vertices(_t(ids, dev))
        ref.delete_vertices(ids)
        check_state(g, ref, "vertex delete")
        assert (g.cores()[ids] == -1).all()
        nids, alive = g.num_vertices()
        assert nids == n + 201 and alive == n + 201 - 300
        # errors: dead id, duplicate, out of range
        for bad, code in (([int(ids[0])], cm.E_DEAD), ([1, 1], cm.E_DUP), ([10 ** 6], cm.E_RANGE)):
            live = [v for v in [1] if v not in set(ids.tolist())]
            st, _ = g.delete_vertices(np.array(bad, dtype=np.int32), check=False)
            assert st == code or (code == cm.E_DUP and 1 in set(ids.tolist()))
            del live
        # invalid neighbour rejects the whole vertex insert
        st, fid, _ = g.insert_vertices(np.array([0, 2], np.int64), np.array([0, int(ids[0])], np.int32),
                                       check=False)
        assert st == cm.E_DEAD
        assert g.num_vertices()[0] == n + 201
        check_state(g, ref, "after rejected vertex insert")


@pytest.mark.parametrize("mode", [0, 1])
def test_uplists_across_batches(cm, dev, oracle_mod, mode):
    """Long lists keep up-lists (neighbours at or above their owner's core)
    across batches; every change that could add a neighbour at or above a
    vertex's core outside its up-list invalidates it: a neighbour rising to
    that core, the vertex's own core falling, an edge of it deleted, its list
    moved, a fresh decomposition.  Many degree-weighted batches on one handle
    with lists split into 8-slot chunks (so most lists keep up-lists), vertex
    insertions and hub deletions, and a second decomposition between them:
    cores and SD equal the oracle's after every step."""
    rng = graphgen.rng_for("uplists")
    n = 3000
    s, d = graphgen.chung_lu_graph(n, 15_000, 2.1, 400.0, rng)
    ref = oracle_mod.DynamicGraph(n, s, d)
    es = graphgen.EdgeSet(s, d)
    nid = n
    with new_graph(cm, n, s, d, dev, mode=mode, small_degree=4, large_degree=8, chunk=8) as g:
        for step in range(24):
            if step % 2 == 0:
                a, b = graphgen.weighted_non_edges(int(rng.integers(20, 400)), es, rng)
                g.insert_edges(_t(a, dev), _t(b, dev))
                ref.insert_edges(a, b)
                es.insert(a, b)
            else:
                a, b = graphgen.existing_edges(int(rng.integers(20, 300)), es, rng)
                g.delete_edges(_t(a, dev), _t(b, dev))
                ref.delete_edges(a, b)
                es.delete(a, b)
            check_state(g, ref, f"step {step}")
            if step == 7:
                degs = graphgen.power_law_degrees(30, 1, 40, 2.1, rng)
                off, nb = graphgen.vertex_insert_payload(nid, 30, degs, es, rng)
                g.insert_vertices(_t(off, dev), _t(nb, dev))
                ref.insert_vertices(off, nb)
                nid += 30
                es = graphgen.EdgeSet(*ref.edges())
                check_state(g, ref, f"step {step} vertex insert")
            if step == 13:
                deg = np.bincount(np.concatenate(ref.edges()).astype(np.int64), minlength=nid)
                hubs = np.argsort(-deg)[:12].astype(np.int32)
                g.delete_vertices(_t(hubs, dev))
                ref.delete_vertices(hubs)
                es = graphgen.EdgeSet(*ref.edges())
                check_state(g, ref, f"step {step} hub delete")
            if step == 17:
                g.decompose()
                check_state(g, ref, f"step {step} decompose again")


def test_growth_and_spill(cm, dev, oracle_mod):
    """Lists outgrow their slack many times (spill blocks, pool repack)."""
    rng = graphgen.rng_for("grow")
    n = 2000
    s, d = graphgen.er_graph(n, 2000, rng)
    ref = oracle_mod.DynamicGraph(n, s, d)
    es = graphgen.EdgeSet(s, d)
    with new_graph(cm, n, s, d, dev) as g:
        for step in range(6):
            a, b = graphgen.weighted_non_edges(4000, es, rng)
            g.insert_edges(_t(a, dev), _t(b, dev))
            ref.insert_edges(a, b)
            es.insert(a, b)
            check_state(g, ref, f"grow {step}")
        xs, ys = g.export_edges()
        assert np.array_equal(np.sort(graphgen.keys_of(xs, ys)), np.sort(ref.keys))


@pytest.mark.slow
def test_chung_lu_full_size(cm, dev, oracle_mod):
    """Chung-Lu n = 1,000,000, m = 10,000,000, exponent 2.1, max weight 50,000;
    100,000 degree-weighted non-edges inserted, then 100,000 existing edges
    deleted: full core vectors compared (the benchmark's workload)."""
    rng = graphgen.rng_for("cl-1m")
    n = 1_000_000
    s, d = graphgen.chung_lu_graph(n, 10_000_000, 2.1, 50_000.0, rng)
    es = graphgen.EdgeSet(s, d)
    ref = oracle_mod.DynamicGraph(n, s, d)
    with new_graph(cm, n, s, d, dev) as g:
        assert np.array_equal(g.cores(), ref.cores())
        a, b = graphgen.weighted_non_edges(100_000, es, rng)
        g.insert_edges(_t(a, dev), _t(b, dev))
        ref.insert_edges(a, b)
        es.insert(a, b)
        assert np.array_equal(g.cores(), ref.cores())
        a, b = graphgen.existing_edges(100_000, es, rng)
        g.delete_edges(_t(a, dev), _t(b, dev))
        ref.delete_edges(a, b)
        check_state(g, ref, "cl full")


@pytest.mark.parametrize("mode", [0, 1])
def test_root_list_grows_during_apply(cm, dev, oracle_mod, mode):
    """A root whose own list receives many other edges of the same superior
    edge set (it is their unconstrained endpoint): its length is final only
    after the apply phase, and the chunked CSD count must cover every entry.
    Two K6 (core 5) joined by a perfect matching rise to core 6; vertex 0 also
    gains 300 edges to isolated vertices in the same iteration."""
    a_, b_ = [], []
    for blk in (0, 6):
        for i in range(6):
            for j in range(i + 1, 6):
                a_.append(blk + i)
                b_.append(blk + j)
    for x in range(12, 312):  # pendants of vertex 0 (core 1)
        a_.append(0)
        b_.append(x)
    n = 612
    s = np.asarray(a_, dtype=np.int32)
    d = np.asarray(b_, dtype=np.int32)
    ins_a = np.asarray(list(range(6)) + [0] * 300, dtype=np.int32)
    ins_b = np.asarray([6 + i for i in range(6)] + list(range(312, 612)), dtype=np.int32)
    ref = oracle_mod.DynamicGraph(n, s, d)
    with new_graph(cm, n, s, d, dev, mode=mode, small_degree=4, large_degree=8, chunk=8) as g:
        check_state(g, ref, "initial")
        st = g.insert_edges(_t(ins_a, dev), _t(ins_b, dev))
        ref.insert_edges(ins_a, ins_b)
        check_state(g, ref, "after insert")
        assert (g.cores()[:12] == 6).all()
        g.delete_edges(_t(ins_b, dev), _t(ins_a, dev))
        ref.delete_edges(ins_b, ins_a)
        check_state(g, ref, "after delete")


@pytest.mark.parametrize("mode", [0, 1])
def test_vertex_ops_dense(cm, dev, oracle_mod, mode):
    """Many new vertices of high degree sharing neighbours, then deletions
    of the highest-degree vertices (adjacent to each other): cores after
    every operation equal the oracle's in both forms."""
    rng = graphgen.rng_for("vops-dense")
    n = 4000
    s, d = graphgen.chung_lu_graph(n, 40_000, 2.1, 800.0, rng)
    ref = oracle_mod.DynamicGraph(n, s, d)
    es = graphgen.EdgeSet(s, d)
    with new_graph(cm, n, s, d, dev, mode=mode) as g:
        nid = n
        for step in range(4):
            degs = graphgen.power_law_degrees(300, 5, 400, 1.6, rng)
            off, nb = graphgen.vertex_insert_payload(nid, 300, degs, es, rng)
            first, _ = g.insert_vertices(_t(off, dev), _t(nb, dev))
            assert ref.insert_vertices(off, nb)[0] == 0
            own = np.repeat(np.arange(nid, nid + 300), np.diff(off))
            es.insert(own, nb)
            nid += 300
            check_state(g, ref, f"dense vertex insert {step}")
            cores = g.cores()
            deg = np.bincount(np.concatenate(es.edges()), minlength=nid)
            top = np.argsort(-deg)[:60]
            top = top[cores[top] >= 0][:40].astype(np.int32)
            g.delete_vertices(_t(top, dev))
            assert ref.delete_vertices(top)[0] == 0
            ks = graphgen.keys_of(*es.edges())
            lo, hi = ks >> 32, ks & 0xFFFFFFFF
            hit = np.isin(lo, top) | np.isin(hi, top)
            es = graphgen.EdgeSet(*graphgen.split_keys(ks[~hit]))
            check_state(g, ref, f"dense vertex delete {step}")


def test_single_edge_regime(cm, dev, oracle_mod):
    """One edge per iteration (the sequential regime the paper compares
    against): same cores, and exactly one iteration per valid edge."""
    rng = graphgen.rng_for("single-edge")
    n = 1500
    s, d = graphgen.chung_lu_graph(n, 6000, 2.2, 200.0, rng)
    ref = oracle_mod.DynamicGraph(n, s, d)
    with new_graph(cm, n, s, d, dev, mode=1, single_edge=True) as g:
        for kind, a, b in _batches(ref, rng, n, 4, 150):
            if a.size == 0:
                continue
            st = (g.insert_edges if kind == "insert" else g.delete_edges)(_t(a, dev), _t(b, dev))
            (ref.insert_edges if kind == "insert" else ref.delete_edges)(a, b)
            assert st.iterations == a.size, (kind, st.iterations, a.size)
            check_state(g, ref, f"single-edge {kind}")


@pytest.mark.parametrize("mode", [0, 1])
def test_core_targeted_updates(cm, dev, oracle_mod, mode):
    """Updates concentrated on one core level (the paper's experiment on the
    core distribution of the updates): 20% of the edges of each typical edge
    core number, deleted as one batch then inserted back as one batch."""
    rng = graphgen.rng_for("core-levels")
    n, s, d = graphgen.rmat_graph(12, 16, rng)
    ref = oracle_mod.DynamicGraph(n, s, d)
    cores0 = ref.cores()
    levels = graphgen.typical_levels(s, d, cores0, 5)
    assert len(levels) >= 3
    with new_graph(cm, n, s, d, dev, mode=mode) as g:
        for k in levels:
            a, b = graphgen.edges_at_level(s, d, cores0, k, 0.2, rng)
            st = g.delete_edges(_t(a, dev), _t(b, dev))
            assert ref.delete_edges(a, b)[0] == 0 and st.status == 0
            check_state(g, ref, f"level {k} delete")
            st = g.insert_edges(_t(a, dev), _t(b, dev))
            assert ref.insert_edges(a, b)[0] == 0 and st.status == 0
            check_state(g, ref, f"level {k} insert")
        assert np.array_equal(g.cores(), cores0)


@pytest.mark.parametrize("mode", [0, 1])
def test_empty_and_degenerate_batches(cm, dev, oracle_mod, mode):
    """Empty graph and empty batches; a clique built in one batch (every
    vertex is the constrained endpoint of all its edges: one level, the
    largest conflict) and torn down in one batch; an all-invalid batch in
    filter mode; a graph of one vertex."""
    n = 50
    e = np.zeros(0, dtype=np.int32)
    with new_graph(cm, n, e, e, dev, mode=mode) as g:
        assert (g.cores() == 0).all() and g.num_edges() == 0
        st = g.insert_edges(_t(e, dev), _t(e, dev))
        assert st.applied == 0 and st.iterations == 0
        st = g.delete_edges(_t(e, dev), _t(e, dev))
        assert st.applied == 0 and st.iterations == 0
        pairs = np.array(list(itertools.combinations(range(3, 13), 2)), dtype=np.int32)
        a, b = pairs[:, 0].copy(), pairs[:, 1].copy()
        ref = oracle_mod.DynamicGraph(n, e, e)
        st = g.insert_edges(_t(a, dev), _t(b, dev))
        ref.insert_edges(a, b)
        assert st.applied == a.size
        check_state(g, ref, "clique insert")
        want = np.zeros(n, np.int32)
        want[3:13] = 9
        assert np.array_equal(g.cores(), want)   # closed form: K_10 has core 9
        st = g.delete_edges(_t(b, dev), _t(a, dev))
        ref.delete_edges(b, a)
        assert st.applied == a.size
        check_state(g, ref, "clique delete")
        assert (g.cores() == 0).all() and g.num_edges() == 0
    with new_graph(cm, n, e, e, dev, mode=mode, strict=False) as g:
        bad_a = np.array([0, 7, 60, -1, 4], dtype=np.int32)
        bad_b = np.array([0, 7, 1, 2, 4], dtype=np.int32)
        st = g.insert_edges(_t(bad_a, dev), _t(bad_b, dev))
        assert st.applied == 0 and st.dropped == bad_a.size and st.first_bad == 0
        st = g.delete_edges(_t(np.array([1, 2], np.int32), dev), _t(np.array([2, 3], np.int32), dev))
        assert st.applied == 0 and st.dropped == 2
        assert (g.cores() == 0).all() and g.num_edges() == 0
    one = np.zeros(0, dtype=np.int32)
    with new_graph(cm, 1, one, one, dev, mode=mode) as g:
        assert np.array_equal(g.cores(), np.zeros(1, np.int32))
        st, stats = g.insert_edges(_t(np.zeros(1, np.int32), dev), _t(np.zeros(1, np.int32), dev), check=False)
        assert st == cm.E_SELF_LOOP and stats.first_bad == 0


@pytest.mark.slow
def test_chung_lu_full_size_batched(cm, dev, oracle_mod):
    """The benchmark's Chung-Lu configuration (n = 1,000,000, m = 10,000,000)
    in the batched form: one insertion batch of 100,000 degree-weighted
    non-edges and one deletion batch of 100,000 existing edges in one
    persistent launch replayed from a hipGraph; the final core numbers and
    SD against the oracle."""
    rng = graphgen.rng_for("cl-1m-batched")
    n = 1_000_000
    s, d = graphgen.chung_lu_graph(n, 10_000_000, 2.1, 50_000.0, rng)
    es = graphgen.EdgeSet(s, d)
    ref = oracle_mod.DynamicGraph(n, s, d)
    a, b = graphgen.weighted_non_edges(100_000, es, rng)
    es.insert(a, b)
    x, y = graphgen.existing_edges(100_000, es, rng)
    ref.insert_edges(a, b)
    ref.delete_edges(x, y)
    xs, ys = np.concatenate([a, x]), np.concatenate([b, y])
    with new_graph(cm, n, s, d, dev, mode=1, use_graph=True) as g:
        res, _ = g.run_batches([cm.BATCH_INSERT, cm.BATCH_DELETE], [0, a.size, a.size + x.size],
                               _t(xs, dev), _t(ys, dev))
        assert [r.status for r in res] == [0, 0] and [r.applied for r in res] == [a.size, x.size]
        check_state(g, ref, "cl full batched")


@pytest.mark.parametrize("mode", [0, 1])
def test_two_workgroups_per_cu(cm, dev, oracle_mod, mode):
    """The cooperative grid with two workgroups per compute unit (a launch
    parameter the autotuner may pick): the grid barrier then groups 64
    workgroups per XCC; decomposition and mixed batches against the oracle,
    in the per-call form and in one batch program."""
    rng = graphgen.rng_for("bpc2")
    n = 20_000
    s, d = graphgen.chung_lu_graph(n, 120_000, 2.2, 2000.0, rng)
    ref = oracle_mod.DynamicGraph(n, s, d)
    with new_graph(cm, n, s, d, dev, mode=mode, blocks_per_cu=2) as g:
        check_state(g, ref, "decompose")
        for kind, a, b in _batches(ref, rng, n, 4, 3000):
            st = (g.insert_edges if kind == "insert" else g.delete_edges)(_t(a, dev), _t(b, dev))
            (ref.insert_edges if kind == "insert" else ref.delete_edges)(a, b)
            check_state(g, ref, f"bpc2 {kind}")
        if mode == 1:
            es = graphgen.EdgeSet(*ref.edges())
            a, b = graphgen.weighted_non_edges(2000, es, rng)
            es.insert(a, b)
            x, y = graphgen.existing_edges(2000, es, rng)
            res, _ = g.run_batches([cm.BATCH_INSERT, cm.BATCH_DELETE], [0, a.size, a.size + x.size],
                                   _t(np.concatenate([a, x]), dev), _t(np.concatenate([b, y]), dev))
            ref.insert_edges(a, b)
            ref.delete_edges(x, y)
            assert [r.status for r in res] == [0, 0]
            check_state(g, ref, "bpc2 program")
