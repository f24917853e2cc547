"""Multi-batch launches (cm_run_batches) and packed independent graphs: the
persistent launch, its hipGraph replay and the plain host loop give the
oracle's core numbers after a whole batch sequence, skip exactly the invalid
(sub-)batches, and survive an adjacency-pool repack mid-launch."""
import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    import torch
    assert torch.cuda.is_available()
    import paper_1612_09368_amd as cm
    cm.library()
    return cm


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _sequence(rng, n, s, d, nbatches, lo, hi):
    es = graphgen.EdgeSet(s, d)
    kinds, xs, ys = [], [], []
    sizes = graphgen.log_uniform_sizes(nbatches, lo, hi, rng)
    order = rng.permutation(np.arange(nbatches) % 2)
    for j in range(nbatches):
        if order[j] == 0:
            a, b = graphgen.weighted_non_edges(int(sizes[j]), es, rng)
            es.insert(a, b)
        else:
            a, b = graphgen.existing_edges(int(sizes[j]), es, rng)
            es.delete(a, b)
        kinds.append(int(order[j]))
        xs.append(a)
        ys.append(b)
    offs = np.concatenate([[0], np.cumsum([len(x) for x in xs])]).astype(np.int64)
    return np.asarray(kinds, np.int32), offs, np.concatenate(xs), np.concatenate(ys)


@pytest.mark.parametrize("form", ["plain", "persistent", "graph", "async"])
def test_sequence_matches_oracle(cm, oracle_mod, form):
    rng = graphgen.rng_for("seq-" + form)
    n = 20_000
    s, d = graphgen.chung_lu_graph(n, 120_000, 2.1, 2000.0, rng)
    kinds, offs, xs, ys = _sequence(rng, n, s, d, 12, 10, 8000)
    ref = oracle_mod.DynamicGraph(n, s, d)
    for j in range(len(kinds)):
        fn = ref.insert_edges if kinds[j] == 0 else ref.delete_edges
        st = fn(xs[offs[j]:offs[j + 1]], ys[offs[j]:offs[j + 1]])
        assert st[0] == 0
    mode = cm.MODE_PLAIN if form == "plain" else cm.MODE_PERSISTENT
    with cm.Graph(mode=mode, use_graph=form == "graph", async_steps=form == "async") as g:
        g.load(n, _dev(s), _dev(d))
        g.decompose()
        res, _ = g.run_batches(kinds, offs, _dev(xs), _dev(ys))
        assert all(r.status == 0 for r in res)
        assert [r.applied for r in res] == list(np.diff(offs))
        assert np.array_equal(g.cores(), ref.cores())
        assert g.num_edges() == ref.num_edges()
        if form == "graph":
            assert res[0].graph_launch == 1
            # a second call replays the instantiated graph
            kinds2, offs2, xs2, ys2 = _sequence(rng, n, *ref.edges(), 4, 10, 2000)
            res2, _ = g.run_batches(kinds2, offs2, _dev(xs2), _dev(ys2))
            for j in range(len(kinds2)):
                fn = ref.insert_edges if kinds2[j] == 0 else ref.delete_edges
                fn(xs2[offs2[j]:offs2[j + 1]], ys2[offs2[j]:offs2[j + 1]])
            assert np.array_equal(g.cores(), ref.cores())


@pytest.mark.parametrize("mode", [0, 1])
def test_invalid_batch_is_skipped(cm, oracle_mod, mode):
    rng = graphgen.rng_for("skip")
    n = 3000
    s, d = graphgen.er_graph(n, 12_000, rng)
    es = graphgen.EdgeSet(s, d)
    a1, b1 = graphgen.uniform_non_edges(n, 500, es, rng)
    es.insert(a1, b1)
    bad_a, bad_b = graphgen.uniform_non_edges(n, 50, es, rng)
    bad_a = bad_a.copy()
    bad_a[7] = n + 5                     # out of range: the whole batch is rejected
    a3, b3 = graphgen.existing_edges(400, es, rng)
    kinds = np.array([0, 0, 1], np.int32)
    offs = np.array([0, 500, 550, 950], np.int64)
    xs = np.concatenate([a1, bad_a, a3])
    ys = np.concatenate([b1, bad_b, b3])
    ref = oracle_mod.DynamicGraph(n, s, d)
    ref.insert_edges(a1, b1)
    ref.delete_edges(a3, b3)
    with cm.Graph(mode=mode) as g:
        g.load(n, s, d)
        g.decompose()
        res, _ = g.run_batches(kinds, offs, _dev(xs), _dev(ys))
        assert [r.status for r in res] == [0, cm.E_RANGE, 0]
        assert res[1].first_bad == 7
        assert np.array_equal(g.cores(), ref.cores())


@pytest.mark.parametrize("mode", [0, 1])
def test_packed_pool_of_graphs(cm, oracle_mod, mode):
    rng = graphgen.rng_for("pool")
    graphs, refs, batches = [], [], []
    for i in range(24):
        n = int(graphgen.log_uniform_sizes(1, 200, 5000, rng)[0])
        deg = rng.uniform(4, 16)
        m = int(n * deg / 2)
        s, d = graphgen.chung_lu_graph(n, m, 2.3, 0.05 * n, rng)
        graphs.append((n, s, d))
        refs.append(oracle_mod.DynamicGraph(n, s, d))
        es = graphgen.EdgeSet(s, d)
        a, b = graphgen.weighted_non_edges(max(1, m // 20), es, rng)
        es.insert(a, b)
        x, y = graphgen.existing_edges(max(1, m // 20), es, rng)
        if i == 5:   # an invalid member batch: only this member's batch is dropped
            a = a.copy()
            a[0] = b[0]
        batches.append((i, 0, a, b))
        batches.append((i, 1, x, y))
    pool = cm.GraphPool(graphs, mode=mode)
    try:
        statuses, stats = pool.run(batches, device="cuda:0")
        for k, (gid, kind, a, b) in enumerate(batches):
            fn = refs[gid].insert_edges if kind == 0 else refs[gid].delete_edges
            st = fn(a, b)[0]
            if gid == 5 and kind == 0:
                assert statuses[k] == cm.E_SELF_LOOP and st == cm.E_SELF_LOOP
            elif gid == 5 and kind == 1:
                # the insert was dropped, so some deleted edges may be missing now
                assert statuses[k] == st
            else:
                assert statuses[k] == 0 and st == 0, (k, statuses[k], st)
        for gid in range(len(graphs)):
            assert np.array_equal(pool.cores(gid), refs[gid].cores()), gid
    finally:
        pool.close()


def test_program_survives_pool_repack(cm, oracle_mod):
    rng = graphgen.rng_for("prog-grow")
    n = 4000
    s, d = graphgen.er_graph(n, 4000, rng)
    kinds, offs, xs, ys = [], [0], [], []
    es = graphgen.EdgeSet(s, d)
    ref = oracle_mod.DynamicGraph(n, s, d)
    for j in range(6):
        a, b = graphgen.weighted_non_edges(5000, es, rng)
        es.insert(a, b)
        ref.insert_edges(a, b)
        kinds.append(0)
        xs.append(a)
        ys.append(b)
        offs.append(offs[-1] + len(a))
    with cm.Graph(mode=cm.MODE_PERSISTENT) as g:
        g.load(n, s, d)
        g.decompose()
        res, _ = g.run_batches(np.array(kinds, np.int32), np.array(offs, np.int64),
                               np.concatenate(xs), np.concatenate(ys))
        assert all(r.status == 0 for r in res)
        assert np.array_equal(g.cores(), ref.cores())
        xs2, ys2 = g.export_edges()
        assert np.array_equal(np.sort(graphgen.keys_of(xs2, ys2)), np.sort(ref.keys))
