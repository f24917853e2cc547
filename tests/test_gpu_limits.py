"""Long runs and waits that are legal and must not trip the kernels' bounds:
- iteration stamps restarting many times (a tiny stamp limit) in every form,
  core numbers exact after every batch;
- an O(n)-round cascade at one level (deleting one edge of a cycle of 10^6
  vertices, closing a path of 10^6 vertices into a cycle), whose chain of
  small steps outlasts any single barrier wait;
- a serving launch idling longer than the default barrier bound's slack."""
import time

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


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


@pytest.mark.parametrize("form", ["plain", "persistent", "program", "async", "single_edge"])
@pytest.mark.parametrize("limit", [1, 3, 7])
def test_stamp_restarts_keep_cores_exact(cm, oracle_mod, form, limit):
    rng = graphgen.rng_for(f"restamp-{form}-{limit}")
    n = 3000
    s, d = graphgen.er_graph(n, 12000, rng)
    es = graphgen.EdgeSet(s, d)
    ref = oracle_mod.DynamicGraph(n, s, d)
    kw = dict(stamp_limit=limit, mode=0 if form == "plain" else 1)
    if form == "async":
        kw["async_steps"] = True
    if form == "single_edge":
        kw["single_edge"] = True
    g = cm.Graph(**kw)
    try:
        g.load(n, _t(s), _t(d))
        g.decompose()
        for j in range(6):
            size = 60 if form == "single_edge" else 400
            if j % 2 == 0:
                a, b = graphgen.uniform_non_edges(n, size, es, rng)
                es.insert(a, b)
            else:
                a, b = graphgen.existing_edges(size, es, rng)
                es.delete(a, b)
            kind = cm.BATCH_INSERT if j % 2 == 0 else cm.BATCH_DELETE
            if form == "program":
                res, _ = g.run_batches(np.array([kind], np.int32), np.array([0, a.size], np.int64), _t(a), _t(b))
                assert res[0].status == 0
            else:
                (g.insert_edges if kind == cm.BATCH_INSERT else g.delete_edges)(_t(a), _t(b))
            (ref.insert_edges if kind == cm.BATCH_INSERT else ref.delete_edges)(a, b)
            assert np.array_equal(g.cores(), ref.cores()), f"batch {j}"
        if form == "persistent":
            # vertex stars restart stamps too
            off = np.array([0, 40, 90], np.int64)
            nb = rng.choice(n, 90, replace=False).astype(np.int32)
            g.insert_vertices(off, nb)
            ref.insert_vertices(off, nb)
            ids = rng.choice(n, 25, replace=False).astype(np.int32)
            g.delete_vertices(ids)
            ref.delete_vertices(ids)
            assert np.array_equal(g.cores(), ref.cores()), "vertex stars"
    finally:
        g.close()


@pytest.mark.parametrize("mode,async_steps", [(0, False), (1, False), (1, True)],
                         ids=["plain", "persistent", "async"])
def test_long_cycle_cascades(cm, mode, async_steps):
    """Every vertex of C_n has core 2; removing one edge peels the whole
    cycle to core 1 in about n/2 rounds, and putting it back raises it again
    through an expansion of about n/2 rounds (Algorithms 6-7, 3-4)."""
    n = 1_000_000
    v = np.arange(n, dtype=np.int32)
    s, d = v, np.roll(v, -1)
    g = cm.Graph(mode=mode, async_steps=async_steps)
    try:
        g.load(n, _t(s), _t(d))
        g.decompose()
        assert (g.cores() == 2).all()
        cut = (np.array([n - 1], np.int32), np.array([0], np.int32))
        st = g.delete_edges(_t(cut[0]), _t(cut[1]))
        assert (g.cores() == 1).all() and st.changed == n
        st = g.insert_edges(_t(cut[0]), _t(cut[1]))
        assert (g.cores() == 2).all() and st.changed == n
    finally:
        g.close()


def test_serving_idles_longer_than_the_old_wait_bound(cm, oracle_mod):
    """A serving launch whose idle limit (3 s) exceeds a second: the launch
    waits for the host well past a second between two requests while every
    other workgroup sits at the grid barrier; both requests must apply."""
    from paper_1612_09368_amd import serve
    rng = graphgen.rng_for("serve-idle")
    n = 5000
    s, d = graphgen.er_graph(n, 20000, rng)
    es = graphgen.EdgeSet(s, d)
    ref = oracle_mod.DynamicGraph(n, s, d)
    g = cm.Graph(mode=cm.MODE_PERSISTENT)
    try:
        g.load(n, _t(s), _t(d))
        g.decompose()
        srv = serve.Server(g, ring_items=1 << 16, max_items=1 << 14, idle_ms=3000)
        a, b = graphgen.uniform_non_edges(n, 300, es, rng)
        es.insert(a, b)
        t1 = srv.submit_edges(cm.REQ_INSERT_EDGES, a, b)
        ref.insert_edges(a, b)
        while srv.poll() <= t1:
            time.sleep(0.001)
        time.sleep(1.8)  # the launch idles, waiting for the next request
        x, y = graphgen.existing_edges(300, es, rng)
        t2 = srv.submit_edges(cm.REQ_DELETE_EDGES, x, y)
        ref.delete_edges(x, y)
        while srv.poll() <= t2:
            time.sleep(0.001)
        assert srv.result(t1).status == 0 and srv.result(t2).status == 0
        srv.stop()
        assert np.array_equal(g.cores(), ref.cores())
    finally:
        g.close()
