"""Serving (continuous batching): every request's outcome and the core
numbers are the oracle's, whether a request runs alone or in a mix of
requests that arrive while others are on the GPU; admission by memory
(busy ring, payload and budget), pool repacks and vertex-capacity growth
during serving keep the results exact."""
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


def _oracle(ref, req):
    """Apply one request to the oracle (serving conventions); returns status."""
    if req[0] == "ins":
        return ref.insert_edges(req[1], req[2])[0]
    if req[0] == "del":
        return ref.delete_edges(req[1], req[2])[0]
    if req[0] == "vins":
        return ref.insert_vertices(req[1], req[2], keep_failed_ids=True)[0]
    return ref.delete_vertices(req[1])[0]


def _stream(scale, nreq, max_size, tag, spoil=()):
    n, s, d, reqs = graphgen.serve_stream(scale, nreq, graphgen.rng_for(tag), max_size=max_size)
    reqs = list(reqs)
    for j in spoil:   # make request j invalid (strict: it must change nothing)
        r = reqs[j]
        if r[0] in ("ins", "del"):
            a = r[1].copy()
            a[-1] = r[2][-1]          # self-loop
            reqs[j] = (r[0], a, r[2])
        elif r[0] == "vdel":
            reqs[j] = ("vdel", np.concatenate([r[1], r[1][:1]]))   # repeated id
        else:
            nb = r[2].copy()
            if nb.size:
                nb[0] = -5            # out of range
            reqs[j] = ("vins", r[1], nb)
    return n, s, d, reqs


def _run_served(cm, n, s, d, reqs, one_at_a_time, async_steps=False, **scfg):
    from paper_1612_09368_amd import serve
    g = cm.Graph(mode=cm.MODE_PERSISTENT, async_steps=async_steps)
    g.load(n, s, d)
    g.decompose()
    cfg = {"ring_items": 1 << 18, "max_items": 1 << 16}
    cfg.update(scfg)
    srv = serve.Server(g, **cfg)
    out = []
    if one_at_a_time:
        for r in reqs:
            res = serve.run_stream(srv, [r])
            out.append(res["stats"][0])
    else:
        res = serve.run_stream(srv, reqs)
        out = res["stats"]
    srv.stop()
    cores = g.cores()
    m = g.num_edges()
    g.close()
    return [(x.status, x.applied, x.changed) for x in out], cores, m


def test_serve_each_request_matches_oracle(cm, oracle_mod):
    from paper_1612_09368_amd import serve
    n, s, d, reqs = _stream(10, 60, 120, "serve-each", spoil=(7, 23, 41))
    ref = oracle_mod.DynamicGraph(n, s, d)
    g = cm.Graph(mode=cm.MODE_PERSISTENT)
    g.load(n, s, d)
    g.decompose()
    for j, r in enumerate(reqs):
        srv = serve.Server(g, idle_ms=5, ring_items=1 << 14, max_items=1 << 13)
        res = serve.run_stream(srv, [r])
        srv.stop()
        st = _oracle(ref, r)
        assert res["stats"][0].status == st, (j, r[0], res["stats"][0].status, st)
        assert np.array_equal(g.cores(), ref.cores()), (j, r[0])
    assert g.num_edges() == ref.num_edges()
    g.close()


@pytest.mark.parametrize("async_steps", [False, True])
def test_serve_mix_equals_alone(cm, oracle_mod, async_steps):
    n, s, d, reqs = _stream(12, 240, 600, "serve-mix", spoil=(5, 77, 150))
    ref = oracle_mod.DynamicGraph(n, s, d)
    want = [_oracle(ref, r) for r in reqs]
    alone, c_alone, m_alone = _run_served(cm, n, s, d, reqs, True, async_steps=async_steps)
    mix, c_mix, m_mix = _run_served(cm, n, s, d, reqs, False, async_steps=async_steps)
    assert [a[0] for a in alone] == want
    assert alone == mix
    assert np.array_equal(c_alone, ref.cores()) and np.array_equal(c_mix, ref.cores())
    assert m_alone == m_mix == ref.num_edges()


def test_serve_admission_waits_and_relaunches(cm, oracle_mod):
    # a 3-slot ring, a small payload ring and budget: submits must wait;
    # idle_ms = 1 lets the launch leave between bursts and come back.
    # max_items also bounds the edges one vertex deletion may gather, so it
    # is kept well above the largest request.
    n, s, d, reqs = _stream(11, 120, 400, "serve-busy")
    ref = oracle_mod.DynamicGraph(n, s, d)
    want = [_oracle(ref, r) for r in reqs]
    big = max(len(r[1]) if r[0] != "vins" else int(r[1][-1]) for r in reqs)
    got, cores, m = _run_served(cm, n, s, d, reqs, False, ring_requests=3, ring_items=16 * big,
                                max_items=16 * big, budget_bytes=64 * big, idle_ms=1)
    assert [x[0] for x in got] == want
    assert np.array_equal(cores, ref.cores()) and m == ref.num_edges()


def test_serve_pool_repack_and_vertex_growth(cm, oracle_mod):
    rng = graphgen.rng_for("serve-grow")
    n = 1500
    s, d = graphgen.er_graph(n, 1500, rng)
    n, s, d, reqs = graphgen.serve_stream(0, 150, rng, max_size=800, mix=(0.6, 0.1, 0.3, 0.0),
                                          graph=(n, s, d), deg_hi=40)
    ref = oracle_mod.DynamicGraph(n, s, d)
    want = [_oracle(ref, r) for r in reqs]
    got, cores, m = _run_served(cm, n, s, d, reqs, False, vertex_headroom=16)
    assert [x[0] for x in got] == want
    assert np.array_equal(cores, ref.cores()) and m == ref.num_edges()


def test_serve_refuses_other_calls(cm):
    from paper_1612_09368_amd import serve
    rng = graphgen.rng_for("serve-state")
    s, d = graphgen.er_graph(500, 2000, rng)
    g = cm.Graph()
    g.load(500, s, d)
    g.decompose()
    srv = serve.Server(g, ring_items=1 << 14, max_items=1 << 13)
    with pytest.raises(cm.CoreMaintError) as e:
        g.cores()
    assert e.value.status == cm.E_STATE
    srv.stop()
    assert g.cores().size == 500
    g.close()


def test_serve_stream_replica_scale18(cm, oracle_mod):
    """The serving workload's stream on a scale-18 R-MAT replica (200
    requests, sizes log-uniform in [1, 10^5], 40% edge insert, 40% edge
    delete, 10% vertex insert, 10% vertex delete), served in 20 chunks, each
    chunk continuously batched: every request's status (and the applied count
    of edge requests) equals the oracle's, and the core numbers equal the
    oracle's at the end of every chunk (20 checkpoints, the last one the final
    state)."""
    from paper_1612_09368_amd import serve
    n, s, d, reqs = graphgen.serve_stream(18, 200, graphgen.rng_for("serve-c5-replica"))
    ref = oracle_mod.DynamicGraph(n, s, d)
    new_ids = sum(len(r[1]) - 1 for r in reqs if r[0] == "vins")
    g = cm.Graph(mode=cm.MODE_PERSISTENT)
    g.load(n, s, d)
    g.decompose()
    assert np.array_equal(g.cores(), ref.cores())
    nchunk = 20
    bounds = np.linspace(0, len(reqs), nchunk + 1).astype(int)
    for c in range(nchunk):
        chunk = reqs[bounds[c]:bounds[c + 1]]
        srv = serve.Server(g, ring_requests=256, ring_items=1 << 24, max_items=1 << 23,
                           vertex_headroom=new_ids + 1024, idle_ms=20)
        res = serve.run_stream(srv, chunk)
        srv.stop()
        for j, (r, x) in enumerate(zip(chunk, res["stats"])):
            if r[0] == "ins":
                want = ref.insert_edges(r[1], r[2])
            elif r[0] == "del":
                want = ref.delete_edges(r[1], r[2])
            elif r[0] == "vins":
                want = ref.insert_vertices(r[1], r[2], keep_failed_ids=True)
            else:
                want = ref.delete_vertices(r[1])
            tag = (c, j, r[0])
            assert x.status == want[0], tag
            if r[0] in ("ins", "del"):
                assert x.applied == want[2], tag
        assert np.array_equal(g.cores(), ref.cores()), f"checkpoint {c}"
    assert g.num_edges() == ref.num_edges()
    g.close()
