"""Parity on the paper's scalability graphs (Section VII): ER, Barabasi-Albert
and R-MAT with n = 2^15 .. 2^17 and m/n = 8 (BA: every vertex at core 8, the
paper's worst case), 10^4 random edge insertions as one batch and then 10^4
random deletions as one batch, with superior edge sets and in the sequential
regime (one edge per iteration); the full core vector is compared with the
oracle after each batch, and the sequential regime must take one iteration
per edge."""
import numpy as np
import pytest

import graphgen

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

UPDATES = 10_000


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


def _graph(kind, sc):
    rng = graphgen.rng_for(f"sweep-{kind}-{sc}")
    n = 1 << sc
    if kind == "er":
        s, d = graphgen.er_graph(n, 8 * n, rng)
    elif kind == "ba":
        s, d = graphgen.ba_graph_blocks(n, 8, rng)
    else:
        n, s, d = graphgen.rmat_graph(sc, 8, rng)
    es = graphgen.EdgeSet(s, d)
    ins = graphgen.uniform_non_edges(n, UPDATES, es, rng)
    es.insert(*ins)
    dl = graphgen.existing_edges(UPDATES, es, rng)
    return n, s, d, ins, dl


@pytest.mark.parametrize("regime", ["superior", "sequential"])
@pytest.mark.parametrize("kind", ["er", "ba", "rmat"])
@pytest.mark.parametrize("sc", [15, 16, 17])
def test_scalability_graphs(cm, oracle_mod, kind, sc, regime):
    n, s, d, ins, dl = _graph(kind, sc)
    ref = oracle_mod.DynamicGraph(n, s, d)
    g = cm.Graph(mode=cm.MODE_PERSISTENT, single_edge=regime == "sequential")
    try:
        g.load(n, _t(s), _t(d))
        g.decompose()
        c0 = g.cores()
        assert np.array_equal(c0, ref.cores())
        if kind == "ba":
            assert c0.max() == 8 and (c0 == 8).mean() > 0.99
        for inserting, (a, b) in ((True, ins), (False, dl)):
            st = (g.insert_edges if inserting else g.delete_edges)(_t(a), _t(b))
            (ref.insert_edges if inserting else ref.delete_edges)(a, b)
            assert st.applied == UPDATES
            if regime == "sequential":
                assert st.iterations == UPDATES
            else:
                assert st.iterations < UPDATES
            got, want = g.cores(), ref.cores()
            bad = np.nonzero(got != want)[0]
            assert bad.size == 0, f"{'insert' if inserting else 'delete'}: {bad.size} cores differ, first {bad[:5]}"
    finally:
        g.close()
