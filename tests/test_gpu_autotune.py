"""The autotuner on a small sample: coordinate descent over a reduced space
(expansion form, partition rounds, chunking), results stored and loaded back
by workload signature; every trial must reproduce the first trial's cores
(the tuner refuses otherwise), and the stored parameters must give the
oracle's cores on the whole stream."""
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


def test_tune_store_and_reuse(cm, oracle_mod, tmp_path):
    import torch
    from paper_1612_09368_amd import autotune
    rng = graphgen.rng_for("autotune-test")
    n, s, d = graphgen.rmat_graph(14, 8, rng)
    es = graphgen.DynamicEdgeSet(s, d)
    kinds, xs, ys = [], [], []
    for j in range(6):
        if j % 2 == 0:
            a, b = graphgen.rmat_non_edges(14, 3000, es, rng)
            es.insert(a, b)
        else:
            a, b = graphgen.existing_edges(3000, es, rng)
            es.delete(a, b)
        kinds.append(j % 2)
        xs.append(a)
        ys.append(b)
    offs = np.concatenate([[0], np.cumsum([x.size for x in xs])]).astype(np.int64)
    xs, ys = np.concatenate(xs).astype(np.int32), np.concatenate(ys).astype(np.int32)
    dev = torch.device("cuda:0")
    ds, dd, dx, dy = (torch.from_numpy(z).to(dev) for z in (s, d, xs, ys))
    kinds = np.asarray(kinds, np.int32)
    space = {"expand_mode": [1, 2, 4], "partition_rounds": [1, 2, 3], "large_degree": [64, 256],
             "chunk": [128, 256]}
    best, best_t, trials = autotune.tune(n, ds, dd, kinds, offs, dx, dy, space=space,
                                         order=list(space), sweeps=1)
    assert len(trials) >= 1 + sum(len(v) - 1 for v in space.values())
    key = autotune.signature(n, s.size, np.diff(offs))
    path = str(tmp_path / "tuning.json")
    autotune.save_tuning(key, best, best_t, path=path, note="test")
    params, source = autotune.params_for(n, s.size, np.diff(offs), path=path)
    assert params == best and "tuning.json" in source
    ref = oracle_mod.DynamicGraph(n, s, d)
    for j in range(len(kinds)):
        a, b = xs[offs[j]:offs[j + 1]], ys[offs[j]:offs[j + 1]]
        (ref.insert_edges if kinds[j] == 0 else ref.delete_edges)(a, b)
    g = cm.Graph(mode=cm.MODE_PERSISTENT, **params)
    try:
        g.load(n, ds, dd)
        g.decompose()
        res, _ = g.run_batches(kinds, offs, dx, dy)
        assert all(r.status == 0 for r in res)
        assert np.array_equal(g.cores(), ref.cores())
    finally:
        g.close()
