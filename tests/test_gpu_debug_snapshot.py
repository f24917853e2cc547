"""Debug-mode replay and checkpoint / restore, through the C ABI.

Replay: with cfg.debug the library logs every superior edge set it applied
and every core change it made, iteration by iteration.  The test replays the
sets on the host: G_i = G_{i-1} plus (minus) S_i.  It checks that

- S_i is a superior edge set (Section IV, definition of the k-superior edge
  set: each edge's endpoints with the edge's core number k = min(core u,
  core v) take no other edge of the set) and not empty (progress);
- the cores after iteration i equal the oracle's BZ(G_i) -- each iteration
  ends at the exact core numbers of G_i (lemmas and theorems on superior
  edge set insertion and deletion, Section IV-A);
- every core moved by exactly one, in the batch's direction, and only at a
  level k of an edge of S_i;
- the sets partition the valid batch.

Checkpoint: cm_snapshot in the middle of an update stream, cm_restore into a
new handle, and both handles continue; cores, SD and edge sets stay bit-exact
to each other and to the oracle after every batch.
"""
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


def sd_definition(n, s, d, core):
    s = s.astype(np.int64)
    d = d.astype(np.int64)
    sd = np.bincount(s, weights=(core[d] >= core[s]), minlength=n)
    sd += np.bincount(d, weights=(core[s] >= core[d]), minlength=n)
    sd[core < 0] = 0
    return sd.astype(np.int32)


def replay(oracle_mod, n, keys0, cores0, batch_keys, inserting, sel, chg, single_edge=False):
    """Check the iteration log of one edge batch against the oracle; returns
    the number of iterations."""
    keys = set(keys0.tolist())
    cores = cores0.copy()
    stamps = np.unique(sel[:, 0])
    assert set(np.unique(chg[:, 0]).tolist()) <= set(stamps.tolist()), "a core moved outside every iteration"
    done = set()
    for ep in stamps.tolist():
        S = sel[sel[:, 0] == ep][:, 1:].astype(np.int64)
        assert S.shape[0] >= 1
        if single_edge:
            assert S.shape[0] == 1, f"iteration {ep}: {S.shape[0]} edges in the sequential regime"
        assert (S[:, 0] < S[:, 1]).all()
        cu, cv = cores[S[:, 0]], cores[S[:, 1]]
        k = np.minimum(cu, cv)
        constrained = np.concatenate([S[cu == k, 0], S[cv == k, 1]])
        assert np.unique(constrained).size == constrained.size, \
            f"iteration {ep}: a constrained endpoint has two edges of the set"
        sk = ((S[:, 0] << 32) | S[:, 1]).tolist()
        assert not (set(sk) & done), f"iteration {ep}: an edge was selected twice"
        done |= set(sk)
        for key in sk:
            if inserting:
                assert key not in keys
                keys.add(key)
            else:
                assert key in keys
                keys.remove(key)
        C = chg[chg[:, 0] == ep][:, 1:]
        assert np.unique(C[:, 0]).size == C.shape[0], f"iteration {ep}: a vertex moved twice"
        old = cores[C[:, 0]]
        step = 1 if inserting else -1
        assert (C[:, 1] - old == step).all(), f"iteration {ep}: a core moved by other than {step}"
        assert set(old.tolist()) <= set(k.tolist()), f"iteration {ep}: a core moved outside the set's levels"
        cores[C[:, 0]] = C[:, 1]
        karr = np.fromiter(keys, dtype=np.int64, count=len(keys))
        want = oracle_mod.bz_cores(n, (karr >> 32).astype(np.int32), (karr & 0xFFFFFFFF).astype(np.int32))
        bad = np.nonzero(cores != want)[0]
        assert bad.size == 0, f"iteration {ep}: cores differ from BZ(G_i) at {bad[:5]}"
    assert done == set(batch_keys.tolist()), "the selected sets do not partition the batch"
    return stamps.size


def _case(kind, seed):
    rng = graphgen.rng_for(f"debug-{kind}-{seed}")
    if kind == "er":
        n, m = 10_000, 50_000
        s, d = graphgen.er_graph(n, m, rng)
        es = graphgen.EdgeSet(s, d)
        ins = graphgen.uniform_non_edges(n, 1000, es, rng)
    elif kind == "rmat":
        n, s, d = graphgen.rmat_graph(12, 8, rng)
        es = graphgen.EdgeSet(s, d)
        ins = graphgen.rmat_non_edges(12, 2000, es, rng)
    else:  # tiny dense graphs: adjacent levels in one set
        n = 40
        s, d = graphgen.er_graph(n, 150, rng)
        es = graphgen.EdgeSet(s, d)
        ins = graphgen.uniform_non_edges(n, 120, es, rng)
    es.insert(*ins)
    dl = graphgen.existing_edges(ins[0].size, es, rng)
    return n, s, d, ins, dl


@pytest.mark.parametrize("mode", [0, 1], ids=["plain", "persistent"])
@pytest.mark.parametrize("kind,seed", [("er", 0), ("rmat", 0), ("tiny", 0), ("tiny", 1), ("tiny", 2),
                                       ("tiny", 3)])
@pytest.mark.parametrize("async_steps", [False, True], ids=["rounds", "async"])
def test_iteration_replay(cm, oracle_mod, mode, kind, seed, async_steps):
    n, s, d, ins, dl = _case(kind, seed)
    ref = oracle_mod.DynamicGraph(n, s, d)
    g = cm.Graph(mode=mode, debug=1, async_steps=async_steps)
    try:
        g.load(n, _t(s), _t(d))
        g.decompose()
        for inserting, (a, b) in ((True, ins), (False, dl)):
            keys0 = ref.keys
            cores0 = g.cores()
            st = (g.insert_edges if inserting else g.delete_edges)(_t(a), _t(b))
            sel, chg = g.debug_log()
            (ref.insert_edges if inserting else ref.delete_edges)(a, b)
            iters = replay(oracle_mod, n, keys0, cores0, graphgen.keys_of(a, b), inserting, sel, chg)
            assert iters == st.iterations
            assert np.array_equal(g.cores(), ref.cores())
    finally:
        g.close()


def test_iteration_replay_single_edge(cm, oracle_mod):
    n, s, d, ins, dl = _case("er", 1)
    ref = oracle_mod.DynamicGraph(n, s, d)
    g = cm.Graph(mode=1, debug=1, single_edge=True)
    try:
        g.load(n, _t(s), _t(d))
        g.decompose()
        # deletions among the edges present after the 200 insertions
        keep = np.isin(graphgen.keys_of(*dl), np.concatenate([graphgen.keys_of(s, d),
                                                               graphgen.keys_of(ins[0][:200], ins[1][:200])]))
        dl = (dl[0][keep], dl[1][keep])
        for inserting, (a, b) in ((True, (ins[0][:200], ins[1][:200])), (False, (dl[0][:200], dl[1][:200]))):
            keys0 = ref.keys
            cores0 = g.cores()
            (g.insert_edges if inserting else g.delete_edges)(_t(a), _t(b))
            sel, chg = g.debug_log()
            (ref.insert_edges if inserting else ref.delete_edges)(a, b)
            assert replay(oracle_mod, n, keys0, cores0, graphgen.keys_of(a, b), inserting, sel, chg,
                          single_edge=True) == a.size
    finally:
        g.close()


def test_debug_log_batches_and_capacity(cm, oracle_mod):
    """A batch program logs every batch's sets (stamps keep growing across
    batches); a log too small for a call reports CM_E_CAPACITY."""
    n, s, d, ins, dl = _case("er", 2)
    g = cm.Graph(mode=1, debug=1)
    try:
        g.load(n, _t(s), _t(d))
        g.decompose()
        kinds = np.array([0, 1], np.int32)
        offs = np.array([0, ins[0].size, ins[0].size + dl[0].size], np.int64)
        res, _ = g.run_batches(kinds, offs, _t(np.concatenate([ins[0], dl[0]])),
                               _t(np.concatenate([ins[1], dl[1]])))
        sel, chg = g.debug_log()
        assert sel.shape[0] == ins[0].size + dl[0].size
        assert np.unique(sel[:, 0]).size == res[0].iterations + res[1].iterations
    finally:
        g.close()
    g = cm.Graph(mode=0, debug=16)
    try:
        g.load(n, _t(s), _t(d))
        g.decompose()
        g.insert_edges(_t(ins[0]), _t(ins[1]))
        with pytest.raises(cm.CoreMaintError) as e:
            g.debug_log()
        assert e.value.status == cm.E_CAPACITY
    finally:
        g.close()


def _stream(seed, n=4000, m=16000):
    rng = graphgen.rng_for(f"snapshot-{seed}")
    s, d = graphgen.er_graph(n, m, rng)
    es = graphgen.EdgeSet(s, d)
    ops = []
    for j in range(6):
        if j % 2 == 0:
            a, b = graphgen.uniform_non_edges(n, 600, es, rng)
            es.insert(a, b)
            ops.append(("ins", a, b))
        else:
            a, b = graphgen.existing_edges(600, es, rng)
            es.delete(a, b)
            ops.append(("del", a, b))
    return n, s, d, ops, rng


def _check_same(g, g2, ref, tag):
    c1, c2 = g.cores(), g2.cores()
    assert np.array_equal(c1, c2), tag
    assert np.array_equal(c1, ref.cores()), tag
    es, ed = ref.edges()
    want_sd = sd_definition(ref.n, es, ed, c1)
    assert np.array_equal(g.superior_degrees(), want_sd), tag
    assert np.array_equal(g2.superior_degrees(), want_sd), tag
    x1 = np.sort(graphgen.keys_of(*g.export_edges()))
    x2 = np.sort(graphgen.keys_of(*g2.export_edges()))
    assert np.array_equal(x1, x2) and np.array_equal(x1, ref.keys), tag
    assert g.num_vertices() == g2.num_vertices(), tag


@pytest.mark.parametrize("mode2", [0, 1], ids=["restored-plain", "restored-persistent"])
def test_snapshot_restore_continues_bit_exact(cm, oracle_mod, tmp_path, mode2):
    n, s, d, ops, rng = _stream(0)
    ref = oracle_mod.DynamicGraph(n, s, d)
    g = cm.Graph(mode=0)
    g2 = None
    try:
        g.load(n, _t(s), _t(d))
        g.decompose()
        for kind, a, b in ops[:3]:
            (g.insert_edges if kind == "ins" else g.delete_edges)(_t(a), _t(b))
            (ref.insert_edges if kind == "ins" else ref.delete_edges)(a, b)
        # vertex operations leave dead and fresh ids in the snapshot
        off = np.array([0, 3, 5], np.int64)
        nb = np.array([1, 2, 3, 4, 5], np.int32)
        g.insert_vertices(off, nb)
        ref.insert_vertices(off, nb)
        # ids that no later batch touches
        later = np.concatenate([np.concatenate([a, b]) for _, a, b in ops[3:]])
        gone = np.setdiff1d(np.arange(6, n), later)[:3].astype(np.int32)
        assert gone.size == 3
        g.delete_vertices(gone)
        ref.delete_vertices(gone)
        path = tmp_path / "mid.snap"
        g.snapshot(path)
        g2 = cm.Graph.restore(path, mode=mode2)
        _check_same(g, g2, ref, "restored")
        for j, (kind, a, b) in enumerate(ops[3:]):
            for h in (g, g2):
                (h.insert_edges if kind == "ins" else h.delete_edges)(_t(a), _t(b))
            (ref.insert_edges if kind == "ins" else ref.delete_edges)(a, b)
            _check_same(g, g2, ref, f"batch {3 + j} after the restore")
        # a snapshot of the restored handle reproduces the same file content
        g.snapshot(tmp_path / "a.snap")
        g2.snapshot(tmp_path / "b.snap")
        g3 = cm.Graph.restore(tmp_path / "b.snap")
        try:
            _check_same(g, g3, ref, "second restore")
        finally:
            g3.close()
    finally:
        g.close()
        if g2 is not None:
            g2.close()


def test_restore_empty_and_corrupt(cm, tmp_path):
    g = cm.Graph()
    try:
        g.load(5, np.empty(0, np.int32), np.empty(0, np.int32))
        g.decompose()
        g.snapshot(tmp_path / "e.snap")
    finally:
        g.close()
    g2 = cm.Graph.restore(tmp_path / "e.snap")
    try:
        assert g2.cores().tolist() == [0] * 5
        g2.insert_edges(np.array([0, 0, 1], np.int32), np.array([1, 2, 2], np.int32))
        assert g2.cores().tolist() == [2, 2, 2, 0, 0]
    finally:
        g2.close()
    data = bytearray((tmp_path / "e.snap").read_bytes())
    data[-1] ^= 1
    (tmp_path / "c.snap").write_bytes(bytes(data))
    with pytest.raises(cm.CoreMaintError) as e:
        cm.Graph.restore(tmp_path / "c.snap")
    assert e.value.status == cm.E_IO
