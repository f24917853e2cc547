"""Continuous batching across sessions: requests of independent sessions
(disjoint graphs packed into one handle) that wait together run fused in one
served batch.  Every request's own result -- status, applied count and its
changed-vertex delta (each moved vertex with its new core number) -- must be
the same when it runs alone (fuse = 1) and in the mix (fuse = 16), and equal
to the oracle's, which applies the requests one by one; the final core
numbers too.  The delta of a request is read from the debug log: the core
changes stamped with its batch's iterations, restricted to its session's
vertices (a fused batch's iterations are shared, and a disjoint union's
members cannot move each other's cores)."""
import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu

ROUNDS = 6


@pytest.fixture(scope="module")
def cm():
    import torch
    assert torch.cuda.is_available()
    import paper_1612_09368_amd as cm
    cm.library()
    return cm


def _workload(cm):
    rng = graphgen.rng_for("serve-fused")
    graphs = []
    for i in range(10):
        kind = i % 3
        if kind == 0:
            n = int(rng.integers(1500, 5000))
            s, d = graphgen.er_graph(n, 5 * n, rng)
        elif kind == 1:
            n = int(rng.integers(2000, 6000))
            s, d = graphgen.chung_lu_graph(n, 6 * n, 2.3, 0.05 * n, rng)
        else:
            n, s, d = graphgen.rmat_graph(11, 8, rng)
        graphs.append((n, s, d))
    base, us, ud = cm.union_edges(graphs)
    sets = [graphgen.EdgeSet(s, d) for _, s, d in graphs]
    reqs, sess = [], []
    spoiled = {(3, 2), (7, 2)}
    for k in range(ROUNDS):
        for g, (n, s, d) in enumerate(graphs):
            size = int(rng.integers(5, 400))
            if k % 2 == 0:
                a, b = graphgen.uniform_non_edges(n, size, sets[g], rng)
            else:
                a, b = graphgen.existing_edges(size, sets[g], rng)
            if (g, k) in spoiled:
                a = a.copy()
                a[-1] = b[-1]  # self-loop: the request is invalid and changes nothing
            elif k % 2 == 0:
                sets[g].insert(a, b)
            else:
                sets[g].delete(a, b)
            reqs.append(("ins" if k % 2 == 0 else "del", (a + base[g]).astype(np.int32),
                         (b + base[g]).astype(np.int32)))
            sess.append(g)
        if k == 2:
            # a vertex insertion in session 5 (two new vertices joined to its ids)
            g = 5
            nb = (rng.choice(graphs[g][0], 12, replace=False) + base[g]).astype(np.int32)
            reqs.append(("vins", np.array([0, 5, 12], np.int64), nb))
            sess.append(-1)
        if k == 3:
            # a vertex deletion in session 8 of two ids no later request uses
            g = 8
            reqs.append(("vdel", None))
            sess.append(-1)
    # ids for the deletion: untouched by the requests after it
    at = next(i for i, r in enumerate(reqs) if r[0] == "vdel")
    later = np.concatenate([np.concatenate([r[1], r[2]]) for r in reqs[at + 1:] if r[0] in ("ins", "del")])
    cand = np.setdiff1d(np.arange(base[8], base[9]), later)[:2].astype(np.int32)
    reqs[at] = ("vdel", cand)
    return int(base[-1]), us, ud, base, reqs, sess


def _oracle_run(oracle_mod, n, us, ud, reqs):
    ref = oracle_mod.DynamicGraph(n, us, ud)
    out = []
    before = ref.cores()
    for r in reqs:
        if r[0] == "ins":
            st = ref.insert_edges(r[1], r[2])[0]
        elif r[0] == "del":
            st = ref.delete_edges(r[1], r[2])[0]
        elif r[0] == "vins":
            st = ref.insert_vertices(r[1], r[2], keep_failed_ids=True)[0]
        else:
            st = ref.delete_vertices(r[1])[0]
        after = ref.cores()
        m = min(before.size, after.size)
        moved = np.nonzero((before[:m] != after[:m]) & (before[:m] >= 0) & (after[:m] >= 0))[0]
        out.append((st, {int(v): int(after[v]) for v in moved}))
        before = after
    return out, ref.cores()


def _served(cm, n, us, ud, reqs, sess, fuse):
    from paper_1612_09368_amd import serve
    g = cm.Graph(mode=cm.MODE_PERSISTENT, debug=1)
    try:
        g.load(n, us, ud)
        g.decompose()
        srv = serve.Server(g, ring_items=1 << 18, max_items=1 << 16, fuse=fuse)
        res = serve.run_stream(srv, reqs, None, sessions=sess)
        srv.stop()
        _, chg = g.debug_log()
        return res["stats"], chg, g.cores()
    finally:
        g.close()


def _delta(st, chg, members, alive_before, alive_after):
    lo, hi = st.first_stamp, st.first_stamp + st.iterations
    sel = chg[(chg[:, 0] >= lo) & (chg[:, 0] < hi)]
    sel = sel[np.argsort(sel[:, 0], kind="stable")]
    out = {}
    for _, v, c in sel.tolist():
        if members(v) and v < alive_before.size and alive_before[v] and alive_after[v]:
            out[v] = c
    return out


def test_fused_serving_results_equal_alone_and_oracle(cm, oracle_mod):
    n, us, ud, base, reqs, sess = _workload(cm)
    want, final = _oracle_run(oracle_mod, n, us, ud, reqs)
    runs = {}
    for fuse in (1, 16):
        stats, chg, cores = _served(cm, n, us, ud, reqs, sess, fuse)
        assert np.array_equal(cores, final), f"fuse {fuse}: final cores differ from the oracle"
        runs[fuse] = (stats, chg)
    groups = [st.group for st in runs[16][0]]
    assert max(groups) > 1, "no request was fused"
    assert max(st.group for st in runs[1][0]) == 1
    # per-request deltas: alive masks before / after each request from the oracle replay
    ref = oracle_mod.DynamicGraph(n, us, ud)
    for i, r in enumerate(reqs):
        alive_before = ref.alive.copy()
        if r[0] == "ins":
            ref.insert_edges(r[1], r[2])
        elif r[0] == "del":
            ref.delete_edges(r[1], r[2])
        elif r[0] == "vins":
            ref.insert_vertices(r[1], r[2], keep_failed_ids=True)
        else:
            ref.delete_vertices(r[1])
        alive_after = ref.alive
        if sess[i] >= 0:
            lo, hi = int(base[sess[i]]), int(base[sess[i] + 1])
            members = (lambda v, lo=lo, hi=hi: lo <= v < hi)
        else:
            members = (lambda v: True)
        st_w, d_w = want[i]
        for fuse in (1, 16):
            st = runs[fuse][0][i]
            assert st.status == st_w, f"request {i} (fuse {fuse}): status {st.status}, oracle {st_w}"
            if r[0] in ("ins", "del"):
                assert st.applied == (r[1].size if st_w == 0 else 0), f"request {i} (fuse {fuse})"
            got = _delta(st, runs[fuse][1], members, alive_before, alive_after)
            assert got == d_w, (f"request {i} ({r[0]}, session {sess[i]}, fuse {fuse}, group {st.group}): "
                                f"delta differs from the oracle ({len(got)} vs {len(d_w)} vertices)")
