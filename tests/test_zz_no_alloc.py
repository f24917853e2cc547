"""The allocation-free entry point (cm_update_edges_noalloc) against the
entry points it is a variant of (cm_insert_edges / cm_delete_edges): two
handles on the same graph take the same calls, one through each path; core
numbers, SD, edge counts and the per-call outcome must be identical after
every call, and both must equal the oracle.  Two calls in a row, the second
smaller, then a strict rejection and an oversized batch."""
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


def _same(g1, g2, ref, tag):
    c1, c2 = g1.cores(), g2.cores()
    assert np.array_equal(c1, c2), tag
    assert np.array_equal(c1, ref.cores()), tag
    assert np.array_equal(g1.superior_degrees(), g2.superior_degrees()), tag
    assert g1.num_edges() == g2.num_edges() == ref.num_edges(), tag


@pytest.mark.parametrize("mode", [0, 1], ids=["plain", "persistent"])
def test_noalloc_matches_allocating_entry_points(cm, oracle_mod, mode):
    rng = graphgen.rng_for("noalloc")
    n, m = 30_000, 150_000
    s, d = graphgen.er_graph(n, m, rng)
    es = graphgen.EdgeSet(s, d)
    ins = graphgen.uniform_non_edges(n, 40_000, es, rng)
    es.insert(*ins)
    dl = graphgen.existing_edges(7_000, es, rng)
    ref = oracle_mod.DynamicGraph(n, s, d)
    ga, gb = cm.Graph(mode=mode), cm.Graph(mode=mode)
    try:
        for h in (ga, gb):
            h.load(n, _t(s), _t(d))
            h.decompose()
        # call 1: 40,000 insertions; call 2: 7,000 deletions (smaller)
        for kind, (a, b) in ((cm.BATCH_INSERT, ins), (cm.BATCH_DELETE, dl)):
            da, db = _t(a), _t(b)
            st_a = (ga.insert_edges if kind == cm.BATCH_INSERT else ga.delete_edges)(da, db)
            st_b = gb.update_edges_noalloc(kind, da, db)
            (ref.insert_edges if kind == cm.BATCH_INSERT else ref.delete_edges)(a, b)
            assert st_b.status == 0 and st_b.applied == st_a.applied == a.size
            assert st_b.first_bad == st_a.first_bad == -1
            _same(ga, gb, ref, f"kind {kind}")
        # a strict rejection: same code and index, nothing applied
        a = np.concatenate([dl[0][:50], dl[0][:1]]).astype(np.int32)
        b = np.concatenate([dl[1][:50], dl[1][:1]]).astype(np.int32)
        ra, sa = ga.insert_edges(_t(a), _t(b), check=False)
        rb, sb = gb.update_edges_noalloc(cm.BATCH_INSERT, _t(a), _t(b), check=False)
        assert ra == rb == cm.E_DUP and sa.first_bad == sb.first_bad == 50
        _same(ga, gb, ref, "rejected")
        # oversized: refused before any work
        big = np.zeros(cm_max(cm) + 1, np.int32)
        rb, _ = gb.update_edges_noalloc(cm.BATCH_INSERT, _t(big), _t(big + 1), check=False)
        assert rb == cm.E_CAPACITY
        _same(ga, gb, ref, "oversized")
    finally:
        ga.close()
        gb.close()


def cm_max(cm):
    import os
    import re
    text = open(os.path.join(os.path.dirname(cm.HERE), "include", "coremaint.h")).read()
    return eval(re.search(r"#define CM_NOALLOC_MAX_ITEMS \((.*?)\)", text).group(1))
