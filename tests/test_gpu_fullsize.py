"""Full-size parity of the HIP path with the CPU oracle on the benchmark's
default workload: R-MAT scale 22 (edge factor 16, (a, b, c, d) = (.57, .19,
.19, .05), deduplicated, loops dropped, ids relabelled) and its stream of 64
batches with sizes log-uniform in [1,000, 1,000,000], half R-MAT-sampled
insertions and half uniform deletions, shuffled -- the same seeded stream
``bench.py`` times, run in the launch configuration it times.

Every check compares the full core vector with the oracle's Batagelj-Zaversnik
recomputation (exact core numbers after every update, Section III problem
statement) and the full maintained SD vector with its definition (superior
degree, Section IV-B) on the oracle's cores.
"""
import os
import sys
import time

import numpy as np
import pytest

import graphgen

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

RM_SCALE, RM_BATCHES, RM_LO, RM_HI = 22, 64, 1000, 1_000_000
GROUP = 8            # batches per cm_run_batches call in the batched form
PLAIN_CHECKED = 8    # leading batches run one call each in the plain form
WORKERS = max(1, min(16, os.cpu_count() or 1))


def progress(msg):
    """Progress line outside pytest's capture (long fixture work)."""
    sys.__stderr__.write(f"[fullsize] {msg}\n")
    sys.__stderr__.flush()


def sd_definition(n, s, d, core):
    """SD(v) = #{w in N(v) : core(w) >= core(v)}; dead ids report 0."""
    s = s.astype(np.int64)
    d = d.astype(np.int64)
    sd = np.bincount(s, weights=(core[d] >= core[s]), minlength=n)
    sd += np.bincount(d, weights=(core[s] >= core[d]), minlength=n)
    sd[core < 0] = 0
    return sd.astype(np.int32)


@pytest.fixture(scope="module")
def cm():
    import torch
    assert torch.cuda.is_available()
    import paper_1612_09368_amd as cm
    cm.library()
    return cm


@pytest.fixture(scope="module")
def rmat22(oracle_mod):
    """The stream plus the oracle's (cores, SD) after batch j for every j
    that a test checks (0 = the loaded graph)."""
    t = time.time()
    n, s, d, kinds, offs, xs, ys = graphgen.rmat_stream(
        RM_SCALE, RM_BATCHES, RM_LO, RM_HI, graphgen.rng_for("bench-rmat22"), workers=WORKERS)
    progress(f"stream generated in {time.time() - t:.0f}s: m={s.size}, {int(offs[-1])} updates")
    ref = oracle_mod.DynamicGraph(n, s, d)
    check = {0} | set(range(1, PLAIN_CHECKED + 1)) | set(range(GROUP, RM_BATCHES + 1, GROUP))
    states = {}

    def snap(j):
        c = ref.cores()
        es, ed = ref.edges()
        states[j] = (c, sd_definition(n, es, ed, c), ref.num_edges())

    snap(0)
    for j in range(RM_BATCHES):
        a, b = xs[offs[j]:offs[j + 1]], ys[offs[j]:offs[j + 1]]
        st = (ref.insert_edges if kinds[j] == 0 else ref.delete_edges)(a, b)
        assert st[0] == 0, f"stream batch {j} is invalid for the oracle"
        if j + 1 in check:
            snap(j + 1)
    progress(f"oracle states ready after {time.time() - t:.0f}s")
    return dict(n=n, s=s, d=d, kinds=kinds, offs=offs, xs=xs, ys=ys, states=states)


def bench_params(cm, w):
    from paper_1612_09368_amd import autotune
    params, _ = autotune.params_for(w["n"], w["s"].size, np.diff(w["offs"]))
    return params


def compare(g, w, j, tag):
    core, sd, m = w["states"][j]
    got = g.cores()
    bad = np.nonzero(got != core)[0]
    assert bad.size == 0, (f"{tag}: after batch {j} {bad.size} cores differ, first {bad[:5]} "
                           f"got {got[bad[:5]]} want {core[bad[:5]]}")
    gsd = g.superior_degrees()
    bad = np.nonzero(gsd != sd)[0]
    assert bad.size == 0, f"{tag}: after batch {j} SD differs at {bad[:5]} got {gsd[bad[:5]]} want {sd[bad[:5]]}"
    assert g.num_edges() == m, tag


def load(cm, w, torch, **kw):
    g = cm.Graph(**kw)
    dev = torch.device("cuda:0")
    g.load(w["n"], torch.from_numpy(w["s"]).to(dev), torch.from_numpy(w["d"]).to(dev))
    g.decompose()
    return g


# launch parameters on top of the tuned ones: as timed, and each other
# expansion form that keeps state across batches
STREAM_FORMS = {"tuned": {}, "sublists": {"expand_mode": 3}}


@pytest.mark.parametrize("form", list(STREAM_FORMS))
def test_rmat22_stream_batched(cm, rmat22, form):
    """The whole stream through cm_run_batches in the persistent form
    replayed from a hipGraph (as timed), GROUP batches per call, the full
    core and SD vectors compared after every call."""
    import torch
    w = rmat22
    dev = torch.device("cuda:0")
    params = {**bench_params(cm, w), **STREAM_FORMS[form]}
    g = load(cm, w, torch, mode=cm.MODE_PERSISTENT, use_graph=True, timing=True, **params)
    try:
        compare(g, w, 0, "decomposition")
        dx = torch.from_numpy(w["xs"]).to(dev)
        dy = torch.from_numpy(w["ys"]).to(dev)
        offs = w["offs"]
        for j0 in range(0, RM_BATCHES, GROUP):
            j1 = j0 + GROUP
            lo, hi = int(offs[j0]), int(offs[j1])
            res, _ = g.run_batches(w["kinds"][j0:j1], offs[j0:j1 + 1] - lo, dx[lo:hi], dy[lo:hi])
            assert all(r.status == 0 for r in res), [r.status for r in res]
            assert [r.applied for r in res] == np.diff(offs[j0:j1 + 1]).tolist()
            assert res[0].graph_launch == 1
            compare(g, w, j1, "batched")
            progress(f"batched: batches {j0}..{j1 - 1} match the oracle")
    finally:
        g.close()


def test_rmat22_stream_plain_leading_batches(cm, rmat22):
    """The first PLAIN_CHECKED batches in the plain form (one cooperative
    launch per superior edge set), one call per batch, checked after each."""
    import torch
    w = rmat22
    dev = torch.device("cuda:0")
    g = load(cm, w, torch, mode=cm.MODE_PLAIN, timing=True, **bench_params(cm, w))
    try:
        offs = w["offs"]
        for j in range(PLAIN_CHECKED):
            a = torch.from_numpy(w["xs"][offs[j]:offs[j + 1]]).to(dev)
            b = torch.from_numpy(w["ys"][offs[j]:offs[j + 1]]).to(dev)
            st = (g.insert_edges if w["kinds"][j] == 0 else g.delete_edges)(a, b)
            assert st.applied == offs[j + 1] - offs[j]
            compare(g, w, j + 1, "plain")
        progress(f"plain: batches 0..{PLAIN_CHECKED - 1} match the oracle")
    finally:
        g.close()


POOL_COUNT = 512


@pytest.fixture(scope="module")
def pool512(oracle_mod):
    """The benchmark's 512 Chung-Lu graphs (n log-uniform in [1000, 200000],
    mean degree U[4, 32], exponent 2.3), each with an insertion batch and a
    deletion batch of 5% of its edges, plus the oracle's cores of every
    member after its insertion batch and after its deletion batch (members
    in parallel threads; BZ releases the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    t = time.time()
    pool = graphgen.chung_lu_pool(POOL_COUNT, graphgen.rng_for("bench-pool512"), workers=WORKERS)
    progress(f"pool generated in {time.time() - t:.0f}s")

    def member(m):
        n, s, d, ins, dele = m
        ref = oracle_mod.DynamicGraph(n, s, d)
        assert ref.insert_edges(*ins)[0] == 0
        c1 = ref.cores()
        assert ref.delete_edges(*dele)[0] == 0
        return c1, ref.cores()

    with ThreadPoolExecutor(max_workers=WORKERS) as ex:
        states = list(ex.map(member, pool))
    progress(f"pool oracle ready after {time.time() - t:.0f}s")
    return pool, states


def test_pool512_every_member(cm, pool512):
    """The 512 graphs packed as one disjoint union, every member batch a
    sub-batch: stage 1 (all insertion batches) and stage 2 (all deletion
    batches) as two calls, each member's cores compared with the oracle
    after each stage; then both stages in one call replayed from a hipGraph
    (as timed) on a fresh handle, compared at the end."""
    import torch
    pool, states = pool512
    dev = torch.device("cuda:0")
    graphs = [(n, s, d) for n, s, d, _, _ in pool]
    batches = []
    for gid, (_, _, _, ins, dele) in enumerate(pool):
        batches.append((gid, cm.BATCH_INSERT, ins[0], ins[1]))
        batches.append((gid, cm.BATCH_DELETE, dele[0], dele[1]))
    base, us, ud = cm.union_edges(graphs)
    kinds, offs, xs, ys, sub, nsub, order = cm.pack_batches(base, batches)
    assert kinds.tolist() == [cm.BATCH_INSERT, cm.BATCH_DELETE]
    want = [np.concatenate([st[k] for st in states]) for k in (0, 1)]
    dus, dud, dx, dy, dsub = (torch.from_numpy(z).to(dev) for z in (us, ud, xs, ys, sub))
    from paper_1612_09368_amd import autotune
    params, _ = autotune.params_for(int(base[-1]), us.size, [b[2].size for b in batches])

    def load():
        g = cm.Graph(mode=cm.MODE_PERSISTENT, use_graph=True, timing=True, **params)
        g.load(int(base[-1]), dus, dud)
        g.decompose()
        return g

    g = load()
    try:
        for stage in (0, 1):
            lo, hi = int(offs[stage]), int(offs[stage + 1])
            res, sst = g.run_batches(kinds[stage:stage + 1], np.array([0, hi - lo], np.int64), dx[lo:hi],
                                     dy[lo:hi], sub=dsub[lo:hi], nsub=nsub)
            assert res[0].status == 0 and (sst == 0).all()
            got = g.cores()
            bad = np.nonzero(got != want[stage])[0]
            assert bad.size == 0, (f"stage {stage}: {bad.size} cores differ, first in graph "
                                   f"{np.searchsorted(base, bad[0], side='right') - 1}")
            progress(f"pool stage {stage}: every member matches the oracle")
    finally:
        g.close()
    g = load()
    try:
        res, sst = g.run_batches(kinds, offs, dx, dy, sub=dsub, nsub=nsub)
        assert all(r.status == 0 for r in res) and (sst == 0).all() and res[0].graph_launch == 1
        assert np.array_equal(g.cores(), want[1])
    finally:
        g.close()
