"""Benchmark: edge updates per second of batched core maintenance on one MI355X.

Workloads (``--workload``; every graph and update stream is seeded and
synthetic, and inputs are resident in device memory before the timed region):

chunglu-1m
    Chung-Lu power-law graph, n = 1,000,000, m = 10,000,000, degree exponent
    2.1, largest weight 50,000.  One step inserts 100,000 degree-weighted
    non-edges and then deletes 100,000 uniformly drawn existing edges, with
    exact core numbers after each batch.  `value` is the plain form (one
    cooperative launch per superior edge set, the host checks termination);
    the persistent form (one launch per batch) and the batched form (every
    timed batch in one launch) run beside it on the same batches.
rmat22-stream (default)
    R-MAT scale 22 (edge factor 16, a=0.57 b=0.19 c=0.19, dedup, no loops,
    random relabel) and 64 batches, sizes log-uniform in [1,000, 1,000,000],
    half R-MAT-sampled insertions, half uniform deletions, shuffled.  One step
    = the whole stream from the freshly loaded graph.  `value` is the batched
    form (one persistent launch replayed from a hipGraph); the plain host
    loop runs beside it.
chunglu-pool512
    512 independent Chung-Lu graphs (n log-uniform in [1,000, 200,000], mean
    degree uniform in [4, 32], exponent 2.3), each with one insertion batch
    of 5% of its edges and then one deletion batch of 5%.  One step = every
    graph's two batches.  `value` is the batched form: the graphs packed as
    one disjoint union, every batch as a sub-batch, one hipGraph launch; the
    plain form runs the 1024 batches one after another.

Prints one JSON line (fields below).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Measured HBM bytes per launch of the dominant kernel, per workload, from two rocprofv3 counter
# passes (FETCH_SIZE, then WRITE_SIZE) scaled by calibration kernels of known footprint; each entry
# names the kernel sources it was measured on and is reported only while their hash matches (the
# summaries and commands are under profiles/).
TRAFFIC = {
    "rmat22-stream": {"kernel": "k_program", "bytes_per_launch": 1717.1e9,
                      "sources_sha256": "6df6baeb8d7b2da9d5ec359367b2947d0c8427066fac50b41d8bb7b7ebd267df"},
}
KERNEL_SOURCES = ["cm_internal.h", "cm_kernels.hip", "cm_phases.h", "cm_walk.h"]


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in sorted(KERNEL_SOURCES):
        with open(os.path.join(ROOT, "paper_1612_09368_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()
METRIC = "edge updates/sec (insert & delete, exact cores) batched vs plain on 1 GPU; p99 latency"
WORKERS = max(1, min(16, os.cpu_count() or 1))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pct(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else 0.0


def contract(workload, value, steps, warmup, ms_per_step, global_batch, form):
    return {
        "metric": METRIC,
        "value": value,
        "unit": "edge_updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": workload, "form": form, "global_batch": global_batch,
                   "parallelism": "single-gpu"},
    }


def roofline(kernel, stats, note, traffic_key=None, method_bytes=None):
    """Algorithmic bytes of the launches over their HIP-event time; the
    measured HBM traffic per launch is attached when it was taken on the
    current kernel sources.  method_bytes (per launch), when given, replaces
    the bytes the timed launches counted: the method's own bytes counted on
    a pass that visits exactly Algorithm 3's sets."""
    kms = sum(x["kernel_ms"] for x in stats)
    launches = sum(x["launches"] for x in stats)
    abytes = sum(x["alg_bytes"] for x in stats) if method_bytes is None else method_bytes * launches
    achieved = (abytes / (kms * 1e-3)) / 1e9 if kms > 0 else 0.0
    out = {
        "bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS, "traffic": None,
        "alg_bytes_per_launch": abytes / max(launches, 1),
        "avg_launch_us": kms * 1e3 / max(launches, 1), "launches": launches, "per_launch": note,
    }
    tr = TRAFFIC.get(traffic_key)
    if tr is not None and tr["kernel"] == kernel:
        if tr["sources_sha256"] == kernel_sources_sha256():
            out["traffic"] = tr["bytes_per_launch"]
            out["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)"
            out["traffic_gbs"] = tr["bytes_per_launch"] / (out["avg_launch_us"] * 1e-6) / 1e9
            out["traffic_frac"] = out["traffic_gbs"] / HBM_PEAK_GBS
            out["traffic_over_alg"] = tr["bytes_per_launch"] / max(out["alg_bytes_per_launch"], 1.0)
        else:
            out["traffic_note"] = "kernel sources changed since the counters were taken"
    return out


def to_dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def tuned_params(args, n, m, batch_sizes, sample):
    """Launch and work-split parameters for this workload: tuned now
    (--tune, on `sample` = a function returning the tuning sample), else the
    stored entry for the workload's signature, else the library defaults."""
    from paper_1612_09368_amd import autotune
    key = autotune.signature(n, m, batch_sizes)
    params, info = _tuned_params(args, key, sample)
    if args.set:
        over = json.loads(args.set)
        params = {**params, **over}
        info = {**info, "params": params, "overrides": over}
    return params, info


def _tuned_params(args, key, sample):
    from paper_1612_09368_amd import autotune
    if args.tune and sample is not None:
        t0 = time.time()
        best, bt, trials = autotune.tune(*sample(), sweeps=2, log=log, budget_s=args.tune_budget)
        autotune.save_tuning(key, best, bt, note=f"{len(trials)} trials on the workload's tuning sample")
        return best, {"source": "tuned in this run", "key": key, "trials": len(trials),
                      "tune_s": time.time() - t0, "params": best}
    stored = autotune.load_tuning(key)
    if stored is not None:
        return stored, {"source": "tuning.json", "key": key, "params": stored}
    return dict(autotune.DEFAULTS), {"source": "library defaults", "key": key,
                                     "params": dict(autotune.DEFAULTS)}


# ---------------------------------------------------------------------------
# chunglu-1m
# ---------------------------------------------------------------------------
CL_N, CL_M, CL_GAMMA, CL_WMAX, CL_BATCH = 1_000_000, 10_000_000, 2.1, 50_000.0, 100_000


def cl1m_workload(steps):
    """The graph and `steps` (insert batch, delete batch) pairs, each pair
    drawn against the edge set the earlier pairs leave."""
    import graphgen
    rng = graphgen.rng_for("bench-cl-1m")
    t = time.time()
    s, d = graphgen.chung_lu_graph(CL_N, CL_M, CL_GAMMA, CL_WMAX, rng)
    log(f"graph generated in {time.time() - t:.1f}s (m={s.size})")
    es = graphgen.EdgeSet(s, d)
    batches = []
    for _ in range(steps):
        a, b = graphgen.weighted_non_edges(CL_BATCH, es, rng)
        es.insert(a, b)
        x, y = graphgen.existing_edges(CL_BATCH, es, rng)
        es.delete(x, y)
        batches.append(((a, b), (x, y)))
    log(f"{steps} batch pairs generated")
    return s, d, batches


def cl1m_per_batch(cm, torch, s, d, dev_batches, mode, warmup, steps, params):
    g = cm.Graph(mode=mode, timing=True, **params)
    g.load(CL_N, to_dev(torch, s), to_dev(torch, d))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dst = g.decompose()
    torch.cuda.synchronize()
    dec_ms = (time.perf_counter() - t0) * 1e3
    for k in range(warmup):
        (a, b), (x, y) = dev_batches[k]
        g.insert_edges(a, b)
        g.delete_edges(x, y)
    torch.cuda.synchronize()
    g.phase_times(reset=True)
    lat, stats = [], []
    t0 = time.perf_counter()
    for k in range(warmup, warmup + steps):
        (a, b), (x, y) = dev_batches[k]
        t1 = time.perf_counter()
        si = g.insert_edges(a, b)
        t2 = time.perf_counter()
        sd = g.delete_edges(x, y)
        t3 = time.perf_counter()
        lat += [(t2 - t1) * 1e3, (t3 - t2) * 1e3]
        stats += [si.as_dict(), sd.as_dict()]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    phases = g.phase_times()
    cores = g.cores()
    g.close()
    return {"elapsed": elapsed, "lat": lat, "stats": stats, "dec_ms": dec_ms,
            "dec_stats": dst.as_dict(), "cores": cores, "phases": phases}


def cl1m_program(cm, torch, s, d, batches, warmup, steps, params):
    """Warm-up batches one by one, then every timed batch in one launch."""
    g = cm.Graph(mode=cm.MODE_PERSISTENT, timing=True, use_graph=True, **params)
    g.load(CL_N, to_dev(torch, s), to_dev(torch, d))
    g.decompose()
    kinds, xs, ys = [], [], []
    for k in range(warmup + steps):
        (a, b), (x, y) = batches[k]
        kinds += [cm.BATCH_INSERT, cm.BATCH_DELETE]
        xs += [a, x]
        ys += [b, y]
    offs = np.concatenate([[0], np.cumsum([v.size for v in xs])]).astype(np.int64)
    dx, dy = to_dev(torch, np.concatenate(xs)), to_dev(torch, np.concatenate(ys))
    w = 2 * warmup
    g.run_batches(kinds[:w], offs[:w + 1], dx[:offs[w]], dy[:offs[w]])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, _ = g.run_batches(kinds[w:], offs[w:] - offs[w], dx[offs[w]:], dy[offs[w]:])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cores = g.cores()
    g.close()
    assert all(r.status == 0 for r in res)
    return {"elapsed": elapsed, "stats": [r.as_dict() for r in res], "cores": cores}


def cl1m_cpu_baseline(s, d, pairs, budget_s=10.0):
    """The oracle as it stands: apply each batch to its host edge set and
    recompute every core number (BZ), pair after pair of the workload (an
    insert batch, then a delete batch) until about `budget_s` seconds."""
    import oracle
    oracle.build(force=False)
    ref = oracle.DynamicGraph(CL_N, s, d)
    t0 = time.perf_counter()
    done = 0
    for (a, b), (x, y) in pairs:
        ref.insert_edges(a, b)
        ref.cores()
        ref.delete_edges(x, y)
        ref.cores()
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    upd = 2 * CL_BATCH * done
    return {"value": upd / el, "unit": "edge_updates/s", "cores": 1, "kind": "oracle",
            "sample": f"the workload's first {done} batch pairs ({upd} updates, {el:.1f}s): host edge-set "
                      "apply + Batagelj-Zaversnik recompute after each batch"}


CL_CPU_PAIRS = 12   # batch pairs the oracle may run for the CPU baseline (about 10 s)


def bench_cl1m(args, cm, torch):
    ntimed = args.warmup + args.steps
    s, d, batches = cl1m_workload(ntimed if args.no_cpu_baseline else max(ntimed, CL_CPU_PAIRS))
    cpu_batches, batches = batches, batches[:ntimed]
    dev_batches = [tuple(tuple(to_dev(torch, z) for z in pair) for pair in step) for step in batches]
    torch.cuda.synchronize()

    def sample():
        (a, b), (x, y) = batches[0]
        xs, ys = np.concatenate([a, x]), np.concatenate([b, y])
        return (CL_N, to_dev(torch, s), to_dev(torch, d), np.array([0, 1], np.int32),
                np.array([0, a.size, a.size + x.size], np.int64), to_dev(torch, xs), to_dev(torch, ys))
    params, tuning = tuned_params(args, CL_N, CL_M, [CL_BATCH], sample)
    plain = cl1m_per_batch(cm, torch, s, d, dev_batches, cm.MODE_PLAIN, args.warmup, args.steps, params)
    log(f"plain: {plain['elapsed']:.3f}s for {args.steps} steps")
    updates = 2 * CL_BATCH * args.steps
    st = plain["stats"]
    out = contract("chung-lu n=1000000 m=10000000 gamma=2.1 wmax=50000; per step insert 100000 "
                   "degree-weighted non-edges then delete 100000 existing edges",
                   updates / plain["elapsed"], args.steps, args.warmup,
                   plain["elapsed"] * 1e3 / args.steps, 2 * CL_BATCH,
                   "plain (one cooperative launch per superior edge set)")
    out["roofline"] = roofline("k_maintain", st, "one superior edge set (partition, apply, cascade, "
                                                "core and SD update)", traffic_key="chunglu-1m")
    out["latency_ms"] = {"p50": pct(plain["lat"], 50), "p99": pct(plain["lat"], 99),
                         "per": "batch of 100000 edges"}
    out["tuning"] = tuning
    out["phase_ms"] = {k: round(v[0], 3) for k, v in plain["phases"].items()}
    out["iterations_per_batch"] = [x["iterations"] for x in st]
    out["rounds_per_batch"] = [x["rounds"] for x in st]
    out["steps_per_batch"] = [x["grid_steps"] + x["local_steps"] for x in st]
    out["decompose"] = {"ms": plain["dec_ms"], "kernel_ms": plain["dec_stats"]["kernel_ms"],
                        "edges_per_s": CL_M / (plain["dec_ms"] * 1e-3)}
    if not args.no_persistent:
        pers = cl1m_per_batch(cm, torch, s, d, dev_batches, cm.MODE_PERSISTENT, args.warmup, args.steps,
                              params)
        log(f"persistent: {pers['elapsed']:.3f}s")
        assert np.array_equal(plain["cores"], pers["cores"]), "plain and persistent forms disagree"
        prog = cl1m_program(cm, torch, s, d, batches, args.warmup, args.steps, params)
        log(f"batched: {prog['elapsed']:.3f}s")
        assert np.array_equal(plain["cores"], prog["cores"]), "plain and batched forms disagree"
        pst = pers["stats"]
        out["persistent"] = {
            "form": "persistent (one cooperative launch per batch)",
            "value": updates / pers["elapsed"],
            "ms_per_step": pers["elapsed"] * 1e3 / args.steps,
            "latency_ms": {"p50": pct(pers["lat"], 50), "p99": pct(pers["lat"], 99)},
            "roofline_achieved_gbs": roofline("k_maintain", pst, "")["achieved"],
            "avg_launch_us": roofline("k_maintain", pst, "")["avg_launch_us"],
        }
        out["batched"] = {
            "form": "batched (every timed batch in one persistent launch, hipGraph replay)",
            "value": updates / prog["elapsed"],
            "ms_per_step": prog["elapsed"] * 1e3 / args.steps,
            "speedup_vs_plain": plain["elapsed"] / prog["elapsed"],
            "roofline_achieved_gbs": roofline("k_program", prog["stats"], "")["achieved"],
        }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cl1m_cpu_baseline(s, d, cpu_batches)
    return out


# ---------------------------------------------------------------------------
# rmat22-stream
# ---------------------------------------------------------------------------
RM_SCALE, RM_BATCHES, RM_LO, RM_HI = 22, 64, 1000, 1_000_000


def host_cpu():
    """Model name and logical CPU count of the host (for the CPU baseline)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def bench_rmat22(args, cm, torch):
    import graphgen
    t = time.time()
    n, s, d, kinds, offs, xs, ys = graphgen.rmat_stream(
        RM_SCALE, RM_BATCHES, RM_LO, RM_HI, graphgen.rng_for("bench-rmat22"), workers=WORKERS,
        progress=lambda m: log(f"{time.time() - t:.0f}s {m}"))
    total = int(offs[-1])
    log(f"stream ready: {total} updates in {RM_BATCHES} batches")
    ds, dd, dx, dy = (to_dev(torch, z) for z in (s, d, xs, ys))
    torch.cuda.synchronize()
    ns = 16  # tuning sample: the first 16 batches of the stream

    def sample():
        return n, ds, dd, kinds[:ns], offs[:ns + 1], dx[:offs[ns]], dy[:offs[ns]]
    params, tuning = tuned_params(args, n, s.size, np.diff(offs), sample)

    def run(mode, use_graph, reps, per_batch=False, extra=None):
        """reps passes over the stream from the freshly loaded graph: one
        cm_run_batches call for the whole stream, or (per_batch) one call per
        batch with its latency."""
        g = cm.Graph(mode=mode, timing=True, use_graph=use_graph, **{**params, **(extra or {})})
        times, allstats, lat = [], [], []
        try:
            for rep in range(reps):
                g.load(n, ds, dd)
                g.decompose()
                g.phase_times(reset=True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if per_batch:
                    res, lat = [], []
                    for j in range(RM_BATCHES):
                        tb = time.perf_counter()
                        r, _ = g.run_batches(kinds[j:j + 1], offs[j:j + 2] - offs[j],
                                             dx[offs[j]:offs[j + 1]], dy[offs[j]:offs[j + 1]])
                        lat.append((time.perf_counter() - tb) * 1e3)
                        res += r
                else:
                    res, _ = g.run_batches(kinds, offs, dx, dy)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
                assert all(r.status == 0 for r in res), [r.status for r in res]
                allstats.append([r.as_dict() for r in res])
                log(f"mode {mode}{' per batch' if per_batch else ''}: pass {rep} {times[-1]:.3f}s")
            phases = g.phase_times()
            cores = g.cores()
        finally:
            g.close()
        return times, allstats, cores, phases, lat

    bt, bstats, bcores, bph, _ = run(cm.MODE_PERSISTENT, True, args.warmup + args.steps)
    bt, bstats = bt[args.warmup:], bstats[args.warmup:]
    pt, pstats, pcores, pph, _ = run(cm.MODE_PLAIN, False, 1 + (args.steps > 1))
    assert np.array_equal(bcores, pcores), "plain and batched forms disagree"
    pt, pstats = pt[-1:], pstats[-1:]
    qt, qstats, qcores, _, qlat = run(cm.MODE_PERSISTENT, False, 1, per_batch=True)
    assert np.array_equal(bcores, qcores), "persistent and batched forms disagree"
    # the method's own bytes: one untimed pass whose expansion visits exactly
    # Algorithm 3's sets (pruned); partitions and cores are the same in every form
    mt, mstats, mcores, _, _ = run(cm.MODE_PERSISTENT, True, 1, extra={"expand_mode": 1})
    assert np.array_equal(bcores, mcores), "pruned and one-pass expansions disagree"
    method_bytes = sum(x["alg_bytes"] for x in mstats[0])
    value = total * len(bt) / sum(bt)
    plain_value = total / pt[0]
    out = contract(f"r-mat scale 22 edge factor 16 (n={n} m={s.size}); stream of 64 batches, sizes "
                   "log-uniform [1000, 1000000], half r-mat non-edge inserts, half uniform deletes "
                   f"({total} updates); one step = the whole stream from the freshly loaded graph",
                   value, args.steps, args.warmup, sum(bt) * 1e3 / len(bt), total,
                   "batched (the whole stream in one persistent launch, hipGraph replay)")
    flat = [x for run_ in bstats for x in run_]
    out["roofline"] = roofline("k_program", flat, "the whole 64-batch stream", traffic_key="rmat22-stream",
                               method_bytes=method_bytes)
    out["roofline"]["alg_bytes_source"] = ("the method's sets (Algorithm 3's pruned expansion), counted on "
                                           f"an untimed pass of the same stream ({mt[0]:.2f}s)")
    out["roofline"]["timed_form_counted_bytes_per_launch"] = sum(x["alg_bytes"] for x in flat) / max(len(bt), 1)
    out["roofline"]["scanned_over_method_entries"] = (
        sum(x["scanned"] for x in flat) / max(len(bt), 1) /
        max(sum(x["cand_degree"] + x["evicted_degree"] + x["changed_degree"] for x in mstats[0]), 1))
    plat = [x["ms_total"] for x in pstats[0]]
    out["speedup_batched_vs_plain"] = value / plain_value
    out["latency_ms"] = {"p50": pct(plat, 50), "p99": pct(plat, 99),
                         "per": "batch, plain form (call to exact cores)"}
    out["plain"] = {
        "form": "plain (host loop, one cooperative launch per superior edge set)",
        "value": plain_value, "ms_per_step": pt[0] * 1e3,
        "latency_ms": {"p50": pct(plat, 50), "p99": pct(plat, 99), "per": "batch"},
        "roofline": roofline("k_maintain", pstats[0], "one superior edge set",
                             method_bytes=method_bytes / max(sum(x["launches"] for x in pstats[0]), 1)),
    }
    out["persistent"] = {
        "form": "persistent (one cooperative launch per batch, one call per batch)",
        "value": total / qt[0], "ms_per_step": qt[0] * 1e3,
        "latency_ms": {"p50": pct(qlat, 50), "p99": pct(qlat, 99), "per": "batch"},
    }
    out["tuning"] = tuning
    out["phase_ms"] = {k: round(v[0], 3) for k, v in bph.items()}
    out["phase_count"] = {k: v[1] for k, v in bph.items()}
    ps0 = pstats[0]
    out["iterations_per_batch"] = [x["iterations"] for x in ps0]
    out["steps_per_batch"] = [x["grid_steps"] + x["local_steps"] for x in bstats[-1]]
    out["batch_sizes"] = np.diff(offs).tolist()
    out["per_batch"] = {k: [x[k] for x in ps0] for k in
                        ("rounds", "candidates", "evicted", "changed", "scanned", "remaining_sum")}
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        ref = oracle.DynamicGraph(n, s, d)
        t0 = time.perf_counter()
        done, used = 0, 0
        for j in range(RM_BATCHES):
            a, b = xs[offs[j]:offs[j + 1]], ys[offs[j]:offs[j + 1]]
            (ref.insert_edges if kinds[j] == 0 else ref.delete_edges)(a, b)
            ref.cores()
            done += a.size
            used += 1
            if time.perf_counter() - t0 >= args.cpu_budget:
                break
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": done / el, "unit": "edge_updates/s", "cores": 1, "kind": "oracle",
                               "host": host_cpu(),
                               "sample": f"first {used} batches of the stream ({done} updates, {el:.1f}s): "
                                         "host edge-set apply + Batagelj-Zaversnik recompute after each "
                                         "batch, one thread"}
    return out


# ---------------------------------------------------------------------------
# chunglu-pool512
# ---------------------------------------------------------------------------
POOL_COUNT = 512


def bench_pool512(args, cm, torch):
    import graphgen
    t = time.time()
    pool = graphgen.chung_lu_pool(POOL_COUNT, graphgen.rng_for("bench-pool512"), workers=WORKERS)
    graphs = [(n, s, d) for n, s, d, _, _ in pool]
    batches = []
    for gid, (_, _, _, ins, dele) in enumerate(pool):
        batches.append((gid, cm.BATCH_INSERT, ins[0], ins[1]))
        batches.append((gid, cm.BATCH_DELETE, dele[0], dele[1]))
    total = int(sum(b[2].size for b in batches))
    log(f"{POOL_COUNT} graphs, {sum(g[1].size for g in graphs)} edges, {total} updates "
        f"generated in {time.time() - t:.0f}s")

    base, us, ud = cm.union_edges(graphs)
    union_n = int(base[-1])
    kinds, offs, xs, ys, sub, nsub, order = cm.pack_batches(base, batches)
    dus, dud, dx, dy, dsub = (to_dev(torch, z) for z in (us, ud, xs, ys, sub))
    torch.cuda.synchronize()
    log(f"packed: union n={union_n} m={us.size}, {len(kinds)} union batches, {nsub} sub-batches")

    def sample():
        return union_n, dus, dud, kinds, offs, dx, dy, dsub, nsub
    params, tuning = tuned_params(args, union_n, us.size, [b[2].size for b in batches], sample)

    def batched(reps):
        g = cm.Graph(mode=cm.MODE_PERSISTENT, timing=True, use_graph=True, **params)
        times, stats = [], []
        for rep in range(reps):
            g.load(union_n, dus, dud)
            g.decompose()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res, sst = g.run_batches(kinds, offs, dx, dy, sub=dsub, nsub=nsub)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            assert all(r.status == 0 for r in res) and (sst == 0).all()
            stats.append([r.as_dict() for r in res])
            phases = g.phase_times()
            log(f"batched pass {rep}: {times[-1]:.3f}s")
        cores = g.cores()
        g.close()
        return times, stats, cores, phases

    def plain():
        """The same 1024 member batches one after another (graph by graph)."""
        g = cm.Graph(mode=cm.MODE_PLAIN, timing=True, **params)
        g.load(union_n, dus, dud)
        g.decompose()
        pk = np.array([b[1] for b in batches], np.int32)
        px = np.concatenate([b[2].astype(np.int64) + base[b[0]] for b in batches]).astype(np.int32)
        py = np.concatenate([b[3].astype(np.int64) + base[b[0]] for b in batches]).astype(np.int32)
        po = np.concatenate([[0], np.cumsum([b[2].size for b in batches])]).astype(np.int64)
        dpx, dpy = to_dev(torch, px), to_dev(torch, py)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, _ = g.run_batches(pk, po, dpx, dpy)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        assert all(r.status == 0 for r in res)
        cores = g.cores()
        g.close()
        return el, [r.as_dict() for r in res], cores

    bt, bstats, bcores, bph = batched(args.warmup + args.steps)
    bt, bstats = bt[args.warmup:], bstats[args.warmup:]
    pel, pstats, pcores = plain()
    log(f"plain: {pel:.3f}s")
    assert np.array_equal(bcores, pcores), "plain and batched forms disagree"
    value = total * len(bt) / sum(bt)
    out = contract(f"{POOL_COUNT} independent chung-lu graphs (n log-uniform [1000, 200000], mean degree "
                   f"U[4, 32], gamma 2.3; union n={union_n} m={us.size}); per graph insert 5% "
                   f"degree-weighted non-edges then delete 5% existing edges ({total} updates)",
                   value, args.steps, args.warmup, sum(bt) * 1e3 / len(bt), total,
                   "batched (graphs packed as one disjoint union, one hipGraph launch)")
    out["roofline"] = roofline("k_program", [x for r in bstats for x in r],
                               "every graph's insertion and deletion batch")
    out["tuning"] = tuning
    out["phase_ms"] = {k: round(v[0], 3) for k, v in bph.items()}
    plat = [x["ms_total"] for x in pstats]
    out["plain"] = {"form": "plain (1024 member batches one after another, one launch per superior "
                            "edge set)", "value": total / pel, "ms_per_step": pel * 1e3,
                    "speedup_batched_vs_plain": value / (total / pel),
                    "latency_ms": {"p50": pct(plat, 50), "p99": pct(plat, 99), "per": "member batch"}}
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        t0 = time.perf_counter()
        done, used = 0, 0
        for gid, (n, s, d, ins, dele) in enumerate(pool):
            ref = oracle.DynamicGraph(n, s, d)
            ref.insert_edges(*ins)
            ref.cores()
            ref.delete_edges(*dele)
            c2 = ref.cores()
            assert np.array_equal(c2, bcores[base[gid]:base[gid + 1]]), f"graph {gid} differs"
            done += ins[0].size + dele[0].size
            used += 1
            if time.perf_counter() - t0 > 20.0:
                break
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": done / el, "unit": "edge_updates/s", "cores": 1, "kind": "oracle",
                               "sample": f"first {used} graphs' two batches ({done} updates, {el:.1f}s): "
                                         "host edge-set apply + Batagelj-Zaversnik recompute per batch; "
                                         "their final cores also checked against the batched form"}
    return out


# ---------------------------------------------------------------------------
# rmat-serve
# ---------------------------------------------------------------------------
def bench_serve(args, cm, torch):
    import graphgen
    from paper_1612_09368_amd import serve
    scale, nreq = args.scale, args.requests
    t = time.time()
    n, s, d, reqs = graphgen.serve_stream(scale, nreq, graphgen.rng_for("bench-serve"), workers=WORKERS,
                                          progress=lambda m: log(f"{time.time() - t:.0f}s {m}"))
    kinds = [r[0] for r in reqs]
    new_ids = sum(len(r[1]) - 1 for r in reqs if r[0] == "vins")
    log(f"stream ready in {time.time() - t:.0f}s: " +
        ", ".join(f"{k} {kinds.count(k)}" for k in ("ins", "del", "vins", "vdel")))
    ds, dd = to_dev(torch, s), to_dev(torch, d)
    sizes = [len(r[1]) for r in reqs]
    params, tuning = tuned_params(args, n, s.size, sizes, None)
    scfg = dict(ring_requests=4096, ring_items=1 << 25, max_items=1 << 23, budget_bytes=4 << 30,
                vertex_headroom=new_ids + 1024, idle_ms=20)

    def one_run(arrivals):
        g = cm.Graph(mode=cm.MODE_PERSISTENT, **params)
        g.load(n, ds, dd)
        g.decompose()
        torch.cuda.synchronize()
        srv = serve.Server(g, **scfg)
        res = serve.run_stream(srv, reqs, arrivals)
        srv.stop()
        cores = g.cores()
        g.close()
        st = res["stats"]
        assert all(x.status == 0 for x in st), "a served request failed"
        upd = sum(int(x.applied) for x in st)
        lat = (res["t_done"] - res["t_arrival"]) * 1e3
        return res["elapsed"], upd, lat, cores

    el, upd, lat_c, cores_c = one_run(None)
    rate = nreq / el
    log(f"closed loop: {el:.2f}s, {upd / el / 1e6:.2f} M updates/s, {rate:.0f} requests/s")
    lam = 0.8 * rate
    arrivals = np.cumsum(np.random.Generator(np.random.PCG64(7)).exponential(1.0 / lam, nreq))
    el2, upd2, lat, cores_p = one_run(arrivals)
    log(f"poisson at {lam:.0f}/s: {el2:.2f}s, p50 {np.percentile(lat, 50):.2f} ms, "
        f"p99 {np.percentile(lat, 99):.2f} ms")
    assert np.array_equal(cores_c, cores_p), "served results depend on arrival timing"
    out = contract(f"serving: r-mat scale {scale} (n={n} m={s.size}); {nreq} requests, sizes log-uniform "
                   "[1, 100000]: 40% edge insert, 40% edge delete, 10% vertex insert (power-law degree "
                   "1-1000), 10% vertex delete; continuous batching in one persistent launch",
                   upd / el, 1, 0, el * 1e3, upd, "served (closed loop: every request submitted at once, "
                                                   "admitted as the ring and memory budget allow)")
    out["served_poisson"] = {
        "arrival_rate_per_s": lam, "rate_rule": "0.8 x the closed-loop request rate",
        "value": upd2 / el2, "requests_per_s": nreq / el2,
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "per": "request, arrival to result"},
    }
    out["closed_loop"] = {"requests_per_s": rate, "latency_ms": {"p50": pct(lat_c, 50), "p99": pct(lat_c, 99)}}
    out["tuning"] = tuning
    out["roofline"] = None
    if args.checkpoints:
        out["checkpoints"] = serve_checkpoints(cm, torch, serve, n, ds, dd, reqs, params, scfg, scale, nreq)
    return out


def serve_checkpoints(cm, torch, serve, n, ds, dd, reqs, params, scfg, scale, nreq):
    """An untimed closed-loop pass that stops serving at the request counts
    of the stored checkpoints (tests/golden/serve_checkpoints_r<scale>.json,
    written on the host by `python -m oracle.serve_checkpoints` for the same
    seeded stream: 21 evenly spaced counts), hashes the core vector there
    (SHA-256 of the int32 cores, dead ids -1) and compares it, the id and
    edge counts and the per-request statuses with the stored values."""
    import hashlib
    golden = os.path.join(ROOT, "tests", "golden", f"serve_checkpoints_r{scale}.json")
    if not os.path.exists(golden):
        return {"compared": False, "note": f"no stored checkpoints ({os.path.basename(golden)})"}
    with open(golden) as f:
        want = json.load(f)
    if want["workload"] != {"scale": scale, "requests": nreq, "seed_tag": "bench-serve"}:
        return {"compared": False, "note": "stored checkpoints are for another workload"}
    marks = [c["after"] for c in want["checkpoints"]]

    def digest(a):
        return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()
    g = cm.Graph(mode=cm.MODE_PERSISTENT, **params)
    got, statuses = [], []
    try:
        g.load(n, ds, dd)
        g.decompose()
        done = 0
        for mark in marks:
            srv = serve.Server(g, **scfg)
            res = serve.run_stream(srv, reqs[done:mark], None)
            srv.stop()
            statuses += [int(x.status) for x in res["stats"]]
            c = g.cores()
            got.append({"after": mark, "cores_sha256": digest(c), "n_ids": int(c.size), "m": g.num_edges()})
            done = mark
            log(f"checkpoint after {mark} requests")
    finally:
        g.close()
    st = np.asarray(statuses, dtype=np.int32)
    out = {"count": len(got), "statuses_sha256": hashlib.sha256(st.tobytes()).hexdigest(),
           "failed_requests": int((st != 0).sum())}
    match = [a["cores_sha256"] == b["cores_sha256"] and a["n_ids"] == b["n_ids"] and a["m"] == b["m"]
             for a, b in zip(got, want["checkpoints"])]
    out.update({"compared": True, "matched": int(sum(match)), "of": len(want["checkpoints"]),
                "statuses_match": out["statuses_sha256"] == want["statuses_sha256"],
                "first_mismatch_after": next((a["after"] for a, ok in zip(got, match) if not ok), None)})
    assert all(match) and len(got) == len(want["checkpoints"]), f"served checkpoints differ from the oracle: {out}"
    return out


# ---------------------------------------------------------------------------
# pool-serve
# ---------------------------------------------------------------------------
def bench_pool_serve(args, cm, torch):
    """Serving many independent graphs (sessions) from one handle: the
    512-graph pool packed as one disjoint union, each graph's insertion and
    deletion batches split into requests of its own session (4 + 4), queued
    round-robin over the graphs.  Closed loop with every request alone in its
    batch (fuse = 1), then Poisson arrivals at 0.8 x that request rate, with
    fuse = 1 and with continuous batching across sessions (fuse = 32); p50 /
    p99 latency from arrival to result."""
    import graphgen
    from paper_1612_09368_amd import serve
    t = time.time()
    pool = graphgen.chung_lu_pool(POOL_COUNT, graphgen.rng_for("bench-pool512"), workers=WORKERS)
    graphs = [(n, s, d) for n, s, d, _, _ in pool]
    base, us, ud = cm.union_edges(graphs)
    parts = 4
    per_graph = []
    for gid, (_, _, _, ins, dele) in enumerate(pool):
        reqs = []
        for kind, (a, b) in (("ins", ins), ("del", dele)):
            for a2, b2 in zip(np.array_split(a, parts), np.array_split(b, parts)):
                reqs.append((kind, (a2 + base[gid]).astype(np.int32), (b2 + base[gid]).astype(np.int32)))
        per_graph.append(reqs)
    reqs, sess = [], []
    for k in range(2 * parts):
        for gid in range(POOL_COUNT):
            reqs.append(per_graph[gid][k])
            sess.append(gid)
    total = sum(r[1].size for r in reqs)
    log(f"pool serving: {len(reqs)} requests, {total} updates ({time.time() - t:.0f}s)")
    ds, dd = to_dev(torch, us), to_dev(torch, ud)
    union_n = int(base[-1])
    params, tuning = tuned_params(args, union_n, us.size, [r[1].size for r in reqs], None)
    scfg = dict(ring_requests=8192, ring_items=1 << 25, max_items=1 << 22, budget_bytes=8 << 30,
                vertex_headroom=1024, idle_ms=20)

    def one_run(arrivals, fuse):
        g = cm.Graph(mode=cm.MODE_PERSISTENT, **params)
        try:
            g.load(union_n, ds, dd)
            g.decompose()
            torch.cuda.synchronize()
            srv = serve.Server(g, fuse=fuse, **scfg)
            res = serve.run_stream(srv, reqs, arrivals, sessions=sess)
            srv.stop()
            cores = g.cores()
        finally:
            g.close()
        st = res["stats"]
        assert all(x.status == 0 for x in st), "a served request failed"
        lat = (res["t_done"] - res["t_arrival"]) * 1e3
        groups = np.array([x.group for x in st])
        return res["elapsed"], lat, cores, groups

    el, lat_c, cores_c, _ = one_run(None, 1)
    rate = len(reqs) / el
    log(f"closed loop, alone: {el:.2f}s, {total / el / 1e6:.2f} M updates/s, {rate:.0f} requests/s")
    elf, lat_cf, cores_cf, grp_cf = one_run(None, 32)
    log(f"closed loop, fused: {elf:.2f}s, {total / elf / 1e6:.2f} M updates/s, mean group {grp_cf.mean():.1f}")
    lam = 0.8 * rate
    arrivals = np.cumsum(np.random.Generator(np.random.PCG64(9)).exponential(1.0 / lam, len(reqs)))
    el1, lat1, cores1, _ = one_run(arrivals, 1)
    el2, lat2, cores2, grp2 = one_run(arrivals, 32)
    for c in (cores_cf, cores1, cores2):
        assert np.array_equal(cores_c, c), "served results depend on fusion or arrival timing"
    log(f"poisson at {lam:.0f}/s: alone p50 {pct(lat1, 50):.2f} p99 {pct(lat1, 99):.2f} ms; "
        f"fused p50 {pct(lat2, 50):.2f} p99 {pct(lat2, 99):.2f} ms")
    out = contract(f"serving {POOL_COUNT} independent chung-lu graphs as sessions of one handle (union n={union_n} "
                   f"m={us.size}); {len(reqs)} requests (each graph's 5% insertion and 5% deletion batches in "
                   f"{parts} requests each), round-robin over the graphs",
                   total / elf, 1, 0, elf * 1e3, total,
                   "served with continuous batching across sessions (fuse 32), closed loop")
    out["closed_loop_alone"] = {"value": total / el, "requests_per_s": rate,
                                "latency_ms": {"p50": pct(lat_c, 50), "p99": pct(lat_c, 99)}}
    out["closed_loop_fused"] = {"value": total / elf, "requests_per_s": len(reqs) / elf,
                                "mean_group": float(grp_cf.mean()),
                                "latency_ms": {"p50": pct(lat_cf, 50), "p99": pct(lat_cf, 99)}}
    out["poisson"] = {"arrival_rate_per_s": lam, "rate_rule": "0.8 x the closed-loop rate with fuse 1",
                      "alone": {"value": total / el1, "latency_ms": {"p50": pct(lat1, 50), "p99": pct(lat1, 99)}},
                      "fused": {"value": total / el2, "mean_group": float(grp2.mean()),
                                "latency_ms": {"p50": pct(lat2, 50), "p99": pct(lat2, 99)}},
                      "per": "request, arrival to result"}
    out["tuning"] = tuning
    out["roofline"] = None
    return out


# ---------------------------------------------------------------------------
# paper-sweep
# ---------------------------------------------------------------------------
SWEEP_UPDATES = 10_000
SWEEP_SEQ_UPDATES = 1_000


def bench_sweep(args, cm, torch):
    """The paper's scalability experiment on synthetic graphs: ER, BA and
    R-MAT with n = 2^15 .. 2^21 and m/n = 8; 10,000 random edge insertions,
    then 10,000 random deletions, timed per edge; beside it the sequential
    regime (one edge per iteration) on 1,000 of them, with iteration counts."""
    import graphgen
    sizes = [int(x) for x in args.sweep_scales.split(",")]
    rows = []
    for kind in ("er", "ba", "rmat"):
        for sc in sizes:
            rng = graphgen.rng_for(f"sweep-{kind}-{sc}")
            n = 1 << sc
            t0 = time.time()
            if kind == "er":
                s, d = graphgen.er_graph(n, 8 * n, rng)
            elif kind == "ba":
                s, d = graphgen.ba_graph_blocks(n, 8, rng)
            else:
                n, s, d = graphgen.rmat_graph(sc, 8, rng, workers=WORKERS)
            es = graphgen.EdgeSet(s, d)
            ia, ib = graphgen.uniform_non_edges(n, SWEEP_UPDATES, es, rng)
            es.insert(ia, ib)
            da, db = graphgen.existing_edges(SWEEP_UPDATES, es, rng)
            dev = [to_dev(torch, z) for z in (s, d, ia, ib, da, db)]
            row = {"graph": kind, "n": n, "m": int(s.size), "gen_s": round(time.time() - t0, 1)}
            for regime, cnt in (("superior", SWEEP_UPDATES), ("sequential", SWEEP_SEQ_UPDATES)):
                g = cm.Graph(mode=cm.MODE_PERSISTENT, single_edge=regime == "sequential")
                g.load(n, dev[0], dev[1])
                g.decompose()
                if regime == "superior":
                    # generator sanity: the paper reports BA all at core 8, ER with max core ~10
                    c0 = g.cores()
                    row["kmax"] = int(c0.max())
                    row["top_level_share"] = round(float((c0 == c0.max()).mean()), 4)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                si = g.insert_edges(dev[2][:cnt], dev[3][:cnt])
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                # deletions of edges that exist in this regime's graph
                if cnt == SWEEP_UPDATES:
                    xa, xb = dev[4], dev[5]
                else:
                    keep = np.isin(graphgen.keys_of(da, db), graphgen.keys_of(s, d)) | \
                        np.isin(graphgen.keys_of(da, db), graphgen.keys_of(ia[:cnt], ib[:cnt]))
                    xa, xb = to_dev(torch, da[keep][:cnt]), to_dev(torch, db[keep][:cnt])
                t3 = time.perf_counter()
                sd = g.delete_edges(xa, xb)
                torch.cuda.synchronize()
                t4 = time.perf_counter()
                g.close()
                row[regime] = {"insert_us_per_edge": 1e6 * (t2 - t1) / cnt,
                               "delete_us_per_edge": 1e6 * (t4 - t3) / max(int(xa.numel()), 1),
                               "insert_iterations": si.iterations, "delete_iterations": sd.iterations,
                               "edges": cnt}
            rows.append(row)
            log(f"{kind} n=2^{sc}: superior {row['superior']['insert_us_per_edge']:.3f}/"
                f"{row['superior']['delete_us_per_edge']:.3f} us/edge ({row['superior']['insert_iterations']}/"
                f"{row['superior']['delete_iterations']} it), sequential "
                f"{row['sequential']['insert_us_per_edge']:.1f}/{row['sequential']['delete_us_per_edge']:.1f} us/edge")
    big = [r for r in rows if r["graph"] == "rmat"][-1]
    per_edge_us = (big["superior"]["insert_us_per_edge"] + big["superior"]["delete_us_per_edge"]) / 2
    out = contract(f"paper scalability sweep: ER / BA / R-MAT, n = 2^{sizes[0]}..2^{sizes[-1]}, m/n = 8; "
                   f"{SWEEP_UPDATES} random insertions then {SWEEP_UPDATES} random deletions per graph "
                   f"(value: R-MAT n=2^{sizes[-1]}, superior edge sets)",
                   1e6 / per_edge_us, 1, 0, per_edge_us * 2 * SWEEP_UPDATES / 1e3, 2 * SWEEP_UPDATES,
                   "persistent (one launch per batch), superior edge sets vs one edge per iteration")
    out["sweep"] = rows
    out["roofline"] = None
    return out


# ---------------------------------------------------------------------------
# core-levels
# ---------------------------------------------------------------------------
LV_LEVELS, LV_FRAC = 5, 0.2


def bench_levels(args, cm, torch):
    """Per-edge time against the core number of the updated edges (the
    paper's experiment on the core distribution of the updates): on the
    R-MAT scale-22 graph, five typical edge core numbers K1 < ... < K5 (the
    edge core distribution's quantiles 0.1, 0.3, ..., 0.9); for each, 20% of
    the edges of that core number, chosen at random, are deleted as one
    batch and then inserted back as one batch (the graph, and so every core
    number, is back to the start afterwards).  Persistent form."""
    import graphgen
    t = time.time()
    rng = graphgen.rng_for("bench-levels")
    n, s, d = graphgen.rmat_graph(RM_SCALE, 16, rng, workers=WORKERS)
    log(f"r-mat scale {RM_SCALE}: {s.size} edges ({time.time() - t:.0f}s)")
    ds, dd = to_dev(torch, s), to_dev(torch, d)
    params, tuning = tuned_params(args, n, s.size, [LV_FRAC * s.size / 50], None)
    g = cm.Graph(mode=cm.MODE_PERSISTENT, timing=True, **params)
    g.load(n, ds, dd)
    g.decompose()
    cores0 = g.cores()
    levels = graphgen.typical_levels(s, d, cores0, LV_LEVELS)
    ec = graphgen.edge_levels(s, d, cores0)
    rows, tot_edges, tot_s = [], 0, 0.0
    for k in levels:
        a, b = graphgen.edges_at_level(s, d, cores0, k, LV_FRAC, rng)
        xa, xb = to_dev(torch, a), to_dev(torch, b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sd = g.delete_edges(xa, xb)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        si = g.insert_edges(xa, xb)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        assert sd.status == 0 and si.status == 0, (sd.status, si.status)
        back = bool(np.array_equal(g.cores(), cores0))
        assert back, f"level {k}: core numbers differ after deleting and re-inserting the same edges"
        rows.append({"level": k, "level_edges": int((ec == k).sum()), "edges": int(a.size),
                     "delete_us_per_edge": 1e6 * (t1 - t0) / a.size,
                     "insert_us_per_edge": 1e6 * (t2 - t1) / a.size,
                     "delete_iterations": sd.iterations, "insert_iterations": si.iterations,
                     "delete_changed": sd.changed, "insert_changed": si.changed})
        tot_edges += 2 * int(a.size)
        tot_s += t2 - t0
        r = rows[-1]
        log(f"level {k}: {a.size} of {r['level_edges']} edges; delete {r['delete_us_per_edge']:.3f} us/edge "
            f"({sd.iterations} it), insert {r['insert_us_per_edge']:.3f} us/edge ({si.iterations} it)")
    g.close()
    out = contract(f"r-mat scale {RM_SCALE} (edge factor 16, {s.size} edges); per typical edge core number "
                   f"(quantiles 0.1..0.9 of the edge core distribution), {int(LV_FRAC * 100)}% of that "
                   f"level's edges deleted as one batch then inserted back as one batch",
                   tot_edges / tot_s, len(rows), 0, 1e3 * tot_s / max(len(rows), 1),
                   tot_edges // max(len(rows), 1), "persistent (one launch per batch)")
    out["levels"] = rows
    out["tuning"] = tuning
    out["roofline"] = None
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat22-stream",
                    choices=["chunglu-1m", "rmat22-stream", "chunglu-pool512", "rmat-serve", "pool-serve",
                             "paper-sweep", "core-levels"])
    ap.add_argument("--sweep-scales", default="15,16,17,18,19,20,21", help="paper-sweep: log2 n values")
    ap.add_argument("--scale", type=int, default=24, help="rmat-serve: R-MAT scale")
    ap.add_argument("--requests", type=int, default=10_000, help="rmat-serve: requests")
    ap.add_argument("--checkpoints", action="store_true",
                    help="rmat-serve: also compare 21 checkpoints of a served pass with the stored oracle states")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the launch parameters on the workload's sample first and store them")
    ap.add_argument("--tune-budget", type=float, default=300.0, help="seconds for --tune")
    ap.add_argument("--set", default="",
                    help='JSON object of launch parameters that override the tuned or default ones, '
                         'e.g. \'{"expand_mode": 3}\'')
    ap.add_argument("--no-persistent", action="store_true",
                    help="chunglu-1m: time the plain form only")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run the calibration kernels (1 GiB copy, random gather) first")
    ap.add_argument("--calibration-only", action="store_true",
                    help="run only the calibration kernels (references for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is described but not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1612_09368_amd as cm
    cm.library()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration or args.calibration_only:
        cal = calibration(torch)
        if args.calibration_only:
            print(json.dumps({"calibration": cal}), flush=True)
            teardown(torch)
            return
    fn = {"chunglu-1m": bench_cl1m, "rmat22-stream": bench_rmat22, "chunglu-pool512": bench_pool512,
          "rmat-serve": bench_serve, "pool-serve": bench_pool_serve, "paper-sweep": bench_sweep,
          "core-levels": bench_levels}
    out = fn[args.workload](args, cm, torch)
    print(json.dumps(out), flush=True)
    teardown(torch)


def calibration(torch):
    """Two kernels of known HBM footprint, the references for scaling the
    rocprofv3 byte counters: a device copy of 1 GiB (reads 1 GiB, writes
    1 GiB), and a gather of 2^21 random 4-byte values from a 1 GiB array
    whose indices hit 2^21 distinct 128-byte lines, at most one value per
    line, in random order -- the access pattern of the traversal kernels'
    neighbour gathers, with no line reused.  It reads its 16 MiB of int64
    indices plus one fetch unit per value, and writes 8 MiB."""
    n = 1 << 28
    src = torch.empty(n, dtype=torch.int32, device="cuda:0")
    dst = torch.empty_like(src)
    src.fill_(1)
    dst.copy_(src)
    rng = np.random.Generator(np.random.PCG64(11))
    lines = rng.choice(n // 32, 1 << 21, replace=False).astype(np.int64)
    idx = lines * 32 + rng.integers(0, 32, lines.size)
    didx = torch.from_numpy(idx).to("cuda:0")
    torch.cuda.synchronize()
    got = torch.take(src, didx)
    torch.cuda.synchronize()
    del src, dst, didx, got
    return {"copy": {"read_bytes": 4 * n, "write_bytes": 4 * n},
            "gather": {"values": int(idx.size), "distinct_128b_lines": int(idx.size),
                       "index_read_bytes": 8 * int(idx.size), "write_bytes": 4 * int(idx.size)}}


def teardown(torch):
    """Explicit end of the process's GPU work: every handle was closed by its
    workload; wait for the device, release torch's cached blocks and flush
    the output before the interpreter unwinds."""
    import gc
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    sys.stdout.flush()
    sys.stderr.flush()


if __name__ == "__main__":
    main()
