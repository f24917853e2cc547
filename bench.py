"""Benchmark: edge updates per second of batched core maintenance on one MI355X.

Workload (one step = the whole maintenance path over one batch pair):
Chung-Lu power-law graph, n = 1,000,000, m = 10,000,000, degree exponent 2.1,
largest weight 50,000 (seeded, synthetic); every step inserts 100,000
degree-weighted non-edges and then deletes 100,000 uniformly drawn existing
edges, with exact core numbers after each batch.  `value` is the plain form
(one cooperative launch per superior edge set, host checks termination);
the persistent form (one launch per batch) is reported beside it on the same
batches.  Inputs are resident in device memory before the timed region.

Prints one JSON line (see the fields below).
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

N_VERT = 1_000_000
N_EDGE = 10_000_000
GAMMA = 2.1
W_MAX = 50_000.0
BATCH = 100_000
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(steps: int):
    import graphgen
    rng = graphgen.rng_for("bench-cl-1m")
    t = time.time()
    s, d = graphgen.chung_lu_graph(N_VERT, N_EDGE, GAMMA, W_MAX, rng)
    log(f"graph generated in {time.time() - t:.1f}s (m={s.size})")
    es = graphgen.EdgeSet(s, d)
    batches = []
    for k in range(steps):
        a, b = graphgen.weighted_non_edges(BATCH, es, rng)
        es.insert(a, b)
        x, y = graphgen.existing_edges(BATCH, es, rng)
        es.delete(x, y)
        batches.append(((a, b), (x, y)))
    log(f"{steps} batch pairs generated")
    return s, d, batches


def run_form(cm, torch, s, d, dev_batches, mode, warmup, steps, timing):
    dev = torch.device("cuda:0")
    g = cm.Graph(mode=mode, timing=timing)
    g.load(N_VERT, torch.from_numpy(s).to(dev), torch.from_numpy(d).to(dev))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dst = g.decompose()
    torch.cuda.synchronize()
    dec_ms = (time.perf_counter() - t0) * 1e3
    lat = []
    stats = []
    for k in range(warmup):
        (a, b), (x, y) = dev_batches[k]
        g.insert_edges(a, b)
        g.delete_edges(x, y)
    torch.cuda.synchronize()
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
    cores = g.cores()
    g.close()
    return {"elapsed": elapsed, "lat": lat, "stats": stats, "dec_ms": dec_ms,
            "dec_stats": dst.as_dict(), "cores": cores}


def cpu_baseline(s, d, batch):
    """The oracle as it stands: apply the batch to its host edge set and
    recompute every core number (BZ), for one insert and one delete batch."""
    import oracle
    oracle.build(force=False)
    ref = oracle.DynamicGraph(N_VERT, s, d)
    (a, b), (x, y) = batch
    t0 = time.perf_counter()
    ref.insert_edges(a, b)
    ref.cores()
    ref.delete_edges(x, y)
    c = ref.cores()
    el = time.perf_counter() - t0
    return 2 * BATCH / el, el, c


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-persistent", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is described but not built)", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import torch
    import paper_1612_09368_amd as cm
    cm.library()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    s, d, batches = make_workload(args.warmup + args.steps)
    dev_batches = [tuple(tuple(torch.from_numpy(np.ascontiguousarray(z)).to(dev) for z in pair)
                         for pair in step) for step in batches]
    torch.cuda.synchronize()

    plain = run_form(cm, torch, s, d, dev_batches, cm.MODE_PLAIN, args.warmup, args.steps, True)
    log(f"plain: {plain['elapsed']:.3f}s for {args.steps} steps")
    pers = None
    if not args.no_persistent:
        pers = run_form(cm, torch, s, d, dev_batches, cm.MODE_PERSISTENT, args.warmup, args.steps, True)
        log(f"persistent: {pers['elapsed']:.3f}s")
        assert np.array_equal(plain["cores"], pers["cores"]), "plain and persistent forms disagree"

    updates = 2 * BATCH * args.steps
    value = updates / plain["elapsed"]
    st = plain["stats"]
    kms = sum(x["kernel_ms"] for x in st)
    launches = sum(x["launches"] for x in st)
    abytes = sum(x["alg_bytes"] for x in st)
    achieved = (abytes / (kms * 1e-3)) / 1e9 if kms > 0 else 0.0
    lat = np.asarray(plain["lat"])
    out = {
        "metric": "edge updates/sec (insert & delete, exact cores) batched vs plain on 1 GPU; p99 latency",
        "value": value,
        "unit": "edge_updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": plain["elapsed"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "chung-lu n=1000000 m=10000000 gamma=2.1 wmax=50000; per step insert 100000 "
                        "degree-weighted non-edges then delete 100000 existing edges",
            "form": "plain (one cooperative launch per superior edge set)",
            "global_batch": 2 * BATCH,
            "parallelism": "single-gpu",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_maintain",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "alg_bytes_per_launch": abytes / max(launches, 1),
            "avg_launch_us": kms * 1e3 / max(launches, 1),
            "launches": launches,
        },
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "per": "batch of 100000 edges"},
        "iterations_per_batch": [x["iterations"] for x in st],
        "rounds_per_batch": [x["rounds"] for x in st],
        "steps_per_batch": [x["grid_steps"] + x["local_steps"] for x in st],
        "decompose": {"ms": plain["dec_ms"], "kernel_ms": plain["dec_stats"]["kernel_ms"],
                      "edges_per_s": N_EDGE / (plain["dec_ms"] * 1e-3)},
    }
    if pers is not None:
        pst = pers["stats"]
        pk = sum(x["kernel_ms"] for x in pst)
        pl = sum(x["launches"] for x in pst)
        pb = sum(x["alg_bytes"] for x in pst)
        plat = np.asarray(pers["lat"])
        out["batched"] = {
            "form": "persistent (one cooperative launch per batch)",
            "value": updates / pers["elapsed"],
            "ms_per_step": pers["elapsed"] * 1e3 / args.steps,
            "speedup_vs_plain": plain["elapsed"] / pers["elapsed"],
            "latency_ms": {"p50": float(np.percentile(plat, 50)), "p99": float(np.percentile(plat, 99))},
            "roofline_achieved_gbs": (pb / (pk * 1e-3)) / 1e9 if pk > 0 else 0.0,
            "avg_launch_us": pk * 1e3 / max(pl, 1),
        }
    if rank == 0 and not args.no_cpu_baseline:
        v, el, cref = cpu_baseline(s, d, batches[0])
        out["cpu_baseline"] = {"value": v, "unit": "edge_updates/s", "cores": 1, "kind": "oracle",
                               "sample": "one insert batch + one delete batch of the workload "
                                         f"(200000 updates, {el:.1f}s): host edge-set apply + "
                                         "Batagelj-Zaversnik recompute after each batch"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
