"""Autotuner for the launch and work-split parameters of the maintenance kernels.

The parameters are the ones of ``cm_config`` that change speed but never
results: workgroups per compute unit of the cooperative grid, the list
length above which a list is split into chunks and the chunk length
(``large_degree``, ``chunk``; shorter lists are walked flattened, up to 64
per wave), the list length walked by one lane in whole-graph passes and in
the asynchronous cascade form (``small_degree``), the cascade form itself
(``async_steps``), the expansion form (``expand_mode``: Algorithm 3's
pruned two-pass walk, the one-pass walk, the one-pass walk that records
each candidate's level-k supporters for the eviction, and that form with
up-lists kept for long lists), the claim rounds of the partition, and the sizes up to
which a step runs inside one workgroup (``local_edges``, ``local_items``,
``local_work``).

Search: coordinate descent from the library defaults.  For each parameter in
turn every candidate value is tried with the others held at the best values
so far, and a candidate replaces the best only when it is at least 3%
faster (trial-to-trial noise is a few percent).  A trial loads the graph
into a fresh handle, decomposes it and times the sample batches in the
persistent form; the defaults run once more beforehand, untimed, to warm the
device and the allocator.  Every trial's final core numbers must
equal the first trial's (a tuning change that altered a result would be a
bug, and the tuner refuses to go on).  Results are kept in a JSON file keyed
by a workload signature (device, size classes of n, m and the batches).
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import Graph, MODE_PERSISTENT, library

SPACE = {
    "large_degree": [16, 32, 64, 128, 256],
    "chunk": [32, 64, 128, 256],
    "small_degree": [2, 4, 8],
    "blocks_per_cu": [1, 2],
    "partition_rounds": [1, 2, 3],
    "local_items": [128, 512, 2048],
    "local_work": [1024, 4096, 16384],
    "local_edges": [512, 2048, 8192],
    "async_steps": [0, 1],
    "expand_mode": [1, 2, 3, 4],
}
ORDER = ["async_steps", "expand_mode", "large_degree", "chunk", "small_degree", "blocks_per_cu", "partition_rounds",
         "local_items", "local_work", "local_edges"]
DEFAULTS = {"blocks_per_cu": 1, "chunk": 256, "large_degree": 256, "small_degree": 4,
            "partition_rounds": 2, "local_items": 128, "local_work": 16384, "local_edges": 2048,
            "async_steps": 0, "expand_mode": 4}

DEFAULT_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def _class(x):
    return int(round(math.log2(max(int(x), 1))))


def signature(n, m, batch_sizes, device_name=None):
    """Workload key: device plus log2 size classes of n, m and the mean batch."""
    if device_name is None:
        import torch
        device_name = (torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
                       if torch.cuda.is_available() else "cpu")
    mean_b = float(np.mean(batch_sizes)) if len(batch_sizes) else 1.0
    return f"{device_name}|n2^{_class(n)}|m2^{_class(m)}|b2^{_class(mean_b)}"


def load_tuning(key, path=DEFAULT_FILE):
    """Best parameters stored for `key`, else None."""
    try:
        with open(path) as f:
            table = json.load(f)
    except (OSError, ValueError):
        return None
    entry = table.get(key)
    return dict(entry["params"]) if entry else None


def save_tuning(key, params, seconds, path=DEFAULT_FILE, note=""):
    try:
        with open(path) as f:
            table = json.load(f)
    except (OSError, ValueError):
        table = {}
    table[key] = {"params": params, "seconds": seconds, "note": note}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _trial(n, src, dst, kinds, offs, xs, ys, params, sub=None, nsub=0):
    import torch
    g = Graph(mode=MODE_PERSISTENT, timing=True, **params)
    try:
        g.load(n, src, dst)
        g.decompose()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, _ = g.run_batches(kinds, offs, xs, ys, sub=sub, nsub=nsub)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if any(r.status not in (0,) for r in res) and sub is None:
            raise RuntimeError("a sample batch failed validation")
        return el, g.cores()
    finally:
        g.close()


def tune(n, src, dst, kinds, offs, xs, ys, sub=None, nsub=0, space=None, order=None, sweeps=1,
         log=None, budget_s=None):
    """Coordinate-descent search; returns (best params, best seconds, trials).

    src/dst/xs/ys (and sub) should already be device tensors so that trials
    time the kernels, not transfers."""
    library()
    space = space or SPACE
    order = order or ORDER
    best = dict(DEFAULTS)
    t_start = time.time()
    # warm the device and the allocator once
    _trial(n, src, dst, kinds, offs, xs, ys, best, sub, nsub)
    best_t, ref_cores = _trial(n, src, dst, kinds, offs, xs, ys, best, sub, nsub)
    trials = [(dict(best), best_t)]
    if log:
        log(f"tune: defaults {best_t * 1e3:.1f} ms")
    for _ in range(sweeps):
        improved = False
        for name in order:
            for v in space[name]:
                if v == best[name]:
                    continue
                if budget_s is not None and time.time() - t_start > budget_s:
                    return best, best_t, trials
                cand = dict(best)
                cand[name] = v
                t, cores = _trial(n, src, dst, kinds, offs, xs, ys, cand, sub, nsub)
                if not np.array_equal(cores, ref_cores):
                    raise RuntimeError(f"tuning parameters {cand} changed the core numbers")
                trials.append((cand, t))
                if log:
                    log(f"tune: {name}={v} {t * 1e3:.1f} ms (best {best_t * 1e3:.1f})")
                if t < best_t * 0.97:
                    best, best_t, improved = cand, t, True
        if not improved:
            break
    return best, best_t, trials


def params_for(n, m, batch_sizes, path=DEFAULT_FILE):
    """(parameters, source) for a workload: the stored entry for its
    signature when there is one, else the library defaults."""
    key = signature(n, m, batch_sizes)
    stored = load_tuning(key, path)
    if stored is not None:
        return stored, f"tuning.json[{key}]"
    return dict(DEFAULTS), "library defaults"
