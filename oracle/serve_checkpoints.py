"""Expected state of the served R-MAT stream at evenly spaced checkpoints --
TEST INFRASTRUCTURE ONLY (the oracle applied to the same seeded request stream
the serving benchmark generates; nothing from the GPU path is read).

For `requests` requests, checkpoints fall after requests round(i * N / 21),
i = 1..20, and after the last one (21 states).  Each checkpoint records the
SHA-256 of the int32 core vector (dead ids -1, Batagelj-Zaversnik from
scratch on the oracle's own edge set), the id count and the edge count; the
per-request statuses (serving conventions: a rejected vertex insertion keeps
its ids as dead ids) are recorded as a digest and a count of failures.

    python -m oracle.serve_checkpoints --scale 24 --requests 10000 \\
        --out tests/golden/serve_checkpoints_r24.json
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import graphgen  # noqa: E402
import oracle  # noqa: E402


def checkpoints(nreq, parts=21):
    return sorted({int(round(i * nreq / parts)) for i in range(1, parts)} | {nreq})


def cores_digest(cores):
    return hashlib.sha256(np.ascontiguousarray(cores, dtype=np.int32).tobytes()).hexdigest()


def apply(ref, req):
    if req[0] == "ins":
        return ref.insert_edges(req[1], req[2])[0]
    if req[0] == "del":
        return ref.delete_edges(req[1], req[2])[0]
    if req[0] == "vins":
        return ref.insert_vertices(req[1], req[2], keep_failed_ids=True)[0]
    return ref.delete_vertices(req[1])[0]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--requests", type=int, default=10_000)
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    t = time.time()

    def log(m):
        print(f"[{time.time() - t:.0f}s] {m}", flush=True)

    oracle.build(force=False)
    n, s, d, reqs = graphgen.serve_stream(args.scale, args.requests, graphgen.rng_for("bench-serve"),
                                          workers=args.workers, progress=log)
    log(f"stream: n={n} m={s.size}, {len(reqs)} requests")
    ref = oracle.DynamicGraph(n, s, d)
    del s, d
    marks = checkpoints(len(reqs))
    statuses, states = [], []
    for j, r in enumerate(reqs):
        statuses.append(int(apply(ref, r)))
        if j + 1 in marks:
            c = ref.cores()
            states.append({"after": j + 1, "cores_sha256": cores_digest(c), "n_ids": int(c.size),
                           "m": ref.num_edges(), "kmax": int(c.max()) if c.size else 0})
            log(f"checkpoint after {j + 1}: m={ref.num_edges()}")
    st = np.asarray(statuses, dtype=np.int32)
    out = {"workload": {"scale": args.scale, "requests": args.requests, "seed_tag": "bench-serve"},
           "checkpoints": states,
           "statuses_sha256": hashlib.sha256(st.tobytes()).hexdigest(),
           "failed_requests": int((st != 0).sum()),
           "written_by": "python -m oracle.serve_checkpoints"}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    log(f"wrote {args.out}")


if __name__ == "__main__":
    main()
