"""Reader for the hand-derived fixtures in this folder.

Each fixture lists a start graph and its core numbers, then a sequence of
batches (``insert`` / ``delete`` lines of ``a-b`` pairs), each followed by the
expected core numbers.  The expected values are derived by hand in each file's
header comment, from the definitions of Section III, not by running code."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _pairs(tokens):
    s, d = [], []
    for t in tokens:
        a, b = t.split("-")
        s.append(int(a))
        d.append(int(b))
    return np.asarray(s, dtype=np.int32), np.asarray(d, dtype=np.int32)


def load(name):
    n = None
    edges = None
    start = None
    steps = []
    pending = None
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            head, *rest = line.split()
            if head == "n":
                n = int(rest[0])
            elif head == "edges":
                edges = _pairs(rest)
            elif head == "cores":
                vals = np.asarray([int(x) for x in rest], dtype=np.int32)
                if pending is None:
                    start = vals
                else:
                    steps.append((pending[0], pending[1], pending[2], vals))
                    pending = None
            elif head in ("insert", "delete"):
                s, d = _pairs(rest)
                pending = (head, s, d)
    return {"n": n, "edges": edges, "cores": start, "steps": steps}


def all_cases():
    return sorted(f for f in os.listdir(HERE) if f.endswith(".txt"))
