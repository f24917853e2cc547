"""Serving: continuous batching of update requests on one resident graph.

``Server`` wraps the ``cm_serve_*`` calls: requests are copied into the
library's pinned request ring and published; one persistent launch picks
each one up as soon as it is published (requests arriving while others run
join the running launch) and applies them in ticket order.  With ``fuse`` >
1, edge requests of distinct independent sessions that are waiting together
run fused in one batch, sharing its iterations.  A submit that
the library cannot admit yet (ring, payload space or memory budget full)
returns None; the caller polls and submits it again.

``run_stream`` drives a request stream against a server: each request is
submitted at its arrival time (or at once, closed loop), completions are
timestamped when a poll sees them, and per-request latency runs from
arrival to the poll that saw it finished.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from . import (E_BUSY, OK, BatchStats, CoreMaintError, REQ_DELETE_EDGES, REQ_DELETE_VERTICES,
               REQ_INSERT_EDGES, REQ_INSERT_VERTICES, ServeConfig, library)


def _c(a, dt):
    a = np.ascontiguousarray(a, dtype=dt)
    return a, ctypes.c_void_p(a.ctypes.data) if a.size else None


class Server:
    def __init__(self, graph, **cfg):
        self.graph = graph
        self._lib = library()
        c = ServeConfig()
        self._lib.cm_serve_config_default(ctypes.byref(c))
        for k, v in cfg.items():
            setattr(c, k, v)
        self.config = c
        graph._check(self._lib.cm_serve_start(graph._h, ctypes.byref(c)), "cm_serve_start")
        self.active = True

    def _submit(self, st, ticket, what):
        if st == E_BUSY:
            return None
        self.graph._check(st, what)
        return int(ticket.value)

    def submit_edges(self, kind, src, dst, session=-1):
        """kind REQ_INSERT_EDGES / REQ_DELETE_EDGES; session >= 0 names an
        independent session (see cm_serve_submit_edges); returns the ticket
        or None (busy)."""
        s, ps = _c(src, np.int32)
        d, pd = _c(dst, np.int32)
        if s.size != d.size:
            raise ValueError("src and dst differ in length")
        t = ctypes.c_int64()
        return self._submit(self._lib.cm_serve_submit_edges(self.graph._h, int(session), kind, s.size, ps, pd,
                                                            ctypes.byref(t)),
                            t, "cm_serve_submit_edges")

    def submit_insert_vertices(self, off, nbrs):
        """Returns (ticket, first new id) or None (busy)."""
        o, po = _c(off, np.int64)
        nb, pn = _c(nbrs, np.int32)
        first = ctypes.c_int32()
        t = ctypes.c_int64()
        st = self._lib.cm_serve_submit_insert_vertices(self.graph._h, o.size - 1, po, pn, ctypes.byref(first),
                                                       ctypes.byref(t))
        r = self._submit(st, t, "cm_serve_submit_insert_vertices")
        return None if r is None else (r, int(first.value))

    def submit_delete_vertices(self, ids):
        i, pi = _c(ids, np.int32)
        t = ctypes.c_int64()
        return self._submit(self._lib.cm_serve_submit_delete_vertices(self.graph._h, i.size, pi, ctypes.byref(t)),
                            t, "cm_serve_submit_delete_vertices")

    def poll(self):
        """Requests finished so far (every ticket below the returned count)."""
        n = ctypes.c_int64()
        self.graph._check(self._lib.cm_serve_poll(self.graph._h, ctypes.byref(n)), "cm_serve_poll")
        return int(n.value)

    def result(self, ticket):
        r = BatchStats()
        st = self._lib.cm_serve_result(self.graph._h, int(ticket), ctypes.byref(r))
        if st == E_BUSY:
            return None
        self.graph._check(st, "cm_serve_result")
        return r

    def stop(self):
        if self.active:
            self.active = False
            self.graph._check(self._lib.cm_serve_stop(self.graph._h), "cm_serve_stop")


def submit_request(server, req, session=-1):
    """req: ("ins", src, dst) | ("del", src, dst) | ("vins", off, nbrs) | ("vdel", ids).
    Returns (ticket, first new id or -1) or None when busy."""
    kind = req[0]
    if kind == "ins":
        t = server.submit_edges(REQ_INSERT_EDGES, req[1], req[2], session)
        return None if t is None else (t, -1)
    if kind == "del":
        t = server.submit_edges(REQ_DELETE_EDGES, req[1], req[2], session)
        return None if t is None else (t, -1)
    if kind == "vins":
        return server.submit_insert_vertices(req[1], req[2])
    if kind == "vdel":
        t = server.submit_delete_vertices(req[1])
        return None if t is None else (t, -1)
    raise ValueError(kind)


def request_updates(req):
    """Edge updates a request stands for (a vertex op counts its edges; a
    vertex deletion's count is only known after it ran: use `applied`)."""
    if req[0] in ("ins", "del"):
        return len(req[1])
    if req[0] == "vins":
        return int(req[1][-1])
    return 0


def run_stream(server, requests, arrivals=None, poll_sleep=0.0, sessions=None):
    """Submit `requests` in order at `arrivals` (seconds from the start; None
    = as fast as admission allows) and wait for all of them; sessions[i]
    (optional) is request i's independent session.

    Returns dict with per-request arrays: ticket, first_id, t_arrival,
    t_submit, t_done (seconds) and the BatchStats of each request."""
    n = len(requests)
    t_arr = np.zeros(n) if arrivals is None else np.asarray(arrivals, dtype=np.float64)
    t_sub = np.full(n, np.nan)
    t_done = np.full(n, np.nan)
    tickets = np.full(n, -1, dtype=np.int64)
    first_ids = np.full(n, -1, dtype=np.int64)
    t0 = time.perf_counter()
    nxt = 0
    done_seen = server.poll()  # tickets of this stream start at or after it
    last = -1
    by_ticket = {}
    while nxt < n or done_seen <= last:
        now = time.perf_counter() - t0
        while nxt < n and t_arr[nxt] <= now:
            r = submit_request(server, requests[nxt], -1 if sessions is None else int(sessions[nxt]))
            if r is None:
                break
            tickets[nxt], first_ids[nxt] = r
            by_ticket[r[0]] = nxt
            last = r[0]
            t_sub[nxt] = time.perf_counter() - t0
            nxt += 1
        fin = server.poll()
        if fin > done_seen:
            tnow = time.perf_counter() - t0
            for tk in range(done_seen, fin):
                if tk in by_ticket:
                    t_done[by_ticket[tk]] = tnow
            done_seen = fin
        elif poll_sleep:
            time.sleep(poll_sleep)
    stats = [server.result(int(tk)) for tk in tickets]
    return {"ticket": tickets, "first_id": first_ids, "t_arrival": t_arr, "t_submit": t_sub,
            "t_done": t_done, "stats": stats, "elapsed": time.perf_counter() - t0}
