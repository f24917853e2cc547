// Load-balanced walks over frontier queues (gfx950, wave64).
//
// A frontier is a list of vertices plus a list of chunk items for long
// adjacency lists.  Each wave takes a batch of up to 64 queue entries and
// walks their lists laid end to end, one slot per lane per step, so short
// and medium lists keep every lane busy; lists longer than `large` never
// enter the vertex list -- the pusher splits them into chunk items that
// separate waves walk.  Pushes go through per-wave LDS buffers so that a
// queue tail takes one atomic per 64 or more entries.
#pragma once
#include "cm_internal.h"

namespace cm {

// Append the chunk items (w, 0), .., (w, nch - 1) of every lane (nch = 0
// for none) to a chunk queue with one tail atomic per wave: returning
// atomics on one word serialise (about 11 ns each), and one per long list
// bound the rounds that push many of them.  The wave writes the items
// together, lane i taking items i, i + 64, ..., so a very long list does
// not serialise on its own lane.  A wave with inactive lanes (the last pass
// of a strided loop) pushes lane by lane instead.
__device__ __forceinline__ void push_chunks(const KArgs &a, int64_t *hq, int32_t *htail, int32_t w,
                                            int32_t nch) {
    if (__ballot(nch > 0) == 0ull) return;
    if (__ballot(1) != ~0ull) {
        if (nch > 0) {
            const int32_t base = atomicAdd(htail, nch);
            for (int32_t c = 0; c < nch; ++c) {
                if (base + c < a.q.hcap) hq[base + c] = chunk_item(w, c);
                else atomicOr(&a.ctl->overflow, 1);
            }
        }
        return;
    }
    int32_t incl = nch;
    for (int o = 1; o < WAVE; o <<= 1) {
        const int32_t t = __shfl_up(incl, o);
        if (lane() >= o) incl += t;
    }
    const int32_t total = __shfl(incl, WAVE - 1);
    const int32_t excl = incl - nch;
    int32_t base = 0;
    if (lane() == 0) base = atomicAdd(htail, total);
    base = __shfl(base, 0);
    for (int32_t e0 = 0; e0 < total; e0 += WAVE) {
        const int32_t e = e0 + lane();
        // owner of item e: the last lane whose items start at or before e
        // (a lane with no items shares its start with the next lane, so
        // the owner of a valid item always has items)
        int32_t j = 0;
        for (int s = WAVE / 2; s > 0; s >>= 1) {
            const int32_t xc = __shfl(excl, j + s);
            if (xc <= e) j += s;
        }
        const int32_t xj = __shfl(excl, j);
        const int32_t wj = __shfl(w, j);
        if (e < total) {
            const int32_t pos = base + e;
            if (pos < a.q.hcap) hq[pos] = chunk_item(wj, e - xj);
            else atomicOr(&a.ctl->overflow, 1);
        }
    }
}

// Route a pushed vertex: short/medium lists to the vertex queue, long lists
// as `nchunks` items to the chunk queue.  All lanes may call it (pred
// selects the pushing lanes).
__device__ __forceinline__ void push_vertex(const KArgs &a, int32_t *vq, int32_t *vtail, int64_t *hq,
                                            int32_t *htail, int32_t w, bool pred) {
    int32_t L = pred ? a.g.len[w] : 0;
    bool big = pred && L > a.t.large_deg;
    push_agg<int32_t>(vq, a.q.vcap, vtail, w, pred && !big, &a.ctl->overflow);
    push_chunks(a, hq, htail, w, big ? nchunks(L, a.t.chunk) : 0);
}

// Per-wave push buffers in LDS.  A queue tail is one word that every wave
// appends to, and returning atomics on one address serialise (about 11 ns
// each on gfx950), so a traversal step that pushed with one atomic per wave
// per step was bound by that word.  A wave instead collects its pushes in
// LDS and appends them with one atomic per 64 or more entries; a round
// flushes its buffers before its barrier.  wb_push / push_vertex_wb must be
// called by every lane of the wave (pred selects the pushing lanes).
constexpr int PUSH_SLOTS = 3;
struct WaveBuf {
    int32_t *buf;  // 2 * WAVE entries of this wave's slot
    int32_t n;     // entries held (uniform over the wave)
};
__device__ __forceinline__ WaveBuf wave_buf(int slot) {
    __shared__ int32_t lds_push[PUSH_SLOTS][COOP_THREADS / WAVE][2 * WAVE];
    return WaveBuf{lds_push[slot][threadIdx.x / WAVE], 0};
}
__device__ __forceinline__ void wb_flush(WaveBuf &b, int32_t *q, int32_t qcap, int32_t *tail, int32_t *overflow) {
    if (b.n == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // other lanes' LDS writes come first
    int base = 0;
    if (lane() == 0) base = atomicAdd(tail, b.n);
    base = __shfl(base, 0);
    for (int i = lane(); i < b.n; i += WAVE) {
        const int pos = base + i;
        if (pos < qcap) q[pos] = b.buf[i];
        else atomicOr(overflow, 1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // reads done before the slots are reused
    b.n = 0;
}
__device__ __forceinline__ void wb_push(WaveBuf &b, int32_t *q, int32_t qcap, int32_t *tail, int32_t val,
                                        bool pred, int32_t *overflow) {
    const unsigned long long m = __ballot(pred);
    if (m == 0ull) return;
    if (pred) b.buf[b.n + __popcll(m & ((1ull << lane()) - 1ull))] = val;
    b.n += __popcll(m);
    if (b.n >= WAVE) wb_flush(b, q, qcap, tail, overflow);
}
// push_vertex through a wave buffer (long lists go straight to the chunk
// queue, one atomic per wave), for a walk of L entries of w (the caller
// gives L: the list length, or the length of another per-vertex run) and
// runs longer than `large` split into items of `chunk` entries.
__device__ __forceinline__ void push_vertex_wb_len(const KArgs &a, WaveBuf &b, int32_t *vq, int32_t *vtail,
                                                   int64_t *hq, int32_t *htail, int32_t w, int32_t L,
                                                   bool pred, int32_t large, int32_t chunk) {
    const bool big = pred && L > large;
    wb_push(b, vq, a.q.vcap, vtail, w, pred && !big, &a.ctl->overflow);
    push_chunks(a, hq, htail, w, big ? nchunks(L, chunk) : 0);
}
// ... for a walk of w's whole list
__device__ __forceinline__ void push_vertex_wb(const KArgs &a, WaveBuf &b, int32_t *vq, int32_t *vtail,
                                               int64_t *hq, int32_t *htail, int32_t w, bool pred) {
    push_vertex_wb_len(a, b, vq, vtail, hq, htail, w, pred ? a.g.len[w] : 0, pred, a.t.large_deg, a.t.chunk);
}

// Team-stride over the implicit identity list 0..n-1 (whole-graph passes).
// fl(v, L) runs on the owning lane for lists of length <= small; fw(v, L)
// runs on the whole wave (uniform) for the others, of any length.
template <class FL, class FW>
__device__ __forceinline__ void for_all_vertices(const Team &T, int32_t n, const DevGraph &g, int32_t small,
                                                 FL &&fl, FW &&fw) {
    const int step = T.nwaves() * WAVE;
    for (int32_t base = T.wave() * WAVE; base < n; base += step) {
        int32_t v = base + lane();
        bool ok = v < n && g.core[v] != -1;  // -1 marks a dead id
        int32_t L = ok ? g.len[v] : 0;
        if (ok && L <= small) fl(v, L);
        unsigned long long m = __ballot(ok && L > small);
        while (m) {
            int src = __ffsll((long long)m) - 1;
            m &= m - 1ull;
            int32_t vv = __shfl(v, src);
            int32_t LL = __shfl(L, src);
            fw(vv, LL);
        }
    }
}

// Team-stride over chunk items, one wave per item: fc(v, lo, hi, nch).
template <class FC>
__device__ __forceinline__ void for_chunks(const Team &T, const int64_t *q, int32_t n, const DevGraph &g,
                                           int32_t chunk, FC &&fc) {
    for (int32_t j = T.wave(); j < n; j += T.nwaves()) {
        int64_t it = q[j];
        int32_t v = item_v(it), c = item_c(it);
        int32_t L = g.len[v];
        int32_t lo = c * chunk;
        int32_t hi = lo + chunk < L ? lo + chunk : L;
        fc(v, lo, hi, nchunks(L, chunk));
    }
}

// Wave walk of slots [lo, hi) of v: every lane calls f(w, slot) each step
// (w < 0 for padding lanes and tombstones) so f may use wave votes.
template <class F>
__device__ __forceinline__ void wave_walk(const DevGraph &g, int32_t v, int32_t lo, int32_t hi, F &&f) {
    const int32_t *p = g.nbr + g.off[v];
    for (int32_t s = lo; s < hi; s += WAVE) {
        int32_t i = s + lane();
        int32_t w = (i < hi) ? p[i] : -1;
        f(w, i);
    }
}

// Wave walk of slots [lo, hi) of v, up to WALK_STEPS steps at a time: the
// entries of those steps are loaded, then pre(w) gathers one word per entry
// (it must read data that f does not change during the walk), before
// f(w, pre(w)) runs step by step on every lane (w < 0: padding or a
// tombstone).  The reads of a step then overlap those of the next ones: a
// walk of a long list is bound by the latency of its dependent reads.
constexpr int WALK_STEPS = 4;
template <class P, class F>
__device__ __forceinline__ void wave_walk_pre(const DevGraph &g, int32_t v, int32_t lo, int32_t hi, P &&pre,
                                              F &&f) {
    const int32_t *p = g.nbr + g.off[v];
    for (int32_t s0 = lo; s0 < hi; s0 += WALK_STEPS * WAVE) {
        int32_t w[WALK_STEPS], x[WALK_STEPS];
#pragma unroll
        for (int u = 0; u < WALK_STEPS; ++u) {
            const int32_t i = s0 + u * WAVE + lane();
            w[u] = i < hi ? p[i] : -1;
        }
#pragma unroll
        for (int u = 0; u < WALK_STEPS; ++u) x[u] = w[u] >= 0 ? pre(w[u]) : -1;
#pragma unroll
        for (int u = 0; u < WALK_STEPS; ++u)
            if (s0 + u * WAVE < hi) f(w[u], x[u]);
    }
}

// Wave walk of chunk [lo, hi) of v through v's up-list (ub = ubl[v] >= 0):
// the chunk's compacted up-list entries, built from slots [lo, min(hi, ub))
// and ending at a negative entry when fewer, then the slots appended since
// (from ub on).  f(w) runs on every lane each step (w < 0: none).  Returns
// the entries read (uniform).
template <class F>
__device__ __forceinline__ int32_t walk_chunk_up(const DevGraph &g, int32_t v, int32_t lo, int32_t hi,
                                                 int32_t ub, F &&f) {
    int32_t seen = 0;
    const int32_t hb = hi < ub ? hi : ub;
    const int32_t *up = g.upl + g.off[v] + lo;
    for (int32_t s = 0; lo + s < hb; s += WAVE) {
        const int32_t i = s + lane();
        int32_t w = lo + i < hb ? up[i] : -1;
        const unsigned long long neg = __ballot(w < 0);
        if (neg && lane() >= __ffsll((long long)neg) - 1) w = -1;
        seen += neg ? __ffsll((long long)neg) - 1 : WAVE;
        f(w);
        if (neg) break;
    }
    const int32_t ab = lo > ub ? lo : ub;
    if (ab < hi) {
        seen += hi - ab;
        wave_walk(g, v, ab, hi, [&](int32_t w, int32_t) { f(w); });
    }
    return seen;
}

// Team-stride over a vertex queue in batches of up to 64 entries per wave:
// a wave takes `per` consecutive entries, per = ceil(n / waves) capped at
// 64, so a queue shorter than 64 entries per wave is spread over every wave
// instead of leaving most waves idle.  fb(v) runs on the whole wave with
// lane j holding entry j of the batch (v < 0 past the end).  n must be the
// same in every thread of the team.
template <class FB>
__device__ __forceinline__ void for_batches(const Team &T, const int32_t *q, int32_t n, FB &&fb) {
    const int nw = T.nwaves();
    int per = (int)(((int64_t)n + nw - 1) / nw);
    per = per < 1 ? 1 : (per > WAVE ? WAVE : per);
    const int step = nw * per;
    for (int32_t base = T.wave() * per; base < n; base += step) {
        const int32_t i = base + lane();
        fb((lane() < per && i < n) ? q[i] : -1);
    }
}

// Flattened walk over the lists of a wave's batch: lane j holds vertex v_j
// and the number L_j of leading slots of its list to walk (0 for none).
// The lists are laid end to end and every lane takes one slot per step, so
// a batch of short and medium lists keeps all 64 lanes busy with 64 loads
// in flight instead of walking the lists one after another.  f(j, w, own,
// oj, lo) runs on every lane each step (it may use wave votes): j = the lane
// whose list holds the slot this lane reads (-1 when it reads none), w = the
// slot's entry of `arr` (< 0 for a tombstone or none), own = the lanes that
// read a slot of THIS lane's list in this step, so that
// popcount(ballot(p) & own) counts p over this lane's slots; oj = the first
// slot of lane j's list and lo = the first lane of this step that reads
// from lane j's list (lanes lo .. this lane - 1 read the slots just before
// this one), for writing compacted per-list output.  arr is the adjacency
// pool or an array with its slot ranges.
template <class F>
__device__ __forceinline__ void flat_walk_pos(const int32_t *arr, const DevGraph &g, int32_t v, int32_t L,
                                              F &&f) {
    int32_t incl = L;
    for (int o = 1; o < WAVE; o <<= 1) {
        const int32_t t = __shfl_up(incl, o);
        if (lane() >= o) incl += t;
    }
    const int32_t total = __shfl(incl, WAVE - 1);
    const int32_t excl = incl - L;
    const int64_t off = v >= 0 ? g.off[v] : 0;  // independent of L: issues with the length load
    for (int32_t base = 0; base < total; base += WAVE) {
        const int32_t e = base + lane();
        // owner of slot e: the last lane whose list starts at or before e
        int32_t j = 0;
        for (int s = WAVE / 2; s > 0; s >>= 1) {
            const int32_t xc = __shfl(excl, j + s);
            if (xc <= e) j += s;
        }
        const int32_t xj = __shfl(excl, j);
        const int64_t oj = __shfl(off, j);
        const bool has = e < total;
        const int32_t w = has ? arr[oj + (e - xj)] : -1;
        int32_t lo = excl - base, hi = incl - base;
        lo = lo < 0 ? 0 : (lo > WAVE ? WAVE : lo);
        hi = hi < 0 ? 0 : (hi > WAVE ? WAVE : hi);
        const unsigned long long own =
            hi > lo ? ((hi - lo == WAVE ? ~0ull : ((1ull << (hi - lo)) - 1ull)) << lo) : 0ull;
        const int32_t loj = xj - base > 0 ? xj - base : 0;
        f(has ? j : -1, w, own, oj, loj);
    }
}
// The same over the adjacency pool, without the position arguments.
template <class F>
__device__ __forceinline__ void flat_walk(const DevGraph &g, int32_t v, int32_t L, F &&f) {
    flat_walk_pos(g.nbr, g, v, L, [&](int32_t j, int32_t w, unsigned long long own, int64_t, int32_t) {
        f(j, w, own);
    });
}

// Team-stride over a vertex queue visiting every slot of every list:
// fs(w, k) runs on every lane per step, k = core number of the list's
// owner (w < 0: no slot or a tombstone).  Lists of up to `large` slots are
// walked flattened, batch by batch; a longer one (possible only for queue
// entries not routed through push_vertex) is walked by the wave alone.
// Returns the slots visited by this lane's owned lists (for statistics).
template <class FS>
__device__ __forceinline__ long long for_vertex_slots(const Team &T, const int32_t *q, int32_t n,
                                                      const DevGraph &g, int32_t large, FS &&fs) {
    long long seen = 0;
    for_batches(T, q, n, [&](int32_t v) {
        const int32_t L = v >= 0 ? g.len[v] : 0;
        const int32_t k = v >= 0 ? g.core[v] : 0;
        const bool big = L > large;
        seen += L;
        flat_walk(g, v, big ? 0 : L, [&](int32_t j, int32_t w, unsigned long long) {
            fs(w, __shfl(k, j < 0 ? 0 : j));
        });
        unsigned long long m = __ballot(big);
        while (m) {
            const int src = __ffsll((long long)m) - 1;
            m &= m - 1ull;
            const int32_t vv = __shfl(v, src);
            const int32_t kk = __shfl(k, src);
            wave_walk(g, vv, 0, __shfl(L, src), [&](int32_t w, int32_t) { fs(w, kk); });
        }
    });
    return seen;
}

}  // namespace cm
