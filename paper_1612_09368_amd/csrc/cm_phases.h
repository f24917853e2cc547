// Device phases of batched core maintenance.  Each phase is a grid-stride
// __device__ function; the plain driver runs an iteration's phases inside one
// cooperative launch (grid barriers between phases), the persistent driver
// loops over iterations inside one launch.
//
// Notation follows the paper: core(v); SD(v) = superior degree, neighbours w
// with core(w) >= core(v) (kept in `mcd`); CSD(v) = constraint superior
// degree, neighbours w with core(w) > core(v) or core(w) == core(v) and
// SD(w) > core(v); cd = the working counter of Algorithms 3/4 and 6/7.
#pragma once
#include "cm_walk.h"

namespace cm {

// Status codes (match coremaint.h).
constexpr int32_t ST_RANGE = -2, ST_SELF = -3, ST_DUP = -4, ST_EXISTS = -5, ST_MISSING = -6,
                  ST_DEAD = -7;

__device__ __forceinline__ void flush_stat(unsigned long long *dst, long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane() == 0 && v) atomicAdd(dst, (unsigned long long)v);
}

// Queue length as published by its tail, clamped to the buffer capacity
// (a tail can pass the capacity only after an overflow, which aborts the batch).
__device__ __forceinline__ int32_t qlen(const int32_t *tail, int32_t cap) {
    int32_t n = ld_acq(tail);
    return n < cap ? n : cap;
}

// Count the active lanes with pred set into *ctr (one atomic per wave).
__device__ __forceinline__ void count_agg(int32_t *ctr, bool pred) {
    unsigned long long m = __ballot(pred);
    unsigned long long act = __ballot(1);
    if (m && lane() == __ffsll((long long)act) - 1) atomicAdd(ctr, __popcll(m));
}

// ===========================================================================
// Batch validation (boundary convention; simple graph, Section III)
// ===========================================================================

// V1: range / dead / self-loop checks, canonical (min, max), hash insert
// (the smallest item index of each pair wins the slot).
__device__ void val_canon(const KArgs &a) {
    const int32_t n = a.g.n_ids;
    const uint32_t mask = (uint32_t)a.b.hcap - 1u;
    for (int32_t i = gtid(); i < a.s; i += gthreads()) {
        int32_t u = a.b.src_in[i], v = a.b.dst_in[i];
        int32_t e = 0;
        if (u < 0 || v < 0 || u >= n || v >= n) e = ST_RANGE;
        else if (a.g.core[u] < 0 || a.g.core[v] < 0) e = ST_DEAD;
        else if (u == v) e = ST_SELF;
        int32_t lo = u < v ? u : v, hi = u < v ? v : u;
        a.b.eu[i] = lo;
        a.b.ev[i] = hi;
        a.b.su[i] = -1;
        a.b.sv[i] = -1;
        a.b.err[i] = e;
        a.b.hslot[i] = -1;
        if (e == 0) {
            unsigned long long key = edge_key(lo, hi);
            uint32_t h = hash_key(key) & mask;
            for (uint32_t probe = 0; probe <= mask; ++probe) {
                unsigned long long old = atomicCAS(&a.b.hkey[h], EMPTY_KEY, key);
                if (old == EMPTY_KEY || old == key) break;
                h = (h + 1u) & mask;
            }
            a.b.hslot[i] = (int32_t)h;
            atomicMin(&a.b.hval[h], i);
        }
    }
}

__device__ __forceinline__ void mark_scan(const KArgs &a, int32_t x) {
    if (atomicExch(&a.g.bmark[x], a.bstamp) != a.bstamp) {
        int32_t L = a.g.len[x];
        int nch = nchunks(L, a.t.chunk);
        if (nch > 0) {
            int base = atomicAdd(&a.ctl->scan_tail, nch);
            for (int c = 0; c < nch; ++c) {
                if (base + c < a.b.scap) a.b.scanq[base + c] = chunk_item(x, c);
                else atomicOr(&a.ctl->overflow, 1);
            }
        }
    }
}

// V2: duplicates inside the batch; choose the lists the locate scan reads
// (insertion: the shorter endpoint list is enough to test existence;
// deletion: both lists, to find both slots).
__device__ void val_dup_mark(const KArgs &a) {
    for (int32_t i = gtid(); i < a.s; i += gthreads()) {
        int32_t e = a.b.err[i];
        if (e != 0) continue;
        if (a.b.hval[a.b.hslot[i]] != i) {
            a.b.err[i] = ST_DUP;
            continue;
        }
        int32_t u = a.b.eu[i], v = a.b.ev[i];
        if (a.inserting) {
            mark_scan(a, a.g.len[u] <= a.g.len[v] ? u : v);
        } else {
            mark_scan(a, u);
            mark_scan(a, v);
        }
    }
}

// V3: locate scan.  Each (vertex, chunk) item is read by one wave; every
// live neighbour probes the batch hash.  Insertion: a hit means the edge
// exists.  Deletion: a hit records the slot of the entry.
__device__ void val_scan(const KArgs &a) {
    const uint32_t mask = (uint32_t)a.b.hcap - 1u;
    const int32_t n = qlen(&a.ctl->scan_tail, a.b.scap);
    for_chunks(a.b.scanq, n, a.g, a.t.chunk,
               [&](int32_t x, int32_t lo, int32_t hi, int32_t) {
                   const int64_t base = a.g.off[x];
                   wave_walk(a.g, x, lo, hi, [&](int32_t w, int32_t slot) {
                       if (w < 0) return;
                       unsigned long long key = edge_key(x, w);
                       uint32_t h = hash_key(key) & mask;
                       for (uint32_t probe = 0; probe <= mask; ++probe) {
                           unsigned long long k2 = a.b.hkey[h];
                           if (k2 == EMPTY_KEY) break;
                           if (k2 == key) {
                               int32_t i = a.b.hval[h];
                               if (a.inserting) {
                                   a.b.err[i] = ST_EXISTS;
                               } else if (x == a.b.eu[i]) {
                                   a.b.su[i] = base + slot;
                               } else {
                                   a.b.sv[i] = base + slot;
                               }
                               break;
                           }
                           h = (h + 1u) & mask;
                       }
                   });
               });
}

// V4: missing edges, smallest invalid index, emit valid item indices into
// the remaining list `cur`.
__device__ void val_final(const KArgs &a) {
    for (int32_t i = gtid(); i < a.s; i += gthreads()) {
        int32_t e = a.b.err[i];
        if (!a.inserting && e == 0 && (a.b.su[i] < 0 || a.b.sv[i] < 0)) {
            e = ST_MISSING;
            a.b.err[i] = e;
        }
        if (e != 0) atomicMin(&a.ctl->first_bad, i);
        push_agg<int32_t>(a.b.rem[a.cur], a.b.cap, &a.ctl->rem_count[a.cur], i, e == 0,
                          &a.ctl->overflow);
    }
}

// ===========================================================================
// Capacity reservation before an insertion batch mutates anything, and
// tombstone compaction after a deletion batch.
// ===========================================================================

__device__ __forceinline__ void mark_endpoint(const KArgs &a, int32_t x) {
    atomicAdd(&a.g.gain[x], 1);
    bool first = atomicExch(&a.g.bmark[x], a.bstamp + 1) != a.bstamp + 1;
    push_agg<int32_t>(a.b.vlist, a.g.n_cap, &a.ctl->vlist_count, x, first, &a.ctl->overflow);
}

// R1: per-vertex count of batch edges (gain) and the distinct endpoints.
__device__ void res_gain(const KArgs &a) {
    const int32_t n = qlen(&a.ctl->rem_count[a.cur], a.b.cap);
    const int32_t *R = a.b.rem[a.cur];
    for (int32_t idx = gtid(); idx < n; idx += gthreads()) {
        int32_t i = R[idx];
        mark_endpoint(a, a.b.eu[i]);
        mark_endpoint(a, a.b.ev[i]);
    }
}

// R2: a list that cannot take its gain moves to a spill block at the pool tail.
__device__ void res_alloc(const KArgs &a) {
    const int32_t n = qlen(&a.ctl->vlist_count, a.g.n_cap);
    for (int32_t j = gtid(); j < n; j += gthreads()) {
        int32_t x = a.b.vlist[j];
        int32_t need = a.g.len[x] + a.g.gain[x];
        a.g.gain[x] = 0;
        if (need > a.g.cap[x]) {
            int32_t nc = need + (need >> 3 > 4 ? need >> 3 : 4);
            nc = (nc + 3) & ~3;
            unsigned long long pos = atomicAdd(&a.ctl->pool_tail, (unsigned long long)nc);
            if (pos + (unsigned long long)nc > (unsigned long long)a.g.pool_size) {
                atomicOr(&a.ctl->pool_fail, 1);
            } else {
                int32_t r = atomicAdd(&a.ctl->reloc_count, 1);
                a.b.reloc[r] = x;
                a.b.reloc_off[r] = (int64_t)pos;
                a.b.reloc_cap[r] = nc;
            }
        }
    }
}

// R3: copy relocated lists (one wave per list).
__device__ void res_copy(const KArgs &a) {
    const int32_t n = qlen(&a.ctl->reloc_count, a.g.n_cap);
    for (int32_t j = gwave(); j < n; j += nwaves()) {
        int32_t x = a.b.reloc[j];
        int32_t L = a.g.len[x];
        const int32_t *src = a.g.nbr + a.g.off[x];
        int32_t *dst = a.g.nbr + a.b.reloc_off[j];
        for (int32_t s = lane(); s < L; s += WAVE) dst[s] = src[s];
        if (lane() == 0) {
            atomicAdd(&a.ctl->garbage, (unsigned long long)a.g.cap[x]);
            a.g.off[x] = a.b.reloc_off[j];
            a.g.cap[x] = a.b.reloc_cap[j];
        }
    }
}

// After a deletion batch: squeeze tombstones out of the touched lists whose
// tombstone share is large (one wave per list, in place, order kept).
__device__ void del_compact(const KArgs &a) {
    const int32_t n = qlen(&a.ctl->vlist_count, a.g.n_cap);
    for (int32_t j = gwave(); j < n; j += nwaves()) {
        int32_t x = a.b.vlist[j];
        int32_t L = a.g.len[x];
        int32_t T = a.g.gain[x];
        if (lane() == 0) a.g.gain[x] = 0;
        if (!(T * 8 >= L || L <= 1024)) continue;
        int32_t *p = a.g.nbr + a.g.off[x];
        int32_t wpos = 0;
        for (int32_t s = 0; s < L; s += WAVE) {
            int32_t i = s + lane();
            int32_t w = i < L ? p[i] : -1;
            unsigned long long m = __ballot(w >= 0);
            int rank = __popcll(m & ((1ull << lane()) - 1ull));
            if (w >= 0) p[wpos + rank] = w;
            wpos += __popcll(m);
        }
        if (lane() == 0) a.g.len[x] = wpos;
    }
}

// ===========================================================================
// One iteration = one superior edge set (Algorithm 1 / Algorithm 5 loop body)
// ===========================================================================

struct Iter {
    int32_t ep;    // iteration stamp
    int32_t cur;   // remaining list read by this iteration
    int32_t n_r;   // its length
};

__device__ __forceinline__ bool matched_before(uint32_t m, int32_t ep, int rounds, int r) {
    uint32_t lo = (uint32_t)ep * (uint32_t)rounds + 1u;
    uint32_t hi = (uint32_t)ep * (uint32_t)rounds + (uint32_t)r;
    return m >= lo && m <= hi;
}

// Selection of a superior edge set from the remaining edges (Algorithms 1-2
// and 5, lines selecting E_k for every level; Definition of the k-superior
// edge set).  An edge <u,v> has core number k = min(core u, core v); the
// endpoints with core k are its constrained endpoints.  Every constrained
// endpoint keeps at most one selected edge: each edge claims its constrained
// endpoints with a pseudo-random priority and is selected when it wins all
// of them (several claim rounds fill in more edges).  Levels are not
// separated: a vertex is constrained only at its own level, so one pass
// builds the union of all k-superior edge sets.
__device__ void part_claim(const KArgs &a, const Iter &it, int r) {
    Ctl *c = a.ctl;
    if (r == 0 && gtid() == 0) {
        c->sel_count = 0;
        c->rem_count[it.cur ^ 1] = 0;
        for (int j = 0; j < 3; ++j) {
            c->fq_tail[j] = 0; c->fh_tail[j] = 0; c->fx_tail[j] = 0;
            c->eq_tail[j] = 0; c->eh_tail[j] = 0;
        }
        c->cand_count = 0; c->chg_count = 0; c->chh_count = 0;
        c->touched_count = 0; c->changed_count = 0;
    }
    const int32_t *R = a.b.rem[it.cur];
    const uint32_t sr = (uint32_t)it.ep * (uint32_t)a.t.rounds + (uint32_t)r;
    const unsigned long long hi = (unsigned long long)(0xFFFFFFFFu - sr) << 32;
    for (int32_t idx = gtid(); idx < it.n_r; idx += gthreads()) {
        int32_t i = R[idx];
        if (r > 0 && a.b.esel[i] == it.ep) continue;
        int32_t u = a.b.eu[i], v = a.b.ev[i];
        int32_t cu = a.g.core[u], cv = a.g.core[v];
        int32_t k = cu < cv ? cu : cv;
        bool fu = cu == k, fv = cv == k;
        if (r > 0 && ((fu && matched_before(a.g.matched[u], it.ep, a.t.rounds, r)) ||
                      (fv && matched_before(a.g.matched[v], it.ep, a.t.rounds, r))))
            continue;
        unsigned long long key = hi | mix32((uint32_t)i);
        if (fu) atomicMin(&a.g.claim[u], key);
        if (fv) atomicMin(&a.g.claim[v], key);
    }
}

__device__ void part_select(const KArgs &a, const Iter &it, int r, bool last) {
    Ctl *c = a.ctl;
    const int32_t *R = a.b.rem[it.cur];
    const uint32_t sr = (uint32_t)it.ep * (uint32_t)a.t.rounds + (uint32_t)r;
    const unsigned long long hi = (unsigned long long)(0xFFFFFFFFu - sr) << 32;
    const uint32_t mstamp = sr + 1u;
    for (int32_t idx = gtid(); idx < it.n_r; idx += gthreads()) {
        int32_t i = R[idx];
        if (r > 0 && a.b.esel[i] == it.ep) continue;  // taken in an earlier round
        int32_t u = a.b.eu[i], v = a.b.ev[i];
        int32_t cu = a.g.core[u], cv = a.g.core[v];
        int32_t k = cu < cv ? cu : cv;
        bool fu = cu == k, fv = cv == k;
        bool part = !(r > 0 && ((fu && matched_before(a.g.matched[u], it.ep, a.t.rounds, r)) ||
                                (fv && matched_before(a.g.matched[v], it.ep, a.t.rounds, r))));
        unsigned long long key = hi | mix32((uint32_t)i);
        bool win = part && (!fu || a.g.claim[u] == key) && (!fv || a.g.claim[v] == key);
        if (win) {
            a.b.esel[i] = it.ep;
            if (fu) a.g.matched[u] = mstamp;
            if (fv) a.g.matched[v] = mstamp;
        }
        push_agg<int32_t>(a.b.sel, a.b.cap, &c->sel_count, i, win, &c->overflow);
        push_agg<int32_t>(a.b.rem[it.cur ^ 1], a.b.cap, &c->rem_count[it.cur ^ 1], i, last && !win,
                          &c->overflow);
    }
}

// Insert the selected set into G (Algorithm 1, insertion of the union of
// E_k) and update SD of the constrained endpoints; roots of the traversal
// are constrained endpoints whose new SD exceeds their core (a vertex with
// SD <= k cannot rise, Section IV-B).
__device__ void apply_insert(const KArgs &a, const Iter &it) {
    Ctl *c = a.ctl;
    const int32_t n = qlen(&c->sel_count, a.b.cap);
    for (int32_t idx = gtid(); idx < n; idx += gthreads()) {
        int32_t i = a.b.sel[idx];
        int32_t u = a.b.eu[i], v = a.b.ev[i];
        int32_t cu = a.g.core[u], cv = a.g.core[v];
        int32_t k = cu < cv ? cu : cv;
        int32_t pu = atomicAdd(&a.g.len[u], 1);
        if (pu < a.g.cap[u]) a.g.nbr[a.g.off[u] + pu] = v;
        else atomicOr(&c->overflow, 2);
        int32_t pv = atomicAdd(&a.g.len[v], 1);
        if (pv < a.g.cap[v]) a.g.nbr[a.g.off[v] + pv] = u;
        else atomicOr(&c->overflow, 2);
        bool ru = false, rv = false;
        if (cu == k) {
            int32_t m = atomicAdd(&a.g.mcd[u], 1) + 1;
            if (m > k) { a.g.stamp[u] = it.ep; a.g.cd[u] = 0; ru = true; }
        }
        if (cv == k) {
            int32_t m = atomicAdd(&a.g.mcd[v], 1) + 1;
            if (m > k) { a.g.stamp[v] = it.ep; a.g.cd[v] = 0; rv = true; }
        }
        // Roots enter the vertex queue whatever their length: other threads
        // may still be appending to the same list in this phase, so a chunk
        // count taken now could be stale.  The first expansion round splits
        // long root lists into chunks once lengths are final.
        push_agg<int32_t>(a.q.fq[0], a.q.vcap, &c->fq_tail[0], u, ru, &c->overflow);
        push_agg<int32_t>(a.q.fq[0], a.q.vcap, &c->fq_tail[0], v, rv, &c->overflow);
    }
}

// Delete the selected set from G (Algorithm 5) and update SD of the
// constrained endpoints; a root whose SD on G minus the set falls below its
// core is peeled at once (Algorithm 6, test cd < k).
__device__ void apply_delete(const KArgs &a, const Iter &it) {
    Ctl *c = a.ctl;
    const int32_t n = qlen(&c->sel_count, a.b.cap);
    for (int32_t idx = gtid(); idx < n; idx += gthreads()) {
        int32_t i = a.b.sel[idx];
        int32_t u = a.b.eu[i], v = a.b.ev[i];
        int32_t cu = a.g.core[u], cv = a.g.core[v];
        int32_t k = cu < cv ? cu : cv;
        a.g.nbr[a.b.su[i]] = TOMB;
        a.g.nbr[a.b.sv[i]] = TOMB;
        bool pu = false, pv = false;
        if (cu == k) {
            int32_t m = atomicSub(&a.g.mcd[u], 1) - 1;
            if (m < k) { a.g.stamp[u] = it.ep; pu = true; }
        }
        if (cv == k) {
            int32_t m = atomicSub(&a.g.mcd[v], 1) - 1;
            if (m < k) { a.g.stamp[v] = it.ep; pv = true; }
        }
        push_vertex(a, a.q.eq[0], &c->eq_tail[0], a.q.eh[0], &c->eh_tail[0], u, pu);
        push_vertex(a, a.q.eq[0], &c->eq_tail[0], a.q.eh[0], &c->eh_tail[0], v, pv);
        push_vertex(a, a.q.chg, &c->chg_count, a.q.chh, &c->chh_count, u, pu);
        push_vertex(a, a.q.chg, &c->chg_count, a.q.chh, &c->chh_count, v, pv);
    }
}

// Positive traversal (Algorithm 3) as level-synchronous rounds over all
// levels at once.  A visited vertex v computes cd[v] = CSD(v); if CSD(v) > k
// it visits its core-k neighbours w with SD(w) > k, otherwise it is queued
// for eviction (Lemma on CSD: CSD <= k keeps v out of the (k+1)-core).
// Every candidate's counter counts exactly its candidate neighbours at level
// k plus its higher-core neighbours, so the later peel is exact whatever the
// visiting order.
__device__ __forceinline__ bool is_support(const DevGraph &g, int32_t w, int32_t k) {
    int32_t cw = g.core[w];
    return cw > k || (cw == k && g.mcd[w] > k);
}

__device__ void expand_round(const KArgs &a, const Iter &it, int r, long long &scanned) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    const int sc = r % 3, sn = (r + 1) % 3, sx = (r + 2) % 3;
    const int bc = r & 1, bn = bc ^ 1;
    const int32_t nq = qlen(&c->fq_tail[sc], a.q.vcap);
    const int32_t nh = qlen(&c->fh_tail[sc], a.q.hcap);
    const int32_t nx = qlen(&c->fx_tail[sc], a.q.hcap);
    if (gtid() == 0) { c->fq_tail[sx] = 0; c->fh_tail[sx] = 0; c->fx_tail[sx] = 0; }
    const int32_t ep = it.ep;

    auto claim = [&](int32_t w, int32_t k) -> bool {
        if (w < 0) return false;
        if (g.core[w] != k || g.mcd[w] <= k) return false;
        if (atomicExch(&g.stamp[w], ep) == ep) return false;
        g.cd[w] = 0;
        return true;
    };
    auto push_next = [&](int32_t w, bool p) {
        push_vertex(a, a.q.fq[bn], &c->fq_tail[sn], a.q.fh[bn], &c->fh_tail[sn], w, p);
    };
    auto push_evict = [&](int32_t v, bool p) {
        push_vertex(a, a.q.eq[0], &c->eq_tail[0], a.q.eh[0], &c->eh_tail[0], v, p);
    };

    for_vertices(
        a.q.fq[bc], nq, g, a.t.small_deg,
        [&](int32_t v, int32_t L) {
            int32_t k = g.core[v];
            const int32_t *p = g.nbr + g.off[v];
            int32_t pcd = 0;
            for (int32_t s = 0; s < L; ++s) {
                int32_t w = p[s];
                if (w >= 0 && is_support(g, w, k)) ++pcd;
            }
            g.cd[v] = pcd;
            scanned += L;
            push_agg<int32_t>(a.q.cand, a.q.vcap, &c->cand_count, v, true, &c->overflow);
            if (pcd > k) {
                scanned += L;
                for (int32_t s = 0; s < L; ++s) push_next(p[s], claim(p[s], k));
            } else {
                push_evict(v, true);
            }
        },
        [&](int32_t v, int32_t L) {
            if (L > a.t.large_deg) {
                // a long root list: count its CSD chunk by chunk next round
                if (lane() == 0) {
                    int nch = nchunks(L, a.t.chunk);
                    int base = atomicAdd(&c->fh_tail[sn], nch);
                    for (int q = 0; q < nch; ++q) {
                        if (base + q < a.q.hcap) a.q.fh[bn][base + q] = chunk_item(v, q);
                        else atomicOr(&c->overflow, 1);
                    }
                }
                return;
            }
            int32_t k = g.core[v];
            int32_t pcd = 0;
            wave_walk(g, v, 0, L, [&](int32_t w, int32_t) {
                if (w >= 0 && is_support(g, w, k)) ++pcd;
            });
            pcd = wave_sum(pcd);
            if (lane() == 0) { g.cd[v] = pcd; scanned += L; }
            push_agg<int32_t>(a.q.cand, a.q.vcap, &c->cand_count, v, lane() == 0, &c->overflow);
            if (pcd > k) {
                if (lane() == 0) scanned += L;
                wave_walk(g, v, 0, L, [&](int32_t w, int32_t) { push_next(w, claim(w, k)); });
            } else {
                push_evict(v, lane() == 0);
            }
        });

    // CSD of long lists, chunk by chunk; the last chunk to finish decides.
    for_chunks(a.q.fh[bc], nh, g, a.t.chunk, [&](int32_t v, int32_t lo, int32_t hi, int32_t nch) {
        int32_t k = g.core[v];
        int32_t part = 0;
        wave_walk(g, v, lo, hi, [&](int32_t w, int32_t) {
            if (w >= 0 && is_support(g, w, k)) ++part;
        });
        part = wave_sum(part);
        int last = 0;
        if (lane() == 0) {
            scanned += hi - lo;
            atomicAdd(&g.cd[v], part);
            __threadfence();
            last = atomicAdd(&g.done[v], 1) == nch - 1;
        }
        last = __shfl(last, 0);
        if (last) {
            int32_t tot = 0;
            if (lane() == 0) {
                __threadfence();
                g.done[v] = 0;
                tot = __hip_atomic_load(&g.cd[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            tot = __shfl(tot, 0);
            push_agg<int32_t>(a.q.cand, a.q.vcap, &c->cand_count, v, lane() == 0, &c->overflow);
            if (tot > k) {
                if (lane() == 0) {
                    int base = atomicAdd(&c->fx_tail[sn], nch);
                    for (int q = 0; q < nch; ++q) {
                        if (base + q < a.q.hcap) a.q.fx[bn][base + q] = chunk_item(v, q);
                        else atomicOr(&c->overflow, 1);
                    }
                }
            } else {
                push_evict(v, lane() == 0);
            }
        }
    });

    // Expansion of long lists whose CSD exceeded k (decided last round).
    for_chunks(a.q.fx[bc], nx, g, a.t.chunk, [&](int32_t v, int32_t lo, int32_t hi, int32_t) {
        int32_t k = g.core[v];
        if (lane() == 0) scanned += hi - lo;
        wave_walk(g, v, lo, hi, [&](int32_t w, int32_t) { push_next(w, claim(w, k)); });
    });
}

// Negative traversal (Algorithm 4) as rounds: an evicted candidate lowers the
// counter of each candidate neighbour at its level; a neighbour is evicted
// exactly once, when its counter crosses from k+1 to k.
__device__ void evict_round(const KArgs &a, const Iter &it, int r, long long &scanned) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    const int sc = r % 3, sn = (r + 1) % 3, sx = (r + 2) % 3;
    const int bc = r & 1, bn = bc ^ 1;
    const int32_t nq = qlen(&c->eq_tail[sc], a.q.vcap);
    const int32_t nh = qlen(&c->eh_tail[sc], a.q.hcap);
    if (gtid() == 0) { c->eq_tail[sx] = 0; c->eh_tail[sx] = 0; }
    const int32_t ep = it.ep;
    auto hit = [&](int32_t w, int32_t k) -> bool {
        if (w < 0 || g.core[w] != k || g.stamp[w] != ep) return false;
        return atomicSub(&g.cd[w], 1) == k + 1;
    };
    auto push_next = [&](int32_t w, bool p) {
        push_vertex(a, a.q.eq[bn], &c->eq_tail[sn], a.q.eh[bn], &c->eh_tail[sn], w, p);
    };
    for_vertices(
        a.q.eq[bc], nq, g, a.t.small_deg,
        [&](int32_t x, int32_t L) {
            int32_t k = g.core[x];
            const int32_t *p = g.nbr + g.off[x];
            scanned += L;
            for (int32_t s = 0; s < L; ++s) {
                int32_t w = p[s];
                push_next(w, hit(w, k));
            }
        },
        [&](int32_t x, int32_t L) {
            int32_t k = g.core[x];
            if (lane() == 0) scanned += L;
            wave_walk(g, x, 0, L, [&](int32_t w, int32_t) { push_next(w, hit(w, k)); });
        });
    for_chunks(a.q.eh[bc], nh, g, a.t.chunk, [&](int32_t x, int32_t lo, int32_t hi, int32_t) {
        int32_t k = g.core[x];
        if (lane() == 0) scanned += hi - lo;
        wave_walk(g, x, lo, hi, [&](int32_t w, int32_t) { push_next(w, hit(w, k)); });
    });
}

// Peel cascade of the deletion (Algorithms 6-7) as rounds.  A peeled vertex
// adds one to dec[w] of each core-k neighbour w not yet peeled; w's counter
// is cd = SD(w) - dec[w] (SD on G minus the set) and w is peeled exactly
// once, when cd crosses from k to k-1.  dec is cleared after the iteration
// through the `touched` list.
__device__ void peel_round(const KArgs &a, const Iter &it, int r, long long &scanned) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    const int sc = r % 3, sn = (r + 1) % 3, sx = (r + 2) % 3;
    const int bc = r & 1, bn = bc ^ 1;
    const int32_t nq = qlen(&c->eq_tail[sc], a.q.vcap);
    const int32_t nh = qlen(&c->eh_tail[sc], a.q.hcap);
    if (gtid() == 0) { c->eq_tail[sx] = 0; c->eh_tail[sx] = 0; }
    const int32_t ep = it.ep;
    auto body = [&](int32_t w, int32_t k) {
        bool first = false, fire = false;
        if (w >= 0 && g.core[w] == k && g.stamp[w] != ep) {
            int32_t old = atomicAdd(&g.dec[w], 1);
            first = old == 0;
            fire = g.mcd[w] - old - 1 == k - 1;
            if (fire) g.stamp[w] = ep;
        }
        push_agg<int32_t>(a.q.touched, a.q.vcap, &c->touched_count, w, first, &c->overflow);
        push_vertex(a, a.q.eq[bn], &c->eq_tail[sn], a.q.eh[bn], &c->eh_tail[sn], w, fire);
        push_vertex(a, a.q.chg, &c->chg_count, a.q.chh, &c->chh_count, w, fire);
    };
    for_vertices(
        a.q.eq[bc], nq, g, a.t.small_deg,
        [&](int32_t x, int32_t L) {
            int32_t k = g.core[x];
            const int32_t *p = g.nbr + g.off[x];
            scanned += L;
            for (int32_t s = 0; s < L; ++s) body(p[s], k);
        },
        [&](int32_t x, int32_t L) {
            int32_t k = g.core[x];
            if (lane() == 0) scanned += L;
            wave_walk(g, x, 0, L, [&](int32_t w, int32_t) { body(w, k); });
        });
    for_chunks(a.q.eh[bc], nh, g, a.t.chunk, [&](int32_t x, int32_t lo, int32_t hi, int32_t) {
        int32_t k = g.core[x];
        if (lane() == 0) scanned += hi - lo;
        wave_walk(g, x, lo, hi, [&](int32_t w, int32_t) { body(w, k); });
    });
}

// Core update (Algorithm 1: +1 for every surviving candidate; Algorithm 5:
// -1 for every peeled vertex).  SD of a moved vertex is rebuilt next phase.
__device__ void apply_core(const KArgs &a, const Iter &it) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    if (a.inserting) {
        const int32_t n = qlen(&c->cand_count, a.q.vcap);
        for (int32_t idx = gtid(); idx < n; idx += gthreads()) {
            int32_t v = a.q.cand[idx];
            int32_t k = g.core[v];
            bool up = g.cd[v] > k;
            if (up) {
                g.core[v] = k + 1;
                g.chg[v] = it.ep;
                g.mcd[v] = 0;
            }
            count_agg(&c->changed_count, up);
            push_vertex(a, a.q.chg, &c->chg_count, a.q.chh, &c->chh_count, v, up);
        }
    } else {
        const int32_t n = qlen(&c->chg_count, a.q.vcap);
        for (int32_t idx = gtid(); idx < n; idx += gthreads()) {
            int32_t v = a.q.chg[idx];
            g.core[v] -= 1;
            g.chg[v] = it.ep;
            g.mcd[v] = 0;
        }
        if (gtid() == 0) atomicAdd(&c->changed_count, n);
        const int32_t nh = qlen(&c->chh_count, a.q.hcap);
        for (int32_t idx = gtid(); idx < nh; idx += gthreads()) {
            int64_t item = a.q.chh[idx];
            bool first = item_c(item) == 0;
            if (first) {
                int32_t v = item_v(item);
                g.core[v] -= 1;
                g.chg[v] = it.ep;
                g.mcd[v] = 0;
            }
            count_agg(&c->changed_count, first);
        }
        const int32_t nt = qlen(&c->touched_count, a.q.vcap);
        for (int32_t idx = gtid(); idx < nt; idx += gthreads()) g.dec[a.q.touched[idx]] = 0;
    }
}

// SD maintenance after the core update: a moved vertex recounts SD from its
// list; an unmoved neighbour w gains (insert) or loses (delete) one when the
// moved vertex crossed w's core.
__device__ void mcd_phase(const KArgs &a, const Iter &it, long long &scanned) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    const int32_t ep = it.ep;
    const bool ins = a.inserting != 0;
    auto nb = [&](int32_t w, int32_t cv) -> int32_t {
        if (w < 0) return 0;
        int32_t cw = g.core[w];
        if (g.chg[w] != ep) {
            if (ins && cw == cv) atomicAdd(&g.mcd[w], 1);
            if (!ins && cw == cv + 1) atomicSub(&g.mcd[w], 1);
        }
        return cw >= cv ? 1 : 0;
    };
    const int32_t n = qlen(&c->chg_count, a.q.vcap);
    for_vertices(
        a.q.chg, n, g, a.t.small_deg,
        [&](int32_t v, int32_t L) {
            int32_t cv = g.core[v];
            const int32_t *p = g.nbr + g.off[v];
            int32_t cnt = 0;
            for (int32_t s = 0; s < L; ++s) cnt += nb(p[s], cv);
            g.mcd[v] = cnt;
            scanned += L;
        },
        [&](int32_t v, int32_t L) {
            int32_t cv = g.core[v];
            int32_t cnt = 0;
            wave_walk(g, v, 0, L, [&](int32_t w, int32_t) { cnt += nb(w, cv); });
            cnt = wave_sum(cnt);
            if (lane() == 0) { g.mcd[v] = cnt; scanned += L; }
        });
    const int32_t nh = qlen(&c->chh_count, a.q.hcap);
    for_chunks(a.q.chh, nh, g, a.t.chunk, [&](int32_t v, int32_t lo, int32_t hi, int32_t) {
        int32_t cv = g.core[v];
        int32_t cnt = 0;
        wave_walk(g, v, lo, hi, [&](int32_t w, int32_t) { cnt += nb(w, cv); });
        cnt = wave_sum(cnt);
        if (lane() == 0) { atomicAdd(&g.mcd[v], cnt); scanned += hi - lo; }
    });
}

// Runs up to a.max_iters iterations (one superior edge set each) of the
// current batch.  Returns the iterations run.  Grid-uniform control flow:
// every decision reads counters published before a grid barrier.
__device__ int run_iterations(const KArgs &a) {
    Ctl *c = a.ctl;
    const int32_t ep0 = ld_acq(&c->epoch);
    int it_n = 0;
    long long scanned = 0;
    for (; it_n < a.max_iters; ++it_n) {
        Iter it;
        it.ep = ep0 + it_n + 1;
        it.cur = it.ep & 1;
        it.n_r = qlen(&c->rem_count[it.cur], a.b.cap);
        if (it.n_r == 0 || ld_acq(&c->overflow) != 0) break;
        for (int r = 0; r < a.t.rounds; ++r) {
            part_claim(a, it, r);
            gsync();
            part_select(a, it, r, r == a.t.rounds - 1);
            gsync();
        }
        if (a.inserting) {
            apply_insert(a, it);
            gsync();
            for (int r = 0;; ++r) {
                int s = r % 3;
                if (ld_acq(&c->fq_tail[s]) + ld_acq(&c->fh_tail[s]) + ld_acq(&c->fx_tail[s]) == 0) break;
                expand_round(a, it, r, scanned);
                gsync();
            }
            for (int r = 0;; ++r) {
                int s = r % 3;
                if (ld_acq(&c->eq_tail[s]) + ld_acq(&c->eh_tail[s]) == 0) break;
                evict_round(a, it, r, scanned);
                gsync();
            }
        } else {
            apply_delete(a, it);
            gsync();
            for (int r = 0;; ++r) {
                int s = r % 3;
                if (ld_acq(&c->eq_tail[s]) + ld_acq(&c->eh_tail[s]) == 0) break;
                peel_round(a, it, r, scanned);
                gsync();
            }
        }
        apply_core(a, it);
        gsync();
        mcd_phase(a, it, scanned);
        if (gtid() == 0) {
            int32_t ns = ld_acq(&c->sel_count);
            int32_t nch = ld_acq(&c->changed_count);
            int32_t ncand = ld_acq(&c->cand_count);
            c->st_iters += 1;
            c->st_remaining += (unsigned long long)it.n_r;
            c->st_selected += (unsigned long long)ns;
            if (a.inserting) {
                c->st_candidates += (unsigned long long)ncand;
                c->st_changed += (unsigned long long)nch;
                c->st_evicted += (unsigned long long)(ncand - nch);
            } else {
                c->st_candidates += (unsigned long long)ld_acq(&c->touched_count);
                c->st_changed += (unsigned long long)nch;
                c->st_evicted += (unsigned long long)nch;
            }
        }
        gsync();
    }
    flush_stat(&c->st_scanned, scanned);
    if (gtid() == 0) {
        c->epoch = ep0 + it_n;
        c->iters_done = it_n;
    }
    return it_n;
}

// ===========================================================================
// Static core decomposition (initial state): level-synchronous peeling.
// Level k: every remaining vertex whose current degree is <= k gets core k
// and is removed; removing a vertex lowers its remaining neighbours'
// degrees, and a neighbour joins the level when its degree crosses from k+1
// to k (exactly once).  Empty levels are skipped by jumping k to the
// smallest remaining degree.  cd[] holds the current degree; core = -2 marks
// "not yet peeled".  Vertex lists: q.fq[0..1] (remaining, ping-pong);
// frontier: q.eq / q.eh.
// ===========================================================================
__device__ int decompose(const KArgs &a) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    int32_t k = 0;
    int j = 0;       // sweep index (rotating rm_count / min_deg slots)
    int rr = 0;      // frontier round index (rotating eq/eh slots)
    long long scanned = 0;
    int32_t kmax = 0;
    for (;;) {
        // Sweep: split the remaining vertices into this level's frontier
        // (degree <= k) and the rest; track the smallest remaining degree.
        {
            const int s0 = j % 3, s1 = (j + 1) % 3, s2 = (j + 2) % 3;
            const int fs = rr % 3, fb = rr & 1;
            const int32_t n = qlen(&c->rm_count[s0], a.q.vcap);
            if (gtid() == 0) {
                c->rm_count[s2] = 0;
                c->min_deg[s2] = 0x7fffffff;
                c->eq_tail[(rr + 1) % 3] = 0; c->eh_tail[(rr + 1) % 3] = 0;
                c->eq_tail[(rr + 2) % 3] = 0; c->eh_tail[(rr + 2) % 3] = 0;
            }
            const int32_t *src = a.q.fq[j & 1];
            int32_t *dst = a.q.fq[(j + 1) & 1];
            int32_t mymin = 0x7fffffff;
            for (int32_t idx = gtid(); idx < n; idx += gthreads()) {
                int32_t v = src[idx];
                bool keep = false, take = false;
                if (g.core[v] == -2) {
                    int32_t d = g.cd[v];
                    if (d <= k) { g.core[v] = k; take = true; }
                    else { keep = true; mymin = d < mymin ? d : mymin; }
                }
                push_vertex(a, a.q.eq[fb], &c->eq_tail[fs], a.q.eh[fb], &c->eh_tail[fs], v, take);
                push_agg<int32_t>(dst, a.q.vcap, &c->rm_count[s1], v, keep, &c->overflow);
            }
            for (int o = 32; o > 0; o >>= 1) {
                int32_t t = __shfl_xor(mymin, o);
                mymin = t < mymin ? t : mymin;
            }
            if (lane() == 0 && mymin != 0x7fffffff) atomicMin(&c->min_deg[s1], mymin);
        }
        gsync();
        const int s1 = (j + 1) % 3;
        ++j;
        if (ld_acq(&c->eq_tail[rr % 3]) + ld_acq(&c->eh_tail[rr % 3]) == 0) {
            if (ld_acq(&c->rm_count[s1]) == 0) break;
            int32_t md = ld_acq(&c->min_deg[s1]);
            k = md > k + 1 ? md : k + 1;
            continue;
        }
        kmax = k;
        // Frontier rounds of level k.
        for (;;) {
            const int sc = rr % 3, sn = (rr + 1) % 3, sx = (rr + 2) % 3;
            const int bc = rr & 1, bn = bc ^ 1;
            const int32_t nq = qlen(&c->eq_tail[sc], a.q.vcap);
            const int32_t nh = qlen(&c->eh_tail[sc], a.q.hcap);
            if (gtid() == 0) { c->eq_tail[sx] = 0; c->eh_tail[sx] = 0; }
            auto body = [&](int32_t w) -> bool {
                if (w < 0 || g.core[w] != -2) return false;
                if (atomicSub(&g.cd[w], 1) != k + 1) return false;
                g.core[w] = k;
                return true;
            };
            auto push_next = [&](int32_t w, bool p) {
                push_vertex(a, a.q.eq[bn], &c->eq_tail[sn], a.q.eh[bn], &c->eh_tail[sn], w, p);
            };
            for_vertices(
                a.q.eq[bc], nq, g, a.t.small_deg,
                [&](int32_t x, int32_t L) {
                    const int32_t *p = g.nbr + g.off[x];
                    scanned += L;
                    for (int32_t s = 0; s < L; ++s) push_next(p[s], body(p[s]));
                },
                [&](int32_t x, int32_t L) {
                    if (lane() == 0) scanned += L;
                    wave_walk(g, x, 0, L, [&](int32_t w, int32_t) { push_next(w, body(w)); });
                });
            for_chunks(a.q.eh[bc], nh, g, a.t.chunk, [&](int32_t x, int32_t lo, int32_t hi, int32_t) {
                if (lane() == 0) scanned += hi - lo;
                wave_walk(g, x, lo, hi, [&](int32_t w, int32_t) { push_next(w, body(w)); });
            });
            gsync();
            ++rr;
            if (ld_acq(&c->eq_tail[rr % 3]) + ld_acq(&c->eh_tail[rr % 3]) == 0) break;
        }
        k += 1;
    }
    flush_stat(&c->st_scanned, scanned);
    if (gtid() == 0) { c->kmax = kmax; c->dec_rounds = rr; }
    return rr;
}

}  // namespace cm
