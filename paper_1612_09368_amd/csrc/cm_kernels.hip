// Kernels of libcoremaint and their host launch helpers.
#include "cm_launch.h"
#include "cm_phases.h"

namespace cm {

// ---------------------------------------------------------------------------
// Small utilities
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_i64(int64_t *p, int64_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Reset the per-batch control fields (the persistent ones -- epoch, pool
// tail, garbage -- are kept).
__global__ void k_ctl_batch_reset(Ctl *c, int cur) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->rem_count[0] = 0;
        c->rem_count[1] = 0;
        c->sel_count = 0;
        for (int j = 0; j < 3; ++j) {
            c->fq_tail[j] = 0; c->fh_tail[j] = 0;
            c->eq_tail[j] = 0; c->eh_tail[j] = 0;
            c->rm_count[j] = 0; c->min_deg[j] = 0x7fffffff;
        }
        c->cand_count = 0; c->chg_count = 0; c->chh_count = 0;
        c->touched_count = 0; c->changed_count = 0;
        c->overflow = 0;
        c->iters_done = 0;
        c->pool_fail = 0;
        c->first_bad = 0x7fffffff;
        c->valid_count = 0;
        c->scan_tail = 0;
        c->vlist_count = 0;
        c->reloc_count = 0;
        c->kmax = 0;
        c->dec_rounds = 0;
        c->st_iters = 0; c->st_remaining = 0; c->st_selected = 0;
        c->st_candidates = 0; c->st_evicted = 0; c->st_changed = 0; c->st_scanned = 0;
        c->st_rounds = 0; c->st_grid_steps = 0; c->st_local_steps = 0;
        c->st_icand = 0; c->st_cdeg = 0; c->st_edeg = 0; c->st_hdeg = 0;
        (void)cur;
    }
}

// Reservation counters (validation results are kept).
__global__ void k_ctl_reserve_reset(Ctl *c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->vlist_count = 0;
        c->reloc_count = 0;
        c->pool_fail = 0;
    }
}
__global__ void k_ctl_set_pool(Ctl *c, unsigned long long tail) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->pool_tail = tail;
        c->garbage = 0;
    }
}

// Exclusive scan of int64 values (three passes; SCAN_TILE items per block).
constexpr int SCAN_TILE = 1024;

__device__ __forceinline__ long long block_incl_scan(long long v, long long *sh) {
    // 256 threads: wave scan, then scan of the 4 wave totals
    int ln = lane();
    for (int o = 1; o < WAVE; o <<= 1) {
        long long t = __shfl_up(v, o);
        if (ln >= o) v += t;
    }
    int w = threadIdx.x / WAVE;
    if (ln == WAVE - 1) sh[w] = v;
    __syncthreads();
    long long add = 0;
    for (int i = 0; i < w; ++i) add += sh[i];
    __syncthreads();
    return v + add;
}

__global__ void k_scan_reduce(const int64_t *in, int64_t n, int64_t *bsum) {
    __shared__ long long sh[8];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    long long s = 0;
    for (int i = threadIdx.x; i < SCAN_TILE; i += blockDim.x) {
        int64_t j = base + i;
        if (j < n) s += in[j];
    }
    s = block_incl_scan(s, sh);
    if (threadIdx.x == blockDim.x - 1) bsum[blockIdx.x] = s;
}

__global__ void k_scan_blocks(int64_t *bsum, int64_t nb, int64_t *total) {
    // single block: exclusive scan of nb block sums in place
    __shared__ long long sh[8];
    __shared__ long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += blockDim.x) {
        int64_t j = base + threadIdx.x;
        long long v = j < nb ? bsum[j] : 0;
        long long incl = block_incl_scan(v, sh);
        long long c0 = carry;
        if (j < nb) bsum[j] = c0 + incl - v;
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) carry = c0 + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_apply(const int64_t *in, int64_t n, const int64_t *bsum, int64_t *out) {
    __shared__ long long sh[8];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    // each thread owns 4 consecutive items
    long long vals[4];
    long long s = 0;
    for (int q = 0; q < 4; ++q) {
        int64_t j = base + threadIdx.x * 4 + q;
        vals[q] = j < n ? in[j] : 0;
        s += vals[q];
    }
    long long incl = block_incl_scan(s, sh);
    long long run = bsum[blockIdx.x] + incl - s;
    for (int q = 0; q < 4; ++q) {
        int64_t j = base + threadIdx.x * 4 + q;
        if (j < n) out[j] = run;
        run += vals[q];
    }
}

// ---------------------------------------------------------------------------
// Graph store: load from an edge list
// ---------------------------------------------------------------------------
__device__ __forceinline__ void note_bad(unsigned long long *first_bad, int64_t i, int code) {
    atomicMin(first_bad, ((unsigned long long)i << 8) | (unsigned long long)(-code));
}

__global__ void k_load_hash(const int32_t *src, const int32_t *dst, int64_t m, int32_t n,
                            unsigned long long *hkey, int64_t *hval, uint32_t mask,
                            unsigned long long *first_bad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t u = src[i], v = dst[i];
        if (u < 0 || v < 0 || u >= n || v >= n) { note_bad(first_bad, i, ST_RANGE); continue; }
        if (u == v) { note_bad(first_bad, i, ST_SELF); continue; }
        unsigned long long key = edge_key(u, v);
        uint32_t h = hash_key(key) & mask;
        for (uint32_t probe = 0; probe <= mask; ++probe) {
            unsigned long long old = atomicCAS(&hkey[h], EMPTY_KEY, key);
            if (old == EMPTY_KEY || old == key) break;
            h = (h + 1u) & mask;
        }
        atomicMin((unsigned long long *)&hval[h], (unsigned long long)i);
    }
}

__global__ void k_load_dup(const int32_t *src, const int32_t *dst, int64_t m, int32_t n,
                           const unsigned long long *hkey, const int64_t *hval, uint32_t mask,
                           unsigned long long *first_bad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t u = src[i], v = dst[i];
        if (u < 0 || v < 0 || u >= n || v >= n || u == v) continue;
        unsigned long long key = edge_key(u, v);
        uint32_t h = hash_key(key) & mask;
        for (uint32_t probe = 0; probe <= mask; ++probe) {
            unsigned long long k2 = hkey[h];
            if (k2 == key) {
                if (hval[h] != i) note_bad(first_bad, i, ST_DUP);
                break;
            }
            if (k2 == EMPTY_KEY) break;
            h = (h + 1u) & mask;
        }
    }
}

__global__ void k_count_deg(const int32_t *src, const int32_t *dst, int64_t m, int32_t *len) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        atomicAdd(&len[src[i]], 1);
        atomicAdd(&len[dst[i]], 1);
    }
}

__device__ __forceinline__ int32_t slack_cap(int32_t live) {
    int32_t extra = live >> 3;
    if (extra < 4) extra = 4;
    return (live + extra + 3) & ~3;
}

// caps64[v] = capacity with slack for `cnt[v]` live entries (0 for unused ids).
__global__ void k_caps(const int32_t *cnt, int32_t n, int32_t n_cap, int64_t *caps64, int32_t *cap) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n_cap; v += gridDim.x * blockDim.x) {
        int32_t c = v < n ? slack_cap(cnt[v]) : 0;
        caps64[v] = c;
        cap[v] = c;
    }
}

__global__ void k_scatter(const int32_t *src, const int32_t *dst, int64_t m, const int64_t *off,
                          int32_t *len, int32_t *nbr) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t u = src[i], v = dst[i];
        int32_t pu = atomicAdd(&len[u], 1);
        nbr[off[u] + pu] = v;
        int32_t pv = atomicAdd(&len[v], 1);
        nbr[off[v] + pv] = u;
    }
}

// Live entries per list (tombstones excluded) into cnt.
__global__ void k_count_live(KArgs a, int32_t *cnt) {
    const DevGraph &g = a.g;
    for_all_vertices(
        grid_team(), g.n_ids, g, a.t.small_deg,
        [&](int32_t v, int32_t L) {
            const int32_t *p = g.nbr + g.off[v];
            int32_t c = 0;
            for (int32_t s = 0; s < L; ++s) c += p[s] >= 0;
            cnt[v] = c;
        },
        [&](int32_t v, int32_t L) {
            int32_t c = 0;
            wave_walk(g, v, 0, L, [&](int32_t w, int32_t) { c += w >= 0; });
            c = wave_sum(c);
            if (lane() == 0) cnt[v] = c;
        });
    // dead ids: zero
    for (int32_t v = gtid(); v < g.n_ids; v += gthreads())
        if (g.core[v] == -1) cnt[v] = 0;
}

// Copy live entries of every list to the new pool (order kept).
__global__ void k_repack_copy(KArgs a, const int64_t *newoff, int32_t *newnbr) {
    const DevGraph &g = a.g;
    for (int32_t v = gwave(); v < g.n_ids; v += nwaves()) {
        if (g.core[v] == -1) continue;
        int32_t L = g.len[v];
        const int32_t *p = g.nbr + g.off[v];
        int32_t *q = newnbr + newoff[v];
        int32_t wpos = 0;
        for (int32_t s = 0; s < L; s += WAVE) {
            int32_t i = s + lane();
            int32_t w = i < L ? p[i] : -1;
            unsigned long long m = __ballot(w >= 0);
            int rank = __popcll(m & ((1ull << lane()) - 1ull));
            if (w >= 0) q[wpos + rank] = w;
            wpos += __popcll(m);
        }
    }
}

__global__ void k_repack_finish(KArgs a, const int64_t *newoff, const int32_t *cnt) {
    const DevGraph &g = a.g;
    for (int32_t v = gtid(); v < g.n_cap; v += gthreads()) {
        bool live = v < g.n_ids && g.core[v] != -1;
        g.off[v] = newoff[v];
        g.len[v] = live ? cnt[v] : 0;
        if (g.ubl) g.ubl[v] = -1;  // lists moved
    }
}

// Every edge once as (min, max).
__global__ void k_export(KArgs a, int32_t *xs, int32_t *ys, int64_t cap, unsigned long long *tail) {
    const DevGraph &g = a.g;
    for (int32_t v = gwave(); v < g.n_ids; v += nwaves()) {
        if (g.core[v] == -1) continue;
        int32_t L = g.len[v];
        wave_walk(g, v, 0, L, [&](int32_t w, int32_t) {
            bool take = w > v;
            unsigned long long m = __ballot(take);
            int rank = __popcll(m & ((1ull << lane()) - 1ull));
            unsigned long long base = 0;
            if (lane() == 0 && m) base = atomicAdd(tail, (unsigned long long)__popcll(m));
            base = __shfl(base, 0);
            if (take && (int64_t)(base + rank) < cap) {
                xs[base + rank] = v;
                ys[base + rank] = w;
            }
        });
    }
}

// ---------------------------------------------------------------------------
// Decomposition
// ---------------------------------------------------------------------------
__global__ void k_dec_prep(KArgs a) {
    const DevGraph &g = a.g;
    Ctl *c = a.ctl;
    // cores are recomputed from scratch: no up-list survives
    if (g.ubl)
        for (int32_t v = gtid(); v < g.n_cap; v += gthreads()) g.ubl[v] = -1;
    for_all_vertices(
        grid_team(), g.n_ids, g, a.t.small_deg,
        [&](int32_t v, int32_t L) {
            const int32_t *p = g.nbr + g.off[v];
            int32_t d = 0;
            for (int32_t s = 0; s < L; ++s) d += p[s] >= 0;
            g.cd[v] = d;
        },
        [&](int32_t v, int32_t L) {
            int32_t d = 0;
            wave_walk(g, v, 0, L, [&](int32_t w, int32_t) { d += w >= 0; });
            d = wave_sum(d);
            if (lane() == 0) g.cd[v] = d;
        });
    for (int32_t base = gwave() * WAVE; base < g.n_ids; base += nwaves() * WAVE) {
        int32_t v = base + lane();
        bool alive = v < g.n_ids && g.core[v] != -1;
        if (alive) g.core[v] = -2;
        push_agg<int32_t>(a.q.fq[0], a.q.vcap, &c->rm_count[0], v, alive, &c->overflow);
    }
}

__global__ void __launch_bounds__(COOP_THREADS) k_decompose(KArgs a) {
    gbar_setup(a.bar);
    Acc acc{};
    decompose(a, acc);
    flush_acc(a.ctl, acc);
}

__global__ void k_mcd_init(KArgs a) {
    const DevGraph &g = a.g;
    for_all_vertices(
        grid_team(), g.n_ids, g, a.t.small_deg,
        [&](int32_t v, int32_t L) {
            int32_t cv = g.core[v];
            const int32_t *p = g.nbr + g.off[v];
            int32_t cnt = 0;
            for (int32_t s = 0; s < L; ++s) {
                int32_t w = p[s];
                if (w >= 0 && g.core[w] >= cv) ++cnt;
            }
            g.mcd[v] = cnt;
        },
        [&](int32_t v, int32_t L) {
            int32_t cv = g.core[v];
            int32_t cnt = 0;
            wave_walk(g, v, 0, L, [&](int32_t w, int32_t) {
                if (w >= 0 && g.core[w] >= cv) ++cnt;
            });
            cnt = wave_sum(cnt);
            if (lane() == 0) g.mcd[v] = cnt;
        });
}

// ---------------------------------------------------------------------------
// Batch validation, reservation, compaction, maintenance
// ---------------------------------------------------------------------------
__global__ void k_val_canon(KArgs a) { val_canon(a, batch_of(a), grid_team()); }
__global__ void k_val_dup_mark(KArgs a) { val_dup_mark(a, batch_of(a), grid_team()); }
__global__ void k_val_scan(KArgs a) { val_scan(a, batch_of(a), grid_team()); }
__global__ void k_val_final(KArgs a) { val_final(a, batch_of(a), grid_team()); }
__global__ void k_val_subfilter(KArgs a) { val_subfilter(a, batch_of(a), grid_team()); }
__global__ void k_res_gain(KArgs a) { res_gain(a, batch_of(a), grid_team()); }
__global__ void k_res_alloc(KArgs a) { res_alloc(a, grid_team()); }
__global__ void k_res_copy(KArgs a) { res_copy(a, grid_team()); }
__global__ void k_del_compact(KArgs a) { del_compact(a, grid_team()); }
__global__ void __launch_bounds__(COOP_THREADS) k_maintain(KArgs a) {
    gbar_setup(a.bar);
    int32_t ep = ld_rlx(&a.ctl->epoch);
    Acc acc{};
    int pubs = 0;
    int n = run_iterations(a, a.inserting, a.max_iters, ep, acc, pubs);
    flush_acc(a.ctl, acc);
    if (gtid() == 0) {
        a.ctl->epoch = ep;
        a.ctl->iters_done = n;
        if (a.lout) {
            // every step ended at a grid barrier, so the counters are final
            a.lout->epoch = ep;
            a.lout->iters = n;
            a.lout->rem_next = ld_rlx(&a.ctl->rem_count[(ep + 1) & 1]);
            a.lout->overflow = ld_rlx(&a.ctl->overflow);
            a.lout->aborted = bar_aborted(a.bar) ? 1 : 0;
        }
    }
}

__global__ void __launch_bounds__(COOP_THREADS) k_program(KArgs a) {
    gbar_setup(a.bar);
    run_program(a);
}
__global__ void __launch_bounds__(COOP_THREADS) k_serve(KArgs a) {
    gbar_setup(a.bar);
    run_server(a);
}

// ---------------------------------------------------------------------------
// Vertex operations
// ---------------------------------------------------------------------------
// New ids [first, first + c): empty lists, core 0, SD 0.
__global__ void k_vins_init(KArgs a, int32_t first, int32_t c) {
    const DevGraph &g = a.g;
    for (int32_t i = gtid(); i < c; i += gthreads()) {
        int32_t v = first + i;
        g.core[v] = 0;
        g.mcd[v] = 0;
        g.len[v] = 0;
        g.cap[v] = 0;
        g.off[v] = 0;
    }
}
__global__ void k_vins_revert(KArgs a, int32_t first, int32_t c) {
    for (int32_t i = gtid(); i < c; i += gthreads()) a.g.core[first + i] = -1;
}
// src[j] = first + i for j in [off[i], off[i+1]).
__global__ void k_vins_expand(const int64_t *off, int32_t c, int32_t first, int32_t *src) {
    for (int32_t i = gwave(); i < c; i += nwaves()) {
        int64_t lo = off[i], hi = off[i + 1];
        for (int64_t j = lo + lane(); j < hi; j += WAVE) src[j] = first + i;
    }
}
__global__ void k_vins_check_off(const int64_t *off, int32_t c, unsigned long long *first_bad) {
    for (int32_t i = gtid(); i < c; i += gthreads())
        if (off[i + 1] < off[i]) atomicMin(first_bad, (unsigned long long)i);
}

// Deleted ids: range, dead, duplicates (smallest index wins).
__global__ void k_vdel_check(KArgs a, const int32_t *ids, int32_t c, int32_t *firstidx,
                             unsigned long long *first_bad) {
    const DevGraph &g = a.g;
    for (int32_t i = gtid(); i < c; i += gthreads()) {
        int32_t x = ids[i];
        if (x < 0 || x >= g.n_ids) { note_bad(first_bad, i, ST_RANGE); continue; }
        if (g.core[x] < 0) { note_bad(first_bad, i, ST_DEAD); continue; }
        atomicMin(&firstidx[x], i);
    }
}
__global__ void k_vdel_dup(KArgs a, const int32_t *ids, int32_t c, const int32_t *firstidx,
                           unsigned long long *first_bad, unsigned long long *total) {
    const DevGraph &g = a.g;
    for (int32_t i = gtid(); i < c; i += gthreads()) {
        int32_t x = ids[i];
        if (x < 0 || x >= g.n_ids || g.core[x] < 0) continue;
        if (firstidx[x] != i) { note_bad(first_bad, i, ST_DUP); continue; }
        atomicAdd(total, (unsigned long long)g.len[x]);
    }
}
__global__ void k_vdel_reset_first(KArgs a, const int32_t *ids, int32_t c, int32_t *firstidx) {
    for (int32_t i = gtid(); i < c; i += gthreads()) {
        int32_t x = ids[i];
        if (x >= 0 && x < a.g.n_ids) firstidx[x] = 0x7fffffff;
    }
}
// Every live edge of the deleted ids (an edge between two deleted ids appears
// twice; the second copy is dropped as a duplicate by validation).
__global__ void k_vdel_gather(KArgs a, const int32_t *ids, int32_t c, int32_t *xs, int32_t *ys,
                              int64_t cap, unsigned long long *tail) {
    const DevGraph &g = a.g;
    for (int32_t i = gwave(); i < c; i += nwaves()) {
        int32_t x = ids[i];
        int32_t L = g.len[x];
        wave_walk(g, x, 0, L, [&](int32_t w, int32_t) {
            bool take = w >= 0;
            unsigned long long m = __ballot(take);
            int rank = __popcll(m & ((1ull << lane()) - 1ull));
            unsigned long long base = 0;
            if (lane() == 0 && m) base = atomicAdd(tail, (unsigned long long)__popcll(m));
            base = __shfl(base, 0);
            if (take && (int64_t)(base + rank) < cap) {
                xs[base + rank] = x;
                ys[base + rank] = w;
            }
        });
    }
}
__global__ void k_vdel_finish(KArgs a, const int32_t *ids, int32_t c) {
    const DevGraph &g = a.g;
    for (int32_t i = gtid(); i < c; i += gthreads()) {
        int32_t x = ids[i];
        g.core[x] = -1;
        g.mcd[x] = 0;
        g.len[x] = 0;
    }
}

// ---------------------------------------------------------------------------
// Host launch helpers
// ---------------------------------------------------------------------------
static inline int grid_for(int64_t n, int maxb) {
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > maxb) b = maxb;
    return (int)b;
}

hipError_t fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (!p) return hipErrorInvalidValue;
    k_fill_i32<<<grid_for(n, 4096), 256, 0, st>>>(p, v, n);
    return hipGetLastError();
}
hipError_t fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (!p) return hipErrorInvalidValue;
    k_fill_u64<<<grid_for(n, 4096), 256, 0, st>>>(p, v, n);
    return hipGetLastError();
}
hipError_t fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (!p) return hipErrorInvalidValue;
    k_fill_i64<<<grid_for(n, 4096), 256, 0, st>>>(p, v, n);
    return hipGetLastError();
}
hipError_t ctl_batch_reset(Ctl *c, int cur, hipStream_t st) {
    if (!c) return hipErrorInvalidValue;
    k_ctl_batch_reset<<<1, 64, 0, st>>>(c, cur);
    return hipGetLastError();
}

hipError_t ctl_reserve_reset(Ctl *c, hipStream_t st) {
    if (!c) return hipErrorInvalidValue;
    k_ctl_reserve_reset<<<1, 64, 0, st>>>(c);
    return hipGetLastError();
}
hipError_t ctl_set_pool(Ctl *c, unsigned long long tail, hipStream_t st) {
    if (!c) return hipErrorInvalidValue;
    k_ctl_set_pool<<<1, 64, 0, st>>>(c, tail);
    return hipGetLastError();
}

// in-place exclusive scan of n int64 values; *total_dev receives the sum.
hipError_t exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp,
                              int64_t *total_dev, hipStream_t st) {
    if (!in || !out || !tmp || !total_dev) return hipErrorInvalidValue;
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb < 1) nb = 1;
    k_scan_reduce<<<(unsigned)nb, 256, 0, st>>>(in, n, tmp);
    k_scan_blocks<<<1, 256, 0, st>>>(tmp, nb, total_dev);
    k_scan_apply<<<(unsigned)nb, 256, 0, st>>>(in, n, tmp, out);
    return hipGetLastError();
}
int64_t scan_tmp_len(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

hipError_t load_check(const int32_t *src, const int32_t *dst, int64_t m, int32_t n,
                      unsigned long long *hkey, int64_t *hval, uint32_t mask,
                      unsigned long long *first_bad, hipStream_t st) {
    if (!src || !dst || !hkey || !hval || !first_bad) return hipErrorInvalidValue;
    k_load_hash<<<grid_for(m, 8192), 256, 0, st>>>(src, dst, m, n, hkey, hval, mask, first_bad);
    k_load_dup<<<grid_for(m, 8192), 256, 0, st>>>(src, dst, m, n, hkey, hval, mask, first_bad);
    return hipGetLastError();
}
hipError_t count_deg(const int32_t *src, const int32_t *dst, int64_t m, int32_t *len, hipStream_t st) {
    k_count_deg<<<grid_for(m, 8192), 256, 0, st>>>(src, dst, m, len);
    return hipGetLastError();
}
hipError_t caps_from_counts(const int32_t *cnt, int32_t n, int32_t n_cap, int64_t *caps64,
                            int32_t *cap, hipStream_t st) {
    k_caps<<<grid_for(n_cap, 8192), 256, 0, st>>>(cnt, n, n_cap, caps64, cap);
    return hipGetLastError();
}
hipError_t scatter_edges(const int32_t *src, const int32_t *dst, int64_t m, const int64_t *off,
                         int32_t *len, int32_t *nbr, hipStream_t st) {
    k_scatter<<<grid_for(m, 8192), 256, 0, st>>>(src, dst, m, off, len, nbr);
    return hipGetLastError();
}
hipError_t count_live(const KArgs &a, int32_t *cnt, int blocks, hipStream_t st) {
    k_count_live<<<blocks, 256, 0, st>>>(a, cnt);
    return hipGetLastError();
}
hipError_t repack_copy(const KArgs &a, const int64_t *newoff, int32_t *newnbr, int blocks, hipStream_t st) {
    k_repack_copy<<<blocks, 256, 0, st>>>(a, newoff, newnbr);
    return hipGetLastError();
}
hipError_t repack_finish(const KArgs &a, const int64_t *newoff, const int32_t *cnt, int blocks,
                         hipStream_t st) {
    k_repack_finish<<<blocks, 256, 0, st>>>(a, newoff, cnt);
    return hipGetLastError();
}
hipError_t export_edges(const KArgs &a, int32_t *xs, int32_t *ys, int64_t cap,
                        unsigned long long *tail, int blocks, hipStream_t st) {
    k_export<<<blocks, 256, 0, st>>>(a, xs, ys, cap, tail);
    return hipGetLastError();
}

static hipError_t coop(const void *fn, const KArgs &a, int blocks, hipStream_t st) {
    KArgs copy = a;
    void *args[] = {&copy};
    return hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(COOP_THREADS), args, 0, st);
}

hipError_t dec_prep(const KArgs &a, int blocks, hipStream_t st) {
    k_dec_prep<<<blocks, 256, 0, st>>>(a);
    return hipGetLastError();
}
hipError_t decompose_coop(const KArgs &a, int blocks, hipStream_t st) {
    return coop((const void *)k_decompose, a, blocks, st);
}
hipError_t mcd_init(const KArgs &a, int blocks, hipStream_t st) {
    k_mcd_init<<<blocks, 256, 0, st>>>(a);
    return hipGetLastError();
}
hipError_t validate_batch(const KArgs &a, int blocks, hipStream_t st) {
    k_val_canon<<<blocks, 256, 0, st>>>(a);
    k_val_dup_mark<<<blocks, 256, 0, st>>>(a);
    k_val_scan<<<blocks, 256, 0, st>>>(a);
    k_val_final<<<blocks, 256, 0, st>>>(a);
    if (a.b.sub_in) k_val_subfilter<<<blocks, 256, 0, st>>>(a);
    return hipGetLastError();
}
hipError_t reserve_gain(const KArgs &a, int blocks, hipStream_t st) {
    k_res_gain<<<blocks, 256, 0, st>>>(a);
    return hipGetLastError();
}
hipError_t reserve_alloc_copy(const KArgs &a, int blocks, hipStream_t st) {
    k_res_alloc<<<blocks, 256, 0, st>>>(a);
    k_res_copy<<<blocks, 256, 0, st>>>(a);
    return hipGetLastError();
}
hipError_t delete_compact(const KArgs &a, int blocks, hipStream_t st) {
    k_del_compact<<<blocks, 256, 0, st>>>(a);
    return hipGetLastError();
}
hipError_t maintain_coop(const KArgs &a, int blocks, hipStream_t st) {
    return coop((const void *)k_maintain, a, blocks, st);
}
hipError_t program_coop(const KArgs &a, int blocks, hipStream_t st) {
    return coop((const void *)k_program, a, blocks, st);
}
const void *program_kernel() { return (const void *)k_program; }
hipError_t serve_coop(const KArgs &a, int blocks, hipStream_t st) {
    return coop((const void *)k_serve, a, blocks, st);
}
hipError_t vins_init(const KArgs &a, int32_t first, int32_t c, hipStream_t st) {
    k_vins_init<<<grid_for(c, 4096), 256, 0, st>>>(a, first, c);
    return hipGetLastError();
}
hipError_t vins_revert(const KArgs &a, int32_t first, int32_t c, hipStream_t st) {
    k_vins_revert<<<grid_for(c, 4096), 256, 0, st>>>(a, first, c);
    return hipGetLastError();
}
hipError_t vins_expand(const int64_t *off, int32_t c, int32_t first, int32_t *src, int blocks,
                       hipStream_t st) {
    k_vins_expand<<<blocks, 256, 0, st>>>(off, c, first, src);
    return hipGetLastError();
}
hipError_t vins_check_off(const int64_t *off, int32_t c, unsigned long long *first_bad, hipStream_t st) {
    k_vins_check_off<<<grid_for(c, 4096), 256, 0, st>>>(off, c, first_bad);
    return hipGetLastError();
}
hipError_t vdel_check(const KArgs &a, const int32_t *ids, int32_t c, int32_t *firstidx,
                      unsigned long long *first_bad, unsigned long long *total, hipStream_t st) {
    k_vdel_check<<<grid_for(c, 4096), 256, 0, st>>>(a, ids, c, firstidx, first_bad);
    k_vdel_dup<<<grid_for(c, 4096), 256, 0, st>>>(a, ids, c, firstidx, first_bad, total);
    k_vdel_reset_first<<<grid_for(c, 4096), 256, 0, st>>>(a, ids, c, firstidx);
    return hipGetLastError();
}
hipError_t vdel_gather(const KArgs &a, const int32_t *ids, int32_t c, int32_t *xs, int32_t *ys,
                       int64_t cap, unsigned long long *tail, int blocks, hipStream_t st) {
    k_vdel_gather<<<blocks, 256, 0, st>>>(a, ids, c, xs, ys, cap, tail);
    return hipGetLastError();
}
hipError_t vdel_finish(const KArgs &a, const int32_t *ids, int32_t c, hipStream_t st) {
    k_vdel_finish<<<grid_for(c, 4096), 256, 0, st>>>(a, ids, c);
    return hipGetLastError();
}

hipError_t coop_occupancy(int which, int *blocks_per_cu) {
    const void *fn = which == 0   ? (const void *)k_maintain
                     : which == 1 ? (const void *)k_decompose
                     : which == 2 ? (const void *)k_program
                                  : (const void *)k_serve;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, COOP_THREADS, 0);
}

}  // namespace cm
