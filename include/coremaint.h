/*
 * coremaint.h -- C ABI of libcoremaint.so: batched core maintenance of a
 * dynamic undirected graph on one AMD Instinct MI355X (gfx950).
 *
 * Method: "Parallel Algorithms for Core Maintenance in Dynamic Graphs"
 * (Wang, Yu, Jin, Qian, Xie, Hua).  A batch of inserted (deleted) edges is
 * processed in iterations; each iteration selects a superior edge set
 * (Section IV, definition of the k-superior edge set), applies it to the
 * graph, finds for every core level k in parallel the core-k vertices whose
 * core number moves (Algorithms 3-4 for insertion, 6-7 for deletion) and
 * moves them by exactly one (Algorithms 1 and 5).  Vertex insertion and
 * deletion reduce to edge insertion and deletion (Introduction).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Status: every call returns an int; CM_OK (0) on success, a negative
 *   CM_E_* code otherwise.  No C++ exception crosses this boundary.
 *   cm_last_error(g) gives a text message for the last failure on g.
 * - Ids: vertices are dense int32 ids in [0, n_ids).  Deleted ids stay dead
 *   (core reported as -1) and are never reused; inserted vertices receive
 *   fresh ids n_ids, n_ids+1, ...
 * - Edges: an undirected edge is given once, in either orientation; pairs
 *   are canonicalised to (min, max).  The graph stays simple.
 * - Batch validation (strict mode, the default): an item is invalid when an
 *   endpoint is outside [0, n_ids) (CM_E_RANGE), an endpoint is dead
 *   (CM_E_DEAD), it is a self-loop (CM_E_SELF_LOOP), its pair occurred at an
 *   earlier index of the same batch (CM_E_DUP), or for insertion the edge
 *   already exists (CM_E_EXISTS) / for deletion it does not (CM_E_MISSING);
 *   checks apply in that order.  A batch with any invalid item is rejected
 *   as a whole, the graph is left unchanged, the call returns the code of
 *   the smallest invalid index and stats->first_bad holds that index.
 *   Filter mode (cm_config.strict = 0) drops invalid items, counts them in
 *   stats->dropped and applies the rest.
 * - Memory: `on_device` = 1 means the pointer is device memory of the
 *   current HIP device (e.g. a torch tensor's data_ptr), 0 means host memory.
 *   Inputs are borrowed for the duration of the call; outputs are
 *   caller-allocated.  Every call has returned only after the work it
 *   enqueued on the handle's stream has completed.
 * - Threading: one call at a time per handle.
 * - Core numbers are exact int32 values: after every successful update call
 *   they equal the core numbers of the updated graph (core number
 *   definition, Section III).
 */
#ifndef COREMAINT_H
#define COREMAINT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CM_OK 0
#define CM_E_ARG (-1)       /* bad argument (null pointer, negative size, bad mode) */
#define CM_E_RANGE (-2)     /* vertex id outside [0, n_ids) */
#define CM_E_SELF_LOOP (-3) /* edge <v, v> */
#define CM_E_DUP (-4)       /* pair (or id) repeated inside one batch */
#define CM_E_EXISTS (-5)    /* inserted edge already in the graph */
#define CM_E_MISSING (-6)   /* deleted edge not in the graph */
#define CM_E_DEAD (-7)      /* id of a deleted vertex */
#define CM_E_NOMEM (-8)     /* device or host allocation failed */
#define CM_E_CAPACITY (-9)  /* configured vertex capacity exceeded */
#define CM_E_STATE (-10)    /* call not valid in the handle's state (e.g. no graph loaded) */
#define CM_E_DEVICE (-11)   /* HIP runtime error; the handle is poisoned */
#define CM_E_INTERNAL (-12) /* internal invariant violated (queue overflow); handle poisoned */
#define CM_E_BUSY (-13)     /* serving: the request must wait (ring, payload space or budget full) */
#define CM_E_IO (-14)       /* snapshot file missing, unreadable, corrupt or inconsistent */

/* Execution forms of the update path. */
#define CM_MODE_PLAIN 0     /* host loop: one cooperative launch per superior edge set */
#define CM_MODE_PERSISTENT 1 /* one cooperative launch loops over all sets of the batch */

typedef struct cm_graph cm_graph; /* opaque; owned by the library */

typedef struct cm_config {
    int32_t vertex_capacity;    /* max vertex ids over the handle's lifetime; 0 = auto (grows) */
    int64_t edge_capacity_hint; /* adjacency slots to reserve up front; 0 = auto */
    int32_t strict;             /* 1 = reject an invalid batch whole (default), 0 = drop items */
    int32_t mode;               /* CM_MODE_PLAIN or CM_MODE_PERSISTENT */
    int32_t partition_rounds;   /* selection rounds per superior edge set (1..8; 0 = default) */
    int32_t blocks_per_cu;      /* cooperative grid occupancy (0 = default) */
    int32_t small_degree;       /* whole-graph passes and the asynchronous cascade form walk lists up to
                                   this length with one lane, longer ones with a wave (0 = default) */
    int32_t large_degree;       /* lists above this length are split into chunks; shorter ones are walked
                                   flattened, up to 64 lists per wave (0 = default) */
    int32_t chunk;              /* chunk length for long lists (0 = default) */
    int32_t local_edges;        /* selection / apply steps up to this many edges run in one
                                   workgroup instead of the whole grid (0 = default) */
    int32_t local_items;        /* frontier steps up to this many items run in one workgroup
                                   (0 = default) */
    int32_t local_work;         /* ... if their lists hold at most this many entries (0 = default) */
    int32_t timing;             /* 1 = time each maintenance launch with HIP events */
    int32_t use_graph;          /* 1 = cm_run_batches replays its persistent launch from an
                                   instantiated hipGraph (rebuilt when buffers move) */
    int32_t async_steps;        /* 1 = each expansion / eviction / peel cascade runs as one
                                   work-queue step instead of one grid-wide step per round */
    int32_t single_edge;        /* 1 = one edge per iteration (the sequential regime the
                                   paper compares against) instead of a superior edge set */
    int32_t debug;              /* > 0 = keep the iteration log of the last update call
                                   (cm_debug_log) with room for 2^20 entries of each kind,
                                   or for `debug` entries when debug > 1 */
    int32_t expand_mode;        /* insertion's subcore expansion (Algorithm 3): 1 = a candidate
                                   visits its neighbours only once its CSD exceeds its core (the
                                   algorithm's pruning: two passes over an expanding list); 2 = it
                                   claims them while counting its CSD (one pass per list, a
                                   larger visited set, same cores); 3 = as 2, and the pass also
                                   records the candidate's neighbours at its level with SD above
                                   it, the only ones whose counters its eviction (Algorithm 4)
                                   lowers, so that an eviction walks those instead of the whole
                                   list (one more int32 per adjacency slot of device memory);
                                   4 = as 3, and every list split into chunks keeps, per chunk,
                                   the neighbours whose core was at least its owner's at its last
                                   whole scan, which later expansions read instead of the chunk
                                   (kept until a change could add a neighbour outside it; one
                                   more int32 per adjacency slot); 0 = default (4; 2 with
                                   async_steps) */
    int32_t stamp_limit;        /* iteration stamps restart (the kernels clear the arrays that hold
                                   them, at an iteration boundary) before a stamp passes this;
                                   0 = default (2^28, also the largest allowed) */
    void *stream;               /* hipStream_t to run on; NULL = the null stream */
} cm_config;

typedef struct cm_batch_stats {
    int32_t status;         /* same value the call returned */
    int32_t iterations;     /* superior edge sets processed */
    int64_t first_bad;      /* smallest invalid item index, -1 if none */
    int64_t applied;        /* edges applied to the graph */
    int64_t dropped;        /* invalid items dropped (filter mode) */
    int64_t remaining_sum;  /* sum over iterations of edges still to place (partition work) */
    int64_t candidates;     /* sum over iterations of candidate vertices visited */
    int64_t evicted;        /* sum of evicted (insert) / peeled (delete) vertices */
    int64_t changed;        /* sum of vertices whose core moved */
    int64_t scanned;        /* adjacency entries read by traversal phases */
    int64_t alg_bytes;      /* algorithmic HBM bytes of the method's own work on the batch:
                               32 per remaining edge per iteration (partition), 40 per applied
                               edge (validation and apply), per candidate and per evicted vertex
                               16 + 12 per list entry (CSD count; counter decrements), per
                               changed vertex 20 per list entry (SD recount, neighbour deltas) */
    int64_t rounds;         /* cascade rounds (expansion, eviction, peel) */
    int64_t cand_degree;    /* sum of list lengths over the insertion candidates visited */
    int64_t evicted_degree; /* sum of list lengths over the evicted / peeled vertices */
    int64_t changed_degree; /* sum of list lengths over the vertices whose core moved */
    int64_t grid_steps;     /* steps run by the whole grid (each ends in a grid barrier) */
    int64_t local_steps;    /* steps run inside one workgroup */
    int32_t launches;       /* maintenance kernel launches (plain mode: one per superior edge
                               set plus the empty one that ends the batch, queued before the
                               host knew no edges were left) */
    int32_t graph_launch;   /* 1 when the launch was replayed from a hipGraph */
    int32_t group;          /* serving: requests that ran in one fused batch with this one
                               (1 = alone; the statistics above are the batch's) */
    int32_t first_stamp;    /* iteration stamp of the batch's first iteration (debug log) */
    double kernel_ms;       /* summed HIP-event time of those launches (timing = 1; the
                               plain mode times every launch) */
    double ms_total;        /* wall time of the call */
} cm_batch_stats;

/* Fill *cfg with defaults (strict, plain mode, auto capacities, null stream). */
void cm_config_default(cm_config *cfg);

/* Create an empty handle on the current HIP device.  cfg may be NULL. */
int cm_create(const cm_config *cfg, cm_graph **out);

/* Release every device and host resource of g.  g may be NULL. */
void cm_destroy(cm_graph *g);

/* Text for a status code. */
const char *cm_strerror(int status);

/* Message of the last failing call on g (empty if none). */
const char *cm_last_error(const cm_graph *g);

/* Load the simple graph G = (V, E) with V = [0, n) and E given as m pairs
 * (src[i], dst[i]) (problem definition, Section III).  Replaces any graph
 * already held.  Pairs must be distinct and loop-free: CM_E_RANGE,
 * CM_E_SELF_LOOP or CM_E_DUP otherwise (graph left empty).  Core numbers
 * are not computed until cm_core_decompose. */
int cm_load_graph(cm_graph *g, int32_t n, int64_t m, const int32_t *src,
                  const int32_t *dst, int on_device);

/* Initial state: core number of every vertex (core number definition,
 * Section III) by parallel level-synchronous peeling on the device, plus
 * each vertex's superior degree SD (Section IV-B definition).  stats may
 * be NULL (only ms_total, scanned, kernel_ms are filled). */
int cm_core_decompose(cm_graph *g, cm_batch_stats *stats);

/* Incremental core maintenance (Section V): insert s edges, then bring every
 * core number up to date.  stats may be NULL. */
int cm_insert_edges(cm_graph *g, int64_t s, const int32_t *src, const int32_t *dst,
                    int on_device, cm_batch_stats *stats);

/* Decremental core maintenance (Section VI): delete s edges, then bring
 * every core number up to date.  stats may be NULL. */
int cm_delete_edges(cm_graph *g, int64_t s, const int32_t *src, const int32_t *dst,
                    int on_device, cm_batch_stats *stats);

/* Largest batch of cm_update_edges_noalloc. */
#define CM_NOALLOC_MAX_ITEMS (1 << 16)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * update as cm_insert_edges (kind CM_BATCH_INSERT) or cm_delete_edges (kind
 * CM_BATCH_DELETE), with src / dst in device memory, that allocates nothing:
 * the per-call batch arrays, batch hash and locate-scan queue live in one
 * file-scope device array of the library (about 13 MiB, held by every GPU
 * the library runs on until the process ends).  Limits: s <=
 * CM_NOALLOC_MAX_ITEMS, and 2 s + (adjacency pool slots) / chunk + 1024 <=
 * 2^20 (about 2.3 x 10^8 pool slots with the default chunk of 256), else
 * CM_E_CAPACITY before any work; an insertion that would need
 * a larger adjacency pool returns CM_E_CAPACITY with the graph unchanged
 * (cm_insert_edges grows the pool instead).  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (from any handle, on any
 * stream) race and must not be issued. */
int cm_update_edges_noalloc(cm_graph *g, int32_t kind, int64_t s, const int32_t *src, const int32_t *dst,
                            cm_batch_stats *stats);

/* Vertex insertion (Introduction: a new vertex enters with core 0, then its
 * edges are inserted).  c new vertices get ids first..first+c-1 where
 * first = n_ids on entry (*first_new_id receives it, may be NULL).  Vertex i
 * is joined to nbrs[off[i] .. off[i+1]); off has c+1 entries starting at 0.
 * Neighbours may be live ids or ids of this call's new vertices; an edge
 * between two new vertices is listed once.  Invalid items are reported by
 * their index in nbrs (validation convention above); in strict mode no
 * vertex is created on error. */
int cm_insert_vertices(cm_graph *g, int32_t c, const int64_t *off, const int32_t *nbrs,
                       int on_device, int32_t *first_new_id, cm_batch_stats *stats);

/* Vertex deletion (Introduction: the vertex's edges are deleted, then the
 * vertex).  ids must be live, in range and distinct (CM_E_DEAD, CM_E_RANGE,
 * CM_E_DUP, index in stats->first_bad).  Deleted ids report core -1. */
int cm_delete_vertices(cm_graph *g, int32_t c, const int32_t *ids, int on_device,
                       cm_batch_stats *stats);

/* Copy the core numbers of ids [0, n) to out (n <= n_ids; dead ids -> -1). */
int cm_get_cores(cm_graph *g, int32_t *out, int32_t n, int on_device);

/* Current id count (live + dead) and live vertex count. */
int cm_num_vertices(cm_graph *g, int32_t *n_ids, int32_t *n_alive);

/* Current number of undirected edges. */
int cm_num_edges(cm_graph *g, int64_t *m);

/* Export the edge set: every undirected edge once as (min, max), in no
 * particular order, into caller buffers of capacity cap; *m_out receives
 * the edge count (CM_E_ARG if cap is too small, *m_out still set). */
int cm_export_edges(cm_graph *g, int32_t *src, int32_t *dst, int64_t cap,
                    int64_t *m_out, int on_device);

/* Batch kinds of cm_run_batches. */
#define CM_BATCH_INSERT 0
#define CM_BATCH_DELETE 1

/* Run nb edge batches in order (Algorithms 1 and 5 per batch).  Batch j is
 * items [offsets[j], offsets[j+1]) of src/dst with kind kinds[j]
 * (CM_BATCH_INSERT / CM_BATCH_DELETE); kinds and offsets are host arrays
 * (offsets has nb+1 entries, starting at 0), src/dst follow on_device.
 * Each batch is validated against the graph as left by the batches before
 * it; in strict mode an invalid batch is skipped whole (results[j].status
 * holds the code of its smallest invalid item) and later batches still run.
 *
 * Packed independent batches: sub (optional, same location as src) gives
 * every item a sub-batch id in [0, nsub); a sub-batch lies inside one batch.
 * Strictness then applies per sub-batch: a sub-batch with an invalid item
 * is dropped whole and sub_status[b] (host, nsub entries, may be NULL)
 * receives its code; the other sub-batches of the batch proceed.  This is
 * how many independent graphs, packed as one disjoint union, are updated
 * by one launch.
 *
 * CM_MODE_PLAIN: host loop, one cooperative launch per superior edge set.
 * CM_MODE_PERSISTENT: one cooperative launch runs every batch (validation,
 * reservation, all iterations, compaction); with use_graph it is replayed
 * from a hipGraph.  results (nb entries) may be NULL.  Timing fields: in
 * the plain mode every entry holds its own batch (ms_total, kernel_ms,
 * launches); in the persistent mode results[0] holds the whole call (the one
 * launch, its HIP-event time and the wall time) and the other entries zero.
 * Returns CM_OK unless the call itself failed (bad arguments, device error). */
int cm_run_batches(cm_graph *g, int32_t nb, const int32_t *kinds, const int64_t *offsets,
                   const int32_t *src, const int32_t *dst, const int32_t *sub, int32_t nsub,
                   int on_device, cm_batch_stats *results, int32_t *sub_status);

/* Copy the maintained superior degree SD(v) (Section IV-B definition) of
 * ids [0, n) to out; dead ids report 0. */
int cm_get_superior_degrees(cm_graph *g, int32_t *out, int32_t n, int on_device);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of update requests on one resident graph.
 *
 * Requests (edge insertions or deletions, vertex insertions or deletions,
 * in the Introduction's reduction to edge updates) are copied into a ring of
 * pinned host memory and published; one persistent cooperative launch reads
 * each request from the ring as soon as it is published, applies it exactly
 * as the one-call API would (validation through compaction; in strict mode
 * an invalid request changes nothing), records its outcome and moves on,
 * so requests that arrive while others run join the running launch without
 * a host round trip.  Requests apply in ticket order.  The launch leaves
 * after idle_ms without work, when stopped, or when the adjacency pool must
 * be repacked or vertex capacity grown; the next submit or poll launches it
 * again.  Admission is by memory: a request waits (CM_E_BUSY) while the
 * ring has no free slot, the payload ring no room, or the device bytes that
 * unfinished requests may claim (payload plus an estimate of adjacency
 * growth for insertions) would exceed budget_bytes.  While serving, the
 * other calls on the handle return CM_E_STATE (cm_num_* excepted); call
 * cm_serve_stop first.
 * ------------------------------------------------------------------------- */
typedef struct cm_serve_config {
    int32_t ring_requests;    /* request slots (default 4096) */
    int32_t idle_ms;          /* launch leaves after this long without work (default 20) */
    int64_t ring_items;       /* payload slots of the pinned ring, int32 pairs (default 2^24) */
    int64_t max_items;        /* largest request, in items (edges; ids for a vertex deletion); also
                                 the most incident edges one vertex deletion may gather (default 2^22) */
    int64_t budget_bytes;     /* device bytes unfinished requests may claim (default 2^30) */
    int32_t vertex_headroom;  /* vertex capacity kept beyond the ids in use (default 2^20) */
    int32_t fuse;             /* continuous batching across sessions: most requests fused into one
                                 batch (<= 32; 0 or 1 = every request runs alone; strict mode only) */
} cm_serve_config;

#define CM_REQ_INSERT_EDGES 0
#define CM_REQ_DELETE_EDGES 1
#define CM_REQ_INSERT_VERTICES 2
#define CM_REQ_DELETE_VERTICES 3

void cm_serve_config_default(cm_serve_config *cfg);

/* Enter serving on a decomposed graph (cfg may be NULL for the defaults). */
int cm_serve_start(cm_graph *g, const cm_serve_config *cfg);

/* Submit an edge request (kind CM_REQ_INSERT_EDGES / CM_REQ_DELETE_EDGES; s
 * pairs in host arrays, copied before return).  *ticket receives its
 * position in the request order.  CM_E_BUSY: not admitted now, submit it
 * again later; CM_E_CAPACITY: larger than max_items.
 *
 * session >= 0 names an independent session: the caller guarantees that
 * requests of different sessions touch disjoint vertex sets with no edge
 * between them (e.g. independent graphs packed into one handle).  With
 * cfg.fuse > 1, consecutive published edge requests of one kind from
 * distinct sessions run fused in one batch (continuous batching): they are
 * validated together, each keeping its own strictness (an invalid request
 * changes nothing and gets its own status), share their iterations, and
 * each gets the result it would get alone, since the sessions cannot
 * influence each other's core numbers (a disjoint union's cores are its
 * members' cores).  Requests of one session never share a batch, and a
 * session < 0 never fuses. */
int cm_serve_submit_edges(cm_graph *g, int32_t session, int32_t kind, int64_t s, const int32_t *src,
                          const int32_t *dst, int64_t *ticket);

/* Submit a vertex insertion: c new vertices with neighbour lists in CSR
 * form (off int64[c+1] with off[0] = 0, nbrs int32[off[c]], host memory).
 * Ids are assigned at submission (*first_new_id); if the request is
 * rejected when it runs, its ids stay allocated as dead ids. */
int cm_serve_submit_insert_vertices(cm_graph *g, int32_t c, const int64_t *off, const int32_t *nbrs,
                                    int32_t *first_new_id, int64_t *ticket);

/* Submit a vertex deletion of c ids (host memory).  A request whose ids
 * have more than max_items incident edges fails with CM_E_CAPACITY. */
int cm_serve_submit_delete_vertices(cm_graph *g, int32_t c, const int32_t *ids, int64_t *ticket);

/* Progress: collect finished requests, relaunch if work is pending; never
 * blocks.  *finished (may be NULL) = number of requests finished (every
 * ticket below it). */
int cm_serve_poll(cm_graph *g, int64_t *finished);

/* Outcome of a finished request (CM_E_BUSY while it is unfinished).
 * status is the request's own status; applied counts its edges. */
int cm_serve_result(cm_graph *g, int64_t ticket, cm_batch_stats *out);

/* Finish every admitted request, end the launch and leave serving. */
int cm_serve_stop(cm_graph *g);

/* Checkpoint: write the graph's state to the file at path -- id count, live
 * count, the core number of every id (-1 for dead ids), the maintained SD
 * of every id, and the edge set -- so that cm_restore can continue the
 * update stream exactly where it stopped (core numbers are a function of
 * the graph, Section III, and SD of the cores, Section IV-B).  Needs a
 * decomposed graph; the graph is not changed.  CM_E_IO when the file cannot
 * be written. */
int cm_snapshot(cm_graph *g, const char *path);

/* Create a handle (cfg as for cm_create, may be NULL) holding the state
 * written by cm_snapshot, without a new decomposition.  CM_E_IO when the
 * file is missing, truncated, fails its checksum or is inconsistent (a
 * core outside [-1, n_ids), an edge at a dead or out-of-range id, a live
 * count that does not match).  *out is NULL on failure. */
int cm_restore(const cm_config *cfg, const char *path, cm_graph **out);

/* Iteration log of the last update call on a handle created with
 * cfg.debug > 0 (Algorithms 1 and 5 step by step): sel receives sel_cap
 * entries of 3 int32 (iteration stamp, u, v), one per edge of a selected
 * superior edge set, u < v; chg receives chg_cap entries (iteration stamp,
 * v, new core), one per core number moved by an iteration.  Stamps grow by
 * one per iteration, so the entries of one stamp are one superior edge set
 * and the core changes it caused.  *n_sel / *n_chg receive the counts
 * recorded.  The sets of vertex-star iterations (vertex operations in the
 * persistent form, batch programs and serving) are not logged, their core
 * changes of existing vertices are (a new vertex's starting core and a
 * deleted vertex's -1 are not).  In serving, the log covers everything
 * since cm_serve_start.  CM_E_STATE
 * without debug mode; CM_E_CAPACITY when the log overflowed (entries past
 * its capacity are lost; the counts still report the totals). */
int cm_debug_log(cm_graph *g, int64_t *n_sel, int32_t *sel, int64_t sel_cap, int64_t *n_chg, int32_t *chg,
                 int64_t chg_cap);

/* Phase clock of the maintenance kernels, for profiling one persistent
 * launch from the inside: ms[i] (host, n <= 16 entries) receives the device
 * wall-clock time summed over every phase i since the graph was loaded or
 * the clock was last reset, counts[i] (may be NULL) how often it ran.
 * Slots 0..7 are grid-wide steps of an iteration (claim, select, apply,
 * expansion round, eviction round, peel round, core update, SD update),
 * 8 chains of steps run inside one workgroup, 9..11 validation, capacity
 * reservation and compaction inside cm_run_batches' persistent launch.
 * reset != 0 clears the clock afterwards.  No device work is started. */
int cm_phase_times(cm_graph *g, double *ms, int64_t *counts, int32_t n, int reset);

#ifdef __cplusplus
}
#endif
#endif /* COREMAINT_H */
