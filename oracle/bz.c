/*
 * Core-decomposition oracle: the O(m) bucket algorithm of Batagelj and
 * Zaversnik, which the paper cites as the linear-time static decomposition
 * (Introduction; Related Work).  Test infrastructure only: the GPU library
 * never links or calls this file.
 *
 * The method, restated from its published description:
 *   1. deg[v] = |N(v)| for every live vertex; D = max deg.
 *   2. Counting-sort the live vertices by deg into vert[]; bin[d] is the first
 *      index of the degree-d block and pos[v] the index of v in vert[].
 *   3. Walk vert[] in order.  The current deg of the visited vertex v is final
 *      (its core number).  For every neighbour u whose deg is still larger
 *      than deg[v], move u to the front of its bin (swap with the vertex at
 *      bin[deg[u]]), advance that bin's start by one and decrement deg[u]:
 *      u has lost the support of v.
 *   4. core[v] = deg[v]; isolated live vertices get 0; dead ids get -1.
 *
 * Input is a symmetric CSR (each undirected edge in both lists) over ids
 * 0..n-1.  Entries < 0 in adj are ignored (they are never produced by the
 * oracle's own CSR builder, but the check keeps the routine total).
 * Returns 0 on success, -1 on allocation failure.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int oracle_bz_cores(int32_t n, const int64_t *off, const int32_t *adj,
                    const uint8_t *alive, int32_t *core) {
    if (n <= 0) return 0;
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *vert = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!deg || !pos || !vert) {
        free(deg); free(pos); free(vert);
        return -1;
    }
    int32_t maxd = 0;
    int32_t nlive = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (alive && !alive[v]) { deg[v] = -1; continue; }
        int32_t d = 0;
        for (int64_t e = off[v]; e < off[v + 1]; ++e)
            if (adj[e] >= 0) ++d;
        deg[v] = d;
        if (d > maxd) maxd = d;
        ++nlive;
    }
    int64_t *bin = (int64_t *)calloc((size_t)maxd + 2, sizeof(int64_t));
    if (!bin) { free(deg); free(pos); free(vert); return -1; }
    for (int32_t v = 0; v < n; ++v)
        if (deg[v] >= 0) bin[deg[v]]++;
    /* exclusive prefix: bin[d] = first slot of degree-d block */
    int64_t start = 0;
    for (int32_t d = 0; d <= maxd; ++d) {
        int64_t c = bin[d];
        bin[d] = start;
        start += c;
    }
    for (int32_t v = 0; v < n; ++v) {
        if (deg[v] < 0) continue;
        pos[v] = (int32_t)bin[deg[v]];
        vert[pos[v]] = v;
        bin[deg[v]]++;
    }
    /* restore starts */
    for (int32_t d = maxd; d >= 1; --d) bin[d] = bin[d - 1];
    bin[0] = 0;

    for (int32_t i = 0; i < nlive; ++i) {
        int32_t v = vert[i];
        for (int64_t e = off[v]; e < off[v + 1]; ++e) {
            int32_t u = adj[e];
            if (u < 0 || deg[u] < 0) continue;
            if (deg[u] > deg[v]) {
                int32_t du = deg[u];
                int32_t pu = pos[u];
                int32_t pw = (int32_t)bin[du];
                int32_t w = vert[pw];
                if (u != w) {
                    pos[u] = pw; vert[pw] = u;
                    pos[w] = pu; vert[pu] = w;
                }
                bin[du]++;
                deg[u]--;
            }
        }
    }
    for (int32_t v = 0; v < n; ++v) core[v] = deg[v];  /* dead stay -1 */
    free(bin); free(deg); free(pos); free(vert);
    return 0;
}

/* Symmetric CSR from an undirected edge list (each pair given once).
 * off must hold n+1 entries, adj 2*m.  Pairs with an endpoint outside
 * [0, n) are skipped.  Returns the number of adjacency entries written. */
int64_t oracle_build_csr(int32_t n, int64_t m, const int32_t *src,
                         const int32_t *dst, int64_t *off, int32_t *adj) {
    memset(off, 0, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t i = 0; i < m; ++i) {
        int32_t a = src[i], b = dst[i];
        if (a < 0 || b < 0 || a >= n || b >= n) continue;
        off[a + 1]++;
        off[b + 1]++;
    }
    for (int32_t v = 0; v < n; ++v) off[v + 1] += off[v];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!fill) return -1;
    memcpy(fill, off, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t i = 0; i < m; ++i) {
        int32_t a = src[i], b = dst[i];
        if (a < 0 || b < 0 || a >= n || b >= n) continue;
        adj[fill[a]++] = b;
        adj[fill[b]++] = a;
    }
    free(fill);
    return off[n];
}
