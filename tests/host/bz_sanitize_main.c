/* Host sanitizer run of the oracle's C code (oracle/bz.c), built with
 * -fsanitize=address,undefined by tests/test_sanitize.py: random graphs of
 * many shapes (empty, isolated ids, dead ids, dense, sparse, stars), each
 * decomposed by oracle_bz_cores, and the result checked against the core
 * number property itself: every live vertex v with core k has at least k
 * neighbours of core >= k (v lies in the k-core) and fewer than k + 1
 * neighbours of core >= k + 1 ... checked through threshold peeling of the
 * (k+1)-core written out here. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_bz_cores(int32_t n, const int64_t *off, const int32_t *adj, const uint8_t *alive, int32_t *core);
int64_t oracle_build_csr(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int64_t *off,
                         int32_t *adj);

static uint64_t state = 88172645463325252ull;
static uint32_t rnd(void) {
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (uint32_t)state;
}

/* Peel every live vertex of degree < k repeatedly; out[v] = 1 if v survives. */
static void kcore(int32_t n, const int64_t *off, const int32_t *adj, const uint8_t *alive, int32_t k,
                  uint8_t *out) {
    int32_t *deg = calloc((size_t)n + 1, sizeof(int32_t));
    for (int32_t v = 0; v < n; ++v) {
        out[v] = alive[v];
        if (alive[v]) deg[v] = (int32_t)(off[v + 1] - off[v]);
    }
    int changed = 1;
    while (changed) {
        changed = 0;
        for (int32_t v = 0; v < n; ++v) {
            if (!out[v] || deg[v] >= k) continue;
            out[v] = 0;
            changed = 1;
            for (int64_t e = off[v]; e < off[v + 1]; ++e)
                if (out[adj[e]]) deg[adj[e]]--;
        }
    }
    free(deg);
}

int main(void) {
    int fails = 0;
    for (int t = 0; t < 300; ++t) {
        int32_t n = 1 + (int32_t)(rnd() % 120);
        int64_t cap = (int64_t)n * (n - 1) / 2;
        int64_t m = cap ? (int64_t)(rnd() % (uint32_t)(cap + 1)) : 0;
        if (t % 3 == 0) m /= 8;
        int32_t *src = malloc(sizeof(int32_t) * ((size_t)m + 1));
        int32_t *dst = malloc(sizeof(int32_t) * ((size_t)m + 1));
        uint8_t *alive = malloc((size_t)n);
        uint8_t *seen = calloc((size_t)n * (size_t)n, 1);
        for (int32_t v = 0; v < n; ++v) alive[v] = (t % 4 == 0) ? (rnd() % 5 != 0) : 1;
        int64_t k = 0;
        for (int64_t i = 0; i < m; ++i) {
            int32_t a = (int32_t)(rnd() % (uint32_t)n), b = (int32_t)(rnd() % (uint32_t)n);
            if (t % 5 == 1) a = 0; /* stars */
            if (a == b || !alive[a] || !alive[b] || seen[(size_t)a * n + b]) continue;
            seen[(size_t)a * n + b] = seen[(size_t)b * n + a] = 1;
            src[k] = a;
            dst[k] = b;
            ++k;
        }
        int64_t *off = malloc(sizeof(int64_t) * ((size_t)n + 1));
        int32_t *adj = malloc(sizeof(int32_t) * ((size_t)(2 * k) + 1));
        int32_t *core = malloc(sizeof(int32_t) * (size_t)n);
        uint8_t *in = malloc((size_t)n);
        if (oracle_build_csr(n, k, src, dst, off, adj) != 2 * k) { printf("csr %d\n", t); ++fails; }
        if (oracle_bz_cores(n, off, adj, alive, core) != 0) { printf("bz %d\n", t); ++fails; }
        int32_t kmax = 0;
        for (int32_t v = 0; v < n; ++v) {
            if (!alive[v] && core[v] != -1) { printf("dead %d %d\n", t, v); ++fails; }
            if (alive[v] && core[v] > kmax) kmax = core[v];
        }
        for (int32_t kk = 1; kk <= kmax + 1; ++kk) {
            kcore(n, off, adj, alive, kk, in);
            for (int32_t v = 0; v < n; ++v)
                if (alive[v] && (in[v] != 0) != (core[v] >= kk)) { printf("core %d v%d k%d\n", t, v, kk); ++fails; }
        }
        free(src); free(dst); free(alive); free(seen); free(off); free(adj); free(core); free(in);
        if (fails > 10) break;
    }
    printf(fails ? "bz: %d failures\n" : "bz: ok\n", fails);
    return fails ? 1 : 0;
}
