/*
 * Seeded synthetic graph generators: input generation only.
 *
 * This file computes nothing of the betweenness method. It builds edge lists
 * that the oracle and the GPU library both consume as identical CSR bytes.
 * The random stream is SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), used
 * here only to draw graph structure.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Uniform integer in [0, bound) by the 128-bit multiply-high map. */
static uint64_t below(uint64_t *state, uint64_t bound)
{
    unsigned __int128 p = (unsigned __int128)splitmix64_next(state) * bound;
    return (uint64_t)(p >> 64);
}

/*
 * Barabasi-Albert preferential attachment.
 * Seed graph: the clique on m+1 vertices. Every later vertex i attaches to m
 * distinct earlier vertices, each drawn with probability proportional to its
 * current degree (uniform draw from the list of all edge endpoints so far;
 * a repeated pick is redrawn). The endpoints of vertex i's own edges join the
 * list only after all m targets are fixed.
 *
 * src/dst receive m(m+1)/2 + m(n-m-1) undirected edges (each once).
 * Returns the number of edges written, or -1 on bad arguments / no memory.
 */
int64_t graphgen_ba(int64_t n, int32_t m, uint64_t seed, int32_t *src, int32_t *dst)
{
    if (m < 1 || n < (int64_t)m + 1 || n > 0x7fffffffLL) return -1;
    int64_t n_edges = (int64_t)m * (m + 1) / 2 + (int64_t)m * (n - m - 1);
    int32_t *ends = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)n_edges);
    int32_t *pick = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    if (!ends || !pick) { free(ends); free(pick); return -1; }
    uint64_t st = seed;
    int64_t ne = 0, nends = 0;
    for (int32_t a = 0; a <= m; ++a)
        for (int32_t b = a + 1; b <= m; ++b) {
            src[ne] = a; dst[ne] = b; ++ne;
            ends[nends++] = a; ends[nends++] = b;
        }
    for (int64_t i = m + 1; i < n; ++i) {
        int32_t got = 0;
        while (got < m) {
            int32_t t = ends[below(&st, (uint64_t)nends)];
            int dup = 0;
            for (int32_t j = 0; j < got; ++j) if (pick[j] == t) { dup = 1; break; }
            if (!dup) pick[got++] = t;
        }
        for (int32_t j = 0; j < m; ++j) {
            src[ne] = (int32_t)i; dst[ne] = pick[j]; ++ne;
            ends[nends++] = (int32_t)i; ends[nends++] = pick[j];
        }
    }
    free(ends); free(pick);
    return ne;
}

/*
 * Build a symmetric CSR from an undirected edge list: both directions are
 * inserted, self-loops dropped, duplicates merged, rows sorted ascending.
 * row has n+1 entries; col must hold 2*n_edges entries. Returns nnz or -1.
 */
static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

int64_t graphgen_csr(int64_t n, int64_t n_edges, const int32_t *src, const int32_t *dst,
                     int64_t *row, int32_t *col)
{
    int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!deg) return -1;
    for (int64_t e = 0; e < n_edges; ++e) {
        int32_t a = src[e], b = dst[e];
        if (a < 0 || b < 0 || a >= n || b >= n) { free(deg); return -1; }
        if (a == b) continue;
        deg[a]++; deg[b]++;
    }
    row[0] = 0;
    for (int64_t v = 0; v < n; ++v) row[v + 1] = row[v] + deg[v];
    for (int64_t v = 0; v < n; ++v) deg[v] = row[v];
    for (int64_t e = 0; e < n_edges; ++e) {
        int32_t a = src[e], b = dst[e];
        if (a == b) continue;
        col[deg[a]++] = b;
        col[deg[b]++] = a;
    }
    /* sort + unique each row, compacting in place */
    int64_t out = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t lo = row[v], hi = row[v + 1];
        qsort(col + lo, (size_t)(hi - lo), sizeof(int32_t), cmp_i32);
        int64_t start = out;
        for (int64_t e = lo; e < hi; ++e)
            if (e == lo || col[e] != col[e - 1]) col[out++] = col[e];
        row[v] = start;
    }
    row[n] = out;
    free(deg);
    return out;
}
