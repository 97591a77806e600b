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
 * R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004): each of the
 * edge_factor * 2^scale edges picks, bit by bit from the top, one of the four
 * quadrants with probabilities a, b, c, 1-a-b-c (no noise, no relabelling).
 * Quadrant b sets the column bit, c the row bit, d both.
 */
int64_t graphgen_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c,
                      uint64_t seed, int32_t *src, int32_t *dst)
{
    if (scale < 1 || scale > 30 || edge_factor < 1) return -1;
    const int64_t ne = (int64_t)edge_factor << scale;
    uint64_t st = seed;
    /* quadrant thresholds on a 32-bit uniform draw (two draws per 64-bit word) */
    const uint64_t ta = (uint64_t)(a * 4294967296.0);
    const uint64_t tab = (uint64_t)((a + b) * 4294967296.0);
    const uint64_t tabc = (uint64_t)((a + b + c) * 4294967296.0);
    for (int64_t e = 0; e < ne; ++e) {
        uint32_t r = 0, q = 0;
        uint64_t word = 0;
        for (int32_t bit = scale - 1, k = 0; bit >= 0; --bit, ++k) {
            if ((k & 1) == 0) word = splitmix64_next(&st);
            const uint64_t u = (k & 1) ? (word >> 32) : (word & 0xffffffffULL);
            const uint32_t down = u >= tab;
            const uint32_t right = (u >= ta && u < tab) || u >= tabc;
            r |= down << bit;
            q |= right << bit;
        }
        src[e] = (int32_t)r;
        dst[e] = (int32_t)q;
    }
    return ne;
}

/*
 * Build a symmetric CSR from an undirected edge list: both directions are
 * inserted, self-loops dropped, duplicates merged, rows sorted ascending.
 * Two stable counting-sort passes (by neighbour, then by row) order the
 * directed entries; equal neighbours of a row become adjacent and are merged.
 * row has n+1 entries; col must hold 2*n_edges entries. Returns nnz or -1.
 */
int64_t graphgen_csr(int64_t n, int64_t n_edges, const int32_t *src, const int32_t *dst,
                     int64_t *row, int32_t *col)
{
    int64_t d = 0;
    for (int64_t e = 0; e < n_edges; ++e) {
        int32_t a = src[e], b = dst[e];
        if (a < 0 || b < 0 || a >= n || b >= n) return -1;
        if (a != b) d += 2;
    }
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *ra = (int32_t *)malloc(sizeof(int32_t) * (size_t)(d ? d : 1));
    int32_t *rb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(d ? d : 1));
    if (!cnt || !ra || !rb) { free(cnt); free(ra); free(rb); return -1; }
    /* pass 1: bucket the directed entries (a -> b) by b */
    for (int64_t e = 0; e < n_edges; ++e) {
        int32_t a = src[e], b = dst[e];
        if (a == b) continue;
        cnt[b + 1]++;
        cnt[a + 1]++;
    }
    for (int64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
    for (int64_t e = 0; e < n_edges; ++e) {
        int32_t a = src[e], b = dst[e];
        if (a == b) continue;
        int64_t p = cnt[b]++;
        ra[p] = a; rb[p] = b;
        p = cnt[a]++;
        ra[p] = b; rb[p] = a;
    }
    /* pass 2: stable bucket by a; entries of a row come out ordered by b */
    memset(cnt, 0, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t i = 0; i < d; ++i) cnt[ra[i] + 1]++;
    for (int64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
    for (int64_t i = 0; i < d; ++i) col[cnt[ra[i]]++] = rb[i];
    /* cnt[v] now holds the end of row v; merge duplicates in place */
    int64_t out = 0, lo = 0;
    for (int64_t v = 0; v < n; ++v) {
        const int64_t hi = cnt[v];
        row[v] = out;
        for (int64_t i = lo; i < hi; ++i)
            if (i == lo || col[i] != col[i - 1]) col[out++] = col[i];
        lo = hi;
    }
    row[n] = out;
    free(cnt); free(ra); free(rb);
    return out;
}
