/*
 * CPU oracle for sampled betweenness centrality.
 *
 * TEST INFRASTRUCTURE ONLY: plain, slow, obviously correct. Only the tests,
 * the smoke check and the benchmark's CPU-baseline leg may call it; the GPU
 * library never links or loads it and shares no code with it.
 *
 * Paper: S. Ji and Z. Yan, "Refining Approximating Betweenness Centrality
 * Based on Samplings" (arXiv 1608.04472). Each function cites the passage it
 * follows. Readings of silent or ambiguous points:
 *   - unweighted graphs: the single-source shortest paths of Brandes' first
 *     step are a breadth-first search; weighted graphs (the *_weighted
 *     entry points): Dijkstra's algorithm, weights positive integers with
 *     max weight * (n - 1) < 2^30, so distances, their sums and ties are
 *     exact;
 *   - BC sums over ordered pairs (s, t), s, t, v pairwise distinct;
 *   - the predecessor condition of Definition 3 is read as "if and only if";
 *   - sampling is uniform with replacement over all n vertices (sources) or
 *     all n(n-1) ordered pairs of distinct vertices (pairs);
 *   - the loop runs while S <= c*n, so it stops at the first S > c*n, and the
 *     sample that crosses the threshold is counted.
 * Built with -ffp-contract=off: no fused multiply-add anywhere.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ Philox */

/* Philox4x64-10 as published by Salmon et al. (SC'11): ten rounds of two
 * 64x64->128 multiplies with the round keys bumped by the Weyl constants. */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, x0, &hi0, &lo0);
        mulhilo64(M1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0; k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static int64_t scale_draw(uint64_t w, int64_t range)
{
    unsigned __int128 p = (unsigned __int128)w * (uint64_t)range;
    return (int64_t)(p >> 64);
}

int32_t oracle_draw_source(uint64_t seed, int64_t j, int64_t n)
{
    uint64_t ctr[4] = {(uint64_t)j, 0, 0, 0}, key[2] = {seed, 0}, w[4];
    oracle_philox4x64_10(ctr, key, w);
    return (int32_t)scale_draw(w[0], n);
}

void oracle_draw_pair(uint64_t seed, int64_t j, int64_t n, int32_t *u, int32_t *v)
{
    uint64_t ctr[4] = {(uint64_t)j, 0, 0, 0}, key[2] = {seed, 1}, w[4];
    oracle_philox4x64_10(ctr, key, w);
    int64_t a = scale_draw(w[0], n);
    int64_t b = scale_draw(w[1], n - 1);
    if (b >= a) b += 1;
    *u = (int32_t)a;
    *v = (int32_t)b;
}

/* ------------------------------------------- FP64 with unbounded exponent */

typedef struct { double m; int32_t e; } xnum;   /* m * 2^e; m == 0 or 1 <= m < 2 */

static xnum xnum_make(double m, int64_t e)
{
    xnum r = {0.0, 0};
    if (m == 0.0) return r;
    int k;
    double f = frexp(m, &k);            /* m = f * 2^k, 0.5 <= f < 1 */
    r.m = f * 2.0;
    r.e = (int32_t)(e + k - 1);
    return r;
}

static xnum xnum_add(xnum a, xnum b)
{
    if (a.m == 0.0) return b;
    if (b.m == 0.0) return a;
    int32_t e = a.e > b.e ? a.e : b.e;
    return xnum_make(ldexp(a.m, a.e - e) + ldexp(b.m, b.e - e), e);
}

static xnum xnum_mul(xnum a, xnum b)
{
    return xnum_make(a.m * b.m, (int64_t)a.e + b.e);
}

/* a / b as a plain double (may underflow to 0 or a subnormal). */
static double xnum_div(xnum a, xnum b)
{
    return ldexp(a.m / b.m, a.e - b.e);
}

/* ------------------------------------------------------------ Brandes pass */

/* A graph as a pass reads it: out-neighbour rows (the search and the
 * dependency sums follow edges forward) and in-neighbour rows (path counts
 * sum over predecessors, Definition 3). An undirected graph is its own
 * reverse: both pairs of arrays are the same. */
typedef struct {
    int64_t n;
    const int64_t *row;     /* out-neighbours */
    const int32_t *col;
    const int64_t *rrow;    /* in-neighbours */
    const int32_t *rcol;
    const int32_t *wt;      /* weights of the out-arcs (row/col order), or NULL */
    const int32_t *rwt;     /* weights of the in-arcs (rrow/rcol order), or NULL */
} graph_t;

static graph_t undirected(int64_t n, const int64_t *row, const int32_t *col)
{
    graph_t g = {n, row, col, row, col};
    return g;
}

/* the same graph with every edge reversed */
static graph_t reversed(const graph_t *g)
{
    graph_t r = {g->n, g->rrow, g->rcol, g->row, g->col};
    r.wt = g->rwt;
    r.rwt = g->wt;
    return r;
}

/* In-neighbour rows of a directed CSR (rows sorted ascending, as the out
 * rows are). Returns 0, or -2 when out of memory. */
static int transpose(int64_t n, const int64_t *row, const int32_t *col, int64_t **trow,
                     int32_t **tcol)
{
    const int64_t nnz = row[n];
    int64_t *tr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *tc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!tr || !tc || !fill) { free(tr); free(tc); free(fill); return -2; }
    for (int64_t e = 0; e < nnz; ++e) tr[col[e] + 1] += 1;
    for (int64_t v = 0; v < n; ++v) tr[v + 1] += tr[v];
    for (int64_t v = 0; v < n; ++v) fill[v] = tr[v];
    for (int64_t u = 0; u < n; ++u)          /* sources ascending: rows come out sorted */
        for (int64_t e = row[u]; e < row[u + 1]; ++e) tc[fill[col[e]]++] = (int32_t)u;
    free(fill);
    *trow = tr;
    *tcol = tc;
    return 0;
}

typedef struct {
    int32_t *dist;
    xnum *sig;
    double *delta;
    int32_t *order;     /* vertices in BFS order: non-decreasing distance */
    int64_t reached;
    /* weighted graphs: Dijkstra's heap of (distance, vertex) entries with
     * lazy deletion (one entry per improving relaxation: at most nnz + 1),
     * and the tentative distances */
    int64_t *hkey;
    int32_t *hval;
    int32_t *tent;
} pass_t;

static int pass_alloc(pass_t *p, int64_t n)
{
    p->dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    p->sig = (xnum *)malloc(sizeof(xnum) * (size_t)n);
    p->delta = (double *)malloc(sizeof(double) * (size_t)n);
    p->order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    p->reached = 0;
    p->hkey = NULL;
    p->hval = NULL;
    p->tent = NULL;
    return (p->dist && p->sig && p->delta && p->order) ? 0 : -1;
}

/* the heap and tentative distances of a weighted graph's passes */
static int pass_alloc_heap(pass_t *p, const graph_t *g)
{
    if (!g->wt) return 0;
    const size_t cap = (size_t)g->row[g->n] + 1;
    p->hkey = (int64_t *)malloc(sizeof(int64_t) * cap);
    p->hval = (int32_t *)malloc(sizeof(int32_t) * cap);
    p->tent = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->n);
    return (p->hkey && p->hval && p->tent) ? 0 : -1;
}

static void pass_free(pass_t *p)
{
    free(p->dist); free(p->sig); free(p->delta); free(p->order);
    free(p->hkey); free(p->hval); free(p->tent);
}

static int check_graph(int64_t n, const int64_t *row, const int32_t *col)
{
    return (n > 0 && n < 0x7fffffffLL && row && (col || row[n] == 0)) ? 0 : -1;
}

/* Brandes' first step for an unweighted graph: breadth-first search from s
 * along out-edges, giving d(s, .) and the visiting order. */
static void bfs(const graph_t *g, int32_t s, pass_t *p)
{
    const int64_t *row = g->row;
    const int32_t *col = g->col;
    for (int64_t v = 0; v < g->n; ++v) p->dist[v] = -1;
    int64_t head = 0, tail = 0;
    p->dist[s] = 0;
    p->order[tail++] = s;
    while (head < tail) {
        int32_t u = p->order[head++];
        for (int64_t e = row[u]; e < row[u + 1]; ++e) {
            int32_t w = col[e];
            if (p->dist[w] < 0) {
                p->dist[w] = p->dist[u] + 1;
                p->order[tail++] = w;
            }
        }
    }
    p->reached = tail;
}

/* sigma_sw = sum of sigma_su over the predecessors u of w (Definition 3:
 * in-neighbours with d(s,u) = d(s,w) - 1), in BFS order so that every
 * predecessor is final before it is read. */
static void path_counts(const graph_t *g, pass_t *p)
{
    const int64_t *row = g->rrow;
    const int32_t *col = g->rcol;
    for (int64_t v = 0; v < g->n; ++v) { p->sig[v].m = 0.0; p->sig[v].e = 0; }
    int32_t s = p->order[0];
    p->sig[s] = xnum_make(1.0, 0);
    for (int64_t i = 1; i < p->reached; ++i) {
        int32_t w = p->order[i];
        xnum acc = {0.0, 0};
        for (int64_t e = row[w]; e < row[w + 1]; ++e) {
            int32_t u = col[e];
            if (p->dist[u] == p->dist[w] - 1) acc = xnum_add(acc, p->sig[u]);
        }
        p->sig[w] = acc;
    }
}

/* Theorem 1: delta_s(v) = sum over t with v in P_s(t) (out-neighbours of v
 * one level further) of (sigma_sv / sigma_st) * (1 + delta_s(t)), evaluated
 * in non-increasing distance (Brandes' second step) so every successor t is
 * final. The source itself is excluded from its own dependency (s != t != v),
 * so delta_s(s) = 0. */
static void dependencies(const graph_t *g, pass_t *p)
{
    const int64_t *row = g->row;
    const int32_t *col = g->col;
    for (int64_t v = 0; v < g->n; ++v) p->delta[v] = 0.0;
    for (int64_t i = p->reached - 1; i >= 1; --i) {
        int32_t v = p->order[i];
        double acc = 0.0;
        for (int64_t e = row[v]; e < row[v + 1]; ++e) {
            int32_t t = col[e];
            if (p->dist[t] == p->dist[v] + 1) {
                double q = xnum_div(p->sig[v], p->sig[t]);
                double r = 1.0 + p->delta[t];
                acc += q * r;
            }
        }
        p->delta[v] = acc;
    }
}

/* ------------------------------------------------------- weighted graphs */

/* binary min-heap on (key, vertex) in hkey/hval, `size` entries */
static void heap_push(pass_t *p, int64_t *size, int64_t key, int32_t v)
{
    int64_t i = (*size)++;
    while (i > 0) {
        const int64_t up = (i - 1) / 2;
        if (p->hkey[up] <= key) break;
        p->hkey[i] = p->hkey[up];
        p->hval[i] = p->hval[up];
        i = up;
    }
    p->hkey[i] = key;
    p->hval[i] = v;
}

static void heap_pop(pass_t *p, int64_t *size, int64_t *key, int32_t *v)
{
    *key = p->hkey[0];
    *v = p->hval[0];
    const int64_t last = --(*size);
    const int64_t k = p->hkey[last];
    const int32_t x = p->hval[last];
    int64_t i = 0;
    for (;;) {
        int64_t c = 2 * i + 1;
        if (c >= last) break;
        if (c + 1 < last && p->hkey[c + 1] < p->hkey[c]) c += 1;
        if (p->hkey[c] >= k) break;
        p->hkey[i] = p->hkey[c];
        p->hval[i] = p->hval[c];
        i = c;
    }
    if (last > 0) {
        p->hkey[i] = k;
        p->hval[i] = x;
    }
}

/* Brandes' first step on a weighted graph (Section 3 names Dijkstra's
 * algorithm): vertices are settled in non-decreasing distance; a stale heap
 * entry (its vertex settled, or its key above the tentative distance) is
 * skipped. p->order lists the settled vertices in that order. */
static void dijkstra(const graph_t *g, int32_t s, pass_t *p)
{
    for (int64_t v = 0; v < g->n; ++v) { p->dist[v] = -1; p->tent[v] = -1; }
    int64_t size = 0;
    p->reached = 0;
    p->tent[s] = 0;
    heap_push(p, &size, 0, s);
    while (size > 0) {
        int64_t key;
        int32_t u;
        heap_pop(p, &size, &key, &u);
        if (p->dist[u] >= 0 || key != p->tent[u]) continue;
        p->dist[u] = (int32_t)key;
        p->order[p->reached++] = u;
        for (int64_t e = g->row[u]; e < g->row[u + 1]; ++e) {
            const int32_t w = g->col[e];
            const int32_t through = p->dist[u] + g->wt[e];
            if (p->dist[w] < 0 && (p->tent[w] < 0 || through < p->tent[w])) {
                p->tent[w] = through;
                heap_push(p, &size, through, w);
            }
        }
    }
}

/* Definition 3 with weights: u precedes w when the arc u->w lies on a
 * shortest path, d(s,u) + w(u,w) = d(s,w). Settled order puts every
 * predecessor (strictly closer: weights are positive) first. */
static void weighted_counts(const graph_t *g, pass_t *p)
{
    for (int64_t v = 0; v < g->n; ++v) { p->sig[v].m = 0.0; p->sig[v].e = 0; }
    p->sig[p->order[0]] = xnum_make(1.0, 0);
    for (int64_t i = 1; i < p->reached; ++i) {
        const int32_t w = p->order[i];
        xnum sum = {0.0, 0};
        for (int64_t e = g->rrow[w]; e < g->rrow[w + 1]; ++e) {
            const int32_t u = g->rcol[e];
            if (p->dist[u] >= 0 && p->dist[u] + g->rwt[e] == p->dist[w])
                sum = xnum_add(sum, p->sig[u]);
        }
        p->sig[w] = sum;
    }
}

/* Theorem 1 with weights: the successors of v are the heads t of arcs
 * v->t with d(s,v) + w(v,t) = d(s,t); reverse settled order; delta_s(s) = 0. */
static void weighted_dependencies(const graph_t *g, pass_t *p)
{
    for (int64_t v = 0; v < g->n; ++v) p->delta[v] = 0.0;
    for (int64_t i = p->reached - 1; i > 0; --i) {
        const int32_t v = p->order[i];
        double sum = 0.0;
        for (int64_t e = g->row[v]; e < g->row[v + 1]; ++e) {
            const int32_t t = g->col[e];
            if (p->dist[v] + g->wt[e] == p->dist[t])
                sum += xnum_div(p->sig[v], p->sig[t]) * (1.0 + p->delta[t]);
        }
        p->delta[v] = sum;
    }
}

static void brandes_pass(const graph_t *g, int32_t s, pass_t *p)
{
    if (g->wt) {
        dijkstra(g, s, p);
        weighted_counts(g, p);
        weighted_dependencies(g, p);
        return;
    }
    bfs(g, s, p);
    path_counts(g, p);
    dependencies(g, p);
}

static int brandes_g(const graph_t *g, int32_t s, int32_t *dist, double *sig_m, int32_t *sig_e,
                     double *delta)
{
    if (s < 0 || s >= g->n) return -1;
    pass_t p;
    if (pass_alloc(&p, g->n) | pass_alloc_heap(&p, g)) { pass_free(&p); return -2; }
    brandes_pass(g, s, &p);
    for (int64_t v = 0; v < g->n; ++v) {
        if (dist) dist[v] = p.dist[v];
        if (sig_m) sig_m[v] = p.sig[v].m;
        if (sig_e) sig_e[v] = p.sig[v].e;
        if (delta) delta[v] = p.delta[v];
    }
    pass_free(&p);
    return 0;
}

/* Exact BC as the sum of source dependencies (Section 3). */
static int bc_exact_g(const graph_t *g, double *bc)
{
    if (!bc) return -1;
    pass_t p;
    if (pass_alloc(&p, g->n) | pass_alloc_heap(&p, g)) { pass_free(&p); return -2; }
    for (int64_t v = 0; v < g->n; ++v) bc[v] = 0.0;
    for (int64_t s = 0; s < g->n; ++s) {
        brandes_pass(g, (int32_t)s, &p);
        for (int64_t v = 0; v < g->n; ++v) bc[v] += p.delta[v];
    }
    pass_free(&p);
    return 0;
}

static int dependencies_g(const graph_t *g, const int32_t *sources, int64_t k, double *full,
                          double *sum)
{
    const int64_t n = g->n;
    if (k < 0 || (k > 0 && !sources)) return -1;
    for (int64_t i = 0; i < k; ++i)
        if (sources[i] < 0 || sources[i] >= n) return -1;
    pass_t p;
    if (pass_alloc(&p, n) | pass_alloc_heap(&p, g)) { pass_free(&p); return -2; }
    if (sum) for (int64_t v = 0; v < n; ++v) sum[v] = 0.0;
    for (int64_t i = 0; i < k; ++i) {
        brandes_pass(g, sources[i], &p);
        for (int64_t v = 0; v < n; ++v) {
            if (full) full[i * n + v] = p.delta[v];
            if (sum) sum[v] += p.delta[v];
        }
    }
    pass_free(&p);
    return 0;
}

/* -------------------------------------------------------- pair dependency */

/* pu: search from u; pv: search from v over reversed edges, so pv->dist[t] =
 * d(t, v) and pv->sig[t] = sigma_tv. */
static void pair_from_passes(int64_t n, int32_t u, int32_t v, const pass_t *pu,
                             const pass_t *pv, double *y)
{
    for (int64_t t = 0; t < n; ++t) y[t] = 0.0;
    int32_t duv = pu->dist[v];
    if (duv < 0) return;
    for (int64_t t = 0; t < n; ++t) {
        if (t == u || t == v) continue;
        if (pu->dist[t] < 0 || pv->dist[t] < 0) continue;
        if (pu->dist[t] + pv->dist[t] != duv) continue;
        xnum through = xnum_mul(pu->sig[t], pv->sig[t]);
        y[t] = xnum_div(through, pu->sig[v]);
    }
}

static void sssp_counts(const graph_t *g, int32_t s, pass_t *p)
{
    if (g->wt) {
        dijkstra(g, s, p);
        weighted_counts(g, p);
        return;
    }
    bfs(g, s, p);
    path_counts(g, p);
}

static int pair_dependency_g(const graph_t *g, int32_t u, int32_t v, double *y)
{
    const int64_t n = g->n;
    if (!y || u < 0 || v < 0 || u >= n || v >= n || u == v) return -1;
    const graph_t r = reversed(g);
    pass_t pu, pv;
    int bad = pass_alloc(&pu, n) | pass_alloc(&pv, n) | pass_alloc_heap(&pu, g) |
              pass_alloc_heap(&pv, &r);
    if (bad) { pass_free(&pu); pass_free(&pv); return -2; }
    sssp_counts(g, u, &pu);
    sssp_counts(&r, v, &pv);
    pair_from_passes(n, u, v, &pu, &pv, y);
    pass_free(&pu); pass_free(&pv);
    return 0;
}

/* ---------------------------------------------------------------- samplers */

enum { ST_RUNNING = 255, ST_DONE = 0, ST_CAPPED = 1 };

/* Section 4, Bader's loop as restated in the paper: S starts at 0; each
 * iteration samples a vertex, runs the shortest paths from it and adds its
 * dependency on the target; the loop repeats while S <= c*n; the estimate
 * is n*S/k. Targets share the sample stream, so one pass per draw serves all
 * targets that are still running. */
static int adaptive_source_g(const graph_t *g, const int32_t *targets, int32_t T, double c,
                             uint64_t seed, int64_t k_max, double *est, int64_t *samples,
                             double *S, uint8_t *status)
{
    const int64_t n = g->n;
    if (T < 0 || (T > 0 && !targets) || !(c >= 1.0) || k_max < 1 || !est || !samples || !S ||
        !status)
        return -1;
    for (int32_t i = 0; i < T; ++i)
        if (targets[i] < 0 || targets[i] >= n) return -1;
    pass_t p;
    if (pass_alloc(&p, n) | pass_alloc_heap(&p, g)) { pass_free(&p); return -2; }
    const double threshold = c * (double)n;
    for (int32_t i = 0; i < T; ++i) { S[i] = 0.0; samples[i] = 0; status[i] = ST_RUNNING; }
    int32_t running = T;
    for (int64_t j = 0; running > 0; ++j) {
        int32_t s = oracle_draw_source(seed, j, n);
        brandes_pass(g, s, &p);
        for (int32_t i = 0; i < T; ++i) {
            if (status[i] != ST_RUNNING) continue;
            S[i] += p.delta[targets[i]];
            samples[i] += 1;
            if (S[i] > threshold) { status[i] = ST_DONE; --running; }
            else if (samples[i] == k_max) { status[i] = ST_CAPPED; --running; }
        }
    }
    for (int32_t i = 0; i < T; ++i) est[i] = ((double)n * S[i]) / (double)samples[i];
    pass_free(&p);
    return 0;
}

/* Algorithm 1: pick an ordered pair of distinct vertices, count the share of
 * its shortest paths through the target, add it to S, count the sample.
 * Rule 0 keeps the loop's literal condition (repeat while S <= c*n). Rule 1
 * stops once k reaches Lemma 5's sample count eps*(n^2(n-1)/A)^(2/3) with A
 * read as the running estimate n(n-1)S/k, which rearranges to
 * k*S^2 >= eps^3*n^2. */
static int adaptive_pair_g(const graph_t *g, const int32_t *targets, int32_t T, int rule,
                           double eps, double c, uint64_t seed, int64_t k_max, double *est,
                           int64_t *samples, double *S, uint8_t *status)
{
    const int64_t n = g->n;
    if (n < 2 || T < 0 || (T > 0 && !targets) || k_max < 1 || !est || !samples || !S || !status)
        return -1;
    if (rule == 0 && !(c >= 1.0)) return -1;
    if (rule == 1 && !(eps > 0.0 && eps < 0.5)) return -1;
    if (rule != 0 && rule != 1) return -1;
    for (int32_t i = 0; i < T; ++i)
        if (targets[i] < 0 || targets[i] >= n) return -1;
    const graph_t r = reversed(g);
    pass_t pu, pv;
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    int bad = pass_alloc(&pu, n) | pass_alloc(&pv, n) | pass_alloc_heap(&pu, g) |
              pass_alloc_heap(&pv, &r);
    if (bad || !y) { pass_free(&pu); pass_free(&pv); free(y); return -2; }
    const double threshold = c * (double)n;
    const double eps_rhs = ((eps * eps) * eps) * ((double)n * (double)n);
    for (int32_t i = 0; i < T; ++i) { S[i] = 0.0; samples[i] = 0; status[i] = ST_RUNNING; }
    int32_t running = T;
    for (int64_t j = 0; running > 0; ++j) {
        int32_t u, v;
        oracle_draw_pair(seed, j, n, &u, &v);
        sssp_counts(g, u, &pu);
        sssp_counts(&r, v, &pv);
        pair_from_passes(n, u, v, &pu, &pv, y);
        for (int32_t i = 0; i < T; ++i) {
            if (status[i] != ST_RUNNING) continue;
            S[i] += y[targets[i]];
            samples[i] += 1;
            int stop;
            if (rule == 0) stop = S[i] > threshold;
            else stop = S[i] > 0.0 && ((double)samples[i] * (S[i] * S[i])) >= eps_rhs;
            if (stop) { status[i] = ST_DONE; --running; }
            else if (samples[i] == k_max) { status[i] = ST_CAPPED; --running; }
        }
    }
    const double pairs = (double)n * (double)(n - 1);
    for (int32_t i = 0; i < T; ++i) est[i] = (pairs * S[i]) / (double)samples[i];
    pass_free(&pu); pass_free(&pv); free(y);
    return 0;
}

/* ------------------------------------------------- undirected entry points */

int oracle_brandes(int64_t n, const int64_t *row, const int32_t *col, int32_t s,
                   int32_t *dist, double *sig_m, int32_t *sig_e, double *delta)
{
    if (check_graph(n, row, col)) return -1;
    const graph_t g = undirected(n, row, col);
    return brandes_g(&g, s, dist, sig_m, sig_e, delta);
}

int oracle_bc_exact(int64_t n, const int64_t *row, const int32_t *col, double *bc)
{
    if (check_graph(n, row, col)) return -1;
    const graph_t g = undirected(n, row, col);
    return bc_exact_g(&g, bc);
}

int oracle_dependencies(int64_t n, const int64_t *row, const int32_t *col,
                        const int32_t *sources, int64_t k, double *full, double *sum)
{
    if (check_graph(n, row, col)) return -1;
    const graph_t g = undirected(n, row, col);
    return dependencies_g(&g, sources, k, full, sum);
}

int oracle_pair_dependency(int64_t n, const int64_t *row, const int32_t *col,
                           int32_t u, int32_t v, double *y)
{
    if (check_graph(n, row, col)) return -1;
    const graph_t g = undirected(n, row, col);
    return pair_dependency_g(&g, u, v, y);
}

int oracle_adaptive_source(int64_t n, const int64_t *row, const int32_t *col,
                           const int32_t *targets, int32_t T, double c, uint64_t seed,
                           int64_t k_max, double *est, int64_t *samples, double *S,
                           uint8_t *status)
{
    if (check_graph(n, row, col)) return -1;
    const graph_t g = undirected(n, row, col);
    return adaptive_source_g(&g, targets, T, c, seed, k_max, est, samples, S, status);
}

int oracle_adaptive_pair(int64_t n, const int64_t *row, const int32_t *col,
                         const int32_t *targets, int32_t T, int rule, double eps, double c,
                         uint64_t seed, int64_t k_max, double *est, int64_t *samples,
                         double *S, uint8_t *status)
{
    if (check_graph(n, row, col)) return -1;
    const graph_t g = undirected(n, row, col);
    return adaptive_pair_g(&g, targets, T, rule, eps, c, seed, k_max, est, samples, S, status);
}

/* --------------------------------------------------- directed entry points
 * row/col hold out-neighbours; the in-neighbour rows are built here. */

#define WITH_DIRECTED(n, row, col, CALL)                                           \
    do {                                                                           \
        if (check_graph(n, row, col)) return -1;                                   \
        int64_t *trow_ = NULL;                                                     \
        int32_t *tcol_ = NULL;                                                     \
        if (transpose(n, row, col, &trow_, &tcol_)) return -2;                     \
        const graph_t g = {n, row, col, trow_, tcol_};                             \
        const int rc_ = (CALL);                                                    \
        free(trow_);                                                               \
        free(tcol_);                                                               \
        return rc_;                                                                \
    } while (0)

int oracle_brandes_directed(int64_t n, const int64_t *row, const int32_t *col, int32_t s,
                            int32_t *dist, double *sig_m, int32_t *sig_e, double *delta)
{
    WITH_DIRECTED(n, row, col, brandes_g(&g, s, dist, sig_m, sig_e, delta));
}

int oracle_bc_exact_directed(int64_t n, const int64_t *row, const int32_t *col, double *bc)
{
    WITH_DIRECTED(n, row, col, bc_exact_g(&g, bc));
}

int oracle_dependencies_directed(int64_t n, const int64_t *row, const int32_t *col,
                                 const int32_t *sources, int64_t k, double *full, double *sum)
{
    WITH_DIRECTED(n, row, col, dependencies_g(&g, sources, k, full, sum));
}

int oracle_pair_dependency_directed(int64_t n, const int64_t *row, const int32_t *col,
                                    int32_t u, int32_t v, double *y)
{
    WITH_DIRECTED(n, row, col, pair_dependency_g(&g, u, v, y));
}

int oracle_adaptive_source_directed(int64_t n, const int64_t *row, const int32_t *col,
                                    const int32_t *targets, int32_t T, double c, uint64_t seed,
                                    int64_t k_max, double *est, int64_t *samples, double *S,
                                    uint8_t *status)
{
    WITH_DIRECTED(n, row, col,
                  adaptive_source_g(&g, targets, T, c, seed, k_max, est, samples, S, status));
}

int oracle_adaptive_pair_directed(int64_t n, const int64_t *row, const int32_t *col,
                                  const int32_t *targets, int32_t T, int rule, double eps,
                                  double c, uint64_t seed, int64_t k_max, double *est,
                                  int64_t *samples, double *S, uint8_t *status)
{
    WITH_DIRECTED(n, row, col, adaptive_pair_g(&g, targets, T, rule, eps, c, seed, k_max, est,
                                               samples, S, status));
}

/* --------------------------------------------------- weighted entry points
 * wt[e]: the weight of arc e of row/col, a positive integer with
 * max weight * (n - 1) < 2^30. directed = 0: an undirected CSR whose two
 * arcs of an edge carry equal weights; directed != 0: out-neighbour rows,
 * the in-neighbour rows and their weights built here. */

static int check_weights(int64_t n, const int64_t *row, const int32_t *col, const int32_t *wt,
                         int directed)
{
    if (!wt && row[n] > 0) return -1;
    int32_t most = 0;
    for (int64_t e = 0; e < row[n]; ++e) {
        if (wt[e] <= 0) return -1;
        if (wt[e] > most) most = wt[e];
    }
    if ((int64_t)most * (n - 1) >= (1ll << 30)) return -1;
    if (directed) return 0;
    for (int64_t u = 0; u < n; ++u)
        for (int64_t e = row[u]; e < row[u + 1]; ++e) {
            const int32_t v = col[e];
            int64_t f = row[v];
            while (f < row[v + 1] && col[f] != u) ++f;
            if (f == row[v + 1] || wt[f] != wt[e]) return -1;
        }
    return 0;
}

/* weights of the in-neighbour rows that transpose() builds, in its order */
static int transpose_weights(int64_t n, const int64_t *row, const int32_t *col,
                             const int32_t *wt, const int64_t *trow, int32_t **twt)
{
    const int64_t nnz = row[n];
    int32_t *tw = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!tw || !next) { free(tw); free(next); return -2; }
    for (int64_t v = 0; v < n; ++v) next[v] = trow[v];
    for (int64_t u = 0; u < n; ++u)
        for (int64_t e = row[u]; e < row[u + 1]; ++e) tw[next[col[e]]++] = wt[e];
    free(next);
    *twt = tw;
    return 0;
}

#define WITH_WEIGHTS(n, row, col, wt, directed, CALL)                              \
    do {                                                                           \
        if (check_graph(n, row, col) || check_weights(n, row, col, wt, directed))  \
            return -1;                                                             \
        int64_t *trow_ = NULL;                                                     \
        int32_t *tcol_ = NULL, *twt_ = NULL;                                       \
        graph_t g = {n, row, col, row, col, wt, wt};                               \
        if (directed) {                                                            \
            if (transpose(n, row, col, &trow_, &tcol_)) return -2;                 \
            if (transpose_weights(n, row, col, wt, trow_, &twt_)) {                \
                free(trow_);                                                       \
                free(tcol_);                                                       \
                return -2;                                                         \
            }                                                                      \
            g.rrow = trow_;                                                        \
            g.rcol = tcol_;                                                        \
            g.rwt = twt_;                                                          \
        }                                                                          \
        const int rc_ = (CALL);                                                    \
        free(trow_);                                                               \
        free(tcol_);                                                               \
        free(twt_);                                                                \
        return rc_;                                                                \
    } while (0)

int oracle_brandes_weighted(int64_t n, const int64_t *row, const int32_t *col,
                            const int32_t *wt, int directed, int32_t s, int32_t *dist,
                            double *sig_m, int32_t *sig_e, double *delta)
{
    WITH_WEIGHTS(n, row, col, wt, directed, brandes_g(&g, s, dist, sig_m, sig_e, delta));
}

int oracle_bc_exact_weighted(int64_t n, const int64_t *row, const int32_t *col,
                             const int32_t *wt, int directed, double *bc)
{
    WITH_WEIGHTS(n, row, col, wt, directed, bc_exact_g(&g, bc));
}

int oracle_dependencies_weighted(int64_t n, const int64_t *row, const int32_t *col,
                                 const int32_t *wt, int directed, const int32_t *sources,
                                 int64_t k, double *full, double *sum)
{
    WITH_WEIGHTS(n, row, col, wt, directed, dependencies_g(&g, sources, k, full, sum));
}

int oracle_pair_dependency_weighted(int64_t n, const int64_t *row, const int32_t *col,
                                    const int32_t *wt, int directed, int32_t u, int32_t v,
                                    double *y)
{
    WITH_WEIGHTS(n, row, col, wt, directed, pair_dependency_g(&g, u, v, y));
}

int oracle_adaptive_source_weighted(int64_t n, const int64_t *row, const int32_t *col,
                                    const int32_t *wt, int directed, const int32_t *targets,
                                    int32_t T, double c, uint64_t seed, int64_t k_max,
                                    double *est, int64_t *samples, double *S, uint8_t *status)
{
    WITH_WEIGHTS(n, row, col, wt, directed,
                 adaptive_source_g(&g, targets, T, c, seed, k_max, est, samples, S, status));
}

int oracle_adaptive_pair_weighted(int64_t n, const int64_t *row, const int32_t *col,
                                  const int32_t *wt, int directed, const int32_t *targets,
                                  int32_t T, int rule, double eps, double c, uint64_t seed,
                                  int64_t k_max, double *est, int64_t *samples, double *S,
                                  uint8_t *status)
{
    WITH_WEIGHTS(n, row, col, wt, directed,
                 adaptive_pair_g(&g, targets, T, rule, eps, c, seed, k_max, est, samples, S,
                                 status));
}

/* ------------------------------------------------------------ work counts */

int oracle_source_work(int64_t n, const int64_t *row, const int32_t *col, int32_t s,
                       int64_t *reached, int64_t *edges_undirected, int64_t *dag_edges)
{
    if (check_graph(n, row, col) || s < 0 || s >= n) return -1;
    pass_t p;
    if (pass_alloc(&p, n)) { pass_free(&p); return -2; }
    const graph_t g = undirected(n, row, col);
    bfs(&g, s, &p);
    int64_t deg = 0, dag = 0;
    for (int64_t i = 0; i < p.reached; ++i) {
        int32_t u = p.order[i];
        deg += row[u + 1] - row[u];
        for (int64_t e = row[u]; e < row[u + 1]; ++e)
            if (p.dist[col[e]] == p.dist[u] + 1) ++dag;
    }
    if (reached) *reached = p.reached;
    if (edges_undirected) *edges_undirected = deg / 2;
    if (dag_edges) *dag_edges = dag;
    pass_free(&p);
    return 0;
}

int oracle_pair_work(int64_t n, const int64_t *row, const int32_t *col, int32_t u, int32_t v,
                     int64_t *edges_undirected)
{
    if (check_graph(n, row, col) || u < 0 || v < 0 || u >= n || v >= n || u == v) return -1;
    pass_t p;
    if (pass_alloc(&p, n)) { pass_free(&p); return -2; }
    const graph_t g = undirected(n, row, col);
    bfs(&g, u, &p);
    int32_t limit = p.dist[v] < 0 ? 0x7fffffff : p.dist[v];
    int64_t cnt = 0;
    for (int64_t i = 0; i < p.reached; ++i) {
        int32_t a = p.order[i];
        for (int64_t e = row[a]; e < row[a + 1]; ++e) {
            int32_t b = col[e];
            int32_t da = p.dist[a], db = p.dist[b];
            /* count each undirected edge once, from its lower-distance end
             * (ties: lower id) when that end lies below the limit */
            int lead = (da < db) || (da == db && a < b);
            if (lead && da < limit) ++cnt;
        }
    }
    *edges_undirected = cnt;
    pass_free(&p);
    return 0;
}

/* Work of the two-sided pair search, counted over the walks the library's
 * search takes. Section 6.2 stops a pair's search once the destination is
 * reached; growing it from both ends in this balanced order is the
 * library's design, not the paper's, and this count is a measurement check
 * only. The rules, step by step:
 *   - side 0 grows from u over out-arcs, side 1 from v over in-arcs; each
 *     step the side whose frontier has fewer arcs to walk (side 0 on ties)
 *     walks every arc of its frontier, adding each vertex it had not held as
 *     its next level; the step meets the other side when any arc's head is
 *     held by the other side;
 *   - a step also reads, over the other direction, the row of each vertex it
 *     added (after a meeting step: only those the other side holds);
 *   - the search ends without a meeting when the chosen side has no arcs to
 *     walk or adds no vertex;
 *   - after a meeting, with D the sum of the two depths, side 0's levels and
 *     then side 1's are swept from the deepest up: at level L, every vertex
 *     of level L+1 that the other side holds at distance D-L-1 reads its row
 *     over the other direction and gives each neighbour of this side's level
 *     L the other side's distance D-L; then every level-L vertex the other
 *     side now holds at D-L reads its row over this side's direction.
 * found = vertices the steps add (the two ends excluded); arcs = the arcs of
 * every row read. */
static int bidir_work_g(const graph_t *g, int32_t u, int32_t v, int64_t *found, int64_t *arcs)
{
    const int64_t n = g->n;
    const int64_t *row[2] = {g->row, g->rrow};
    const int32_t *col[2] = {g->col, g->rcol};
    int32_t *dist[2] = {NULL, NULL}, *list[2] = {NULL, NULL};
    int64_t *lo[2] = {NULL, NULL};
    int rc = 0;
    for (int s = 0; s < 2; ++s) {
        dist[s] = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        list[s] = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        lo[s] = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 2));
        if (!dist[s] || !list[s] || !lo[s]) rc = -2;
    }
    if (rc == 0) {
        for (int s = 0; s < 2; ++s)
            for (int64_t x = 0; x < n; ++x) dist[s][x] = -1;
        const int32_t end[2] = {u, v};
        int depth[2] = {0, 0};
        int64_t f0[2] = {0, 0}, f1[2] = {1, 1}, vol[2];
        for (int s = 0; s < 2; ++s) {
            dist[s][end[s]] = 0;
            list[s][0] = end[s];
            lo[s][0] = 0;
            lo[s][1] = 1;
            vol[s] = row[s][end[s] + 1] - row[s][end[s]];
        }
        int64_t nf = 0, na = 0;
        int met = 0;
        for (;;) {
            const int s = vol[0] <= vol[1] ? 0 : 1, o = 1 - s;
            if (vol[s] == 0) break;
            int meet = 0;
            int64_t put = f1[s], cnt = 0, nv = 0;
            for (int64_t i = f0[s]; i < f1[s]; ++i) {
                const int32_t x = list[s][i];
                na += row[s][x + 1] - row[s][x];
                for (int64_t e = row[s][x]; e < row[s][x + 1]; ++e) {
                    const int32_t y = col[s][e];
                    if (dist[s][y] < 0) {
                        dist[s][y] = depth[s] + 1;
                        list[s][put + cnt++] = y;
                        nv += row[s][y + 1] - row[s][y];
                        ++nf;
                    }
                    if (dist[o][y] >= 0) meet = 1;
                }
            }
            vol[s] = nv;
            if (cnt == 0) break;
            depth[s] += 1;
            f0[s] = put;
            f1[s] = put + cnt;
            lo[s][depth[s] + 1] = put + cnt;
            for (int64_t i = put; i < put + cnt; ++i) {
                const int32_t w = list[s][i];
                if (!meet || dist[o][w] >= 0) na += row[o][w + 1] - row[o][w];
            }
            if (meet) {
                met = 1;
                break;
            }
        }
        if (met) {
            const int D = depth[0] + depth[1];
            for (int s = 0; s < 2; ++s) {
                const int o = 1 - s;
                for (int L = depth[s] - 1; L >= 0; --L) {
                    for (int64_t i = lo[s][L + 1]; i < lo[s][L + 2]; ++i) {
                        const int32_t x = list[s][i];
                        if (dist[o][x] != D - L - 1) continue;
                        na += row[o][x + 1] - row[o][x];
                        for (int64_t e = row[o][x]; e < row[o][x + 1]; ++e)
                            if (dist[s][col[o][e]] == L) dist[o][col[o][e]] = D - L;
                    }
                    for (int64_t i = lo[s][L]; i < lo[s][L + 1]; ++i) {
                        const int32_t w = list[s][i];
                        if (dist[o][w] == D - L) na += row[s][w + 1] - row[s][w];
                    }
                }
            }
        }
        *found = nf;
        *arcs = na;
    }
    for (int s = 0; s < 2; ++s) {
        free(dist[s]);
        free(list[s]);
        free(lo[s]);
    }
    return rc;
}

int oracle_bidir_work(int64_t n, const int64_t *row, const int32_t *col, int directed, int32_t u,
                      int32_t v, int64_t *found, int64_t *arcs)
{
    if (check_graph(n, row, col) || u < 0 || v < 0 || u >= n || v >= n || u == v) return -1;
    if (!directed) {
        const graph_t g = undirected(n, row, col);
        return bidir_work_g(&g, u, v, found, arcs);
    }
    WITH_DIRECTED(n, row, col, bidir_work_g(&g, u, v, found, arcs));
}
