/*
 * CPU oracle for sampled betweenness centrality (Ji and Yan, "Refining
 * Approximating Betweenness Centrality Based on Samplings").
 *
 * TEST INFRASTRUCTURE ONLY. Plain, slow, obviously correct C used to check the
 * GPU library; it shares no code, header, table or constant with it. Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may call it.
 *
 * Graph: undirected, unweighted, symmetric CSR (row: int64[n+1], col:
 * int32[nnz], rows sorted ascending, no self-loops or duplicates).
 *
 * Arithmetic: IEEE FP64, round to nearest even, built without FMA contraction.
 * Shortest-path counts use an FP64 significand with an unbounded int32
 * exponent (value = m * 2^e, m = 0 or 1 <= m < 2), identical to plain FP64
 * while below 2^1024. All neighbour sums run in ascending CSR order.
 *
 * Every function returns 0 on success and a negative value on bad arguments
 * or allocation failure.
 */
#ifndef BC_ORACLE_H
#define BC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x64 with 10 rounds (Salmon, Moraes, Dror and Shaw, SC'11). */
void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* One Brandes pass from source s (Section 3: BFS for the unweighted shortest
 * paths, then the dependency recursion of Theorem 1 in non-increasing
 * distance). Any output pointer may be NULL.
 *   dist[v]  : hop distance, -1 if unreachable
 *   sig_m/e  : sigma_sv = sig_m[v] * 2^sig_e[v] (0 if unreachable)
 *   delta[v] : delta_{s.}(v) (Definition 2); delta[s] = 0 and 0 if unreachable */
int oracle_brandes(int64_t n, const int64_t *row, const int32_t *col, int32_t s,
                   int32_t *dist, double *sig_m, int32_t *sig_e, double *delta);

/* Exact BC over ordered pairs (Definition 1): bc[v] = sum over s != v of
 * delta_{s.}(v), s ascending. */
int oracle_bc_exact(int64_t n, const int64_t *row, const int32_t *col, double *bc);

/* Dependencies of a source list. full (k*n, source-major) and sum (n, the sum
 * over the list in list order) may each be NULL. */
int oracle_dependencies(int64_t n, const int64_t *row, const int32_t *col,
                        const int32_t *sources, int64_t k, double *full, double *sum);

/* Pair dependency of every vertex on the pair (u, v), u != v (Algorithm 1):
 * y[t] = sigma_uv(t) / sigma_uv, with y[u] = y[v] = 0 and y = 0 everywhere if v
 * is unreachable from u. Computed from its definition: a shortest u-v path
 * passes t iff d(u,t) + d(t,v) = d(u,v), and then sigma_uv(t) =
 * sigma_ut * sigma_tv. */
int oracle_pair_dependency(int64_t n, const int64_t *row, const int32_t *col,
                           int32_t u, int32_t v, double *y);

/* Sample draws (key = (seed, stream), counter = (j, 0, 0, 0)):
 *   source j : floor(w0 * n / 2^64), stream 0
 *   pair j   : u = floor(w0 * n / 2^64), v' = floor(w1 * (n-1) / 2^64),
 *              v = v' + (v' >= u), stream 1 */
int32_t oracle_draw_source(uint64_t seed, int64_t j, int64_t n);
void oracle_draw_pair(uint64_t seed, int64_t j, int64_t n, int32_t *u, int32_t *v);

/* Adaptive source sampling (Section 4), T targets sharing one sample stream.
 * Per target: S += delta_{s_k}(v); k += 1; stop at the first k with
 * S > c*n (DONE) or at k = k_max (CAPPED). est = (n*S)/k.
 * Requires c >= 1, k_max >= 1, 0 <= targets[i] < n. */
int oracle_adaptive_source(int64_t n, const int64_t *row, const int32_t *col,
                           const int32_t *targets, int32_t T, double c, uint64_t seed,
                           int64_t k_max, double *est, int64_t *samples, double *S,
                           uint8_t *status);

/* Adaptive pair sampling (Algorithm 1), T targets sharing one stream.
 * Per target: S += sigma_uv(t)/sigma_uv; k += 1; stop rule:
 *   rule 0 (literal Algorithm 1): S > c*n
 *   rule 1 (epsilon): S > 0 and k*S*S >= eps^3 * n^2, the sample count of
 *          Lemma 5 with BC replaced by the running estimate
 * or k = k_max (CAPPED). est = (n*(n-1))*S/k.
 * Requires c >= 1 (rule 0), 0 < eps < 1/2 (rule 1), n >= 2. */
int oracle_adaptive_pair(int64_t n, const int64_t *row, const int32_t *col,
                         const int32_t *targets, int32_t T, int rule, double eps, double c,
                         uint64_t seed, int64_t k_max, double *est, int64_t *samples,
                         double *S, uint8_t *status);

/* Directed graphs (Definition 1 over ordered pairs, shortest paths following
 * edge directions): row/col hold each vertex's out-neighbours (rows sorted,
 * no self-loops or duplicates); the in-neighbour rows are built inside. The
 * search and Theorem 1's successor sums follow out-edges, the path counts of
 * Definition 3 sum over in-neighbours, and a pair's sigma_tv comes from a
 * search from v over reversed edges. Arguments and results as in the
 * undirected functions above. */
int oracle_brandes_directed(int64_t n, const int64_t *row, const int32_t *col, int32_t s,
                            int32_t *dist, double *sig_m, int32_t *sig_e, double *delta);
int oracle_bc_exact_directed(int64_t n, const int64_t *row, const int32_t *col, double *bc);
int oracle_dependencies_directed(int64_t n, const int64_t *row, const int32_t *col,
                                 const int32_t *sources, int64_t k, double *full, double *sum);
int oracle_pair_dependency_directed(int64_t n, const int64_t *row, const int32_t *col,
                                    int32_t u, int32_t v, double *y);
int oracle_adaptive_source_directed(int64_t n, const int64_t *row, const int32_t *col,
                                    const int32_t *targets, int32_t T, double c, uint64_t seed,
                                    int64_t k_max, double *est, int64_t *samples, double *S,
                                    uint8_t *status);
int oracle_adaptive_pair_directed(int64_t n, const int64_t *row, const int32_t *col,
                                  const int32_t *targets, int32_t T, int rule, double eps,
                                  double c, uint64_t seed, int64_t k_max, double *est,
                                  int64_t *samples, double *S, uint8_t *status);

/* Weighted graphs (Brandes' first step by Dijkstra's algorithm, Section 3):
 * wt[e] is the weight of arc e (row/col order), a positive integer with
 * max weight * (n - 1) < 2^30. directed = 0 takes an undirected CSR whose two
 * arcs of an edge carry the same weight; directed != 0 a CSR of out-arcs.
 * dist holds weighted distances. Results as the unweighted calls. */
int oracle_brandes_weighted(int64_t n, const int64_t *row, const int32_t *col,
                            const int32_t *wt, int directed, int32_t s, int32_t *dist,
                            double *sig_m, int32_t *sig_e, double *delta);
int oracle_bc_exact_weighted(int64_t n, const int64_t *row, const int32_t *col,
                             const int32_t *wt, int directed, double *bc);
int oracle_dependencies_weighted(int64_t n, const int64_t *row, const int32_t *col,
                                 const int32_t *wt, int directed, const int32_t *sources,
                                 int64_t k, double *full, double *sum);
int oracle_pair_dependency_weighted(int64_t n, const int64_t *row, const int32_t *col,
                                    const int32_t *wt, int directed, int32_t u, int32_t v,
                                    double *y);
int oracle_adaptive_source_weighted(int64_t n, const int64_t *row, const int32_t *col,
                                    const int32_t *wt, int directed, const int32_t *targets,
                                    int32_t T, double c, uint64_t seed, int64_t k_max,
                                    double *est, int64_t *samples, double *S, uint8_t *status);
int oracle_adaptive_pair_weighted(int64_t n, const int64_t *row, const int32_t *col,
                                  const int32_t *wt, int directed, const int32_t *targets,
                                  int32_t T, int rule, double eps, double c, uint64_t seed,
                                  int64_t k_max, double *est, int64_t *samples, double *S,
                                  uint8_t *status);

/* Work counters for the throughput metric: for source s, the number of
 * vertices reached and the undirected edges of s's component; for a pair
 * (u, v), the undirected edges with an endpoint at distance < d(u,v)
 * from u (all of u's component when v is unreachable). */
int oracle_source_work(int64_t n, const int64_t *row, const int32_t *col, int32_t s,
                       int64_t *reached, int64_t *edges_undirected, int64_t *dag_edges);
int oracle_pair_work(int64_t n, const int64_t *row, const int32_t *col, int32_t u, int32_t v,
                     int64_t *edges_undirected);
/* Work of the library's two-sided search for the pair (u, v), u != v, over
 * the same walks (the balanced order is the library's design; a measurement
 * check, not the paper's arithmetic): vertices the search adds and arcs of
 * the rows it reads. directed != 0: col lists out-neighbours. */
int oracle_bidir_work(int64_t n, const int64_t *row, const int32_t *col, int directed, int32_t u,
                      int32_t v, int64_t *found, int64_t *arcs);

#ifdef __cplusplus
}
#endif
#endif
