/*
 * bcmi -- sampled betweenness centrality on an MI355X (gfx950), C ABI.
 *
 * Implements the computations of S. Ji and Z. Yan, "Refining Approximating
 * Betweenness Centrality Based on Samplings" (arXiv 1608.04472):
 *   - Brandes' pass (Section 3): breadth-first search from a source giving
 *     distances and shortest-path counts sigma, then the dependency recursion
 *     of Theorem 1 in non-increasing distance;
 *   - exact BC as the sum of source dependencies (Section 3, Definition 1);
 *   - Bader's adaptive source sampling as restated in Section 4;
 *   - adaptive pair sampling (Algorithm 1, Section 6.1) with the early stop of
 *     the pair's search once the destination's level is complete (Section 6.2).
 *
 * Conventions shared by every call:
 *   - Graphs are undirected and unweighted: symmetric CSR with rows sorted
 *     ascending, no self-loops, no duplicate edges, 0 <= col < n < 2^31.
 *   - BC counts ordered pairs (s, t), s, t, v pairwise distinct, so
 *     0 <= BC(v) < n^2 (Definition 1).
 *   - Array arguments of compute calls (bc_exact, bc_dependencies,
 *     bc_pair_dependencies, bc_adaptive_*, bc_draw_*) are DEVICE pointers on
 *     the graph's device, or HOST pointers once bc_graph_set_io(g, BC_IO_HOST)
 *     has been called; the caller owns them either way. bc_graph_create reads
 *     a HOST CSR and keeps its own device copy.
 *   - Device memory the library needs (the graph's copy, its workspace) comes
 *     from the caller's bc_allocator when one is given, else from hipMalloc.
 *   - All work is ordered on the graph's stream; a call returns once its
 *     outputs are complete. One graph handle serves one host thread at a time.
 *   - Errors: no call throws or aborts. Arguments are checked before any
 *     device work: a bad argument returns BC_E_INVALID and leaves the outputs
 *     untouched. A failure found during the computation (BC_E_NOMEM,
 *     BC_E_DEVICE, BC_E_UNSUPPORTED) leaves the outputs unspecified. Either
 *     way bc_last_error() describes it.
 *   - Arithmetic: FP64. Path counts use an FP64 significand with an int32
 *     exponent once any count of a batch reaches 2^1000 (plain FP64 below).
 *   - Random draws: Philox4x64-10 (Salmon et al., SC'11), key (seed, stream),
 *     counter (j, 0, 0, 0) for sample j; stream 0 for sources, 1 for pairs.
 *     Source j = floor(w0 * n / 2^64). Pair j: u = floor(w0 * n / 2^64),
 *     v' = floor(w1 * (n-1) / 2^64), v = v' + (v' >= u).
 */
#ifndef BCMI_H
#define BCMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BC_OK = 0,
    BC_E_INVALID = 1,      /* bad argument or malformed CSR */
    BC_E_NOMEM = 2,        /* device memory exhausted */
    BC_E_DEVICE = 3,       /* HIP runtime error (message in bc_last_error) */
    BC_E_UNSUPPORTED = 4   /* valid request that the library does not serve */
} bc_status;

typedef enum {
    BC_DONE = 0,           /* the stopping rule was met */
    BC_CAPPED = 1          /* k_max samples taken without meeting it */
} bc_target_status;

/* Output layouts of bc_dependencies. */
typedef enum {
    BC_OUT_FULL = 0,       /* out[i*n + v] = delta_{sources[i].}(v), k*n doubles */
    BC_OUT_SUM = 1,        /* out[v] = sum over i of delta_{sources[i].}(v), n doubles */
    BC_OUT_TARGETS = 2     /* out[i*T + t] = delta_{sources[i].}(targets[t]), k*T doubles:
                              the values a sampler takes from each sample (Section 4) */
} bc_out_mode;

/* Where the array arguments of compute calls live (bc_graph_set_io). */
typedef enum {
    BC_IO_DEVICE = 0,      /* device pointers on the graph's device (default) */
    BC_IO_HOST = 1         /* host pointers: the library stages them through
                              device memory from the graph's allocator */
} bc_io;

/* Stopping rules of bc_adaptive_pair. */
typedef enum {
    BC_PAIR_ALG1 = 0,      /* Algorithm 1 as printed: repeat while S <= c*n */
    BC_PAIR_EPS = 1        /* stop at the first k with S > 0 and k*S^2 >= eps^3 n^2:
                              Lemma 5's sample count eps*(n^2(n-1)/A)^(2/3) with A
                              replaced by the running estimate n(n-1)S/k */
} bc_pair_rule;

/* Batch scheduling (the engine's knobs; results do not depend on them beyond
 * FP64 summation order in BC_OUT_SUM and bc_exact). */
typedef enum {
    BC_SCHED_AUTO = 0,     /* BATCHED, or THREADED when a BFS from a highest-degree
                              vertex is deeper than 32 levels; batch width auto */
    BC_SCHED_BATCHED = 1,  /* many sources per launch: one wavefront per
                              (vertex, 64-source word), lanes = sources */
    BC_SCHED_PER_SOURCE = 2, /* one source per launch sequence, one thread per
                              frontier vertex: the plain form, for comparison */
    BC_SCHED_THREADED = 3, /* many sources per launch, one thread per (vertex,
                              source) pair: for graphs of large diameter */
    BC_SCHED_TUNED = 4,    /* the first compute call times candidate plans and
                              keeps the fastest (bc_graph_tune) */
    BC_SCHED_WORKGROUP = 5 /* one workgroup per source, whole passes with
                              workgroup barriers only (no device-wide step per
                              level): for graphs of large diameter; batch =
                              sources in flight (0 = auto, up to 1024 within
                              70 % of free memory, 40 bytes per vertex each).
                              bc_dependencies, bc_exact, bc_pair_dependencies
                              (one-sided); the samplers run the THREADED engine */
} bc_schedule;

typedef struct {
    int32_t schedule;      /* bc_schedule */
    int32_t batch;         /* sources per batch, a power of two in [64, 4096]; 0 = auto */
    double bottom_up;      /* run a level bottom-up when its frontier entries exceed
                              bottom_up * (n * batch/64); 0 = auto, < 0 = never */
    int64_t split_entries; /* ignored (any value): every level sums rows longer
                              than 256 in parts of 256, one wavefront per part over
                              the whole device; the field keeps the struct's layout */
    int32_t level_loop;    /* pair-per-thread engine: > 0 runs all levels of a pass in
                              one persistent cooperative launch (grid barriers between
                              phases, each wait bounded in time: BC_E_DEVICE if one
                              gives up); <= 0 launches each level's phases
                              separately (the default). Values are identical
                              either way. */
    int32_t sampler_batch; /* samples per round of bc_adaptive_source / _pair, a
                              power of two in [64, 4096]; 0 = auto (256 sources,
                              2048 pairs). A round
                              runs ahead of the stop rule by at most its width:
                              results do not depend on it. */
    int32_t pair_search;   /* bc_pair_search: how pair samples (bc_adaptive_pair,
                              bc_pair_dependencies) find their shortest paths */
} bc_config;

/* Pair samples: the search from u that stops once v's level is complete
 * (Section 6.2), run by the engine the schedule picks, or a balanced search
 * from both ends, one workgroup per pair (the side with fewer frontier arcs
 * grows until the two sides meet; the counts on the shortest paths are then
 * completed by one sweep per side). AUTO takes the bidirectional search; a
 * batch whose path counts reach 2^1000 in it is run one-sided. Values are
 * identical either way up to FP64 summation order. */
typedef enum {
    BC_PAIR_SEARCH_AUTO = 0,
    BC_PAIR_SEARCH_ONE_SIDED = 1,
    BC_PAIR_SEARCH_BIDIRECTIONAL = 2
} bc_pair_search;

/* Host CSR. row has n+1 entries, int64 if row_is_i64 else int32. */
typedef struct {
    int64_t n;
    int64_t nnz;
    const void *row;
    int32_t row_is_i64;
    const int32_t *col;
} bc_csr;

typedef struct bc_graph bc_graph;

/* Device memory provider. alloc returns `bytes` of device memory on the
 * current device (aligned to at least 256 bytes), or NULL when it has none;
 * free releases what alloc returned. Both may be called from any library
 * call on the handle that was created with it, on the calling host thread;
 * the memory is used on the handle's stream. The struct is copied: ctx must
 * stay valid until the handle is destroyed. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} bc_allocator;

/* Validate a host CSR and copy it to the current HIP device. alloc supplies
 * all device memory of the handle (NULL = hipMalloc / hipFree). hip_stream is
 * a hipStream_t (NULL = the null stream). On success *out owns the device
 * copy and a lazily grown workspace; release it with bc_graph_destroy.
 * row_is_i64 = 0 takes int32 row offsets (nnz < 2^31). */
bc_status bc_graph_create(const bc_csr *csr, const bc_allocator *alloc, void *hip_stream,
                          bc_graph **out);
/* A directed graph (Definition 1 over ordered pairs, paths following arc
 * directions): csr->row / csr->col list each vertex's out-neighbours (rows
 * sorted ascending, no self-loops or repeated arcs, 0 <= col < n; no symmetry
 * required). The library builds the in-neighbour rows: the search and
 * Theorem 1's successor sums follow out-arcs, the path counts of Definition 3
 * sum over in-neighbours. Every compute call serves the handle; the query
 * server takes undirected graphs. */
bc_status bc_graph_create_directed(const bc_csr *csr, const bc_allocator *alloc,
                                   void *hip_stream, bc_graph **out);
/* A weighted graph (Section 3: Brandes' first step by Dijkstra's algorithm;
 * shortest paths minimise the total arc weight). weights[e] is the weight of
 * arc e of csr->col: positive, with max weight * (n - 1) < 2^30 so distances
 * and their sums are exact in int32; undirected graphs (directed = 0) need
 * equal weights on the two arcs of an edge, directed ones (directed != 0) take
 * a CSR of out-arcs as bc_graph_create_directed. Every compute call serves
 * the handle with one engine (a label-correcting search of the batch's
 * sources, 64 per wavefront word, then path counts and Theorem 1 over the
 * shortest-path DAG in topological rounds; bc_last_stats reports it as
 * BC_SCHED_BATCHED); dist_out holds weighted distances; path counts must
 * stay below 2^1000 (BC_E_UNSUPPORTED otherwise); pair samples search from
 * u to the end of the search (no early stop, no two-sided search). Not
 * served: the query server, bc_dependencies_noalloc. */
bc_status bc_graph_create_weighted(const bc_csr *csr, const int32_t *weights, int32_t directed,
                                   const bc_allocator *alloc, void *hip_stream, bc_graph **out);
void bc_graph_destroy(bc_graph *g);
bc_status bc_graph_set_stream(bc_graph *g, void *hip_stream);
/* Autotuner: times candidate plans on one seeded batch of sources each and
 * installs the fastest per source, by coordinate descent: the engine
 * (BC_SCHED_BATCHED, BC_SCHED_THREADED or BC_SCHED_WORKGROUP, the last one
 * only on graphs deeper than 32 levels or of at most 2^16 vertices) at its
 * default width, then the batch width (256 .. 4096, within 32-bit indices and free
 * memory; for BC_SCHED_WORKGROUP the sources in flight, 64 .. 1024), then the
 * wave engine's bottom_up (0.04, 0.01, 0.15, never), or the pair engine's
 * level_loop. A candidate slower than 1.5x
 * the best so far is abandoned early. Winners are cached per process by graph
 * signature (n, nnz, log2-degree histogram, BFS depth from a highest-degree
 * vertex). The width applies to bc_dependencies and bc_exact; the samplers keep
 * their round widths, and a source sampler on the wave engine whose round width
 * differs from the plan's tries the bottom_up candidates once more on up to
 * eight rounds of that width, twice each (the threshold is kept per graph
 * signature and width, and bc_last_stats reports the one used). Plans change scheduling only:
 * values equal any other plan's (sums up to FP64 summation order). *plan
 * (optional) receives it. */
bc_status bc_graph_tune(bc_graph *g, bc_config *plan);
/* The plan compute calls on g use now, with the schedule resolved to the
 * engine that runs (BC_SCHED_BATCHED, BC_SCHED_THREADED or PER_SOURCE) and
 * batch the tuned width (0 = automatic). */
bc_status bc_graph_plan(bc_graph *g, bc_config *out);
/* bc_io: where the array arguments of later compute calls on g live. */
bc_status bc_graph_set_io(bc_graph *g, int32_t io);
bc_status bc_graph_configure(bc_graph *g, const bc_config *cfg);
bc_status bc_graph_info(const bc_graph *g, int64_t *n, int64_t *nnz);

/* Exact BC of every vertex (Section 3; Definition 1 over ordered pairs):
 * out[v] = sum over s != v of delta_{s.}(v), all n sources. out: n doubles. */
bc_status bc_exact(bc_graph *g, double *out);

/* Brandes' pass from each of k given sources (Definition 2, Theorem 1).
 * sources: k int32 in [0, n), repeats allowed. out: see bc_out_mode.
 * dist_out (k*n int32, -1 = unreachable), sigma_mant and sigma_exp (k*n each,
 * sigma = mant * 2^exp) are optional (NULL) per-source outputs, source-major;
 * they require out_mode == BC_OUT_FULL. targets (T int32 in [0, n)) are read
 * only in BC_OUT_TARGETS mode (else they may be NULL, T = 0).
 * delta_{s.}(s) = 0. */
bc_status bc_dependencies(bc_graph *g, const int32_t *sources, int64_t k, int32_t out_mode,
                          double *out, int32_t *dist_out, double *sigma_mant,
                          int32_t *sigma_exp, const int32_t *targets, int32_t T);

/* Bader's adaptive source sampling as restated in Section 4, for T targets
 * sharing one sample stream (target i's results equal a T = 1 call with the
 * same seed). Per target: S = 0, k = 0; repeat { draw source s_k; S +=
 * delta_{s_k.}(v); k += 1 } while S <= c*n and k < k_max; est = n*S/k.
 * c >= 1, k_max >= 1. Outputs (device, T entries each): est (double),
 * samples (int64), S (double), status (uint8, bc_target_status). */
bc_status bc_adaptive_source(bc_graph *g, const int32_t *targets, int32_t T, double c,
                             uint64_t seed, int64_t k_max, double *out_est,
                             int64_t *out_samples, double *out_S, uint8_t *out_status);

/* Adaptive pair sampling (Algorithm 1) for T targets sharing one stream.
 * Per target: S = 0, k = 0; repeat { draw ordered pair (u, v), u != v;
 * S += sigma_uv(t)/sigma_uv; k += 1 } until the rule stops or k = k_max;
 * est = n(n-1)*S/k. The pair's search stops once v's level is complete
 * (one-sided), or once the searches from u and from v meet (bidirectional;
 * bc_config.pair_search).
 * rule BC_PAIR_ALG1 needs c >= 1; BC_PAIR_EPS needs 0 < eps < 1/2. Outputs as
 * in bc_adaptive_source. */
bc_status bc_adaptive_pair(bc_graph *g, const int32_t *targets, int32_t T, int32_t rule,
                           double eps, double c, uint64_t seed, int64_t k_max,
                           double *out_est, int64_t *out_samples, double *out_S,
                           uint8_t *out_status);

/* ---------------------------------------------------- allocation-free call
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. Computes
 * what bc_dependencies computes in BC_OUT_FULL or BC_OUT_SUM mode without any
 * hipMalloc, hipFree or allocator call: the engine's buffers come from one
 * fixed device array of BC_NOALLOC_SCRATCH_BYTES that the library holds on
 * every device it runs on until the process ends (the graph handle, created
 * beforehand, supplies the CSR). Sources run in batches of 64, in the
 * caller's order. Results equal bc_dependencies' up to FP64 summation order.
 * Limits: about 1.2 KB per vertex in BC_OUT_FULL and 0.7 KB in BC_OUT_SUM must
 * fit the array (extended path counts need 256 B more); a larger graph, a
 * level record beyond what is left, or BC_IO_HOST returns BC_E_UNSUPPORTED.
 * Arrays are device pointers. All calls on one device share its array and
 * it keeps the last call's contents: each call clears what it reads, and
 * calls that overlap on one device (other host threads or streams) race, so
 * the caller must not overlap them. */
#define BC_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
bc_status bc_dependencies_noalloc(bc_graph *g, const int32_t *sources, int64_t k,
                                  int32_t out_mode, double *out);

/* Pair dependencies of k given pairs: out[i*n + t] = sigma_{u_i v_i}(t) /
 * sigma_{u_i v_i} (0 for t in {u_i, v_i} or when v_i is unreachable), by the
 * search bc_config.pair_search selects.
 * us, vs: k int32 each, u_i != v_i. out: k*n doubles (device). */
bc_status bc_pair_dependencies(bc_graph *g, const int32_t *us, const int32_t *vs, int64_t k,
                               double *out);

/* Sample draws as the samplers take them (Philox4x64-10, maps above):
 * out_u[i] (and out_v[i] for pairs) for j = j0 + i, i < count. Device outputs. */
bc_status bc_draw_sources(bc_graph *g, uint64_t seed, int64_t j0, int64_t count,
                          int32_t *out_u);
bc_status bc_draw_pairs(bc_graph *g, uint64_t seed, int64_t j0, int64_t count,
                        int32_t *out_u, int32_t *out_v);

/* Statistics of the most recent compute call on g: samples (sources or pairs)
 * executed, batches, levels, whether extended path counts were needed. */
typedef struct {
    int64_t samples_executed;
    int64_t batches;
    int64_t levels;
    int32_t extended;
    int32_t batch_width;
    int32_t schedule;      /* bc_schedule that ran (never BC_SCHED_AUTO) */
    int32_t pair_search;   /* pair samples: BC_PAIR_SEARCH_BIDIRECTIONAL when every
                              batch took the two-sided search, ONE_SIDED when any
                              ran one-sided, 0 for source samples */
    double bottom_up;      /* bottom-up threshold the wave engine's levels used
                              (fraction of (vertex, word) entries; -1 = top-down
                              only); 0 when that engine did not run */
} bc_stats;
bc_status bc_last_stats(const bc_graph *g, bc_stats *out);

/* Per-kernel profile of the hot path, for roofline accounting. While enabled,
 * every launch of the hot kernels is bracketed by HIP events on the
 * graph's stream, and the kernels count the work units they process:
 *   units_a: (vertex, source) pairs (discovered, counted or swept),
 *   units_b: DAG (edge, source) pairs read (predecessor or successor values).
 * Algorithmic bytes per unit (8-byte path counts and rho, 4-byte levels):
 *   discover_topdown / discover_bottomup: 4 per units_a (level write)
 *   sigma_pull : 8 per units_a (count write) + 8 per units_b (count read)
 *   backward   : 20 per units_a (count read, rho write, level read)
 *                + 8 per units_b (rho read)
 *   hub_parts  : rows longer than 256 of both pulls, summed in parts of 256
 *                by a wavefront each before the pull adds the parts in order:
 *                8 per units_b (count or rho read); the pulls' units_a count
 *                their entries
 *   pair_forward : the pair engine's persistent forward loop (discovery and
 *                path counts of every level): 12 per units_a (level and
 *                count write) + 8 per units_b (count read)
 *   pair_backward: its persistent backward loop, bytes as backward
 *   level_record: 8 per (vertex, word) read + 36 per record entry written
 *   wg_pass    : the one-workgroup-per-source engine (whole passes): 36 per
 *                units_a (vertex reached: distance CAS, list entry, count,
 *                dependency, reset) + 12 per units_b (arc walked: head, its
 *                distance)
 *   w_search   : weighted graphs' search rounds (64 sources per word):
 *                4 per units_a (arc relaxed for one source: the head's
 *                distance) + 8 per units_b (arc walked for a word: head,
 *                weight)
 *   w_counts   : their path-count rounds, both halves (successors released,
 *                counts summed; units from the sums): 16 per units_a (entry
 *                counted: distance, count, pending counter) + 12 per units_b
 *                (in-arc read for an entry: the tail's distance and count)
 *   w_backward : their dependency rounds: 28 per units_a (entry: distance,
 *                count, dependency and rho written) + 12 per units_b (out-arc
 *                read for an entry: the head's distance and rho)
 *   bidir_pair : the two-sided pair search (one launch per batch of pairs):
 *                units_a = vertices found by either side, 36 each (row
 *                bounds, stamp, list entry, path count); units_b = arcs
 *                walked by its expansions, count sums and sweeps, 12 each
 *                (head, head's stamp)
 * Enabling resets the accumulators. Profiling adds one event pair per launch
 * and one counter update per wavefront. */
typedef struct {
    char name[32];
    int64_t launches;
    double ms;          /* sum of event-measured launch durations */
    int64_t units_a;
    int64_t units_b;
    double algo_bytes;  /* from the per-unit figures above */
} bc_kernel_profile;

bc_status bc_profile_enable(bc_graph *g, int32_t enable);
/* Writes up to max entries (one per kernel) to out; *count receives the number. */
bc_status bc_profile_read(bc_graph *g, bc_kernel_profile *out, int32_t max, int32_t *count);

/* ---------------------------------------------------------------- serving
 * A query server over device-resident graphs with continuous batching: each
 * round (bc_server_step) takes one graph and fills the sample slots of one
 * batch with consecutive samples of the active queries on that graph (source
 * and pair queries together), newly arrived queries joining as slots free
 * up. A query's samples come from its own seed and each sample's arithmetic
 * does not depend on its batch mates, so a query's result is bit-identical
 * to running it alone, and to bc_adaptive_source / bc_adaptive_pair with T = 1
 * on the same graph, seed and schedule. Pair samples take the two-sided
 * search (one workgroup per pair, up to an eighth of the graph's batch width
 * at once per lane, at most 512), as the
 * samplers do by default; on a graph where it once met path counts of 2^1000
 * they run one-sided from then on.
 * Admission by HBM budget: resident bytes (every graph's CSR and lane-order
 * key) plus the shared workspace never exceed the budget. The workspace is
 * sized per buffer for the widest need of any admitted graph; a new graph
 * takes the widest batch width (<= max_batch, and within the 32-bit index
 * range of its engine) that keeps that sum within the budget, and
 * bc_server_add_graph fails with BC_E_NOMEM when even width 64 does not fit.
 * A round whose level record would outgrow the budgeted workspace runs its
 * samples in two halves instead (results are unchanged).
 * Scheduling: shortest job first at graph granularity (the graph whose
 * cheapest unfinished query has the smallest bound (k_max - k) * nnz runs the
 * next round), with every eighth round given to the graph of the oldest
 * unfinished query so that no query starves. With several lanes
 * (bc_server_set_lanes) a step runs one round on each of up to that many
 * graphs at once, the next graphs by the same rule, each on its own stream
 * and workspace; every query's samples and results are the same as with one
 * lane (a query's rounds never run concurrently).
 * Not thread-safe: one host thread drives a server (the lanes' host threads
 * are the server's own). */
typedef struct bc_server bc_server;

typedef enum { BC_QUERY_SOURCE = 0, BC_QUERY_PAIR = 1 } bc_query_kind;

typedef struct {
    int32_t graph;        /* id from bc_server_add_graph */
    int32_t target;       /* vertex whose BC is estimated */
    int32_t kind;         /* bc_query_kind */
    int32_t rule;         /* pair queries: bc_pair_rule */
    double c;             /* source queries and BC_PAIR_ALG1: c >= 1 */
    double eps;           /* BC_PAIR_EPS: 0 < eps < 1/2 */
    uint64_t seed;
    int64_t k_max;        /* >= 1 */
    double arrival_s;     /* arrival on the server clock (bc_server_now); < 0 = now */
} bc_query;

typedef struct {
    int64_t id;
    int32_t graph;
    int32_t status;       /* bc_target_status */
    double est;
    int64_t samples;
    double S;
    double arrival_s;     /* server clock, seconds */
    double done_s;
} bc_result;

/* hbm_budget_bytes bounds the device memory the server holds: the resident
 * graphs (CSR, lane-order keys) plus the engine workspace of each lane. alloc
 * as in bc_graph_create (NULL = hipMalloc). */
bc_status bc_server_create(size_t hbm_budget_bytes, int32_t max_batch,
                           const bc_allocator *alloc, void *hip_stream, bc_server **out);
void bc_server_destroy(bc_server *s);
bc_status bc_server_add_graph(bc_server *s, const bc_csr *csr, int32_t *graph_id);
bc_status bc_server_submit(bc_server *s, const bc_query *q, int64_t *id);
/* Run one round per lane (on distinct graphs); *completed receives the number
 * of queries they finished (0 and no device work when nothing is queued). */
bc_status bc_server_step(bc_server *s, int32_t *completed);
/* Lanes: rounds of different graphs run concurrently, each lane with its own
 * stream (created by the server, default priority; lane 0 is the caller's
 * stream) and its own workspace. 1 <= lanes <= 4 (default 1). The budget then
 * holds the resident graphs plus one workspace per lane: BC_E_INVALID when
 * the admitted graphs' widest need times lanes does not fit; graphs added
 * later are sized for the current number of lanes. */
bc_status bc_server_set_lanes(bc_server *s, int32_t lanes);
/* Move up to max finished results (completion order) into out. */
bc_status bc_server_poll(bc_server *s, bc_result *out, int32_t max, int32_t *count);
bc_status bc_server_now(const bc_server *s, double *now_s);
typedef struct {
    int64_t queued;           /* submitted, not yet admitted */
    int64_t active;           /* admitted, still sampling */
    int64_t finished;         /* results produced so far */
    int64_t rounds;
    int64_t samples_executed; /* slots run, including those past a query's stop */
    int64_t samples_used;     /* samples counted by the stopping rules */
    int64_t resident_bytes;   /* graphs' device CSR and lane-order keys */
    int64_t workspace_bytes;  /* the lanes' engine workspaces held now */
    int64_t budget_bytes;     /* the budget: resident + workspace never exceed it */
    int64_t split_rounds;     /* rounds run in halves to stay within the budget */
} bc_server_stats;
bc_status bc_server_stats_get(const bc_server *s, bc_server_stats *out);
/* Batch width and engine (BC_SCHED_BATCHED or BC_SCHED_THREADED) chosen for a
 * graph at admission. */
bc_status bc_server_graph_width(const bc_server *s, int32_t graph, int32_t *width,
                                int32_t *schedule);

/* Thread-local description of the last error (empty string if none). */
const char *bc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
