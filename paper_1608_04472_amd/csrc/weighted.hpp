// Weighted graphs: Brandes' pass over shortest paths by total arc weight.
//
// Section 3 runs Dijkstra's algorithm for the first step on weighted graphs.
// Here the batch's sources share one label-correcting search instead: every
// round relaxes the out-arcs of the (source, vertex) entries whose distance
// fell in the previous round (atomicMin on integer distances, so ties are
// exact), until no distance falls. Path counts (Definition 3 with the
// predecessor condition d(s,u) + w(u,v) = d(s,v)) then follow the shortest-
// path DAG in rounds: an entry joins the next round once its last DAG
// predecessor is done, and sums its predecessors' counts in CSR order (so
// the counts do not depend on the order in which rounds meet an entry).
// Every DAG successor of an entry joins a later round than the entry, so
// Theorem 1's sums run over the rounds in reverse.
//
// Layout: entry o = b * n + v of source lane b, as the pair-per-thread engine
// (whose output kernels read these arrays: dist < 0 unreached, 0 at the
// source, >= 1 elsewhere since weights are positive).

namespace bcmi {

constexpr int32_t kWUnreached = 0x7fffffff;

struct WArgs {
    const int64_t *row;   // out-arcs and their weights
    const int32_t *col;
    const int32_t *wt;
    const int64_t *rrow;  // in-arcs and their weights
    const int32_t *rcol;
    const int32_t *rwt;
    uint32_t n;
    int32_t B;
    int32_t *dist;        // [B][n]: kWUnreached until reached (-1 after the search)
    double *sig;          // [B][n] path counts
    double *dlt;          // [B][n] dependencies
    uint32_t *pend;       // [B][n] DAG predecessors not yet done
    uint32_t *flag;       // [B][n] last search round that queued the entry
    uint32_t *order;      // [B][n] entries in the rounds of the path counts
    unsigned long long *ctl;
    const int32_t *srcs;
    const int32_t *dest;  // [B] pair destinations, or null
    int32_t nvalid;
    unsigned long long *prof;
};

__device__ __forceinline__ void w_split(const WArgs &a, uint32_t o, uint32_t &b, uint32_t &v)
{
    b = o / a.n;
    v = o - b * a.n;
}

// round 0: each lane's source at distance 0, queued for the search and first
// in the order of the path counts
__global__ void k_w_init(WArgs a, uint32_t *frontier)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.nvalid) return;
    const uint32_t o = (uint32_t)b * a.n + (uint32_t)a.srcs[b];
    a.dist[o] = 0;
    frontier[b] = o;
    a.order[b] = o;
}

// One search round over the queued entries F[0, count): relax their out-arcs
// and queue (once per round) every entry whose distance fell.
__global__ void k_w_relax(WArgs a, const uint32_t *F, int64_t count, uint32_t *next,
                          uint32_t round)
{
    unsigned long long units = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t o = F[i];
        uint32_t b, v;
        w_split(a, o, b, v);
        const int32_t dv = a.dist[o];
        const uint32_t base = b * a.n;
        const int64_t e1 = a.row[v + 1];
        units += (unsigned long long)(e1 - a.row[v]);
        for (int64_t e = a.row[v]; e < e1; ++e) {
            const uint32_t ow = base + (uint32_t)a.col[e];
            const int32_t nd = dv + a.wt[e];
            if (nd < a.dist[ow] && nd < atomicMin(&a.dist[ow], nd) &&
                atomicExch(&a.flag[ow], round) != round)
                next[atomicAdd(&a.ctl[CTL_TAIL], 1ull)] = ow;
        }
    }
    if (a.prof) prof_add_raw(a.prof, PROF_W_SEARCH, wave_sum_u64(units), 0);
}

// After the search: unreached entries to -1; per reached entry its number of
// DAG predecessors, path count 1 at the source and 0 elsewhere, dependency 0.
// Sets the order list's tail after the sources (ctl zeroed beforehand).
__global__ void k_w_count(WArgs a)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl[CTL_TAIL] = (unsigned long long)a.nvalid;
    const int64_t total = (int64_t)a.nvalid * a.n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t o = (uint32_t)i;
        uint32_t b, v;
        w_split(a, o, b, v);
        const int32_t d = a.dist[o];
        a.dlt[o] = 0.0;
        if (d == kWUnreached) {
            a.dist[o] = -1;
            a.sig[o] = 0.0;
            continue;
        }
        a.sig[o] = d == 0 ? 1.0 : 0.0;
        uint32_t preds = 0;
        if (d > 0) {
            const uint32_t base = b * a.n;
            for (int64_t e = a.rrow[v]; e < a.rrow[v + 1]; ++e) {
                const int32_t du = a.dist[base + (uint32_t)a.rcol[e]];
                // an unreached in-neighbour holds kWUnreached or -1: never equal
                if (du >= 0 && du != kWUnreached && du + a.rwt[e] == d) ++preds;
            }
        }
        a.pend[o] = preds;
    }
}

// Path counts, one round: the entries order[s0, s1) are done; each DAG
// successor whose last predecessor this is sums its predecessors' counts and
// joins the next round (appended at ctl[CTL_TAIL]).
__global__ void k_w_sigma(WArgs a, int64_t s0, int64_t s1)
{
    unsigned long long ua = 0, ub = 0;
    for (int64_t i = s0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < s1;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t o = a.order[i];
        uint32_t b, v;
        w_split(a, o, b, v);
        const uint32_t base = b * a.n;
        const int32_t dv = a.dist[o];
        for (int64_t e = a.row[v]; e < a.row[v + 1]; ++e) {
            const uint32_t x = (uint32_t)a.col[e];
            const uint32_t ow = base + x;
            if (dv + a.wt[e] != a.dist[ow]) continue;
            if (atomicSub(&a.pend[ow], 1u) != 1u) continue;
            double s = 0.0;
            const int32_t dw = a.dist[ow];
            for (int64_t f = a.rrow[x]; f < a.rrow[x + 1]; ++f) {
                const int32_t du = a.dist[base + (uint32_t)a.rcol[f]];
                if (du >= 0 && du + a.rwt[f] == dw) s += a.sig[base + (uint32_t)a.rcol[f]];
            }
            ub += (unsigned long long)(a.rrow[x + 1] - a.rrow[x]);
            ++ua;
            a.sig[ow] = s;
            if (!(s < 0x1p1000)) a.ctl[CTL_SIG_OVERFLOW] = 1ull;
            a.order[atomicAdd(&a.ctl[CTL_TAIL], 1ull)] = ow;
        }
    }
    if (a.prof) prof_add_raw(a.prof, PROF_W_COUNTS, wave_sum_u64(ua), wave_sum_u64(ub));
}

// Theorem 1 for the entries order[s0, s1) of one round (every successor is in
// a later round): delta(v) = sum over DAG successors w of sigma(v)/sigma(w) *
// (term(w) + delta(w)), term 1 (pair mode: 1 only at the lane's destination).
__global__ void k_w_backward(WArgs a, int64_t s0, int64_t s1)
{
    unsigned long long ua = 0, ub = 0;
    for (int64_t i = s0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < s1;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t o = a.order[i];
        uint32_t b, v;
        w_split(a, o, b, v);
        const uint32_t base = b * a.n;
        const int32_t dv = a.dist[o];
        const int32_t dst = a.dest ? a.dest[b] : -1;
        const double sv = a.sig[o];
        double acc = 0.0;
        for (int64_t e = a.row[v]; e < a.row[v + 1]; ++e) {
            const int32_t x = a.col[e];
            const uint32_t ow = base + (uint32_t)x;
            if (dv + a.wt[e] != a.dist[ow]) continue;
            const double term = a.dest ? (x == dst ? 1.0 : 0.0) : 1.0;
            acc += sv / a.sig[ow] * (term + a.dlt[ow]);
        }
        ub += (unsigned long long)(a.row[v + 1] - a.row[v]);
        ++ua;
        a.dlt[o] = acc;
    }
    if (a.prof) prof_add_raw(a.prof, PROF_W_BACKWARD, wave_sum_u64(ua), wave_sum_u64(ub));
}

}  // namespace bcmi
