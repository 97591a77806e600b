// Weighted graphs: Brandes' pass over shortest paths by total arc weight.
//
// Section 3 runs Dijkstra's algorithm for the first step on weighted graphs.
// Here the batch's sources share one label-correcting search instead: every
// round relaxes the out-arcs of the (source, vertex) entries whose distance
// fell in the previous round (atomicMin on integer distances, so ties are
// exact), until no distance falls. Path counts (Definition 3 with the
// predecessor condition d(s,u) + w(u,v) = d(s,v)) then follow the shortest-
// path DAG in rounds: an entry joins the next round once its last DAG
// predecessor is done, and then sums its predecessors' counts in CSR order
// (so the counts do not depend on the order in which rounds meet an entry).
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

// rows up to this many arcs are walked by one thread, longer ones by a wavefront
constexpr int kWSmall = 32;

// Entries i in [i0, i1), grid-strided a wavefront's 64 at a time: get(i, r0,
// r1) names the entry's row (false: nothing to do); a row of at most kWSmall
// arcs goes to the entry's lane as small(i, r0, r1), a longer one to the
// whole wavefront as big(i, r0, r1, lane).
template <class Get, class Small, class Big>
__device__ __forceinline__ void w_rows(int64_t i0, int64_t i1, Get get, Small small, Big big)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t c = i0 + wave * kWave; c < i1; c += waves * kWave) {
        const int64_t i = c + lane;
        int64_t r0 = 0, r1 = 0;
        const bool on = i < i1 && get(i, r0, r1);
        const bool longrow = on && r1 - r0 > kWSmall;
        if (on && !longrow) small(i, r0, r1);
        uint64_t m = __ballot(longrow);
        while (m) {
            const int src = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            big(__shfl(i, src, kWave), __shfl(r0, src, kWave), __shfl(r1, src, kWave), lane);
        }
    }
}

// Append to a global list among the active lanes of a wavefront: one atomic
// on *tail for all lanes with want set (a contended counter serialises every
// atomic on it); returns each such lane's position. Safe in divergent code.
__device__ __forceinline__ unsigned long long w_append(bool want, unsigned long long *tail)
{
    const uint64_t bal = __ballot(want);
    if (!want) return 0;
    const int leader = __ffsll((unsigned long long)bal) - 1;
    const int lane = threadIdx.x & (kWave - 1);
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(tail, (unsigned long long)__popcll(bal));
    base = __shfl(base, leader, kWave);
    return base + (unsigned long long)__popcll(bal & ((1ull << lane) - 1ull));
}

// lane 0 receives the wavefront's sum, added in a fixed tree
__device__ __forceinline__ double w_wave_sum(double x)
{
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) x += __shfl_down(x, off, kWave);
    return x;
}

// One search round over the queued entries F[0, count): relax their out-arcs
// and queue (once per round) every entry whose distance fell.
__global__ void k_w_relax(WArgs a, const uint32_t *F, int64_t count, uint32_t *next,
                          uint32_t round)
{
    unsigned long long units = 0;
    auto relax = [&](uint32_t base, int32_t dv, int64_t e) {
        const uint32_t ow = base + (uint32_t)a.col[e];
        const int32_t nd = dv + a.wt[e];
        const bool queue = nd < a.dist[ow] && nd < atomicMin(&a.dist[ow], nd) &&
                           atomicExch(&a.flag[ow], round) != round;
        const unsigned long long at = w_append(queue, &a.ctl[CTL_TAIL]);
        if (queue) next[at] = ow;
    };
    w_rows(
        0, count,
        [&](int64_t i, int64_t &r0, int64_t &r1) {
            uint32_t b, v;
            w_split(a, F[i], b, v);
            r0 = a.row[v];
            r1 = a.row[v + 1];
            return true;
        },
        [&](int64_t i, int64_t r0, int64_t r1) {
            const uint32_t o = F[i];
            const int32_t dv = a.dist[o];
            const uint32_t base = o / a.n * a.n;
            units += (unsigned long long)(r1 - r0);
            for (int64_t e = r0; e < r1; ++e) relax(base, dv, e);
        },
        [&](int64_t i, int64_t r0, int64_t r1, int lane) {
            const uint32_t o = F[i];
            const int32_t dv = a.dist[o];
            const uint32_t base = o / a.n * a.n;
            for (int64_t e = r0 + lane; e < r1; e += kWave) {
                ++units;
                relax(base, dv, e);
            }
        });
    if (a.prof) prof_add_raw(a.prof, PROF_W_SEARCH, wave_sum_u64(units), 0);
}

// After the search: unreached entries to -1; per reached entry its number of
// DAG predecessors, path count 1 at the source and 0 elsewhere, dependency 0.
// Sets the order list's tail after the sources (ctl zeroed beforehand).
__global__ void k_w_count(WArgs a)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl[CTL_TAIL] = (unsigned long long)a.nvalid;
    // an unreached in-neighbour holds kWUnreached or (once converted) -1
    auto is_pred = [&](uint32_t base, int64_t e, int32_t d) {
        const int32_t du = a.dist[base + (uint32_t)a.rcol[e]];
        return du >= 0 && du != kWUnreached && du + a.rwt[e] == d;
    };
    w_rows(
        0, (int64_t)a.nvalid * a.n,
        [&](int64_t i, int64_t &r0, int64_t &r1) {
            const uint32_t o = (uint32_t)i;
            uint32_t b, v;
            w_split(a, o, b, v);
            const int32_t d = a.dist[o];
            a.dlt[o] = 0.0;
            if (d == kWUnreached) {
                a.dist[o] = -1;
                a.sig[o] = 0.0;
                return false;
            }
            a.sig[o] = d == 0 ? 1.0 : 0.0;
            if (d == 0) {
                a.pend[o] = 0u;
                return false;
            }
            r0 = a.rrow[v];
            r1 = a.rrow[v + 1];
            return true;
        },
        [&](int64_t i, int64_t r0, int64_t r1) {
            const uint32_t o = (uint32_t)i;
            const uint32_t base = o / a.n * a.n;
            const int32_t d = a.dist[o];
            uint32_t preds = 0;
            for (int64_t e = r0; e < r1; ++e) preds += is_pred(base, e, d) ? 1u : 0u;
            a.pend[o] = preds;
        },
        [&](int64_t i, int64_t r0, int64_t r1, int lane) {
            const uint32_t o = (uint32_t)i;
            const uint32_t base = o / a.n * a.n;
            const int32_t d = a.dist[o];
            unsigned long long preds = 0;
            for (int64_t e = r0 + lane; e < r1; e += kWave) preds += is_pred(base, e, d) ? 1 : 0;
            preds = wave_sum_u64(preds);
            if (lane == 0) a.pend[o] = (uint32_t)preds;
        });
}

// Path counts, first half of a round: the entries order[s0, s1) are done;
// every DAG successor whose last predecessor this is joins the next round
// (appended at ctl[CTL_TAIL]).
__global__ void k_w_release(WArgs a, int64_t s0, int64_t s1)
{
    auto release = [&](uint32_t base, int32_t dv, int64_t e) {
        const uint32_t ow = base + (uint32_t)a.col[e];
        const bool ready = dv + a.wt[e] == a.dist[ow] && atomicSub(&a.pend[ow], 1u) == 1u;
        const unsigned long long at = w_append(ready, &a.ctl[CTL_TAIL]);
        if (ready) a.order[at] = ow;
    };
    w_rows(
        s0, s1,
        [&](int64_t i, int64_t &r0, int64_t &r1) {
            uint32_t b, v;
            w_split(a, a.order[i], b, v);
            r0 = a.row[v];
            r1 = a.row[v + 1];
            return true;
        },
        [&](int64_t i, int64_t r0, int64_t r1) {
            const uint32_t o = a.order[i];
            const int32_t dv = a.dist[o];
            const uint32_t base = o / a.n * a.n;
            for (int64_t e = r0; e < r1; ++e) release(base, dv, e);
        },
        [&](int64_t i, int64_t r0, int64_t r1, int lane) {
            const uint32_t o = a.order[i];
            const int32_t dv = a.dist[o];
            const uint32_t base = o / a.n * a.n;
            for (int64_t e = r0 + lane; e < r1; e += kWave) release(base, dv, e);
        });
}

// Path counts, second half: each entry of order[s0, s1) (released by the
// previous half) sums its DAG predecessors' counts over its in-row in CSR
// order (a long row by a wavefront with a fixed tree).
__global__ void k_w_sigma(WArgs a, int64_t s0, int64_t s1)
{
    unsigned long long ua = 0, ub = 0;
    auto term = [&](uint32_t base, int64_t e, int32_t dw) {
        const uint32_t ou = base + (uint32_t)a.rcol[e];
        const int32_t du = a.dist[ou];
        return du >= 0 && du + a.rwt[e] == dw ? a.sig[ou] : 0.0;
    };
    auto store = [&](uint32_t o, double x) {
        a.sig[o] = x;
        if (!(x < 0x1p1000)) a.ctl[CTL_SIG_OVERFLOW] = 1ull;
    };
    w_rows(
        s0, s1,
        [&](int64_t i, int64_t &r0, int64_t &r1) {
            uint32_t b, v;
            w_split(a, a.order[i], b, v);
            r0 = a.rrow[v];
            r1 = a.rrow[v + 1];
            return true;
        },
        [&](int64_t i, int64_t r0, int64_t r1) {
            const uint32_t o = a.order[i];
            const uint32_t base = o / a.n * a.n;
            const int32_t dw = a.dist[o];
            double x = 0.0;
            for (int64_t e = r0; e < r1; ++e) x += term(base, e, dw);
            ++ua;
            ub += (unsigned long long)(r1 - r0);
            store(o, x);
        },
        [&](int64_t i, int64_t r0, int64_t r1, int lane) {
            const uint32_t o = a.order[i];
            const uint32_t base = o / a.n * a.n;
            const int32_t dw = a.dist[o];
            double x = 0.0;
            for (int64_t e = r0 + lane; e < r1; e += kWave) {
                ++ub;
                x += term(base, e, dw);
            }
            x = w_wave_sum(x);
            if (lane == 0) {
                ++ua;
                store(o, x);
            }
        });
    if (a.prof) prof_add_raw(a.prof, PROF_W_COUNTS, wave_sum_u64(ua), wave_sum_u64(ub));
}

// Theorem 1 for the entries order[s0, s1) of one round (every successor is in
// a later round): delta(v) = sum over DAG successors w of sigma(v)/sigma(w) *
// (term(w) + delta(w)), term 1 (pair mode: 1 only at the lane's destination).
__global__ void k_w_backward(WArgs a, int64_t s0, int64_t s1)
{
    unsigned long long ua = 0, ub = 0;
    auto part = [&](uint32_t o, uint32_t base, int32_t dv, int32_t dst, int64_t e) {
        const int32_t x = a.col[e];
        const uint32_t ow = base + (uint32_t)x;
        if (dv + a.wt[e] != a.dist[ow]) return 0.0;
        const double term = a.dest ? (x == dst ? 1.0 : 0.0) : 1.0;
        return a.sig[o] / a.sig[ow] * (term + a.dlt[ow]);
    };
    w_rows(
        s0, s1,
        [&](int64_t i, int64_t &r0, int64_t &r1) {
            uint32_t b, v;
            w_split(a, a.order[i], b, v);
            r0 = a.row[v];
            r1 = a.row[v + 1];
            return true;
        },
        [&](int64_t i, int64_t r0, int64_t r1) {
            const uint32_t o = a.order[i];
            const uint32_t b = o / a.n, base = b * a.n;
            const int32_t dv = a.dist[o];
            const int32_t dst = a.dest ? a.dest[b] : -1;
            double x = 0.0;
            for (int64_t e = r0; e < r1; ++e) x += part(o, base, dv, dst, e);
            ++ua;
            ub += (unsigned long long)(r1 - r0);
            a.dlt[o] = x;
        },
        [&](int64_t i, int64_t r0, int64_t r1, int lane) {
            const uint32_t o = a.order[i];
            const uint32_t b = o / a.n, base = b * a.n;
            const int32_t dv = a.dist[o];
            const int32_t dst = a.dest ? a.dest[b] : -1;
            double x = 0.0;
            for (int64_t e = r0 + lane; e < r1; e += kWave) {
                ++ub;
                x += part(o, base, dv, dst, e);
            }
            x = w_wave_sum(x);
            if (lane == 0) {
                ++ua;
                a.dlt[o] = x;
            }
        });
    if (a.prof) prof_add_raw(a.prof, PROF_W_BACKWARD, wave_sum_u64(ua), wave_sum_u64(ub));
}

}  // namespace bcmi
