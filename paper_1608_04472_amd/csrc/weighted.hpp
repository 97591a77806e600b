// Weighted graphs: Brandes' pass over shortest paths by total arc weight.
//
// Section 3 runs Dijkstra's algorithm for the first step on weighted graphs.
// Here the batch's sources share one label-correcting search instead, in the
// layout of the batched engine: the 64 lanes of a wavefront are 64 sources
// (one word), so that one arc of a vertex is relaxed for all of them with one
// coalesced read and coalesced atomicMin's on integer distances (ties are
// exact). Every round expands the words that have lanes whose distance fell
// in the previous round, until no distance falls; the search's atomics return
// nothing, so no wavefront waits on one. Path counts (Definition 3
// with the predecessor condition d(s,u) + w(u,v) = d(s,v)) then follow the
// shortest-path DAG in rounds: a lane joins the next round once its last DAG
// predecessor is done, and then sums its predecessors' counts in CSR order (so
// the counts do not depend on the order in which rounds meet it). Every DAG
// successor of a lane joins a later round, so Theorem 1's sums run over the
// rounds in reverse, in the rho form delta(v) = sigma(v) * sum of rho(w),
// rho(w) = (term(w) + delta(w)) / sigma(w).
//
// Layout: B = 64 * W sources; entry (v, b) at v * B + b, i.e. word (v, j) at
// v * W + j holds lanes b = 64 j .. 64 j + 63 contiguously. Word masks mark
// the lanes a list entry stands for.

namespace bcmi {

constexpr int32_t kWUnreached = 0x7fffffff;
constexpr int kWChunk = 64;    // arcs per task of the search
constexpr int kWFlight = 8;    // arcs whose loads a wavefront keeps in flight

struct WArgs {
    const int64_t *row;   // out-arcs and their weights
    const int32_t *col;
    const int32_t *wt;
    const int64_t *rrow;  // in-arcs and their weights
    const int32_t *rcol;
    const int32_t *rwt;
    int64_t n;
    int32_t logW;         // W = 2^logW words of 64 sources
    int32_t *dist;        // [n][B]: kWUnreached until reached
    double *sig;          // [n][B] path counts
    double *dlt;          // [n][B] dependencies
    double *rho;          // [n][B] (term + delta) / sigma, once swept
    uint32_t *pend;       // [n][B] DAG predecessors not yet counted
    uint64_t *chg;        // [n][W] lanes whose distance fell since the word was expanded
    uint64_t *rdy;        // [n][W] lanes released into the next round of the counts
    uint64_t *tmask;      // [list] lanes of a search list entry, taken at the round's start
    uint64_t *task;       // search tasks: list position << 32 | arc chunk
    uint32_t *ord;        // words of the counts' rounds, round after round
    uint64_t *omask;      // their lanes
    unsigned long long *ctl;
    const int32_t *srcs;  // [nvalid] source of lane b
    const int32_t *dest;  // [nvalid] pair destination of lane b, or null
    int32_t nvalid;
    unsigned long long *prof;
};

__device__ __forceinline__ int64_t w_wave_id()
{
    return ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
}
__device__ __forceinline__ int64_t w_waves() { return ((int64_t)gridDim.x * blockDim.x) / kWave; }

// entry (x, lane) of word j: x's word j, this lane
__device__ __forceinline__ int64_t w_at(const WArgs &a, int64_t x, uint32_t j, int lane)
{
    return (((x << a.logW) + j) << 6) + lane;
}

// A wavefront's appends to a list, 64 at a time: item k waits in lane k's
// registers, and a full (or final) group takes its place with one atomic on
// the tail (a contended counter serialises every atomic on it). Called with
// all lanes active and wave-uniform arguments.
struct WPush {
    uint32_t item = 0;
    uint64_t mask = 0;
    int cnt = 0;
    __device__ __forceinline__ void flush(unsigned long long *tail, uint32_t *items,
                                          uint64_t *masks, int lane)
    {
        if (cnt == 0) return;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(tail, (unsigned long long)cnt);
        base = __shfl(base, 0, kWave);
        if (lane < cnt) {
            items[base + lane] = item;
            if (masks) masks[base + lane] = mask;
        }
        cnt = 0;
    }
    __device__ __forceinline__ void push(uint32_t it, uint64_t m, unsigned long long *tail,
                                         uint32_t *items, uint64_t *masks, int lane)
    {
        if (lane == cnt) {
            item = it;
            mask = m;
        }
        if (++cnt == kWave) flush(tail, items, masks, lane);
    }
};

// lane 0 receives the wavefront's sum, added in a fixed tree
__device__ __forceinline__ double w_wave_sum(double x)
{
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) x += __shfl_down(x, off, kWave);
    return x;
}

// Lane 0 ORs the wavefront's ballot into a word mask; true (on every lane)
// when the mask was empty before, i.e. the word is new to its list.
__device__ __forceinline__ bool w_mark(uint64_t *word, uint64_t bal, int lane)
{
    unsigned long long prev = 0;
    if (lane == 0) prev = atomicOr((unsigned long long *)word, (unsigned long long)bal);
    return __shfl(prev, 0, kWave) == 0ull;
}

// Round 0 of the search: lane b's source at distance 0, its lane changed.
__global__ void k_ww_init(WArgs a)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.nvalid) return;
    const int64_t s = a.srcs[b];
    const uint32_t j = (uint32_t)b >> 6;
    a.dist[w_at(a, s, j, b & 63)] = 0;
    atomicOr((unsigned long long *)&a.chg[(s << a.logW) + j], 1ull << (b & 63));
}

// Appends one item per lane with `want` set and `count` items per lane to two
// lists with one atomic each per wavefront; returns the lane's first position
// in each (all lanes active).
__device__ __forceinline__ void w_append2(bool want, int32_t count, unsigned long long *tail1,
                                          unsigned long long *tail2, int lane,
                                          unsigned long long &at1, unsigned long long &at2)
{
    int32_t i1 = want ? 1 : 0, i2 = count;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int32_t y1 = __shfl_up(i1, off, kWave);
        const int32_t y2 = __shfl_up(i2, off, kWave);
        if (lane >= off) {
            i1 += y1;
            i2 += y2;
        }
    }
    const int32_t t1 = __shfl(i1, kWave - 1, kWave), t2 = __shfl(i2, kWave - 1, kWave);
    unsigned long long b1 = 0, b2 = 0;
    if (lane == 0 && t1) b1 = atomicAdd(tail1, (unsigned long long)t1);
    if (lane == 0 && t2) b2 = atomicAdd(tail2, (unsigned long long)t2);
    at1 = __shfl(b1, 0, kWave) + (unsigned long long)(i1 - (want ? 1 : 0));
    at2 = __shfl(b2, 0, kWave) + (unsigned long long)(i2 - count);
}

// Start of a search round: every word with changed lanes takes them (the
// word leaves the pending set, so later falls mark it again), joins the
// round's list (ctl[CTL_TAIL]) and is cut into tasks of kWChunk arcs
// (ctl[CTL_WTASKS]); both zeroed beforehand.
__global__ void k_ww_collect(WArgs a, uint32_t *list)
{
    const int lane = lane_id();
    const int64_t words = a.n << a.logW;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x; c < words;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t wi = c + threadIdx.x;
        uint64_t m = 0;
        int32_t chunks = 0;
        if (wi < words) {
            m = a.chg[wi];
            if (m) {
                a.chg[wi] = 0ull;
                const int64_t v = wi >> a.logW;
                chunks = (int32_t)((a.row[v + 1] - a.row[v] + kWChunk - 1) / kWChunk);
            }
        }
        unsigned long long at = 0, tb = 0;
        w_append2(m != 0, chunks, &a.ctl[CTL_TAIL], &a.ctl[CTL_WTASKS], lane, at, tb);
        if (m) {
            list[at] = (uint32_t)wi;
            a.tmask[at] = m;
            for (int32_t k = 0; k < chunks; ++k)
                a.task[tb + k] = ((uint64_t)at << 32) | (uint32_t)k;
        }
    }
}

// A search round: one wavefront per task relaxes its arc chunk for the
// entry's lanes. A lane whose candidate beats the distance it read marks its
// word changed: then its distance falls in this round (to the candidate or
// below), so every round lowers some distance and the search ends.
__global__ __launch_bounds__(kBlock) void k_ww_relax(WArgs a, const uint32_t *list)
{
    const int lane = lane_id();
    const int64_t ntask = (int64_t)a.ctl[CTL_WTASKS];
    const uint32_t jm = (1u << a.logW) - 1u;
    unsigned long long units = 0, arcs = 0;
    for (int64_t t = w_wave_id(); t < ntask; t += w_waves()) {
        const uint64_t tk = uniform_u64(a.task[t]);
        const int64_t i = (int64_t)(tk >> 32);
        const uint32_t wi = (uint32_t)__builtin_amdgcn_readfirstlane((int)list[i]);
        const uint64_t m = uniform_u64(a.tmask[i]);
        const int64_t v = wi >> a.logW;
        const uint32_t j = wi & jm;
        const int64_t r0 = a.row[v] + (int64_t)(uint32_t)tk * kWChunk;
        const int64_t rend = a.row[v + 1];
        const int64_t r1 = r0 + kWChunk < rend ? r0 + kWChunk : rend;
        const bool on = (m >> lane) & 1ull;
        const int32_t dv = a.dist[((int64_t)wi << 6) + lane];
        units += (unsigned long long)__popcll(m) * (unsigned long long)(r1 - r0);
        arcs += (unsigned long long)(r1 - r0);
        for (int64_t e = r0; e < r1; e += kWFlight) {
            int32_t xs[kWFlight], ws[kWFlight], old[kWFlight];
#pragma unroll
            for (int f = 0; f < kWFlight; ++f) {
                const bool ok = e + f < r1;
                xs[f] = ok ? a.col[e + f] : -1;
                ws[f] = ok ? a.wt[e + f] : 0;
            }
#pragma unroll
            for (int f = 0; f < kWFlight; ++f)
                old[f] = xs[f] >= 0 ? a.dist[w_at(a, xs[f], j, lane)] : kWUnreached;
#pragma unroll
            for (int f = 0; f < kWFlight; ++f) {
                if (xs[f] < 0) break;
                const int32_t nd = dv + ws[f];
                const bool imp = on && nd < old[f];
                if (imp) atomicMin(&a.dist[w_at(a, xs[f], j, lane)], nd);
                const uint64_t bal = wave_ballot(imp);
                if (bal && lane == 0)
                    atomicOr((unsigned long long *)&a.chg[((int64_t)xs[f] << a.logW) + j],
                             (unsigned long long)bal);
            }
        }
    }
    if (a.prof) prof_add_raw(a.prof, PROF_W_SEARCH, units, arcs);
}

// After the search, one wavefront per word (all n * W): path count 1 at the
// source and 0 elsewhere, dependency 0, the number of DAG predecessors of
// every reached lane; words holding sources form round 0 of the counts
// (ord / omask from ctl[CTL_TAIL], zeroed beforehand).
__global__ __launch_bounds__(kBlock) void k_ww_prep(WArgs a)
{
    const int lane = lane_id();
    const int64_t words = a.n << a.logW;
    const uint32_t jm = (1u << a.logW) - 1u;
    WPush q;
    for (int64_t wi = w_wave_id(); wi < words; wi += w_waves()) {
        const int64_t e = (wi << 6) + lane;
        const int32_t d = a.dist[e];
        a.sig[e] = d == 0 ? 1.0 : 0.0;
        a.dlt[e] = 0.0;
        const bool need = d != kWUnreached && d > 0;
        uint32_t preds = 0;
        if (wave_ballot(need)) {
            const int64_t v = wi >> a.logW;
            const uint32_t j = (uint32_t)wi & jm;
            const int64_t r1 = a.rrow[v + 1];
            for (int64_t r = a.rrow[v]; r < r1; r += kWFlight) {
                int32_t us[kWFlight], ws[kWFlight], du[kWFlight];
#pragma unroll
                for (int f = 0; f < kWFlight; ++f) {
                    const bool ok = r + f < r1;
                    us[f] = ok ? a.rcol[r + f] : -1;
                    ws[f] = ok ? a.rwt[r + f] : 0;
                }
#pragma unroll
                for (int f = 0; f < kWFlight; ++f)
                    du[f] = us[f] >= 0 ? a.dist[w_at(a, us[f], j, lane)] : kWUnreached;
#pragma unroll
                for (int f = 0; f < kWFlight; ++f)
                    preds += (need && du[f] != kWUnreached && du[f] + ws[f] == d) ? 1u : 0u;
            }
        }
        a.pend[e] = preds;
        const uint64_t src = wave_ballot(d == 0);
        if (src) q.push((uint32_t)wi, src, &a.ctl[CTL_TAIL], a.ord, a.omask, lane);
    }
    q.flush(&a.ctl[CTL_TAIL], a.ord, a.omask, lane);
}

// Path counts, first half of a round: the lanes of ord[s0, s1) are done;
// every DAG successor lane whose last predecessor this is joins the next
// round: its word's rdy mask gains the lane, and a word new to the round is
// appended to ord at ctl[CTL_TAIL].
__global__ __launch_bounds__(kBlock) void k_ww_release(WArgs a, int64_t s0, int64_t s1)
{
    const int lane = lane_id();
    const uint32_t jm = (1u << a.logW) - 1u;
    WPush q;
    for (int64_t i = s0 + w_wave_id(); i < s1; i += w_waves()) {
        const uint32_t wi = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.ord[i]);
        const uint64_t m = uniform_u64(a.omask[i]);
        const int64_t v = wi >> a.logW;
        const uint32_t j = wi & jm;
        const bool on = (m >> lane) & 1ull;
        const int32_t dv = a.dist[((int64_t)wi << 6) + lane];
        const int64_t r1 = a.row[v + 1];
        for (int64_t r = a.row[v]; r < r1; r += kWFlight) {
            int32_t xs[kWFlight], ws[kWFlight], dx[kWFlight];
#pragma unroll
            for (int f = 0; f < kWFlight; ++f) {
                const bool ok = r + f < r1;
                xs[f] = ok ? a.col[r + f] : -1;
                ws[f] = ok ? a.wt[r + f] : 0;
            }
#pragma unroll
            for (int f = 0; f < kWFlight; ++f)
                dx[f] = xs[f] >= 0 ? a.dist[w_at(a, xs[f], j, lane)] : kWUnreached;
            // the batch's decrements are issued together; a lane whose
            // decrement took the last predecessor (left 1) is released
            uint32_t left[kWFlight];
#pragma unroll
            for (int f = 0; f < kWFlight; ++f) {
                left[f] = 0u;
                if (xs[f] >= 0 && on && dv + ws[f] == dx[f])
                    left[f] = atomicSub(&a.pend[w_at(a, xs[f], j, lane)], 1u);
            }
#pragma unroll
            for (int f = 0; f < kWFlight; ++f) {
                if (xs[f] < 0) break;
                const uint64_t bal = wave_ballot(left[f] == 1u);
                if (bal) {
                    const uint32_t xw = ((uint32_t)xs[f] << a.logW) + j;
                    if (w_mark(&a.rdy[xw], bal, lane))
                        q.push(xw, 0ull, &a.ctl[CTL_TAIL], a.ord, nullptr, lane);
                }
            }
        }
    }
    q.flush(&a.ctl[CTL_TAIL], a.ord, nullptr, lane);
}

// Path counts, second half: each word of ord[s0, s1) (queued by the previous
// half) takes its released lanes, and each such lane sums its DAG
// predecessors' counts over the in-row in CSR order.
__global__ __launch_bounds__(kBlock) void k_ww_sigma(WArgs a, int64_t s0, int64_t s1)
{
    const int lane = lane_id();
    const uint32_t jm = (1u << a.logW) - 1u;
    unsigned long long ua = 0, ub = 0;
    for (int64_t i = s0 + w_wave_id(); i < s1; i += w_waves()) {
        const uint32_t wi = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.ord[i]);
        const uint64_t m = uniform_u64(a.rdy[wi]);
        if (lane == 0) {
            a.rdy[wi] = 0ull;
            a.omask[i] = m;
        }
        const int64_t v = wi >> a.logW;
        const uint32_t j = wi & jm;
        const bool on = (m >> lane) & 1ull;
        const int64_t e = ((int64_t)wi << 6) + lane;
        const int32_t dv = a.dist[e];
        const int64_t r0 = a.rrow[v], r1 = a.rrow[v + 1];
        ua += (unsigned long long)__popcll(m);
        ub += (unsigned long long)__popcll(m) * (unsigned long long)(r1 - r0);
        double acc = 0.0;
        for (int64_t r = r0; r < r1; r += kWFlight) {
            int32_t us[kWFlight], ws[kWFlight], du[kWFlight];
            bool pr[kWFlight];
            double su[kWFlight];
#pragma unroll
            for (int f = 0; f < kWFlight; ++f) {
                const bool ok = r + f < r1;
                us[f] = ok ? a.rcol[r + f] : -1;
                ws[f] = ok ? a.rwt[r + f] : 0;
            }
#pragma unroll
            for (int f = 0; f < kWFlight; ++f)
                du[f] = us[f] >= 0 ? a.dist[w_at(a, us[f], j, lane)] : kWUnreached;
#pragma unroll
            for (int f = 0; f < kWFlight; ++f) {
                pr[f] = on && du[f] != kWUnreached && du[f] + ws[f] == dv;
                su[f] = wave_ballot(pr[f]) ? a.sig[w_at(a, us[f], j, lane)] : 0.0;
            }
#pragma unroll
            for (int f = 0; f < kWFlight; ++f)
                if (pr[f]) acc += su[f];
        }
        if (on) {
            a.sig[e] = acc;
            if (!(acc < 0x1p1000)) a.ctl[CTL_SIG_OVERFLOW] = 1ull;
        }
    }
    if (a.prof) prof_add_raw(a.prof, PROF_W_COUNTS, ua, ub);
}

// Theorem 1 for the words of ord[s0, s1), one round (every successor lane is
// in a later round): delta(v) = sigma(v) * sum over DAG successors w, in CSR
// order, of rho(w); then rho(v) = (term(v) + delta(v)) / sigma(v), term 1 (pair
// mode: 1 only at the lane's destination).
__global__ __launch_bounds__(kBlock) void k_ww_backward(WArgs a, int64_t s0, int64_t s1)
{
    const int lane = lane_id();
    const uint32_t jm = (1u << a.logW) - 1u;
    unsigned long long ua = 0, ub = 0;
    for (int64_t i = s0 + w_wave_id(); i < s1; i += w_waves()) {
        const uint32_t wi = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.ord[i]);
        const uint64_t m = uniform_u64(a.omask[i]);
        const int64_t v = wi >> a.logW;
        const uint32_t j = wi & jm;
        const bool on = (m >> lane) & 1ull;
        const int64_t e = ((int64_t)wi << 6) + lane;
        const int32_t dv = a.dist[e];
        const int64_t r0 = a.row[v], r1 = a.row[v + 1];
        ua += (unsigned long long)__popcll(m);
        ub += (unsigned long long)__popcll(m) * (unsigned long long)(r1 - r0);
        double acc = 0.0;
        for (int64_t r = r0; r < r1; r += kWFlight) {
            int32_t xs[kWFlight], ws[kWFlight], dx[kWFlight];
            bool sc[kWFlight];
            double rx[kWFlight];
#pragma unroll
            for (int f = 0; f < kWFlight; ++f) {
                const bool ok = r + f < r1;
                xs[f] = ok ? a.col[r + f] : -1;
                ws[f] = ok ? a.wt[r + f] : 0;
            }
#pragma unroll
            for (int f = 0; f < kWFlight; ++f)
                dx[f] = xs[f] >= 0 ? a.dist[w_at(a, xs[f], j, lane)] : kWUnreached;
#pragma unroll
            for (int f = 0; f < kWFlight; ++f) {
                sc[f] = on && xs[f] >= 0 && dv + ws[f] == dx[f];
                rx[f] = wave_ballot(sc[f]) ? a.rho[w_at(a, xs[f], j, lane)] : 0.0;
            }
#pragma unroll
            for (int f = 0; f < kWFlight; ++f)
                if (sc[f]) acc += rx[f];
        }
        if (on) {
            const int b = (int)(j << 6) + lane;
            const double sv = a.sig[e];
            const double d = sv * acc;
            const double term = a.dest ? (a.dest[b] == (int32_t)v ? 1.0 : 0.0) : 1.0;
            a.dlt[e] = d;
            a.rho[e] = (term + d) / sv;
        }
    }
    if (a.prof) prof_add_raw(a.prof, PROF_W_BACKWARD, ua, ub);
}

// ------------------------------------------------------------- outputs

// out[v] += the dependencies of v's reached lanes (the source lane holds 0),
// word by word in a fixed tree per word
__global__ __launch_bounds__(kBlock) void k_ww_out_sum(WArgs a, double *out)
{
    const int lane = lane_id();
    const int W = 1 << a.logW;
    for (int64_t v = w_wave_id(); v < a.n; v += w_waves()) {
        double acc = 0.0;
        for (int j = 0; j < W; ++j) {
            const double x = a.dlt[w_at(a, v, (uint32_t)j, lane)];
            acc += w_wave_sum(x);
        }
        if (lane == 0) out[v] += acc;
    }
}

// row b0 + b of a source-major [count][n] output from lane b
template <class F>
__device__ __forceinline__ void w_rows_out(const WArgs &a, int32_t count, F f)
{
    const int64_t total = a.n * count;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(i / a.n);
        const int64_t v = i - (int64_t)b * a.n;
        f(i, (v << (a.logW + 6)) + b);
    }
}

__global__ void k_ww_out_full(WArgs a, int32_t count, int64_t b0, double *out)
{
    w_rows_out(a, count, [&](int64_t i, int64_t e) { out[b0 * a.n + i] = a.dlt[e]; });
}

__global__ void k_ww_out_dist(WArgs a, int32_t count, int64_t b0, int32_t *out)
{
    w_rows_out(a, count, [&](int64_t i, int64_t e) {
        const int32_t d = a.dist[e];
        out[b0 * a.n + i] = d == kWUnreached ? -1 : d;
    });
}

__global__ void k_ww_out_sigma(WArgs a, int32_t count, int64_t b0, double *mant, int32_t *ex)
{
    w_rows_out(a, count, [&](int64_t i, int64_t e) {
        const XNum x = xnorm(a.dist[e] == kWUnreached ? 0.0 : a.sig[e], 0);
        if (mant) mant[b0 * a.n + i] = x.m;
        if (ex) ex[b0 * a.n + i] = x.e;
    });
}

// out[(b0 + b) * T + t] = delta of lane b at targets[t]
__global__ void k_ww_out_targets(WArgs a, const int32_t *targets, int32_t T, int32_t count,
                                 int64_t b0, double *out)
{
    const int64_t total = (int64_t)count * T;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(i / T);
        const int t = (int)(i - (int64_t)b * T);
        out[(b0 + b) * T + t] = a.dlt[((int64_t)targets[t] << (a.logW + 6)) + b];
    }
}

// X[t * stride + b] = delta of lane b at targets[t] (0 past the valid lanes)
__global__ void k_ww_gather_targets(WArgs a, const int32_t *targets, int32_t T, int32_t stride,
                                    double *X)
{
    const int64_t total = (int64_t)T * stride;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(i / stride);
        const int b = (int)(i - (int64_t)t * stride);
        X[i] = b < a.nvalid ? a.dlt[((int64_t)targets[t] << (a.logW + 6)) + b] : 0.0;
    }
}

}  // namespace bcmi
