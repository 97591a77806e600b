// Balanced bidirectional search for pair samples.
//
// A pair sample (u, v) needs, for every vertex t, the fraction of shortest
// u-v paths through t: sigma_ut * sigma_tv / sigma_uv where d(u,t) + d(t,v) =
// d(u,v) (Algorithm 1's term; Section 6.2 stops the pair's search once v is
// reached). Here the search grows from both ends: side 0 from u over
// out-arcs, side 1 from v over in-arcs, each step expanding the side whose
// frontier has fewer arcs to walk, until an expansion finds a vertex the other
// side holds. Then d(u,v) = D = d0 + d1 (the two depths), and the vertices
// found by that expansion that the other side holds (the meeting set M) lie
// at distance d0 from u and d1 from v. Two backward sweeps complete the counts
// on the shortest paths only:
//   side 0, levels L = d0-1 .. 0: sigma_wv = sum of sigma_xv over the out-
//     neighbours x of w at level L+1 that lie on a shortest path;
//   side 1, levels L = d1-1 .. 0: sigma_uw = sum of sigma_ux over the in-
//     neighbours x of w at level L+1 that lie on a shortest path.
// A vertex lies on a shortest path when both sides hold it with distances
// summing to D: the sweeps give every such vertex the other side's stamp
// before its sum is pulled (a mark step from the level above), so the
// stamps alone say which values to read. Each side's ball inside the meeting
// level is disjoint from the other side's, so a vertex's sigma toward the far
// end is stored in the other side's count array. sigma_uv is side 0's sweep
// value at u.
//
// One workgroup serves one pair at a time in its own slot of per-vertex state.
// A stamp holds (epoch << 32 | distance); every pair a slot serves gets a new
// epoch, so nothing is cleared between pairs. Sums walk a row in CSR order
// (one thread) or strided over a wavefront's lanes with a fixed reduction
// tree (rows longer than kBiSmall), so results do not depend on the order in
// which vertices were found.

namespace bcmi {

constexpr int kBiBlock = 256;
static_assert(kBiBlock == kBlock, "k_bidir runs on the common workgroup size");
constexpr int kBiSmall = 32;   // rows up to this many arcs are walked by one thread

// long rows a phase queues in LDS; more take a second scan of the range
constexpr int kRowQ = 512;

// The queue of long rows shared by a workgroup's phases (bi_rows). Its count
// rotates over three slots: phase k appends to slot k % 3 and clears slot
// (k+1) % 3 before its barrier; the last read of that slot (phase k-2, after
// its own barrier) and the next appends (phase k+1, after phase k's barrier)
// are both ordered with the clear by barriers.
struct RowQ {
    int32_t w[kRowQ];
    int cnt[3];
    int ovf[3];
};

// before the first phase; a barrier must follow before the first bi_rows
__device__ __forceinline__ void rowq_init(RowQ &rq)
{
    if (threadIdx.x < 3) {
        rq.cnt[threadIdx.x] = 0;
        rq.ovf[threadIdx.x] = 0;
    }
}


struct BiArgs {
    // adjacency by direction: [0] out-arcs, [1] in-arcs. Side s expands over
    // adj[s] and sums path counts over adj[1 - s].
    const int64_t *row[2];
    const int32_t *col[2];
    int64_t n;
    const int32_t *us;     // [count] pair ends
    const int32_t *vs;
    int32_t count;
    uint64_t *st[2];       // [slots][n] stamps
    double *val[2];        // [slots][n] side 0: sigma_uw; side 1: sigma_wv
    int32_t *q[2];         // [slots][n] vertices in the order the side found them
    int32_t *lo[2];        // [slots][n + 2] first list position of each level
    uint32_t epoch0;       // a slot's i-th pair of this launch has epoch epoch0 + i + 1
    unsigned long long *ctl;
    unsigned long long *prof;
    const int32_t *targets;
    int32_t T;
    int32_t stride;
    double *X;             // X[t * stride + pair] for the T targets, or null
    const int32_t *ptgt;   // [count] one target per pair: X[pair] = its value (T = 0), or null
    double *full;          // full[pair * n + w] (zero on entry), or null
};

struct BiShared {
    RowQ rq;
    int cnt;                 // vertices found by the current expansion
    int meet;                // the expansion found a vertex of the other side
    unsigned long long vol;  // arcs the new frontier will walk
};

__device__ __forceinline__ uint64_t bi_stamp(uint32_t ep, uint32_t d)
{
    return ((uint64_t)ep << 32) | d;
}

__device__ __forceinline__ bool bi_held(uint64_t st, uint32_t ep)
{
    return (uint32_t)(st >> 32) == ep;
}

// Append among the active lanes of a wavefront: one LDS atomic on *cnt for
// all lanes with want set; returns each such lane's slot (others: unused).
// Safe in divergent code (only active lanes take part).
__device__ __forceinline__ int bi_append(bool want, int *cnt)
{
    const uint64_t bal = __ballot(want);
    if (!want) return 0;
    const int leader = __ffsll((unsigned long long)bal) - 1;
    const int lane = threadIdx.x & (kWave - 1);
    int base = 0;
    if (lane == leader) base = atomicAdd(cnt, __popcll(bal));
    base = __shfl(base, leader, kWave);
    return base + __popcll(bal & ((1ull << lane) - 1ull));
}

// lane 0 receives the sum over the wavefront, added in a fixed tree
__device__ __forceinline__ double bi_wave_sum(double x)
{
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) x += __shfl_down(x, off, kWave);
    return x;
}

// For each list entry w = q[i], i in [a, b), that take(w) accepts: a row of at
// most kBiSmall arcs goes to one thread as small(w, r0, r1); a longer one to a
// wavefront as big(w, r0, r1, lane), from the LDS queue (or, when more than
// kRowQ long rows came up, by a second scan in which each wavefront's ballot
// finds them 64 entries at a time). A long row is walked the same way either
// way. Ends with a barrier (two when long rows came up); a, b must be uniform
// over the workgroup, take(w) must read nothing the phase writes, and every
// thread passes the same phase counter (from 0, after rowq_init).
template <int kThreads = kBiBlock, class Take, class Small, class Big>
__device__ __forceinline__ void bi_rows(RowQ &rq, int &phase, const int32_t *q, int a, int b,
                                        const int64_t *row, Take take, Small small, Big big)
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int k = phase % 3;
    phase += 1;
    if (threadIdx.x == 0) {
        rq.cnt[(k + 1) % 3] = 0;
        rq.ovf[(k + 1) % 3] = 0;
    }
    for (int i = a + (int)threadIdx.x; i < b; i += kThreads) {
        const int32_t w = q[i];
        if (!take(w)) continue;
        const int64_t r0 = row[w], r1 = row[w + 1];
        if (r1 - r0 <= kBiSmall) {
            small(w, r0, r1);
        } else {
            const int at = bi_append(true, &rq.cnt[k]);
            if (at < kRowQ) rq.w[at] = w;
            else rq.ovf[k] = 1;
        }
    }
    __syncthreads();
    const int qc = rq.cnt[k];
    if (qc == 0) return;
    if (!rq.ovf[k]) {
        for (int j = wave; j < qc; j += kThreads / kWave) {
            const int32_t w = rq.w[j];
            big(w, row[w], row[w + 1], lane);
        }
    } else {
        for (int c = a + wave * kWave; c < b; c += kThreads) {
            const int i = c + lane;
            int32_t w = 0;
            int64_t r0 = 0, r1 = 0;
            bool longrow = false;
            if (i < b) {
                w = q[i];
                if (take(w)) {
                    r0 = row[w];
                    r1 = row[w + 1];
                    longrow = r1 - r0 > kBiSmall;
                }
            }
            uint64_t m = __ballot(longrow);
            while (m) {
                const int src = __ffsll((unsigned long long)m) - 1;
                m &= m - 1;
                const int32_t wb = __shfl(w, src, kWave);
                const int64_t b0 = __shfl(r0, src, kWave), b1 = __shfl(r1, src, kWave);
                big(wb, b0, b1, lane);
            }
        }
    }
    __syncthreads();
}

// Sum of val[x] over the arcs [r0, r1) of `col` whose head x passes ok(x):
// in CSR order by one thread, or by a wavefront (lanes strided, lane 0 gets
// the total) for long rows.
template <class Ok>
__device__ __forceinline__ double bi_sum_thread(const int32_t *col, int64_t r0, int64_t r1,
                                                const double *val, Ok ok)
{
    double x = 0.0;
    for (int64_t e = r0; e < r1; ++e) {
        const int32_t y = col[e];
        if (ok(y)) x += val[y];
    }
    return x;
}

template <class Ok>
__device__ __forceinline__ double bi_sum_wave(const int32_t *col, int64_t r0, int64_t r1,
                                              const double *val, Ok ok, int lane)
{
    double x = 0.0;
    for (int64_t e = r0 + lane; e < r1; e += kWave) {
        const int32_t y = col[e];
        if (ok(y)) x += val[y];
    }
    return bi_wave_sum(x);
}

__device__ __forceinline__ void bi_check(const BiArgs &a, double x)
{
    if (!(x < 0x1p1000)) a.ctl[CTL_SIG_OVERFLOW] = 1ull;
}

__global__ void __launch_bounds__(kBiBlock) k_bidir(BiArgs a)
{
    __shared__ BiShared sh;
    const int64_t base = (int64_t)blockIdx.x * a.n;
    uint64_t *st[2] = {a.st[0] + base, a.st[1] + base};
    double *val[2] = {a.val[0] + base, a.val[1] + base};
    int32_t *q[2] = {a.q[0] + base, a.q[1] + base};
    int32_t *lo[2] = {a.lo[0] + (int64_t)blockIdx.x * (a.n + 2),
                      a.lo[1] + (int64_t)blockIdx.x * (a.n + 2)};
    unsigned long long ua = 0, ub = 0;
    int phase = 0;
    rowq_init(sh.rq);   // ordered before the first phase by the loop's barriers

    uint32_t i = 0;
    for (int p = blockIdx.x; p < a.count; p += gridDim.x, ++i) {
        const uint32_t ep = a.epoch0 + i + 1u;
        const int32_t u = a.us[p], v = a.vs[p];
        __syncthreads();   // the previous pair's output is read
        if (threadIdx.x == 0 && u != v) {
            st[0][u] = bi_stamp(ep, 0);
            val[0][u] = 1.0;
            q[0][0] = u;
            lo[0][0] = 0;
            lo[0][1] = 1;
            st[1][v] = bi_stamp(ep, 0);
            val[1][v] = 1.0;
            q[1][0] = v;
            lo[1][0] = 0;
            lo[1][1] = 1;
        }
        __syncthreads();
        int depth[2] = {0, 0};
        int f0[2] = {0, 0}, f1[2] = {1, 1};   // list range of each side's frontier
        unsigned long long vol[2] = {(unsigned long long)(a.row[0][u + 1] - a.row[0][u]),
                                     (unsigned long long)(a.row[1][v + 1] - a.row[1][v])};
        bool met = false;
        while (u != v) {
            const int s = vol[0] <= vol[1] ? 0 : 1;
            if (vol[s] == 0) break;            // that side cannot grow: v unreachable
            const int o = 1 - s;
            const int L = depth[s];
            if (threadIdx.x == 0) {
                sh.cnt = 0;
                sh.meet = 0;
                sh.vol = 0;
            }
            __syncthreads();
            const uint64_t nst = bi_stamp(ep, (uint32_t)(L + 1));
            const int32_t *ecol = a.col[s];
            const int64_t *erow = a.row[s];
            const int put = f1[s];
            auto visit = [&](int32_t y) {
                const uint64_t old = st[s][y];
                const bool got = !bi_held(old, ep) &&
                                 atomicCAS((unsigned long long *)&st[s][y],
                                           (unsigned long long)old,
                                           (unsigned long long)nst) == old;
                const int at = bi_append(got, &sh.cnt);
                if (got) {
                    q[s][put + at] = y;
                    atomicAdd(&sh.vol, (unsigned long long)(erow[y + 1] - erow[y]));
                    ++ua;
                }
                if (bi_held(st[o][y], ep)) sh.meet = 1;
            };
            bi_rows(
                sh.rq, phase, q[s], f0[s], f1[s], erow, [](int32_t) { return true; },
                [&](int32_t, int64_t r0, int64_t r1) {
                    ub += (unsigned long long)(r1 - r0);
                    for (int64_t e = r0; e < r1; ++e) visit(ecol[e]);
                },
                [&](int32_t, int64_t r0, int64_t r1, int lane) {
                    for (int64_t e = r0 + lane; e < r1; e += kWave) {
                        ++ub;
                        visit(ecol[e]);
                    }
                });
            const int cnt = sh.cnt;
            const bool meet = sh.meet != 0;
            vol[s] = sh.vol;
            if (cnt == 0) break;               // nothing new: v unreachable
            depth[s] = L + 1;
            f0[s] = put;
            f1[s] = put + cnt;
            if (threadIdx.x == 0) lo[s][L + 2] = put + cnt;
            // path counts of the new level (only the meeting set's once the
            // sides have met: no other vertex of that level is on a path)
            const uint64_t pst = bi_stamp(ep, (uint32_t)L);
            const int32_t *pcol = a.col[o];
            auto from_level = [&](int32_t x) { return st[s][x] == pst; };
            bi_rows(
                sh.rq, phase, q[s], put, put + cnt, a.row[o],
                [&](int32_t w) { return !meet || bi_held(st[o][w], ep); },
                [&](int32_t w, int64_t r0, int64_t r1) {
                    ub += (unsigned long long)(r1 - r0);
                    const double x = bi_sum_thread(pcol, r0, r1, val[s], from_level);
                    val[s][w] = x;
                    bi_check(a, x);
                },
                [&](int32_t w, int64_t r0, int64_t r1, int lane) {
                    ub += (unsigned long long)((r1 - r0 + kWave - 1 - lane) / kWave);
                    const double x = bi_sum_wave(pcol, r0, r1, val[s], from_level, lane);
                    if (lane == 0) {
                        val[s][w] = x;
                        bi_check(a, x);
                    }
                });
            if (meet) {
                met = true;
                break;
            }
        }

        const uint32_t D = (uint32_t)(depth[0] + depth[1]);
        if (met) {
            // the sweeps, side 0 then side 1, each from its deepest level up
            for (int s = 0; s < 2; ++s) {
                const int o = 1 - s;
                for (int L = depth[s] - 1; L >= 0; --L) {
                    const uint64_t here = bi_stamp(ep, (uint32_t)L);
                    const uint64_t above = bi_stamp(ep, (uint32_t)(L + 1));
                    const uint64_t far_here = bi_stamp(ep, D - (uint32_t)L);
                    const uint64_t far_above = bi_stamp(ep, D - (uint32_t)L - 1u);
                    const int lA = lo[s][L + 1], lB = lo[s][L + 2], l0 = lo[s][L];
                    // mark: level-L neighbours (over adj[o]) of the on-path
                    // vertices of level L+1 are on a path
                    const int32_t *mcol = a.col[o];
                    auto mark = [&](int32_t y) {
                        if (st[s][y] == here) st[o][y] = far_here;
                    };
                    bi_rows(
                        sh.rq, phase, q[s], lA, lB, a.row[o],
                        [&](int32_t x) { return st[o][x] == far_above; },
                        [&](int32_t, int64_t r0, int64_t r1) {
                            ub += (unsigned long long)(r1 - r0);
                            for (int64_t e = r0; e < r1; ++e) mark(mcol[e]);
                        },
                        [&](int32_t, int64_t r0, int64_t r1, int lane) {
                            for (int64_t e = r0 + lane; e < r1; e += kWave) {
                                ++ub;
                                mark(mcol[e]);
                            }
                        });
                    // pull: a marked vertex sums its on-path successors (over adj[s])
                    const int32_t *scol = a.col[s];
                    auto on_above = [&](int32_t x) {
                        return st[s][x] == above && st[o][x] == far_above;
                    };
                    bi_rows(
                        sh.rq, phase, q[s], l0, lA, a.row[s],
                        [&](int32_t w) { return st[o][w] == far_here; },
                        [&](int32_t w, int64_t r0, int64_t r1) {
                            ub += (unsigned long long)(r1 - r0);
                            const double x = bi_sum_thread(scol, r0, r1, val[o], on_above);
                            val[o][w] = x;
                            bi_check(a, x);
                        },
                        [&](int32_t w, int64_t r0, int64_t r1, int lane) {
                            ub += (unsigned long long)((r1 - r0 + kWave - 1 - lane) / kWave);
                            const double x = bi_sum_wave(scol, r0, r1, val[o], on_above, lane);
                            if (lane == 0) {
                                val[o][w] = x;
                                bi_check(a, x);
                            }
                        });
                }
            }
        }

        // outputs: sigma_uw * sigma_wv / sigma_uv on the shortest paths
        const double suv = met ? val[1][u] : 0.0;
        auto value = [&](int32_t w) {
            if (!met || w == u || w == v) return 0.0;
            const uint64_t s0 = st[0][w], s1 = st[1][w];
            if (!bi_held(s0, ep) || !bi_held(s1, ep) || (uint32_t)s0 + (uint32_t)s1 != D)
                return 0.0;
            return val[0][w] * val[1][w] / suv;
        };
        if (a.X)
            for (int t = threadIdx.x; t < a.T; t += kBiBlock)
                a.X[(int64_t)t * a.stride + p] = value(a.targets[t]);
        if (a.ptgt && threadIdx.x == 0) a.X[p] = value(a.ptgt[p]);
        if (a.full && met)
            for (int s = 0; s < 2; ++s) {
                const int end = lo[s][depth[s] + 1];
                for (int k = threadIdx.x; k < end; k += kBiBlock) {
                    const int32_t w = q[s][k];
                    const double x = value(w);
                    if (x != 0.0) a.full[(int64_t)p * a.n + w] = x;
                }
            }
    }
    if (a.prof) prof_add_raw(a.prof, PROF_BIDIR, wave_sum_u64(ua), wave_sum_u64(ub));
}

}  // namespace bcmi
