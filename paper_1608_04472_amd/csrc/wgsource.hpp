// One workgroup per source: Brandes' pass with workgroup barriers only.
//
// On graphs of large diameter (a 2048 x 2048 grid has about 4,000 BFS
// levels) the batched engines spend their time on one device-wide step per
// level. Here each workgroup runs whole passes (Section 3's two steps,
// Definition 3's counts, Theorem 1's sums) for its sources, one after another,
// in its own slot of per-vertex state: a level is a range of the slot's
// visiting list, its vertices are found by walking the previous level's rows
// (a CAS on the distance admits each vertex once), and the barriers between
// levels are the workgroup's own. Counts and dependencies are pulled in CSR
// order (one thread per row, or a wavefront with a fixed reduction tree for
// rows longer than kBiSmall), so values do not depend on the order in which
// a level's vertices were found. A slot's distances are stored above a base
// that each pass moves past the levels it used, so a vertex is new to the
// pass when its stored value is below the base and nothing is reset between
// sources (when the base nears the int32 range the slot is cleared once).

namespace bcmi {

// threads per workgroup: a pass's levels are walked by all of them, so a wide
// workgroup keeps more of a level's loads in flight per source
constexpr int kWgBlock = 1024;
// arcs of a thread's row whose loads are issued together (a group's heads,
// then their records, before any is used)
constexpr int kWgFlight = 8;

// a vertex's state in a slot: the fields a pull reads together share one line
struct WgVert {
    int32_t dist;   // base of the pass + level; below the base = unseen
    int32_t sige;   // count exponent (extended mode)
    double sig;     // count (mantissa in extended mode)
    double dlt;     // dependency
    double sum;     // the slot's dependency sum over its passes (BC_OUT_SUM)
};
static_assert(sizeof(WgVert) == 32, "two vertices per 64-byte sector");

struct WgArgs {
    const int64_t *row;    // out-arcs: discovery, Theorem 1's successors
    const int32_t *col;
    const int64_t *rrow;   // in-arcs: Definition 3's predecessors
    const int32_t *rcol;
    int64_t n;
    const int32_t *srcs;   // [count]
    const int32_t *dest;   // [count] pair destinations (pair mode), or null
    int32_t count;
    WgVert *vert;          // [slots][n] per-vertex state
    int32_t *base;         // [slots] the next pass's base (0 with every dist -1 at first)
    int32_t *q;            // [slots][n] vertices in visiting order
    int32_t *lo;           // [slots][n + 1] first list position of each level
    int32_t sum;           // BC_OUT_SUM: add each pass's dependencies to WgVert::sum
    double *full;          // full[i * n + v] (rows zeroed by the caller), or null
    double *tgt;           // tgt[i * T + t] for the targets, or null
    const int32_t *targets;
    int32_t T;
    int32_t *dist_out;     // rows of distances (-1 filled by the caller), or null
    double *sig_m;         // rows of count mantissas / exponents (0 filled), or null
    int32_t *sig_e;
    unsigned long long *ctl;
    unsigned long long *prof;
};

struct WgShared {
    RowQ rq;
    int cnt;      // vertices found by the current level
    int found;    // pair mode: the destination is among them
};

template <bool kExt>
__global__ void __launch_bounds__(kWgBlock) k_wg(WgArgs a)
{
    __shared__ WgShared sh;
    const int64_t n = a.n;
    const int64_t base = (int64_t)blockIdx.x * n;
    WgVert *vx = a.vert + base;
    int32_t *q = a.q + base;
    int32_t *lo = a.lo + (int64_t)blockIdx.x * (n + 1);
    unsigned long long ua = 0, ub = 0;
    int phase = 0;
    rowq_init(sh.rq);   // ordered before the first phase by the loop's barriers
    int32_t b0 = a.base[blockIdx.x];
    const bool rows_out = a.full || a.dist_out || a.sig_m || a.sig_e;

    for (int i = blockIdx.x; i < a.count; i += gridDim.x) {
        const int32_t s = a.srcs[i];
        const int32_t dst = a.dest ? a.dest[i] : -1;
        if (b0 > 0x7fffffff - (int32_t)n - 2) {
            // the base would leave the int32 range: clear the slot once
            __syncthreads();
            for (int64_t v = threadIdx.x; v < n; v += kWgBlock) vx[v].dist = -1;
            b0 = 0;
        }
        __syncthreads();   // the previous pass's outputs are read
        if (threadIdx.x == 0) {
            vx[s].dist = b0;
            vx[s].sig = 1.0;
            if (kExt) vx[s].sige = 0;
            vx[s].dlt = 0.0;
            q[0] = s;
            lo[0] = 0;
            lo[1] = 1;
        }
        int L = 0, f0 = 0, f1 = 1;
        // forward: discovery, then the new level's counts
        for (;;) {
            if (threadIdx.x == 0) {
                sh.cnt = 0;
                sh.found = 0;
            }
            __syncthreads();
            const int32_t nd = b0 + L + 1;
            auto visit_from = [&](int32_t w, int32_t old) {
                const bool got = old < b0 && atomicCAS(&vx[w].dist, old, nd) == old;
                const int at = bi_append(got, &sh.cnt);
                if (got) {
                    q[f1 + at] = w;
                    ++ua;
                    if (w == dst) sh.found = 1;
                }
            };
            bi_rows<kWgBlock>(
                sh.rq, phase, q, f0, f1, a.row, [](int32_t) { return true; },
                [&](int32_t, int64_t r0, int64_t r1) {
                    ub += (unsigned long long)(r1 - r0);
                    for (int64_t e = r0; e < r1; e += kWgFlight) {
                        int32_t y[kWgFlight], old[kWgFlight];
#pragma unroll
                        for (int f = 0; f < kWgFlight; ++f) y[f] = e + f < r1 ? a.col[e + f] : -1;
#pragma unroll
                        for (int f = 0; f < kWgFlight; ++f) old[f] = vx[y[f] >= 0 ? y[f] : y[0]].dist;
#pragma unroll
                        for (int f = 0; f < kWgFlight; ++f)
                            if (y[f] >= 0) visit_from(y[f], old[f]);
                    }
                },
                [&](int32_t, int64_t r0, int64_t r1, int lane) {
                    for (int64_t e = r0 + lane; e < r1; e += kWave) {
                        ++ub;
                        const int32_t w = a.col[e];
                        visit_from(w, vx[w].dist);
                    }
                });
            const int cnt = sh.cnt;
            const bool found = sh.found != 0;
            if (cnt == 0) break;
            if (threadIdx.x == 0) lo[L + 2] = f1 + cnt;
            const int32_t pl = b0 + L;
            auto pred = [&](int32_t u) { return vx[u].dist == pl; };
            bi_rows<kWgBlock>(
                sh.rq, phase, q, f1, f1 + cnt, a.rrow, [](int32_t) { return true; },
                [&](int32_t w, int64_t r0, int64_t r1) {
                    ub += (unsigned long long)(r1 - r0);
                    // the same additions in CSR order; a group's records are
                    // loaded together (a non-predecessor adds +0.0 to a
                    // non-negative sum, or nothing in extended form)
                    XNum x{0.0, 0};
                    double xp = 0.0;
                    for (int64_t e = r0; e < r1; e += kWgFlight) {
                        int32_t u[kWgFlight], d[kWgFlight], ue[kWgFlight];
                        double us[kWgFlight];
#pragma unroll
                        for (int f = 0; f < kWgFlight; ++f) u[f] = e + f < r1 ? a.rcol[e + f] : -1;
#pragma unroll
                        for (int f = 0; f < kWgFlight; ++f) {
                            const WgVert &r = vx[u[f] >= 0 ? u[f] : u[0]];
                            d[f] = r.dist;
                            us[f] = r.sig;
                            ue[f] = kExt ? r.sige : 0;
                        }
#pragma unroll
                        for (int f = 0; f < kWgFlight; ++f) {
                            const bool p = u[f] >= 0 && d[f] == pl;
                            if (kExt) {
                                if (p) x = xadd(x, XNum{us[f], ue[f]});
                            } else {
                                xp += p ? us[f] : 0.0;
                            }
                        }
                    }
                    if (kExt) {
                        vx[w].sig = x.m;
                        vx[w].sige = x.e;
                    } else {
                        vx[w].sig = xp;
                        if (!(xp < 0x1p1000)) a.ctl[CTL_SIG_OVERFLOW] = 1ull;
                    }
                },
                [&](int32_t w, int64_t r0, int64_t r1, int lane) {
                    ub += (unsigned long long)((r1 - r0 + kWave - 1 - lane) / kWave);
                    if (kExt) {
                        // lanes strided, then the lane sums in a fixed tree
                        XNum x{0.0, 0};
                        for (int64_t e = r0 + lane; e < r1; e += kWave) {
                            const int32_t u = a.rcol[e];
                            if (pred(u)) x = xadd(x, XNum{vx[u].sig, vx[u].sige});
                        }
#pragma unroll
                        for (int off = kWave / 2; off >= 1; off >>= 1) {
                            const XNum y{__shfl_down(x.m, off, kWave),
                                         __shfl_down(x.e, off, kWave)};
                            x = xadd(x, y);
                        }
                        if (lane == 0) {
                            vx[w].sig = x.m;
                            vx[w].sige = x.e;
                        }
                    } else {
                        double x = 0.0;
                        for (int64_t e = r0 + lane; e < r1; e += kWave) {
                            const int32_t u = a.rcol[e];
                            if (pred(u)) x += vx[u].sig;
                        }
                        x = bi_wave_sum(x);
                        if (lane == 0) {
                            vx[w].sig = x;
                            if (!(x < 0x1p1000)) a.ctl[CTL_SIG_OVERFLOW] = 1ull;
                        }
                    }
                });
            f0 = f1;
            f1 += cnt;
            ++L;
            if (found) break;   // pair mode: the destination's level is complete
        }
        // backward, deepest level first (the source keeps 0): Theorem 1 with
        // term 1, or in pair mode 1 only at the destination
        for (int l = L; l >= 1; --l) {
            const int32_t nl = b0 + l + 1;
            auto contrib = [&](int32_t v, int32_t w) -> double {
                const double term = dst >= 0 ? (w == dst ? 1.0 : 0.0) : 1.0;
                double r;
                if (kExt) r = ldexp(vx[v].sig / vx[w].sig, vx[v].sige - vx[w].sige);
                else r = vx[v].sig / vx[w].sig;
                return r * (term + vx[w].dlt);
            };
            bi_rows<kWgBlock>(
                sh.rq, phase, q, lo[l], lo[l + 1], a.row, [](int32_t) { return true; },
                [&](int32_t v, int64_t r0, int64_t r1) {
                    ub += (unsigned long long)(r1 - r0);
                    // contrib(v, w) from a group's records loaded together,
                    // added in CSR order for the successors only
                    const double sv = vx[v].sig;
                    const int32_t ev = kExt ? vx[v].sige : 0;
                    double x = 0.0;
                    for (int64_t e = r0; e < r1; e += kWgFlight) {
                        int32_t w[kWgFlight], d[kWgFlight], we[kWgFlight];
                        double ws[kWgFlight], wd[kWgFlight];
#pragma unroll
                        for (int f = 0; f < kWgFlight; ++f) w[f] = e + f < r1 ? a.col[e + f] : -1;
#pragma unroll
                        for (int f = 0; f < kWgFlight; ++f) {
                            const WgVert &r = vx[w[f] >= 0 ? w[f] : w[0]];
                            d[f] = r.dist;
                            ws[f] = r.sig;
                            wd[f] = r.dlt;
                            we[f] = kExt ? r.sige : 0;
                        }
#pragma unroll
                        for (int f = 0; f < kWgFlight; ++f) {
                            if (w[f] < 0 || d[f] != nl) continue;
                            const double term = dst >= 0 ? (w[f] == dst ? 1.0 : 0.0) : 1.0;
                            const double rr = kExt ? ldexp(sv / ws[f], ev - we[f]) : sv / ws[f];
                            x += rr * (term + wd[f]);
                        }
                    }
                    vx[v].dlt = x;
                    if (a.sum) vx[v].sum += x;
                },
                [&](int32_t v, int64_t r0, int64_t r1, int lane) {
                    ub += (unsigned long long)((r1 - r0 + kWave - 1 - lane) / kWave);
                    double x = 0.0;
                    for (int64_t e = r0 + lane; e < r1; e += kWave) {
                        const int32_t w = a.col[e];
                        if (vx[w].dist == nl) x += contrib(v, w);
                    }
                    x = bi_wave_sum(x);
                    if (lane == 0) {
                        vx[v].dlt = x;
                        if (a.sum) vx[v].sum += x;
                    }
                });
        }
        // rows of source i (every visited vertex: list positions [0, f1)); the
        // sum mode's additions were made by the backward
        if (rows_out)
            for (int k = threadIdx.x; k < f1; k += kWgBlock) {
                const int32_t v = q[k];
                const int64_t o = (int64_t)i * n + v;
                if (a.full) a.full[o] = k == 0 ? 0.0 : vx[v].dlt;
                if (a.dist_out) a.dist_out[o] = vx[v].dist - b0;
                if (a.sig_m || a.sig_e) {
                    const XNum x = xnorm(vx[v].sig, kExt ? vx[v].sige : 0);
                    if (a.sig_m) a.sig_m[o] = x.m;
                    if (a.sig_e) a.sig_e[o] = x.e;
                }
            }
        for (int t = threadIdx.x; t < a.T; t += kWgBlock) {
            const int32_t v = a.targets[t];
            a.tgt[(int64_t)i * a.T + t] = vx[v].dist > b0 ? vx[v].dlt : 0.0;
        }
        b0 += L + 2;   // past every level of this pass
    }
    if (threadIdx.x == 0) a.base[blockIdx.x] = b0;
    if (a.prof) prof_add_raw(a.prof, PROF_WG, wave_sum_u64(ua), wave_sum_u64(ub));
}

// every vertex of `cells` slots' states unseen (below any base)
__global__ void k_wg_clear(WgVert *vert, int64_t cells)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cells;
         i += (int64_t)gridDim.x * blockDim.x)
        vert[i].dist = -1;
}

// the slots' dependency sums to zero
__global__ void k_wg_zero_sum(WgVert *vert, int64_t cells)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cells;
         i += (int64_t)gridDim.x * blockDim.x)
        vert[i].sum = 0.0;
}

// out[v] += sum over slots (in slot order) of the slots' dependency sums
__global__ void k_wg_reduce(const WgVert *vert, int32_t slots, int64_t n, double *out)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        double acc = out[v];
        for (int32_t s = 0; s < slots; ++s) acc += vert[(int64_t)s * n + v].sum;
        out[v] = acc;
    }
}

}  // namespace bcmi
