// bcmi C ABI: graph handles, the batched level-synchronous Brandes engine,
// the per-source plain form, and the two adaptive samplers.
//
// Engine (one batch of B = 64 * 2^logW sources or pairs):
//   forward, level by level: discover the next level top-down (narrow
//   frontiers) or bottom-up (wide ones) as dense words, lay out the level's
//   record entries and pool segments by a prefix sum, pull path counts from
//   all predecessors, clear the retired frontier words;
//   backward, from the deepest recorded level up to level 1: pull rho from
//   successors (Theorem 1), write delta and the vertex's own rho.
// The host reads one 64-byte control block per level (queue tail, flags).
#include "../../include/bcmi.h"
#include "kernels.hpp"
#include "bidir.hpp"
#include "weighted.hpp"
#include "wgsource.hpp"

#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <array>
#include <chrono>
#include <limits>
#include <map>
#include <tuple>
#include <cmath>
#include <cstring>
#include <deque>
#include <exception>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <utility>
#include <vector>

using namespace bcmi;

namespace {

thread_local std::string tl_error;

struct Failure {
    bc_status status;
    std::string msg;
};

[[noreturn]] void fail(bc_status s, std::string m) { throw Failure{s, std::move(m)}; }

void hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess) return;
    fail(e == hipErrorOutOfMemory ? BC_E_NOMEM : BC_E_DEVICE,
         std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPX(expr) hip_check((expr), #expr)

// Device memory provider of a handle: the caller's bc_allocator, or hipMalloc.
// `forbid` marks the allocation-free entry point, where any attempt to
// allocate is an error.
struct Alloc {
    bc_allocator a{nullptr, nullptr, nullptr};
    bool forbid = false;
    void *get(size_t bytes) const
    {
        if (forbid) fail(BC_E_UNSUPPORTED, "the scratch array is too small for this request");
        void *p = nullptr;
        if (a.alloc) {
            p = a.alloc(bytes, a.ctx);
            if (!p) fail(BC_E_NOMEM, "the caller's allocator returned no memory");
        } else {
            HIPX(hipMalloc(&p, bytes));
        }
        return p;
    }
    void put(void *p) const
    {
        if (!p) return;
        if (a.free) a.free(p, a.ctx);
        else (void)hipFree(p);
    }
};

// The allocator of the handle the current ABI call works on (one per host
// thread; null = hipMalloc).
thread_local const Alloc *tl_alloc = nullptr;
// A stream whose work may still use buffers this thread frees: set while a
// server runs rounds on several streams, so that memory the caller's allocator
// hands out again is idle (buffers freed on one lane are not reused under
// another lane's pending work).
thread_local hipStream_t tl_sync = nullptr;

struct UseAlloc {
    const Alloc *prev;
    explicit UseAlloc(const Alloc *a) : prev(tl_alloc) { tl_alloc = a; }
    ~UseAlloc() { tl_alloc = prev; }
};

// A lazily grown device array. It remembers the allocator it came from, so it
// is released through that one. A view (set by `view`) borrows memory it does
// not own: it never grows and is never freed.
template <class T>
struct DBuf {
    T *p = nullptr;
    size_t cap = 0;
    const Alloc *from = nullptr;
    bool borrowed = false;
    void ensure(size_t count)
    {
        if (count <= cap) return;
        if (borrowed) fail(BC_E_UNSUPPORTED, "the scratch array is too small for this request");
        release();
        static const Alloc plain;
        const Alloc *al = tl_alloc ? tl_alloc : &plain;
        p = (T *)al->get(std::max<size_t>(count, 1) * sizeof(T));
        from = al == &plain ? nullptr : al;
        cap = count;
    }
    void view(T *mem, size_t count)
    {
        release();
        p = mem;
        cap = count;
        borrowed = true;
    }
    void release()
    {
        if (p && !borrowed) {
            if (tl_sync) (void)hipStreamSynchronize(tl_sync);
            if (from) from->put(p);
            else (void)hipFree(p);
        }
        p = nullptr;
        cap = 0;
        from = nullptr;
        borrowed = false;
    }
    size_t bytes() const { return cap * sizeof(T); }
};

int grid_for(int64_t threads)
{
    const int64_t b = (threads + kBlock - 1) / kBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 20));
}
// wave-per-entry kernels stride over their entries with at most 64K wavefronts
int grid_waves(int64_t waves)
{
    return std::min(grid_for(waves * kWave), 16384);
}

// tiled pull kernels: one workgroup per kTile entries, grid-strided
int grid_tiles(int64_t entries)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((entries + kTile - 1) / kTile, 32768));
}

template <class K, class... A>
void launch(hipStream_t st, dim3 grid, K kernel, A... args)
{
    hipLaunchKernelGGL(kernel, grid, dim3(kBlock), 0, st, args...);
    HIPX(hipGetLastError());
}

}  // namespace

// landmark vertices of the lane-order key (8 bits of distance each)
constexpr int kLandmarks = 8;
// batches of at least this many samples are reordered by the key
constexpr int64_t kOrderMin = 128;

// Device buffers of the engines. A graph owns one; graphs of a server share
// the server's (rounds on a server run one at a time on one stream).
struct Work {
    // wave engine
    DBuf<double> sig, dlt;
    DBuf<int32_t> sige;
    // F0, F1: the two rotating levels' (vertex, word) records, kFS words each
    // (lane mask, pool segment)
    DBuf<uint64_t> vis, F0, F1, active, valid, live;
    // a level's long-row parts (tasks) and their sums ([part][B])
    DBuf<uint64_t> hubs;
    DBuf<double> pm;
    DBuf<int32_t> pe;
    DBuf<double> vsum;
    DBuf<uint32_t> ridx;
    DBuf<uint64_t> rmask, rseg;
    DBuf<unsigned long long> bcnt, bpop;   // per-block record / pool offsets of a level
    DBuf<unsigned long long> ctl;
    DBuf<int32_t> srcs, dest;
    // samplers
    DBuf<double> X, S;
    DBuf<int64_t> K;
    DBuf<uint8_t> st;
    // pair-per-thread engine (shares sig/dlt/sige/ridx with the wave engine)
    DBuf<int32_t> lv;
    DBuf<uint8_t> pactive;
    DBuf<unsigned long long> loff;   // level offsets written by the persistent loops
    // per-source plain form
    DBuf<int32_t> ss_d, ss_q;
    DBuf<double> ss_sig, ss_dlt;
    DBuf<int32_t> probe_src;
    // lane order: sort keys and permutation of the requested samples
    DBuf<uint64_t> okey_in, okey_out;
    DBuf<int32_t> oidx_in, operm, lane_row;
    DBuf<int32_t> draw_src, draw_dst;   // a round's draws in draw order
    DBuf<uint8_t> sort_tmp;
    // two-sided pair search: per-slot stamps, counts, lists and level starts
    // of both sides ([2][slots][n], level starts [2][slots][n + 2])
    DBuf<uint64_t> bst;
    DBuf<double> bval;
    DBuf<int32_t> bq, blo;
    // weighted graphs ([n][B] entries, [n][W] words): rho and predecessors
    // pending per entry; changed and released lanes per word; the search's
    // lists (words), their taken lanes and arc tasks; the lanes of the counts'
    // rounds (distances, counts, dependencies and the rounds' words use lv,
    // sig, dlt and ridx)
    DBuf<double> wrho;
    DBuf<uint32_t> wpend, wfa, wfb;
    DBuf<uint64_t> wchg, wrdy, wtmask, wtask, womask;
    // one workgroup per source: per-slot distances (-1 between passes),
    // counts, exponents, dependencies, visiting lists, level starts, sums
    DBuf<WgVert> wgv;
    DBuf<int32_t> wgq, wglo, wgbase;
    int64_t wgn = 0;        // n the distances were filled for (0: refill)
    int32_t bslots = 0;
    int64_t bn = 0;
    uint32_t bepoch = 0;   // epochs up to this one are used in every slot
    unsigned long long *h_ctl = nullptr;  // pinned mirror of ctl
    // largest level record (entries) a batch may grow to; 0 = no limit. A
    // server sets it from its budget; a batch that would need more raises
    // RecordLimit.
    int64_t cap_limit = 0;
    // bytes the two-sided search's slots may hold; 0 = no limit (a server sets it)
    size_t bi_budget = 0;

    void init()
    {
        ctl.ensure(CTL_WORDS);
        if (!h_ctl) HIPX(hipHostMalloc((void **)&h_ctl, CTL_WORDS * sizeof(unsigned long long), 0));
    }
    // the engines' per-vertex buffers (not the control block or small arrays)
    void release_engines()
    {
        sig.release(); dlt.release(); sige.release();
        vis.release(); F0.release(); F1.release();
        vsum.release(); ridx.release(); rmask.release(); rseg.release();
        hubs.release(); pm.release(); pe.release();
        lv.release();
        bst.release(); bval.release(); bq.release(); blo.release();
        bslots = 0;
        bn = 0;
        bepoch = 0;
        wrho.release(); wpend.release(); wfa.release(); wfb.release();
        wchg.release(); wrdy.release(); wtmask.release(); wtask.release(); womask.release();
        wgv.release(); wgq.release(); wglo.release(); wgbase.release();
        wgn = 0;
    }
    void release()
    {
        sig.release(); dlt.release(); sige.release();
        vis.release(); F0.release(); F1.release();
        active.release(); valid.release(); live.release();
        hubs.release(); pm.release(); pe.release();
        vsum.release(); ridx.release(); rmask.release(); rseg.release(); ctl.release();
        bcnt.release(); bpop.release();
        srcs.release();
        dest.release(); X.release(); S.release(); K.release(); st.release();
        lv.release(); pactive.release(); loff.release();
        ss_d.release(); ss_q.release(); ss_sig.release(); ss_dlt.release(); probe_src.release();
        okey_in.release(); okey_out.release(); oidx_in.release(); operm.release();
        lane_row.release(); sort_tmp.release(); draw_src.release(); draw_dst.release();
        bst.release(); bval.release(); bq.release(); blo.release();
        wrho.release(); wpend.release(); wfa.release(); wfb.release();
        wchg.release(); wrdy.release(); wtmask.release(); wtask.release(); womask.release();
        wgv.release(); wgq.release(); wglo.release(); wgbase.release();
        wgn = 0;
        bslots = 0;
        bn = 0;
        bepoch = 0;
        if (h_ctl) (void)hipHostFree(h_ctl);
        h_ctl = nullptr;
    }
};

struct bc_graph {
    int64_t n = 0, nnz = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    Alloc alloc;                 // device memory of this handle
    int32_t io = BC_IO_DEVICE;   // where compute calls' arrays live
    DBuf<int64_t> row;
    DBuf<int32_t> col;
    bool directed = false;    // row/col hold out-neighbours; rrow/rcol in-neighbours
    DBuf<int64_t> rrow_buf;
    DBuf<int32_t> rcol_buf;
    const int64_t *rrow() const { return directed ? rrow_buf.p : row.p; }
    const int32_t *rcol() const { return directed ? rcol_buf.p : col.p; }
    bool weighted = false;    // wt_buf: out-arc weights; rwt_buf: in-arc weights (directed)
    DBuf<int32_t> wt_buf, rwt_buf;
    const int32_t *rwt() const { return directed ? rwt_buf.p : wt_buf.p; }
    // rows longer than kHub, per direction (out: row/col, in: rrow/rcol): the
    // first part of each in the part-sum slab (-1 for shorter rows), how many
    // such rows, their parts, the most parts of one row
    DBuf<int32_t> hpart_buf, rhpart_buf;
    int64_t hubs_out = 0, hubs_in = 0, parts_out = 0, parts_in = 0;
    int32_t most_out = 0, most_in = 0;
    const int32_t *rhpart() const { return directed ? rhpart_buf.p : hpart_buf.p; }
    // the vertices of those rows, ascending (hubs_out / hubs_in of them)
    DBuf<int32_t> hlist_buf, rhlist_buf;
    const int32_t *rhlist() const { return directed ? rhlist_buf.p : hlist_buf.p; }
    bc_config cfg{BC_SCHED_AUTO, 0, 0.0, 0, 0, 0, BC_PAIR_SEARCH_AUTO};
    Work own;
    Work *w = &own;
    int64_t cap_hint = 0;
    bc_stats stats{};
    int32_t hub = 0;          // a highest-degree vertex (depth probe)
    int64_t hub_degree = 0;
    int32_t engine = -1;      // cached automatic engine choice
    int32_t depth = -1;       // BFS depth from the hub (probe), -1 until probed
    bool tuned = false;       // cfg holds a plan chosen by the autotuner
    int32_t tuned_batch = 0;  // batch width of the tuned plan (bc_dependencies, bc_exact)
    std::array<int64_t, 33> deg_hist{};   // vertices per floor(log2(degree + 1))
    bool timed = false;       // a tuning candidate is running against `deadline`
    std::chrono::steady_clock::time_point deadline{};
    bool ext_sticky = false;  // an earlier batch on this graph needed extended counts
    bool bidir_off = false;   // a two-sided pair search here reached 2^1000
    // lane-order key: distances to up to kLandmarks highest-degree vertices
    std::vector<int32_t> landmarks;
    DBuf<uint64_t> skey;
    bool skey_ready = false;
    // profiler: event pairs around hot launches, device work-unit counters
    bool prof_on = false;
    DBuf<unsigned long long> prof_dev;
    double prof_ms[PROF_KERNELS] = {};
    int64_t prof_launches[PROF_KERNELS] = {};
    int64_t prof_host_units[2 * PROF_KERNELS] = {};   // work units counted on the host
    struct Pending {
        int kernel;
        hipEvent_t start, stop;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> ev_free;

    void release_all()
    {
        row.release(); col.release();
        rrow_buf.release(); rcol_buf.release();
        wt_buf.release(); rwt_buf.release();
        hpart_buf.release(); rhpart_buf.release();
        hlist_buf.release(); rhlist_buf.release();
        skey.release();
        own.release();
        prof_dev.release();
        for (auto &p : pending) {
            (void)hipEventDestroy(p.start);
            (void)hipEventDestroy(p.stop);
        }
        for (auto e : ev_free) (void)hipEventDestroy(e);
        pending.clear();
        ev_free.clear();
    }
};

namespace {

template <class F>
bc_status guarded(F &&f)
{
    try {
        f();
        tl_error.clear();
        return BC_OK;
    } catch (const Failure &e) {
        tl_error = e.msg;
        return e.status;
    } catch (const std::bad_alloc &) {
        tl_error = "host allocation failed";
        return BC_E_NOMEM;
    } catch (...) {
        tl_error = "unexpected error";
        return BC_E_DEVICE;
    }
}

void need(bool ok, const char *msg)
{
    if (!ok) fail(BC_E_INVALID, msg);
}

void use_device(bc_graph *g) { HIPX(hipSetDevice(g->device)); }

// A tuning candidate that runs past its deadline is abandoned at the next
// level boundary.
struct TuneTimeout {};

void check_deadline(const bc_graph *g)
{
    if (g->timed && std::chrono::steady_clock::now() > g->deadline) throw TuneTimeout{};
}


// Host arrays of a compute call in BC_IO_HOST mode, staged through device
// memory from the handle's allocator: inputs are copied in when staged,
// outputs copied back by finish(). In BC_IO_DEVICE mode pointers pass through.
class Staging {
public:
    Staging(bc_graph *g) : g_(g), host_(g->io == BC_IO_HOST) {}
    ~Staging()
    {
        if (!bufs_.empty()) (void)hipStreamSynchronize(g_->stream);
        for (auto &b : bufs_) b.release();
    }
    template <class T>
    const T *in(const T *h, int64_t count)
    {
        if (!host_ || !h || count <= 0) return h;
        T *d = take<T>(count);
        HIPX(hipMemcpyAsync(d, h, (size_t)count * sizeof(T), hipMemcpyHostToDevice, g_->stream));
        return d;
    }
    template <class T>
    T *out(T *h, int64_t count)
    {
        if (!host_ || !h || count <= 0) return h;
        T *d = take<T>(count);
        outs_.push_back({(void *)h, (const void *)d, (size_t)count * sizeof(T)});
        return d;
    }
    void finish()
    {
        for (auto &o : outs_)
            HIPX(hipMemcpyAsync(o.host, o.dev, o.bytes, hipMemcpyDeviceToHost, g_->stream));
        HIPX(hipStreamSynchronize(g_->stream));
    }
    // a host array read on the host (u != v checks): copied when on the device
    template <class T>
    std::vector<T> to_host(const T *p, int64_t count)
    {
        std::vector<T> v((size_t)std::max<int64_t>(count, 0));
        if (count <= 0) return v;
        if (host_) std::memcpy(v.data(), p, (size_t)count * sizeof(T));
        else HIPX(hipMemcpy(v.data(), p, (size_t)count * sizeof(T), hipMemcpyDeviceToHost));
        return v;
    }

private:
    template <class T>
    T *take(int64_t count)
    {
        bufs_.emplace_back();
        bufs_.back().ensure((size_t)count * sizeof(T));
        return (T *)bufs_.back().p;
    }
    struct Out {
        void *host;
        const void *dev;
        size_t bytes;
    };
    bc_graph *g_;
    bool host_;
    std::deque<DBuf<uint8_t>> bufs_;
    std::vector<Out> outs_;
};

// ------------------------------------------------------------------ profiler

hipEvent_t take_event(bc_graph *g)
{
    if (!g->ev_free.empty()) {
        hipEvent_t e = g->ev_free.back();
        g->ev_free.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPX(hipEventCreate(&e));
    return e;
}

// Collect the durations of finished profiled launches.
void prof_flush(bc_graph *g)
{
    if (g->pending.empty()) return;
    HIPX(hipStreamSynchronize(g->stream));
    for (auto &p : g->pending) {
        float ms = 0.f;
        HIPX(hipEventElapsedTime(&ms, p.start, p.stop));
        g->prof_ms[p.kernel] += ms;
        g->prof_launches[p.kernel] += 1;
        g->ev_free.push_back(p.start);
        g->ev_free.push_back(p.stop);
    }
    g->pending.clear();
}

// Launch one of the hot kernels, bracketed by events while profiling.
template <class K, class... A>
void launch_hot(bc_graph *g, int kernel, dim3 grid, K fn, A... args)
{
    if (!g->prof_on) {
        launch(g->stream, grid, fn, args...);
        return;
    }
    bc_graph::Pending p{kernel, take_event(g), take_event(g)};
    HIPX(hipEventRecord(p.start, g->stream));
    launch(g->stream, grid, fn, args...);
    HIPX(hipEventRecord(p.stop, g->stream));
    g->pending.push_back(p);
    if (g->pending.size() >= 256) prof_flush(g);
}

// launch_hot for a kernel whose workgroups are `block` threads wide
template <class K, class... A>
void launch_wide(bc_graph *g, int kernel, int grid, int block, K fn, A... args)
{
    bc_graph::Pending p{kernel, nullptr, nullptr};
    if (g->prof_on) {
        p.start = take_event(g);
        p.stop = take_event(g);
        HIPX(hipEventRecord(p.start, g->stream));
    }
    hipLaunchKernelGGL(fn, dim3(grid), dim3(block), 0, g->stream, args...);
    HIPX(hipGetLastError());
    if (g->prof_on) {
        HIPX(hipEventRecord(p.stop, g->stream));
        g->pending.push_back(p);
        if (g->pending.size() >= 256) prof_flush(g);
    }
}

// Part sums of the rows longer than kHub among the record entries [e0, e1),
// for the pull that follows: a's row / col / hpart in the pull's direction,
// F / SG the pulled level's words, `most` the most parts of one such row.
void hub_parts(bc_graph *g, const BatchArgs &a, int64_t e0, int64_t e1, const uint64_t *F,
               const uint64_t *SG, bool ext, int32_t most)
{
    if (e1 <= e0 || most <= 0) return;
    hipStream_t s = g->stream;
    launch(s, 1, k_fill_i32, (int32_t *)(g->w->ctl.p + CTL_HUBS), (int32_t)0, (int64_t)2);
    launch(s, grid_for(e1 - e0), k_hub_find, a, e0, e1, g->w->hubs.p);
    // one wavefront per task, at most as many as the level's entries could make
    const int64_t bound = std::min<int64_t>((e1 - e0) * most, (int64_t)g->w->hubs.cap);
    if (ext)
        launch_hot(g, PROF_HUB_PARTS, grid_waves(bound), k_hub_parts<true>, a, F, SG,
                   (const uint64_t *)g->w->hubs.p);
    else
        launch_hot(g, PROF_HUB_PARTS, grid_waves(bound), k_hub_parts<false>, a, F, SG,
                   (const uint64_t *)g->w->hubs.p);
}

// Lay out the record entries and pool segments of the level now in `nxt`
// (one profiled unit: count, scan, write).
void build_level(bc_graph *g, const BatchArgs &a, const uint64_t *nxt, int64_t cap)
{
    hipStream_t s = g->stream;
    const int64_t total = g->n << a.logW;
    const int64_t nb = (total + (1 << kLevelShift) - 1) >> kLevelShift;
    bc_graph::Pending p{PROF_LEVEL, nullptr, nullptr};
    if (g->prof_on) {
        p.start = take_event(g);
        p.stop = take_event(g);
        HIPX(hipEventRecord(p.start, s));
    }
    launch(s, (int)nb, k_level_count, nxt, total, g->w->bcnt.p, g->w->bpop.p);
    hipLaunchKernelGGL(k_level_scan, dim3(1), dim3(1024), 0, s, g->w->bcnt.p, g->w->bpop.p, nb,
                       g->w->ctl.p, cap, g->w->live.p, (int32_t)(1 << a.logW));
    HIPX(hipGetLastError());
    launch(s, (int)nb, k_level_write, a, nxt, (const unsigned long long *)g->w->bcnt.p,
           (const unsigned long long *)g->w->bpop.p);
    if (g->prof_on) {
        HIPX(hipEventRecord(p.stop, s));
        g->pending.push_back(p);
        g->prof_host_units[2 * PROF_LEVEL] += total;
        if (g->pending.size() >= 256) prof_flush(g);
    }
}

void read_ctl(bc_graph *g)
{
    HIPX(hipMemcpyAsync(g->w->h_ctl, g->w->ctl.p, CTL_WORDS * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, g->stream));
    HIPX(hipStreamSynchronize(g->stream));
}

void zero_ctl(bc_graph *g)
{
    HIPX(hipMemsetAsync(g->w->ctl.p, 0, CTL_WORDS * sizeof(unsigned long long), g->stream));
}

// Device-side range check of an index array (sources, targets, pair ends).
void check_indices(bc_graph *g, const int32_t *x, int64_t count, const char *what)
{
    if (count <= 0) return;
    zero_ctl(g);
    launch(g->stream, grid_for(count), k_check_range, x, count, g->n, &g->w->ctl.p[CTL_REC_OVERFLOW]);
    read_ctl(g);
    if (g->w->h_ctl[CTL_REC_OVERFLOW]) fail(BC_E_INVALID, std::string(what) + " outside [0, n)");
}

// ------------------------------------------------------------ batch planning

struct Plan {
    int logW = 0;
    int B = 64;
};

size_t free_device_bytes()
{
    size_t fr = 0, tot = 0;
    HIPX(hipMemGetInfo(&fr, &tot));
    return fr;
}

Plan plan_batch(bc_graph *g, int64_t want, int default_cap)
{
    int B = g->cfg.batch;
    if (B == 0) {
        B = 64;
        while (B < want && B < default_cap) B *= 2;
    }
    // (vertex, word) indices are 32-bit
    while (B > 64 && g->n * (int64_t)(B / 64) >= (1ll << 32)) B /= 2;
    // slabs: sig + dlt (+ exponents) per (vertex, source); keep within free memory
    const size_t budget = free_device_bytes() / 10 * 7 + g->w->sig.cap * 8 + g->w->dlt.cap * 8 +
                          g->w->sige.cap * 4;
    while (B > 64 && (size_t)g->n * B * 20 > budget) B /= 2;
    Plan p;
    p.B = B;
    p.logW = 0;
    while ((64 << p.logW) < B) ++p.logW;
    return p;
}

// What the backward pass leaves behind: the full dependency slab (per-source
// outputs, target gathers) or only per-(vertex, word) sums (BC_OUT_SUM).
enum OutKind { OUT_DELTA = 0, OUT_VSUM = 1 };

void ensure_batch(bc_graph *g, const Plan &p, bool ext, int64_t cap, OutKind kind)
{
    const int64_t n = g->n, W = 1ll << p.logW;
    g->w->sig.ensure((size_t)(n * p.B));
    if (kind == OUT_DELTA) g->w->dlt.ensure((size_t)(n * p.B));
    else g->w->vsum.ensure((size_t)(n * W));
    if (ext) g->w->sige.ensure((size_t)(n * p.B));
    g->w->vis.ensure((size_t)(n * W));
    g->w->F0.ensure((size_t)(kFS * n * W));
    g->w->F1.ensure((size_t)(kFS * n * W));
    g->w->active.ensure((size_t)W);
    g->w->valid.ensure((size_t)W);
    g->w->live.ensure((size_t)W);
    if (g->hubs_out || g->hubs_in) {
        const int64_t pp = std::max(g->parts_out, g->parts_in);
        g->w->hubs.ensure((size_t)(pp * W));
        g->w->pm.ensure((size_t)(pp * p.B));
        if (ext) g->w->pe.ensure((size_t)(pp * p.B));
    }
    g->w->srcs.ensure((size_t)p.B);
    g->w->dest.ensure((size_t)p.B);
    g->w->ridx.ensure((size_t)cap);
    g->w->rmask.ensure((size_t)cap);
    g->w->rseg.ensure((size_t)cap);
    g->w->bcnt.ensure((size_t)(((n * W) >> kLevelShift) + 2));
    g->w->bpop.ensure((size_t)(((n * W) >> kLevelShift) + 2));
}

// valid, active and live (level 0 holds every source) lanes of each word
__global__ void k_lane_masks(uint64_t *valid, uint64_t *active, uint64_t *live, int32_t W,
                             int32_t nvalid)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= W) return;
    const int rest = nvalid - 64 * j;
    const int lanes = rest < 0 ? 0 : (rest > 64 ? 64 : rest);
    const uint64_t m = lanes == 64 ? ~0ull : ((1ull << lanes) - 1ull);
    valid[j] = m;
    active[j] = m;
    live[j] = m;
}

BatchArgs make_args(bc_graph *g, const Plan &p, bool ext, int nvalid, bool pair, int64_t cap,
                    OutKind kind)
{
    BatchArgs a;
    a.row = g->row.p;
    a.col = g->col.p;
    a.rrow = g->rrow();
    a.rcol = g->rcol();
    a.n = g->n;
    a.logW = p.logW;
    a.B = p.B;
    a.sig = g->w->sig.p;
    a.sige = ext ? g->w->sige.p : nullptr;
    a.dlt = kind == OUT_DELTA ? g->w->dlt.p : nullptr;
    a.vsum = kind == OUT_VSUM ? g->w->vsum.p : nullptr;
    a.prof = g->prof_on ? g->prof_dev.p : nullptr;
    a.vis = g->w->vis.p;
    a.ridx = g->w->ridx.p;
    a.rmask = g->w->rmask.p;
    a.rseg = g->w->rseg.p;
    a.cap = cap;
    a.ctl = g->w->ctl.p;
    a.active = g->w->active.p;
    a.valid = g->w->valid.p;
    a.live = g->w->live.p;
    a.hpart = g->hpart_buf.p;
    a.rhpart = g->rhpart();
    a.pm = g->w->pm.p;
    a.pe = ext ? g->w->pe.p : nullptr;
    a.srcs = g->w->srcs.p;
    a.dest = pair ? g->w->dest.p : nullptr;
    a.lane_row = nullptr;
    a.nvalid = nvalid;
    return a;
}

// Raised by run_batch when the level record would outgrow Work::cap_limit.
struct RecordLimit {};

// The record capacity after an overflow: `want`, clamped to the work's limit.
int64_t grow_cap(const bc_graph *g, int64_t cap, int64_t want)
{
    const int64_t limit = g->w->cap_limit;
    if (limit <= 0) return want;
    if (cap >= limit) throw RecordLimit{};
    return std::min(want, limit);
}

// Hook between the forward and backward passes (per-source path counts).
struct SigmaOut {
    double *mant = nullptr;
    int32_t *ex = nullptr;
    int32_t count = 0;
    int64_t b0 = 0;
    const int32_t *lane_row = nullptr;   // caller's row of each lane, or null
};

double bottom_up_fraction(const bc_graph *g)
{
    if (g->cfg.bottom_up < 0) return -1.0;
    return g->cfg.bottom_up > 0 ? g->cfg.bottom_up : 0.04;
}

// Forward + backward for the nvalid sources (pair mode: u in srcs, v in
// dest) already placed in g->w->srcs / g->w->dest. Returns the level offsets and
// sets *ext_used. Grows the record and switches to extended path counts as
// needed, redoing the batch.
std::vector<int64_t> run_batch(bc_graph *g, const Plan &p, int nvalid, bool pair, bool *ext_used,
                               const SigmaOut *sigout, OutKind kind)
{
    const int64_t n = g->n, W = 1ll << p.logW;
    bool ext = g->ext_sticky;
    int64_t cap = std::max<int64_t>(g->cap_hint, std::max<int64_t>(4 * n * W, 1 << 16));
    if (g->w->cap_limit > 0) cap = std::min(cap, g->w->cap_limit);
    const double bu_frac = bottom_up_fraction(g);
    g->stats.bottom_up = bu_frac;
    for (;;) {
        ensure_batch(g, p, ext, cap, kind);
        BatchArgs a = make_args(g, p, ext, nvalid, pair, cap, kind);
        hipStream_t s = g->stream;
        HIPX(hipMemsetAsync(g->w->vis.p, 0, (size_t)(n * W) * 8, s));
        if (kind == OUT_VSUM) HIPX(hipMemsetAsync(g->w->vsum.p, 0, (size_t)(n * W) * 8, s));
        HIPX(hipMemsetAsync(g->w->F0.p, 0, (size_t)(kFS * n * W) * 8, s));
        HIPX(hipMemsetAsync(g->w->F1.p, 0, (size_t)(kFS * n * W) * 8, s));
        zero_ctl(g);
        launch(s, 1, k_lane_masks, g->w->valid.p, g->w->active.p, g->w->live.p, (int32_t)W,
               nvalid);
        launch(s, grid_for(p.B), k_init_sources, a, g->w->F0.p);
        read_ctl(g);
        std::vector<int64_t> off{0, (int64_t)g->w->h_ctl[CTL_TAIL]};
        if (g->w->h_ctl[CTL_REC_OVERFLOW]) {
            cap = grow_cap(g, cap, cap * 2);
            continue;
        }
        launch(s, grid_for(off[1]), k_init_level0, a, (int64_t)0, off[1],
               (const uint64_t *)g->w->F0.p, g->w->F0.p + 1);

        uint64_t *cur = g->w->F0.p, *nxt = g->w->F1.p;
        uint64_t *sgcur = g->w->F0.p + 1, *sgnxt = g->w->F1.p + 1;   // segments: word 1
        bool redo = false;
        for (int level = 0;; ++level) {
            const int64_t e0 = off[level], e1 = off[level + 1];
            const int64_t nent = e1 - e0;
            if (bu_frac > 0 && (double)nent > bu_frac * (double)(n * W)) {
                launch_hot(g, PROF_BOTTOMUP, grid_for(n * W), k_discover_bottomup, a,
                           (const uint64_t *)cur, nxt);
                if (g->hubs_in)
                    launch_hot(g, PROF_BOTTOMUP, grid_waves(g->hubs_in * W),
                               k_discover_bottomup_long, a, (const uint64_t *)cur, nxt,
                               g->rhlist(), g->hubs_in);
            } else
                launch_hot(g, PROF_TOPDOWN, grid_waves(nent), k_discover_topdown, a, e0, e1, nxt);
            build_level(g, a, nxt, cap);
            read_ctl(g);
            check_deadline(g);
            const int64_t e2 = (int64_t)g->w->h_ctl[CTL_TAIL];
            if (g->prof_on) g->prof_host_units[2 * PROF_LEVEL + 1] += e2 - e1;
            if (g->w->h_ctl[CTL_REC_OVERFLOW]) {
                cap = grow_cap(g, cap, std::max<int64_t>(cap * 2, e2 + (e2 >> 2)));
                redo = true;
                break;
            }
            if (e2 == e1) break;
            if (g->hubs_in) {
                BatchArgs ain = a;
                ain.row = a.rrow;
                ain.col = a.rcol;
                ain.hpart = a.rhpart;
                hub_parts(g, ain, e1, e2, cur, sgcur, ext, g->most_in);
            }
            if (ext)
                launch_hot(g, PROF_SIGMA, grid_tiles(e2 - e1), k_sigma_pull<true>, a, e1, e2,
                           (const uint64_t *)cur, (const uint64_t *)sgcur, sgnxt);
            else
                launch_hot(g, PROF_SIGMA, grid_tiles(e2 - e1), k_sigma_pull<false>, a, e1, e2,
                           (const uint64_t *)cur, (const uint64_t *)sgcur, sgnxt);
            launch(s, grid_for(nent), k_clear, a, e0, e1, cur);
            off.push_back(e2);
            std::swap(cur, nxt);
            std::swap(sgcur, sgnxt);
        }
        if (redo) continue;
        if (!ext) {
            read_ctl(g);
            if (g->w->h_ctl[CTL_SIG_OVERFLOW]) {
                ext = true;
                g->ext_sticky = true;
                continue;
            }
        }
        g->cap_hint = std::max<int64_t>(g->cap_hint, off.back() + off.back() / 4);
        // (the caller has zeroed the output rows: unreached vertices stay 0)
        if (sigout && (sigout->mant || sigout->ex)) {
            BatchArgs ao = a;
            ao.lane_row = sigout->lane_row;
            launch(s, grid_for(off.back()), k_out_sigma, ao, (int64_t)0, off.back(),
                   sigout->count, sigout->b0, sigout->mant, sigout->ex);
        }

        // backward: cur holds the deepest level's masks, nxt is clear
        const int L = (int)off.size() - 1;
        uint64_t *fnext = nxt, *fown = cur;
        uint64_t *sgnext = sgnxt, *sgown = sgcur;
        for (int level = L - 1; level >= 1; --level) {
            const int64_t e0 = off[level], e1 = off[level + 1];
            if (g->hubs_out) hub_parts(g, a, e0, e1, fnext, sgnext, ext, g->most_out);
            if (ext)
                launch_hot(g, PROF_BACKWARD, grid_tiles(e1 - e0), k_backward<true>, a, e0, e1,
                           (const uint64_t *)fnext, (const uint64_t *)sgnext, fown, sgown);
            else
                launch_hot(g, PROF_BACKWARD, grid_tiles(e1 - e0), k_backward<false>, a, e0, e1,
                           (const uint64_t *)fnext, (const uint64_t *)sgnext, fown, sgown);
            if (level + 1 < L)
                launch(s, grid_for(off[level + 2] - e1), k_clear, a, e1, off[level + 2], fnext);
            std::swap(fnext, fown);
            std::swap(sgnext, sgown);
        }
        *ext_used = ext;
        g->stats.levels += L;
        g->stats.extended |= ext ? 1 : 0;
        return off;
    }
}

// --------------------------------------------------------- per-source form

void ensure_single(bc_graph *g)
{
    g->w->ss_d.ensure((size_t)g->n);
    g->w->ss_q.ensure((size_t)g->n);
    g->w->ss_sig.ensure((size_t)g->n);
    g->w->ss_dlt.ensure((size_t)g->n);
}

__global__ void k_ss_start(int32_t *d, double *sig, double *dlt, int32_t *queue,
                           const int32_t *src, unsigned long long *ctl)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int32_t s = *src;
        d[s] = 0;
        sig[s] = 1.0;
        dlt[s] = 0.0;
        queue[0] = s;
        ctl[CTL_TAIL] = 1ull;
    }
}

// One source: level-synchronous BFS with one thread per frontier vertex,
// sigma pull, then the dependency sweep, each level its own launch.
std::vector<int64_t> run_single(bc_graph *g, const int32_t *src_dev, bool forward_only = false)
{
    const int64_t n = g->n;
    hipStream_t s = g->stream;
    ensure_single(g);
    HIPX(hipMemsetAsync(g->w->ss_d.p, 0xff, (size_t)n * 4, s));
    zero_ctl(g);
    launch(s, 1, k_ss_start, g->w->ss_d.p, g->w->ss_sig.p, g->w->ss_dlt.p, g->w->ss_q.p, src_dev, g->w->ctl.p);
    std::vector<int64_t> off{0, 1};
    for (int level = 0;; ++level) {
        const int64_t q0 = off[level], q1 = off[level + 1];
        launch(s, grid_for(q1 - q0), k_ss_topdown, (const int64_t *)g->row.p,
               (const int32_t *)g->col.p, g->w->ss_d.p, g->w->ss_q.p, q0, q1, (int32_t)level, g->w->ctl.p);
        read_ctl(g);
        const int64_t q2 = (int64_t)g->w->h_ctl[CTL_TAIL];
        if (q2 == q1) break;
        launch(s, grid_for(q2 - q1), k_ss_sigma, g->rrow(), g->rcol(),
               (const int32_t *)g->w->ss_d.p, g->w->ss_sig.p,
               (const int32_t *)g->w->ss_q.p, q1, q2, (int32_t)level, g->w->ctl.p);
        off.push_back(q2);
    }
    if (forward_only) return off;
    read_ctl(g);
    if (g->w->h_ctl[CTL_SIG_OVERFLOW])
        fail(BC_E_UNSUPPORTED, "path counts reach 2^1000: the per-source form has no "
                               "extended counts; use the batched schedule");
    const int L = (int)off.size() - 1;
    for (int level = L - 1; level >= 1; --level)
        launch(s, grid_for(off[level + 1] - off[level]), k_ss_backward, (const int64_t *)g->row.p,
               (const int32_t *)g->col.p, (const int32_t *)g->w->ss_d.p,
               (const double *)g->w->ss_sig.p, g->w->ss_dlt.p, (const int32_t *)g->w->ss_q.p, off[level],
               off[level + 1], (int32_t)level);
    g->stats.levels += L;
    return off;
}

bool per_source_schedule(const bc_graph *g) { return g->cfg.schedule == BC_SCHED_PER_SOURCE; }

// ------------------------------------------------------ engine selection

enum Engine { ENG_WAVE = 0, ENG_PAIR = 1, ENG_WG = 2 };
constexpr int kDeepGraphLevels = 32;
// the tuner times the workgroup engine on graphs of at most kDeepGraphLevels
// levels only up to this many vertices
constexpr int64_t kWgTrialMaxShallow = 1 << 16;

// Wave-per-word batching pays off when a vertex sits at few distinct levels
// across a batch's sources (small-world graphs); for deep graphs each
// (vertex, source) is on its own, so pairs get one thread each. The automatic
// choice probes the BFS depth from a highest-degree vertex once per graph.
// BFS depth from a highest-degree vertex (once per graph). A path count is at
// most maxdeg^distance and distances are at most twice that depth: counts
// start extended when that bound reaches 2^1000 (they agree bit for bit with
// plain FP64 in range).
int probe_depth(bc_graph *g)
{
    if (g->depth < 0) {
        g->w->probe_src.ensure(1);
        HIPX(hipMemcpy(g->w->probe_src.p, &g->hub, 4, hipMemcpyHostToDevice));
        std::vector<int64_t> off = run_single(g, g->w->probe_src.p, true);
        g->depth = (int)off.size() - 2;
        g->stats.levels = 0;
        const double bound =
            2.0 * g->depth * std::log2(std::max<double>(2.0, (double)g->hub_degree));
        if (bound >= 1000.0) g->ext_sticky = true;
    }
    return g->depth;
}

Engine engine_for(bc_graph *g)
{
    if (g->weighted) return ENG_WAVE;   // the weighted engine's 64-source words
    if (g->cfg.schedule == BC_SCHED_BATCHED) return ENG_WAVE;
    if (g->cfg.schedule == BC_SCHED_THREADED) return ENG_PAIR;
    if (g->cfg.schedule == BC_SCHED_WORKGROUP) return ENG_WG;
    if (g->engine < 0) g->engine = probe_depth(g) > kDeepGraphLevels ? ENG_PAIR : ENG_WAVE;
    return (Engine)g->engine;
}

int32_t schedule_of(Engine e)
{
    return e == ENG_PAIR ? BC_SCHED_THREADED
                         : e == ENG_WG ? BC_SCHED_WORKGROUP : BC_SCHED_BATCHED;
}

// ------------------------------------------------------ pair-per-thread engine

int plan_pairs(bc_graph *g, int64_t want, int default_cap)
{
    int B = g->cfg.batch;
    if (B == 0) {
        B = 64;
        while (B < want && B < default_cap) B *= 2;
    }
    while (B > 1 && (int64_t)B * g->n >= (1ll << 32)) B /= 2;
    // level, count, dependency, exponent, record: 28 bytes per pair
    const size_t budget = free_device_bytes() / 10 * 7 + g->w->sig.cap * 8 + g->w->dlt.cap * 8 +
                          g->w->lv.cap * 4 + g->w->sige.cap * 4 + g->w->ridx.cap * 4;
    while (B > 1 && (size_t)g->n * B * 28 > budget) B /= 2;
    return B;
}

PairArgs make_pair_args(bc_graph *g, int B, bool ext, int nvalid, bool pair)
{
    PairArgs a;
    a.row = g->row.p;
    a.col = g->col.p;
    a.rrow = g->rrow();
    a.rcol = g->rcol();
    a.n = (uint32_t)g->n;
    a.B = B;
    a.lv = g->w->lv.p;
    a.sig = g->w->sig.p;
    a.sige = ext ? g->w->sige.p : nullptr;
    a.dlt = g->w->dlt.p;
    a.rec = g->w->ridx.p;
    a.cap = (int64_t)B * g->n;
    a.ctl = g->w->ctl.p;
    a.active = g->w->pactive.p;
    a.srcs = g->w->srcs.p;
    a.dest = pair ? g->w->dest.p : nullptr;
    a.nvalid = nvalid;
    a.prof = g->prof_on ? g->prof_dev.p : nullptr;
    return a;
}

void ensure_pairs(bc_graph *g, int B, bool ext)
{
    const size_t np = (size_t)B * g->n;
    g->w->lv.ensure(np);
    g->w->sig.ensure(np);
    g->w->dlt.ensure(np);
    if (ext) g->w->sige.ensure(np);
    g->w->ridx.ensure(np);
    g->w->pactive.ensure((size_t)B);
    g->w->srcs.ensure((size_t)B);
    g->w->dest.ensure((size_t)B);
}

struct PairSigmaOut {
    double *mant = nullptr;
    int32_t *ex = nullptr;
    int32_t count = 0;
    int64_t b0 = 0;
};

// Persistent level loops of the pair engine: when to use them, on what grid.
// The loops are opt-in: on the 2048^2 grid (thousands of levels of ~0.5 M
// pairs) they measured 2.3x slower than one launch per phase, the halved
// resident grid hiding less latency and every block's barrier fence writing
// back and invalidating its L2.
bool use_level_loop(const bc_graph *g)
{
    if (g->cfg.level_loop <= 0) return false;
    int coop = 0;
    HIPX(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, g->device));
    if (!coop && g->cfg.level_loop > 0)
        fail(BC_E_UNSUPPORTED, "the device has no cooperative launch for the level loop");
    return coop != 0;
}

// A grid that is resident as a whole. The occupancy query's blocks per CU is
// the theoretical figure; at a kernel's register-file limit fewer blocks are
// resident in practice (a grid of the full figure left blocks waiting for
// others to exit), so the loops take half of it on every CU.
template <class K>
int resident_grid(const bc_graph *g, K kernel)
{
    int per_cu = 0, cus = 0;
    HIPX(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0));
    HIPX(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device));
    if (per_cu < 1 || cus < 1) fail(BC_E_UNSUPPORTED, "the level loop kernel cannot be resident");
    return std::max(1, per_cu / 2) * cus;
}

// A grid barrier wait longer than this is taken as a failure (no level of
// any graph here takes a fraction of it).
constexpr double kBarrierSeconds = 5.0;

uint64_t barrier_ticks(const bc_graph *g)
{
    int khz = 0;
    HIPX(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, g->device));
    return (uint64_t)(kBarrierSeconds * 1e3 * (double)std::max(khz, 1));
}

// One cooperative launch of a persistent loop (profiled like a hot kernel).
template <class K, class... A>
void launch_loop(bc_graph *g, int kernel, K fn, int grid, A... args)
{
    void *params[] = {(void *)&args...};
    bc_graph::Pending p{kernel, nullptr, nullptr};
    if (g->prof_on) {
        p.start = take_event(g);
        p.stop = take_event(g);
        HIPX(hipEventRecord(p.start, g->stream));
    }
    HIPX(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(fn), dim3(grid), dim3(kBlock),
                                    params, 0, g->stream));
    if (g->prof_on) {
        HIPX(hipEventRecord(p.stop, g->stream));
        g->pending.push_back(p);
        if (g->pending.size() >= 256) prof_flush(g);
    }
}

// After a persistent loop: a barrier that timed out is an error; the message
// names the loop, the barriers completed and the blocks that had arrived at
// the one that failed.
void check_barrier(bc_graph *g, const char *loop, int grid)
{
    const unsigned long long *h = g->w->h_ctl;
    if (h[CTL_BAR + 2])
        fail(BC_E_DEVICE, std::string("a grid barrier of the ") + loop +
                              " level loop timed out after " + std::to_string(h[CTL_BAR + 1]) +
                              " completed barriers, with " + std::to_string(h[CTL_BAR]) + " of " +
                              std::to_string(grid) + " blocks arrived at the next one");
}

std::vector<int64_t> run_pairs(bc_graph *g, int B, int nvalid, bool pair, bool *ext_used,
                               const PairSigmaOut *sigout)
{
    const int64_t n = g->n;
    hipStream_t s = g->stream;
    bool ext = g->ext_sticky;
    const bool loop = use_level_loop(g);
    for (;;) {
        ensure_pairs(g, B, ext);
        PairArgs a = make_pair_args(g, B, ext, nvalid, pair);
        HIPX(hipMemsetAsync(g->w->lv.p, 0xff, (size_t)B * n * 4, s));
        zero_ctl(g);
        launch(s, grid_for(B), k_p_init, a);
        std::vector<int64_t> off;
        bool redo = false;
        PairLoop L{};
        int grid_b = 0;
        if (loop) {
            // every level of the forward pass in one launch
            g->w->loff.ensure((size_t)n + 2);
            L.a = a;
            L.loff = g->w->loff.p;
            L.max_levels = (int64_t)g->w->loff.cap;
            const int grid_f = ext ? resident_grid(g, k_p_forward_loop<true>)
                                   : resident_grid(g, k_p_forward_loop<false>);
            grid_b = ext ? resident_grid(g, k_p_backward_loop<true>)
                         : resident_grid(g, k_p_backward_loop<false>);
            L.gs.bar = g->w->ctl.p + CTL_BAR;
            L.gs.nblocks = (unsigned long long)grid_f;
            L.gs.limit = barrier_ticks(g);
            if (ext) launch_loop(g, PROF_PAIR_FWD, k_p_forward_loop<true>, grid_f, L);
            else launch_loop(g, PROF_PAIR_FWD, k_p_forward_loop<false>, grid_f, L);
            read_ctl(g);
            check_barrier(g, "forward", grid_f);
            if (g->w->h_ctl[CTL_REC_OVERFLOW]) fail(BC_E_DEVICE, "pair record overflow");
            if (!ext && g->w->h_ctl[CTL_SIG_OVERFLOW]) {
                redo = true;
            } else {
                off.resize((size_t)g->w->h_ctl[CTL_LEVELS] + 1);
                HIPX(hipMemcpy(off.data(), g->w->loff.p, off.size() * 8, hipMemcpyDeviceToHost));
            }
        } else {
            read_ctl(g);
            off = {0, (int64_t)g->w->h_ctl[CTL_TAIL]};
            for (int level = 0;; ++level) {
                const int64_t e0 = off[level], e1 = off[level + 1];
                launch_hot(g, PROF_TOPDOWN, grid_for(e1 - e0), k_p_topdown, a, e0, e1,
                           (int32_t)level);
                read_ctl(g);
                check_deadline(g);
                const int64_t e2 = (int64_t)g->w->h_ctl[CTL_TAIL];
                if (g->w->h_ctl[CTL_REC_OVERFLOW]) fail(BC_E_DEVICE, "pair record overflow");
                if (!ext && g->w->h_ctl[CTL_SIG_OVERFLOW]) {
                    redo = true;
                    break;
                }
                if (e2 == e1) break;
                if (ext)
                    launch_hot(g, PROF_SIGMA, grid_for(e2 - e1), k_p_sigma<true>, a, e1, e2,
                               (int32_t)level);
                else
                    launch_hot(g, PROF_SIGMA, grid_for(e2 - e1), k_p_sigma<false>, a, e1, e2,
                               (int32_t)level);
                off.push_back(e2);
            }
            if (!redo && !ext) {
                read_ctl(g);
                redo = g->w->h_ctl[CTL_SIG_OVERFLOW] != 0;
            }
        }
        if (redo) {
            ext = true;
            g->ext_sticky = true;
            continue;
        }
        if (sigout && (sigout->mant || sigout->ex))
            launch(s, grid_for(n * sigout->count), k_p_out_sigma, a, sigout->count, sigout->b0,
                   sigout->mant, sigout->ex);
        const int nlev = (int)off.size() - 1;
        if (loop) {
            if (nlev >= 2) {
                L.gs.nblocks = (unsigned long long)grid_b;
                zero_ctl(g);
                if (ext)
                    launch_loop(g, PROF_PAIR_BWD, k_p_backward_loop<true>, grid_b, L, (int32_t)nlev);
                else
                    launch_loop(g, PROF_PAIR_BWD, k_p_backward_loop<false>, grid_b, L,
                                (int32_t)nlev);
                read_ctl(g);
                check_barrier(g, "backward", grid_b);
            }
        } else {
            for (int level = nlev - 1; level >= 1; --level) {
                if (ext)
                    launch_hot(g, PROF_BACKWARD, grid_for(off[level + 1] - off[level]),
                               k_p_backward<true>, a, off[level], off[level + 1], (int32_t)level);
                else
                    launch_hot(g, PROF_BACKWARD, grid_for(off[level + 1] - off[level]),
                               k_p_backward<false>, a, off[level], off[level + 1], (int32_t)level);
            }
        }
        *ext_used = ext;
        g->stats.levels += nlev;
        g->stats.extended |= ext ? 1 : 0;
        return off;
    }
}

// ------------------------------------------------------------ weighted graphs

// Bytes of a weighted batch of width B (words W = B / 64): per entry the
// distance, count, dependency, rho and pending predecessors (32) and a slot of
// the counts' rounds (12: a word appears in a round only with a lane that
// joins it, so the rounds hold at most n * B words); per word its two masks
// and the search's two lists and taken lanes (32); the search's tasks (one per
// list entry and chunk of kWChunk arcs, at most n * W + nnz * W / kWChunk + W).
size_t weighted_tasks(const bc_graph *g, int B)
{
    const size_t W = (size_t)B / 64;
    return (size_t)g->n * W + (size_t)g->nnz * W / kWChunk + W;
}

size_t weighted_bytes(const bc_graph *g, int B)
{
    const size_t np = (size_t)B * g->n, words = np / 64;
    return np * 44 + words * 32 + weighted_tasks(g, B) * 8;
}

// Width of a weighted batch: a power of two from 64, up to the request or
// default_cap, within 70 % of the free device memory (held buffers count) and
// with word indices below 2^32.
int plan_weighted(bc_graph *g, int64_t want, int default_cap)
{
    int B = g->cfg.batch;
    if (B == 0) {
        B = 64;
        while (B < want && B < default_cap) B *= 2;
    }
    B = std::max(B, 64);
    while (B > 64 && (int64_t)(B / 64) * g->n >= (1ll << 32)) B /= 2;
    const Work &w = *g->w;
    const size_t held = w.sig.bytes() + w.dlt.bytes() + w.lv.bytes() + w.ridx.bytes() +
                        w.wrho.bytes() + w.wpend.bytes() + w.wfa.bytes() + w.wfb.bytes() +
                        w.wchg.bytes() + w.wrdy.bytes() + w.wtmask.bytes() + w.wtask.bytes() +
                        w.womask.bytes();
    const size_t budget = (free_device_bytes() + held) / 10 * 7;
    while (B > 64 && weighted_bytes(g, B) > budget) B /= 2;
    return B;
}

void ensure_weighted(bc_graph *g, int B)
{
    const size_t np = (size_t)B * g->n, words = np / 64;
    Work &w = *g->w;
    w.lv.ensure(np);
    w.sig.ensure(np);
    w.dlt.ensure(np);
    w.wrho.ensure(np);
    w.wpend.ensure(np);
    w.ridx.ensure(np);
    w.womask.ensure(np);
    w.wchg.ensure(words);
    w.wrdy.ensure(words);
    w.wfa.ensure(words);
    w.wfb.ensure(words);
    w.wtmask.ensure(words);
    w.wtask.ensure(weighted_tasks(g, B));
    w.srcs.ensure((size_t)B);
    w.dest.ensure((size_t)B);
}

WArgs make_weighted_args(bc_graph *g, int B, int nvalid, bool pair)
{
    WArgs a;
    a.row = g->row.p;
    a.col = g->col.p;
    a.wt = g->wt_buf.p;
    a.rrow = g->rrow();
    a.rcol = g->rcol();
    a.rwt = g->rwt();
    a.n = g->n;
    a.logW = 0;
    while ((64 << a.logW) < B) ++a.logW;
    a.dist = g->w->lv.p;
    a.sig = g->w->sig.p;
    a.dlt = g->w->dlt.p;
    a.rho = g->w->wrho.p;
    a.pend = g->w->wpend.p;
    a.chg = g->w->wchg.p;
    a.rdy = g->w->wrdy.p;
    a.tmask = g->w->wtmask.p;
    a.task = g->w->wtask.p;
    a.ord = g->w->ridx.p;
    a.omask = g->w->womask.p;
    a.ctl = g->w->ctl.p;
    a.srcs = g->w->srcs.p;
    a.dest = pair ? g->w->dest.p : nullptr;
    a.nvalid = nvalid;
    a.prof = g->prof_on ? g->prof_dev.p : nullptr;
    return a;
}

// Brandes' pass (pair mode: toward each lane's destination) for the nvalid
// sources in g->w->srcs (and destinations in g->w->dest), B lanes wide.
// Returns the rounds of the path counts.
int64_t run_weighted(bc_graph *g, int B, int nvalid, bool pair)
{
    hipStream_t s = g->stream;
    Work &w = *g->w;
    const int64_t np = (int64_t)B * g->n, words = np / 64;
    WArgs a = make_weighted_args(g, B, nvalid, pair);
    launch(s, grid_for(np), k_fill_i32, a.dist, kWUnreached, np);
    launch(s, grid_for(2 * words), k_fill_i32, (int32_t *)a.chg, (int32_t)0, 2 * words);
    launch(s, grid_for(2 * words), k_fill_i32, (int32_t *)a.rdy, (int32_t)0, 2 * words);
    launch(s, grid_for(nvalid), k_ww_init, a);
    // the search: rounds until no distance falls
    for (;;) {
        zero_ctl(g);
        launch(s, grid_for(words), k_ww_collect, a, w.wfa.p);
        read_ctl(g);
        if (w.h_ctl[CTL_TAIL] == 0) break;
        launch_hot(g, PROF_W_SEARCH, grid_waves((int64_t)w.h_ctl[CTL_WTASKS]), k_ww_relax, a,
                   (const uint32_t *)w.wfa.p);
        if (g->timed) check_deadline(g);
    }
    // path counts in rounds; ord grows behind each round
    zero_ctl(g);
    launch(s, grid_waves(words), k_ww_prep, a);
    read_ctl(g);
    std::vector<int64_t> off{0, (int64_t)w.h_ctl[CTL_TAIL]};
    for (;;) {
        const int64_t s0 = off[off.size() - 2], s1 = off.back();
        launch_hot(g, PROF_W_COUNTS, grid_waves(s1 - s0), k_ww_release, a, s0, s1);
        read_ctl(g);
        const int64_t t = (int64_t)w.h_ctl[CTL_TAIL];
        if (t == s1) break;
        launch_hot(g, PROF_W_COUNTS, grid_waves(t - s1), k_ww_sigma, a, s1, t);
        off.push_back(t);
    }
    read_ctl(g);
    if (w.h_ctl[CTL_SIG_OVERFLOW])
        fail(BC_E_UNSUPPORTED, "path counts reach 2^1000 on a weighted graph");
    // Theorem 1, latest round first (round 0 holds the sources: delta 0)
    for (size_t r = off.size() - 1; r >= 2; --r)
        launch_hot(g, PROF_W_BACKWARD, grid_waves(off[r] - off[r - 1]), k_ww_backward, a,
                   off[r - 1], off[r]);
    const int64_t rounds = (int64_t)off.size() - 1;
    g->stats.levels += rounds;
    return rounds;
}

// dependencies_impl for weighted graphs (every schedule: one engine)
void weighted_dependencies(bc_graph *g, const int32_t *sources, int64_t k, int32_t mode,
                           double *out, int32_t *dist_out, double *sig_m, int32_t *sig_e,
                           bool pair, const int32_t *dests, const int32_t *targets, int32_t T)
{
    const int64_t n = g->n;
    hipStream_t s = g->stream;
    const int B = plan_weighted(g, k, g->tuned_batch ? g->tuned_batch : 512);
    g->stats.batch_width = B;
    g->stats.schedule = BC_SCHED_BATCHED;
    for (int64_t b0 = 0; b0 < k; b0 += B) {
        const int count = (int)std::min<int64_t>(B, k - b0);
        ensure_weighted(g, B);
        HIPX(hipMemcpyAsync(g->w->srcs.p, sources + b0, (size_t)count * 4,
                            hipMemcpyDeviceToDevice, s));
        if (pair)
            HIPX(hipMemcpyAsync(g->w->dest.p, dests + b0, (size_t)count * 4,
                                hipMemcpyDeviceToDevice, s));
        run_weighted(g, B, count, pair);
        const WArgs a = make_weighted_args(g, B, count, pair);
        if (mode == BC_OUT_SUM) launch(s, grid_waves(n), k_ww_out_sum, a, out);
        else if (mode == BC_OUT_TARGETS)
            launch(s, grid_for((int64_t)count * T), k_ww_out_targets, a, targets, T,
                   (int32_t)count, b0, out);
        else launch(s, grid_for(n * count), k_ww_out_full, a, (int32_t)count, b0, out);
        if (dist_out)
            launch(s, grid_for(n * count), k_ww_out_dist, a, (int32_t)count, b0, dist_out);
        if (sig_m || sig_e)
            launch(s, grid_for(n * count), k_ww_out_sigma, a, (int32_t)count, b0, sig_m, sig_e);
        g->stats.batches += 1;
        g->stats.samples_executed += count;
    }
    HIPX(hipStreamSynchronize(s));
    prof_flush(g);
}

// ------------------------------------------------- one workgroup per source

constexpr int kWgSlotsMax = 1024;
// sources per slot per launch (bounds a launch's duration)
constexpr int64_t kWgPerSlot = 64;

size_t wg_slot_bytes(int64_t n)
{
    // vertex record, list entry, level start; base
    return (size_t)n * (sizeof(WgVert) + 8) + 8;
}

// Sources in flight: the configured width or up to kWgSlotsMax, at most the
// request, within 70 % of the free device memory (held slots count).
int plan_wg(bc_graph *g, int64_t want, int default_cap)
{
    const Work &w = *g->w;
    const size_t held = w.wgv.bytes() + w.wgq.bytes() + w.wglo.bytes() + w.wgbase.bytes();
    const size_t budget = (free_device_bytes() + held) / 10 * 7;
    int S = g->cfg.batch ? g->cfg.batch : std::min(default_cap, kWgSlotsMax);
    S = (int)std::max<int64_t>(1, std::min<int64_t>(S, want));
    while (S > 1 && (size_t)S * wg_slot_bytes(g->n) > budget) S /= 2;
    return S;
}

void ensure_wg(bc_graph *g, int S, bool ext, bool sum)
{
    Work &w = *g->w;
    const int64_t n = g->n;
    const size_t cells = (size_t)S * n;
    if (w.wgv.cap < cells || w.wgn != n) {
        // distances all below every slot's base (0)
        w.wgv.release();
        w.wgv.ensure(cells);
        launch(g->stream, grid_for((int64_t)cells), k_wg_clear, w.wgv.p, (int64_t)cells);
        w.wgbase.release();
        w.wgbase.ensure((size_t)S);
        launch(g->stream, grid_for(S), k_fill_i32, w.wgbase.p, (int32_t)0, (int64_t)S);
        w.wgn = n;
    }
    w.wgq.ensure(cells);
    w.wglo.ensure((size_t)S * (n + 1));
}

// dependencies_impl on the one-workgroup-per-source engine. A pass whose plain
// counts reach 2^1000 restarts the call with extended counts.
void wg_dependencies(bc_graph *g, const int32_t *sources, int64_t k, int32_t mode, double *out,
                     int32_t *dist_out, double *sig_m, int32_t *sig_e, bool pair,
                     const int32_t *dests, const int32_t *targets, int32_t T)
{
    const int64_t n = g->n;
    hipStream_t s = g->stream;
    Work &w = *g->w;
    const int S = plan_wg(g, k, g->tuned_batch ? g->tuned_batch : kWgSlotsMax);
    const bool sum = mode == BC_OUT_SUM;
    bool ext = g->ext_sticky;
    int64_t launches = 0;
    for (;;) {
        ensure_wg(g, S, ext, sum);
        if (sum) launch(s, grid_for((int64_t)S * n), k_wg_zero_sum, w.wgv.p, (int64_t)S * n);
        if (mode == BC_OUT_FULL && out) launch(s, grid_for(k * n), k_fill_f64, out, 0.0, k * n);
        zero_ctl(g);
        w.wgn = 0;   // a launch that does not complete leaves the slots unknown
        for (int64_t c0 = 0; c0 < k; c0 += (int64_t)S * kWgPerSlot) {
            const int count = (int)std::min<int64_t>((int64_t)S * kWgPerSlot, k - c0);
            WgArgs a;
            a.row = g->row.p;
            a.col = g->col.p;
            a.rrow = g->rrow();
            a.rcol = g->rcol();
            a.n = n;
            a.srcs = sources + c0;
            a.dest = pair ? dests + c0 : nullptr;
            a.count = count;
            a.vert = w.wgv.p;
            a.base = w.wgbase.p;
            a.q = w.wgq.p;
            a.lo = w.wglo.p;
            a.sum = sum ? 1 : 0;
            a.full = mode == BC_OUT_FULL && out ? out + c0 * n : nullptr;
            a.tgt = mode == BC_OUT_TARGETS ? out + c0 * T : nullptr;
            a.targets = targets;
            a.T = mode == BC_OUT_TARGETS ? T : 0;
            a.dist_out = dist_out ? dist_out + c0 * n : nullptr;
            a.sig_m = sig_m ? sig_m + c0 * n : nullptr;
            a.sig_e = sig_e ? sig_e + c0 * n : nullptr;
            a.ctl = w.ctl.p;
            a.prof = g->prof_on ? g->prof_dev.p : nullptr;
            const int grid = std::min(S, count);
            if (ext) launch_wide(g, PROF_WG, grid, kWgBlock, k_wg<true>, a);
            else launch_wide(g, PROF_WG, grid, kWgBlock, k_wg<false>, a);
            ++launches;
            if (g->timed) {
                HIPX(hipStreamSynchronize(s));
                check_deadline(g);
            }
        }
        read_ctl(g);
        w.wgn = n;
        if (!ext && w.h_ctl[CTL_SIG_OVERFLOW]) {
            ext = true;
            g->ext_sticky = true;
            continue;
        }
        break;
    }
    if (sum) launch(s, grid_for(n), k_wg_reduce, (const WgVert *)w.wgv.p, (int32_t)S, n, out);
    g->stats.schedule = BC_SCHED_WORKGROUP;
    g->stats.batch_width = S;
    g->stats.batches = launches;
    g->stats.samples_executed = k;
    g->stats.extended = ext ? 1 : 0;
    HIPX(hipStreamSynchronize(s));
    prof_flush(g);
}

// ------------------------------------------------------ two-sided pair search

// Pairs in flight at once: one workgroup and one slot of per-vertex state each.
constexpr int kBiSlotsMax = 2048;
// pairs per launch of bc_pair_dependencies' two-sided search
constexpr int64_t kBiChunk = 1 << 16;

size_t bidir_slot_bytes(int64_t n)
{
    return (size_t)n * 2 * (8 + 8 + 4) + (size_t)(n + 2) * 2 * 4;
}

// Pair samples take the two-sided search unless the caller asked for the
// one-sided one or its path counts once reached 2^1000 on this graph.
bool use_bidir(const bc_graph *g)
{
    return g->cfg.pair_search != BC_PAIR_SEARCH_ONE_SIDED && !g->bidir_off && !g->weighted;
}

// Slots for `want` pairs: at most kBiSlotsMax, within a quarter of the free device
// memory (what the slots hold already counts as free).
int plan_bidir(bc_graph *g, int64_t want)
{
    const Work &w = *g->w;
    const size_t held = w.bst.bytes() + w.bval.bytes() + w.bq.bytes() + w.blo.bytes();
    const size_t budget = (free_device_bytes() + held) / 4;
    const size_t per = bidir_slot_bytes(g->n);
    int S = (int)std::max<int64_t>(1, std::min<int64_t>(want, kBiSlotsMax));
    while (S > 1 && (size_t)S * per > budget) S /= 2;
    return S;
}

// The two-sided search of `count` pairs (device arrays us, vs): target values
// into X[t * stride + i] when X is given, or into X[i] for pair i's own target
// ptgt[i] when ptgt is given; rows into full[i * n + w] (zeroed by the
// caller) when full is given. Returns false when a path count reached 2^1000
// (plain FP64 only): the caller runs those pairs one-sided.
bool run_bidir(bc_graph *g, const int32_t *us, const int32_t *vs, int count,
               const int32_t *targets, int32_t T, int32_t stride, double *X, double *full,
               const int32_t *ptgt = nullptr)
{
    if (count <= 0) return true;
    Work &w = *g->w;
    const int64_t n = g->n;
    hipStream_t s = g->stream;
    int want = plan_bidir(g, count);
    if (w.bi_budget)
        want = (int)std::max<size_t>(1, std::min<size_t>((size_t)want,
                                                         w.bi_budget / bidir_slot_bytes(n)));
    // Slots are laid out [side][slot][n] for this graph and width; buffers
    // large enough are kept across graphs and widths: a stale stamp holds an
    // older epoch than any pair of this launch, so it never reads as found.
    const size_t cells = (size_t)2 * want * n, lo_cells = (size_t)2 * want * (n + 2);
    if (w.bst.cap < cells || w.bval.cap < cells || w.bq.cap < cells || w.blo.cap < lo_cells) {
        w.bst.release(); w.bval.release(); w.bq.release(); w.blo.release();
        w.bst.ensure(cells);
        w.bval.ensure(cells);
        w.bq.ensure(cells);
        w.blo.ensure(lo_cells);
        HIPX(hipMemsetAsync(w.bst.p, 0, cells * sizeof(uint64_t), s));
        w.bepoch = 0;
    }
    w.bslots = want;
    w.bn = n;
    const int grid = std::min(w.bslots, count);
    const uint32_t per_slot = (uint32_t)((count + grid - 1) / grid);
    if ((uint64_t)w.bepoch + per_slot + 1 >= 0xffffffffull) {
        HIPX(hipMemsetAsync(w.bst.p, 0, w.bst.bytes(), s));
        w.bepoch = 0;
    }
    const size_t half = (size_t)w.bslots * n, half_lo = (size_t)w.bslots * (n + 2);
    BiArgs a;
    a.row[0] = g->row.p;
    a.col[0] = g->col.p;
    a.row[1] = g->rrow();
    a.col[1] = g->rcol();
    a.n = n;
    a.us = us;
    a.vs = vs;
    a.count = count;
    a.st[0] = w.bst.p;
    a.st[1] = w.bst.p + half;
    a.val[0] = w.bval.p;
    a.val[1] = w.bval.p + half;
    a.q[0] = w.bq.p;
    a.q[1] = w.bq.p + half;
    a.lo[0] = w.blo.p;
    a.lo[1] = w.blo.p + half_lo;
    a.epoch0 = w.bepoch;
    a.ctl = w.ctl.p;
    a.prof = g->prof_on ? g->prof_dev.p : nullptr;
    a.targets = targets;
    a.T = T;
    a.stride = stride;
    a.X = X;
    a.full = full;
    a.ptgt = ptgt;
    zero_ctl(g);
    launch_hot(g, PROF_BIDIR, grid, k_bidir, a);
    w.bepoch += per_slot;
    read_ctl(g);
    if (w.h_ctl[CTL_SIG_OVERFLOW] == 0) return true;
    g->bidir_off = true;
    return false;
}

// ------------------------------------------------------------ lane order

// key[v]: the BFS distances from the landmarks interleaved in Morton order,
// computed once per graph by one multi-source BFS.
void ensure_source_keys(bc_graph *g)
{
    if (g->skey_ready) return;
    const int64_t n = g->n;
    const int nl = (int)g->landmarks.size();
    hipStream_t s = g->stream;
    g->skey.ensure((size_t)n);
    DBuf<uint8_t> f0, f1, seen;
    DBuf<int32_t> lm;
    DBuf<unsigned long long> grew;
    f0.ensure((size_t)n);
    f1.ensure((size_t)n);
    seen.ensure((size_t)n);
    lm.ensure((size_t)std::max(nl, 1));
    grew.ensure(1);
    try {
        HIPX(hipMemcpy(lm.p, g->landmarks.data(), (size_t)nl * 4, hipMemcpyHostToDevice));
        launch(s, grid_for(n), k_key_init, (const int32_t *)lm.p, (int32_t)nl, n, f0.p, seen.p,
               g->skey.p);
        const uint8_t all = (uint8_t)((1u << nl) - 1u);
        uint8_t *f = f0.p, *fn = f1.p;
        int32_t depth = 0;
        for (int32_t level = 1;; ++level) {
            HIPX(hipMemsetAsync(grew.p, 0, 8, s));
            // a vertex joins a landmark's next level from an in-neighbour
            launch(s, grid_for(n), k_key_level, g->rrow(), g->rcol(), n, all, level,
                   (const uint8_t *)f, fn, seen.p, g->skey.p, grew.p);
            unsigned long long h = 0;
            HIPX(hipMemcpyAsync(&h, grew.p, 8, hipMemcpyDeviceToHost, s));
            HIPX(hipStreamSynchronize(s));
            if (!h) break;
            depth = level;
            std::swap(f, fn);
        }
        // bits per landmark: enough for the deepest level (unreached clamps)
        int32_t bits = 1;
        while (bits < 8 && (1 << bits) <= depth) ++bits;
        launch(s, grid_for(n), k_key_morton, g->skey.p, n, bits);
    } catch (...) {
        (void)hipStreamSynchronize(s);
        f0.release(); f1.release(); seen.release(); lm.release(); grew.release();
        throw;
    }
    f0.release(); f1.release(); seen.release(); lm.release(); grew.release();
    g->skey_ready = true;
}

// Temporary bytes of the lane-order sort of k keys (no device work).
size_t sort_temp_bytes(int64_t k)
{
    size_t bytes = 0;
    HIPX(rocprim::radix_sort_pairs(nullptr, bytes, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                   (const int32_t *)nullptr, (int32_t *)nullptr, (size_t)k, 0u,
                                   8u * (unsigned)sizeof(uint64_t), (hipStream_t)0));
    return bytes;
}

// g->w->operm[0..k) = the sample indices in ascending (key of source, index)
// order (a stable radix sort: deterministic for a given graph and input).
void order_samples(bc_graph *g, const int32_t *sources, int64_t k)
{
    ensure_source_keys(g);
    hipStream_t s = g->stream;
    Work &w = *g->w;
    w.okey_in.ensure((size_t)k);
    w.okey_out.ensure((size_t)k);
    w.oidx_in.ensure((size_t)k);
    w.operm.ensure((size_t)k);
    launch(s, grid_for(k), k_key_gather, (const uint64_t *)g->skey.p, sources, k, w.okey_in.p,
           w.oidx_in.p);
    size_t bytes = sort_temp_bytes(k);
    w.sort_tmp.ensure(std::max<size_t>(bytes, 1));
    HIPX(rocprim::radix_sort_pairs(w.sort_tmp.p, bytes, w.okey_in.p, w.okey_out.p, w.oidx_in.p,
                                   w.operm.p, (size_t)k, 0u, 8u * (unsigned)sizeof(uint64_t), s));
}

// Lane order inside a sampler or server round: the nb samples drawn into
// g->w->srcs (and g->w->dest for pairs) are sorted by the lane-order key in
// place; lane_row[b] is lane b's position in draw order, so gathers can hand
// the stop rule its values in draw order. Returns null when the round keeps
// draw order (small rounds, graphs without edges).
const int32_t *order_round(bc_graph *g, int nb, bool pair, int B)
{
    if (nb < kOrderMin || g->landmarks.empty()) return nullptr;
    Work &w = *g->w;
    hipStream_t s = g->stream;
    w.draw_src.ensure((size_t)nb);
    w.draw_dst.ensure((size_t)nb);
    w.lane_row.ensure((size_t)B);
    HIPX(hipMemcpyAsync(w.draw_src.p, w.srcs.p, (size_t)nb * 4, hipMemcpyDeviceToDevice, s));
    if (pair)
        HIPX(hipMemcpyAsync(w.draw_dst.p, w.dest.p, (size_t)nb * 4, hipMemcpyDeviceToDevice, s));
    order_samples(g, w.draw_src.p, nb);
    launch(s, grid_for(nb), k_take_batch, (const int32_t *)w.operm.p, (int64_t)0, (int32_t)nb,
           (const int32_t *)w.draw_src.p, pair ? (const int32_t *)w.draw_dst.p : nullptr,
           w.srcs.p, w.dest.p, w.lane_row.p);
    return w.lane_row.p;
}

// ------------------------------------------------------------ dependencies

// The record capacity a batch starts from: what earlier batches on the graph
// needed, within the work's limit.
int64_t start_cap(const bc_graph *g)
{
    const int64_t c = std::max<int64_t>(g->cap_hint, 1 << 16);
    return g->w->cap_limit > 0 ? std::min(c, g->w->cap_limit) : c;
}

// `fixed`: run the wave engine at that plan, in the caller's sample order (no
// depth probe, no lane-order sort): the allocation-free entry point's form.
void dependencies_impl(bc_graph *g, const int32_t *sources, int64_t k, int32_t mode, double *out,
                       int32_t *dist_out, double *sig_m, int32_t *sig_e, bool pair,
                       const int32_t *dests, const int32_t *targets = nullptr, int32_t T = 0,
                       const Plan *fixed = nullptr)
{
    const int64_t n = g->n;
    hipStream_t s = g->stream;
    g->stats = bc_stats{};
    // the sum over an empty source list is zero
    if (mode == BC_OUT_SUM && out) HIPX(hipMemsetAsync(out, 0, (size_t)n * 8, s));
    if (k == 0) {
        HIPX(hipStreamSynchronize(s));
        return;
    }
    if (dist_out) launch(s, grid_for(k * n), k_fill_i32, dist_out, (int32_t)-1, k * n);
    if (sig_m) launch(s, grid_for(k * n), k_fill_f64, sig_m, 0.0, k * n);
    if (sig_e) launch(s, grid_for(k * n), k_fill_i32, sig_e, (int32_t)0, k * n);
    if (g->weighted) {
        weighted_dependencies(g, sources, k, mode, out, dist_out, sig_m, sig_e, pair, dests,
                              targets, T);
        return;
    }

    if (!fixed && per_source_schedule(g) && !pair) {
        for (int64_t i = 0; i < k; ++i) {
            std::vector<int64_t> off = run_single(g, sources + i);
            if (mode == BC_OUT_SUM)
                launch(s, grid_for(off.back() - 1), k_ss_out_sum, (const double *)g->w->ss_dlt.p,
                       (const int32_t *)g->w->ss_q.p, (int64_t)1, off.back(), out);
            else if (mode == BC_OUT_TARGETS)
                launch(s, grid_for(T), k_ss_out_targets, (const int32_t *)g->w->ss_d.p,
                       (const double *)g->w->ss_dlt.p, targets, T, out + i * T);
            else
                launch(s, grid_for(n), k_ss_out_full, (const int32_t *)g->w->ss_d.p,
                       (const double *)g->w->ss_dlt.p, n, out + i * n);
            if (dist_out)
                HIPX(hipMemcpyAsync(dist_out + i * n, g->w->ss_d.p, (size_t)n * 4,
                                    hipMemcpyDeviceToDevice, s));
        }
        g->stats.samples_executed = k;
        g->stats.batches = k;
        g->stats.batch_width = 1;
        g->stats.schedule = BC_SCHED_PER_SOURCE;
        HIPX(hipStreamSynchronize(s));
        return;
    }

    if (!fixed && engine_for(g) == ENG_WG) {
        wg_dependencies(g, sources, k, mode, out, dist_out, sig_m, sig_e, pair, dests, targets,
                        T);
        return;
    }
    if (!fixed && engine_for(g) == ENG_PAIR) {
        const int B = plan_pairs(g, k, g->tuned_batch ? g->tuned_batch : 512);
        g->stats.batch_width = B;
        g->stats.schedule = BC_SCHED_THREADED;
        for (int64_t b0 = 0; b0 < k; b0 += B) {
            const int count = (int)std::min<int64_t>(B, k - b0);
            ensure_pairs(g, B, false);
            HIPX(hipMemcpyAsync(g->w->srcs.p, sources + b0, (size_t)count * 4,
                                hipMemcpyDeviceToDevice, s));
            if (pair)
                HIPX(hipMemcpyAsync(g->w->dest.p, dests + b0, (size_t)count * 4,
                                    hipMemcpyDeviceToDevice, s));
            PairSigmaOut so;
            so.mant = sig_m;
            so.ex = sig_e;
            so.count = count;
            so.b0 = b0;
            bool ext = false;
            run_pairs(g, B, count, pair, &ext, &so);
            PairArgs a = make_pair_args(g, B, ext, count, pair);
            if (mode == BC_OUT_SUM) launch(s, grid_for(n), k_p_out_sum, a, out);
            else if (mode == BC_OUT_TARGETS)
                launch(s, grid_for((int64_t)count * T), k_p_out_targets, a, targets, T,
                       (int32_t)count, b0, out);
            else launch(s, grid_for(n * count), k_p_out_full, a, (int32_t)count, b0, out);
            if (dist_out)
                HIPX(hipMemcpyAsync(dist_out + b0 * n, g->w->lv.p, (size_t)count * n * 4,
                                    hipMemcpyDeviceToDevice, s));
            g->stats.batches += 1;
            g->stats.samples_executed += count;
        }
        HIPX(hipStreamSynchronize(s));
        prof_flush(g);
        return;
    }

    const Plan p = fixed ? *fixed : plan_batch(g, k, g->tuned_batch ? g->tuned_batch : 2048);
    g->stats.batch_width = p.B;
    g->stats.schedule = BC_SCHED_BATCHED;
    // samples sorted by the clustering key, cut into batches, rows mapped back
    const bool ordered = !fixed && k >= kOrderMin && !g->landmarks.empty();
    if (ordered) order_samples(g, sources, k);
    for (int64_t b0 = 0; b0 < k; b0 += p.B) {
        const int count = (int)std::min<int64_t>(p.B, k - b0);
        const OutKind kind = mode == BC_OUT_SUM ? OUT_VSUM : OUT_DELTA;
        ensure_batch(g, p, false, start_cap(g), kind);
        if (ordered) {
            g->w->lane_row.ensure((size_t)p.B);
            launch(s, grid_for(count), k_take_batch, (const int32_t *)g->w->operm.p, b0, count,
                   sources, pair ? dests : (const int32_t *)nullptr, g->w->srcs.p, g->w->dest.p,
                   g->w->lane_row.p);
        } else {
            HIPX(hipMemcpyAsync(g->w->srcs.p, sources + b0, (size_t)count * 4,
                                hipMemcpyDeviceToDevice, s));
            if (pair)
                HIPX(hipMemcpyAsync(g->w->dest.p, dests + b0, (size_t)count * 4,
                                    hipMemcpyDeviceToDevice, s));
        }
        const int32_t *lane_row = ordered ? (const int32_t *)g->w->lane_row.p : nullptr;
        SigmaOut so;
        so.mant = sig_m;
        so.ex = sig_e;
        so.count = count;
        so.b0 = b0;
        so.lane_row = lane_row;
        bool ext = false;
        std::vector<int64_t> off = run_batch(g, p, count, pair, &ext, &so, kind);
        BatchArgs a = make_args(g, p, ext, count, pair, (int64_t)g->w->ridx.cap, kind);
        a.lane_row = lane_row;
        if (mode == BC_OUT_SUM) {
            const int64_t vb = vsum_tile_vertices(a.logW);
            launch(s, (int)std::min<int64_t>((n + vb - 1) / vb, 1 << 16), k_out_vsum, a, out);
        } else if (mode == BC_OUT_TARGETS)
            launch(s, grid_for((int64_t)count * T), k_out_targets, a, targets, T, (int32_t)count,
                   b0, out);
        else launch(s, grid_for(n * count), k_out_full, a, (int32_t)count, b0, out);
        if (dist_out)
            for (size_t l = 0; l + 1 < off.size(); ++l)
                launch(s, grid_for(off[l + 1] - off[l]), k_out_dist, a, off[l], off[l + 1],
                       (int32_t)l, (int32_t)count, b0, dist_out);
        g->stats.batches += 1;
        g->stats.samples_executed += count;
    }
    HIPX(hipStreamSynchronize(s));
    prof_flush(g);
}

// bc_pair_dependencies by the two-sided search, in launches of kBiChunk pairs;
// a launch whose counts reached 2^1000 is run again one-sided.
void pair_dependencies_bidir(bc_graph *g, const int32_t *us, const int32_t *vs, int64_t k,
                             double *out)
{
    const int64_t n = g->n;
    hipStream_t s = g->stream;
    if (k > 0) launch(s, grid_for(k * n), k_fill_f64, out, 0.0, k * n);
    bc_stats st{};
    st.pair_search = BC_PAIR_SEARCH_BIDIRECTIONAL;
    for (int64_t b0 = 0; b0 < k; b0 += kBiChunk) {
        const int count = (int)std::min<int64_t>(kBiChunk, k - b0);
        if (use_bidir(g) && run_bidir(g, us + b0, vs + b0, count, nullptr, 0, 0, nullptr,
                                      out + b0 * n)) {
            st.batches += 1;
            st.samples_executed += count;
            st.batch_width = std::max(st.batch_width, std::min(g->w->bslots, count));
            continue;
        }
        dependencies_impl(g, us + b0, count, BC_OUT_FULL, out + b0 * n, nullptr, nullptr,
                          nullptr, true, vs + b0);
        st.batches += g->stats.batches;
        st.samples_executed += g->stats.samples_executed;
        st.levels += g->stats.levels;
        st.extended |= g->stats.extended;
        st.batch_width = std::max(st.batch_width, g->stats.batch_width);
        st.bottom_up = g->stats.bottom_up;
        st.pair_search = BC_PAIR_SEARCH_ONE_SIDED;
    }
    st.schedule = schedule_of(engine_for(g));
    HIPX(hipStreamSynchronize(s));
    prof_flush(g);
    g->stats = st;
}

// -------------------------------------------------------------- autotuner
//
// Times candidate plans on one seeded batch of sources each and keeps the
// fastest per source, by coordinate descent: the engine (wave per word,
// thread per pair, or workgroup per source on deep or small graphs) at its
// default width, then the batch width, then, for the wave engine, the
// bottom-up threshold, or, for the pair engine, the persistent level loop. A candidate that runs
// past 1.5x the best time for its batch is abandoned at a level boundary.
// Winners are cached per process by graph signature (size, log2-degree
// histogram, BFS depth from the hub). Every plan only changes how sources
// are scheduled: results are those of any other plan (sums up to FP64
// summation order).

struct TuneKey {
    int64_t n, nnz;
    int32_t depth;
    std::array<int64_t, 33> hist;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(n, nnz, depth, hist) < std::tie(o.n, o.nnz, o.depth, o.hist);
    }
};

std::mutex tune_mu;
std::map<TuneKey, bc_config> tune_cache;

constexpr int kTuneWidths[] = {4096, 2048, 1024, 512, 256};
constexpr double kTuneBottomUp[] = {0.04, 0.01, 0.15, -1.0};
constexpr uint64_t kTuneSeed = 0x74756e65ull;   // the sample sources' Philox key

// Widest width <= want that an engine serves on this graph (32-bit indices,
// 70 % of free device memory).
int fit_width(bc_graph *g, Engine e, int want)
{
    bc_config keep = g->cfg;
    g->cfg.batch = want;
    const int B = e == ENG_PAIR ? plan_pairs(g, want, want)
                  : e == ENG_WG ? plan_wg(g, want, want) : plan_batch(g, want, want).B;
    g->cfg = keep;
    return B;
}

bc_config tune_plan(bc_graph *g)
{
    if (g->weighted) {
        // one engine serves weighted graphs: nothing to choose but the width
        bc_config c = g->cfg;
        c.schedule = BC_SCHED_BATCHED;
        c.batch = 0;
        return c;
    }
    const TuneKey key{g->n, g->nnz, probe_depth(g), g->deg_hist};
    {
        std::lock_guard<std::mutex> lock(tune_mu);
        auto it = tune_cache.find(key);
        if (it != tune_cache.end()) return it->second;
    }
    const int64_t n = g->n;
    hipStream_t s = g->stream;
    DBuf<int32_t> sample;
    DBuf<double> out;
    sample.ensure(4096);
    out.ensure((size_t)n);
    launch(s, grid_for(4096), k_draw_sources, kTuneSeed, (int64_t)0, (int64_t)4096, n, sample.p);
    const bc_config user = g->cfg;
    const int32_t user_batch = g->tuned_batch;
    double best_per = 0.0;
    bc_config best{};
    bool have = false;
    // seconds per source of k sources (default: one batch of width c.batch)
    // under plan c, or < 0 when abandoned
    auto trial = [&](bc_config c, int64_t k) -> double {
        if (k <= 0) k = std::min<int64_t>(n, c.batch);
        g->cfg = c;
        g->tuned_batch = 0;
        double per = -1.0;
        try {
            // size the plan's buffers first, so that allocation is not timed
            if (c.schedule == BC_SCHED_THREADED) {
                ensure_pairs(g, c.batch, g->ext_sticky);
            } else if (c.schedule == BC_SCHED_WORKGROUP) {
                ensure_wg(g, plan_wg(g, k, c.batch), g->ext_sticky, true);
            } else {
                const Plan p = plan_batch(g, k, c.batch);
                ensure_batch(g, p, g->ext_sticky, start_cap(g), OUT_VSUM);
            }
            HIPX(hipStreamSynchronize(s));
            g->timed = have;
            g->deadline = std::chrono::steady_clock::now() +
                          std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                              std::chrono::duration<double>(std::max(0.05, 1.5 * best_per * k)));
            const auto t0 = std::chrono::steady_clock::now();
            dependencies_impl(g, sample.p, k, BC_OUT_SUM, out.p, nullptr, nullptr, nullptr, false,
                              nullptr);
            per = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() /
                  (double)k;
        } catch (const TuneTimeout &) {
            (void)hipStreamSynchronize(s);
        } catch (...) {
            g->timed = false;
            g->cfg = user;
            g->tuned_batch = user_batch;
            throw;
        }
        g->timed = false;
        if (per > 0.0 && (!have || per < best_per)) {
            best_per = per;
            best = c;
            have = true;
        }
        return per;
    };
    auto make = [&](Engine e, int B) {
        bc_config c{};
        c.schedule = schedule_of(e);
        c.batch = fit_width(g, e, B);
        return c;
    };
    try {
        // 1. engine, the heuristic one first, on the same 256 sources
        const Engine first = probe_depth(g) > kDeepGraphLevels ? ENG_PAIR : ENG_WAVE;
        const Engine second = first == ENG_PAIR ? ENG_WAVE : ENG_PAIR;
        const int64_t k_eng = std::min<int64_t>(n, 256);
        trial(make(first, first == ENG_PAIR ? 512 : 2048), k_eng);
        trial(make(second, second == ENG_PAIR ? 512 : 2048), k_eng);
        // one workgroup per source: a single launch that cannot be abandoned,
        // and on a large shallow graph one pass walks wide levels with one
        // workgroup (~0.26 s on 2^20 vertices): tried on deep or small graphs
        if (probe_depth(g) > kDeepGraphLevels || n <= kWgTrialMaxShallow)
            trial(make(ENG_WG, 1024), k_eng);
        // 2. batch width, widest first (buffers grow once), up to the first
        // width that holds all n sources; each timed on a batch of its width
        const Engine e = best.schedule == BC_SCHED_THREADED    ? ENG_PAIR
                         : best.schedule == BC_SCHED_WORKGROUP ? ENG_WG
                                                               : ENG_WAVE;
        have = false;
        int prev = 0;
        // one workgroup per source: fewer passes in flight keep more of the
        // slots' records in cache, so narrower widths are candidates too
        static const int kWgWidths[] = {1024, 512, 256, 128, 64};
        const bool wg = e == ENG_WG;
        for (int W : wg ? std::vector<int>(std::begin(kWgWidths), std::end(kWgWidths))
                        : std::vector<int>(std::begin(kTuneWidths), std::end(kTuneWidths))) {
            if (W > 2 * n && W > 256) continue;
            bc_config c = make(e, W);
            if (c.batch == prev) continue;
            prev = c.batch;
            trial(c, 0);
        }
        // 3. the engine's own knobs at the best width
        const bc_config width = best;
        const double width_per = best_per;
        if (e == ENG_WAVE) {
            for (double bu : kTuneBottomUp) {
                if (bu == 0.04) continue;
                bc_config c = width;
                c.bottom_up = bu;
                trial(c, 0);
            }
        } else if (e == ENG_PAIR) {
            // a persistent loop cannot be abandoned mid-launch: it is tried
            // where a batch takes under 50 ms (many short levels)
            int coop = 0;
            HIPX(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, g->device));
            if (coop && width_per * std::min<int64_t>(n, width.batch) < 0.05) {
                bc_config c = width;
                c.level_loop = 1;
                trial(c, 0);
            }
        }
    } catch (...) {
        sample.release();
        out.release();
        throw;
    }
    sample.release();
    out.release();
    // the candidates' buffers go back: the winner sizes its own from free memory
    g->w->release_engines();
    g->cfg = user;
    g->tuned_batch = user_batch;
    if (!have) fail(BC_E_DEVICE, "no tuning candidate finished");
    {
        std::lock_guard<std::mutex> lock(tune_mu);
        tune_cache[key] = best;
    }
    return best;
}

// Install a tuned plan: engine and knobs in cfg, width for bc_dependencies and
// bc_exact only (the samplers keep their own round widths).
void apply_plan(bc_graph *g, const bc_config &plan)
{
    // the caller's sampler width and pair search, not tuned
    const int32_t sampler_batch = g->cfg.sampler_batch, pair_search = g->cfg.pair_search;
    g->cfg = plan;
    g->tuned_batch = plan.batch;
    g->cfg.batch = 0;
    g->cfg.sampler_batch = sampler_batch;
    g->cfg.pair_search = pair_search;
    g->tuned = true;
}

void ensure_tuned(bc_graph *g)
{
    if (g->cfg.schedule == BC_SCHED_TUNED && !g->tuned) apply_plan(g, tune_plan(g));
}

std::map<std::pair<TuneKey, int>, double> round_bu_cache;

// Bottom-up threshold for the wave engine's source rounds of width B under a
// tuned plan. The plan's threshold was chosen at the plan's own width; a
// bottom-up level scans every unvisited (vertex, word) entry while a top-down
// one follows the frontier, and the balance between them moves with the
// number of words per vertex, so the candidates are tried again at the round
// width: each is timed on up to eight rounds of the tuner's seeded sources,
// twice, the candidates alternating (nearby thresholds differ by a few per
// cent, about what one short trial varies by), and the fastest of each
// candidate's two times decides, the plan's own threshold winning ties. The
// choice is kept per graph shape and width. Values do not depend on the
// threshold, only the time does.
double round_bottom_up(bc_graph *g, const Plan &p)
{
    const double planned = g->cfg.bottom_up;
    if (p.B == g->tuned_batch) return planned;
    const TuneKey tk{g->n, g->nnz, probe_depth(g), g->deg_hist};
    const auto key = std::make_pair(tk, p.B);
    {
        std::lock_guard<std::mutex> lock(tune_mu);
        auto it = round_bu_cache.find(key);
        if (it != round_bu_cache.end()) return it->second;
    }
    const int64_t n = g->n;
    const int64_t k = std::min<int64_t>(n, 8 * (int64_t)p.B);
    hipStream_t s = g->stream;
    DBuf<int32_t> sample;
    DBuf<double> out;
    sample.ensure((size_t)k);
    out.ensure((size_t)n);
    launch(s, grid_for(k), k_draw_sources, kTuneSeed, (int64_t)0, k, n, sample.p);
    const bc_config user = g->cfg;
    const int32_t user_batch = g->tuned_batch;
    auto restore = [&] {
        g->timed = false;
        g->cfg = user;
        g->tuned_batch = user_batch;
    };
    std::vector<double> cand{planned};
    for (double bu : kTuneBottomUp)
        if (bu != bottom_up_fraction(g)) cand.push_back(bu);
    // each candidate's fastest time; < 0 until timed, infinite once abandoned
    std::vector<double> best_t(cand.size(), -1.0);
    double best_all = 0.0;
    bool have = false;
    try {
        // one untimed round first, so that no candidate is timed cold
        g->cfg.batch = p.B;
        g->tuned_batch = 0;
        dependencies_impl(g, sample.p, std::min<int64_t>(k, p.B), BC_OUT_SUM, out.p, nullptr,
                          nullptr, nullptr, false, nullptr);
        for (int pass = 0; pass < 2; ++pass) {
            for (size_t c = 0; c < cand.size(); ++c) {
                if (std::isinf(best_t[c])) continue;
                g->cfg.batch = p.B;
                g->cfg.bottom_up = cand[c];
                g->tuned_batch = 0;
                ensure_batch(g, plan_batch(g, k, p.B), g->ext_sticky, start_cap(g), OUT_VSUM);
                HIPX(hipStreamSynchronize(s));
                g->timed = have;
                g->deadline = std::chrono::steady_clock::now() +
                              std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                                  std::chrono::duration<double>(std::max(0.05, 1.5 * best_all)));
                const auto t0 = std::chrono::steady_clock::now();
                try {
                    dependencies_impl(g, sample.p, k, BC_OUT_SUM, out.p, nullptr, nullptr,
                                      nullptr, false, nullptr);
                } catch (const TuneTimeout &) {
                    (void)hipStreamSynchronize(s);
                    if (best_t[c] < 0) best_t[c] = std::numeric_limits<double>::infinity();
                    continue;
                }
                const double t =
                    std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                if (best_t[c] < 0 || t < best_t[c]) best_t[c] = t;
                if (!have || t < best_all) best_all = t;
                have = true;
            }
        }
    } catch (...) {
        restore();
        sample.release();
        out.release();
        throw;
    }
    restore();
    sample.release();
    out.release();
    double best = planned, bt = std::numeric_limits<double>::infinity();
    for (size_t c = 0; c < cand.size(); ++c)
        if (best_t[c] >= 0 && best_t[c] < bt) {
            bt = best_t[c];
            best = cand[c];
        }
    {
        std::lock_guard<std::mutex> lock(tune_mu);
        round_bu_cache[key] = best;
    }
    return best;
}

// --------------------------------------------------------------- samplers

void sampler_impl(bc_graph *g, const int32_t *targets, int32_t T, bool pair, int32_t rule,
                  double c, double eps, uint64_t seed, int64_t k_max, double *out_est,
                  int64_t *out_samples, double *out_S, uint8_t *out_status)
{
    const int64_t n = g->n;
    hipStream_t s = g->stream;
    g->stats = bc_stats{};
    if (T == 0) return;
    // the one-workgroup-per-source engine hands sampler rounds to the pair engine
    const bool use_pairs = engine_for(g) != ENG_WAVE;
    // round width: the configured one, else 256 source samples or 2048 pair
    // samples (a sampler's stop rule sees samples in draw order, so a round
    // runs ahead of it by up to its width; pair searches stop early, and wider
    // rounds of them measured faster: 0.92 s against 1.17 s at 256 on the BA
    // n = 2^20 pair workload)
    const int32_t keep_batch = g->cfg.batch;
    if (g->cfg.sampler_batch > 0) g->cfg.batch = g->cfg.sampler_batch;
    const int round = pair ? 2048 : 256;
    Plan p = plan_batch(g, k_max, round);
    if (g->weighted) {
        p.B = plan_weighted(g, k_max, round);
    } else if (use_pairs) {
        // the pair engine takes any power-of-two width; keep the sampler's stride
        p.B = plan_pairs(g, k_max, round);
    }
    g->cfg.batch = keep_batch;
    // source rounds of a width other than the tuned plan's take a bottom-up
    // threshold tried at their own width, for this call only
    struct KeepBottomUp {
        bc_graph *g;
        double v;
        ~KeepBottomUp() { g->cfg.bottom_up = v; }
    } keep_bu{g, g->cfg.bottom_up};
    if (g->tuned && !pair && !use_pairs && !g->weighted) {
        g->cfg.bottom_up = round_bottom_up(g, p);
        g->stats = bc_stats{};
    }
    g->stats.batch_width = p.B;
    g->stats.schedule = use_pairs ? BC_SCHED_THREADED : BC_SCHED_BATCHED;
    g->w->X.ensure((size_t)T * p.B);
    g->w->S.ensure((size_t)T);
    g->w->K.ensure((size_t)T);
    g->w->st.ensure((size_t)T);
    StopArgs sa;
    sa.T = T;
    sa.rule = rule;
    sa.threshold = c * (double)n;
    sa.eps_rhs = ((eps * eps) * eps) * ((double)n * (double)n);
    sa.k_max = k_max;
    sa.S = g->w->S.p;
    sa.K = g->w->K.p;
    sa.status = g->w->st.p;
    launch(s, grid_for(T), k_stop_init, sa);
    int64_t j0 = 0;
    bool one_sided = pair && !use_bidir(g);
    for (;;) {
        const int nb = (int)std::min<int64_t>(p.B, k_max - j0);
        const bool bidir = pair && use_bidir(g);
        if (g->weighted) {
            ensure_weighted(g, p.B);
        } else if (bidir) {
            g->w->srcs.ensure((size_t)p.B);
            g->w->dest.ensure((size_t)p.B);
        } else if (use_pairs) {
            ensure_pairs(g, p.B, false);
        } else {
            ensure_batch(g, p, false, start_cap(g), OUT_DELTA);
        }
        if (pair)
            launch(s, grid_for(nb), k_draw_pairs, seed, j0, (int64_t)nb, n, g->w->srcs.p, g->w->dest.p);
        else
            launch(s, grid_for(nb), k_draw_sources, seed, j0, (int64_t)nb, n, g->w->srcs.p);
        bool ext = false;
        bool done = false;
        if (bidir) {
            done = run_bidir(g, g->w->srcs.p, g->w->dest.p, nb, targets, T, p.B, g->w->X.p,
                             nullptr);
            if (!done) {
                // counts reached 2^1000: this round (its draws are in place) one-sided
                one_sided = true;
                if (use_pairs) ensure_pairs(g, p.B, false);
                else ensure_batch(g, p, false, start_cap(g), OUT_DELTA);
            }
        }
        if (done) {
        } else if (g->weighted) {
            run_weighted(g, p.B, nb, pair);
            const WArgs a = make_weighted_args(g, p.B, nb, pair);
            launch(s, grid_for((int64_t)T * p.B), k_ww_gather_targets, a, targets, T,
                   (int32_t)p.B, g->w->X.p);
        } else if (use_pairs) {
            run_pairs(g, p.B, nb, pair, &ext, nullptr);
            PairArgs a = make_pair_args(g, p.B, ext, nb, pair);
            launch(s, grid_for((int64_t)T * p.B), k_p_gather_targets, a, targets, T,
                   (int32_t)p.B, g->w->X.p);
        } else {
            const int32_t *lane_row = order_round(g, nb, pair, p.B);
            run_batch(g, p, nb, pair, &ext, nullptr, OUT_DELTA);
            BatchArgs a = make_args(g, p, ext, nb, pair, (int64_t)g->w->ridx.cap, OUT_DELTA);
            a.lane_row = lane_row;
            launch(s, grid_for((int64_t)T * p.B), k_gather_targets, a, targets, T, g->w->X.p);
        }
        launch(s, grid_for(T), k_stop_rule, sa, (const double *)g->w->X.p, (int32_t)p.B, (int32_t)nb,
               g->w->ctl.p);
        read_ctl(g);
        j0 += nb;
        g->stats.batches += 1;
        if (g->w->h_ctl[CTL_RUNNING] == 0) break;
        if (j0 >= k_max) fail(BC_E_DEVICE, "stop rule left targets running at k_max");
    }
    g->stats.samples_executed = j0;
    if (pair) g->stats.pair_search = one_sided ? BC_PAIR_SEARCH_ONE_SIDED : BC_PAIR_SEARCH_BIDIRECTIONAL;
    const double scale = pair ? (double)n * (double)(n - 1) : (double)n;
    launch(s, grid_for(T), k_stop_finish, sa, scale, out_est, out_samples, out_S, out_status);
    HIPX(hipStreamSynchronize(s));
    prof_flush(g);
}

// ---------------------------------------------------------- CSR validation

template <class R>
void validate_csr(const bc_csr *c, const R *row, bool symmetric)
{
    const int64_t n = c->n, nnz = c->nnz;
    need(row[0] == 0, "row[0] must be 0");
    need((int64_t)row[n] == nnz, "row[n] must equal nnz");
    for (int64_t v = 0; v < n; ++v) {
        const int64_t b = (int64_t)row[v], e = (int64_t)row[v + 1];
        need(b <= e, "row offsets must be non-decreasing");
        for (int64_t i = b; i < e; ++i) {
            const int32_t w = c->col[i];
            need(w >= 0 && w < n, "column index outside [0, n)");
            need(w != v, "self-loop");
            need(i == b || c->col[i - 1] < w, "rows must be sorted ascending without duplicates");
        }
    }
    if (!symmetric) return;
    // symmetry: every (v, w) needs (w, v)
    for (int64_t v = 0; v < n; ++v) {
        for (int64_t i = (int64_t)row[v]; i < (int64_t)row[v + 1]; ++i) {
            const int32_t w = c->col[i];
            const int32_t *lo = c->col + (int64_t)row[w], *hi = c->col + (int64_t)row[w + 1];
            need(std::binary_search(lo, hi, (int32_t)v), "CSR is not symmetric");
        }
    }
}

}  // namespace

// ------------------------------------------------ allocation-free variant

// Scratch of bc_dependencies_noalloc: a file-scope device array, one copy on
// each device, held until the process ends. Host code reaches it only through
// the address hipGetSymbolAddress gives for the current device.
static __device__ __align__(256) unsigned char scratch[BC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
unsigned char *scratch_dev[kMaxDevices] = {};

// The scratch array's device address on device `dev`, which must be current
// (looked up once per device).
unsigned char *scratch_on(int dev)
{
    need(dev >= 0 && dev < kMaxDevices, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        HIPX(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        need(p != nullptr, "no address for the scratch array");
        scratch_dev[dev] = (unsigned char *)p;
    }
    return scratch_dev[dev];
}

// Consecutive 256-byte-aligned pieces of the scratch array, as buffer views.
struct Carve {
    unsigned char *base;
    size_t cap;
    size_t used = 0;
    size_t left() const
    {
        const size_t at = (used + 255) & ~(size_t)255;
        return at >= cap ? 0 : cap - at;
    }
    template <class T>
    bool take(DBuf<T> &b, size_t count)
    {
        const size_t at = (used + 255) & ~(size_t)255;
        const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        if (at > cap || bytes > cap - at) return false;
        b.view((T *)(base + at), count);
        used = at + bytes;
        return true;
    }
};

}  // namespace

// ===================================================================== ABI

extern "C" {

const char *bc_last_error(void) { return tl_error.c_str(); }

}  // extern "C"

namespace {

// Validate a host CSR (symmetric unless directed) and build the handle: the
// device copy of the rows and, for a directed graph, of its in-neighbour rows.
// Arc weights: positive, max weight * (n - 1) < 2^30 (distances and their
// sums stay exact in int32), and on an undirected graph equal on both arcs of
// an edge.
void validate_weights(const bc_csr *c, const std::vector<int64_t> &row, const int32_t *wt,
                      bool directed)
{
    int32_t most = 0;
    for (int64_t e = 0; e < c->nnz; ++e) {
        need(wt[e] > 0, "arc weights must be positive");
        most = std::max(most, wt[e]);
    }
    need((int64_t)most * (c->n - 1) < (1ll << 30), "max weight * (n - 1) must be below 2^30");
    if (directed) return;
    for (int64_t v = 0; v < c->n; ++v)
        for (int64_t e = row[(size_t)v]; e < row[(size_t)v + 1]; ++e) {
            const int32_t w = c->col[e];
            const int32_t *lo = c->col + row[(size_t)w], *hi = c->col + row[(size_t)w + 1];
            const int32_t *f = std::lower_bound(lo, hi, (int32_t)v);
            need(wt[f - c->col] == wt[e], "the two arcs of an edge carry different weights");
        }
}

// The rows longer than kHub in `row`: the first part (of kPart neighbours)
// of each in the part-sum slab, rows in vertex order, -1 for shorter rows,
// uploaded to `out`; their vertices, ascending, uploaded to `list`; their
// number, their parts and the most parts of one row.
void hub_table(const std::vector<int64_t> &row, DBuf<int32_t> &out, DBuf<int32_t> &list,
               int64_t &hubs, int64_t &parts, int32_t &most)
{
    const size_t n = row.size() - 1;
    std::vector<int32_t> h(n, -1), vs;
    hubs = parts = 0;
    most = 0;
    for (size_t v = 0; v < n; ++v) {
        const int64_t d = row[v + 1] - row[v];
        if (d <= kHub) continue;
        h[v] = (int32_t)parts;
        vs.push_back((int32_t)v);
        const int64_t q = (d + kPart - 1) / kPart;
        parts += q;
        hubs += 1;
        most = (int32_t)std::max<int64_t>(most, q);
        need(parts < (1ll << 31), "too many long rows");
    }
    out.ensure(n);
    HIPX(hipMemcpy(out.p, h.data(), n * 4, hipMemcpyHostToDevice));
    list.ensure(std::max<size_t>(vs.size(), 1));
    if (!vs.empty())
        HIPX(hipMemcpy(list.p, vs.data(), vs.size() * 4, hipMemcpyHostToDevice));
}

void create_graph(const bc_csr *csr, const bc_allocator *alloc, void *hip_stream, bc_graph **out,
                  bool directed, const int32_t *weights = nullptr)
{
    {
        need(csr && out, "null argument");
        need(csr->n >= 1 && csr->n < 0x7fffffffll, "n must be in [1, 2^31 - 1)");
        need(csr->nnz >= 0 && csr->row && (csr->col || csr->nnz == 0), "bad CSR arrays");
        need(!alloc || (alloc->alloc && alloc->free), "allocator needs both alloc and free");
        std::vector<int64_t> row((size_t)csr->n + 1);
        if (csr->row_is_i64) {
            const int64_t *r = (const int64_t *)csr->row;
            validate_csr(csr, r, !directed);
            std::copy(r, r + csr->n + 1, row.begin());
        } else {
            need(csr->nnz < 0x7fffffffll, "int32 row offsets need nnz < 2^31");
            const int32_t *r = (const int32_t *)csr->row;
            validate_csr(csr, r, !directed);
            std::copy(r, r + csr->n + 1, row.begin());
        }
        if (weights) validate_weights(csr, row, weights, directed);
        bc_graph *g = new bc_graph();
        if (alloc) g->alloc.a = *alloc;
        UseAlloc ua(&g->alloc);
        try {
            HIPX(hipGetDevice(&g->device));
            g->n = csr->n;
            g->nnz = csr->nnz;
            int64_t best = -1;
            for (int64_t v = 0; v < csr->n; ++v)
                if (row[v + 1] - row[v] > best) {
                    best = row[v + 1] - row[v];
                    g->hub = (int32_t)v;
                }
            g->hub_degree = best;
            for (int64_t v = 0; v < csr->n; ++v) {
                int64_t d = row[v + 1] - row[v] + 1;
                int b = 0;
                while (d > 1) {
                    d >>= 1;
                    ++b;
                }
                g->deg_hist[(size_t)std::min(b, 32)] += 1;
            }
            {
                // landmarks: the kLandmarks highest degrees (ties by vertex id)
                std::vector<int32_t> ids((size_t)csr->n);
                for (int64_t v = 0; v < csr->n; ++v) ids[(size_t)v] = (int32_t)v;
                const size_t nl = std::min<size_t>(kLandmarks, ids.size());
                std::partial_sort(ids.begin(), ids.begin() + nl, ids.end(), [&](int32_t x, int32_t y) {
                    const int64_t dx = row[x + 1] - row[x], dy = row[y + 1] - row[y];
                    return dx != dy ? dx > dy : x < y;
                });
                for (size_t i = 0; i < nl; ++i)
                    if (row[ids[i] + 1] > row[ids[i]]) g->landmarks.push_back(ids[i]);
            }
            g->stream = (hipStream_t)hip_stream;
            g->row.ensure(row.size());
            g->col.ensure((size_t)csr->nnz);
            g->own.init();
            HIPX(hipMemcpy(g->row.p, row.data(), row.size() * 8, hipMemcpyHostToDevice));
            if (csr->nnz)
                HIPX(hipMemcpy(g->col.p, csr->col, (size_t)csr->nnz * 4, hipMemcpyHostToDevice));
            hub_table(row, g->hpart_buf, g->hlist_buf, g->hubs_out, g->parts_out, g->most_out);
            g->hubs_in = g->hubs_out;
            g->parts_in = g->parts_out;
            g->most_in = g->most_out;
            if (weights) {
                g->weighted = true;
                g->wt_buf.ensure((size_t)std::max<int64_t>(csr->nnz, 1));
                if (csr->nnz)
                    HIPX(hipMemcpy(g->wt_buf.p, weights, (size_t)csr->nnz * 4,
                                   hipMemcpyHostToDevice));
            }
            if (directed) {
                // in-neighbour rows, sorted ascending (sources visited in order)
                const int64_t n = csr->n;
                std::vector<int64_t> trow((size_t)n + 1, 0), fill((size_t)n);
                std::vector<int32_t> tcol((size_t)std::max<int64_t>(csr->nnz, 1));
                for (int64_t e = 0; e < csr->nnz; ++e) trow[(size_t)csr->col[e] + 1] += 1;
                for (int64_t v = 0; v < n; ++v) trow[(size_t)v + 1] += trow[(size_t)v];
                for (int64_t v = 0; v < n; ++v) fill[(size_t)v] = trow[(size_t)v];
                std::vector<int32_t> twt(weights ? tcol.size() : 0);
                for (int64_t u = 0; u < n; ++u)
                    for (int64_t e = row[(size_t)u]; e < row[(size_t)u + 1]; ++e) {
                        const int64_t at = fill[(size_t)csr->col[e]]++;
                        tcol[(size_t)at] = (int32_t)u;
                        if (weights) twt[(size_t)at] = weights[e];
                    }
                if (weights) {
                    g->rwt_buf.ensure(twt.size());
                    HIPX(hipMemcpy(g->rwt_buf.p, twt.data(), twt.size() * 4,
                                   hipMemcpyHostToDevice));
                }
                g->directed = true;
                hub_table(trow, g->rhpart_buf, g->rhlist_buf, g->hubs_in, g->parts_in,
                          g->most_in);
                g->rrow_buf.ensure(trow.size());
                g->rcol_buf.ensure((size_t)csr->nnz);
                HIPX(hipMemcpy(g->rrow_buf.p, trow.data(), trow.size() * 8, hipMemcpyHostToDevice));
                if (csr->nnz)
                    HIPX(hipMemcpy(g->rcol_buf.p, tcol.data(), (size_t)csr->nnz * 4,
                                   hipMemcpyHostToDevice));
            }
        } catch (...) {
            g->release_all();
            delete g;
            throw;
        }
        *out = g;
    }
}

}  // namespace

extern "C" {

bc_status bc_graph_create(const bc_csr *csr, const bc_allocator *alloc, void *hip_stream,
                          bc_graph **out)
{
    return guarded([&] { create_graph(csr, alloc, hip_stream, out, false); });
}

bc_status bc_graph_create_directed(const bc_csr *csr, const bc_allocator *alloc,
                                   void *hip_stream, bc_graph **out)
{
    return guarded([&] { create_graph(csr, alloc, hip_stream, out, true); });
}

bc_status bc_graph_create_weighted(const bc_csr *csr, const int32_t *weights, int32_t directed,
                                   const bc_allocator *alloc, void *hip_stream, bc_graph **out)
{
    return guarded([&] {
        need(csr && (weights || csr->nnz == 0), "null argument");
        static const int32_t none = 1;
        create_graph(csr, alloc, hip_stream, out, directed != 0, weights ? weights : &none);
    });
}

void bc_graph_destroy(bc_graph *g)
{
    if (!g) return;
    (void)hipSetDevice(g->device);
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    g->release_all();
    delete g;
}

bc_status bc_graph_set_stream(bc_graph *g, void *hip_stream)
{
    return guarded([&] {
        need(g, "null graph");
        g->stream = (hipStream_t)hip_stream;
    });
}

bc_status bc_graph_set_io(bc_graph *g, int32_t io)
{
    return guarded([&] {
        need(g, "null graph");
        need(io == BC_IO_DEVICE || io == BC_IO_HOST, "unknown io mode");
        g->io = io;
    });
}

bc_status bc_graph_configure(bc_graph *g, const bc_config *cfg)
{
    return guarded([&] {
        need(g && cfg, "null argument");
        need(cfg->schedule >= BC_SCHED_AUTO && cfg->schedule <= BC_SCHED_WORKGROUP,
             "unknown schedule");
        const int b = cfg->batch;
        need(b == 0 || (b >= 64 && b <= 4096 && (b & (b - 1)) == 0),
             "batch must be 0 or a power of two in [64, 4096]");
        const int sb = cfg->sampler_batch;
        need(sb == 0 || (sb >= 64 && sb <= 4096 && (sb & (sb - 1)) == 0),
             "sampler_batch must be 0 or a power of two in [64, 4096]");
        need(cfg->bottom_up == cfg->bottom_up, "bottom_up is NaN");
        need(cfg->pair_search >= BC_PAIR_SEARCH_AUTO &&
                 cfg->pair_search <= BC_PAIR_SEARCH_BIDIRECTIONAL,
             "unknown pair_search");
        g->cfg = *cfg;
        g->tuned = false;
        g->tuned_batch = 0;
    });
}

bc_status bc_graph_tune(bc_graph *g, bc_config *plan)
{
    return guarded([&] {
        need(g, "null graph");
        use_device(g);
        UseAlloc ua(&g->alloc);
        const bc_config best = tune_plan(g);
        apply_plan(g, best);
        if (plan) *plan = best;
    });
}

bc_status bc_graph_plan(bc_graph *g, bc_config *out)
{
    return guarded([&] {
        need(g && out, "null argument");
        use_device(g);
        UseAlloc ua(&g->alloc);
        ensure_tuned(g);
        bc_config c = g->cfg;
        if (c.schedule == BC_SCHED_AUTO)
            c.schedule = schedule_of(engine_for(g));
        if (c.batch == 0) c.batch = g->tuned_batch;
        *out = c;
    });
}

bc_status bc_graph_info(const bc_graph *g, int64_t *n, int64_t *nnz)
{
    return guarded([&] {
        need(g, "null graph");
        if (n) *n = g->n;
        if (nnz) *nnz = g->nnz;
    });
}

bc_status bc_last_stats(const bc_graph *g, bc_stats *out)
{
    return guarded([&] {
        need(g && out, "null argument");
        *out = g->stats;
    });
}

bc_status bc_profile_enable(bc_graph *g, int32_t enable)
{
    return guarded([&] {
        need(g, "null graph");
        use_device(g);
        UseAlloc ua(&g->alloc);
        prof_flush(g);
        g->prof_dev.ensure(2 * PROF_KERNELS * kProfSlots);
        HIPX(hipMemsetAsync(g->prof_dev.p, 0, 2 * PROF_KERNELS * kProfSlots * 8, g->stream));
        HIPX(hipStreamSynchronize(g->stream));
        for (int k = 0; k < PROF_KERNELS; ++k) {
            g->prof_ms[k] = 0.0;
            g->prof_launches[k] = 0;
            g->prof_host_units[2 * k] = 0;
            g->prof_host_units[2 * k + 1] = 0;
        }
        g->prof_on = enable != 0;
    });
}

bc_status bc_profile_read(bc_graph *g, bc_kernel_profile *out, int32_t max, int32_t *count)
{
    return guarded([&] {
        need(g && count && (max <= 0 || out), "null argument");
        use_device(g);
        prof_flush(g);
        unsigned long long units[2 * PROF_KERNELS] = {};
        if (g->prof_dev.p) {
            std::vector<unsigned long long> slots((size_t)2 * PROF_KERNELS * kProfSlots);
            HIPX(hipMemcpy(slots.data(), g->prof_dev.p, slots.size() * 8, hipMemcpyDeviceToHost));
            for (int k = 0; k < 2 * PROF_KERNELS; ++k)
                for (int q = 0; q < kProfSlots; ++q) units[k] += slots[(size_t)k * kProfSlots + q];
        }
        for (int k = 0; k < 2 * PROF_KERNELS; ++k) units[k] += (unsigned long long)g->prof_host_units[k];
        static const char *names[PROF_KERNELS] = {"discover_topdown", "discover_bottomup",
                                                  "sigma_pull", "backward", "level_record",
                                                  "hub_parts", "pair_forward",
                                                  "pair_backward", "bidir_pair", "w_search",
                                                  "w_counts", "w_backward", "wg_pass"};
        // level_record: each word read once (8 B); per entry the record
        // (4 + 8 + 8 B) and the visited word read and written (16 B)
        static const double per_a[PROF_KERNELS] = {4.0, 4.0, 8.0, 20.0, 8.0, 0.0, 12.0, 20.0,
                                                   36.0, 4.0, 16.0, 28.0, 36.0};
        static const double per_b[PROF_KERNELS] = {0.0, 0.0, 8.0, 8.0, 36.0, 8.0, 8.0, 8.0,
                                                   12.0, 8.0, 12.0, 12.0, 12.0};
        int32_t c = 0;
        for (int k = 0; k < PROF_KERNELS && c < max; ++k, ++c) {
            bc_kernel_profile &r = out[c];
            std::memset(&r, 0, sizeof(r));
            std::strncpy(r.name, names[k], sizeof(r.name) - 1);
            r.launches = g->prof_launches[k];
            r.ms = g->prof_ms[k];
            r.units_a = (int64_t)units[2 * k];
            r.units_b = (int64_t)units[2 * k + 1];
            r.algo_bytes = per_a[k] * (double)r.units_a + per_b[k] * (double)r.units_b;
        }
        *count = c;
    });
}

bc_status bc_exact(bc_graph *g, double *out)
{
    return guarded([&] {
        need(g && out, "null argument");
        use_device(g);
        UseAlloc ua(&g->alloc);
        ensure_tuned(g);
        Staging io(g);
        double *d_out = io.out(out, g->n);
        DBuf<int32_t> all;
        all.ensure((size_t)g->n);
        try {
            launch(g->stream, grid_for(g->n), k_iota, all.p, (int64_t)0, g->n);
            dependencies_impl(g, all.p, g->n, BC_OUT_SUM, d_out, nullptr, nullptr, nullptr, false,
                              nullptr);
            io.finish();
        } catch (...) {
            (void)hipStreamSynchronize(g->stream);
            all.release();
            throw;
        }
        all.release();
    });
}

bc_status bc_dependencies(bc_graph *g, const int32_t *sources, int64_t k, int32_t out_mode,
                          double *out, int32_t *dist_out, double *sigma_mant, int32_t *sigma_exp,
                          const int32_t *targets, int32_t T)
{
    return guarded([&] {
        need(g, "null graph");
        need(k >= 0, "k must be >= 0");
        need(out_mode == BC_OUT_FULL || out_mode == BC_OUT_SUM || out_mode == BC_OUT_TARGETS,
             "unknown out_mode");
        need(out_mode == BC_OUT_FULL || (!dist_out && !sigma_mant && !sigma_exp),
             "per-source outputs need BC_OUT_FULL");
        need(out_mode != BC_OUT_TARGETS || (T >= 0 && (T == 0 || targets)),
             "BC_OUT_TARGETS needs T >= 0 targets");
        const int64_t want = out_mode == BC_OUT_SUM ? g->n
                             : out_mode == BC_OUT_FULL ? k * g->n : k * (int64_t)T;
        need(want == 0 || out, "null argument");
        need(k == 0 || sources, "null argument");
        use_device(g);
        UseAlloc ua(&g->alloc);
        ensure_tuned(g);
        Staging io(g);
        const int32_t *d_src = io.in(sources, k);
        const int32_t *d_tg = out_mode == BC_OUT_TARGETS ? io.in(targets, T) : nullptr;
        check_indices(g, d_src, k, "source");
        if (out_mode == BC_OUT_TARGETS) check_indices(g, d_tg, T, "target");
        if (per_source_schedule(g) && (sigma_mant || sigma_exp))
            fail(BC_E_UNSUPPORTED, "path-count output is served by the batched schedule");
        double *d_out = io.out(out, want);
        int32_t *d_dist = io.out(dist_out, k * g->n);
        double *d_sm = io.out(sigma_mant, k * g->n);
        int32_t *d_se = io.out(sigma_exp, k * g->n);
        if (out_mode == BC_OUT_TARGETS && (k == 0 || T == 0)) {
            io.finish();
            return;
        }
        dependencies_impl(g, d_src, k, out_mode, d_out, d_dist, d_sm, d_se, false, nullptr, d_tg,
                          T);
        io.finish();
    });
}

bc_status bc_dependencies_noalloc(bc_graph *g, const int32_t *sources, int64_t k,
                                  int32_t out_mode, double *out)
{
    return guarded([&] {
        need(g, "null graph");
        need(k >= 0, "k must be >= 0");
        need(out_mode == BC_OUT_FULL || out_mode == BC_OUT_SUM,
             "out_mode must be BC_OUT_FULL or BC_OUT_SUM");
        need(k == 0 || sources, "null argument");
        need(out || (out_mode == BC_OUT_FULL && k == 0), "null argument");
        if (g->io == BC_IO_HOST)
            fail(BC_E_UNSUPPORTED, "the allocation-free call takes device arrays only");
        if (g->weighted) fail(BC_E_UNSUPPORTED, "the allocation-free call takes unweighted graphs");
        use_device(g);
        // any attempt to allocate in this call is an error
        Alloc none;
        none.forbid = true;
        UseAlloc ua(&none);
        const int64_t n = g->n;
        Plan p;
        p.B = 64;
        p.logW = 0;
        // the wave engine's buffers at one word per vertex, carved from the array
        Work nw;
        Carve c{scratch_on(g->device), (size_t)BC_NOALLOC_SCRATCH_BYTES};
        const size_t N = (size_t)n, blocks = (N >> kLevelShift) + 2;
        const size_t min_rec = (size_t)std::max<int64_t>(4 * n, 1 << 16);
        bool ok = c.take(nw.sig, N * 64) &&
                  (out_mode == BC_OUT_FULL ? c.take(nw.dlt, N * 64) : c.take(nw.vsum, N)) &&
                  c.take(nw.vis, N) && c.take(nw.F0, kFS * N) && c.take(nw.F1, kFS * N) &&
                  c.take(nw.active, 1) && c.take(nw.valid, 1) && c.take(nw.live, 1) &&
                  c.take(nw.srcs, 64) && c.take(nw.dest, 64) && c.take(nw.bcnt, blocks) &&
                  c.take(nw.bpop, blocks);
        // long rows: the level's part tasks (one word per vertex) and their sums
        const size_t hubs = (size_t)std::max(g->hubs_out, g->hubs_in);
        const size_t parts = (size_t)std::max(g->parts_out, g->parts_in);
        if (hubs) ok = ok && c.take(nw.hubs, parts) && c.take(nw.pm, parts * 64);
        // the level record (4 + 8 + 8 bytes per entry) takes what is left; it
        // needs at least 4 entries per vertex
        const size_t rec_bytes = 20, pad = 3 * 256;
        ok = ok && c.left() >= min_rec * rec_bytes + pad;
        if (!ok)
            fail(BC_E_UNSUPPORTED, "graph too large for the allocation-free call (" +
                                       std::to_string(n) + " vertices need more than the " +
                                       std::to_string((size_t)BC_NOALLOC_SCRATCH_BYTES) +
                                       "-byte scratch array)");
        // extended path-count exponents when room remains beside that record
        if (c.left() >= (N + parts) * 64 * 4 + 512 + min_rec * rec_bytes + pad) {
            (void)c.take(nw.sige, N * 64);
            if (hubs) (void)c.take(nw.pe, parts * 64);
        }
        const size_t rec = (c.left() - pad) / rec_bytes;
        (void)(c.take(nw.ridx, rec) && c.take(nw.rmask, rec) && c.take(nw.rseg, rec));
        nw.cap_limit = (int64_t)rec;
        nw.ctl.view(g->own.ctl.p, g->own.ctl.cap);   // the handle's control block
        nw.h_ctl = g->own.h_ctl;
        Work *saved = g->w;
        const bool prof = g->prof_on;
        g->w = &nw;
        g->prof_on = false;
        auto restore = [&] {
            g->w = saved;
            g->prof_on = prof;
        };
        try {
            check_indices(g, sources, k, "source");
            dependencies_impl(g, sources, k, out_mode, out, nullptr, nullptr, nullptr, false,
                              nullptr, nullptr, 0, &p);
        } catch (const RecordLimit &) {
            restore();
            (void)hipStreamSynchronize(g->stream);
            fail(BC_E_UNSUPPORTED, "the level record outgrows the allocation-free scratch array");
        } catch (...) {
            restore();
            (void)hipStreamSynchronize(g->stream);
            throw;
        }
        restore();
    });
}

bc_status bc_pair_dependencies(bc_graph *g, const int32_t *us, const int32_t *vs, int64_t k,
                               double *out)
{
    return guarded([&] {
        need(g, "null graph");
        need(k >= 0, "k must be >= 0");
        need(k == 0 || (us && vs && out), "null argument");
        need(g->n >= 2, "pairs need n >= 2");
        use_device(g);
        UseAlloc ua(&g->alloc);
        ensure_tuned(g);
        Staging io(g);
        const int32_t *d_us = io.in(us, k);
        const int32_t *d_vs = io.in(vs, k);
        check_indices(g, d_us, k, "pair start");
        check_indices(g, d_vs, k, "pair end");
        // u != v is checked on the host (k is small in practice)
        {
            const std::vector<int32_t> hu = io.to_host(us, k), hv = io.to_host(vs, k);
            for (int64_t i = 0; i < k; ++i) need(hu[(size_t)i] != hv[(size_t)i], "pair with u == v");
        }
        double *d_out = io.out(out, k * g->n);
        if (use_bidir(g)) pair_dependencies_bidir(g, d_us, d_vs, k, d_out);
        else {
            dependencies_impl(g, d_us, k, BC_OUT_FULL, d_out, nullptr, nullptr, nullptr, true, d_vs);
            g->stats.pair_search = BC_PAIR_SEARCH_ONE_SIDED;
        }
        io.finish();
    });
}

bc_status bc_adaptive_source(bc_graph *g, const int32_t *targets, int32_t T, double c,
                             uint64_t seed, int64_t k_max, double *out_est, int64_t *out_samples,
                             double *out_S, uint8_t *out_status)
{
    return guarded([&] {
        need(g, "null graph");
        need(T >= 0, "T must be >= 0");
        need(T == 0 || (targets && out_est && out_samples && out_S && out_status),
             "null argument");
        need(c >= 1.0, "c must be >= 1 (and not NaN)");
        need(k_max >= 1, "k_max must be >= 1");
        use_device(g);
        UseAlloc ua(&g->alloc);
        ensure_tuned(g);
        Staging io(g);
        const int32_t *d_tg = io.in(targets, T);
        check_indices(g, d_tg, T, "target");
        if (per_source_schedule(g))
            fail(BC_E_UNSUPPORTED, "samplers run on the batched schedule");
        double *d_est = io.out(out_est, T), *d_S = io.out(out_S, T);
        int64_t *d_k = io.out(out_samples, T);
        uint8_t *d_st = io.out(out_status, T);
        sampler_impl(g, d_tg, T, false, RULE_SOURCE, c, 0.0, seed, k_max, d_est, d_k, d_S, d_st);
        io.finish();
    });
}

bc_status bc_adaptive_pair(bc_graph *g, const int32_t *targets, int32_t T, int32_t rule,
                           double eps, double c, uint64_t seed, int64_t k_max, double *out_est,
                           int64_t *out_samples, double *out_S, uint8_t *out_status)
{
    return guarded([&] {
        need(g, "null graph");
        need(T >= 0, "T must be >= 0");
        need(T == 0 || (targets && out_est && out_samples && out_S && out_status),
             "null argument");
        need(rule == BC_PAIR_ALG1 || rule == BC_PAIR_EPS, "unknown rule");
        if (rule == BC_PAIR_ALG1) need(c >= 1.0, "c must be >= 1 (and not NaN)");
        if (rule == BC_PAIR_EPS) need(eps > 0.0 && eps < 0.5, "eps must be in (0, 1/2)");
        need(k_max >= 1, "k_max must be >= 1");
        need(g->n >= 2, "pairs need n >= 2");
        use_device(g);
        UseAlloc ua(&g->alloc);
        ensure_tuned(g);
        Staging io(g);
        const int32_t *d_tg = io.in(targets, T);
        check_indices(g, d_tg, T, "target");
        if (per_source_schedule(g))
            fail(BC_E_UNSUPPORTED, "samplers run on the batched schedule");
        double *d_est = io.out(out_est, T), *d_S = io.out(out_S, T);
        int64_t *d_k = io.out(out_samples, T);
        uint8_t *d_st = io.out(out_status, T);
        sampler_impl(g, d_tg, T, true, rule == BC_PAIR_EPS ? RULE_PAIR_EPS : RULE_PAIR_ALG1, c, eps,
                     seed, k_max, d_est, d_k, d_S, d_st);
        io.finish();
    });
}

bc_status bc_draw_sources(bc_graph *g, uint64_t seed, int64_t j0, int64_t count, int32_t *out_u)
{
    return guarded([&] {
        need(g, "null graph");
        need(j0 >= 0 && count >= 0, "j0 and count must be >= 0");
        need(count == 0 || out_u, "null argument");
        use_device(g);
        if (count == 0) return;
        UseAlloc ua(&g->alloc);
        Staging io(g);
        int32_t *d_u = io.out(out_u, count);
        launch(g->stream, grid_for(count), k_draw_sources, seed, j0, count, g->n, d_u);
        io.finish();
    });
}

bc_status bc_draw_pairs(bc_graph *g, uint64_t seed, int64_t j0, int64_t count, int32_t *out_u,
                        int32_t *out_v)
{
    return guarded([&] {
        need(g, "null graph");
        need(j0 >= 0 && count >= 0, "j0 and count must be >= 0");
        need(count == 0 || (out_u && out_v), "null argument");
        need(g->n >= 2, "pairs need n >= 2");
        use_device(g);
        if (count == 0) return;
        UseAlloc ua(&g->alloc);
        Staging io(g);
        int32_t *d_u = io.out(out_u, count), *d_v = io.out(out_v, count);
        launch(g->stream, grid_for(count), k_draw_pairs, seed, j0, count, g->n, d_u, d_v);
        io.finish();
    });
}

}  // extern "C"

// ================================================================= serving

namespace {

struct ServerQuery {
    int64_t id = 0;
    bc_query q{};
    double S = 0.0;
    int64_t K = 0;
    double arrival = 0.0;
};

// Device buffers a server holds, per kind, so that the shared workspace can
// be budgeted buffer by buffer: the workspace keeps, for each buffer, the
// largest size any admitted graph needs.
enum WsBuf {
    WB_SIG, WB_DLT, WB_SIGE, WB_VIS, WB_F0, WB_F1, WB_ACTIVE, WB_VALID,
    WB_RIDX, WB_RMASK, WB_RSEG, WB_BCNT, WB_BPOP, WB_SRCS, WB_DEST, WB_LV, WB_PACTIVE,
    WB_SS_D, WB_SS_Q, WB_SS_SIG, WB_SS_DLT, WB_PROBE, WB_OKEY_IN, WB_OKEY_OUT, WB_OIDX,
    WB_OPERM, WB_LANE_ROW, WB_DRAW_SRC, WB_DRAW_DST, WB_SORT_TMP, WB_KEY_TMP, WB_QD,
    WB_SLOTQ, WB_TGT, WB_X, WB_CTL, WB_LOFF, WB_LIVE, WB_HUBS, WB_PM, WB_PE, WB_BI, WB_COUNT
};

struct WsNeed {
    size_t b[WB_COUNT] = {};
    size_t total() const
    {
        size_t t = 0;
        for (size_t x : b) t += x;
        return t;
    }
    WsNeed max_with(const WsNeed &o) const
    {
        WsNeed r;
        for (int i = 0; i < WB_COUNT; ++i) r.b[i] = std::max(b[i], o.b[i]);
        return r;
    }
};

// Slots of the two-sided search a server round may use for its pair samples:
// one per eight slots of the batch, 8 to 512 (each holds ~48 bytes per vertex).
int server_bi_slots(int B)
{
    return std::max(8, std::min(B / 8, 512));
}

// Record entries a server batch of W words on n vertices starts with, and
// the most it may grow to (the budgeted size).
int64_t server_record_entries(int64_t n, int64_t W)
{
    return std::max<int64_t>(4 * n * W, 1 << 16);
}

// Upper bound of the device bytes a server round on graph g at width B
// allocates with engine e, per buffer (engine slabs and bitmaps, level record,
// long rows' part sums, lane-order sort, the one-off depth probe and key
// bitmaps, round arrays).
WsNeed need_for(const bc_graph *g, Engine e, int B)
{
    const int64_t n = g->n;
    WsNeed r;
    const size_t N = (size_t)n, Bs = (size_t)B, W = (size_t)std::max(1, B / 64);
    r.b[WB_SIG] = N * Bs * 8;
    r.b[WB_DLT] = N * Bs * 8;
    r.b[WB_SIGE] = N * Bs * 4;
    r.b[WB_SRCS] = Bs * 4;
    r.b[WB_DEST] = Bs * 4;
    if (e == ENG_PAIR) {
        r.b[WB_LV] = N * Bs * 4;
        r.b[WB_RIDX] = N * Bs * 4;
        r.b[WB_PACTIVE] = Bs;
    } else {
        const size_t cap = (size_t)server_record_entries(n, (int64_t)W);
        r.b[WB_VIS] = N * W * 8;
        r.b[WB_F0] = r.b[WB_F1] = N * W * 8 * kFS;
        r.b[WB_ACTIVE] = r.b[WB_VALID] = r.b[WB_LIVE] = W * 8;
        r.b[WB_HUBS] = (size_t)std::max(g->parts_out, g->parts_in) * W * 8;
        r.b[WB_PM] = (size_t)std::max(g->parts_out, g->parts_in) * Bs * 8;
        r.b[WB_PE] = (size_t)std::max(g->parts_out, g->parts_in) * Bs * 4;
        r.b[WB_RIDX] = cap * 4;
        r.b[WB_RMASK] = r.b[WB_RSEG] = cap * 8;
        r.b[WB_BCNT] = r.b[WB_BPOP] = (((N * W) >> kLevelShift) + 2) * 8;
        r.b[WB_OKEY_IN] = r.b[WB_OKEY_OUT] = Bs * 8;
        r.b[WB_OIDX] = r.b[WB_OPERM] = r.b[WB_LANE_ROW] = Bs * 4;
        r.b[WB_DRAW_SRC] = r.b[WB_DRAW_DST] = Bs * 4;
        r.b[WB_SORT_TMP] = std::max<size_t>(sort_temp_bytes(B), 1);
        r.b[WB_KEY_TMP] = 3 * N + kLandmarks * 4 + 8;
    }
    r.b[WB_SS_D] = r.b[WB_SS_Q] = N * 4;
    r.b[WB_SS_SIG] = r.b[WB_SS_DLT] = N * 8;
    r.b[WB_PROBE] = 4;
    r.b[WB_QD] = Bs * sizeof(QueryDesc);
    r.b[WB_SLOTQ] = r.b[WB_TGT] = Bs * 4;
    r.b[WB_X] = Bs * 8;
    r.b[WB_CTL] = CTL_WORDS * sizeof(unsigned long long);
    if (e == ENG_PAIR) r.b[WB_LOFF] = (N + 2) * 8;
    // pair samples: the two-sided search's stamps, counts, lists, level starts
    r.b[WB_BI] = (size_t)server_bi_slots(B) * bidir_slot_bytes(n);
    return r;
}

// Widest width <= max_batch within the 32-bit index range of engine e:
// pair indices b*n + v (pair engine), (vertex, word) indices n*W (wave).
int widest_width(Engine e, int64_t n, int max_batch)
{
    int B = max_batch;
    if (e == ENG_PAIR)
        while (B > 64 && (int64_t)B * n >= (1ll << 32)) B /= 2;
    else
        while (B > 64 && n * (int64_t)(B / 64) >= (1ll << 32)) B /= 2;
    return B;
}

}  // namespace

// One lane of a server: a stream and the workspace of the rounds it runs.
struct ServerLane {
    hipStream_t stream = nullptr;
    bool own_stream = false;   // created by the server (lanes beyond the first)
    Work work;
    DBuf<QueryDesc> qd;
    DBuf<int32_t> slotq, tgt;
    DBuf<double> X;

    size_t bytes() const
    {
        const Work &w = work;
        return w.sig.bytes() + w.dlt.bytes() + w.sige.bytes() + w.vis.bytes() + w.F0.bytes() +
               w.F1.bytes() + w.active.bytes() +
               w.valid.bytes() + w.vsum.bytes() + w.ridx.bytes() + w.rmask.bytes() +
               w.rseg.bytes() + w.bcnt.bytes() + w.bpop.bytes() + w.ctl.bytes() +
               w.srcs.bytes() + w.dest.bytes() + w.X.bytes() + w.S.bytes() + w.K.bytes() +
               w.st.bytes() + w.lv.bytes() + w.pactive.bytes() + w.loff.bytes() + w.ss_d.bytes() +
               w.ss_q.bytes() + w.ss_sig.bytes() + w.ss_dlt.bytes() + w.probe_src.bytes() +
               w.okey_in.bytes() + w.okey_out.bytes() + w.oidx_in.bytes() + w.operm.bytes() +
               w.lane_row.bytes() + w.draw_src.bytes() + w.draw_dst.bytes() +
               w.sort_tmp.bytes() + w.live.bytes() + w.hubs.bytes() + w.pm.bytes() +
               w.pe.bytes() + w.bst.bytes() + w.bval.bytes() + w.bq.bytes() + w.blo.bytes() +
               qd.bytes() + slotq.bytes() + tgt.bytes() + X.bytes();
    }
    void release()
    {
        if (stream) (void)hipStreamSynchronize(stream);
        work.release();
        qd.release();
        slotq.release();
        tgt.release();
        X.release();
        if (own_stream && stream) (void)hipStreamDestroy(stream);
        stream = nullptr;
    }
};

// What one lane's round produced, merged by the calling thread.
struct LaneOut {
    std::vector<bc_result> done;
    int64_t samples_exec = 0, samples_used = 0, split_rounds = 0;
    std::exception_ptr error;
};

struct bc_server {
    int device = 0;
    Alloc alloc;
    size_t budget = 0;
    size_t resident = 0;               // graphs' CSR and lane-order keys
    int max_batch = 256;
    std::vector<std::unique_ptr<ServerLane>> lanes;   // lane 0: the caller's stream
    WsNeed ws;                         // budgeted workspace of one lane, per buffer
    std::vector<bc_graph *> graphs;
    std::vector<int> width;            // batch width per graph
    std::deque<ServerQuery> queued;    // arrival order
    std::vector<std::vector<ServerQuery>> active;
    std::deque<bc_result> done;
    int64_t next_id = 0, finished = 0, rounds = 0, samples_exec = 0, samples_used = 0;
    int64_t split_rounds = 0;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    // device bytes the lanes' workspaces hold now
    size_t workspace_bytes() const
    {
        size_t t = 0;
        for (const auto &l : lanes) t += l->bytes();
        return t;
    }
    void release()
    {
        for (auto g : graphs) bc_graph_destroy(g);
        graphs.clear();
        for (auto &l : lanes) l->release();
        lanes.clear();
    }
};

namespace {

// Slots [lo, hi) of the round's batch on graph g: draw their samples, run
// them as one batch and gather each slot's value at its query's target into
// X[lo..hi). A batch whose level record would outgrow the budgeted workspace
// runs as two halves (each sample's arithmetic does not depend on its batch
// mates, so the values are the same).
void run_slots(ServerLane &ln, LaneOut &out, bc_graph *g, Engine e, int B, int lo, int hi)
{
    const int cnt = hi - lo;
    const int64_t n = g->n;
    hipStream_t st = ln.stream;
    try {
        bool ext = false;
        if (e == ENG_PAIR) {
            ensure_pairs(g, B, false);
            launch(st, grid_for(cnt), k_serve_draw, (const QueryDesc *)ln.qd.p,
                   (const int32_t *)ln.slotq.p, (int32_t)lo, (int32_t)cnt, n, g->w->srcs.p,
                   g->w->dest.p, ln.tgt.p);
            run_pairs(g, B, cnt, true, &ext, nullptr);
            PairArgs a = make_pair_args(g, B, ext, cnt, true);
            launch(st, grid_for(cnt), k_p_gather_slots, a, (const int32_t *)ln.tgt.p,
                   (int32_t)lo, ln.X.p);
        } else {
            Plan p;
            p.B = B;
            while ((64 << p.logW) < B) ++p.logW;
            ensure_batch(g, p, false, start_cap(g), OUT_DELTA);
            launch(st, grid_for(cnt), k_serve_draw, (const QueryDesc *)ln.qd.p,
                   (const int32_t *)ln.slotq.p, (int32_t)lo, (int32_t)cnt, n, g->w->srcs.p,
                   g->w->dest.p, ln.tgt.p);
            const int32_t *lane_row = order_round(g, cnt, true, B);
            run_batch(g, p, cnt, true, &ext, nullptr, OUT_DELTA);
            BatchArgs a = make_args(g, p, ext, cnt, true, (int64_t)g->w->ridx.cap, OUT_DELTA);
            a.lane_row = lane_row;
            launch(st, grid_for(cnt), k_gather_slots, a, (const int32_t *)ln.tgt.p, (int32_t)lo,
                   ln.X.p);
        }
    } catch (const RecordLimit &) {
        // a single sample reaches at most n (vertex, word) entries, within the
        // 4 n W entries budgeted for any width, so halving always ends
        if (cnt <= 1) fail(BC_E_NOMEM, "level record exceeds the server's budget");
        (void)hipStreamSynchronize(st);
        out.split_rounds += 1;
        const int mid = lo + cnt / 2;
        run_slots(ln, out, g, e, B, lo, mid);
        run_slots(ln, out, g, e, B, mid, hi);
    }
}

// Pair slots [lo, hi) of the round: the two-sided search, each slot's value
// at its query's target into X[lo..hi); on a graph where it cannot serve
// (counts once reached 2^1000, now or before) the slots run one-sided.
void run_pair_slots(ServerLane &ln, LaneOut &out, bc_graph *g, Engine e, int B, int lo, int hi)
{
    const int cnt = hi - lo;
    if (cnt <= 0) return;
    if (use_bidir(g)) {
        g->w->srcs.ensure((size_t)B);
        g->w->dest.ensure((size_t)B);
        launch(ln.stream, grid_for(cnt), k_serve_draw, (const QueryDesc *)ln.qd.p,
               (const int32_t *)ln.slotq.p, (int32_t)lo, (int32_t)cnt, g->n, g->w->srcs.p,
               g->w->dest.p, ln.tgt.p);
        if (run_bidir(g, g->w->srcs.p, g->w->dest.p, cnt, nullptr, 0, 0, ln.X.p + lo, nullptr,
                      ln.tgt.p))
            return;
    }
    run_slots(ln, out, g, e, B, lo, hi);
}

// Admit waiting queries of graph gi in arrival order while slots remain.
void admit(bc_server *sv, int gi)
{
    std::vector<ServerQuery> &act = sv->active[(size_t)gi];
    const int B = sv->width[(size_t)gi];
    for (auto it = sv->queued.begin(); it != sv->queued.end() && (int)act.size() < B;) {
        if (it->q.graph == gi) {
            act.push_back(*it);
            it = sv->queued.erase(it);
        } else {
            ++it;
        }
    }
}

// One round of graph gi's active queries on lane ln: fill the batch's slots,
// run them, apply the stop rules. Touches only graph gi's state and the
// lane's, so rounds of different graphs run on different lanes at once;
// finished queries and counts go to `out` for the calling thread to merge.
void server_round(bc_server *sv, ServerLane &ln, int gi, LaneOut &out)
{
    bc_graph *g = sv->graphs[(size_t)gi];
    std::vector<ServerQuery> &act = sv->active[(size_t)gi];
    const int B = sv->width[(size_t)gi];
    const int A = (int)act.size();
    const int64_t n = g->n;
    std::vector<QueryDesc> hd((size_t)A);
    std::vector<int32_t> hslot;
    hslot.reserve((size_t)B);
    const int base = B / A, extra = B % A;
    // the source queries' slots first, then the pair queries' (two engines)
    int ns = 0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int i = 0; i < A; ++i) {
            const ServerQuery &sq = act[(size_t)i];
            const bool pairq = sq.q.kind == BC_QUERY_PAIR;
            if (pairq != (pass == 1)) continue;
            QueryDesc &d = hd[(size_t)i];
            std::memset(&d, 0, sizeof(d));
            d.seed = sq.q.seed;
            d.j0 = sq.K;
            d.k_max = sq.q.k_max;
            d.threshold = sq.q.c * (double)n;
            d.eps_rhs = ((sq.q.eps * sq.q.eps) * sq.q.eps) * ((double)n * (double)n);
            d.scale = pairq ? (double)n * (double)(n - 1) : (double)n;
            d.S = sq.S;
            d.K = sq.K;
            d.target = sq.q.target;
            d.rule = !pairq                      ? RULE_SOURCE
                     : sq.q.rule == BC_PAIR_EPS ? RULE_PAIR_EPS
                                                : RULE_PAIR_ALG1;
            d.slot0 = (int32_t)hslot.size();
            const int64_t need = sq.q.k_max - sq.K;
            d.nslots = (int32_t)std::min<int64_t>(need, base + (i < extra ? 1 : 0));
            d.status = ST_RUNNING;
            for (int k = 0; k < d.nslots; ++k) hslot.push_back(i);
            if (!pairq) ns = (int)hslot.size();
        }
    }
    const int nb = (int)hslot.size();
    hipStream_t st = ln.stream;
    g->stream = st;
    g->w = &ln.work;
    ln.qd.ensure((size_t)B);
    ln.slotq.ensure((size_t)B);
    ln.tgt.ensure((size_t)B);
    ln.X.ensure((size_t)B);
    HIPX(hipMemcpyAsync(ln.qd.p, hd.data(), hd.size() * sizeof(QueryDesc),
                        hipMemcpyHostToDevice, st));
    HIPX(hipMemcpyAsync(ln.slotq.p, hslot.data(), (size_t)nb * 4, hipMemcpyHostToDevice, st));
    if (ns > 0) run_slots(ln, out, g, engine_for(g), B, 0, ns);
    run_pair_slots(ln, out, g, engine_for(g), B, ns, nb);
    launch(st, grid_for(A), k_stop_queries, ln.qd.p, (int32_t)A, (const double *)ln.X.p);
    HIPX(hipMemcpyAsync(hd.data(), ln.qd.p, hd.size() * sizeof(QueryDesc),
                        hipMemcpyDeviceToHost, st));
    HIPX(hipStreamSynchronize(st));
    const double t = sv->now();
    std::vector<ServerQuery> keep;
    keep.reserve(act.size());
    for (int i = 0; i < A; ++i) {
        ServerQuery sq = act[(size_t)i];
        const QueryDesc &d = hd[(size_t)i];
        out.samples_used += d.K - sq.K;
        sq.S = d.S;
        sq.K = d.K;
        if (d.status == ST_RUNNING) {
            keep.push_back(sq);
            continue;
        }
        bc_result r;
        r.id = sq.id;
        r.graph = gi;
        r.status = d.status;
        r.est = d.est;
        r.samples = d.K;
        r.S = d.S;
        r.arrival_s = sq.arrival;
        r.done_s = t;
        out.done.push_back(r);
    }
    act.swap(keep);
    out.samples_exec += nb;
}

// Graph of the next round: shortest job first at graph granularity (the
// graph whose cheapest unfinished query has the least remaining work bound,
// (k_max - k) samples times the CSR size); every eighth round goes to the
// graph of the oldest unfinished query, so no query starves. Graphs in
// `busy` are skipped; -1 when none has work.
int pick_graph(const bc_server *sv, const std::vector<int> &busy, bool oldest_rule)
{
    const int G = (int)sv->graphs.size();
    auto taken = [&](int g) { return std::find(busy.begin(), busy.end(), g) != busy.end(); };
    int gi = -1;
    if (oldest_rule) {
        double oldest = 0.0;
        for (int i = 0; i < G; ++i) {
            if (taken(i)) continue;
            for (const auto &q : sv->active[(size_t)i])
                if (gi < 0 || q.arrival < oldest) {
                    gi = i;
                    oldest = q.arrival;
                }
        }
        for (const auto &q : sv->queued)
            if (!taken(q.q.graph) && (gi < 0 || q.arrival < oldest)) {
                gi = q.q.graph;
                oldest = q.arrival;
            }
        return gi;
    }
    double best = 0.0;
    auto consider = [&](const ServerQuery &q) {
        if (taken(q.q.graph)) return;
        const double work = (double)(q.q.k_max - q.K) *
                            (double)std::max<int64_t>(sv->graphs[(size_t)q.q.graph]->nnz, 1);
        if (gi < 0 || work < best) {
            gi = q.q.graph;
            best = work;
        }
    };
    for (int i = 0; i < G; ++i)
        for (const auto &q : sv->active[(size_t)i]) consider(q);
    for (const auto &q : sv->queued) consider(q);
    return gi;
}

}  // namespace

extern "C" {

constexpr int kServerLanesMax = 4;

bc_status bc_server_create(size_t hbm_budget_bytes, int32_t max_batch, const bc_allocator *alloc,
                           void *hip_stream, bc_server **out)
{
    return guarded([&] {
        need(out != nullptr, "null argument");
        need(max_batch >= 64 && max_batch <= 4096 && (max_batch & (max_batch - 1)) == 0,
             "max_batch must be a power of two in [64, 4096]");
        need(hbm_budget_bytes > 0, "budget must be positive");
        need(!alloc || (alloc->alloc && alloc->free), "allocator needs both alloc and free");
        bc_server *sv = new bc_server();
        if (alloc) sv->alloc.a = *alloc;
        UseAlloc ua(&sv->alloc);
        try {
            HIPX(hipGetDevice(&sv->device));
            sv->budget = hbm_budget_bytes;
            sv->max_batch = max_batch;
            need(hbm_budget_bytes >= CTL_WORDS * sizeof(unsigned long long), "budget below 128 bytes");
            sv->lanes.push_back(std::make_unique<ServerLane>());
            sv->lanes[0]->stream = (hipStream_t)hip_stream;
            sv->lanes[0]->work.init();
            sv->ws.b[WB_CTL] = sv->lanes[0]->work.ctl.bytes();
        } catch (...) {
            sv->release();
            delete sv;
            throw;
        }
        *out = sv;
    });
}

void bc_server_destroy(bc_server *sv)
{
    if (!sv) return;
    (void)hipSetDevice(sv->device);
    UseAlloc ua(&sv->alloc);
    sv->release();
    delete sv;
}

bc_status bc_server_add_graph(bc_server *sv, const bc_csr *csr, int32_t *graph_id)
{
    return guarded([&] {
        need(sv && csr && graph_id, "null argument");
        HIPX(hipSetDevice(sv->device));
        UseAlloc ua(&sv->alloc);
        need(csr->n >= 1 && csr->n < 0x7fffffffll, "n must be in [1, 2^31 - 1)");
        const int64_t n = csr->n;
        // resident: the CSR (int64 rows, int32 columns), the lane-order key, the
        // long-row table and list (at most nnz / (kHub + 1) such rows) and the
        // handle's own control block
        const int64_t nnz = std::max<int64_t>(csr->nnz, 0);
        const size_t res_bytes = (size_t)(n + 1) * 8 + (size_t)nnz * 4 + (size_t)n * 8 +
                                 (size_t)n * 4 + (size_t)(nnz / (kHub + 1) + 1) * 4 +
                                 CTL_WORDS * sizeof(unsigned long long);
        // every lane may hold the widest need (one workspace per lane)
        const size_t L = sv->lanes.size();
        auto fits = [&](const WsNeed &w) {
            return sv->resident + res_bytes + L * w.total() <= sv->budget;
        };
        // the engine choice runs a depth probe in the shared workspace: it must fit first
        WsNeed probe;
        probe.b[WB_SS_D] = probe.b[WB_SS_Q] = (size_t)n * 4;
        probe.b[WB_SS_SIG] = probe.b[WB_SS_DLT] = (size_t)n * 8;
        probe.b[WB_PROBE] = 4;
        if (!fits(sv->ws.max_with(probe)))
            fail(BC_E_NOMEM, "graph does not fit the server's HBM budget");
        bc_graph *g = nullptr;
        bc_allocator *al = sv->alloc.a.alloc ? &sv->alloc.a : nullptr;
        const bc_status rc = bc_graph_create(csr, al, (void *)sv->lanes[0]->stream, &g);
        if (rc != BC_OK) fail(rc, tl_error);
        g->w = &sv->lanes[0]->work;
        try {
            const Engine e = engine_for(g);
            int B = widest_width(e, n, sv->max_batch);
            while (B > 64 && !fits(sv->ws.max_with(need_for(g, e, B)))) B /= 2;
            const WsNeed ws = sv->ws.max_with(need_for(g, e, B));
            if (!fits(ws))
                fail(BC_E_NOMEM, "no batch width fits the server's HBM budget for this graph");
            sv->ws = ws;
            for (auto &ln : sv->lanes) {
                ln->work.cap_limit = (int64_t)(ws.b[WB_RIDX] / 4);
                ln->work.bi_budget = ws.b[WB_BI];
            }
            sv->graphs.push_back(g);
            sv->width.push_back(B);
            sv->active.emplace_back();
            sv->resident += res_bytes;
        } catch (...) {
            g->w = &g->own;
            bc_graph_destroy(g);
            throw;
        }
        *graph_id = (int32_t)sv->graphs.size() - 1;
    });
}

bc_status bc_server_submit(bc_server *sv, const bc_query *q, int64_t *id)
{
    return guarded([&] {
        need(sv && q && id, "null argument");
        need(q->graph >= 0 && q->graph < (int32_t)sv->graphs.size(), "unknown graph id");
        const bc_graph *g = sv->graphs[(size_t)q->graph];
        need(q->target >= 0 && q->target < g->n, "target outside [0, n)");
        need(q->kind == BC_QUERY_SOURCE || q->kind == BC_QUERY_PAIR, "unknown query kind");
        need(q->k_max >= 1, "k_max must be >= 1");
        if (q->kind == BC_QUERY_SOURCE) {
            need(q->c >= 1.0, "c must be >= 1 (and not NaN)");
        } else {
            need(g->n >= 2, "pairs need n >= 2");
            need(q->rule == BC_PAIR_ALG1 || q->rule == BC_PAIR_EPS, "unknown rule");
            if (q->rule == BC_PAIR_ALG1) need(q->c >= 1.0, "c must be >= 1 (and not NaN)");
            else need(q->eps > 0.0 && q->eps < 0.5, "eps must be in (0, 1/2)");
        }
        ServerQuery sq;
        sq.id = sv->next_id++;
        sq.q = *q;
        sq.arrival = q->arrival_s >= 0.0 ? q->arrival_s : sv->now();
        sv->queued.push_back(sq);
        *id = sq.id;
    });
}

bc_status bc_server_step(bc_server *sv, int32_t *completed)
{
    return guarded([&] {
        need(sv && completed, "null argument");
        HIPX(hipSetDevice(sv->device));
        UseAlloc ua(&sv->alloc);
        *completed = 0;
        // one graph per lane, picked in turn by the scheduling rule
        std::vector<int> pick;
        for (size_t k = 0; k < sv->lanes.size(); ++k) {
            const int gi = pick_graph(sv, pick, k == 0 && sv->rounds % 8 == 7);
            if (gi < 0) break;
            pick.push_back(gi);
            admit(sv, gi);
        }
        if (pick.empty()) return;
        const size_t R = pick.size();
        std::vector<LaneOut> out(R);
        auto run = [&](size_t k) {
            try {
                HIPX(hipSetDevice(sv->device));
                UseAlloc lane_alloc(&sv->alloc);
                tl_sync = R > 1 ? sv->lanes[k]->stream : nullptr;
                server_round(sv, *sv->lanes[k], pick[k], out[k]);
            } catch (...) {
                out[k].error = std::current_exception();
                (void)hipStreamSynchronize(sv->lanes[k]->stream);
            }
            tl_sync = nullptr;
        };
        std::vector<std::thread> th;
        for (size_t k = 1; k < R; ++k) th.emplace_back(run, k);
        run(0);
        for (auto &t : th) t.join();
        for (size_t k = 0; k < R; ++k)
            if (out[k].error) std::rethrow_exception(out[k].error);
        // results in lane order
        for (size_t k = 0; k < R; ++k) {
            for (const bc_result &r : out[k].done) sv->done.push_back(r);
            sv->finished += (int64_t)out[k].done.size();
            *completed += (int32_t)out[k].done.size();
            sv->samples_exec += out[k].samples_exec;
            sv->samples_used += out[k].samples_used;
            sv->split_rounds += out[k].split_rounds;
            sv->rounds += 1;
        }
    });
}

bc_status bc_server_set_lanes(bc_server *sv, int32_t lanes)
{
    return guarded([&] {
        need(sv, "null argument");
        need(lanes >= 1 && lanes <= kServerLanesMax, "lanes must be in [1, 4]");
        HIPX(hipSetDevice(sv->device));
        UseAlloc ua(&sv->alloc);
        need(sv->resident + (size_t)lanes * sv->ws.total() <= sv->budget,
             "the lanes' workspaces do not fit the server's HBM budget");
        while ((int)sv->lanes.size() > lanes) {
            sv->lanes.back()->release();
            sv->lanes.pop_back();
        }
        while ((int)sv->lanes.size() < lanes) {
            auto ln = std::make_unique<ServerLane>();
            HIPX(hipStreamCreateWithFlags(&ln->stream, hipStreamNonBlocking));
            ln->own_stream = true;
            try {
                ln->work.init();
                ln->work.cap_limit = sv->lanes[0]->work.cap_limit;
                ln->work.bi_budget = sv->lanes[0]->work.bi_budget;
            } catch (...) {
                ln->release();
                throw;
            }
            sv->lanes.push_back(std::move(ln));
        }
    });
}

bc_status bc_server_poll(bc_server *sv, bc_result *out, int32_t max, int32_t *count)
{
    return guarded([&] {
        need(sv && count && (max <= 0 || out), "null argument");
        int32_t c = 0;
        while (c < max && !sv->done.empty()) {
            out[c++] = sv->done.front();
            sv->done.pop_front();
        }
        *count = c;
    });
}

bc_status bc_server_now(const bc_server *sv, double *now_s)
{
    return guarded([&] {
        need(sv && now_s, "null argument");
        *now_s = sv->now();
    });
}

bc_status bc_server_stats_get(const bc_server *sv, bc_server_stats *out)
{
    return guarded([&] {
        need(sv && out, "null argument");
        int64_t act = 0;
        for (const auto &a : sv->active) act += (int64_t)a.size();
        out->queued = (int64_t)sv->queued.size();
        out->active = act;
        out->finished = sv->finished;
        out->rounds = sv->rounds;
        out->samples_executed = sv->samples_exec;
        out->samples_used = sv->samples_used;
        out->resident_bytes = (int64_t)sv->resident;
        out->workspace_bytes = (int64_t)sv->workspace_bytes();
        out->budget_bytes = (int64_t)sv->budget;
        out->split_rounds = sv->split_rounds;
    });
}

bc_status bc_server_graph_width(const bc_server *sv, int32_t graph, int32_t *width,
                                int32_t *schedule)
{
    return guarded([&] {
        need(sv && (width || schedule), "null argument");
        need(graph >= 0 && graph < (int32_t)sv->graphs.size(), "unknown graph id");
        if (width) *width = sv->width[(size_t)graph];
        if (schedule)
            *schedule = sv->graphs[(size_t)graph]->engine == ENG_PAIR ? BC_SCHED_THREADED
                                                                     : BC_SCHED_BATCHED;
    });
}

}  // extern "C"
