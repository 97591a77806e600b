// Device kernels for Brandes' pass on an unweighted CSR graph, batched over
// many sources, plus the per-source plain form, the sample draws and the
// adaptive stopping rules.
//
// Wave engine layout (a batch of B = 64 * W sources, W = 2^logW words):
//   vis[v*W + j]  bit l set once source b = 64j + l has reached v.
//   F*[v*W + j]   dense frontier bitmap of one level (two rotating arrays);
//   SG*[v*W + j]  beside it, the first pool slot of that (v, j) entry.
//   Level record: entries (v, j) with a nonzero 64-bit mask m, level after
//   level, in (v, j) order within a level (laid out by a prefix sum over the
//   level's dense words); level l occupies [off[l], off[l+1]). It replaces
//   Brandes' distance-ordered stack: the backward sweep walks it from the
//   deepest level.
//   Value pool: entry e owns popcount(m_e) consecutive FP64 slots starting at
//   rseg[e]; lane l of the entry's word (source 64j + l, bit l of m_e) lives at
//   rseg[e] + (number of bits of m_e below l). It holds sigma_{s_b}(v), replaced
//   in place by rho = (1 + delta)/sigma (pair mode: ([v = dest_b] + delta')/sigma)
//   when the backward sweep reaches v's level, the only quantity a predecessor
//   needs from v (Theorem 1). A level's values are one dense region, and the
//   lanes a reader needs from one owner are consecutive slots.
//   dlt[v*B + b]  FP64 dependency, written only for per-source outputs.
// One wavefront works on one entry: its 64 lanes are the 64 sources of word j.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace bcmi {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kInFlight = 8;   // overlapping neighbours whose value loads are issued together

// control words shared with the host (one 64-byte block)
enum : int {
    CTL_TAIL = 0,         // level-record tail
    CTL_REC_OVERFLOW = 1,
    CTL_SIG_OVERFLOW = 2, // some path count reached 2^1000 in plain FP64
    CTL_RUNNING = 3,      // targets still sampling
    CTL_POOL = 4,         // value-pool tail
    CTL_LEVELS = 5,       // levels of a pass run by a persistent loop
    CTL_WTASKS = 6,       // tasks of a weighted search round
    CTL_HUBS = 7,         // long-row entries of a level (k_hub_find)
    CTL_BAR = 8,          // grid barrier of the persistent loops: arrivals,
                          // generation, failure flag (CTL_BAR .. CTL_BAR + 2)
    CTL_WORDS = 16
};

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return (uint64_t)__ballot(p); }

__device__ __forceinline__ int32_t lane_read_i32(int32_t x, int l)
{
    return __builtin_amdgcn_readlane(x, l);
}

__device__ __forceinline__ uint64_t lane_read_u64(uint64_t x, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// the value of x in the first active lane, as a wave-uniform (scalar) value
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// true in the lanes whose bit is set in the wave-uniform mask m
__device__ __forceinline__ bool lane_in(uint64_t m)
{
    return __builtin_amdgcn_inverse_ballot_w64(m);
}

// number of set bits of bal below this lane
__device__ __forceinline__ int rank_below(uint64_t bal)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
}

// number of set bits of m below this lane: the lane's slot in its owner's segment
__device__ __forceinline__ uint32_t slot_rank(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Wave-aggregated append: one atomic per wavefront, slots by ballot rank.
// Every lane of the wavefront must reach this call.
__device__ __forceinline__ int64_t wave_append(bool want, unsigned long long *tail)
{
    const uint64_t bal = wave_ballot(want);
    if (bal == 0) return -1;
    const int leader = __ffsll((long long)bal) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader) base = atomicAdd(tail, (unsigned long long)__popcll(bal));
    base = lane_read_u64(base, leader);
    return want ? (int64_t)base + rank_below(bal) : -1;
}

// A (vertex, word) of a level is one 16-byte record in the frontier arrays:
// its lane mask, then its pool segment. Kernels take the two as pointers F
// and SG = F + 1 into the same array and index both by kFS * (vertex, word),
// so a pull finds a neighbour's mask and segment on one line.
constexpr int64_t kFS = 2;

struct BatchArgs {
    const int64_t *row;   // out-neighbours (the search, Theorem 1's successors)
    const int32_t *col;
    const int64_t *rrow;  // in-neighbours (Definition 3's predecessors); the same
    const int32_t *rcol;  // arrays as row/col for an undirected graph
    int64_t n;
    int32_t logW;        // words per batch = 1 << logW
    int32_t B;           // sources per batch = 64 << logW
    double *sig;         // value pool: sigma, then rho, per entry segment
    int32_t *sige;       // pool exponents (extended mode), else null
    double *dlt;
    uint64_t *vis;
    uint32_t *ridx;
    uint64_t *rmask;
    uint64_t *rseg;      // first pool slot of each record entry
    int64_t cap;
    unsigned long long *ctl;
    uint64_t *active;    // [W] sources still expanding (pair mode clears finished slots)
    const uint64_t *valid;  // [W] lanes holding a real source
    uint64_t *live;      // [W] lanes present in the newest level (its masks OR-ed)
    const int32_t *hpart;   // [n] first part of each row longer than kHub (row/col), -1 else
    const int32_t *rhpart;  // the same for rrow/rcol
    double *pm;          // [part][B] part sums of the level's long rows
    int32_t *pe;         // their exponents (extended mode), else null
    const int32_t *srcs; // [B] source (pair: u)
    const int32_t *dest; // [B] pair destination v, or null in source mode
    double *vsum;        // [n][W] per-(vertex, word) dependency sums, or null
    unsigned long long *prof;  // work-unit counters [kernel][2], or null
    const int32_t *lane_row;   // [B] caller's row of each lane, or null (row b0 + lane)
    int32_t nvalid;
};

// output row of lane b in a batch whose first sample is b0
__device__ __forceinline__ int64_t out_row(const BatchArgs &a, int64_t b0, int b)
{
    return a.lane_row ? (int64_t)a.lane_row[b] : b0 + b;
}

// kernel ids of the work-unit counters
enum : int {
    PROF_TOPDOWN = 0,
    PROF_BOTTOMUP = 1,
    PROF_SIGMA = 2,
    PROF_BACKWARD = 3,
    PROF_LEVEL = 4,   // record layout of a level (k_level_*), counted on the host
    PROF_HUB_PARTS = 5,  // part sums of rows longer than kHub (both pulls)
    PROF_PAIR_FWD = 6,   // pair engine's persistent forward loop (discovery + path counts)
    PROF_PAIR_BWD = 7,   // pair engine's persistent backward loop
    PROF_BIDIR = 8,      // two-sided pair search
    PROF_W_SEARCH = 9,   // weighted graphs: search rounds
    PROF_W_COUNTS = 10,  //   path-count rounds
    PROF_W_BACKWARD = 11,  // dependency rounds
    PROF_WG = 12,        // one workgroup per source
    PROF_KERNELS = 13
};

__device__ __forceinline__ unsigned long long wave_or_u64(unsigned long long x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x |= __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Work-unit counters: prof[(2 * kernel + c) * kProfSlots + slot], c = 0 for
// units a, 1 for units b. A workgroup adds into slot blockIdx % kProfSlots,
// so the counters' atomics spread over kProfSlots addresses (one address
// would serialise every wavefront's add); the host sums the slots.
constexpr int kProfSlots = 64;

__device__ __forceinline__ unsigned long long *prof_slot(unsigned long long *prof, int kernel,
                                                         int c)
{
    return prof + (2 * kernel + c) * kProfSlots + (blockIdx.x & (kProfSlots - 1));
}

// add wave-summed unit counts (lane 0 of each wave adds)
__device__ __forceinline__ void prof_add_raw(unsigned long long *prof, int kernel,
                                             unsigned long long ua, unsigned long long ub)
{
    if ((threadIdx.x & 63) == 0) {
        if (ua) atomicAdd(prof_slot(prof, kernel, 0), ua);
        if (ub) atomicAdd(prof_slot(prof, kernel, 1), ub);
    }
}

// add per-wave unit counts to the profile counters (one atomic pair per wave)
__device__ __forceinline__ void prof_add(const BatchArgs &a, int kernel, unsigned long long ua,
                                         unsigned long long ub, int lane)
{
    if (!a.prof) return;
    if (lane == 0) {
        if (ua) atomicAdd(prof_slot(a.prof, kernel, 0), ua);
        if (ub) atomicAdd(prof_slot(a.prof, kernel, 1), ub);
    }
}

__device__ __forceinline__ void record_push(const BatchArgs &a, int64_t pos, uint32_t idx)
{
    if (pos < a.cap) a.ridx[pos] = idx;
    else a.ctl[CTL_REC_OVERFLOW] = 1ull;
}

// ------------------------------------------------------------ extended FP64
// value = m * 2^e with m normalised into [1, 2) once it leaves the plain range.
struct XNum {
    double m;
    int32_t e;
};

__device__ __forceinline__ XNum xnorm(double m, int32_t e)
{
    XNum r{m, e};
    if (m == 0.0) { r.e = 0; return r; }
    const uint64_t bits = __double_as_longlong(m);
    const int32_t ex = (int32_t)((bits >> 52) & 0x7ff) - 1023;
    if (ex == 0) return r;
    r.m = __longlong_as_double((long long)((bits & ~(0x7ffull << 52)) | (1023ull << 52)));
    r.e = e + ex;
    return r;
}

// Fields are selected one by one: a select of the whole struct (or a return
// of one of several structs) is lowered through a stack slot.
__device__ __forceinline__ XNum xadd(XNum a, XNum b)
{
    const int32_t e = a.e > b.e ? a.e : b.e;
    const XNum s = xnorm(ldexp(a.m, a.e - e) + ldexp(b.m, b.e - e), e);
    const bool az = a.m == 0.0, bz = b.m == 0.0;
    XNum r;
    r.m = az ? b.m : (bz ? a.m : s.m);
    r.e = az ? b.e : (bz ? a.e : s.e);
    return r;
}

// ------------------------------------------------------------------ level 0

__global__ void k_init_sources(BatchArgs a, uint64_t *F0)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    bool want = false;
    uint32_t idx = 0;
    if (b < a.nvalid) {
        const int32_t s = a.srcs[b];
        const int j = b >> 6;
        const uint64_t bit = 1ull << (b & 63);
        const int64_t o = (int64_t)s * a.B + b;
        if (a.dlt) a.dlt[o] = 0.0;
        idx = ((uint32_t)s << a.logW) + (uint32_t)j;
        const uint64_t old = atomicOr((unsigned long long *)&F0[kFS * idx],
                                      (unsigned long long)bit);
        atomicOr((unsigned long long *)&a.vis[idx], (unsigned long long)bit);
        want = (old == 0);
    }
    const int64_t pos = wave_append(want, &a.ctl[CTL_TAIL]);
    if (want) record_push(a, pos, idx);
}

// Level 0: each source entry's final mask, its pool segment and sigma = 1.
__global__ void k_init_level0(BatchArgs a, int64_t e0, int64_t e1, const uint64_t *F0,
                              uint64_t *SG0)
{
    for (int64_t e = e0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < e1;
         e += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t idx = a.ridx[e];
        const uint64_t m = F0[kFS * idx];
        const int c = __popcll(m);
        const uint64_t seg = atomicAdd(&a.ctl[CTL_POOL], (unsigned long long)c);
        for (int r = 0; r < c; ++r) {
            a.sig[seg + r] = 1.0;
            if (a.sige) a.sige[seg + r] = 0;
        }
        a.rmask[e] = m;
        a.rseg[e] = seg;
        SG0[kFS * idx] = seg;
    }
}

__global__ void k_clear(BatchArgs a, int64_t e0, int64_t e1, uint64_t *F)
{
    for (int64_t e = e0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < e1;
         e += (int64_t)gridDim.x * blockDim.x)
        F[kFS * a.ridx[e]] = 0;
}

// ---------------------------------------------------------- forward: discover

// Top-down: each frontier entry (u, j) offers its mask to every neighbour w;
// bits not yet visited are OR-ed into w's next-level word (the level's record
// is built from the words afterwards, by k_level_*).
__global__ void k_discover_topdown(BatchArgs a, int64_t e0, int64_t e1, uint64_t *nxt)
{
    const int lane = lane_id();
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const uint32_t wmask = (1u << a.logW) - 1u;
    unsigned long long found = 0;
    for (int64_t e = e0 + wave; e < e1; e += nwaves) {
        const uint32_t idx = a.ridx[e];
        const int64_t u = idx >> a.logW;
        const uint32_t j = idx & wmask;
        const uint64_t m = a.rmask[e] & a.active[j];
        if (m == 0) continue;
        const int64_t beg = a.row[u], end = a.row[u + 1];
        for (int64_t p = beg + lane; p < end; p += kWave) {
            const uint32_t widx = ((uint32_t)a.col[p] << a.logW) + j;
            const uint64_t fresh = m & ~a.vis[widx];
            if (fresh) {
                const uint64_t old = atomicOr((unsigned long long *)&nxt[kFS * widx],
                                              (unsigned long long)fresh);
                found += __popcll(fresh & ~old);
            }
        }
    }
    if (a.prof) prof_add(a, PROF_TOPDOWN, wave_sum_u64(found), 0, lane);
}

// Bottom-up: every (w, j) with unvisited live sources looks for frontier
// neighbours and stops early once all its unvisited sources are found
// (membership only: the path counts are pulled afterwards from all parents;
// the level's record is built from the words by k_level_*).
__global__ void k_discover_bottomup(BatchArgs a_in, const uint64_t *cur, uint64_t *nxt)
{
    // a vertex looks for frontier predecessors: its in-neighbours
    BatchArgs a = a_in;
    a.row = a_in.rrow;
    a.col = a_in.rcol;
    const int64_t total = a.n << a.logW;
    const uint32_t wmask = (1u << a.logW) - 1u;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long found = 0;
    for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x; i0 < total; i0 += stride) {
        const int64_t idx = i0 + threadIdx.x;
        if (idx < total) {
            const uint32_t j = (uint32_t)idx & wmask;
            // a lane absent from the current level finds nothing (its search
            // has ended, e.g. a source outside this vertex's component)
            const uint64_t want = ~a.vis[idx] & a.valid[j] & a.active[j] & a.live[j];
            const int64_t v = idx >> a.logW;
            // rows longer than kHub take a wavefront each (k_discover_bottomup_long)
            if (want && a.rhpart[v] < 0) {
                uint64_t acc = 0;
                const int64_t beg = a.row[v], end = a.row[v + 1];
                // eight neighbours per step; the next step's neighbour ids are
                // loaded while this step's frontier words are in flight
                int32_t c[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) c[k] = beg + k < end ? a.col[beg + k] : -1;
                for (int64_t e = beg; e < end; e += 8) {
                    uint64_t f[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        f[k] = c[k] >= 0 ? cur[kFS * (((int64_t)c[k] << a.logW) + j)] : 0ull;
#pragma unroll
                    for (int k = 0; k < 8; ++k) c[k] = e + 8 + k < end ? a.col[e + 8 + k] : -1;
#pragma unroll
                    for (int k = 0; k < 8; ++k) acc |= f[k];
                    if ((acc & want) == want) break;
                }
                const uint64_t fresh = acc & want;
                if (fresh) {
                    nxt[kFS * idx] = fresh;
                    found += __popcll(fresh);
                }
            }
        }
    }
    if (a.prof) prof_add(a, PROF_BOTTOMUP, wave_sum_u64(found), 0, lane_id());
}

// Bottom-up for the in-rows longer than kHub: one wavefront per (vertex, word)
// of the `nlong` listed vertices, 256 neighbours a step (four per lane, their
// frontier words ORed over the wavefront), stopping once every wanted source
// is found. A thread alone would walk such a row serially while the rest of
// its wavefront waits.
__global__ void k_discover_bottomup_long(BatchArgs a, const uint64_t *cur, uint64_t *nxt,
                                         const int32_t *longv, int64_t nlong)
{
    const int lane = lane_id();
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const uint32_t wmask = (1u << a.logW) - 1u;
    unsigned long long found = 0;
    for (int64_t t = wave; t < (nlong << a.logW); t += nwaves) {
        const int64_t v = longv[t >> a.logW];
        const uint32_t j = (uint32_t)t & wmask;
        const int64_t idx = (v << a.logW) + j;
        const uint64_t want = ~a.vis[idx] & a.valid[j] & a.active[j] & a.live[j];
        if (want == 0) continue;
        const int64_t beg = a.rrow[v], end = a.rrow[v + 1];
        unsigned long long acc = 0;
        for (int64_t p0 = beg; p0 < end; p0 += 4 * kWave) {
            int32_t c[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t p = p0 + k * kWave + lane;
                c[k] = p < end ? a.rcol[p] : -1;
            }
            unsigned long long f = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                f |= c[k] >= 0 ? cur[kFS * (((int64_t)c[k] << a.logW) + j)] : 0ull;
            acc |= wave_or_u64(f);
            if ((acc & want) == want) break;
        }
        const uint64_t fresh = acc & want;
        if (fresh && lane == 0) {
            nxt[kFS * idx] = fresh;
            found += __popcll(fresh);
        }
    }
    if (a.prof) prof_add(a, PROF_BOTTOMUP, wave_sum_u64(found), 0, lane);
}

// ------------------------------------------------------- level record
//
// After discovery the new level exists only as dense words nxt[v][j]. The
// record entries (one per non-zero word, in (vertex, word) order) and their
// pool segments (popcount(word) consecutive slots each, same order) are laid
// out by a prefix sum: k_level_count totals blocks of 2^kLevelShift words,
// k_level_scan turns the totals into block offsets from the record and pool
// tails, and k_level_write emits the entries. No contended counter is used.
constexpr int kLevelShift = 10;   // 256 threads x 4 words

// scan of (entries, slots) over the block's threads; returns this thread's
// exclusive offsets and leaves the block totals in tot_e / tot_s
__device__ __forceinline__ void block_scan2(int ce, int cs, int &pe, int &ps, int &tot_e,
                                            int &tot_s)
{
    __shared__ int we[4], ws[4];
    const int lane = lane_id();
    const int wv = threadIdx.x >> 6;
    int ie = ce, is = cs;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int ye = __shfl_up(ie, off, 64);
        const int ys = __shfl_up(is, off, 64);
        if (lane >= off) {
            ie += ye;
            is += ys;
        }
    }
    if (lane == 63) {
        we[wv] = ie;
        ws[wv] = is;
    }
    __syncthreads();
    pe = ie - ce;
    ps = is - cs;
    tot_e = 0;
    tot_s = 0;
    for (int w = 0; w < 4; ++w) {
        if (w < wv) {
            pe += we[w];
            ps += ws[w];
        }
        tot_e += we[w];
        tot_s += ws[w];
    }
}

__global__ __launch_bounds__(256) void k_level_count(const uint64_t *nxt, int64_t total,
                                                     unsigned long long *bcnt,
                                                     unsigned long long *bpop)
{
    const int64_t base = ((int64_t)blockIdx.x << kLevelShift) + (int64_t)threadIdx.x * 4;
    int ce = 0, cs = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint64_t m = base + r < total ? nxt[kFS * (base + r)] : 0ull;
        ce += m != 0;
        cs += __popcll(m);
    }
    int pe, ps, te, ts;
    block_scan2(ce, cs, pe, ps, te, ts);
    if (threadIdx.x == 0) {
        bcnt[blockIdx.x] = (unsigned long long)te;
        bpop[blockIdx.x] = (unsigned long long)ts;
    }
}

// One workgroup of 1024 threads: exclusive scan of the block totals from the
// record tail (ctl[CTL_TAIL]) and the pool tail (ctl[CTL_POOL]); both tails
// advance past the level, and a record beyond `cap` raises the overflow flag.
// The level's live lanes start empty (k_level_write fills them).
__global__ __launch_bounds__(1024) void k_level_scan(unsigned long long *bcnt,
                                                     unsigned long long *bpop, int64_t nb,
                                                     unsigned long long *ctl, int64_t cap,
                                                     uint64_t *live, int32_t W)
{
    __shared__ unsigned long long we[16], ws[16];
    const int tid = threadIdx.x;
    for (int j = tid; j < W; j += 1024) live[j] = 0ull;
    const int lane = lane_id();
    const int wv = tid >> 6;
    unsigned long long ce = ctl[CTL_TAIL], cs = ctl[CTL_POOL];
    for (int64_t i0 = 0; i0 < nb; i0 += 1024) {
        const int64_t i = i0 + tid;
        const unsigned long long xe = i < nb ? bcnt[i] : 0ull;
        const unsigned long long xs = i < nb ? bpop[i] : 0ull;
        unsigned long long ie = xe, is = xs;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned long long ye = __shfl_up(ie, off, 64);
            const unsigned long long ys = __shfl_up(is, off, 64);
            if (lane >= off) {
                ie += ye;
                is += ys;
            }
        }
        if (lane == 63) {
            we[wv] = ie;
            ws[wv] = is;
        }
        __syncthreads();
        unsigned long long be = 0, bs = 0, te = 0, ts = 0;
        for (int w = 0; w < 16; ++w) {
            if (w < wv) {
                be += we[w];
                bs += ws[w];
            }
            te += we[w];
            ts += ws[w];
        }
        if (i < nb) {
            bcnt[i] = ce + be + ie - xe;
            bpop[i] = cs + bs + is - xs;
        }
        ce += te;
        cs += ts;
        __syncthreads();
    }
    if (tid == 0) {
        ctl[CTL_TAIL] = ce;
        ctl[CTL_POOL] = cs;
        if (ce > (unsigned long long)cap) ctl[CTL_REC_OVERFLOW] = 1ull;
    }
}

// Entries of the level in (vertex, word) order with their masks and pool
// segments; the words join the visited set, and their lanes the level's live
// lanes (OR-ed per workgroup in LDS, then into a.live only with new bits).
__global__ __launch_bounds__(256) void k_level_write(BatchArgs a, const uint64_t *nxt,
                                                     const unsigned long long *bcnt,
                                                     const unsigned long long *bpop)
{
    __shared__ unsigned long long lw[64];
    const int W = 1 << a.logW;
    if ((int)threadIdx.x < W) lw[threadIdx.x] = 0ull;
    const int64_t total = a.n << a.logW;
    const int64_t base = ((int64_t)blockIdx.x << kLevelShift) + (int64_t)threadIdx.x * 4;
    uint64_t m[4];
    int ce = 0, cs = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        m[r] = base + r < total ? nxt[kFS * (base + r)] : 0ull;
        ce += m[r] != 0;
        cs += __popcll(m[r]);
    }
    int pe, ps, te, ts;
    block_scan2(ce, cs, pe, ps, te, ts);
    uint64_t pos = bcnt[blockIdx.x] + (uint64_t)pe;
    uint64_t seg = bpop[blockIdx.x] + (uint64_t)ps;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (m[r]) {
            const int64_t idx = base + r;
            if ((int64_t)pos < a.cap) {
                a.ridx[pos] = (uint32_t)idx;
                a.rmask[pos] = m[r];
                a.rseg[pos] = seg;
            }
            a.vis[idx] |= m[r];
            pos += 1;
            seg += (uint64_t)__popcll(m[r]);
        }
    }
    // block_scan2's barriers order the LDS clear before these ORs
    const uint32_t wmask = (uint32_t)W - 1u;
    uint64_t own = 0;
    int jo = -1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (!m[r]) continue;
        const int j = (int)((uint64_t)(base + r) & wmask);
        if (j == jo) {
            own |= m[r];
        } else {
            if (own) atomicOr(&lw[jo], (unsigned long long)own);
            own = m[r];
            jo = j;
        }
    }
    if (own) atomicOr(&lw[jo], (unsigned long long)own);
    __syncthreads();
    if ((int)threadIdx.x < W) {
        const uint64_t x = lw[threadIdx.x];
        if (x & ~a.live[threadIdx.x])
            atomicOr((unsigned long long *)&a.live[threadIdx.x], (unsigned long long)x);
    }
}

// ------------------------------------------------- neighbour pull (shared)

// Rows longer than kHub are never staged in LDS: they are summed in parts over
// the whole device before the pull (k_hub_parts).
constexpr int kHub = 256;

// Issue the value loads of up to kIF overlapping neighbours, taken from
// bal (bit k: the neighbour staged in lane k, whose frontier word and pool
// segment are this lane's fm and sx) in ascending order. fk[q] receives the
// q-th neighbour's overlap with the wave-uniform `want` (0 for an unused
// slot). Every lane loads, so the loads are straight-line code and all of a
// batch is in flight together: lanes outside the overlap read the first
// overlapping lane's slot (always valid) and add_batch discards it.
template <bool kExt, int kIF = kInFlight>
__device__ __forceinline__ void issue_batch(const BatchArgs &a, uint64_t fm, uint64_t sx,
                                            uint64_t want, uint64_t &bal, double (&vm)[kIF],
                                            int32_t (&ve)[kIF], uint64_t (&fk)[kIF],
                                            unsigned long long &units)
{
#pragma unroll
    for (int q = 0; q < kIF; ++q) {
        fk[q] = 0;
        vm[q] = 0.0;
        ve[q] = 0;
        if (bal) {
            const int k = __ffsll((long long)bal) - 1;
            bal &= bal - 1;
            const uint64_t mk = lane_read_u64(fm, k);
            const uint64_t sk = lane_read_u64(sx, k);
            fk[q] = mk & want;
            units += __popcll(fk[q]);
            // lanes outside the overlap read the first overlapping lane's slot,
            // a line the overlap needs anyway (the segment's first slot may sit
            // in a line no overlapping lane uses)
            const uint64_t low = fk[q] & (~fk[q] + 1ull);
            const uint32_t first = (uint32_t)__popcll(mk & (low - 1ull));
            const uint64_t o = sk + (lane_in(fk[q]) ? slot_rank(mk) : first);
            vm[q] = a.sig[o];
            if (kExt) ve[q] = a.sige[o];
        }
    }
}

// Add a batch in issue order; lanes outside a neighbour's overlap add nothing.
// In plain FP64 every slot is consumed by every lane without a branch, so no
// load of a batch can be pending when its register is reused by the next one
// (the compiler would otherwise wait for all memory operations first).
template <bool kExt, int kIF = kInFlight>
__device__ __forceinline__ void add_batch(const double (&vm)[kIF], const int32_t (&ve)[kIF],
                                          const uint64_t (&fk)[kIF], double &accp, XNum &accx)
{
#pragma unroll
    for (int q = 0; q < kIF; ++q) {
        const bool on = lane_in(fk[q]);
        if (kExt) {
            if (fk[q]) {
                const XNum y = xadd(accx, XNum{vm[q], ve[q]});
                accx.m = on ? y.m : accx.m;
                accx.e = on ? y.e : accx.e;
            }
        } else {
            accp += on ? vm[q] : 0.0;
        }
    }
}

// Sum, over the neighbours x at row positions [beg, end), in ascending CSR
// order, whose frontier word F[x][j] shares a bit with `want`, of the slab
// value slab[x][64j + lane] for the lanes whose bit is set in that word. Overlapping neighbours are taken
// kIF at a time so their slab loads are in flight together; only the
// lanes inside a neighbour's overlap load and add (the overlap is wave-uniform,
// so it serves directly as the execution mask).
template <bool kExt, int kIF = kInFlight>
__device__ __forceinline__ void pull_sum(const BatchArgs &a, int64_t beg, int64_t end, uint32_t j,
                                         uint64_t want, const uint64_t *F, const uint64_t *SG,
                                         int lane, double &accp, XNum &accx,
                                         unsigned long long &units)
{
    if (beg >= end) return;
    // Pipelined over chunks of kWave neighbours: while chunk c's values are
    // summed, chunk c+1's frontier words and segments and chunk c+2's
    // neighbour ids are in flight. Every lane loads (clamped to the row's last
    // neighbour) so no load sits under a per-lane branch.
    auto nb_at = [&](int64_t base) {
        const int64_t p = base + lane;
        return a.col[p < end ? p : end - 1];
    };
    int32_t x_next = nb_at(beg + kWave);          // ids of chunk c+1
    int64_t xi = ((int64_t)nb_at(beg) << a.logW) + j;
    uint64_t f_cur = F[kFS * xi], s_cur = SG[kFS * xi];   // words of chunk c
    for (int64_t base = beg; base < end; base += kWave) {
        const bool in = base + lane < end;
        const uint64_t fm = in ? f_cur : 0ull;
        const uint64_t sx = (fm & want) ? s_cur : 0ull;
        // issue the next chunk's words and the one after's ids
        const int64_t xin = ((int64_t)x_next << a.logW) + j;
        const uint64_t f_nxt = F[kFS * xin], s_nxt = SG[kFS * xin];
        x_next = nb_at(base + 2 * kWave);
        uint64_t bal = wave_ballot((fm & want) != 0);
        while (bal) {
            double vm[kIF];
            int32_t ve[kIF];
            uint64_t fk[kIF];
            issue_batch<kExt, kIF>(a, fm, sx, want, bal, vm, ve, fk, units);
            add_batch<kExt, kIF>(vm, ve, fk, accp, accx);
        }
        f_cur = f_nxt;
        s_cur = s_nxt;
    }
}

// Rows longer than kHub are summed in parts of kPart neighbours, each part in
// ascending CSR order by a wavefront of its own (k_hub_parts, all parts of a
// level's long rows spread over the device), and the part sums are added in
// part order by the entry's pull: one grouping for every level and kernel.
constexpr int kPart = 256;

__device__ __forceinline__ int32_t row_parts(int64_t deg)
{
    return (int32_t)((deg + kPart - 1) / kPart);
}

// The entry's sum from its row's part sums, in part order.
template <bool kExt>
__device__ __forceinline__ void parts_sum(const BatchArgs &a, int64_t v, uint32_t j, int64_t deg,
                                          const int32_t *hpart, int lane, double &accp,
                                          XNum &accx)
{
    const int32_t parts = row_parts(deg);
    const int64_t first = hpart[v];
#pragma unroll 1
    for (int32_t q = 0; q < parts; ++q) {
        const int64_t o = ((first + q) << (a.logW + 6)) + ((int64_t)j << 6) + lane;
        if (kExt) {
            const XNum y{a.pm[o], a.pe[o]};
            accx = q == 0 ? y : xadd(accx, y);
        } else {
            accp = q == 0 ? a.pm[o] : accp + a.pm[o];
        }
    }
}

// x from the lane DPP control `Ctrl` selects (0 where no lane is selected or
// the row is masked off)
template <int Ctrl, int RowMask, bool BoundCtrl>
__device__ __forceinline__ double dpp_f64(double x)
{
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, Ctrl, RowMask, 0xf, BoundCtrl);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), Ctrl, RowMask, 0xf,
                                               BoundCtrl);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Sum over the 64 lanes in a fixed tree (pairs, quads, half rows, rows, then
// rows 0+1 and 2+3, then all four); the total lands in lane 63. All lanes
// must be active.
__device__ __forceinline__ double wave_sum_to_last(double x)
{
    x += dpp_f64<0xB1, 0xF, true>(x);    // quad_perm [1,0,3,2]
    x += dpp_f64<0x4E, 0xF, true>(x);    // quad_perm [2,3,0,1]
    x += dpp_f64<0x141, 0xF, true>(x);   // row_half_mirror
    x += dpp_f64<0x140, 0xF, true>(x);   // row_mirror
    x += dpp_f64<0x142, 0xA, false>(x);  // row_bcast:15 into rows 1 and 3
    x += dpp_f64<0x143, 0xC, false>(x);  // row_bcast:31 into rows 2 and 3
    return x;
}

// ------------------------------------------------------ tiled pull kernels
//
// A workgroup takes a tile of kTile consecutive record entries and works in
// three phases, so that only the slab loads remain on each entry's critical
// path:
//   1. one thread per entry loads (vertex, word, mask) and the CSR row bounds
//      and makes the entry's read-modify-write updates (visited word, frontier
//      word and segment for the next sweep, running dependency sum), so that
//      no entry waits on them one after another in phase 3;
//   2. all threads walk the tile's concatenated adjacency rows in parallel,
//      loading each neighbour id and its frontier word for the entry's word,
//      and stage (frontier word, pool segment) in LDS;
//   3. each wavefront takes entries in turn: the overlap masks come from LDS,
//      the slab values of overlapping neighbours are loaded eight at a time
//      (lanes = sources) and summed in ascending CSR order.
// Entries whose row is longer than kHub skip staging and take their row's
// part sums (k_hub_parts) in phase 3; entries that no longer fit the tile's
// edge budget gather their neighbours from global memory (the same sums).
constexpr int kTile = 32;
constexpr int kEdgeCap = 1024;

struct TileLds {
    int32_t v[kTile];
    uint32_t j[kTile];
    uint64_t m[kTile];
    uint64_t seg[kTile];
    int64_t beg[kTile];
    int32_t deg[kTile];
    int32_t start[kTile];   // first staged edge (entries not staged: start == end)
    int32_t end[kTile];
    int32_t staged[kTile];
    int32_t total;
    double vs[kTile];       // the entry's running dependency sum before this level
    uint64_t fm[kEdgeCap];  // the neighbour's full frontier word for the entry's word
    uint64_t fs[kEdgeCap];  // the neighbour's pool segment for that word
};

// Sum over staged edges [s0, s1) of the tile: for each neighbour whose
// frontier word shares bits with `want`, the values of the shared lanes.
template <bool kExt, class Lds>
__device__ __forceinline__ void pull_sum_lds(const BatchArgs &a, const Lds &t, int s0, int s1,
                                             uint64_t want, int lane, double &accp, XNum &accx,
                                             unsigned long long &units)
{
    for (int base = s0; base < s1; base += kWave) {
        const int p = base + lane;
        uint64_t fm = 0, sx = 0;
        if (p < s1) {
            fm = t.fm[p];
            sx = t.fs[p];
        }
        uint64_t bal = wave_ballot((fm & want) != 0);
        while (bal) {
            double vm[kInFlight];
            int32_t ve[kInFlight];
            uint64_t fk[kInFlight];
            issue_batch<kExt>(a, fm, sx, want, bal, vm, ve, fk, units);
            add_batch<kExt>(vm, ve, fk, accp, accx);
        }
    }
}

// Phase 3 for entry i of a tile: the sum over its overlapping neighbours in
// ascending CSR order (a row longer than kHub from its part sums, in part
// order), then sigma (forward) or rho and the dependency (backward) for the
// entry's lanes.
template <bool kExt, bool kBackward, class Lds>
__device__ __forceinline__ void entry_sum(const BatchArgs &a, const Lds &t, int i, int lane,
                                          const uint64_t *F, const uint64_t *SG,
                                          unsigned long long &ua, unsigned long long &ub)
{
    const int64_t v = __builtin_amdgcn_readfirstlane(t.v[i]);
    const uint32_t j = (uint32_t)__builtin_amdgcn_readfirstlane((int)t.j[i]);
    const uint64_t m = uniform_u64(t.m[i]);
    const uint64_t seg = uniform_u64(t.seg[i]);
    const int b = (int)(j << 6) + lane;
    const bool mine = lane_in(m);
    // backward: every lane loads its slot (the segment's first slot outside the
    // entry) and computes rho, only the entry's lanes store (a load under a
    // per-lane branch makes the compiler wait for all outstanding memory
    // operations, the previous entry's stores included, before the next one)
    const uint64_t own_slot = seg + ((kBackward && !mine) ? 0u : slot_rank(m));
    double own = 1.0;
    int32_t owne = 0;
    int32_t dstb = -1;
    if (kBackward) {
        own = a.sig[own_slot];
        if (kExt) owne = a.sige[own_slot];
        if (a.dest) dstb = a.dest[b];
    }
    XNum acc{0.0, 0};
    double accp = 0.0;
    ua += __popcll(m);
    if (t.staged[i]) {
        pull_sum_lds<kExt>(a, t, t.start[i], t.start[i] + t.deg[i], m, lane, accp, acc, ub);
    } else if (t.deg[i] > kHub) {
        parts_sum<kExt>(a, v, j, t.deg[i], a.hpart, lane, accp, acc);
    } else {
        // a row the tile could not stage: its neighbours from global memory
        const int64_t beg = (int64_t)uniform_u64((uint64_t)t.beg[i]);
        pull_sum<kExt>(a, beg, beg + __builtin_amdgcn_readfirstlane(t.deg[i]), j, m, F, SG,
                       lane, accp, acc, ub);
    }
    if (!kBackward) {
        if (mine) {
            if (kExt) {
                a.sig[own_slot] = acc.m;
                a.sige[own_slot] = acc.e;
            } else {
                a.sig[own_slot] = accp;
                if (!(accp < 0x1p1000)) a.ctl[CTL_SIG_OVERFLOW] = 1ull;
            }
            if (a.dest && a.dest[b] == (int32_t)v)
                atomicAnd((unsigned long long *)&a.active[j], ~(1ull << lane));
        }
    } else {
        // a slot without a destination (< 0) is a source sample
        const double term = dstb >= 0 ? (dstb == (int32_t)v ? 1.0 : 0.0) : 1.0;
        double d;
        if (kExt) {
            // delta = sigma(v) * sum(rho): exponents add back to the plain range
            d = acc.m == 0.0 ? 0.0 : ldexp(own * acc.m, owne + acc.e);
            const XNum r = xnorm((term + d) / own, -owne);
            if (mine) {
                a.sig[own_slot] = r.m;
                a.sige[own_slot] = r.e;
            }
        } else {
            d = own * accp;
            const double rho = (term + d) / own;
            if (mine) a.sig[own_slot] = rho;
        }
        d = mine ? d : 0.0;
        if (mine && a.dlt) a.dlt[v * a.B + b] = d;
        if (a.vsum) {
            const double tsum = wave_sum_to_last(d);
            if (lane == kWave - 1) a.vsum[((uint32_t)v << a.logW) + j] = t.vs[i] + tsum;
        }
    }
}

// kBackward = false: sigma pull for the new level (F/SG = previous frontier;
//   masks and pool segments from the record written by k_level_write; the
//   segments are published in SGo for the next level's pull).
// kBackward = true: dependency sweep (F/SG = next-deeper frontier, masks and
//   segments from the record; the entry's own word and segment are scattered
//   into Fo/SGo for the next, shallower level).
template <bool kExt, bool kBackward>
__device__ __forceinline__ void pull_tiles(BatchArgs a, int64_t e0, int64_t e1, const uint64_t *F,
                                           const uint64_t *SG, uint64_t *Fo, uint64_t *SGo)
{
    __shared__ TileLds t;
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwv = kBlock / kWave;
    const uint32_t wmask = (1u << a.logW) - 1u;
    unsigned long long ua = 0, ub = 0;
    for (int64_t tile = e0 + (int64_t)blockIdx.x * kTile; tile < e1;
         tile += (int64_t)gridDim.x * kTile) {
        // phase 1 (wave 0): entry headers, pool segments, staging plan
        if (wv == 0) {
            const int64_t e = tile + lane;
            int32_t v = 0, deg = 0;
            uint32_t j = 0;
            uint64_t m = 0, seg = 0;
            int64_t beg = 0;
            if (lane < kTile && e < e1) {
                const uint32_t idx = a.ridx[e];
                v = (int32_t)(idx >> a.logW);
                j = idx & wmask;
                m = a.rmask[e];
                seg = a.rseg[e];
                beg = a.row[v];
                deg = (int32_t)(a.row[v + 1] - beg);
            }
            const int de = deg <= kHub ? deg : 0;
            int incl = de;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int y = __shfl_up(incl, off, 64);
                if (lane >= off) incl += y;
            }
            const bool fits = incl <= kEdgeCap;
            const int endp = fits ? incl : kEdgeCap;
            const int startp = fits ? incl - de : kEdgeCap;
            int maxfit = fits ? incl : 0;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const int y = __shfl_xor(maxfit, off, 64);
                maxfit = maxfit > y ? maxfit : y;
            }
            if (lane < kTile) {
                t.v[lane] = v;
                t.j[lane] = j;
                t.m[lane] = m;
                t.seg[lane] = seg;
                t.beg[lane] = beg;
                t.deg[lane] = deg;
                t.start[lane] = (fits && de == deg) ? startp : endp;
                t.end[lane] = endp;
                t.staged[lane] = (fits && de == deg) ? 1 : 0;
            }
            if (lane == 0) t.total = maxfit;
            // per-entry bookkeeping, one lane per entry (each (v, j) occurs
            // once per level, so these updates do not race)
            if (lane < kTile && e < e1) {
                const uint32_t idx = ((uint32_t)v << a.logW) + j;
                if (!kBackward) {
                    SGo[kFS * idx] = seg;
                } else {
                    Fo[kFS * idx] = m;
                    SGo[kFS * idx] = seg;
                    if (a.vsum) t.vs[lane] = a.vsum[idx];
                }
            }
        }
        __syncthreads();
        // phase 2: stage neighbours with their frontier words and segments
        const int total = t.total;
        for (int p = tid; p < total; p += blockDim.x) {
            int lo = 0, hi = kTile - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (t.end[mid] > p) hi = mid;
                else lo = mid + 1;
            }
            const int i = lo;
            const int32_t x = a.col[t.beg[i] + (p - t.start[i])];
            const int64_t xi = ((int64_t)x << a.logW) + t.j[i];
            // mask and segment share the record's line: both loaded
            const uint64_t fm = F[kFS * xi], sg = SG[kFS * xi];
            t.fm[p] = fm;
            t.fs[p] = (fm & t.m[i]) ? sg : 0;
        }
        __syncthreads();
        // phase 3: value sums, one entry per wavefront at a time (a row longer
        // than kHub from its part sums)
        for (int i = wv; i < kTile; i += nwv) {
            if (tile + i >= e1) break;
            entry_sum<kExt, kBackward>(a, t, i, lane, F, SG, ua, ub);
        }
        __syncthreads();
    }
    prof_add(a, kBackward ? PROF_BACKWARD : PROF_SIGMA, ua, ub,
             lane);
}

// sigma_s(w) = sum over predecessors u (neighbours one level up, Definition 3)
// of sigma_s(u), in ascending CSR order.
// The plain-FP64 pull kernels are latency bound: they are held to 64 VGPRs so
// that eight wavefronts share each SIMD (the scalar registers that do not fit
// are kept in vector-register lanes).
template <bool kExt>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kExt ? 1 : 8, 8))) void k_sigma_pull(BatchArgs a, int64_t e0, int64_t e1,
                                                       const uint64_t *cur, const uint64_t *sgcur,
                                                       uint64_t *sgnxt)
{
    // predecessors are in-neighbours
    BatchArgs b = a;
    b.row = a.rrow;
    b.col = a.rcol;
    b.hpart = a.rhpart;
    pull_tiles<kExt, false>(b, e0, e1, cur, sgcur, nullptr, sgnxt);
}

// Theorem 1 in the rho form: delta(v) = sigma(v) * sum over successors w of
// rho(w), rho(w) = (1 + delta(w)) / sigma(w). Pair mode replaces the 1 by the
// indicator of the pair's destination, which yields sigma_uv(t)/sigma_uv.
// With a.vsum set, the entry's dependencies are also summed over its lanes
// (fixed tree order) into vsum[v][j]; each (v, j) appears once per level and
// levels run in sequence, so the accumulation needs no atomics.
template <bool kExt>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kExt ? 1 : 8, 8))) void k_backward(BatchArgs a, int64_t e0, int64_t e1,
                                                     const uint64_t *fnext, const uint64_t *sgnext,
                                                     uint64_t *fown, uint64_t *sgown)
{
    pull_tiles<kExt, true>(a, e0, e1, fnext, sgnext, fown, sgown);
}

// ------------------------------------------------------- long rows in parts
//
// Before a pull over the record entries [e0, e1), each part of kPart
// neighbours of an entry whose row (in the pull's direction: a.row / a.col /
// a.hpart) is longer than kHub becomes a task, and every task is summed by
// one wavefront.

// task: record entry << kTaskPartBits | part
constexpr int kTaskPartBits = 24;

// the level's long-row parts as tasks, appended at ctl[CTL_HUBS] (zeroed
// beforehand), one atomic per wavefront
__global__ void k_hub_find(BatchArgs a, int64_t e0, int64_t e1, uint64_t *tasks)
{
    const int lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = e0 + blockIdx.x * (int64_t)blockDim.x; b < e1; b += stride) {
        const int64_t e = b + threadIdx.x;
        int32_t parts = 0;
        if (e < e1) {
            const int64_t v = a.ridx[e] >> a.logW;
            if (a.hpart[v] >= 0) parts = row_parts(a.row[v + 1] - a.row[v]);
        }
        int32_t incl = parts;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int32_t y = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += y;
        }
        const int32_t total = __shfl(incl, kWave - 1, kWave);
        unsigned long long base = 0;
        if (lane == 0 && total) base = atomicAdd(&a.ctl[CTL_HUBS], (unsigned long long)total);
        base = __shfl(base, 0, kWave) + (unsigned long long)(incl - parts);
        for (int32_t q = 0; q < parts; ++q)
            tasks[base + q] = ((uint64_t)e << kTaskPartBits) | (uint64_t)q;
    }
}

// One wavefront per task: the sum over the part's neighbours of the
// overlapping lanes' values (as the pulls take them), into the part's slot.
template <bool kExt>
__global__ __launch_bounds__(kBlock) void k_hub_parts(BatchArgs a, const uint64_t *F,
                                                      const uint64_t *SG, const uint64_t *tasks)
{
    const int lane = lane_id();
    const int64_t nt = (int64_t)a.ctl[CTL_HUBS];
    const uint32_t wmask = (1u << a.logW) - 1u;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    unsigned long long ub = 0;
    for (int64_t t = wave; t < nt; t += waves) {
        const uint64_t tk = uniform_u64(tasks[t]);
        const int64_t e = (int64_t)(tk >> kTaskPartBits);
        const int64_t q = (int64_t)(tk & ((1ull << kTaskPartBits) - 1ull));
        const uint32_t idx = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.ridx[e]);
        const int64_t v = idx >> a.logW;
        const uint32_t j = idx & wmask;
        const uint64_t m = uniform_u64(a.rmask[e]);
        const int64_t end = a.row[v + 1];
        const int64_t pb = a.row[v] + q * kPart;
        const int64_t pe = pb + kPart < end ? pb + kPart : end;
        double p = 0.0;
        XNum x{0.0, 0};
        pull_sum<kExt>(a, pb, pe, j, m, F, SG, lane, p, x, ub);
        const int64_t o = ((a.hpart[v] + q) << (a.logW + 6)) + ((int64_t)j << 6) + lane;
        if (kExt) {
            a.pm[o] = x.m;
            a.pe[o] = x.e;
        } else {
            a.pm[o] = p;
        }
    }
    prof_add(a, PROF_HUB_PARTS, 0, ub, lane);
}

// ------------------------------------------------------------- lane order
//
// Which sample sits in which lane does not change any per-sample value, but it
// decides how many (vertex, word) entries and overlapping neighbours a batch
// has: a word whose 64 sources are close to each other meets each vertex at
// fewer distinct levels. Sources are therefore sorted by a clustering key
// (distances to a few landmark vertices) before they are cut into batches.

// The key packs the BFS distance of v from landmark l (capped at 255; 255
// when unreached) into byte 7 - l. All landmarks advance together: bit l of
// a frontier byte marks v as on landmark l's current level.

// level 0: key bytes 255, the landmarks themselves at distance 0
__global__ void k_key_init(const int32_t *lm, int32_t nl, int64_t n, uint8_t *f, uint8_t *seen,
                           uint64_t *key)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        uint8_t bits = 0;
        uint64_t k = ~0ull;
        for (int l = 0; l < nl; ++l)
            if (lm[l] == v) {
                bits |= (uint8_t)(1u << l);
                k &= ~(0xffull << (8 * (7 - l)));
            }
        f[v] = bits;
        seen[v] = bits;
        key[v] = k;
    }
}

// one level (bottom-up): v joins landmark l's next level when a neighbour is
// on its current one; `grew` is set when any vertex joins
__global__ void k_key_level(const int64_t *row, const int32_t *col, int64_t n, uint8_t all,
                            int32_t level, const uint8_t *f, uint8_t *fn, uint8_t *seen,
                            uint64_t *key, unsigned long long *grew)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const uint8_t want = (uint8_t)(all & ~seen[v]);
        uint8_t fresh = 0;
        if (want) {
            uint8_t acc = 0;
            for (int64_t e = row[v], end = row[v + 1]; e < end; ++e) {
                acc |= f[col[e]];
                if ((acc & want) == want) break;
            }
            fresh = acc & want;
        }
        fn[v] = fresh;
        if (fresh) {
            seen[v] |= fresh;
            uint64_t k = key[v];
            const uint64_t d = level < 255 ? (uint64_t)level : 255u;
            for (int l = 0; l < 8; ++l)
                if ((fresh >> l) & 1u) k = (k & ~(0xffull << (8 * (7 - l)))) | (d << (8 * (7 - l)));
            key[v] = k;
            *grew = 1ull;
        }
    }
}

// Final key: the distance bytes interleaved bit by bit (Morton order), most
// significant bits first, each distance clamped to `bits` bits: sources whose
// distances to all landmarks are close get close keys.
__global__ void k_key_morton(uint64_t *key, int64_t n, int32_t bits)
{
    const uint64_t top = (1ull << bits) - 1ull;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = key[v];
        uint64_t m = 0;
        for (int b = bits - 1; b >= 0; --b)
            for (int l = 0; l < 8; ++l) {
                uint64_t d = (k >> (8 * (7 - l))) & 0xffull;
                d = d > top ? top : d;
                m = (m << 1) | ((d >> b) & 1ull);
            }
        key[v] = m;
    }
}

// sort input: out[i] = key[src[i]], idx[i] = i
__global__ void k_key_gather(const uint64_t *key, const int32_t *src, int64_t k, uint64_t *out,
                             int32_t *idx)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * blockDim.x) {
        out[i] = key[src[i]];
        idx[i] = (int32_t)i;
    }
}

// Batch starting at b0 of the sorted order: lane b takes sample perm[b0 + b]
// (its source, its destination in pair mode, and its caller's row).
__global__ void k_take_batch(const int32_t *perm, int64_t b0, int32_t count, const int32_t *src,
                             const int32_t *dst, int32_t *lane_src, int32_t *lane_dst,
                             int32_t *lane_row)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < count) {
        const int32_t r = perm[b0 + b];
        lane_src[b] = src[r];
        if (dst) lane_dst[b] = dst[r];
        lane_row[b] = r;
    }
}

// ------------------------------------------------------------------ outputs

__device__ __forceinline__ bool reached(const BatchArgs &a, int64_t v, int b)
{
    return (a.vis[(v << a.logW) + (b >> 6)] >> (b & 63)) & 1ull;
}

// out[row(b) * n + v] = delta_{s_b}(v) for b < count (0 where unreached)
__global__ void k_out_full(BatchArgs a, int32_t count, int64_t b0, double *out)
{
    const int64_t total = a.n * count;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = i / count;
        const int b = (int)(i - v * count);
        out[out_row(a, b0, b) * a.n + v] = reached(a, v, b) ? a.dlt[v * a.B + b] : 0.0;
    }
}

// out[row(b) * T + t] = delta_{s_b}(targets[t]) for b < count (0 where unreached)
__global__ void k_out_targets(BatchArgs a, const int32_t *targets, int32_t T, int32_t count,
                              int64_t b0, double *out)
{
    const int64_t total = (int64_t)count * T;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(i / T);
        const int t = (int)(i - (int64_t)b * T);
        const int64_t v = targets[t];
        out[out_row(a, b0, b) * T + t] = reached(a, v, b) ? a.dlt[v * a.B + b] : 0.0;
    }
}

// out[v] += sum over j ascending of vsum[v][j]
// out[v] += the per-word dependency sums of v, in word order. A block's
// vertices have their words staged in LDS by coalesced loads (each thread
// reading its own words would stride a wavefront over 64 lines per word);
// rows are padded by one double so that the threads' row reads fall in
// different banks.
constexpr int kVsumTile = 4096;   // words staged per workgroup
// vertices per tile: at most 1024, so that a padded tile fits the LDS array
__host__ __device__ inline int64_t vsum_tile_vertices(int logW)
{
    const int64_t v = kVsumTile >> logW;
    return v < 1024 ? v : 1024;
}
__global__ __launch_bounds__(kBlock) void k_out_vsum(BatchArgs a, double *out)
{
    __shared__ double t[kVsumTile + kVsumTile / 4];
    const int W = 1 << a.logW;
    const int64_t vb = vsum_tile_vertices(a.logW);   // W <= 64
    for (int64_t v0 = blockIdx.x * vb; v0 < a.n; v0 += (int64_t)gridDim.x * vb) {
        const int64_t cnt = a.n - v0 < vb ? a.n - v0 : vb;
        const double *src = a.vsum + (v0 << a.logW);
        for (int64_t i = threadIdx.x; i < (cnt << a.logW); i += kBlock)
            t[(i >> a.logW) * (W + 1) + (i & (W - 1))] = src[i];
        __syncthreads();
        for (int64_t k = threadIdx.x; k < cnt; k += kBlock) {
            double acc = out[v0 + k];
            for (int j = 0; j < W; ++j) acc += t[k * (W + 1) + j];
            out[v0 + k] = acc;
        }
        __syncthreads();
    }
}


// per-source distances from the level record: dist[row(b)*n + v] = level
__global__ void k_out_dist(BatchArgs a, int64_t e0, int64_t e1, int32_t level, int32_t count,
                           int64_t b0, int32_t *dist)
{
    const uint32_t wmask = (1u << a.logW) - 1u;
    for (int64_t e = e0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < e1;
         e += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t idx = a.ridx[e];
        const int64_t v = idx >> a.logW;
        const int j = (int)(idx & wmask);
        uint64_t m = a.rmask[e];
        while (m) {
            const int l = __ffsll((long long)m) - 1;
            m &= m - 1;
            const int b = (j << 6) + l;
            if (b < count) dist[out_row(a, b0, b) * a.n + v] = level;
        }
    }
}

// per-source path counts from the record (between the forward and backward
// passes): mant[row(b)*n + v], ex[...] for b < count, normalised to [1, 2)
__global__ void k_out_sigma(BatchArgs a, int64_t e0, int64_t e1, int32_t count, int64_t b0,
                            double *mant, int32_t *ex)
{
    const uint32_t wmask = (1u << a.logW) - 1u;
    for (int64_t e = e0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < e1;
         e += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t idx = a.ridx[e];
        const int64_t v = idx >> a.logW;
        const int j = (int)(idx & wmask);
        uint64_t m = a.rmask[e];
        const uint64_t seg = a.rseg[e];
        for (int r = 0; m; ++r) {
            const int l = __ffsll((long long)m) - 1;
            m &= m - 1;
            const int b = (j << 6) + l;
            if (b >= count) continue;
            const XNum x = xnorm(a.sig[seg + r], a.sige ? a.sige[seg + r] : 0);
            const int64_t row = out_row(a, b0, b);
            if (mant) mant[row * a.n + v] = x.m;
            if (ex) ex[row * a.n + v] = x.e;
        }
    }
}

// X[t*B + b] = delta_{s_b}(target_t) (pair mode: sigma_{u_b v_b}(t)/sigma_{u_b v_b})
__global__ void k_gather_targets(BatchArgs a, const int32_t *targets, int32_t T, double *X)
{
    const int64_t total = (int64_t)T * a.B;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(i / a.B);
        const int b = (int)(i - (int64_t)t * a.B);
        const int64_t v = targets[t];
        // lanes may hold the round's samples in another order: write sample order
        const int64_t r = (a.lane_row && b < a.nvalid) ? (int64_t)a.lane_row[b] : (int64_t)b;
        X[(int64_t)t * a.B + r] = (b < a.nvalid && reached(a, v, b)) ? a.dlt[v * a.B + b] : 0.0;
    }
}

// ------------------------------------------------------------------- draws

__global__ void k_draw_sources(uint64_t seed, int64_t j0, int64_t count, int64_t n, int32_t *out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const Block4 r = philox4x64_10((uint64_t)(j0 + i), 0, 0, 0, seed, 0);
        out[i] = (int32_t)scale_to_range(r.w[0], (uint64_t)n);
    }
}

__global__ void k_draw_pairs(uint64_t seed, int64_t j0, int64_t count, int64_t n, int32_t *us,
                             int32_t *vs)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const Block4 r = philox4x64_10((uint64_t)(j0 + i), 0, 0, 0, seed, 1);
        const int64_t u = scale_to_range(r.w[0], (uint64_t)n);
        int64_t v = scale_to_range(r.w[1], (uint64_t)(n - 1));
        v += (v >= u) ? 1 : 0;
        us[i] = (int32_t)u;
        vs[i] = (int32_t)v;
    }
}

// ------------------------------------------------------------- stop rules

enum : uint8_t { ST_DONE = 0, ST_CAPPED = 1, ST_RUNNING = 255 };
enum : int32_t { RULE_SOURCE = 0, RULE_PAIR_ALG1 = 1, RULE_PAIR_EPS = 2 };

struct StopArgs {
    int32_t T;
    int32_t rule;
    double threshold;   // c * n
    double eps_rhs;     // eps^3 * n^2
    int64_t k_max;
    double *S;
    int64_t *K;
    uint8_t *status;
};

// One sample of the sequential loop: add, count, then test (the crossing
// sample counts). Source sampling and the literal Algorithm 1 repeat while
// S <= c*n; the epsilon rule stops at S > 0 and k*S^2 >= eps^3 n^2.
__device__ __forceinline__ void stop_step(double &S, int64_t &k, uint8_t &st, double x,
                                          int32_t rule, double threshold, double eps_rhs,
                                          int64_t k_max)
{
    S = S + x;
    k = k + 1;
    bool stop;
    if (rule == RULE_PAIR_EPS) stop = (S > 0.0) && (((double)k * (S * S)) >= eps_rhs);
    else stop = S > threshold;
    if (stop) st = ST_DONE;
    else if (k == k_max) st = ST_CAPPED;
}

// One lane per target walks the round's samples in draw order, exactly as the
// sequential loop would.
__global__ void k_stop_rule(StopArgs s, const double *X, int32_t B, int32_t nb,
                            unsigned long long *ctl)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= s.T) return;
    double S = s.S[t];
    int64_t k = s.K[t];
    uint8_t st = s.status[t];
    for (int b = 0; b < nb && st == ST_RUNNING; ++b)
        stop_step(S, k, st, X[(int64_t)t * B + b], s.rule, s.threshold, s.eps_rhs, s.k_max);
    s.S[t] = S;
    s.K[t] = k;
    s.status[t] = st;
    if (st == ST_RUNNING) atomicAdd(&ctl[CTL_RUNNING], 1ull);
}

__global__ void k_stop_init(StopArgs s)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= s.T) return;
    s.S[t] = 0.0;
    s.K[t] = 0;
    s.status[t] = ST_RUNNING;
}

// est = n*S/k (sources) or n(n-1)*S/k (pairs)
__global__ void k_stop_finish(StopArgs s, double scale, double *est, int64_t *samples,
                              double *S_out, uint8_t *status)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= s.T) return;
    est[t] = (scale * s.S[t]) / (double)s.K[t];
    samples[t] = s.K[t];
    S_out[t] = s.S[t];
    status[t] = s.status[t];
}

// ------------------------------------------------ pair-per-thread engine
//
// For graphs of large diameter the sources of a batch sit at unrelated levels
// of most vertices, so one lane per (vertex, source) pair replaces one
// wavefront per (vertex, 64-source word). Arrays are source-major ([B][n]):
// source b's levels, counts and dependencies are contiguous, so neighbouring
// vertices of one source share cache lines. The level record holds pair
// indices o = b*n + v (32-bit), level by level.

struct PairArgs {
    const int64_t *row;   // out-neighbours
    const int32_t *col;
    const int64_t *rrow;  // in-neighbours (the same arrays when undirected)
    const int32_t *rcol;
    uint32_t n;
    int32_t B;
    int32_t *lv;         // [B][n] level, -1 = unreached
    double *sig;         // [B][n] sigma, then rho after the backward pass of its level
    int32_t *sige;       // [B][n] exponents in extended mode, else null
    double *dlt;         // [B][n] dependency
    uint32_t *rec;       // level record of pair indices
    int64_t cap;
    unsigned long long *ctl;
    uint8_t *active;     // [B] pair mode: slot still expanding
    const int32_t *srcs;
    const int32_t *dest; // [B] pair destinations, or null
    int32_t nvalid;
    unsigned long long *prof;
};

__device__ __forceinline__ void pair_split(const PairArgs &a, uint32_t o, uint32_t &b, uint32_t &v)
{
    b = o / a.n;
    v = o - b * a.n;
}

__global__ void k_p_init(PairArgs a)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    bool want = false;
    uint32_t o = 0;
    if (b < a.nvalid) {
        o = (uint32_t)b * a.n + (uint32_t)a.srcs[b];
        a.lv[o] = 0;
        a.sig[o] = 1.0;
        if (a.sige) a.sige[o] = 0;
        a.dlt[o] = 0.0;
        a.active[b] = 1;
        want = true;
    }
    const int64_t pos = wave_append(want, &a.ctl[CTL_TAIL]);
    if (want) {
        if (pos < a.cap) a.rec[pos] = o;
        else a.ctl[CTL_REC_OVERFLOW] = 1ull;
    }
}

// Top-down discovery: each pair (v, b) of the level claims its unreached
// neighbours for source b (compare-and-swap on the level word). A lane looks
// at four neighbours per step and the wavefront appends all its claims of
// that step with one atomic. Grid-stride over [e0, e1); returns this lane's
// claim count. Every lane of the wavefront must call it.
__device__ __forceinline__ unsigned long long p_topdown(const PairArgs &a, int64_t e0, int64_t e1,
                                                        int32_t level)
{
    const int lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long found = 0;
    for (int64_t i0 = e0 + blockIdx.x * (int64_t)blockDim.x; i0 < e1; i0 += stride) {
        const int64_t i = i0 + threadIdx.x;
        uint32_t b = 0, v = 0;
        int64_t beg = 0;
        int32_t deg = 0;
        if (i < e1) {
            pair_split(a, a.rec[i], b, v);
            if (!a.dest || a.active[b]) {
                beg = a.row[v];
                deg = (int32_t)(a.row[v + 1] - beg);
            }
        }
        for (int k0 = 0;; k0 += 4) {
            if (wave_ballot(k0 < deg) == 0) break;
            uint32_t c[4];
            int cnt = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                c[q] = 0;
                if (k0 + q < deg) {
                    const uint32_t ox = b * a.n + (uint32_t)a.col[beg + k0 + q];
                    if (a.lv[ox] < 0 && atomicCAS(&a.lv[ox], -1, level + 1) == -1) {
                        c[q] = ox + 1u;   // 0 = no claim
                        ++cnt;
                    }
                }
            }
            found += cnt;
            // exclusive prefix of the claim counts across the wavefront
            int incl = cnt;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int y = __shfl_up(incl, off, 64);
                if (lane >= off) incl += y;
            }
            const int tot = __shfl(incl, 63, 64);
            if (tot == 0) continue;
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(&a.ctl[CTL_TAIL], (unsigned long long)tot);
            base = lane_read_u64(base, 0);
            int64_t pos = (int64_t)base + (incl - cnt);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (c[q]) {
                    if (pos < a.cap) a.rec[pos] = c[q] - 1u;
                    else a.ctl[CTL_REC_OVERFLOW] = 1ull;
                    ++pos;
                }
            }
        }
    }
    return found;
}

// sigma for the pairs discovered at level+1, in [e0, e1): sum over
// neighbours one level up (ascending CSR order), four neighbour loads in
// flight. Adds this lane's pair and DAG-edge counts to ua, ub.
template <bool kExt>
__device__ __forceinline__ void p_sigma(const PairArgs &a_in, int64_t e0, int64_t e1,
                                        int32_t level, unsigned long long &ua,
                                        unsigned long long &ub)
{
    // predecessors are in-neighbours
    PairArgs a = a_in;
    a.row = a_in.rrow;
    a.col = a_in.rcol;
    for (int64_t i = e0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < e1;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t o = a.rec[i];
        uint32_t b, x;
        pair_split(a, o, b, x);
        const uint32_t base = b * a.n;
        double accp = 0.0;
        XNum acc{0.0, 0};
        const int64_t end = a.row[x + 1];
        for (int64_t e = a.row[x]; e < end; e += 4) {
            int32_t y[4];
            bool par[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                y[q] = (e + q < end) ? a.col[e + q] : 0;
                par[q] = (e + q < end) && a.lv[base + (uint32_t)y[q]] == level;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (!par[q]) continue;
                ++ub;
                const uint32_t oy = base + (uint32_t)y[q];
                if (kExt) acc = xadd(acc, XNum{a.sig[oy], a.sige[oy]});
                else accp += a.sig[oy];
            }
        }
        ++ua;
        if (kExt) {
            a.sig[o] = acc.m;
            a.sige[o] = acc.e;
        } else {
            a.sig[o] = accp;
            if (!(accp < 0x1p1000)) a.ctl[CTL_SIG_OVERFLOW] = 1ull;
        }
        if (a.dest && a.dest[b] == (int32_t)x) a.active[b] = 0;
    }
}

// Theorem 1 (rho form) for the pairs of one level, in [e0, e1).
template <bool kExt>
__device__ __forceinline__ void p_backward(const PairArgs &a, int64_t e0, int64_t e1,
                                           int32_t level, unsigned long long &ua,
                                           unsigned long long &ub)
{
    for (int64_t i = e0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < e1;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t o = a.rec[i];
        uint32_t b, v;
        pair_split(a, o, b, v);
        const uint32_t base = b * a.n;
        double accp = 0.0;
        XNum acc{0.0, 0};
        const int64_t end = a.row[v + 1];
        for (int64_t e = a.row[v]; e < end; e += 4) {
            int32_t w[4];
            bool suc[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                w[q] = (e + q < end) ? a.col[e + q] : 0;
                suc[q] = (e + q < end) && a.lv[base + (uint32_t)w[q]] == level + 1;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (!suc[q]) continue;
                ++ub;
                const uint32_t ow = base + (uint32_t)w[q];
                if (kExt) acc = xadd(acc, XNum{a.sig[ow], a.sige[ow]});
                else accp += a.sig[ow];
            }
        }
        ++ua;
        const double term =
            (a.dest && a.dest[b] >= 0) ? (a.dest[b] == (int32_t)v ? 1.0 : 0.0) : 1.0;
        double d;
        if (kExt) {
            const XNum s{a.sig[o], a.sige[o]};
            d = acc.m == 0.0 ? 0.0 : ldexp(s.m * acc.m, s.e + acc.e);
            const XNum r = xnorm((term + d) / s.m, -s.e);
            a.sig[o] = r.m;
            a.sige[o] = r.e;
        } else {
            const double s = a.sig[o];
            d = s * accp;
            a.sig[o] = (term + d) / s;
        }
        a.dlt[o] = d;
    }
}

__global__ void k_p_topdown(PairArgs a, int64_t e0, int64_t e1, int32_t level)
{
    const unsigned long long found = p_topdown(a, e0, e1, level);
    if (a.prof) {
        const unsigned long long t = wave_sum_u64(found);
        if (lane_id() == 0 && t) atomicAdd(prof_slot(a.prof, PROF_TOPDOWN, 0), t);
    }
}

template <bool kExt>
__global__ void k_p_sigma(PairArgs a, int64_t e0, int64_t e1, int32_t level)
{
    unsigned long long ua = 0, ub = 0;
    p_sigma<kExt>(a, e0, e1, level, ua, ub);
    if (a.prof) prof_add_raw(a.prof, PROF_SIGMA, wave_sum_u64(ua), wave_sum_u64(ub));
}

template <bool kExt>
__global__ void k_p_backward(PairArgs a, int64_t e0, int64_t e1, int32_t level)
{
    unsigned long long ua = 0, ub = 0;
    p_backward<kExt>(a, e0, e1, level, ua, ub);
    if (a.prof) prof_add_raw(a.prof, PROF_BACKWARD, wave_sum_u64(ua), wave_sum_u64(ub));
}

// ------------------------------------------ pair engine: persistent level loops
//
// A deep graph has thousands of levels, each with little work: one launch
// per level phase spends most of its time starting and draining the grid.
// The loops below run every level of a pass in one launch on a grid that is
// resident as a whole (cooperative launch, sized by occupancy), with a grid
// barrier between phases. The barrier's wait is bounded by wall-clock time:
// a block that waits too long raises the failure flag and leaves, every other
// block then fails its next wait too, and the host reports the error, so
// every wait ends.

// bar[0]: arrivals, bar[1]: generation, bar[2]: failure flag
struct GridSync {
    unsigned long long *bar;
    unsigned long long nblocks;
    uint64_t limit;       // wall-clock ticks a block may wait at one barrier
};

__device__ __forceinline__ unsigned long long ld_acquire(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Returns false once the failure flag is set (by this block or another).
__device__ bool grid_sync(const GridSync &g)
{
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        int good = 1;
        __threadfence();
        const unsigned long long gen = ld_acquire(&g.bar[1]);
        const unsigned long long arrived = atomicAdd(&g.bar[0], 1ull);
        if (arrived == g.nblocks - 1) {
            __hip_atomic_store(&g.bar[0], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&g.bar[1], 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const uint64_t t0 = wall_clock64();
            while (ld_acquire(&g.bar[1]) == gen) {
                if (ld_acquire(&g.bar[2]) != 0ull || wall_clock64() - t0 > g.limit) {
                    atomicOr(&g.bar[2], 1ull);
                    good = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __threadfence();
        if (ld_acquire(&g.bar[2]) != 0ull) good = 0;
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

// loff[l] = first record entry of level l; ctl[CTL_TAIL] = record tail;
// ctl[CTL_LEVELS] receives the number of levels when the pass ends.
struct PairLoop {
    PairArgs a;
    unsigned long long *loff;
    int64_t max_levels;
    GridSync gs;
};

// Forward pass from the level-0 record [0, nvalid): discovery, then
// the path counts of the new level, level after level until a level comes
// out empty (or, in plain FP64, a count reaches 2^1000: the host then redoes
// the batch with extended counts).
template <bool kExt>
__global__ __launch_bounds__(kBlock) void k_p_forward_loop(PairLoop L)
{
    const PairArgs &a = L.a;
    // level 0 holds one entry per valid lane (k_p_init). It must not be read
    // from the record tail: blocks start at different times, and the first
    // ones are already appending level 1 while later ones start.
    int64_t e0 = 0;
    int64_t e1 = a.nvalid;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        L.loff[0] = 0;
        L.loff[1] = (unsigned long long)e1;
    }
    unsigned long long found = 0, ua = 0, ub = 0;
    int32_t level = 0;
    for (;; ++level) {
        found += p_topdown(a, e0, e1, level);
        if (!grid_sync(L.gs)) break;
        const int64_t e2 = (int64_t)__hip_atomic_load(&a.ctl[CTL_TAIL], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
        if (level + 2 >= L.max_levels && blockIdx.x == 0 && threadIdx.x == 0)
            a.ctl[CTL_REC_OVERFLOW] = 1ull;   // no room for the next level's offset
        const bool stop = e2 == e1 || level + 2 >= L.max_levels ||
                          __hip_atomic_load(&a.ctl[CTL_REC_OVERFLOW], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                          (!kExt && __hip_atomic_load(&a.ctl[CTL_SIG_OVERFLOW], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT) != 0);
        if (stop) break;
        if (blockIdx.x == 0 && threadIdx.x == 0) L.loff[level + 2] = (unsigned long long)e2;
        p_sigma<kExt>(a, e1, e2, level, ua, ub);
        if (!grid_sync(L.gs)) break;
        e0 = e1;
        e1 = e2;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl[CTL_LEVELS] = (unsigned long long)(level + 1);
    // every discovered pair gets its path count once: found and ua agree
    (void)found;
    if (a.prof) prof_add_raw(a.prof, PROF_PAIR_FWD, wave_sum_u64(ua), wave_sum_u64(ub));
}

// Backward pass over levels nlev-1 .. 1 of the record laid out by the forward
// loop.
template <bool kExt>
__global__ __launch_bounds__(kBlock) void k_p_backward_loop(PairLoop L, int32_t nlev)
{
    const PairArgs &a = L.a;
    unsigned long long ua = 0, ub = 0;
    for (int32_t level = nlev - 1; level >= 1; --level) {
        p_backward<kExt>(a, (int64_t)L.loff[level], (int64_t)L.loff[level + 1], level, ua, ub);
        if (level > 1 && !grid_sync(L.gs)) break;
    }
    if (a.prof) prof_add_raw(a.prof, PROF_PAIR_BWD, wave_sum_u64(ua), wave_sum_u64(ub));
}

// out[v] += sum over b ascending of the reached pairs' dependencies
__global__ void k_p_out_sum(PairArgs a, double *out)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < a.n;
         v += (int64_t)gridDim.x * blockDim.x) {
        double acc = out[v];
        for (int b = 0; b < a.nvalid; ++b) {
            const uint32_t o = (uint32_t)b * a.n + (uint32_t)v;
            if (a.lv[o] >= 1) acc += a.dlt[o];
        }
        out[v] = acc;
    }
}

__global__ void k_p_out_full(PairArgs a, int32_t count, int64_t b0, double *out)
{
    const int64_t total = (int64_t)a.n * count;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        out[b0 * a.n + i] = a.lv[i] >= 1 ? a.dlt[i] : 0.0;
    }
}

__global__ void k_p_out_targets(PairArgs a, const int32_t *targets, int32_t T, int32_t count,
                                int64_t b0, double *out)
{
    const int64_t total = (int64_t)count * T;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(i / T);
        const int t = (int)(i - (int64_t)b * T);
        const uint32_t o = (uint32_t)b * a.n + (uint32_t)targets[t];
        out[(b0 + b) * T + t] = a.lv[o] >= 1 ? a.dlt[o] : 0.0;
    }
}

__global__ void k_p_out_sigma(PairArgs a, int32_t count, int64_t b0, double *mant, int32_t *ex)
{
    const int64_t total = (int64_t)a.n * count;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const bool r = a.lv[i] >= 0;
        const XNum x = xnorm(r ? a.sig[i] : 0.0, (r && a.sige) ? a.sige[i] : 0);
        if (mant) mant[b0 * a.n + i] = x.m;
        if (ex) ex[b0 * a.n + i] = x.e;
    }
}

__global__ void k_p_gather_targets(PairArgs a, const int32_t *targets, int32_t T, int32_t stride,
                                   double *X)
{
    const int64_t total = (int64_t)T * stride;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(i / stride);
        const int b = (int)(i - (int64_t)t * stride);
        double x = 0.0;
        if (b < a.nvalid) {
            const uint32_t o = (uint32_t)b * a.n + (uint32_t)targets[t];
            if (a.lv[o] >= 1) x = a.dlt[o];
        }
        X[i] = x;
    }
}

// ---------------------------------------------------------------- serving
//
// A serving round fills the B sample slots of one batch with consecutive
// samples of several queries on the same graph: query q owns slots
// [slot0, slot0 + nslots) and draws its samples j0, j0 + 1, ... from its own
// stream. Source and pair samples share the batch (a slot's destination is
// -1 for a source sample). Each slot's value is taken at its own query's
// target, and one lane per query then runs that query's stopping rule over
// its slots in draw order.

struct QueryDesc {
    uint64_t seed;
    int64_t j0;
    int64_t k_max;
    double threshold;
    double eps_rhs;
    double scale;       // n (sources) or n(n-1) (pairs)
    double S;
    int64_t K;
    double est;
    int32_t target;
    int32_t rule;       // RULE_SOURCE, RULE_PAIR_ALG1, RULE_PAIR_EPS
    int32_t slot0;
    int32_t nslots;
    int32_t status;
    int32_t pad;
};

// Draws of slots [b0, b0 + nb) into lanes 0..nb-1 (a round may run its slots
// in parts).
__global__ void k_serve_draw(const QueryDesc *q, const int32_t *slot_query, int32_t b0,
                             int32_t nb, int64_t n, int32_t *srcs, int32_t *dest, int32_t *tgt)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int slot = b0 + b;
    const QueryDesc &d = q[slot_query[slot]];
    const int64_t j = d.j0 + (slot - d.slot0);
    if (d.rule == RULE_SOURCE) {
        const Block4 r = philox4x64_10((uint64_t)j, 0, 0, 0, d.seed, 0);
        srcs[b] = (int32_t)scale_to_range(r.w[0], (uint64_t)n);
        dest[b] = -1;
    } else {
        const Block4 r = philox4x64_10((uint64_t)j, 0, 0, 0, d.seed, 1);
        const int64_t u = scale_to_range(r.w[0], (uint64_t)n);
        int64_t v = scale_to_range(r.w[1], (uint64_t)(n - 1));
        v += (v >= u) ? 1 : 0;
        srcs[b] = (int32_t)u;
        dest[b] = (int32_t)v;
    }
    tgt[b] = d.target;
}

// X[b0 + slot] for the lanes of a part that starts at slot b0
__global__ void k_gather_slots(BatchArgs a, const int32_t *tgt, int32_t b0, double *X)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.nvalid) return;
    const int r = a.lane_row ? a.lane_row[b] : b;   // the lane's slot within the part
    const int64_t v = tgt[r];
    X[b0 + r] = reached(a, v, b) ? a.dlt[v * a.B + b] : 0.0;
}

__global__ void k_p_gather_slots(PairArgs a, const int32_t *tgt, int32_t b0, double *X)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.nvalid) return;
    const uint32_t o = (uint32_t)b * a.n + (uint32_t)tgt[b];
    X[b0 + b] = a.lv[o] >= 1 ? a.dlt[o] : 0.0;
}

__global__ void k_stop_queries(QueryDesc *q, int32_t nq, const double *X)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    QueryDesc d = q[i];
    double S = d.S;
    int64_t k = d.K;
    uint8_t st = (uint8_t)d.status;
    for (int b = d.slot0; b < d.slot0 + d.nslots && st == ST_RUNNING; ++b)
        stop_step(S, k, st, X[b], d.rule, d.threshold, d.eps_rhs, d.k_max);
    q[i].S = S;
    q[i].K = k;
    q[i].status = st;
    q[i].est = st == ST_RUNNING ? 0.0 : (d.scale * S) / (double)k;
}

// -------------------------------------------------- per-source plain form

__global__ void k_ss_init(int32_t *d, double *sig, double *dlt, int32_t *queue, int32_t s)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        d[s] = 0;
        sig[s] = 1.0;
        dlt[s] = 0.0;
        queue[0] = s;
    }
}

__global__ void k_ss_topdown(const int64_t *row, const int32_t *col, int32_t *d, int32_t *queue,
                             int64_t q0, int64_t q1, int32_t level, unsigned long long *ctl)
{
    for (int64_t i = q0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < q1;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = queue[i];
        for (int64_t e = row[u]; e < row[u + 1]; ++e) {
            const int32_t w = col[e];
            if (d[w] < 0 && atomicCAS(&d[w], -1, level + 1) == -1) {
                const unsigned long long pos = atomicAdd(&ctl[CTL_TAIL], 1ull);
                queue[pos] = w;
            }
        }
    }
}

__global__ void k_ss_sigma(const int64_t *row, const int32_t *col, const int32_t *d, double *sig,
                           const int32_t *queue, int64_t q0, int64_t q1, int32_t level,
                           unsigned long long *ctl)
{
    for (int64_t i = q0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < q1;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t w = queue[i];
        double acc = 0.0;
        for (int64_t e = row[w]; e < row[w + 1]; ++e) {
            const int32_t u = col[e];
            if (d[u] == level) acc += sig[u];
        }
        sig[w] = acc;
        if (!(acc < 0x1p1000)) ctl[CTL_SIG_OVERFLOW] = 1ull;
    }
}

__global__ void k_ss_backward(const int64_t *row, const int32_t *col, const int32_t *d,
                              const double *sig, double *dlt, const int32_t *queue, int64_t q0,
                              int64_t q1, int32_t level)
{
    for (int64_t i = q0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < q1;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = queue[i];
        const double sv = sig[v];
        double acc = 0.0;
        for (int64_t e = row[v]; e < row[v + 1]; ++e) {
            const int32_t w = col[e];
            if (d[w] == level + 1) acc += (sv / sig[w]) * (1.0 + dlt[w]);
        }
        dlt[v] = acc;
    }
}

__global__ void k_ss_out_sum(const double *dlt, const int32_t *queue, int64_t q0, int64_t q1,
                             double *out)
{
    for (int64_t i = q0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < q1;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = queue[i];
        out[v] += dlt[v];
    }
}

__global__ void k_ss_out_targets(const int32_t *d, const double *dlt, const int32_t *targets,
                                 int32_t T, double *out_row)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < T;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = targets[t];
        out_row[t] = d[v] > 0 ? dlt[v] : 0.0;
    }
}

__global__ void k_ss_out_full(const int32_t *d, const double *dlt, int64_t n, double *out_row)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        out_row[v] = d[v] > 0 ? dlt[v] : 0.0;
}

// ------------------------------------------------------------------- misc

__global__ void k_iota(int32_t *out, int64_t start, int64_t count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (int32_t)(start + i);
}

__global__ void k_fill_i32(int32_t *out, int32_t value, int64_t count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = value;
}

__global__ void k_fill_f64(double *out, double value, int64_t count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = value;
}

// check sources / targets lie in [0, n); ctl[CTL_REC_OVERFLOW] is reused as
// the "bad index" flag by the host before any batch starts
__global__ void k_check_range(const int32_t *x, int64_t count, int64_t n, unsigned long long *flag)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        if (x[i] < 0 || x[i] >= n) *flag = 1ull;
}

}  // namespace bcmi
