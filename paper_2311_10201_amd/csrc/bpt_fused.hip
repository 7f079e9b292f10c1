// Fused breadth-first probabilistic traversals (paper Section 3, Listing 1)
// for gfx950.
//
// One persistent workgroup owns one "slot" of traversal state and processes
// batches of C = 64*NW samples (colours) one after another, claiming batch
// ids from a device counter until none are left.  Within a batch the
// traversal is level-synchronous (Section 3.2):
//
//   frontier entry   a vertex v with the mask of colours that reached it at
//                    the current depth (Listing 1's frontier[v]).
//   expansion        every in-edge e = (u -> v) of the entry is tried for
//                    every colour of the mask.  Work items are (entry, up to
//                    eight 4-edge quads) spread evenly over the workgroup's
//                    lanes (four quads per item where colours are gathered);
//                    each evaluates one Philox block per colour and quad,
//                    i.e. the coins of four consecutive in-edges.
//                    Coins are flipped before any neighbour data is read
//                    ("flip before gather"): `col[e]` and visited[u] are only
//                    touched for live coins.
//   discovery        a live coin (u, c) sets bit c of visited[u] with a
//                    fetch-old atomic OR; only a truly new bit propagates, into
//                    the next level's frontier mask of u (Listing 1's fusing
//                    OR).  Marking at discovery means each (vertex, colour)
//                    enters a frontier exactly once, so the sets equal the
//                    per-sample reverse BFS of Definition 2 for any schedule.
//
// After the last level the batch's RRR sets are extracted (Listing 1's final
// loop): the touched vertices are sorted (in LDS when few, by a scan of a
// touched-vertex bitmap otherwise), each colour's members are ranked with
// wavefront ballots, written to the output pool in ascending order, and the
// slot's state is reset through the same list.
//
// A second instantiation (kHelp, one-word masks) adds helping at the end of a
// launch: once half the workgroups have no batch left, an owner publishes each
// heavy chunk of its batch to device memory and idle workgroups expand units of
// its work items (help_others).  The host picks it for graphs with large sets.
#include "bpt.h"
#include "bpt_internal.hpp"
#include "bpt_rng.hpp"

namespace bpt {

namespace {

constexpr int kWave = 64;
// Workgroup size BS is a template parameter (128, 256 or 512 threads); a chunk of
// BS frontier entries is staged per pass, and touched lists up to
// sort_cap(BS) vertices are sorted in LDS.
constexpr int sort_cap(int bs) { return bs >= 256 ? 4096 : 2048; }
// Frontier entries each thread stages per pass: fewer for wide masks and wide
// workgroups, to fit LDS and to keep every instantiation within 128 VGPRs.
constexpr int ept(int nw, int bs) {
    return nw == 1 ? (bs <= 512 ? 4 : 2) : (nw == 2 ? (bs <= 256 ? 4 : 2) : (nw == 4 && bs <= 256 ? 2 : 1));
}
constexpr uint32_t kNone = 0xFFFFFFFFu;
// Live coins a wavefront queues in LDS before resolving them: their source
// ids are loaded and their discoveries performed 64 at a time, one per lane,
// so the dependent global round trips of a discovery are paid once per 64
// live coins instead of once per coin loop of every lane that drew one.
constexpr uint32_t kDiscQueue = 256;
constexpr uint32_t kQuadsPerItem = 8;  // 4-edge quads one work item covers at most (one entry lookup)

// Staging of large chunks orders entries by colour count: the lanes of a
// wavefront take consecutive work items, and a lane loops over its entry's
// colours, so a wavefront whose items mix 1-, 2- and 3-colour entries keeps
// lanes idle for the longest (on R-MAT 22 p = 0.01 about a quarter of the
// expansion's lane slots; with entries grouped by colour count, about 6%).
// Buckets, in position order: 64+, 32-63, 16-31, 8-15, 4-7, 3, 2, 1 colours,
// then entries without work items.
constexpr uint32_t kColourBuckets = 9;
__device__ __forceinline__ uint32_t colour_bucket(uint32_t pc) {
    return pc == 0 ? 8u
         : pc >= 64 ? 0u
         : pc >= 32 ? 1u
         : pc >= 16 ? 2u
         : pc >= 8  ? 3u
         : pc >= 4  ? 4u
         : 8u - pc;  // 3 -> 5, 2 -> 6, 1 -> 7
}

// 4-edge quads per work item of an entry with pc colours: kQuadsPerItem in
// general, 4 for entries expected to gather several live colours per edge
// (the test of expand_item), whose quads are heavy: a finer split keeps more
// lanes busy there, a coarser one saves entry lookups elsewhere.
__device__ __forceinline__ uint32_t item_quads(uint32_t pc, uint32_t thr, bool per_edge, uint32_t gather_mode) {
    const uint32_t p_est = per_edge ? 0x80000000u : thr;
    const bool gathers = gather_mode == kGatherAlways ||
                         (gather_mode == kGatherAuto && pc >= 2 && (unsigned long long)pc * p_est >= 0x80000000ull);
    return gathers ? 4u : kQuadsPerItem;
}

template <int NW, int BS>
struct Stage {  // traversal staging of one chunk of ept(NW, BS) * BS frontier entries
    uint32_t beg[BS * ept(NW, BS)];
    uint32_t end[BS * ept(NW, BS)];
    uint32_t thr[BS * ept(NW, BS)];
    uint32_t scan[BS * ept(NW, BS)];
    unsigned long long mask[BS * ept(NW, BS)][NW];
};

template <int NW, int BS>
struct Extract {  // extraction buffers
    uint32_t sorted[sort_cap(BS)];
    uint32_t wprefix[BS / kWave][64 * NW];
};

template <int NW, int BS>
struct FusedShared {
    union {
        Stage<NW, BS> st;
        Extract<NW, BS> ex;
    } u;
    unsigned long long coff[64 * NW];  // first pool position of each colour's set
    uint32_t cnt[64 * NW];             // members per colour (found by this workgroup)
    uint32_t cidx[64 * NW];            // sorted starts: sample index (from the job's first) of each colour
    uint32_t qlen[3];  // frontier sizes of levels L, L+1 (and L+2, reset), indexed by level % 3
    uint32_t tlen;
    unsigned long long batch;
    uint32_t job;
    // helping (one-word masks): the owner's decision and the helpers' commands
    uint32_t tail;     // the launch has no batch left to claim
    uint32_t probes;   // heavy chunks seen before that
    uint32_t go;       // this batch takes helpers from now on
    uint32_t unit;     // unit of work items just claimed
    uint32_t cmd;      // helper: what to do next
    uint32_t pick;     // helper: offset of the slot to join
    uint32_t h_npos, h_nxt, h_qnext;  // helper: the joined chunk's parameters
    unsigned long long claimed;        // helper: value returned by its claim
    uint32_t scan_tmp[2][BS / kWave];
    unsigned long long base;
    unsigned long long stats[kNumStats];
    // live coins waiting for discovery, per wavefront: edge id and colour
    uint32_t dq_e[BS / kWave][kDiscQueue];
    uint16_t dq_c[BS / kWave][kDiscQueue];
    uint32_t dq_len[BS / kWave];
    uint32_t next_item;  // work items of the current chunk handed out to wavefronts so far
    uint32_t bcnt[kColourBuckets];   // staging by colour count: entries per bucket (zero between chunks)
    uint32_t bbase[kColourBuckets];  // ... and each bucket's first position
};

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWave - 1); }

// Values every lane of the wavefront holds alike, moved to scalar registers.
__device__ __forceinline__ uint32_t uni32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    return ((uint64_t)uni32((uint32_t)(x >> 32)) << 32) | uni32((uint32_t)x);
}
template <class T>
__device__ __forceinline__ T* uni_ptr(T* p) {
    return reinterpret_cast<T*>(uni64(reinterpret_cast<uint64_t>(p)));
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, kWave);
        if (lane >= (uint32_t)d) x += y;
    }
    return x;
}

// Exclusive scan over the workgroup; *total receives the sum (all threads).
// One barrier: callers alternate between two `tmp` buffers, and at least one
// other barrier separates two uses of the same buffer.
template <int BS>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* tmp, uint32_t* total) {
    constexpr int kWaves = BS / kWave;
    const uint32_t wid = threadIdx.x / kWave;
    const uint32_t incl = wave_incl_scan(x);
    if (lane_id() == kWave - 1) tmp[wid] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t t = tmp[w];
        before += (w < (int)wid) ? t : 0u;
        all += t;
    }
    *total = all;
    return before + incl - x;
}

__device__ __forceinline__ unsigned long long wave_or64(unsigned long long x) {
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        lo |= __shfl_xor(lo, d, kWave);
        hi |= __shfl_xor(hi, d, kWave);
    }
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long x) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)x, d, kWave);
        const uint32_t hi = __shfl_xor((uint32_t)(x >> 32), d, kWave);
        x += ((unsigned long long)hi << 32) | lo;
    }
    return x;
}

__device__ __forceinline__ unsigned long long bcast64(unsigned long long x, int src) {
    const uint32_t lo = __shfl((uint32_t)x, src, kWave);
    const uint32_t hi = __shfl((uint32_t)(x >> 32), src, kWave);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long lanemask_lt() {
    const uint32_t lane = lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Wavefront issue priority (s_setprio) among the waves resident on a SIMD.
__device__ __forceinline__ void set_wave_priority(int p) {
    switch (p) {
        case 3: __builtin_amdgcn_s_setprio(3); break;
        case 2: __builtin_amdgcn_s_setprio(2); break;
        case 1: __builtin_amdgcn_s_setprio(1); break;
        default: __builtin_amdgcn_s_setprio(0); break;
    }
}

// The slot's traversal state is written with device-scope atomics.  It is
// read back and cleared with agent-scope (device-coherent) loads and stores
// after waiting for this workgroup's own atomics (s_waitcnt): an agent-scope
// acquire/release fence would write back or invalidate a whole L2 on this
// multi-XCD part.
__device__ __forceinline__ void store_coherent(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wait_own_memory_ops() { __builtin_amdgcn_s_waitcnt(0); }
__device__ __forceinline__ unsigned long long load_coherent64(const unsigned long long* p) {
    return __hip_atomic_load(const_cast<unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_coherent64(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_coherent32(const uint32_t* p) {
    return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Where a batch's discovery counters live: the owner's LDS while it runs the
// batch alone, the slot's help record once other workgroups may join (then the
// queue and touched entries are written coherently too).
struct Ctr {
    uint32_t* qlen;  // [3], indexed by level % 3
    uint32_t* tlen;
    uint32_t* cnt;   // [64 * NW]
};

// Traversal state of one slot.  A vertex's masks form one record (visited,
// frontier of even levels, frontier of odd levels: mask_record_words(NW)
// words), so a discovery's fetch-or on the next frontier finds the line its
// fetch-or on visited has just brought in.
template <int NW>
struct BatchCtx {
    unsigned long long* masks;  // n records
    uint32_t* stamp;
    uint32_t* queue0;   // frontier queue of even levels
    uint32_t* queue1;   // frontier queue of odd levels
    uint32_t* touched;  // vertices touched by the batch, in discovery order
    unsigned long long* tbits;
    uint32_t n;
    unsigned int* err;
    bool read_first;  // the batch's job has kJobReadFirst

    static constexpr size_t kRec = mask_record_words(NW);
    __device__ __forceinline__ unsigned long long* vis(uint32_t u, int k) const {
        return masks + (size_t)u * kRec + k;
    }
    // frontier masks of the levels of this parity
    __device__ __forceinline__ unsigned long long* fr(int parity, uint32_t u, int k) const {
        return masks + (size_t)u * kRec + (size_t)(1 + parity) * NW + k;
    }
};

// Slot arrays are strided by the largest n of the launch's graphs; b.n is set
// per batch to the batch's own graph.
template <int NW>
__device__ __forceinline__ BatchCtx<NW> slot_ctx(const FusedArgs& a, uint32_t slot) {
    const uint32_t n = a.n_max;
    BatchCtx<NW> b;
    b.n = n;
    b.err = &a.ctl->err;
    b.read_first = false;
    b.masks = a.ws.masks + (size_t)slot * n * mask_record_words(NW);
    b.stamp = (NW > 1) ? a.ws.stamp + (size_t)slot * n : nullptr;
    b.queue0 = a.ws.queue + (size_t)slot * 2 * n;
    b.queue1 = b.queue0 + n;
    b.touched = a.ws.touched + (size_t)slot * n;
    b.tbits = a.ws.tbits + (size_t)slot * bitmap_words(n);
    return b;
}

// Colours `bits` of word k reached u over live edges: record the new ones once
// (Listing 1's visited / frontier update, one atomic per mask word as in its
// fusing OR, with the visited mark taken at discovery time).  `next` is the
// parity of the level the new frontier entry belongs to, `qslot` its counter.
template <int NW, bool kSh>
__device__ __forceinline__ void discover_word(const BatchCtx<NW>& b, const Ctr& ct, uint32_t u, int k,
                                              unsigned long long bits, int next, uint32_t qslot, uint32_t tag,
                                              uint32_t base_tag) {
    // Read first (jobs with kJobReadFirst): a coin whose colours have all
    // reached u already changes nothing, and a device-coherent load costs well
    // under half a random fetch-or (bits only grow within a batch, so a set
    // bit is never stale).
    unsigned long long* const vp = b.vis(u, k);
    if (b.read_first && !(bits & ~load_coherent64(vp))) return;
    const unsigned long long old = atomicOr(vp, bits);
    unsigned long long fresh = bits & ~old;
    if (!fresh) return;
    const unsigned long long old_next = atomicOr(b.fr(next, u, k), fresh);
    for (unsigned long long f = fresh; f; f &= f - 1)
        atomicAdd(&ct.cnt[k * 64 + (__ffsll((long long)f) - 1)], 1u);
    bool push, first;
    if constexpr (NW == 1) {
        (void)tag;
        (void)base_tag;
        push = (old_next == 0);
        first = (old == 0);
    } else {
        (void)old_next;
        const uint32_t st = atomicMax(&b.stamp[u], tag);
        push = st < tag;
        first = st < base_tag;
    }
    if (push) {
        const uint32_t pos = atomicAdd(&ct.qlen[qslot], 1u);
        uint32_t* q = next ? b.queue1 : b.queue0;
        if (pos >= b.n) atomicOr(b.err, (unsigned)kErrQueueOverflow);
        else if constexpr (kSh) store_coherent(&q[pos], u);
        else q[pos] = u;
    }
    if (first) {
        atomicOr(&b.tbits[u >> 6], 1ull << (u & 63));  // result unused: no wait
        const uint32_t pos = atomicAdd(ct.tlen, 1u);
        if (pos >= b.n) atomicOr(b.err, (unsigned)kErrQueueOverflow);
        else if constexpr (kSh) store_coherent(&b.touched[pos], u);
        else b.touched[pos] = u;
    }
}

// (u, c) became reachable (one colour).
template <int NW, bool kSh>
__device__ __forceinline__ void discover(const BatchCtx<NW>& b, const Ctr& ct, uint32_t u, uint32_t c,
                                         int next, uint32_t qslot, uint32_t tag, uint32_t base_tag) {
    discover_word<NW, kSh>(b, ct, u, (int)(c >> 6), 1ull << (c & 63), next, qslot, tag, base_tag);
}

__device__ __forceinline__ uint32_t live_bits(const Block4& r, const uint4& t) {
    return (coin_live(r.w0, t.x) ? 1u : 0u) | (coin_live(r.w1, t.y) ? 2u : 0u) | (coin_live(r.w2, t.z) ? 4u : 0u) |
           (coin_live(r.w3, t.w) ? 8u : 0u);
}

// Words of a block below one threshold (the p = 1 sentinel is handled by the caller).
__device__ __forceinline__ uint32_t below_bits(const Block4& r, uint32_t t) {
    return (r.w0 < t ? 1u : 0u) | (r.w1 < t ? 2u : 0u) | (r.w2 < t ? 4u : 0u) | (r.w3 < t ? 8u : 0u);
}

// Coins of the work item's quads [q_first, q_end) (at most kQuadsPerItem) of
// the row [beg, end) for every colour in `mask`, and discovery of the live
// ones.  Two schedules, chosen per wavefront (FusedArgs::gather_mode):
//  * mostly one colour per entry: the item's Philox blocks of a colour are
//    independent and are evaluated side by side (in rounds of four when the
//    mask is one word, the row has one threshold and any lane has more than
//    two quads, else in pairs),
//    so that a wavefront alone on its SIMD still keeps the multiplier
//    pipeline busy; each live coin is discovered on its own;
//  * several colours per entry: per (quad, mask word) the blocks of two
//    colours are evaluated side by side and each edge's live colours are
//    gathered into one mask, so visited[u] and the next frontier take one
//    atomic per (edge, word) whatever the number of colours (Listing 1).
template <int NW, int BS, bool kSh>
__device__ __forceinline__ void expand_item(const DevGraph& g, uint64_t seed, uint32_t gather_mode,
                                            const BatchCtx<NW>& b, FusedShared<NW, BS>& s, const Ctr& ct,
                                            const unsigned long long (&mask)[NW], unsigned long long s0,
                                            unsigned long long first, bool ordered,
                                            uint32_t beg, uint32_t end, uint32_t thr_row, uint32_t q_first,
                                            uint32_t q_end, int nxt, uint32_t qslot, uint32_t tag,
                                            uint32_t base_tag, uint32_t& n_philox, uint32_t& n_live) {
    static_assert(kQuadsPerItem % 4 == 0 && kQuadsPerItem <= 8, "an item's coin words must fit 32 bits");
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t nq = q_end - q_first;
    const uint32_t e_first = q_first << 2;
    // coin words of the item that belong to the row
    uint32_t valid = (end - e_first >= 32u) ? 0xFFFFFFFFu : ((1u << (end - e_first)) - 1u);
    if (e_first < beg) valid &= 0xFFFFFFFFu << (beg - e_first);
    const bool per_edge = g.prob_layout == BPT_PROB_EDGE;
    const uint4 t_row = make_uint4(thr_row, thr_row, thr_row, thr_row);
    // one threshold for the whole row: its p = 1 sentinel is tested once per item, and each
    // coin costs one compare (per-edge thresholds test both conditions per coin)
    const uint32_t row_always = (!per_edge && thr_row == kAlwaysLive) ? 0xFu : 0u;
    // thresholds of quad j of the item (per-edge layout: re-read per colour, an L1 hit)
    auto thr_of = [&](uint32_t j) -> uint4 {
        return (per_edge && j < nq) ? *reinterpret_cast<const uint4*>(g.thr_edge + e_first + 4 * j) : t_row;
    };
    // Gathering pays when an edge is expected to be live for several colours at
    // once: colours of the entry x probability >= 1/2 (per-edge thresholds
    // count as 1/2).  A wavefront gathers when a quarter of its lanes would.
    uint32_t pc = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) pc += (uint32_t)__popcll(mask[k]);
    const uint32_t p_est = per_edge ? 0x80000000u : thr_row;
    const bool want = pc >= 2 && (unsigned long long)pc * p_est >= 0x80000000ull;
    const bool gather = gather_mode == kGatherAlways ||
                        (gather_mode == kGatherAuto &&
                         4 * __popcll(__ballot(want)) >= (unsigned)__popcll(__ballot(true)));

    if (gather) {
        for (uint32_t j = 0; j < nq; ++j) {
            const uint32_t quad = q_first + j;
            const uint4 t = thr_of(j);
            const uint32_t vq = (valid >> (4 * j)) & 0xFu;
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                unsigned long long mk = mask[k];
                unsigned long long acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;  // live colours of the 4 edges
                while (mk) {
                    // two colours side by side; an absent second one repeats b0 and is dropped
                    const uint32_t b0 = (uint32_t)(__ffsll((long long)mk) - 1);
                    mk &= mk - 1;
                    const bool h1 = mk != 0;
                    const uint32_t b1 = h1 ? (uint32_t)(__ffsll((long long)mk) - 1) : b0;
                    mk &= h1 ? mk - 1 : mk;
                    const unsigned long long sa = ordered ? first + s.cidx[k * 64 + b0] : s0 + k * 64u + b0;
                    const unsigned long long sb = ordered ? first + s.cidx[k * 64 + b1] : s0 + k * 64u + b1;
                    const Block4 r0 = coin_block(quad, sa, k0, k1);
                    const Block4 r1 = coin_block(quad, sb, k0, k1);
                    n_philox += h1 ? 2u : 1u;
                    const uint32_t l0 = live_bits(r0, t) & vq;
                    const uint32_t l1 = h1 ? live_bits(r1, t) & vq : 0u;
                    const unsigned long long m0 = 1ull << b0, m1 = 1ull << b1;
                    acc0 |= ((l0 & 1u) ? m0 : 0ull) | ((l1 & 1u) ? m1 : 0ull);
                    acc1 |= ((l0 & 2u) ? m0 : 0ull) | ((l1 & 2u) ? m1 : 0ull);
                    acc2 |= ((l0 & 4u) ? m0 : 0ull) | ((l1 & 4u) ? m1 : 0ull);
                    acc3 |= ((l0 & 8u) ? m0 : 0ull) | ((l1 & 8u) ? m1 : 0ull);
                }
                const uint32_t e0 = quad << 2;
                if (acc0) { n_live += __popcll(acc0); discover_word<NW, kSh>(b, ct, g.col[e0], k, acc0, nxt, qslot, tag, base_tag); }
                if (acc1) { n_live += __popcll(acc1); discover_word<NW, kSh>(b, ct, g.col[e0 + 1], k, acc1, nxt, qslot, tag, base_tag); }
                if (acc2) { n_live += __popcll(acc2); discover_word<NW, kSh>(b, ct, g.col[e0 + 2], k, acc2, nxt, qslot, tag, base_tag); }
                if (acc3) { n_live += __popcll(acc3); discover_word<NW, kSh>(b, ct, g.col[e0 + 3], k, acc3, nxt, qslot, tag, base_tag); }
            }
        }
        return;
    }

    // four side by side only where registers allow it (one colour word, one threshold per row); two otherwise
    const bool wide = (NW == 1) && !per_edge && __any(nq > 2);
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        unsigned long long mk = mask[k];
        while (mk) {
            const uint32_t bpos = (uint32_t)(__ffsll((long long)mk) - 1);
            mk &= mk - 1;
            const uint32_t c = (uint32_t)k * 64u + bpos;
            const unsigned long long sc = ordered ? first + s.cidx[c] : s0 + c;  // colour c's sample
            uint32_t live;
            if (wide) {
                live = 0;
                for (uint32_t j = 0; j < nq; j += 4) {  // rounds of four quads
                    const Block4 r0 = coin_block(q_first + j, sc, k0, k1);
                    const Block4 r1 = coin_block(q_first + j + 1, sc, k0, k1);
                    const Block4 r2 = coin_block(q_first + j + 2, sc, k0, k1);
                    const Block4 r3 = coin_block(q_first + j + 3, sc, k0, k1);
                    live |= ((below_bits(r0, thr_row) | (below_bits(r1, thr_row) << 4) |
                              (below_bits(r2, thr_row) << 8) | (below_bits(r3, thr_row) << 12)) |
                             (row_always * 0x1111u)) << (4 * j);
                }
            } else {
                live = 0;
                for (uint32_t j = 0; j < nq; j += 2) {
                    const Block4 r0 = coin_block(q_first + j, sc, k0, k1);
                    const Block4 r1 = coin_block(q_first + j + 1, sc, k0, k1);  // past the row: masked below
                    if (per_edge)
                        live |= (live_bits(r0, thr_of(j)) | (live_bits(r1, thr_of(j + 1)) << 4)) << (4 * j);
                    else
                        live |= (below_bits(r0, thr_row) | (below_bits(r1, thr_row) << 4) | (row_always * 0x11u))
                                << (4 * j);
                }
            }
            n_philox += nq;
            live &= valid;
            if (live) {  // queue the live coins; past the queue's end, discover directly
                const uint32_t k = (uint32_t)__popc(live);
                const uint32_t wid = threadIdx.x / kWave;
                uint32_t p = atomicAdd(&s.dq_len[wid], k);
                n_live += k;
                while (live) {
                    const uint32_t j = (uint32_t)(__ffs((int)live) - 1);
                    live &= live - 1;
                    if (p < kDiscQueue) {
                        s.dq_e[wid][p] = e_first + j;
                        s.dq_c[wid][p] = (uint16_t)c;
                    } else {
                        discover<NW, kSh>(b, ct, g.col[e_first + j], c, nxt, qslot, tag, base_tag);
                    }
                    ++p;
                }
            }
        }
    }
}

// Moves one staged field of this thread's entries (places tid*E .. tid*E+E-1)
// to places at[0..E): all threads read, then all write.  The barrier before
// the reads also orders them after the previous field's writes.
template <uint32_t E, class T>
__device__ __forceinline__ void move_staged(T* field, const uint32_t (&at)[E], uint32_t tid) {
    T v[E];
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < E; ++j) v[j] = field[tid * E + j];
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < E; ++j) field[at[j]] = v[j];
}
template <uint32_t E, int NW>
__device__ __forceinline__ void move_staged_mask(unsigned long long (*mask)[NW], int k, const uint32_t (&at)[E],
                                                 uint32_t tid) {
    unsigned long long v[E];
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < E; ++j) v[j] = mask[tid * E + j][k];
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < E; ++j) mask[at[j]][k] = v[j];
}

// Largest i in [0, cnt) with scan[i] <= t (scan is an exclusive prefix).
__device__ __forceinline__ uint32_t find_entry(const uint32_t* scan, uint32_t cnt, uint32_t t) {
    uint32_t lo = 0, hi = cnt;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (scan[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Resolves the wavefront's queued live coins: every full group of 64 (all of
// them when `all`), one coin per lane (source id, then the discovery).  Called
// by every lane of the wavefront at the same point; the rest stays queued.
template <int NW, int BS, bool kSh>
__device__ __forceinline__ void drain_queue(const DevGraph& g, const BatchCtx<NW>& b, FusedShared<NW, BS>& s,
                                            const Ctr& ct, int nxt, uint32_t qslot, uint32_t tag, uint32_t base_tag,
                                            bool all) {
    const uint32_t wid = threadIdx.x / kWave, lane = lane_id();
    const uint32_t len = uni32(min(s.dq_len[wid], kDiscQueue));
    const uint32_t upto = all ? len : len & ~(kWave - 1);
    if (upto == 0) return;
    for (uint32_t d = 0; d < upto; d += kWave) {
        const uint32_t i = d + lane;
        if (i < upto) discover<NW, kSh>(b, ct, g.col[s.dq_e[wid][i]], (uint32_t)s.dq_c[wid][i], nxt, qslot, tag,
                                        base_tag);
    }
    const uint32_t rem = len - upto;  // fewer than 64, moved to the front
    uint32_t e = 0, c = 0;
    if (lane < rem) {
        e = s.dq_e[wid][upto + lane];
        c = s.dq_c[wid][upto + lane];
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < rem) {
        s.dq_e[wid][lane] = e;
        s.dq_c[wid][lane] = (uint16_t)c;
    }
    if (lane == 0) s.dq_len[wid] = rem;
    __builtin_amdgcn_wave_barrier();
}

// Work item t of the chunk staged in LDS (npos positions).
template <int NW, int BS, bool kSh>
__device__ __forceinline__ void run_item(const DevGraph& g, uint64_t seed, uint32_t gather_mode, const BatchCtx<NW>& b,
                                         FusedShared<NW, BS>& s, const Ctr& ct, unsigned long long s0,
                                         unsigned long long first, bool ordered, uint32_t t, uint32_t npos, int nxt,
                                         uint32_t qnext, uint32_t tag, uint32_t base_tag,
                                         uint32_t& th_philox, uint32_t& th_live) {
    const uint32_t i = find_entry(s.u.st.scan, npos, t);
    const uint32_t beg = s.u.st.beg[i], end = s.u.st.end[i];
    unsigned long long mask[NW];
    uint32_t pc = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        mask[k] = s.u.st.mask[i][k];
        pc += (uint32_t)__popcll(mask[k]);
    }
    const uint32_t qpi = item_quads(pc, s.u.st.thr[i], g.prob_layout == BPT_PROB_EDGE, gather_mode);
    const uint32_t q_first = (beg >> 2) + (t - s.u.st.scan[i]) * qpi;
    const uint32_t q_end = min(q_first + qpi, ((end - 1) >> 2) + 1);
    expand_item<NW, BS, kSh>(g, seed, gather_mode, b, s, ct, mask, s0, first, ordered, beg, end, s.u.st.thr[i],
                             q_first, q_end, nxt, qnext, tag, base_tag, th_philox, th_live);
}

// Helping: a chunk is published when it has at least kHelpMin work items; a
// unit is BS consecutive items.  claim = [63:48] chunk number, [47:20] items,
// [19:0] next unit.
constexpr uint32_t kHelpMinUnits = 4;
__device__ __forceinline__ uint32_t claim_seq(unsigned long long c) { return (uint32_t)(c >> 48); }
__device__ __forceinline__ uint32_t claim_items(unsigned long long c) { return (uint32_t)(c >> 20) & 0x0FFFFFFFu; }
__device__ __forceinline__ uint32_t claim_unit(unsigned long long c) { return (uint32_t)c & 0xFFFFFu; }
constexpr uint32_t kWaitSpins = 1u << 26;   // owner: bound of the wait for helpers (never reached)
constexpr uint32_t kPollRounds = 1u << 15;  // helper: idle polls before it gives up on a batch
constexpr uint32_t kIdleRounds = 1u << 15;  // helper: rounds without an open batch before it stops

// Writes each colour's members (ascending) from the sorted vertex list
// `list[0..T)` into the pool and clears visited[] for the listed vertices.
// With one-word masks, pass 1 keeps each listed vertex's mask at its list
// position in the slot's queue memory (2n words, idle once the traversal has
// ended) and clears it at once, so pass 2 reads the masks in list order
// instead of gathering them from the vertex records a second time.
template <int NW, int BS>
__device__ void write_sets(uint32_t* pool, const BatchCtx<NW>& b, FusedShared<NW, BS>& s, const uint32_t* list,
                           uint32_t T, bool write_ok) {
    unsigned long long* const kept = reinterpret_cast<unsigned long long*>(b.queue0);  // n entries
    constexpr int kWaves = BS / kWave;
    const uint32_t lane = lane_id();
    const uint32_t wid = threadIdx.x / kWave;
    const uint32_t nchunks = (T + kWave - 1) / kWave;
    const uint32_t per_wave = (nchunks + kWaves - 1) / kWaves;
    const uint32_t c_begin = min(nchunks, wid * per_wave);
    const uint32_t c_end = min(nchunks, c_begin + per_wave);

    // pass 1: per-colour member counts of this wave's chunk range; lane l
    // keeps the count of colour k*64 + l.
    // kB chunks per round (one-word masks), their list entries and masks loaded together
    constexpr uint32_t kB = NW == 1 ? 4 : 1;
    uint32_t mycnt[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) mycnt[k] = 0;
    for (uint32_t ch = c_begin; ch < c_end; ch += kB) {
        uint32_t u[kB];
        unsigned long long mk[kB][NW];
#pragma unroll
        for (uint32_t r = 0; r < kB; ++r) {
            const uint32_t idx = (ch + r) * kWave + lane;
            u[r] = (ch + r < c_end && idx < T) ? list[idx] : kNone;
        }
#pragma unroll
        for (uint32_t r = 0; r < kB; ++r)
#pragma unroll
            for (int k = 0; k < NW; ++k)
                mk[r][k] = (u[r] != kNone) ? load_coherent64(b.vis(u[r], k)) : 0ull;
        if constexpr (NW == 1) {
#pragma unroll
            for (uint32_t r = 0; r < kB; ++r) {
                if (u[r] != kNone) {
                    store_coherent64(&kept[(ch + r) * kWave + lane], mk[r][0]);
                    store_coherent64(b.vis(u[r], 0), 0ull);
                }
            }
        }
#pragma unroll
        for (uint32_t r = 0; r < kB; ++r) {
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                unsigned long long present = wave_or64(mk[r][k]);
                while (present) {
                    const int bpos = __ffsll((long long)present) - 1;
                    present &= present - 1;
                    const unsigned long long bal = __ballot((mk[r][k] >> bpos) & 1ull);
                    if ((int)lane == bpos) mycnt[k] += (uint32_t)__popcll(bal);
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NW; ++k) s.u.ex.wprefix[wid][k * 64 + lane] = mycnt[k];
    __syncthreads();
    for (uint32_t c = threadIdx.x; c < 64u * NW; c += BS) {
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t t = s.u.ex.wprefix[w][c];
            s.u.ex.wprefix[w][c] = run;
            run += t;
        }
    }
    __syncthreads();

    // pass 2: write, with lane l holding the next pool position of colour k*64+l
    unsigned long long run[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) run[k] = s.base + s.coff[k * 64 + lane] + s.u.ex.wprefix[wid][k * 64 + lane];
    const unsigned long long lt = lanemask_lt();
    for (uint32_t ch = c_begin; ch < c_end; ch += kB) {
        uint32_t u[kB];
        unsigned long long mk[kB][NW];
#pragma unroll
        for (uint32_t r = 0; r < kB; ++r) {
            const uint32_t idx = (ch + r) * kWave + lane;
            u[r] = (ch + r < c_end && idx < T) ? list[idx] : kNone;
        }
#pragma unroll
        for (uint32_t r = 0; r < kB; ++r)
#pragma unroll
            for (int k = 0; k < NW; ++k)
                mk[r][k] = (u[r] == kNone) ? 0ull
                           : (NW == 1)      ? load_coherent64(&kept[(ch + r) * kWave + lane])
                                            : load_coherent64(b.vis(u[r], k));
#pragma unroll
        for (uint32_t r = 0; r < kB; ++r) {
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                unsigned long long present = wave_or64(mk[r][k]);
                while (present) {
                    const int bpos = __ffsll((long long)present) - 1;
                    present &= present - 1;
                    const bool mine = (mk[r][k] >> bpos) & 1ull;
                    const unsigned long long bal = __ballot(mine);
                    const unsigned long long pos0 = bcast64(run[k], bpos);
                    if (mine && write_ok) pool[pos0 + (unsigned long long)__popcll(bal & lt)] = u[r];
                    if ((int)lane == bpos) run[k] += (unsigned long long)__popcll(bal);
                }
            }
            if (NW > 1 && u[r] != kNone) {
#pragma unroll
                for (int k = 0; k < NW; ++k) store_coherent64(b.vis(u[r], k), 0ull);
            }
        }
    }
}


// The job data of launch-wide batch bt (of job `job`), in scalar registers.
struct BatchJob {
    DevGraph g;
    uint64_t seed, first, n_samples, out_base;
    uint64_t batch;  // index within the job
    uint32_t colors;
    uint32_t flags;
    const uint32_t* order;
};

__device__ __forceinline__ BatchJob batch_job(const FusedArgs& a, uint32_t job, unsigned long long bt) {
    const FusedJob* jp = a.jobs ? a.jobs + uni32(job) : nullptr;
    BatchJob j;
    j.g.rowptr = uni_ptr(jp ? jp->g.rowptr : a.job0.g.rowptr);
    j.g.col = uni_ptr(jp ? jp->g.col : a.job0.g.col);
    j.g.thr_row = uni_ptr(jp ? jp->g.thr_row : a.job0.g.thr_row);
    j.g.thr_edge = uni_ptr(jp ? jp->g.thr_edge : a.job0.g.thr_edge);
    j.g.thr_uniform = uni32(jp ? jp->g.thr_uniform : a.job0.g.thr_uniform);
    j.g.prob_layout = uni32(jp ? jp->g.prob_layout : a.job0.g.prob_layout);
    j.g.n = uni32(jp ? jp->g.n : a.job0.g.n);
    j.g.m = uni32(jp ? jp->g.m : a.job0.g.m);
    j.seed = uni64(jp ? jp->seed : a.job0.seed);
    j.first = uni64(jp ? jp->first_sample : a.job0.first_sample);
    j.n_samples = uni64(jp ? jp->n_samples : a.job0.n_samples);
    j.out_base = uni64(jp ? jp->out_base : a.job0.out_base);
    j.colors = uni32(jp ? jp->colors : a.job0.colors);
    j.flags = uni32(jp ? jp->flags : a.job0.flags);
    j.order = uni_ptr(jp ? jp->order : a.job0.order);
    j.batch = uni64(bt) - uni64(jp ? jp->batch_begin : a.job0.batch_begin);
    return j;
}

// Once no batch is left to claim, a workgroup helps batches still running
// (one-word masks): it joins an open one (the first after its own slot),
// claims units of the chunks its owner publishes and expands them as the owner
// would, with the chunk's queue and touched counters in the help record and
// its per-colour counts in its own LDS (added to the record per unit).  It leaves when the
// batch closes and stops when every batch is finished; owners never wait for
// a helper that has not claimed work, so a helper may also give up at any
// time between claims.
template <int NW, int BS>
__device__ void help_others(const FusedArgs& a, FusedShared<NW, BS>& s, uint32_t& th_philox, uint32_t& th_live) {
    constexpr uint32_t kChunkPos = BS * ept(NW, BS);
    const uint32_t tid = threadIdx.x;
    const uint32_t grid = gridDim.x;
    uint32_t idle = 0, nap = 1;
    for (;;) {
        __syncthreads();
        if (tid == 0) {  // 0: look for an open batch, 1: stop, 2: nothing open yet
            s.pick = kNone;
            if (load_coherent64(&a.ctl->finished) >= a.n_batches || ++idle > kIdleRounds) s.cmd = 1u;
            else s.cmd = load_coherent64(&a.ctl->open) ? 0u : 2u;
        }
        __syncthreads();
        if (s.cmd == 1u) return;
        if (s.cmd == 0u) {
            for (uint32_t off = tid + 1; off < grid; off += BS) {
                if (load_coherent32(&a.ws.help[(blockIdx.x + off) % grid].state) == 1u) {
                    atomicMin(&s.pick, off);
                    break;
                }
            }
            __syncthreads();
        }
        if (s.pick == kNone) {  // back off (up to ~50 us between looks)
            for (uint32_t i = 0; i < nap; ++i) __builtin_amdgcn_s_sleep(127);
            nap = min(2u * nap, 16u);
            continue;
        }
        nap = 1;
        const uint32_t h = (blockIdx.x + s.pick) % grid;
        HelpRec* const hr = a.ws.help + h;
        if (tid == 0) {
            s.batch = load_coherent64(&hr->batch);
            s.job = load_coherent32(&hr->job);
        }
        __syncthreads();
        if (s.batch >= a.n_batches || (a.jobs && s.job >= a.n_jobs)) continue;
        const BatchJob jb = batch_job(a, s.job, s.batch);
        BatchCtx<NW> b = slot_ctx<NW>(a, h);
        b.n = jb.g.n;
        b.read_first = (jb.flags & kJobReadFirst) != 0;
        const unsigned long long s0 = jb.first + jb.batch * jb.colors;
        const Ctr ct{hr->qlen, &hr->tlen, s.cnt};  // colour counts kept here, added to hr->cnt per unit
        for (uint32_t c = tid; c < 64u; c += BS) s.cnt[c] = 0u;
        const uint32_t* stage = a.ws.hstage + (size_t)h * kHelpStagePos * 6;
        uint32_t have = 0, spent = 0, polls = 0, wait = 1;  // staged chunk; exhausted chunk (thread 0)
        for (;;) {
            if (tid == 0) {
                uint32_t cmd = 0;  // 0: wait, 1: leave, 2: expand the claimed unit
                unsigned long long r = 0;
                if (load_coherent32(&hr->state) != 1u) {
                    cmd = 1;
                } else {
                    const unsigned long long c = load_coherent64(&hr->claim);
                    if (claim_seq(c) != 0 && claim_seq(c) != spent &&
                        (unsigned long long)claim_unit(c) * BS < claim_items(c)) {
                        r = atomicAdd(&hr->claim, 1ull);
                        if ((unsigned long long)claim_unit(r) * BS < claim_items(r)) cmd = 2;
                        else spent = claim_seq(r);
                    }
                }
                s.cmd = cmd;
                s.claimed = r;
            }
            __syncthreads();
            const uint32_t cmd = s.cmd;
            const unsigned long long r = s.claimed;
            __syncthreads();
            if (cmd == 1) break;
            if (cmd == 0) {  // the owner has not published its next chunk yet
                if (++polls > kPollRounds) break;
                for (uint32_t i = 0; i < wait; ++i) __builtin_amdgcn_s_sleep(16);
                wait = min(2u * wait, 8u);
                continue;
            }
            polls = 0;
            wait = 1;
            if (claim_seq(r) != have) {  // the chunk's staging: valid while our unit is unfinished
                if (tid == 0) {
                    s.h_npos = min(load_coherent32(&hr->npos), kChunkPos);
                    s.h_nxt = load_coherent32(&hr->nxt);
                    s.h_qnext = load_coherent32(&hr->qnext);
                }
                __syncthreads();
                const uint32_t npos = s.h_npos;
                for (uint32_t p = tid; p < npos; p += BS) {
                    s.u.st.scan[p] = load_coherent32(stage + p);
                    const uint32_t end = min(load_coherent32(stage + 2 * kHelpStagePos + p), jb.g.m);
                    s.u.st.beg[p] = min(load_coherent32(stage + kHelpStagePos + p), end);
                    s.u.st.end[p] = end;
                    s.u.st.thr[p] = load_coherent32(stage + 3 * kHelpStagePos + p);
                    s.u.st.mask[p][0] = (unsigned long long)load_coherent32(stage + 4 * kHelpStagePos + p) |
                                        ((unsigned long long)load_coherent32(stage + 5 * kHelpStagePos + p) << 32);
                }
                __syncthreads();
                have = claim_seq(r);
            }
            const uint32_t total = claim_items(r), unit = claim_unit(r);
            const uint32_t t = unit * BS + tid;
            if (t < total)
                run_item<NW, BS, true>(jb.g, jb.seed, a.gather_mode, b, s, ct, s0, jb.first, false, t, s.h_npos,
                                       (int)s.h_nxt, s.h_qnext, 0u, 0u, th_philox, th_live);
            drain_queue<NW, BS, true>(jb.g, b, s, ct, (int)s.h_nxt, s.h_qnext, 0u, 0u, true);
            if (th_philox >= 0x80000000u || th_live >= 0x80000000u) {
                atomicAdd(&s.stats[kStatPhilox], (unsigned long long)th_philox);
                atomicAdd(&s.stats[kStatLive], (unsigned long long)th_live);
                th_philox = th_live = 0;
            }
            wait_own_memory_ops();  // discoveries and queue entries performed before they are counted
            __syncthreads();
            for (uint32_t c = tid; c < 64u; c += BS) {
                if (s.cnt[c]) atomicAdd(&hr->cnt[c], s.cnt[c]);
                s.cnt[c] = 0u;
            }
            wait_own_memory_ops();
            __syncthreads();
            if (tid == 0) atomicAdd(&hr->done, min((uint32_t)BS, total - unit * BS));
        }
    }
}

// kHelp: the instantiation with helping (one-word masks only).  Kept apart
// because its extra state costs the plain traversal registers.
template <int NW, int BS, bool kHelp>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4))) void fused_bpt_kernel(FusedArgs a) {
    __shared__ FusedShared<NW, BS> s;
    constexpr uint32_t kSortCap = sort_cap(BS);
    const uint32_t tid = threadIdx.x;
    const uint32_t slot = blockIdx.x;
    constexpr uint32_t C = 64u * NW;
    BatchCtx<NW> b = slot_ctx<NW>(a, slot);
    HelpRec* const hr = (kHelp && NW == 1 && a.ws.help) ? a.ws.help + slot : nullptr;

    if (tid < kNumStats) s.stats[tid] = 0;
    if (tid < BS / kWave) s.dq_len[tid] = 0;
    if (tid < kColourBuckets) s.bcnt[tid] = 0;
    if (tid == 0) {
        s.tail = 0;
        s.probes = 0;
    }
    uint32_t th_philox = 0, th_live = 0;  // moved into s.stats before they could overflow

    for (;;) {
        __syncthreads();
        if (tid == 0) {
            const unsigned long long bt = atomicAdd(&a.ctl->work_counter, 1ull);
            uint32_t j = 0;
            if (a.jobs && bt < a.n_batches) {  // the last job whose first batch is <= bt
                uint32_t lo = 0, hi = a.n_jobs;
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (a.jobs[mid].batch_begin <= bt) lo = mid;
                    else hi = mid;
                }
                j = lo;
            }
            s.batch = bt;
            s.job = j;
        }
        __syncthreads();
        if (s.batch >= a.n_batches) break;
        // the batch's job, in scalar registers
        const BatchJob jb = batch_job(a, s.job, s.batch);
        const DevGraph& g = jb.g;
        const uint64_t seed = jb.seed;
        const uint64_t first = jb.first;
        const uint64_t n_samples = jb.n_samples;
        const uint64_t out_base = jb.out_base;
        const uint32_t colors = jb.colors;
        const uint32_t* order = jb.order;
        const bool ordered = order != nullptr;
        const uint64_t batch = jb.batch;
        const uint32_t n = g.n;
        const uint32_t layout = g.prob_layout;
        const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
        b.n = n;
        b.read_first = (jb.flags & kJobReadFirst) != 0;
        // samples s0 .. s0 + ncol - 1 take colours 0 .. ncol - 1 (colors <= C per batch)
        const uint64_t s0 = first + batch * colors;
        const uint32_t ncol = (uint32_t)min((uint64_t)colors, n_samples - batch * colors);

        uint32_t base_tag = 0;
        if constexpr (NW > 1) {
            base_tag = a.ws.slot_tag[slot] + 1;
            if (base_tag > 0xFFFFFFFFu - a.n_max - 8u) {  // tags would wrap: restart them
                for (uint32_t v = tid; v < a.n_max; v += BS) store_coherent(&b.stamp[v], 0u);
                wait_own_memory_ops();
                __syncthreads();
                base_tag = 1;
            }
        }
        for (uint32_t c = tid; c < C; c += BS) s.cnt[c] = 0;
        if (ordered)
            for (uint32_t c = tid; c < ncol; c += BS) s.cidx[c] = order[batch * colors + c];
        if (tid == 0) {
            s.qlen[0] = 0;
            s.qlen[1] = 0;
            s.qlen[2] = 0;
            s.tlen = 0;
        }
        __syncthreads();

        // Frontier initialisation: colour c starts at its sample's start vertex.
        const Ctr ct_own{s.qlen, &s.tlen, s.cnt};
        for (uint32_t c = tid; c < ncol; c += BS)
            discover<NW, false>(b, ct_own, start_of(ordered ? first + s.cidx[c] : s0 + c, n, k0, k1), c, 0, 0,
                                base_tag, base_tag);

        // Helping: once half the workgroups have no batch left, a heavy chunk of this
        // batch is published and idle workgroups expand units of it.  An open batch
        // writes queue and touched entries coherently; its queue and touched
        // counters move to `hr` for the duration of each published chunk.
        const bool help_ok = kHelp && hr != nullptr && !ordered;
        bool shared = false;
        uint32_t hseq = 0;

        // Level-synchronous fused traversal.
        uint32_t level = 0, scan_buf = 0;
        for (;;) {
            __syncthreads();  // every discovery of the previous level is done
            const uint32_t qcur = level % 3, qnext = (level + 1) % 3;
            const uint32_t F = min(s.qlen[qcur], n);
            if (F == 0) break;
            if (level > n) {
                if (tid == 0) atomicOr(&a.ctl->err, (unsigned)kErrLevelBound);
                break;
            }
            if (tid == 0) s.qlen[(level + 2) % 3] = 0;  // used next by level L+1's discoveries
            const int cur = level & 1, nxt = cur ^ 1;
            const uint32_t tag = base_tag + level + 1;
            const uint32_t* qcur_arr = cur ? b.queue1 : b.queue0;

            constexpr uint32_t kEPT = ept(NW, BS);
            constexpr uint32_t kChunk = BS * kEPT;
            for (uint32_t c0 = 0; c0 < F; c0 += kChunk) {
                const uint32_t cnt = min(kChunk, F - c0);
                // Thread tid stages the chunk's queue entries tid, tid + BS, ... into LDS
                // positions tid*kEPT + j (queue order carries no meaning), so a level
                // smaller than the workgroup costs every thread at most one entry, and it
                // issues all of their loads before using any result.
                const uint32_t npos = min((uint32_t)BS, cnt) * kEPT;  // LDS positions in use
                uint32_t vq[kEPT];
#pragma unroll
                for (uint32_t j = 0; j < kEPT; ++j) {
                    const uint32_t e = j * BS + tid;
                    vq[j] = e < cnt ? (shared ? min(load_coherent32(&qcur_arr[c0 + e]), n - 1) : qcur_arr[c0 + e]) : 0u;
                }
                uint32_t rb[kEPT], re[kEPT], rt[kEPT];
                unsigned long long mk[kEPT][NW];
#pragma unroll
                for (uint32_t j = 0; j < kEPT; ++j) {
                    const bool ok = j * BS + tid < cnt;
                    rb[j] = g.rowptr[vq[j]];
                    re[j] = g.rowptr[vq[j] + 1];
                    rt[j] = layout == BPT_PROB_ROW ? g.thr_row[vq[j]]
                                                   : (layout == BPT_PROB_UNIFORM ? g.thr_uniform : 0u);
#pragma unroll
                    for (int k = 0; k < NW; ++k)
                        mk[j][k] = ok ? atomicExch(b.fr(cur, vq[j], k), 0ull) : 0ull;
                }
                uint32_t my_items[kEPT], my_pc[kEPT];
                uint32_t items = 0;
                unsigned long long ch_entries = 0, ch_ea = 0, ch_te = 0, ch_members = 0;
#pragma unroll
                for (uint32_t j = 0; j < kEPT; ++j) {
                    const uint32_t pos = tid * kEPT + j;
                    const bool ok = j * BS + tid < cnt;
                    uint32_t pc = 0;
#pragma unroll
                    for (int k = 0; k < NW; ++k) {
                        s.u.st.mask[pos][k] = mk[j][k];
                        pc += (uint32_t)__popcll(mk[j][k]);
                    }
                    const uint32_t beg = rb[j], end = re[j], deg = end - beg;
                    const bool never = (layout != BPT_PROB_EDGE) && rt[j] == 0;
                    const uint32_t quads =
                        (!ok || deg == 0 || never || pc == 0) ? 0u : ((end - 1) >> 2) - (beg >> 2) + 1;
                    my_items[j] = item_quads(pc, rt[j], layout == BPT_PROB_EDGE, a.gather_mode) == 4u
                                      ? (quads + 3) >> 2
                                      : (quads + kQuadsPerItem - 1) / kQuadsPerItem;
                    my_pc[j] = my_items[j] ? pc : 0u;
                    items += my_items[j];
                    s.u.st.beg[pos] = beg;
                    s.u.st.end[pos] = end;
                    s.u.st.thr[pos] = rt[j];
                    if (ok) {
                        ch_entries += 1;
                        ch_ea += deg;
                        ch_te += (unsigned long long)pc * deg;
                        ch_members += pc;
                    }
                }
                // Chunks of at least BS entries (every position holds one) are regrouped by
                // colour count: each entry takes a place in its bucket (an LDS atomic; the
                // order within a bucket carries no meaning), then the staged fields move
                // there one at a time, each read by all threads before any is overwritten.
                const bool by_colours = cnt >= (uint32_t)BS;
                if (by_colours) {
                    uint32_t at[kEPT];
#pragma unroll
                    for (uint32_t j = 0; j < kEPT; ++j) {
                        my_pc[j] = colour_bucket(my_pc[j]);
                        at[j] = atomicAdd(&s.bcnt[my_pc[j]], 1u);
                    }
                    __syncthreads();  // bucket sizes complete
                    if (tid == 0) {
                        uint32_t run = 0;
                        for (uint32_t bb = 0; bb < kColourBuckets; ++bb) {
                            s.bbase[bb] = run;
                            run += s.bcnt[bb];
                            s.bcnt[bb] = 0;
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (uint32_t j = 0; j < kEPT; ++j) {
                        at[j] += s.bbase[my_pc[j]];
                        s.u.st.scan[at[j]] = my_items[j];  // item count, until the scan below
                    }
                    move_staged(s.u.st.beg, at, tid);
                    move_staged(s.u.st.end, at, tid);
                    move_staged(s.u.st.thr, at, tid);
#pragma unroll
                    for (int k = 0; k < NW; ++k) move_staged_mask(s.u.st.mask, k, at, tid);
                    __syncthreads();
                    items = 0;
#pragma unroll
                    for (uint32_t j = 0; j < kEPT; ++j) {  // the items of the entries now at this thread's places
                        my_items[j] = s.u.st.scan[tid * kEPT + j];
                        items += my_items[j];
                    }
                }
                // the chunk's staging counters, one LDS update per wavefront
                ch_entries = wave_sum64(ch_entries);
                ch_ea = wave_sum64(ch_ea);
                ch_te = wave_sum64(ch_te);
                ch_members = wave_sum64(ch_members);
                if (lane_id() == 0) {
                    atomicAdd(&s.stats[kStatEntries], ch_entries);
                    atomicAdd(&s.stats[kStatEdgeAccesses], ch_ea);
                    atomicAdd(&s.stats[kStatSampleEdges], ch_te);
                    atomicAdd(&s.stats[kStatMembers], ch_members);
                }
                uint32_t total;
                uint32_t excl = block_excl_scan<BS>(items, s.scan_tmp[scan_buf], &total);
                scan_buf ^= 1u;
#pragma unroll
                for (uint32_t j = 0; j < kEPT; ++j) {
                    s.u.st.scan[tid * kEPT + j] = excl;
                    excl += my_items[j];
                }
                if (tid == 0) s.next_item = 0;
                __syncthreads();

                const bool heavy = help_ok && total >= kHelpMinUnits * BS;
                if (heavy && !shared) {  // are half the workgroups idle? (asked at every 8th heavy chunk)
                    if (tid == 0) {
                        if (!s.tail && (++s.probes & 7u) == 0u &&
                            2 * (a.n_batches - load_coherent64(&a.ctl->finished)) <= gridDim.x)
                            s.tail = 1u;
                        s.go = s.tail;
                    }
                    __syncthreads();
                    if (s.go) {  // open the batch to helpers
                        if (tid == 0) __threadfence();  // queue and touched entries so far become device-visible
                        for (uint32_t c = tid; c < 64u; c += BS) store_coherent(&hr->cnt[c], 0u);  // helpers' counts
                        if (tid == 0) {
                            store_coherent64(&hr->batch, s.batch);
                            store_coherent(&hr->job, s.job);
                            store_coherent(&hr->done, 0u);
                            store_coherent64(&hr->claim, 0ull);
                        }
                        wait_own_memory_ops();
                        __syncthreads();
                        if (tid == 0) {
                            store_coherent(&hr->state, 1u);
                            atomicAdd(&a.ctl->open, 1ull);
                        }
                        shared = true;
                    }
                }

                // Heavy expansion levels are compute-bound while light ones wait on
                // memory: give the heavy ones issue priority on their SIMDs.
                set_wave_priority(total >= 8u * BS ? 3 : (total >= 2u * BS ? 2 : (total >= BS / 2 ? 1 : 0)));
                if (shared && heavy) {
                    // publish the chunk, then claim units of it along with the helpers
                    uint32_t* stage = a.ws.hstage + (size_t)slot * kHelpStagePos * 6;
                    for (uint32_t p = tid; p < npos; p += BS) {
                        store_coherent(stage + p, s.u.st.scan[p]);
                        store_coherent(stage + kHelpStagePos + p, s.u.st.beg[p]);
                        store_coherent(stage + 2 * kHelpStagePos + p, s.u.st.end[p]);
                        store_coherent(stage + 3 * kHelpStagePos + p, s.u.st.thr[p]);
                        const unsigned long long m = s.u.st.mask[p][0];
                        store_coherent(stage + 4 * kHelpStagePos + p, (uint32_t)m);
                        store_coherent(stage + 5 * kHelpStagePos + p, (uint32_t)(m >> 32));
                    }
                    if (tid == 0) {  // the queue and touched counters move to the record for this chunk
                        store_coherent(&hr->qlen[qnext], s.qlen[qnext]);
                        store_coherent(&hr->tlen, s.tlen);
                        store_coherent(&hr->npos, npos);
                        store_coherent(&hr->nxt, (uint32_t)nxt);
                        store_coherent(&hr->qnext, qnext);
                        store_coherent(&hr->done, 0u);
                    }
                    wait_own_memory_ops();
                    __syncthreads();
                    ++hseq;
                    if (tid == 0)
                        atomicExch(&hr->claim, ((unsigned long long)hseq << 48) | ((unsigned long long)total << 20));
                    uint32_t mine = 0;
                    for (;;) {
                        if (tid == 0) s.unit = claim_unit(atomicAdd(&hr->claim, 1ull));
                        __syncthreads();
                        const uint32_t unit = s.unit;
                        __syncthreads();
                        if ((unsigned long long)unit * BS >= total) break;
                        const uint32_t t = unit * BS + tid;
                        const Ctr ct_help{hr->qlen, &hr->tlen, s.cnt};
                        if (t < total)
                            run_item<NW, BS, true>(g, seed, a.gather_mode, b, s, ct_help, s0, first, ordered, t, npos,
                                                   nxt, qnext, tag, base_tag, th_philox, th_live);
                        drain_queue<NW, BS, true>(g, b, s, ct_help, nxt, qnext, tag, base_tag, false);
                        mine += min((uint32_t)BS, total - unit * BS);
                    }
                    drain_queue<NW, BS, true>(g, b, s, Ctr{hr->qlen, &hr->tlen, s.cnt}, nxt, qnext, tag, base_tag,
                                              true);
                    wait_own_memory_ops();
                    __syncthreads();
                    if (tid == 0) {  // wait for the units helpers claimed
                        atomicAdd(&hr->done, mine);
                        uint32_t spins = 0;
                        while (load_coherent32(&hr->done) < total) {
                            if (++spins > kWaitSpins) {
                                atomicOr(&a.ctl->err, (unsigned)kErrHelpTimeout);
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                        }
                        s.qlen[qnext] = load_coherent32(&hr->qlen[qnext]);  // back to LDS
                        s.tlen = load_coherent32(&hr->tlen);
                    }
                } else if (shared) {  // alone, counters in LDS, entries written coherently
                    for (uint32_t t0 = 0; t0 < total; t0 += BS) {
                        if (t0 + tid < total)
                            run_item<NW, BS, true>(g, seed, a.gather_mode, b, s, ct_own, s0, first, ordered, t0 + tid,
                                                   npos, nxt, qnext, tag, base_tag, th_philox, th_live);
                        drain_queue<NW, BS, true>(g, b, s, ct_own, nxt, qnext, tag, base_tag, false);
                    }
                    drain_queue<NW, BS, true>(g, b, s, ct_own, nxt, qnext, tag, base_tag, true);
                } else {
                    // wavefronts claim 64 consecutive items at a time, so a wavefront slowed
                    // by its SIMD's other work takes fewer of them
                    for (;;) {
                        uint32_t t0 = 0;
                        if (lane_id() == 0) t0 = atomicAdd(&s.next_item, (uint32_t)kWave);
                        t0 = uni32(__shfl(t0, 0, kWave));
                        if (t0 >= total) break;
                        if (t0 + lane_id() < total)
                            run_item<NW, BS, false>(g, seed, a.gather_mode, b, s, ct_own, s0, first, ordered,
                                                    t0 + lane_id(), npos, nxt, qnext, tag, base_tag, th_philox,
                                                    th_live);
                        drain_queue<NW, BS, false>(g, b, s, ct_own, nxt, qnext, tag, base_tag, false);
                    }
                    drain_queue<NW, BS, false>(g, b, s, ct_own, nxt, qnext, tag, base_tag, true);
                }
                set_wave_priority(0);
                if (th_philox >= 0x80000000u || th_live >= 0x80000000u) {
                    atomicAdd(&s.stats[kStatPhilox], (unsigned long long)th_philox);
                    atomicAdd(&s.stats[kStatLive], (unsigned long long)th_live);
                    th_philox = th_live = 0;
                }
                if (c0 + kChunk < F) __syncthreads();  // the next chunk reuses the staging area
            }

            ++level;
        }

        if (shared) {  // closed to helpers (none holds work); their colour counts join ours
            if (tid == 0) {
                store_coherent(&hr->state, 0u);
                atomicSub(&a.ctl->open, 1ull);
            }
            for (uint32_t c = tid; c < 64u; c += BS) s.cnt[c] += load_coherent32(&hr->cnt[c]);
        }

        // ---- RRR set extraction (Listing 1's final loop) ----
        wait_own_memory_ops();  // this workgroup's last atomics have been performed
        __syncthreads();
        const uint32_t T = min(s.tlen, n);
        if (tid == 0) {
            unsigned long long run = 0;
            for (uint32_t c = 0; c < C; ++c) {
                s.coff[c] = run;
                run += s.cnt[c];
            }
            s.base = atomicAdd(&a.ctl->pool_cursor, run);
            if (s.base + run > a.out.pool_cap) atomicOr(&a.ctl->err, (unsigned)kErrPoolOverflow);
            if constexpr (NW > 1) a.ws.slot_tag[slot] = base_tag + level + 1;
            atomicAdd(&s.stats[kStatLevels], (unsigned long long)level);
            atomicMax(&s.stats[kStatMaxLevels], (unsigned long long)level);
            atomicAdd(&s.stats[kStatBatches], 1ull);
        }
        __syncthreads();
        const bool write_ok = s.base + s.coff[C - 1] + s.cnt[C - 1] <= a.out.pool_cap;
        for (uint32_t c = tid; c < ncol; c += BS) {
            const uint64_t si = ordered ? (uint64_t)s.cidx[c] : (s0 - first) + c;  // the sample's output slot
            a.out.counts[out_base + si] = s.cnt[c];
            a.out.where[out_base + si] = s.base + s.coff[c];
        }

        const uint32_t* list;
        if (T <= kSortCap) {
            uint32_t P = 64;
            while (P < T) P <<= 1;
            for (uint32_t i = tid; i < P; i += BS)
                s.u.ex.sorted[i] = i < T ? (shared ? load_coherent32(&b.touched[i]) : b.touched[i]) : kNone;
            __syncthreads();
            for (uint32_t k = 2; k <= P; k <<= 1) {
                for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                    for (uint32_t i = tid; i < P; i += BS) {
                        const uint32_t ixj = i ^ j;
                        if (ixj > i) {
                            const uint32_t x = s.u.ex.sorted[i], y = s.u.ex.sorted[ixj];
                            const bool up = (i & k) == 0;
                            if ((x > y) == up) {
                                s.u.ex.sorted[i] = y;
                                s.u.ex.sorted[ixj] = x;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            for (uint32_t i = tid; i < T; i += BS) store_coherent64(&b.tbits[s.u.ex.sorted[i] >> 6], 0ull);
            list = s.u.ex.sorted;
        } else {
            // touched-vertex bitmap, scanned in vertex order, gives the sorted list
            const size_t words = bitmap_words(n);
            const size_t per_t = (words + BS - 1) / BS;
            const size_t w0 = min(words, (size_t)tid * per_t), w1 = min(words, w0 + per_t);
            // eight words per round, their loads issued together
            constexpr uint32_t kR = 8;
            uint32_t ones = 0;
            for (size_t w = w0; w < w1; w += kR) {
                unsigned long long x[kR];
#pragma unroll
                for (uint32_t r = 0; r < kR; ++r) x[r] = w + r < w1 ? load_coherent64(&b.tbits[w + r]) : 0ull;
#pragma unroll
                for (uint32_t r = 0; r < kR; ++r) ones += (uint32_t)__popcll(x[r]);
            }
            uint32_t all;
            uint32_t pos = block_excl_scan<BS>(ones, s.scan_tmp[scan_buf], &all);
            for (size_t w = w0; w < w1; w += kR) {
                unsigned long long x[kR];
#pragma unroll
                for (uint32_t r = 0; r < kR; ++r) x[r] = w + r < w1 ? load_coherent64(&b.tbits[w + r]) : 0ull;
#pragma unroll
                for (uint32_t r = 0; r < kR; ++r) {
                    if (!x[r]) continue;
                    store_coherent64(&b.tbits[w + r], 0ull);
                    while (x[r]) {
                        const uint32_t bpos = (uint32_t)(__ffsll((long long)x[r]) - 1);
                        x[r] &= x[r] - 1;
                        if (pos < n) b.touched[pos] = (uint32_t)((w + r) * 64 + bpos);
                        ++pos;
                    }
                }
            }
            __syncthreads();
            list = b.touched;
        }
        __syncthreads();
        write_sets<NW, BS>(a.out.pool, b, s, list, T, write_ok);
        wait_own_memory_ops();  // the slot's resets have been performed before it is reused
        if (tid == 0) atomicAdd(&a.ctl->finished, 1ull);
    }
    if constexpr (kHelp && NW == 1) {
        if (a.ws.help) help_others<NW, BS>(a, s, th_philox, th_live);
    }

    // thread-local counters into the workgroup's totals, then the call's
    atomicAdd(&s.stats[kStatPhilox], (unsigned long long)th_philox);
    atomicAdd(&s.stats[kStatLive], (unsigned long long)th_live);
    __syncthreads();
    if (tid < kNumStats) {
        if (tid == kStatMaxLevels) atomicMax(&a.ctl->stats[tid], s.stats[tid]);
        else atomicAdd(&a.ctl->stats[tid], s.stats[tid]);
    }
}

}  // namespace

hipError_t launch_fused(const FusedArgs& a, int nw, int block, int grid, bool help, hipStream_t stream) {
#define BPT_LAUNCH(NW_, BS_) \
    hipLaunchKernelGGL((fused_bpt_kernel<NW_, BS_, false>), dim3(grid), dim3(BS_), 0, stream, a)
#define BPT_LAUNCH1(BS_)                                                                                        \
    if (help && a.ws.help)                                                                                      \
        hipLaunchKernelGGL((fused_bpt_kernel<1, BS_, true>), dim3(grid), dim3(BS_), 0, stream, a);            \
    else                                                                                                        \
        hipLaunchKernelGGL((fused_bpt_kernel<1, BS_, false>), dim3(grid), dim3(BS_), 0, stream, a)
    if (block == 128) {
        switch (nw) {
            case 1: BPT_LAUNCH1(128); break;
            case 2: BPT_LAUNCH(2, 128); break;
            case 4: BPT_LAUNCH(4, 128); break;
            case 8: BPT_LAUNCH(8, 128); break;
            case 16: BPT_LAUNCH(16, 128); break;
            default: return hipErrorInvalidValue;
        }
    } else if (block == 256) {
        switch (nw) {
            case 1: BPT_LAUNCH1(256); break;
            case 2: BPT_LAUNCH(2, 256); break;
            case 4: BPT_LAUNCH(4, 256); break;
            case 8: BPT_LAUNCH(8, 256); break;
            case 16: BPT_LAUNCH(16, 256); break;
            default: return hipErrorInvalidValue;
        }
    } else if (block == 512) {
        switch (nw) {
            case 1: BPT_LAUNCH1(512); break;
            case 2: BPT_LAUNCH(2, 512); break;
            case 4: BPT_LAUNCH(4, 512); break;
            default: return hipErrorInvalidValue;
        }
    } else if (block == 1024) {
        switch (nw) {
            case 1: BPT_LAUNCH1(1024); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;
    }
#undef BPT_LAUNCH
#undef BPT_LAUNCH1
    return hipGetLastError();
}

}  // namespace bpt
