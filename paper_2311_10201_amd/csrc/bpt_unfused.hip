// Unfused breadth-first probabilistic traversals: one traversal per sample,
// the baseline the paper compares fused BPTs against (Section 4.1 describes
// gIM's unfused kernel: one traversal per thread block, frontier vertices
// processed one after another with their edges spread over the block's
// threads, one visited bit per vertex).
//
// Here each wavefront owns a private visited bitmap and a visit log and runs
// one sample at a time, claimed from a device counter.  Within a level the
// frontier's (vertex, 4-edge quad) work items are spread evenly over the 64
// lanes, so low-degree vertices do not leave lanes idle; each item evaluates
// one Philox block, i.e. the coins of four consecutive in-edges.  The visit
// log, read level by level, is the BFS queue; at the end it is sorted (in LDS
// when short, by a bitmap scan otherwise) into the RRR set.
#include "bpt.h"
#include "bpt_internal.hpp"
#include "bpt_rng.hpp"

namespace bpt {

namespace {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = kUnfusedBlock / kWave;
constexpr uint32_t kWaveSortCap = 1024;
constexpr uint32_t kNone = 0xFFFFFFFFu;

struct WaveShared {
    uint32_t beg[kWave];
    uint32_t end[kWave];
    uint32_t thr[kWave];
    uint32_t scan[kWave];
    uint32_t sorted[kWaveSortCap];
    uint32_t tail;
};

// The visited bitmap is written by atomics; it is read and cleared with
// agent-scope (device-coherent) loads and stores, so no L2-wide fence is needed.
__device__ __forceinline__ unsigned long long load_coherent64(const unsigned long long* p) {
    return __hip_atomic_load(const_cast<unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_coherent64(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, uint32_t lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, kWave);
        if (lane >= (uint32_t)d) x += y;
    }
    return x;
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long x) {
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t olo = __shfl_xor(lo, d, kWave), ohi = __shfl_xor(hi, d, kWave);
        const uint32_t nlo = lo + olo;
        hi = hi + ohi + (nlo < lo ? 1u : 0u);
        lo = nlo;
    }
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t find_entry(const uint32_t* scan, uint32_t cnt, uint32_t t) {
    uint32_t lo = 0, hi = cnt;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (scan[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kUnfusedBlock) void unfused_bpt_kernel(UnfusedArgs a) {
    __shared__ WaveShared shm[kWavesPerBlock];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wid = threadIdx.x / kWave;
    WaveShared& w = shm[wid];
    const uint32_t n = a.g.n;
    const size_t words = bitmap_words(n);
    const size_t slot = (size_t)blockIdx.x * kWavesPerBlock + wid;
    unsigned long long* vbits = a.ws.vbits + slot * words;
    uint32_t* log = a.ws.log + slot * n;
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const uint32_t layout = a.g.prob_layout;

    unsigned long long st_members = 0, st_ea = 0, st_philox = 0, st_live = 0, st_levels = 0, st_maxlev = 0,
                       st_runs = 0;

    for (;;) {
        unsigned long long got = 0;
        if (lane == 0) got = atomicAdd(&a.ctl->work_counter, 1ull);
        got = ((unsigned long long)__shfl((uint32_t)(got >> 32), 0, kWave) << 32) | __shfl((uint32_t)got, 0, kWave);
        if ((uint64_t)got >= a.n_samples) break;
        const uint64_t s = a.first_sample + got;

        const uint32_t start = start_of(s, n, k0, k1);
        if (lane == 0) {
            atomicOr(&vbits[start >> 6], 1ull << (start & 63));
            log[0] = start;
            w.tail = 1;
        }
        __threadfence_block();
        wave_sync();

        uint32_t lb = 0, le = 1, level = 0;
        while (lb < le) {
            for (uint32_t c0 = lb; c0 < le; c0 += kWave) {
                const uint32_t cnt = min((uint32_t)kWave, le - c0);
                uint32_t items = 0;
                if (lane < cnt) {
                    const uint32_t v = log[c0 + lane];
                    const uint32_t beg = a.g.rowptr[v], end = a.g.rowptr[v + 1];
                    uint32_t thr = 0;
                    if (layout == BPT_PROB_ROW) thr = a.g.thr_row[v];
                    else if (layout == BPT_PROB_UNIFORM) thr = a.g.thr_uniform;
                    const bool never = (layout != BPT_PROB_EDGE) && thr == 0;
                    items = (end == beg || never) ? 0u : ((end - 1) >> 2) - (beg >> 2) + 1;
                    w.beg[lane] = beg;
                    w.end[lane] = end;
                    w.thr[lane] = thr;
                    st_ea += end - beg;
                }
                const uint32_t incl = wave_incl_scan(items, lane);
                const uint32_t total = __shfl(incl, kWave - 1, kWave);
                if (lane < cnt) w.scan[lane] = incl - items;
                wave_sync();
                for (uint32_t t = lane; t < total; t += kWave) {
                    const uint32_t i = find_entry(w.scan, cnt, t);
                    const uint32_t beg = w.beg[i], end = w.end[i];
                    const uint32_t quad = (beg >> 2) + (t - w.scan[i]);
                    const uint32_t e0 = quad << 2;
                    uint32_t t0, t1, t2, t3;
                    if (layout == BPT_PROB_EDGE) {
                        const uint4 tt = *reinterpret_cast<const uint4*>(a.g.thr_edge + e0);
                        t0 = tt.x; t1 = tt.y; t2 = tt.z; t3 = tt.w;
                    } else {
                        t0 = t1 = t2 = t3 = w.thr[i];
                    }
                    uint32_t valid = 0xFu;
                    if (e0 < beg) valid &= 0xFu << (beg - e0);
                    if (end - e0 < 4) valid &= (1u << (end - e0)) - 1u;
                    const Block4 r = coin_block(quad, s, k0, k1);
                    ++st_philox;
                    uint32_t live = (coin_live(r.w0, t0) ? 1u : 0u) | (coin_live(r.w1, t1) ? 2u : 0u) |
                                    (coin_live(r.w2, t2) ? 4u : 0u) | (coin_live(r.w3, t3) ? 8u : 0u);
                    live &= valid;
                    while (live) {
                        const uint32_t j = (uint32_t)(__ffs((int)live) - 1);
                        live &= live - 1;
                        ++st_live;
                        const uint32_t u = a.g.col[e0 + j];
                        const unsigned long long bit = 1ull << (u & 63);
                        if (!(atomicOr(&vbits[u >> 6], bit) & bit)) {
                            const uint32_t pos = atomicAdd(&w.tail, 1u);
                            if (pos < n) log[pos] = u;
                            else atomicOr(&a.ctl->err, (unsigned)kErrQueueOverflow);
                        }
                    }
                }
                wave_sync();
            }
            __threadfence_block();
            wave_sync();
            lb = le;
            le = min(w.tail, n);
            ++level;
            if (level > n + 1) {
                if (lane == 0) atomicOr(&a.ctl->err, (unsigned)kErrLevelBound);
                break;
            }
        }
        const uint32_t T = le;

        // ---- the RRR set: sorted visit log ----
        unsigned long long base = 0;
        if (lane == 0) {
            base = atomicAdd(&a.ctl->pool_cursor, (unsigned long long)T);
            if (base + T > a.out.pool_cap) atomicOr(&a.ctl->err, (unsigned)kErrPoolOverflow);
            a.out.counts[got] = T;
            a.out.where[got] = base;
        }
        base = ((unsigned long long)__shfl((uint32_t)(base >> 32), 0, kWave) << 32) |
               __shfl((uint32_t)base, 0, kWave);
        const bool write_ok = base + T <= a.out.pool_cap;
        __builtin_amdgcn_s_waitcnt(0);  // this wave's bitmap atomics have been performed
        if (T <= kWaveSortCap) {
            uint32_t P = kWave;
            while (P < T) P <<= 1;
            for (uint32_t i = lane; i < P; i += kWave) w.sorted[i] = i < T ? log[i] : kNone;
            wave_sync();
            for (uint32_t k = 2; k <= P; k <<= 1) {
                for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                    for (uint32_t i = lane; i < P; i += kWave) {
                        const uint32_t ixj = i ^ j;
                        if (ixj > i) {
                            const uint32_t x = w.sorted[i], y = w.sorted[ixj];
                            if ((x > y) == ((i & k) == 0)) {
                                w.sorted[i] = y;
                                w.sorted[ixj] = x;
                            }
                        }
                    }
                    wave_sync();
                }
            }
            for (uint32_t i = lane; i < T; i += kWave) {
                const uint32_t u = w.sorted[i];
                if (write_ok) a.out.pool[base + i] = u;
                store_coherent64(&vbits[u >> 6], 0ull);
            }
        } else {
            unsigned long long run = 0;
            for (size_t w0 = 0; w0 < words; w0 += kWave) {
                const size_t wi = w0 + lane;
                unsigned long long x = wi < words ? load_coherent64(&vbits[wi]) : 0ull;
                const uint32_t pc = (uint32_t)__popcll(x);
                const uint32_t incl = wave_incl_scan(pc, lane);
                const uint32_t tot = __shfl(incl, kWave - 1, kWave);
                unsigned long long pos = base + run + (incl - pc);
                if (x) store_coherent64(&vbits[wi], 0ull);
                while (x) {
                    const uint32_t bpos = (uint32_t)(__ffsll((long long)x) - 1);
                    x &= x - 1;
                    if (write_ok) a.out.pool[pos] = (uint32_t)(wi * 64 + bpos);
                    ++pos;
                }
                run += tot;
            }
        }
        __builtin_amdgcn_s_waitcnt(0);  // the cleared bitmap is performed before the next sample
        wave_sync();
        st_members += T;
        st_levels += level;
        st_maxlev = max(st_maxlev, (unsigned long long)level);
        st_runs += 1;
    }
    // every lane holds partial counts of its own items; lane 0 holds the per-sample ones
    st_ea = wave_sum64(st_ea);
    st_philox = wave_sum64(st_philox);
    st_live = wave_sum64(st_live);
    if (lane == 0) {
        atomicAdd(&a.ctl->stats[kStatEdgeAccesses], st_ea);
        atomicAdd(&a.ctl->stats[kStatSampleEdges], st_ea);
        atomicAdd(&a.ctl->stats[kStatPhilox], st_philox);
        atomicAdd(&a.ctl->stats[kStatLive], st_live);
        atomicAdd(&a.ctl->stats[kStatMembers], st_members);
        atomicAdd(&a.ctl->stats[kStatEntries], st_members);
        atomicAdd(&a.ctl->stats[kStatLevels], st_levels);
        atomicMax(&a.ctl->stats[kStatMaxLevels], st_maxlev);
        atomicAdd(&a.ctl->stats[kStatBatches], st_runs);
    }
}

}  // namespace

hipError_t launch_unfused(const UnfusedArgs& a, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(unfused_bpt_kernel, dim3(grid), dim3(kUnfusedBlock), 0, stream, a);
    return hipGetLastError();
}

}  // namespace bpt
