// Influence-maximization seed selection over sampled RRR sets (paper
// Section 2: with reverse influence sampling, choosing k seeds is a maximum
// k-coverage over the sets, and the greedy choice gives 1 - 1/e).
//
// Greedy with exact counts, all on the device:
//   count[v]   number of sets not yet covered that hold v (u32);
//   step r     the vertex not chosen yet with the largest count, the lowest
//              id on ties (one packed 64-bit key, (count << 32) | ~v, reduced
//              with a device-wide atomicMax), then every uncovered set that
//              holds it is covered and its members' counts drop by one.
// An inverted index (for each vertex, the sets that hold it: a counting sort
// of the (vertex, set) pairs) lets step r visit only the chosen vertex's sets;
// one wavefront covers a set and decrements its members in parallel.  The
// input CSR is validated first: a malformed one sets an error flag that every
// later kernel checks, so no access leaves the arrays.
#include <algorithm>

#include "bpt_internal.hpp"

namespace bpt {

namespace {

constexpr int kBlock = 256;
constexpr int kWave = 64;

__device__ __forceinline__ unsigned long long wave_max64(unsigned long long x) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)x, d, kWave);
        const uint32_t hi = __shfl_xor((uint32_t)(x >> 32), d, kWave);
        const unsigned long long y = ((unsigned long long)hi << 32) | lo;
        x = y > x ? y : x;
    }
    return x;
}

// offsets must start at 0, be non-decreasing and end at `total`.
__global__ __launch_bounds__(kBlock) void cover_validate(const uint64_t* offsets, uint64_t n_sets, uint64_t total,
                                                         unsigned int* bad) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_sets; s += stride) {
        const uint64_t a = offsets[s], b = offsets[s + 1];
        if (a > b || b > total || (s == 0 && a != 0)) atomicOr(bad, kCoverBadOffsets);
    }
}

__global__ __launch_bounds__(kBlock) void cover_count(const uint32_t* vertices, uint64_t lo, uint64_t hi, uint32_t n,
                                                      uint32_t* count, unsigned int* bad) {
    if (*bad & kCoverBadOffsets) return;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = lo + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += stride) {
        const uint32_t v = vertices[i];
        if (v < n) atomicAdd(&count[v], 1u);
        else atomicOr(bad, kCoverBadVertex);
    }
}

__global__ __launch_bounds__(kBlock) void cover_argmax(const uint32_t* count, const uint8_t* chosen, uint32_t n,
                                                       unsigned long long* best) {
    __shared__ unsigned long long part[kBlock / kWave];
    unsigned long long key = 0;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        if (chosen[v]) continue;
        const unsigned long long k = ((unsigned long long)count[v] << 32) | (0xFFFFFFFFu - v);
        key = k > key ? k : key;
    }
    key = wave_max64(key);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = 0;
        for (int w = 0; w < kBlock / kWave; ++w) m = part[w] > m ? part[w] : m;
        atomicMax(best, m);
    }
}

// One thread: record step r's seed and gain, mark it chosen, reset the key.
__global__ void cover_pick(unsigned long long* best, uint8_t* chosen, uint32_t* seeds, unsigned long long* gains,
                           uint32_t step) {
    const unsigned long long key = *best;
    const uint32_t v = 0xFFFFFFFFu - (uint32_t)key;
    seeds[step] = v;
    gains[step] = key >> 32;
    chosen[v] = 1;
    *best = 0;
}

// start[v] = sets holding a vertex below v (an exclusive scan of the counts,
// one 256-thread workgroup per 2048 vertices, then the tile sums in one
// workgroup, then the tile offsets added).
constexpr int kTile = kBlock * 8;

__device__ __forceinline__ unsigned long long block_scan_excl(unsigned long long x, unsigned long long* tmp,
                                                              unsigned long long* total) {
    const uint32_t lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    unsigned long long incl = x;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const unsigned long long y = __shfl_up(incl, d, kWave);
        if (lane >= (uint32_t)d) incl += y;
    }
    if (lane == kWave - 1) tmp[wid] = incl;
    __syncthreads();
    unsigned long long before = 0, all = 0;
    for (int w = 0; w < kBlock / kWave; ++w) {
        before += (w < (int)wid) ? tmp[w] : 0ull;
        all += tmp[w];
    }
    __syncthreads();
    *total = all;
    return before + incl - x;
}

__global__ __launch_bounds__(kBlock) void index_tile_scan(const uint32_t* count, uint32_t n,
                                                          unsigned long long* start, unsigned long long* tile_sum,
                                                          const unsigned int* bad) {
    __shared__ unsigned long long tmp[kBlock / kWave];
    if (*bad) return;
    const uint64_t t0 = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * 8;
    uint32_t v[8];
    unsigned long long mine = 0;
    for (int k = 0; k < 8; ++k) {
        v[k] = t0 + k < n ? count[t0 + k] : 0u;
        mine += v[k];
    }
    unsigned long long tot;
    unsigned long long run = block_scan_excl(mine, tmp, &tot);
    for (int k = 0; k < 8; ++k) {
        if (t0 + k < n) start[t0 + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void index_tile_carry(unsigned long long* tile_sum, uint64_t ntiles,
                                                           const unsigned int* bad) {
    __shared__ unsigned long long tmp[kBlock / kWave];
    if (*bad) return;
    unsigned long long carry = 0;
    for (uint64_t b = 0; b < ntiles; b += kBlock) {
        const uint64_t i = b + threadIdx.x;
        const unsigned long long x = i < ntiles ? tile_sum[i] : 0ull;
        unsigned long long tot;
        const unsigned long long ex = block_scan_excl(x, tmp, &tot);
        if (i < ntiles) tile_sum[i] = carry + ex;
        carry += tot;
    }
}

// Adds the tile carries; cursor[v] starts equal to start[v].
__global__ __launch_bounds__(kBlock) void index_add_carry(unsigned long long* start, unsigned long long* cursor,
                                                          uint32_t n, uint64_t total, const unsigned long long* tile_sum,
                                                          const unsigned int* bad) {
    if (*bad) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) start[n] = total;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const unsigned long long x = start[v] + tile_sum[v / kTile];
        start[v] = x;
        cursor[v] = x;
    }
}

// inv[cursor[v]++] = s for every member v of every set s (order within a
// vertex's list does not matter).
__global__ __launch_bounds__(kBlock) void index_scatter(const uint64_t* offsets, const uint32_t* vertices,
                                                        uint64_t n_sets, unsigned long long* cursor, uint32_t* inv,
                                                        const unsigned int* bad) {
    if (*bad) return;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t s = wave; s < n_sets; s += nwaves)
        for (uint64_t i = offsets[s] + lane; i < offsets[s + 1]; i += kWave)
            inv[atomicAdd(&cursor[vertices[i]], 1ull)] = (uint32_t)s;
}

// Step `step`: every set holding the chosen vertex that is not covered yet
// becomes covered and its members' counts drop by one, one wavefront per set
// (a set holds the vertex once, so no two wavefronts of a step share a set).
__global__ __launch_bounds__(kBlock) void cover_apply(const uint64_t* offsets, const uint32_t* vertices,
                                                      const unsigned long long* start, const uint32_t* inv,
                                                      const uint32_t* seeds, uint32_t step, uint8_t* covered,
                                                      uint32_t* count, const unsigned int* bad) {
    if (*bad) return;
    const uint32_t v = seeds[step];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    const uint64_t lo = start[v], hi = start[v + 1];
    for (uint64_t i = lo + wave; i < hi; i += nwaves) {
        const uint32_t s = inv[i];
        if (covered[s]) continue;
        if (lane == 0) covered[s] = 1;
        for (uint64_t k = offsets[s] + lane; k < offsets[s + 1]; k += kWave) atomicSub(&count[vertices[k]], 1u);
    }
}

}  // namespace

size_t max_cover_scratch_bytes(uint64_t n_sets, uint32_t n, uint32_t k, uint64_t total) {
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t ntiles = ((size_t)n + kTile - 1) / kTile;
    return up((size_t)n * 4) + up(n) + up(n_sets) + up(16) + up((size_t)k * 4) + up((size_t)k * 8) +
           up(((size_t)n + 1) * 8) + up((size_t)n * 8) + up(ntiles * 8) + up(total * 4);
}

hipError_t launch_max_cover(const uint64_t* offsets, const uint32_t* vertices, uint64_t n_sets, uint64_t total,
                            uint32_t n, uint32_t k, void* scratch, uint32_t** seeds_dev,
                            unsigned long long** gains_dev, unsigned int** bad_dev, hipStream_t stream) {
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const uint64_t ntiles = ((uint64_t)n + kTile - 1) / kTile;
    char* p = static_cast<char*>(scratch);
    uint32_t* count = reinterpret_cast<uint32_t*>(p);
    p += up((size_t)n * 4);
    uint8_t* chosen = reinterpret_cast<uint8_t*>(p);
    p += up(n);
    uint8_t* covered = reinterpret_cast<uint8_t*>(p);
    p += up(n_sets);
    unsigned long long* best = reinterpret_cast<unsigned long long*>(p);
    unsigned int* bad = reinterpret_cast<unsigned int*>(p + 8);
    p += up(16);
    uint32_t* seeds = reinterpret_cast<uint32_t*>(p);
    p += up((size_t)k * 4);
    unsigned long long* gains = reinterpret_cast<unsigned long long*>(p);
    p += up((size_t)k * 8);
    unsigned long long* start = reinterpret_cast<unsigned long long*>(p);  // n + 1
    p += up(((size_t)n + 1) * 8);
    unsigned long long* cursor = reinterpret_cast<unsigned long long*>(p);
    p += up((size_t)n * 8);
    unsigned long long* tile_sum = reinterpret_cast<unsigned long long*>(p);
    p += up(ntiles * 8);
    uint32_t* inv = reinterpret_cast<uint32_t*>(p);
    *seeds_dev = seeds;
    *gains_dev = gains;
    *bad_dev = bad;
    hipError_t e = hipMemsetAsync(scratch, 0, reinterpret_cast<char*>(seeds) - static_cast<char*>(scratch), stream);
    if (e != hipSuccess) return e;
    const unsigned grid_sets = (unsigned)std::min<uint64_t>(65536, (n_sets + kBlock - 1) / kBlock + 1);
    hipLaunchKernelGGL(cover_validate, dim3(grid_sets), dim3(kBlock), 0, stream, offsets, n_sets, total, bad);
    // members counted where the offsets say the sets are
    hipLaunchKernelGGL(cover_count, dim3(65536), dim3(kBlock), 0, stream, vertices, (uint64_t)0, total, n, count, bad);
    // the inverted index: per vertex, the sets that hold it
    hipLaunchKernelGGL(index_tile_scan, dim3((unsigned)ntiles), dim3(kBlock), 0, stream, count, n, start, tile_sum,
                       bad);
    hipLaunchKernelGGL(index_tile_carry, dim3(1), dim3(kBlock), 0, stream, tile_sum, ntiles, bad);
    const unsigned grid_n = (unsigned)std::min<uint64_t>(4096, ((uint64_t)n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(index_add_carry, dim3(grid_n), dim3(kBlock), 0, stream, start, cursor, n, total, tile_sum, bad);
    const unsigned grid_waves = (unsigned)std::min<uint64_t>(65536, (n_sets * kWave + kBlock - 1) / kBlock + 1);
    hipLaunchKernelGGL(index_scatter, dim3(grid_waves), dim3(kBlock), 0, stream, offsets, vertices, n_sets, cursor, inv,
                       bad);
    for (uint32_t r = 0; r < k; ++r) {
        hipLaunchKernelGGL(cover_argmax, dim3(grid_n), dim3(kBlock), 0, stream, count, chosen, n, best);
        hipLaunchKernelGGL(cover_pick, dim3(1), dim3(1), 0, stream, best, chosen, seeds, gains, r);
        hipLaunchKernelGGL(cover_apply, dim3(256), dim3(kBlock), 0, stream, offsets, vertices, start, inv, seeds, r,
                           covered, count, bad);
    }
    return hipGetLastError();
}

}  // namespace bpt
