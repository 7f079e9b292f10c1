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
// A set is searched for the chosen vertex by one wavefront with a 64-way
// search (sets are sorted ascending), and the wavefront then decrements its
// members in parallel.  The input CSR is validated first: a malformed one
// sets an error flag that every later kernel checks, so no access leaves the
// arrays.
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

__global__ __launch_bounds__(kBlock) void cover_apply(const uint64_t* offsets, const uint32_t* vertices,
                                                      uint64_t n_sets, uint32_t n, const uint32_t* seeds,
                                                      uint32_t step, uint8_t* covered, uint32_t* count,
                                                      const unsigned int* bad) {
    if (*bad) return;
    const uint32_t v = seeds[step];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t s = wave; s < n_sets; s += nwaves) {
        if (covered[s]) continue;
        uint64_t a = offsets[s], b = offsets[s + 1];
        const uint64_t lo = a, hi = b;
        // 64-way search for v in the sorted members [a, b)
        while (b - a > kWave) {
            const uint64_t w = (b - a + kWave - 1) / kWave;
            const uint64_t pos = a + (uint64_t)lane * w;
            const uint32_t x = pos < b ? vertices[pos] : 0xFFFFFFFFu;
            const unsigned long long le = __ballot(pos < b && x <= v);
            if (!le) {
                a = b;
                break;
            }
            const uint64_t j = 63u - (uint64_t)__clzll((long long)le);
            const uint64_t na = a + j * w;
            b = (na + w < b) ? na + w : b;
            a = na;
        }
        const uint64_t pos = a + lane;
        const bool found = __ballot(pos < b && vertices[pos] == v) != 0;
        if (!found) continue;
        if (lane == 0) covered[s] = 1;
        for (uint64_t i = lo + lane; i < hi; i += kWave) atomicSub(&count[vertices[i]], 1u);
    }
}

}  // namespace

size_t max_cover_scratch_bytes(uint64_t n_sets, uint32_t n, uint32_t k) {
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return up((size_t)n * 4) + up(n) + up(n_sets) + up(16) + up((size_t)k * 4) + up((size_t)k * 8);
}

hipError_t launch_max_cover(const uint64_t* offsets, const uint32_t* vertices, uint64_t n_sets, uint64_t total,
                            uint32_t n, uint32_t k, void* scratch, uint32_t** seeds_dev,
                            unsigned long long** gains_dev, unsigned int** bad_dev, hipStream_t stream) {
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
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
    *seeds_dev = seeds;
    *gains_dev = gains;
    *bad_dev = bad;
    hipError_t e = hipMemsetAsync(scratch, 0, reinterpret_cast<char*>(seeds) - static_cast<char*>(scratch), stream);
    if (e != hipSuccess) return e;
    const unsigned grid_sets = (unsigned)std::min<uint64_t>(65536, (n_sets + kBlock - 1) / kBlock + 1);
    hipLaunchKernelGGL(cover_validate, dim3(grid_sets), dim3(kBlock), 0, stream, offsets, n_sets, total, bad);
    // members counted where the offsets say the sets are
    hipLaunchKernelGGL(cover_count, dim3(65536), dim3(kBlock), 0, stream, vertices, (uint64_t)0, total, n, count, bad);
    const unsigned grid_n = (unsigned)std::min<uint64_t>(4096, ((uint64_t)n + kBlock - 1) / kBlock);
    const unsigned grid_apply = (unsigned)std::min<uint64_t>(65536, (n_sets * kWave + kBlock - 1) / kBlock + 1);
    for (uint32_t r = 0; r < k; ++r) {
        hipLaunchKernelGGL(cover_argmax, dim3(grid_n), dim3(kBlock), 0, stream, count, chosen, n, best);
        hipLaunchKernelGGL(cover_pick, dim3(1), dim3(1), 0, stream, best, chosen, seeds, gains, r);
        hipLaunchKernelGGL(cover_apply, dim3(grid_apply), dim3(kBlock), 0, stream, offsets, vertices, n_sets, n,
                           seeds, r, covered, count, bad);
    }
    return hipGetLastError();
}

}  // namespace bpt
