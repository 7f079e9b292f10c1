// Sorted starts (the paper's heuristics of Section 5: grouping traversals
// with nearby start vertices into one batch, after a locality-preserving
// vertex order such as RCM, raises colour occupancy).  The start vertex of
// every sample of a job is computed with the same keyed Philox as the
// traversal, and the sample indices are sorted by it (or by its rank in the
// graph's vertex order) with a stable radix sort, so ties keep index order
// and the order is deterministic.  Vertex ids, edge ids and coins are not
// relabelled.  The
// fused kernel then forms batch b from samples order[b*C .. b*C + C); each
// sample's set is the same as in id order, and the output stays in id order.
#include <algorithm>

#include <hipcub/hipcub.hpp>

#include "bpt_internal.hpp"
#include "bpt_rng.hpp"

namespace bpt {

namespace {

// key of sample first + i: its start vertex, or that vertex's rank in a
// caller-supplied vertex order (a permutation of 0 .. n-1, e.g. RCM)
__global__ __launch_bounds__(256) void start_keys(uint64_t first, uint64_t n_samples, uint32_t n, uint32_t k0,
                                                  uint32_t k1, const uint32_t* rank, uint32_t* keys, uint32_t* idx) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_samples; i += stride) {
        const uint32_t v = start_of(first + i, n, k0, k1);
        keys[i] = rank ? rank[v] : v;
        idx[i] = (uint32_t)i;
    }
}

int key_bits(uint32_t n) {
    int b = 1;
    while (b < 32 && ((uint64_t)1 << b) < n) ++b;
    return b;
}

size_t sort_temp_bytes(uint64_t n_samples, uint32_t n) {
    size_t temp = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, temp, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                             (const uint32_t*)nullptr, (uint32_t*)nullptr, (int)n_samples, 0,
                                             key_bits(n));
    return temp;
}

size_t up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t order_scratch_bytes(uint64_t n_samples, uint32_t n) {
    return 4 * up(n_samples * sizeof(uint32_t)) + up(sort_temp_bytes(n_samples, n));
}

hipError_t launch_sort_by_start(uint32_t n, uint64_t seed, uint64_t first, uint64_t n_samples, const uint32_t* rank,
                                void* scratch, size_t scratch_bytes, const uint32_t** order, hipStream_t stream) {
    if (n_samples >= (1ull << 31) || scratch_bytes < order_scratch_bytes(n_samples, n)) return hipErrorInvalidValue;
    char* p = static_cast<char*>(scratch);
    uint32_t* keys_in = reinterpret_cast<uint32_t*>(p);
    p += up(n_samples * sizeof(uint32_t));
    uint32_t* keys_out = reinterpret_cast<uint32_t*>(p);
    p += up(n_samples * sizeof(uint32_t));
    uint32_t* idx_in = reinterpret_cast<uint32_t*>(p);
    p += up(n_samples * sizeof(uint32_t));
    uint32_t* idx_out = reinterpret_cast<uint32_t*>(p);
    p += up(n_samples * sizeof(uint32_t));
    size_t temp = sort_temp_bytes(n_samples, n);
    const unsigned grid = (unsigned)std::min<uint64_t>(4096, (n_samples + 255) / 256 + 1);
    hipLaunchKernelGGL(start_keys, dim3(grid), dim3(256), 0, stream, first, n_samples, n, (uint32_t)seed,
                       (uint32_t)(seed >> 32), rank, keys_in, idx_in);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipcub::DeviceRadixSort::SortPairs(p, temp, keys_in, keys_out, idx_in, idx_out, (int)n_samples, 0,
                                           key_bits(n), stream);
    *order = idx_out;
    return e;
}

}  // namespace bpt
