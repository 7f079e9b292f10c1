// From per-sample sets in claim order to the CSR the caller asked for:
// an exclusive scan of the set sizes gives the offsets (sample-id order),
// then each set is copied from the pool to its final place.
#include "bpt_internal.hpp"

namespace bpt {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanPerThread = 8;
constexpr int kTile = kScanBlock * kScanPerThread;
constexpr int kWave = 64;

__device__ __forceinline__ unsigned long long block_sum(unsigned long long x, unsigned long long* tmp) {
    const uint32_t lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) x += __shfl_xor(x, d, kWave);
    if (lane == 0) tmp[wid] = x;
    __syncthreads();
    unsigned long long all = 0;
    for (int w = 0; w < kScanBlock / kWave; ++w) all += tmp[w];
    __syncthreads();
    return all;
}

__device__ __forceinline__ unsigned long long block_excl_scan(unsigned long long x, unsigned long long* tmp,
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
    for (int w = 0; w < kScanBlock / kWave; ++w) {
        before += (w < (int)wid) ? tmp[w] : 0ull;
        all += tmp[w];
    }
    __syncthreads();
    *total = all;
    return before + incl - x;
}

__global__ __launch_bounds__(kScanBlock) void tile_sums(const uint32_t* counts, uint64_t n, unsigned long long* part) {
    __shared__ unsigned long long tmp[kScanBlock / kWave];
    const uint64_t t0 = (uint64_t)blockIdx.x * kTile;
    unsigned long long x = 0;
    for (int k = 0; k < kScanPerThread; ++k) {
        const uint64_t i = t0 + (uint64_t)k * kScanBlock + threadIdx.x;
        if (i < n) x += counts[i];
    }
    const unsigned long long s = block_sum(x, tmp);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// One workgroup: exclusive scan of the tile sums, starting at *base (0 when
// null), total into *total and offsets[n].  `base` may be `total` itself.
__global__ __launch_bounds__(kScanBlock) void scan_tiles(unsigned long long* part, uint64_t ntiles, uint64_t n,
                                                         unsigned long long* offsets, unsigned long long* total,
                                                         const unsigned long long* base) {
    __shared__ unsigned long long tmp[kScanBlock / kWave];
    unsigned long long carry = base ? *base : 0ull;
    __syncthreads();  // every thread has read *base before thread 0 may overwrite it
    for (uint64_t b = 0; b < ntiles; b += kScanBlock) {
        const uint64_t i = b + threadIdx.x;
        const unsigned long long x = i < ntiles ? part[i] : 0ull;
        unsigned long long tot;
        const unsigned long long ex = block_excl_scan(x, tmp, &tot);
        if (i < ntiles) part[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        offsets[n] = carry;
        *total = carry;
    }
}

__global__ __launch_bounds__(kScanBlock) void tile_offsets(const uint32_t* counts, uint64_t n,
                                                           const unsigned long long* part,
                                                           unsigned long long* offsets) {
    __shared__ unsigned long long tmp[kScanBlock / kWave];
    // each thread takes kScanPerThread consecutive counts
    const uint64_t t0 = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kScanPerThread;
    uint32_t v[kScanPerThread];
    unsigned long long mine = 0;
    for (int k = 0; k < kScanPerThread; ++k) {
        const uint64_t i = t0 + k;
        v[k] = i < n ? counts[i] : 0u;
        mine += v[k];
    }
    unsigned long long tot;
    unsigned long long run = part[blockIdx.x] + block_excl_scan(mine, tmp, &tot);
    for (int k = 0; k < kScanPerThread; ++k) {
        const uint64_t i = t0 + k;
        if (i < n) offsets[i] = run;
        run += v[k];
    }
}

// One wavefront per set: pool[where[s] ..] -> vertices[offsets[s] ..].
__global__ __launch_bounds__(256) void gather_sets(const uint32_t* counts, const unsigned long long* where,
                                                   const uint32_t* pool, uint64_t n,
                                                   const unsigned long long* offsets, uint32_t* vertices,
                                                   unsigned long long capacity, const unsigned long long* total,
                                                   const unsigned int* err) {
    if (*total > capacity || (*err & kErrPoolOverflow)) return;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t s = wave; s < n; s += nwaves) {
        const uint32_t c = counts[s];
        const uint32_t* src = pool + where[s];
        uint32_t* dst = vertices + offsets[s];
        for (uint32_t i = lane; i < c; i += kWave) dst[i] = src[i];
    }
}

// ---- segmented assembly: many (chunk) jobs of one launch in four kernels ----
// Segment j covers counts[count_base .. count_base + n) and owns the tiles
// [tile_base, tile_base + tiles) of the partial-sum array.

// Segment of tile or sample `x` given ascending starts (largest j with start[j] <= x).
__device__ __forceinline__ uint32_t seg_of(const FinSeg* seg, uint32_t nseg, uint64_t x, bool by_tile) {
    uint32_t lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        const uint64_t start = by_tile ? seg[mid].tile_base : seg[mid].count_base;
        if (start <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kScanBlock) void tile_sums_seg(const uint32_t* counts, const FinSeg* seg, uint32_t nseg,
                                                            unsigned long long* part) {
    __shared__ unsigned long long tmp[kScanBlock / kWave];
    const uint64_t tile = blockIdx.x;
    const FinSeg& sg = seg[seg_of(seg, nseg, tile, true)];
    const uint64_t t0 = (tile - sg.tile_base) * kTile;
    unsigned long long x = 0;
    for (int k = 0; k < kScanPerThread; ++k) {
        const uint64_t i = t0 + (uint64_t)k * kScanBlock + threadIdx.x;
        if (i < sg.n) x += counts[sg.count_base + i];
    }
    const unsigned long long sum = block_sum(x, tmp);
    if (threadIdx.x == 0) part[tile] = sum;
}

// One workgroup per segment: its tile sums scanned from the segment's running
// total, which is then advanced; offsets[n] of the segment written.
__global__ __launch_bounds__(kScanBlock) void scan_tiles_seg(unsigned long long* part, const FinSeg* seg) {
    __shared__ unsigned long long tmp[kScanBlock / kWave];
    const FinSeg& sg = seg[blockIdx.x];
    const uint64_t ntiles = (sg.n + kTile - 1) / kTile;
    unsigned long long carry = *sg.total;
    __syncthreads();  // every thread has read the running total before thread 0 advances it
    for (uint64_t b = 0; b < ntiles; b += kScanBlock) {
        const uint64_t i = b + threadIdx.x;
        const unsigned long long x = i < ntiles ? part[sg.tile_base + i] : 0ull;
        unsigned long long tot;
        const unsigned long long ex = block_excl_scan(x, tmp, &tot);
        if (i < ntiles) part[sg.tile_base + i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        sg.offsets[sg.n] = carry;
        *sg.total = carry;
    }
}

__global__ __launch_bounds__(kScanBlock) void tile_offsets_seg(const uint32_t* counts, const FinSeg* seg,
                                                               uint32_t nseg, const unsigned long long* part) {
    __shared__ unsigned long long tmp[kScanBlock / kWave];
    const uint64_t tile = blockIdx.x;
    const FinSeg& sg = seg[seg_of(seg, nseg, tile, true)];
    const uint64_t t0 = (tile - sg.tile_base) * kTile + (uint64_t)threadIdx.x * kScanPerThread;
    uint32_t v[kScanPerThread];
    unsigned long long mine = 0;
    for (int k = 0; k < kScanPerThread; ++k) {
        const uint64_t i = t0 + k;
        v[k] = i < sg.n ? counts[sg.count_base + i] : 0u;
        mine += v[k];
    }
    unsigned long long tot;
    unsigned long long run = part[tile] + block_excl_scan(mine, tmp, &tot);
    for (int k = 0; k < kScanPerThread; ++k) {
        const uint64_t i = t0 + k;
        if (i < sg.n) sg.offsets[i] = run;
        run += v[k];
    }
}

// One wavefront per sample of the launch: pool -> its segment's vertices.
__global__ __launch_bounds__(256) void gather_sets_seg(const uint32_t* counts, const unsigned long long* where,
                                                       const uint32_t* pool, uint64_t n_all, const FinSeg* seg,
                                                       uint32_t nseg, const unsigned int* err) {
    if (*err & kErrPoolOverflow) return;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / kWave;
    for (uint64_t x = wave; x < n_all; x += nwaves) {
        const FinSeg& sg = seg[seg_of(seg, nseg, x, false)];
        if (*sg.total > sg.capacity) continue;
        const uint64_t i = x - sg.count_base;
        const uint32_t c = counts[x];
        const uint32_t* src = pool + where[x];
        uint32_t* dst = sg.vertices + sg.offsets[i];
        for (uint32_t k = lane; k < c; k += kWave) dst[k] = src[k];
    }
}

}  // namespace

hipError_t launch_finalize_segments(const uint32_t* counts, const unsigned long long* where, const uint32_t* pool,
                                    uint64_t n_all, const FinSeg* d_seg, uint32_t nseg, uint64_t ntiles,
                                    const unsigned int* err, void* scratch, size_t scratch_bytes, hipStream_t stream) {
    if (nseg == 0) return hipSuccess;
    if (scratch_bytes < (size_t)(ntiles ? ntiles : 1) * sizeof(unsigned long long)) return hipErrorInvalidValue;
    unsigned long long* part = static_cast<unsigned long long*>(scratch);
    if (ntiles > 0)
        hipLaunchKernelGGL(tile_sums_seg, dim3((unsigned)ntiles), dim3(kScanBlock), 0, stream, counts, d_seg, nseg,
                           part);
    hipLaunchKernelGGL(scan_tiles_seg, dim3(nseg), dim3(kScanBlock), 0, stream, part, d_seg);
    if (ntiles > 0) {
        hipLaunchKernelGGL(tile_offsets_seg, dim3((unsigned)ntiles), dim3(kScanBlock), 0, stream, counts, d_seg,
                           nseg, part);
        const unsigned blocks = (unsigned)(n_all < 262144 ? (n_all + 3) / 4 : 65536);
        hipLaunchKernelGGL(gather_sets_seg, dim3(blocks ? blocks : 1), dim3(256), 0, stream, counts, where, pool,
                           n_all, d_seg, nseg, err);
    }
    return hipGetLastError();
}

uint64_t finalize_tiles(uint64_t n_samples) { return (n_samples + kTile - 1) / kTile; }

size_t finalize_scratch_bytes(uint64_t n_samples) {
    const uint64_t ntiles = (n_samples + kTile - 1) / kTile;
    return (size_t)(ntiles ? ntiles : 1) * sizeof(unsigned long long);
}

hipError_t launch_finalize(const uint32_t* counts, const unsigned long long* where, const uint32_t* pool,
                           uint64_t n_samples, unsigned long long* offsets, uint32_t* vertices,
                           unsigned long long capacity, unsigned long long* total, const unsigned int* err,
                           void* scratch, size_t scratch_bytes, hipStream_t stream,
                           const unsigned long long* base) {
    const uint64_t ntiles = (n_samples + kTile - 1) / kTile;
    if (scratch_bytes < finalize_scratch_bytes(n_samples)) return hipErrorInvalidValue;
    unsigned long long* part = static_cast<unsigned long long*>(scratch);
    if (ntiles > 0) {
        hipLaunchKernelGGL(tile_sums, dim3((unsigned)ntiles), dim3(kScanBlock), 0, stream, counts, n_samples, part);
    }
    hipLaunchKernelGGL(scan_tiles, dim3(1), dim3(kScanBlock), 0, stream, part, ntiles, n_samples, offsets, total,
                       base);
    if (ntiles > 0) {
        hipLaunchKernelGGL(tile_offsets, dim3((unsigned)ntiles), dim3(kScanBlock), 0, stream, counts, n_samples,
                           part, offsets);
        const uint64_t waves_wanted = n_samples;
        const unsigned blocks = (unsigned)(waves_wanted < 262144 ? (waves_wanted + 3) / 4 : 65536);
        hipLaunchKernelGGL(gather_sets, dim3(blocks), dim3(256), 0, stream, counts, where, pool, n_samples, offsets,
                           vertices, capacity, total, err);
    }
    return hipGetLastError();
}

}  // namespace bpt
