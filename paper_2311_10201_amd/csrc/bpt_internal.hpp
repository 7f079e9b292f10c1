// Internal types shared by the host driver and the kernels of libbpt.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "bpt.h"

namespace bpt {

// ---------------------------------------------------------------------------
// Device graph store: transposed CSR (row v = sources of v's in-edges, in
// ascending order; position in `col` = canonical edge id) plus thresholds.
// ---------------------------------------------------------------------------
struct DevGraph {
    const uint32_t* rowptr;    // n+1
    const uint32_t* col;       // m (padded to a multiple of 4)
    const uint32_t* thr_row;   // n, BPT_PROB_ROW layout only
    const uint32_t* thr_edge;  // m padded to a multiple of 4 with 0, BPT_PROB_EDGE only
    uint32_t thr_uniform;      // BPT_PROB_UNIFORM layout only
    uint32_t prob_layout;      // BPT_PROB_*
    uint32_t n;
    uint32_t m;
};

// Counters accumulated by the kernels (device copy: unsigned long long[kNumStats]).
enum StatIndex {
    kStatMembers = 0,
    kStatSampleEdges,
    kStatEdgeAccesses,
    kStatEntries,
    kStatPhilox,
    kStatLive,
    kStatLevels,
    kStatMaxLevels,
    kStatBatches,
    kNumStats
};

// Device-side error bits (unsigned int).
enum ErrorBits : unsigned int {
    kErrPoolOverflow = 1u,   // output pool too small: grow and run again
    kErrQueueOverflow = 2u,  // frontier queue exceeded n entries (cannot happen)
    kErrLevelBound = 4u,     // more than n+1 levels in one batch (cannot happen)
    kErrBadRange = 8u,       // a plan's device-supplied sample range leaves [0, 2^34)
    kErrHelpTimeout = 16u,   // a helped chunk did not complete within the wait bound (cannot happen)
};

// Small per-call control block in device memory.
struct Control {
    unsigned long long pool_cursor;  // output entries claimed so far
    unsigned long long total;        // offsets[n_samples] after the scan
    unsigned long long work_counter; // next batch / sample to claim
    unsigned int err;                // ErrorBits
    unsigned int pad_;
    unsigned long long finished;     // batches whose sets are written
    unsigned long long open;         // batches open to helpers
    unsigned long long stats[kNumStats];
};

// Help record of one slot (one-word masks only).  Once the launch has no
// batch left to claim, the owner of a batch still running publishes each
// heavy chunk's staging, and idle workgroups claim units of BS work items of
// it.  While helpers may join, the batch's discovery counters live here
// instead of in the owner's LDS.
struct HelpRec {
    unsigned long long claim;  // [63:48] chunk number, [47:20] work items, [19:0] next unit to claim
    unsigned long long batch;  // launch-wide batch index of the helped batch
    unsigned int state;        // 1 while helpers may join
    unsigned int done;         // work items of the current chunk finished
    unsigned int npos;         // staged positions of the current chunk
    unsigned int nxt;          // parity of the next level (frontier and queue)
    unsigned int qnext;        // counter of the next level's queue (level + 1) % 3
    unsigned int job;          // job index of the batch
    unsigned int pad_[2];
    unsigned int qlen[3];      // as the owner's LDS counters
    unsigned int tlen;
    unsigned int cnt[64];
    unsigned int pad2_[48];    // 512 bytes
};
static_assert(sizeof(HelpRec) == 512, "help records are 512 bytes");
constexpr unsigned int kHelpStagePos = 2048;  // staged positions per chunk at most (BS * ept for one-word masks)

// Per-slot state of the fused traversal (one slot per resident workgroup).
// All arrays are zero between batches except `stamp`, whose values only grow.
// Words of a vertex's mask record in a fused slot: visited, the frontier of
// even levels and the frontier of odd levels, NW words each; one-word records
// are padded to 32 bytes so that none straddles a 64-byte line.
constexpr __host__ __device__ size_t mask_record_words(int nw) { return nw == 1 ? 4 : 3 * (size_t)nw; }

struct FusedSlots {
    unsigned long long* masks;     // slots * n * mask_record_words(NW): per-vertex mask records
    uint32_t* stamp;               // slots * n           (NW > 1 only)
    uint32_t* queue;               // slots * 2 * n
    uint32_t* touched;             // slots * n
    unsigned long long* tbits;     // slots * words(n)
    uint32_t* slot_tag;            // slots
    HelpRec* help;                 // slots (one-word masks; else null)
    uint32_t* hstage;              // slots * kHelpStagePos * 6 words: scan, beg, end, thr, mask lo/hi
    uint32_t slots;
};

struct Output {
    uint32_t* counts;           // n_samples: |R_s|
    unsigned long long* where;  // n_samples: position of R_s in `pool`
    uint32_t* pool;             // members, set by set, in claim order
    unsigned long long pool_cap;
};

// One job of a fused launch: a graph and a range of sample ids under a seed.
// FusedJob::flags: discoveries read visited[u] before their fetch-or.  It
// pays where most live coins find their colours there already (graphs whose
// sets are large: dense cores reached along many paths) and costs a round
// trip where they do not (small, tree-like sets).  The sets are the same
// either way.
constexpr uint32_t kJobReadFirst = 1u;

struct FusedJob {
    DevGraph g;
    uint64_t seed;
    uint64_t first_sample;
    uint64_t n_samples;
    uint64_t batch_begin;  // first launch-wide batch index of the job
    uint64_t out_base;     // position of the job's first sample in Output::counts / where
    uint32_t colors;       // samples per batch (at most 64 * NW)
    uint32_t flags;        // kJob* bits
    const uint32_t* order; // batch composition: batch b takes samples first + order[b*colors ..] (null: in id order)
};

struct FusedArgs {
    FusedJob job0;          // the job when `jobs` is null (single-job launches)
    const FusedJob* jobs;   // device array of n_jobs jobs, by ascending batch_begin, or null
    uint32_t n_jobs;
    uint32_t n_max;         // slot stride in vertices: the largest n over the jobs
    FusedSlots ws;
    Output out;             // counts / where for all jobs' samples; one shared pool
    Control* ctl;
    uint64_t n_batches;     // over all jobs
    uint32_t gather_mode;   // kGatherAuto, kGatherNever or kGatherAlways
};

// How the fused expansion schedules an entry's colours (see expand_item):
// chosen per wavefront from the expected live colours per edge, or forced.
enum GatherMode : uint32_t { kGatherAuto = 0, kGatherNever = 1, kGatherAlways = 2 };

// Per-wave state of the unfused traversal.
struct UnfusedSlots {
    unsigned long long* vbits;  // slots * words(n): visited bitmap
    uint32_t* log;              // slots * n: visit order (level by level)
    uint32_t slots;
};

struct UnfusedArgs {
    DevGraph g;
    UnfusedSlots ws;
    Output out;
    Control* ctl;
    uint64_t seed;
    uint64_t first_sample;
    uint64_t n_samples;
};

__host__ __device__ inline size_t bitmap_words(uint32_t n) { return ((size_t)n + 63) / 64; }

// Kernel launchers (defined in the .hip files).
// help: with one-word masks, let workgroups without a batch left help the
// batches still running (worth it when sets are large and levels few).
hipError_t launch_fused(const FusedArgs& a, int nw, int block, int grid, bool help, hipStream_t stream);
hipError_t launch_unfused(const UnfusedArgs& a, int grid, hipStream_t stream);
// CSR assembly of one job's sets: offsets by a scan of `counts`, then a
// gather from the pool (skipped when the total exceeds `capacity` or the pool
// overflowed).  The total goes to offsets[n_samples] and *total.  With `base`
// (device memory, may equal `total`) the offsets start at *base instead of 0:
// consecutive sample ranges of one request appended into one CSR.
hipError_t launch_finalize(const uint32_t* counts, const unsigned long long* where, const uint32_t* pool,
                           uint64_t n_samples, unsigned long long* offsets, uint32_t* vertices,
                           unsigned long long capacity, unsigned long long* total, const unsigned int* err,
                           void* scratch, size_t scratch_bytes, hipStream_t stream,
                           const unsigned long long* base = nullptr);
size_t finalize_scratch_bytes(uint64_t n_samples);

// Many jobs' CSR assembly in four kernels (segment j: counts/where entries
// [count_base, count_base + n), partial sums [tile_base, tile_base +
// finalize_tiles(n))), each appended at its own running total (which it
// then advances) into its own offsets / vertices.  Segments by ascending
// count_base and tile_base; the table lives in device memory.
struct FinSeg {
    uint64_t count_base;
    uint64_t n;
    uint64_t tile_base;
    unsigned long long* offsets;  // n + 1 entries written
    uint32_t* vertices;
    unsigned long long capacity;
    unsigned long long* total;    // running member count: base in, total out
};
uint64_t finalize_tiles(uint64_t n_samples);
hipError_t launch_finalize_segments(const uint32_t* counts, const unsigned long long* where, const uint32_t* pool,
                                    uint64_t n_all, const FinSeg* d_seg, uint32_t nseg, uint64_t ntiles,
                                    const unsigned int* err, void* scratch, size_t scratch_bytes, hipStream_t stream);

constexpr int kUnfusedBlock = 256;  // threads per unfused workgroup (4 waves, one sample each)

// Sorted starts (bpt_order.hip): order[i] = indices 0 .. S-1 of samples
// first .. first+S-1 sorted by start vertex (ties by index).
size_t order_scratch_bytes(uint64_t n_samples, uint32_t n);
hipError_t launch_sort_by_start(uint32_t n, uint64_t seed, uint64_t first, uint64_t n_samples, const uint32_t* rank,
                                void* scratch, size_t scratch_bytes, const uint32_t** order, hipStream_t stream);

// Plans (bpt_plan.hip): the kernels that open and close a capturable call.
// plan_setup clears the control block and sets the job's sample range and
// seed (from `params` = {first_sample, seed} in device memory when not null);
// plan_report writes {status, members} for the caller once the CSR is built.
hipError_t launch_plan_setup(FusedJob* job, const uint64_t* params, uint64_t first, uint64_t seed,
                             uint64_t n_samples, uint64_t max_ids, Control* ctl, hipStream_t stream);
hipError_t launch_plan_report(const Control* ctl, unsigned long long capacity, int64_t* result, hipStream_t stream);
// Multi-job plans: the same around a job table (ids[i]: the caller's index of
// table entry i, which selects its params and its result).
hipError_t launch_plan_setup_jobs(FusedJob* jobs, uint32_t n_jobs, const uint64_t* params, const uint32_t* ids,
                                  uint64_t max_ids, Control* ctl, hipStream_t stream);
hipError_t launch_plan_report_jobs(const Control* ctl, const unsigned long long* totals,
                                   const unsigned long long* capacities, const uint32_t* ids, uint32_t n_jobs,
                                   int64_t* result, hipStream_t stream);

// Allocation-free calls (bpt_noalloc.hip): a fixed scratch array per device,
// resolved to its device address once per device (the device must be
// current), and a kernel that zeroes a 16-byte aligned range.
constexpr size_t kNoAllocScratchBytes = (size_t)BPT_NOALLOC_SCRATCH_BYTES;
hipError_t noalloc_scratch(int device, void** addr);
hipError_t launch_zero_fill(void* p, size_t bytes, hipStream_t stream);

// Greedy maximum coverage (bpt_cover.hip).  Error bits of its device flag.
constexpr unsigned int kCoverBadOffsets = 1u;  // offsets not non-decreasing or past the member count
constexpr unsigned int kCoverBadVertex = 2u;   // a member id >= n
size_t max_cover_scratch_bytes(uint64_t n_sets, uint32_t n, uint32_t k, uint64_t total);
hipError_t launch_max_cover(const uint64_t* offsets, const uint32_t* vertices, uint64_t n_sets, uint64_t total,
                            uint32_t n, uint32_t k, void* scratch, uint32_t** seeds_dev,
                            unsigned long long** gains_dev, unsigned int** bad_dev, hipStream_t stream);

}  // namespace bpt
