// Pipelined fused launches of request chunks, for the serving loop.
//
// A lane is one stream with its own traversal workspace, output pool and
// control block.  lane_launch enqueues one persistent fused launch over a set
// of chunks (consecutive sample ranges of requests, possibly on different
// graphs) and returns at once; the CSR assembly of each chunk appends to its
// request's output at the request's running member count, so the chunks of
// one request, spread over many launches on alternating lanes, assemble into
// the same CSR a single call would write.  A launch on one lane fills the GPU
// while the previous launch on the other lane drains.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "bpt.h"

namespace bpt {

struct LaneChunk {
    bpt_graph* graph;
    uint64_t first_sample;
    uint64_t n_samples;
    uint64_t seed;
    uint32_t colors;                 // 8 .. 64 (one mask word)
    unsigned long long* d_offsets;   // the chunk's n_samples + 1 offsets inside its request's CSR
    uint32_t* d_vertices;            // the request's member buffer (capacity entries)
    uint64_t capacity;
    unsigned long long* d_total;     // device: the request's members so far (read, then advanced)
};

struct Lane;

Lane* lane_create(int device, std::string* why);
void lane_destroy(Lane* l);
hipStream_t lane_stream(Lane* l);
// Enqueues the chunks' traversal (one launch) and, once `after` (an event of
// the previous launch on another lane, or null) has completed, their CSR
// assembly.  Returns a BPT_* status without waiting for the device.
int lane_launch(Lane* l, const LaneChunk* chunks, uint32_t n, hipEvent_t after, std::string* why);
// Event recorded after the last kernel of the lane's current launch.
hipEvent_t lane_done(Lane* l);
// True once the current launch has completed (does not block).
bool lane_finished(Lane* l);
// Traversal slots of the lane's workspace (0 before its first launch).
uint32_t lane_slots(const Lane* l);
// Waits for the current launch.  *overflow: its output pool overflowed, so
// the chunks' members were not written (their offsets and totals were): the
// caller samples those requests again.  Returns a BPT_* status.
int lane_wait(Lane* l, bool* overflow, std::string* why);

// Greedy maximum coverage (as bpt_max_cover) with caller-provided device
// scratch of max_cover_scratch(n_sets, n, k, total) bytes, where total is the
// sets' member count.
int max_cover_run(const uint64_t* d_offsets, const uint32_t* d_vertices, uint64_t n_sets, uint32_t n, uint32_t k,
                  hipStream_t stream, uint32_t* seeds, uint64_t* gains, void* scratch, size_t scratch_bytes,
                  std::string* why);
size_t max_cover_scratch(uint64_t n_sets, uint32_t n, uint32_t k, uint64_t total);

}  // namespace bpt
