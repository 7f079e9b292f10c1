// Host-side declarations of libbpt (graph store builder, sampling driver).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "bpt.h"

namespace bpt {

constexpr uint32_t kAlwaysLiveHost = 0xFFFFFFFFu;
constexpr uint64_t kMaxEdges = 0xFFFFFFFFull - 4;
constexpr uint64_t kMaxSamples = 1ull << 34;

struct HostCsr {
    uint32_t n = 0;
    uint64_t m = 0;
    uint32_t layout = BPT_PROB_UNIFORM;
    uint32_t thr_uniform = 0;
    std::vector<uint32_t> rowptr;    // n+1
    std::vector<uint32_t> col;       // m rounded up to a multiple of 4
    std::vector<uint32_t> thr_row;   // n (BPT_PROB_ROW)
    std::vector<uint32_t> thr_edge;  // m rounded up to a multiple of 4 (BPT_PROB_EDGE)
};

uint32_t threshold_of(float p);
int build_host_csr(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst, const float* prob,
                   HostCsr* out, std::string* why);

}  // namespace bpt
