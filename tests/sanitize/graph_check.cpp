// Host sanitizer check of the library's graph-store builder (build_host_csr
// and the threshold conversion), built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py.  Random edge
// lists of every probability layout, self-loops and empty rows are built and
// the transposed CSR is checked against a direct count; invalid inputs must
// be rejected with BPT_EINVAL.
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "bpt_host.hpp"

using bpt::HostCsr;

static uint64_t rng_state = 0xD1B54A32D192ED03ull;
static uint64_t next_u64() {  // splitmix64
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c);    \
            return 1;                                                       \
        }                                                                   \
    } while (0)

static int one_graph(uint32_t n, uint64_t draws, int layout) {
    std::set<std::pair<uint32_t, uint32_t>> seen;
    std::vector<uint32_t> src, dst;
    std::vector<float> prob;
    for (uint64_t i = 0; i < draws; ++i) {
        const uint32_t u = (uint32_t)(next_u64() % n), v = (uint32_t)(next_u64() % n);
        if (!seen.insert({u, v}).second) continue;
        src.push_back(u);
        dst.push_back(v);
        float p = 0.25f;                                          // uniform
        if (layout == 1) p = 1.0f / (float)(1 + v % 7);           // depends on the destination only
        if (layout == 2) p = (float)(next_u64() % 1001) / 1000.0f;  // per edge, 0 and 1 included
        prob.push_back(p);
    }
    HostCsr csr;
    std::string why;
    const int rc = bpt::build_host_csr(n, src.size(), src.data(), dst.data(), prob.data(), &csr, &why);
    CHECK(rc == BPT_OK);
    CHECK(csr.n == n && csr.m == src.size());
    CHECK(csr.rowptr.size() == (size_t)n + 1 && csr.rowptr[0] == 0 && csr.rowptr[n] == csr.m);
    std::vector<uint32_t> indeg(n, 0);
    for (uint32_t v : dst) indeg[v]++;
    for (uint32_t v = 0; v < n; ++v) {
        CHECK(csr.rowptr[v + 1] - csr.rowptr[v] == indeg[v]);
        for (uint32_t e = csr.rowptr[v]; e < csr.rowptr[v + 1]; ++e) {
            CHECK(seen.count({csr.col[e], v}) == 1);
            if (e > csr.rowptr[v]) CHECK(csr.col[e] > csr.col[e - 1]);
        }
    }
    CHECK(csr.col.size() % 4 == 0);
    if (csr.layout == BPT_PROB_EDGE) CHECK(csr.thr_edge.size() == csr.col.size());
    if (csr.layout == BPT_PROB_ROW) CHECK(csr.thr_row.size() == n);
    return 0;
}

int main() {
    for (int t = 0; t < 9; ++t)
        if (one_graph(1 + (uint32_t)(next_u64() % 400), next_u64() % 4000, t % 3)) return 1;
    HostCsr csr;
    std::string why;
    uint32_t s[2] = {0, 7}, d[2] = {1, 1};
    float p[2] = {0.5f, 0.5f};
    CHECK(bpt::build_host_csr(3, 2, s, d, p, &csr, &why) == BPT_EINVAL);  // vertex id >= n
    uint32_t s2[2] = {0, 0};
    CHECK(bpt::build_host_csr(3, 2, s2, d, p, &csr, &why) == BPT_EINVAL);  // repeated edge
    float nan = 0.0f / 0.0f;
    float p2[1] = {nan};
    CHECK(bpt::build_host_csr(3, 1, s, d, p2, &csr, &why) == BPT_EINVAL);  // NaN probability
    CHECK(bpt::build_host_csr(0, 0, nullptr, nullptr, nullptr, &csr, &why) == BPT_EINVAL);  // no vertices
    CHECK(bpt::build_host_csr(5, 0, nullptr, nullptr, nullptr, &csr, &why) == BPT_OK);  // no edges
    CHECK(bpt::threshold_of(1.0f) == 0xFFFFFFFFu && bpt::threshold_of(0.0f) == 0u &&
          bpt::threshold_of(0.5f) == 0x80000000u);
    printf("graph builder sanitizer check ok\n");
    return 0;
}
