// Host half of the graph store: validates the edge list, puts the edges in
// canonical (dst, src) order, and builds the transposed CSR with per-edge
// thresholds plus the most compact threshold layout (paper Section 2: G with
// p(e); the traversal of Listing 1 walks the edges of each frontier vertex,
// which for reverse-reachable sets are its in-edges).
#include "bpt_host.hpp"

#include <string.h>

#include <algorithm>
#include <vector>

namespace bpt {

// floor(p * 2^32) for fp32 p in [0, 1), from the float's significand and
// exponent; p = 1 maps to the always-live sentinel.
uint32_t threshold_of(float p) {
    if (!(p < 1.0f)) return kAlwaysLiveHost;
    if (!(p > 0.0f)) return 0u;
    uint32_t bits;
    memcpy(&bits, &p, sizeof(bits));
    const uint32_t exp_field = (bits >> 23) & 0xFFu;
    const uint64_t frac = bits & 0x7FFFFFu;
    const uint64_t sig = exp_field ? (frac | (1ull << 23)) : frac;
    const int pow2 = (exp_field ? (int)exp_field - 150 : -149) + 32;  // p * 2^32 = sig * 2^pow2
    if (pow2 >= 0) return (uint32_t)(sig << pow2);
    if (pow2 <= -40) return 0u;
    return (uint32_t)(sig >> (-pow2));
}

namespace {

int bits_for(uint64_t x) {  // bits needed to represent values < x
    int b = 0;
    while (b < 64 && (x - 1) >> b) ++b;
    return b;
}

// LSD radix sort of (key, value) pairs on the low `key_bits` bits, 16 bits a pass.
void radix_sort_pairs(std::vector<uint64_t>& key, std::vector<uint32_t>& val, int key_bits) {
    const size_t m = key.size();
    std::vector<uint64_t> k2(m);
    std::vector<uint32_t> v2(m);
    std::vector<size_t> count(1u << 16);
    for (int shift = 0; shift < key_bits; shift += 16) {
        std::fill(count.begin(), count.end(), 0);
        for (size_t i = 0; i < m; ++i) ++count[(key[i] >> shift) & 0xFFFFu];
        size_t run = 0;
        for (auto& c : count) {
            const size_t t = c;
            c = run;
            run += t;
        }
        for (size_t i = 0; i < m; ++i) {
            const size_t d = count[(key[i] >> shift) & 0xFFFFu]++;
            k2[d] = key[i];
            v2[d] = val[i];
        }
        key.swap(k2);
        val.swap(v2);
    }
}

}  // namespace

int build_host_csr(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst, const float* prob,
                   HostCsr* out, std::string* why) {
    if (n == 0) {
        *why = "n must be at least 1";
        return BPT_EINVAL;
    }
    if (m > kMaxEdges) {
        *why = "too many edges (m must be below 2^32 - 4)";
        return BPT_EINVAL;
    }
    if (m > 0 && (!src || !dst || !prob)) {
        *why = "src, dst and prob must be non-NULL when m > 0";
        return BPT_EINVAL;
    }
    for (uint64_t i = 0; i < m; ++i) {
        if (src[i] >= n || dst[i] >= n) {
            *why = "edge " + std::to_string(i) + " has a vertex id >= n";
            return BPT_EINVAL;
        }
        const float p = prob[i];
        if (!(p >= 0.0f && p <= 1.0f)) {
            *why = "edge " + std::to_string(i) + " has a probability that is NaN or outside [0, 1]";
            return BPT_EINVAL;
        }
    }
    try {
        std::vector<uint64_t> key(m);
        std::vector<uint32_t> thr(m);
        for (uint64_t i = 0; i < m; ++i) {
            key[i] = (uint64_t)dst[i] * n + src[i];
            thr[i] = threshold_of(prob[i]);
        }
        radix_sort_pairs(key, thr, bits_for((uint64_t)n * n));
        for (uint64_t e = 1; e < m; ++e) {
            if (key[e] == key[e - 1]) {
                *why = "repeated edge " + std::to_string(key[e] % n) + " -> " + std::to_string(key[e] / n);
                return BPT_EINVAL;
            }
        }
        out->n = n;
        out->m = m;
        out->rowptr.assign((size_t)n + 1, 0u);
        out->col.assign((size_t)((m + 3) & ~3ull), 0u);
        for (uint64_t e = 0; e < m; ++e) {
            out->rowptr[key[e] / n + 1] += 1;
            out->col[e] = (uint32_t)(key[e] % n);
        }
        for (uint32_t v = 0; v < n; ++v) out->rowptr[v + 1] += out->rowptr[v];

        bool uniform = true, per_row = true;
        for (uint64_t e = 1; e < m && uniform; ++e) uniform = thr[e] == thr[0];
        if (!uniform) {
            for (uint32_t v = 0; v < n && per_row; ++v)
                for (uint32_t e = out->rowptr[v] + 1; e < out->rowptr[v + 1]; ++e)
                    if (thr[e] != thr[out->rowptr[v]]) {
                        per_row = false;
                        break;
                    }
        }
        out->thr_row.clear();
        out->thr_edge.clear();
        out->thr_uniform = 0;
        if (uniform) {
            out->layout = BPT_PROB_UNIFORM;
            out->thr_uniform = m ? thr[0] : 0u;
        } else if (per_row) {
            out->layout = BPT_PROB_ROW;
            out->thr_row.assign(n, 0u);
            for (uint32_t v = 0; v < n; ++v)
                if (out->rowptr[v + 1] > out->rowptr[v]) out->thr_row[v] = thr[out->rowptr[v]];
        } else {
            out->layout = BPT_PROB_EDGE;
            out->thr_edge.assign((size_t)((m + 3) & ~3ull), 0u);
            std::copy(thr.begin(), thr.end(), out->thr_edge.begin());
        }
    } catch (const std::bad_alloc&) {
        *why = "host allocation failed while building the graph";
        return BPT_ENOMEM;
    }
    return BPT_OK;
}

}  // namespace bpt
