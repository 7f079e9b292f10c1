/* Host sanitizer check of the CPU oracle (test infrastructure): built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py.
 * Builds small random graphs (with self-loops, isolated vertices, p = 0 and
 * p = 1 edges), samples them on several threads, and checks what holds for
 * any RRR set: ascending members, the start among them at distance 0, and
 * the quad accounting run over the result.  Invalid inputs must be rejected. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct or_graph or_graph;
typedef struct or_result or_result;
or_graph* or_graph_build(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst, const float* prob,
                         int* status);
void or_graph_free(or_graph* g);
or_result* or_sample_ids(const or_graph* g, uint64_t seed, const uint64_t* ids, uint64_t count, int nthreads,
                         int* status);
void or_result_free(or_result* r);
uint64_t or_result_count(const or_result* r);
uint64_t or_result_total(const or_result* r);
void or_result_export(const or_result* r, uint64_t* offsets, uint32_t* members, int32_t* dist, uint64_t* te);
void or_quad_accounting(const or_graph* g, uint64_t count, const uint64_t* offsets, const uint32_t* members,
                        const int32_t* dist, int one_threshold_rows, int32_t* scratch, uint64_t* all,
                        uint64_t* listing);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64(void) {  /* splitmix64 */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

#define CHECK(c)                                                  \
    do {                                                          \
        if (!(c)) {                                               \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                             \
        }                                                         \
    } while (0)

static int one_graph(uint32_t n, uint64_t m_draw, int trial) {
    uint32_t* src = malloc(m_draw * sizeof(uint32_t));
    uint32_t* dst = malloc(m_draw * sizeof(uint32_t));
    float* prob = malloc(m_draw * sizeof(float));
    uint8_t* seen = calloc((size_t)n * n, 1);
    uint64_t m = 0;
    for (uint64_t i = 0; i < m_draw; ++i) {
        const uint32_t u = (uint32_t)(next_u64() % n), v = (uint32_t)(next_u64() % n);
        if (seen[(size_t)u * n + v]) continue;
        seen[(size_t)u * n + v] = 1;
        src[m] = u;
        dst[m] = v;
        const uint64_t k = next_u64() % 8;
        prob[m] = k == 0 ? 0.0f : (k == 1 ? 1.0f : (float)(next_u64() % 1000) / 1000.0f);
        ++m;
    }
    int st = 0;
    or_graph* g = or_graph_build(n, m, src, dst, prob, &st);
    CHECK(g && st == 0);
    const uint64_t count = 97;
    uint64_t* ids = malloc(count * sizeof(uint64_t));
    for (uint64_t i = 0; i < count; ++i) ids[i] = next_u64() >> 30;
    or_result* r = or_sample_ids(g, 1000u + (uint64_t)trial, ids, count, 3, &st);
    CHECK(r && st == 0 && or_result_count(r) == count);
    const uint64_t total = or_result_total(r);
    uint64_t* off = malloc((count + 1) * sizeof(uint64_t));
    uint32_t* mem = malloc((total ? total : 1) * sizeof(uint32_t));
    int32_t* dist = malloc((total ? total : 1) * sizeof(int32_t));
    uint64_t* te = malloc(count * sizeof(uint64_t));
    or_result_export(r, off, mem, dist, te);
    CHECK(off[0] == 0 && off[count] == total);
    for (uint64_t s = 0; s < count; ++s) {
        CHECK(off[s + 1] > off[s]);
        int starts = 0;
        for (uint64_t j = off[s]; j < off[s + 1]; ++j) {
            CHECK(mem[j] < n);
            if (j > off[s]) CHECK(mem[j] > mem[j - 1]);
            CHECK(dist[j] >= 0);
            starts += dist[j] == 0;
        }
        CHECK(starts == 1);
    }
    int32_t* scratch = malloc(n * sizeof(int32_t));
    for (uint32_t v = 0; v < n; ++v) scratch[v] = -1;
    uint64_t* all = malloc(count * sizeof(uint64_t));
    uint64_t* listing = malloc(count * sizeof(uint64_t));
    or_quad_accounting(g, count, off, mem, dist, 0, scratch, all, listing);
    for (uint64_t s = 0; s < count; ++s) CHECK(listing[s] <= all[s]);
    or_result_free(r);
    or_graph_free(g);
    free(src), free(dst), free(prob), free(seen), free(ids), free(off), free(mem), free(dist), free(te);
    free(scratch), free(all), free(listing);
    return 0;
}

int main(void) {
    for (int t = 0; t < 6; ++t)
        if (one_graph(1 + (uint32_t)(next_u64() % 300), 1 + next_u64() % 3000, t)) return 1;
    /* invalid inputs are rejected, not read out of bounds */
    uint32_t s2[2] = {0, 5}, d2[2] = {1, 1};
    float p2[2] = {0.5f, 0.5f};
    int st = 0;
    CHECK(!or_graph_build(3, 2, s2, d2, p2, &st) && st != 0); /* source >= n */
    uint32_t s3[2] = {0, 0}, d3[2] = {1, 1};
    CHECK(!or_graph_build(3, 2, s3, d3, p2, &st) && st != 0); /* duplicate edge */
    float p3[1] = {1.5f};
    CHECK(!or_graph_build(3, 1, s3, d3, p3, &st) && st != 0); /* probability above 1 */
    printf("oracle sanitizer check ok\n");
    return 0;
}
