/*
 * CPU oracle for RRR-set sampling under the Independent Cascade model.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * package smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * What it computes (paper: Section 2, Definition 2 and the paragraph after
 * it; Section 2 IC model paragraph):
 *
 *   For every sample id s, one live-edge world G_s is fixed: each edge e of
 *   the input graph is kept ("live") with probability p(e), decided by a
 *   keyed counter-based coin that depends only on (seed, s, e).  The RRR set
 *   of s is the set of vertices that have a directed path to the start vertex
 *   start_s inside G_s.  It is computed here by one textbook breadth-first
 *   search per sample over the reversed (incoming) edges, which is exactly
 *   the "visited array of a probabilistic BFS" the paper describes.  Because
 *   the coins are keyed, the set does not depend on the order in which edges
 *   are examined (the IC model's permutation invariance), so any correct
 *   traversal - fused or not, level-synchronous or not - must return the same
 *   set.
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes):
 *   - Edge direction: an RRR set follows edges backwards, so the search walks
 *     in-edges u->v of each reached vertex v.
 *   - Coin: edge e is live for sample s iff  thr(e) == 0xFFFFFFFF  or
 *     r(s,e) < thr(e), where thr(e) = floor(p(e) * 2^32) for p < 1 and the
 *     sentinel 0xFFFFFFFF for p >= 1; r is a 32-bit Philox output word.  This
 *     keeps an edge with probability exactly p for every fp32 p >= 2^-9 (the
 *     paper drops a colour when a uniform draw exceeds p, Listing 1).
 *   - Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
 *     "Parallel Random Numbers: As Easy as 1, 2, 3", SC 2011) with
 *     key = (seed mod 2^32, seed >> 32).
 *       coin word of (s, e):  counter (e >> 2, s mod 2^32, s >> 32, 0),
 *                             output word e & 3
 *       start of sample s:    counter ((s >> 2) mod 2^32, s >> 34, 0, 1),
 *                             output word s & 3, start = (r * n) >> 32
 *   - Starts are drawn with replacement, uniformly over V (Section 3 text;
 *     several traversals may share a start).
 *   - Canonical edge id: the rank of (dst, src) in ascending order.  Input
 *     order therefore does not change any result.
 *   - Output: each set in ascending vertex order, sets in sample-id order.
 *
 * Also reported per sample, for the fused-traversal work accounting of
 * Section 3.1 / 3.2: the BFS distance of every member from the start, and
 * TE_s = sum of in-degrees over the members (the edges an unfused traversal
 * of sample s examines).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

/* ------------------------------------------------------------------ */
/* Edge probability -> 32-bit threshold.                              */
/* ------------------------------------------------------------------ */
uint32_t or_thr32(float p)
{
    if (p >= 1.0f)
        return 0xFFFFFFFFu;
    /* p < 1 in fp32 has a 24-bit significand, so p * 2^32 is exact in double */
    double scaled = (double)p * 4294967296.0;
    return (uint32_t)scaled; /* truncation = floor for non-negative values */
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (SC 2011).                                            */
/* ------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

uint32_t or_coin_word(uint64_t seed, uint64_t s, uint64_t e)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)(e >> 2), (uint32_t)s, (uint32_t)(s >> 32), 0u};
    uint32_t out[4];
    or_philox4x32_10(ctr, key, out);
    return out[e & 3];
}

int or_edge_live(uint64_t seed, uint64_t s, uint64_t e, uint32_t thr)
{
    if (thr == 0xFFFFFFFFu)
        return 1;
    return or_coin_word(seed, s, e) < thr;
}

uint32_t or_start_vertex(uint64_t seed, uint64_t s, uint32_t n)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)(s >> 2), (uint32_t)(s >> 34), 0u, 1u};
    uint32_t out[4];
    or_philox4x32_10(ctr, key, out);
    uint64_t r = out[s & 3];
    return (uint32_t)((r * (uint64_t)n) >> 32);
}

/* ------------------------------------------------------------------ */
/* Graph: incoming adjacency in canonical (dst, src) order.           */
/* ------------------------------------------------------------------ */
typedef struct or_graph {
    uint32_t n;
    uint64_t m;
    uint64_t* in_begin; /* n+1 entries: in-edges of v are [in_begin[v], in_begin[v+1]) */
    uint32_t* in_src;   /* source u of canonical edge e */
    uint32_t* in_thr;   /* threshold of canonical edge e */
} or_graph;

/* Stable counting sort of the edge indices in `in` by key[] (values < n),
 * written to `out`. */
static int counting_sort(const uint32_t* key, uint32_t n, uint64_t m, const uint64_t* in, uint64_t* out)
{
    uint64_t* start = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
    if (!start)
        return OR_ENOMEM;
    for (uint64_t i = 0; i < m; ++i)
        start[key[in[i]] + 1] += 1;
    for (uint32_t v = 0; v < n; ++v)
        start[v + 1] += start[v];
    for (uint64_t i = 0; i < m; ++i)
        out[start[key[in[i]]]++] = in[i];
    free(start);
    return OR_OK;
}

void or_graph_free(or_graph* g)
{
    if (!g)
        return;
    free(g->in_begin);
    free(g->in_src);
    free(g->in_thr);
    free(g);
}

/* Returns NULL and sets *status on invalid input (vertex out of range,
 * probability NaN or outside [0,1], repeated (src,dst) pair, n == 0). */
or_graph* or_graph_build(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                         const float* prob, int* status)
{
    *status = OR_OK;
    if (n == 0 || (m > 0 && (!src || !dst || !prob))) {
        *status = OR_EINVAL;
        return NULL;
    }
    for (uint64_t i = 0; i < m; ++i) {
        float p = prob[i];
        if (src[i] >= n || dst[i] >= n || !(p >= 0.0f && p <= 1.0f)) {
            *status = OR_EINVAL;
            return NULL;
        }
    }
    /* canonical order: by dst, ties by src (sort by src, then stably by dst) */
    uint64_t* order = (uint64_t*)malloc((m ? m : 1) * sizeof(uint64_t));
    uint64_t* by_src = (uint64_t*)malloc((m ? m : 1) * sizeof(uint64_t));
    or_graph* g = (or_graph*)calloc(1, sizeof(or_graph));
    if (!order || !by_src || !g) {
        free(order); free(by_src); free(g);
        *status = OR_ENOMEM;
        return NULL;
    }
    for (uint64_t i = 0; i < m; ++i)
        order[i] = i;
    if (counting_sort(src, n, m, order, by_src) != OR_OK ||
        counting_sort(dst, n, m, by_src, order) != OR_OK) {
        free(order); free(by_src); free(g);
        *status = OR_ENOMEM;
        return NULL;
    }
    free(by_src);
    for (uint64_t e = 1; e < m; ++e) {
        if (src[order[e]] == src[order[e - 1]] && dst[order[e]] == dst[order[e - 1]]) {
            free(order); free(g);
            *status = OR_EINVAL;
            return NULL;
        }
    }
    g->n = n;
    g->m = m;
    g->in_begin = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
    g->in_src = (uint32_t*)malloc((m ? m : 1) * sizeof(uint32_t));
    g->in_thr = (uint32_t*)malloc((m ? m : 1) * sizeof(uint32_t));
    if (!g->in_begin || !g->in_src || !g->in_thr) {
        free(order);
        or_graph_free(g);
        *status = OR_ENOMEM;
        return NULL;
    }
    for (uint64_t e = 0; e < m; ++e) {
        uint64_t i = order[e];
        g->in_begin[dst[i] + 1] += 1;
        g->in_src[e] = src[i];
        g->in_thr[e] = or_thr32(prob[i]);
    }
    for (uint32_t v = 0; v < n; ++v)
        g->in_begin[v + 1] += g->in_begin[v];
    free(order);
    return g;
}

uint32_t or_graph_n(const or_graph* g) { return g->n; }
uint64_t or_graph_m(const or_graph* g) { return g->m; }

/* Copies the canonical incoming adjacency out (for tests). */
void or_graph_export(const or_graph* g, uint64_t* in_begin, uint32_t* in_src, uint32_t* in_thr)
{
    memcpy(in_begin, g->in_begin, ((size_t)g->n + 1) * sizeof(uint64_t));
    if (g->m) {
        memcpy(in_src, g->in_src, g->m * sizeof(uint32_t));
        memcpy(in_thr, g->in_thr, g->m * sizeof(uint32_t));
    }
}

/* ------------------------------------------------------------------ */
/* One RRR set: reverse BFS from the start in the live-edge world.     */
/* ------------------------------------------------------------------ */
typedef struct bfs_scratch {
    int32_t* dist;  /* n entries, -1 = not reached */
    uint32_t* queue; /* n entries */
} bfs_scratch;

static int cmp_u32(const void* a, const void* b)
{
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Fills members[0..k) (ascending) and their distances; returns k and the
 * sum of in-degrees of the members in *te. */
static uint32_t rrr_one(const or_graph* g, uint64_t seed, uint64_t s, bfs_scratch* sc,
                        uint32_t* members, int32_t* member_dist, uint64_t* te)
{
    uint32_t start = or_start_vertex(seed, s, g->n);
    uint32_t head = 0, tail = 0;
    sc->dist[start] = 0;
    sc->queue[tail++] = start;
    while (head < tail) {
        uint32_t v = sc->queue[head++];
        for (uint64_t e = g->in_begin[v]; e < g->in_begin[v + 1]; ++e) {
            uint32_t u = g->in_src[e];
            if (sc->dist[u] >= 0)
                continue;
            if (!or_edge_live(seed, s, e, g->in_thr[e]))
                continue;
            sc->dist[u] = sc->dist[v] + 1;
            sc->queue[tail++] = u;
        }
    }
    uint32_t k = tail;
    memcpy(members, sc->queue, k * sizeof(uint32_t));
    qsort(members, k, sizeof(uint32_t), cmp_u32);
    uint64_t sum = 0;
    for (uint32_t i = 0; i < k; ++i) {
        uint32_t v = members[i];
        member_dist[i] = sc->dist[v];
        sum += g->in_begin[v + 1] - g->in_begin[v];
    }
    for (uint32_t i = 0; i < k; ++i)
        sc->dist[sc->queue[i]] = -1;
    *te = sum;
    return k;
}

/* ------------------------------------------------------------------ */
/* Many samples, optionally on several threads.                        */
/* ------------------------------------------------------------------ */
typedef struct or_result {
    uint64_t count;     /* number of samples */
    uint64_t* offsets;  /* count+1 */
    uint32_t* members;  /* offsets[count] */
    int32_t* dist;      /* offsets[count], BFS distance of each member */
    uint64_t* te;       /* count: sum of member in-degrees */
} or_result;

typedef struct per_sample {
    uint32_t k;
    uint32_t* members;
    int32_t* dist;
    uint64_t te;
} per_sample;

typedef struct worker_args {
    const or_graph* g;
    uint64_t seed;
    const uint64_t* ids;
    uint64_t count;
    per_sample* out;
    uint64_t next; /* shared work cursor (guarded by lock) */
    pthread_mutex_t lock;
    int failed;
} worker_args;

static void* worker(void* arg)
{
    worker_args* w = (worker_args*)arg;
    const or_graph* g = w->g;
    bfs_scratch sc;
    sc.dist = (int32_t*)malloc((size_t)g->n * sizeof(int32_t));
    sc.queue = (uint32_t*)malloc((size_t)g->n * sizeof(uint32_t));
    uint32_t* tmp_m = (uint32_t*)malloc((size_t)g->n * sizeof(uint32_t));
    int32_t* tmp_d = (int32_t*)malloc((size_t)g->n * sizeof(int32_t));
    if (!sc.dist || !sc.queue || !tmp_m || !tmp_d) {
        pthread_mutex_lock(&w->lock);
        w->failed = 1;
        pthread_mutex_unlock(&w->lock);
        free(sc.dist); free(sc.queue); free(tmp_m); free(tmp_d);
        return NULL;
    }
    for (uint32_t v = 0; v < g->n; ++v)
        sc.dist[v] = -1;
    for (;;) {
        pthread_mutex_lock(&w->lock);
        uint64_t i = w->next;
        int stop = w->failed || i >= w->count;
        if (!stop)
            w->next = i + 1;
        pthread_mutex_unlock(&w->lock);
        if (stop)
            break;
        uint64_t te = 0;
        uint32_t k = rrr_one(g, w->seed, w->ids[i], &sc, tmp_m, tmp_d, &te);
        per_sample* ps = &w->out[i];
        ps->k = k;
        ps->te = te;
        ps->members = (uint32_t*)malloc((size_t)k * sizeof(uint32_t));
        ps->dist = (int32_t*)malloc((size_t)k * sizeof(int32_t));
        if (!ps->members || !ps->dist) {
            pthread_mutex_lock(&w->lock);
            w->failed = 1;
            pthread_mutex_unlock(&w->lock);
            break;
        }
        memcpy(ps->members, tmp_m, (size_t)k * sizeof(uint32_t));
        memcpy(ps->dist, tmp_d, (size_t)k * sizeof(int32_t));
    }
    free(sc.dist); free(sc.queue); free(tmp_m); free(tmp_d);
    return NULL;
}

void or_result_free(or_result* r)
{
    if (!r)
        return;
    free(r->offsets);
    free(r->members);
    free(r->dist);
    free(r->te);
    free(r);
}

/* RRR sets of the listed sample ids, in list order.  nthreads <= 1 runs on
 * the calling thread only. */
or_result* or_sample_ids(const or_graph* g, uint64_t seed, const uint64_t* ids, uint64_t count,
                         int nthreads, int* status)
{
    *status = OR_OK;
    worker_args w;
    memset(&w, 0, sizeof(w));
    w.g = g;
    w.seed = seed;
    w.ids = ids;
    w.count = count;
    w.out = (per_sample*)calloc(count ? count : 1, sizeof(per_sample));
    pthread_mutex_init(&w.lock, NULL);
    if (!w.out) {
        *status = OR_ENOMEM;
        return NULL;
    }
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads == 1) {
        worker(&w);
    } else {
        pthread_t* th = (pthread_t*)malloc((size_t)nthreads * sizeof(pthread_t));
        for (int t = 0; t < nthreads; ++t)
            pthread_create(&th[t], NULL, worker, &w);
        for (int t = 0; t < nthreads; ++t)
            pthread_join(th[t], NULL);
        free(th);
    }
    pthread_mutex_destroy(&w.lock);
    or_result* r = (or_result*)calloc(1, sizeof(or_result));
    uint64_t total = 0;
    for (uint64_t i = 0; i < count; ++i)
        total += w.out[i].k;
    if (r) {
        r->count = count;
        r->offsets = (uint64_t*)malloc((count + 1) * sizeof(uint64_t));
        r->members = (uint32_t*)malloc((total ? total : 1) * sizeof(uint32_t));
        r->dist = (int32_t*)malloc((total ? total : 1) * sizeof(int32_t));
        r->te = (uint64_t*)malloc((count ? count : 1) * sizeof(uint64_t));
    }
    int ok = !w.failed && r && r->offsets && r->members && r->dist && r->te;
    if (ok) {
        uint64_t pos = 0;
        for (uint64_t i = 0; i < count; ++i) {
            r->offsets[i] = pos;
            memcpy(r->members + pos, w.out[i].members, (size_t)w.out[i].k * sizeof(uint32_t));
            memcpy(r->dist + pos, w.out[i].dist, (size_t)w.out[i].k * sizeof(int32_t));
            r->te[i] = w.out[i].te;
            pos += w.out[i].k;
        }
        r->offsets[count] = pos;
    }
    for (uint64_t i = 0; i < count; ++i) {
        free(w.out[i].members);
        free(w.out[i].dist);
    }
    free(w.out);
    if (!ok) {
        or_result_free(r);
        *status = OR_ENOMEM;
        return NULL;
    }
    return r;
}

/* ------------------------------------------------------------------ */
/* Coin-block accounting of a result.  Under the coin layout above one */
/* Philox block yields the coins of the four edges 4q .. 4q+3 ("quad"  */
/* q) of one sample, so expanding member v of sample s for all of v's  */
/* in-edges evaluates one block per quad that v's row meets.           */
/* ------------------------------------------------------------------ */
/* For every set i of a result (count sets in CSR form: offsets, members
 * ascending, member_dist their BFS depths, as or_result_export writes them)
 * and every member v with in-edges:
 *   all[i]     += quads met by v's row [in_begin[v], in_begin[v+1]), unless
 *                 skip_dead and every threshold of the row is 0 (a row whose
 *                 coins can never be live, known from one stored threshold);
 *   listing[i] += quads met by v's row that hold an edge u -> v whose source
 *                 u is not a member at depth <= depth(v).  Listing 1 masks the
 *                 colours of an edge with ~visited[u]; a source at depth <=
 *                 depth(v) has been visited before v's level is expanded in
 *                 any level-synchronous order, so only the other edges need a
 *                 coin.  (A row counted in `listing` always counts in `all`.)
 * dist is scratch of n entries that must hold -1 everywhere on entry; it is
 * left so. */
void or_quad_accounting(const or_graph* g, uint64_t count, const uint64_t* offsets, const uint32_t* members,
                        const int32_t* member_dist, int skip_dead, int32_t* dist, uint64_t* all, uint64_t* listing)
{
    for (uint64_t i = 0; i < count; ++i) {
        uint64_t lo = offsets[i], hi = offsets[i + 1];
        uint64_t a = 0, l = 0;
        for (uint64_t j = lo; j < hi; ++j)
            dist[members[j]] = member_dist[j];
        for (uint64_t j = lo; j < hi; ++j) {
            uint32_t v = members[j];
            uint64_t b = g->in_begin[v], e = g->in_begin[v + 1];
            if (b == e)
                continue;
            if (skip_dead) {
                int dead = 1;
                for (uint64_t x = b; x < e; ++x)
                    dead = dead && g->in_thr[x] == 0;
                if (dead)
                    continue;
            }
            for (uint64_t q = b >> 2; q <= (e - 1) >> 2; ++q) {
                a += 1;
                uint64_t x0 = q << 2 < b ? b : q << 2;
                uint64_t x1 = (q << 2) + 4 > e ? e : (q << 2) + 4;
                int need = 0;
                for (uint64_t x = x0; x < x1; ++x) {
                    int32_t du = dist[g->in_src[x]];
                    need = need || du < 0 || du > member_dist[j];
                }
                l += need ? 1 : 0;
            }
        }
        for (uint64_t j = lo; j < hi; ++j)
            dist[members[j]] = -1;
        all[i] = a;
        listing[i] = l;
    }
}

uint64_t or_result_count(const or_result* r) { return r->count; }
uint64_t or_result_total(const or_result* r) { return r->offsets[r->count]; }
void or_result_export(const or_result* r, uint64_t* offsets, uint32_t* members, int32_t* dist,
                      uint64_t* te)
{
    memcpy(offsets, r->offsets, (r->count + 1) * sizeof(uint64_t));
    uint64_t total = r->offsets[r->count];
    if (total) {
        memcpy(members, r->members, total * sizeof(uint32_t));
        memcpy(dist, r->dist, total * sizeof(int32_t));
    }
    if (r->count)
        memcpy(te, r->te, r->count * sizeof(uint64_t));
}
