/*
 * bpt.h - C ABI of libbpt: fused breadth-first probabilistic traversals (BPTs)
 * that sample random reverse-reachable (RRR) sets under the Independent
 * Cascade (IC) model on an AMD Instinct MI355X (gfx950).
 *
 * Problem statement (paper Section 2, Definitions 1 and 2): a directed graph
 * G = (V, E) with a probability p(e) on each edge is given.  An RRR set is
 * drawn by picking a start vertex v uniformly at random, keeping every edge e
 * independently with probability p(e), and collecting every vertex u that
 * has a directed path u -> ... -> v through kept edges.  Many such sets are
 * the input of influence maximization by reverse influence sampling.
 *
 * Method (paper Section 3, Listing 1): the traversals of C samples (C =
 * colors_per_batch, one bit per sample, "colour") are fused into one
 * breadth-first frontier that carries a C-bit mask per vertex, so a vertex
 * reached by several samples at the same depth has its in-edges expanded
 * once for all of them.
 *
 * Determinism contract.  Each sample s draws its coins from Philox4x32-10
 * (Salmon et al., SC 2011) keyed on (seed, s, canonical edge id), so the
 * result depends only on the edge set with its probabilities, n, the sample
 * ids and the seed.  It is bit-identical for every colors_per_batch, for the
 * fused and the unfused traversal, for any launch shape and across runs.
 *
 * Definitions used throughout:
 *   canonical edge id   rank of (dst, src) in ascending order (input order is
 *                       irrelevant).
 *   threshold           thr(e) = floor(p(e) * 2^32) for p < 1, 0xFFFFFFFF for
 *                       p = 1.  Edge e is live for sample s iff thr(e) ==
 *                       0xFFFFFFFF or r < thr(e), where r is word (e & 3) of
 *                       Philox(counter = (e >> 2, s mod 2^32, s >> 32, 0),
 *                       key = (seed mod 2^32, seed >> 32)).
 *   start vertex        word (s & 3) of Philox(counter = ((s >> 2) mod 2^32,
 *                       s >> 34, 0, 1), same key), mapped to (r * n) >> 32.
 *   RRR set of s        ascending vertex ids u with a live path u -> start_s
 *                       (the start itself included).
 *
 * Errors.  Functions that return a pointer return NULL on failure; functions
 * that return int return one of the BPT_* status codes.  Either way the
 * calling thread's last status and a message are available through
 * bpt_last_status() / bpt_last_error().  No function aborts the process.
 *
 * Threads.  A graph is immutable once created; several threads may sample
 * from the same graph at once (each call takes its own workspace).
 */
#ifndef BPT_H
#define BPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BPT_OK 0
#define BPT_EINVAL (-1)   /* invalid argument                                  */
#define BPT_ENOMEM (-2)   /* host or device allocation failed                  */
#define BPT_EDEVICE (-3)  /* HIP runtime error or no usable gfx950 device      */
#define BPT_ERANGE (-4)   /* caller's output buffer too small (size reported)  */
#define BPT_EINTERNAL (-5)/* a device-side consistency check failed            */

/* Probability layouts detected when a graph is created. */
#define BPT_PROB_UNIFORM 0 /* one threshold for every edge                      */
#define BPT_PROB_ROW 1     /* thresholds depend only on the destination vertex  */
#define BPT_PROB_EDGE 2    /* one threshold per edge                            */

/* Flags of bpt_sample_rrr_device(). */
#define BPT_FLAG_UNFUSED 1u /* one traversal per sample (the unfused baseline)  */
#define BPT_FLAG_SORTED_STARTS 2u /* fused batches of samples with neighbouring start
                                     vertices (paper Section 5); same sets, same order */

typedef struct bpt_graph bpt_graph; /* opaque, device-resident, immutable */
typedef struct bpt_rrr bpt_rrr;     /* opaque, host-resident CSR of RRR sets */

/* Work accounting of one sampling call (paper Section 3.1-3.2 terms). */
typedef struct bpt_counters {
    uint64_t samples;          /* RRR sets produced                                    */
    uint64_t members;          /* sum over samples of |R_s|                             */
    uint64_t sample_edges;     /* TE: sum over samples of the in-degrees of R_s members
                                  = edges an unfused traversal examines                  */
    uint64_t edge_accesses;    /* EA: in-edges examined by the traversal actually run
                                  (one row scan per frontier entry)                     */
    uint64_t frontier_entries; /* (batch, level, vertex) frontier entries expanded      */
    uint64_t philox_blocks;    /* Philox4x32-10 evaluations for edge coins              */
    uint64_t live_coins;       /* coins that came up live                               */
    uint64_t levels;           /* sum over batches of BFS levels                        */
    uint64_t max_levels;       /* deepest batch                                         */
    uint64_t batches;          /* batches (fused) or traversals (unfused) run           */
    uint64_t traversal_ns;     /* duration of the traversal kernel (HIP events on the
                                  call's stream), nanoseconds                           */
    uint64_t finalize_ns;      /* duration of the CSR assembly kernels, nanoseconds     */
    uint64_t workgroup_size;   /* threads per workgroup of the traversal launch         */
    uint64_t workgroups;       /* workgroups of the traversal launch (persistent)       */
} bpt_counters;

/* ------------------------------------------------------------------------
 * bpt_create_graph - build the device-resident graph store (paper Section 2:
 * G = (V, E) with p(e); Listing 1 walks the edges of a frontier vertex, which
 * for RRR sets are its in-edges).
 *
 *   n      number of vertices, 1 <= n < 2^32.
 *   m      number of edges, m < 2^32 - 4.
 *   src    host array, m entries: tail u of edge i (u -> dst[i]); u < n.
 *   dst    host array, m entries: head v of edge i; v < n.
 *   prob   host array, m entries: p(e) in [0, 1] (fp32, not NaN); the
 *          probability that u activates v (IC model).
 *   The three arrays are copied; the caller keeps ownership.  They may be
 *   NULL when m == 0.
 *
 * Stores the transposed CSR on the current HIP device: row v lists the
 * sources u of v's in-edges in ascending order (canonical edge ids), plus
 * thresholds in the most compact of the BPT_PROB_* layouts.  Self-loops are
 * accepted (they never change a set).
 *
 * Returns NULL on error: BPT_EINVAL (n == 0, m too large, NULL array with
 * m > 0, vertex out of range, probability NaN or outside [0, 1], repeated
 * (src, dst) pair), BPT_ENOMEM, BPT_EDEVICE.  Free with bpt_free().
 * ---------------------------------------------------------------------- */
bpt_graph* bpt_create_graph(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                            const float* prob);

/* One request of bpt_sample_rrr_jobs(). */
typedef struct bpt_job {
    bpt_graph* graph;          /* in: graph; all jobs of a call on one device          */
    uint64_t first_sample;     /* in: first sample id                                  */
    uint64_t n_samples;        /* in: sets wanted (ids first_sample .. + n_samples - 1) */
    uint64_t seed;             /* in: Philox key                                       */
    uint32_t colors_per_batch; /* in: as in bpt_sample_rrr (0: library's choice)       */
    uint32_t reserved;         /* in: must be 0                                        */
    uint64_t* d_offsets;       /* in: device array of n_samples + 1 entries            */
    uint32_t* d_vertices;      /* in: device array of `capacity` entries               */
    uint64_t capacity;         /* in                                                   */
    uint64_t total;            /* out: members of the job's sets                       */
    int32_t status;            /* out: BPT_OK, or BPT_ERANGE when capacity < total     */
    uint32_t reserved2;        /* in: must be 0                                        */
} bpt_job;

/* ------------------------------------------------------------------------
 * bpt_sample_rrr - sample RRR sets 0 .. n_samples-1 with fused BPTs
 * (paper Section 3, Listing 1) and return them in host memory.
 *
 *   g                 graph from bpt_create_graph.
 *   n_samples         number of RRR sets, < 2^34.  0 gives an empty result.
 *   colors_per_batch  traversals fused per batch: a power of two from 8 to
 *                     1024 (below 64, a batch uses part of one 64-bit colour
 *                     mask); 0 lets the library choose (bpt_default_colors).
 *                     Does not change the result.
 *   seed              Philox key.
 *
 * Returns a host-resident CSR (see bpt_rrr_* accessors), or NULL on error:
 * BPT_EINVAL (NULL graph, bad colors_per_batch, n_samples >= 2^34),
 * BPT_ENOMEM, BPT_EDEVICE, BPT_EINTERNAL.  Free with bpt_free().  The result
 * does not depend on the graph staying alive.
 * ---------------------------------------------------------------------- */
bpt_rrr* bpt_sample_rrr(bpt_graph* g, uint64_t n_samples, uint32_t colors_per_batch,
                        uint64_t seed);

/* Frees a bpt_graph, a bpt_rrr or a bpt_plan (the handle carries its type).
 * NULL is a no-op.  Sets BPT_EINVAL if the handle is none of these.  Free a
 * plan only when no call on it is in flight, and before its graph. */
void bpt_free(void* handle);

/* Accessors of a result.  offsets has num_samples+1 entries; the members of
 * sample i are vertices[offsets[i] .. offsets[i+1]), ascending.  The arrays
 * belong to the result and stay valid until bpt_free(result). */
uint64_t bpt_rrr_num_samples(const bpt_rrr* r);
uint64_t bpt_rrr_num_members(const bpt_rrr* r);
const uint64_t* bpt_rrr_offsets(const bpt_rrr* r);
const uint32_t* bpt_rrr_vertices(const bpt_rrr* r);

/* Last status / message of the calling thread (message valid until the
 * thread's next libbpt call). */
int bpt_last_status(void);
const char* bpt_last_error(void);

/* ------------------------------------------------------------------------
 * Extensions.
 * ---------------------------------------------------------------------- */

/* bpt_sample_rrr_device - sample RRR sets first_sample .. first_sample +
 * n_samples - 1 into caller-owned DEVICE buffers, on a caller's stream.
 *
 *   first_sample      id of the first sample (a shard of a larger job gives
 *                     its own range; the sets equal those of one big call).
 *   n_samples         as in bpt_sample_rrr.
 *   colors_per_batch  as in bpt_sample_rrr (ignored with BPT_FLAG_UNFUSED).
 *   flags             0; BPT_FLAG_UNFUSED for one traversal per sample; or
 *                     BPT_FLAG_SORTED_STARTS: the fused batches take the
 *                     samples in order of their start vertex (ties by id)
 *                     instead of id order, which can raise colour occupancy;
 *                     the sets and their order are unchanged (n_samples < 2^31,
 *                     not with BPT_FLAG_UNFUSED).
 *   stream            hipStream_t to run on (NULL = the default stream).
 *   d_offsets         device array of n_samples+1 uint64: written with the
 *                     CSR offsets (d_offsets[0] = 0).
 *   d_vertices        device array of `capacity` uint32: written with the
 *                     members, sample after sample, ascending within each.
 *   capacity          entries available in d_vertices.
 *   total_out         host pointer, required: receives the total number of
 *                     members (= d_offsets[n_samples]).
 *   counters          host pointer or NULL: receives the work accounting.
 *
 * Blocks the calling thread until the work on `stream` is done.  If
 * capacity < total, returns BPT_ERANGE with *total_out set and d_vertices
 * untouched (d_offsets is written); call again with a larger buffer.  Other
 * errors: BPT_EINVAL (NULL graph/pointers, bad colors or flags), BPT_ENOMEM,
 * BPT_EDEVICE, BPT_EINTERNAL.
 */
int bpt_sample_rrr_device(bpt_graph* g, uint64_t first_sample, uint64_t n_samples,
                          uint32_t colors_per_batch, uint64_t seed, uint32_t flags, void* stream,
                          uint64_t* d_offsets, uint32_t* d_vertices, uint64_t capacity,
                          uint64_t* total_out, bpt_counters* counters);

/* bpt_sample_rrr_noalloc - bpt_sample_rrr_device (fused traversal, flags 0)
 * for callers that cannot allocate device memory: code that runs between the
 * phases of a tight serving loop, harnesses that forbid allocation during a
 * measured region, and callers that must not disturb the caching allocator of
 * the framework they run under.  The call itself allocates nothing, on the
 * host or the device: the traversal slots, per-sample counters, member pool,
 * scan temporaries and control block are carved from one fixed scratch array
 * of BPT_NOALLOC_SCRATCH_BYTES (256 MiB) that the library holds on every GPU
 * it runs on, from the time its code is loaded until the process ends.
 *
 *   arguments         as bpt_sample_rrr_device without flags and counters;
 *                     colors_per_batch 0 lets the library choose.
 *
 * The sets equal those of bpt_sample_rrr_device for the same graph, range,
 * seed and colours.  The scratch bounds what one call can hold: 12 bytes per
 * sample plus the scan's temporaries, at least one traversal slot (about
 * 44 bytes per vertex for up to 64 colours, more for wider masks), and a pool
 * of 4 bytes per member of all the call's sets; the number of slots (batches
 * in flight) shrinks to leave the pool room.  A call that does not fit returns
 * BPT_ENOMEM with the sizes in the message and writes nothing.  Every call on a
 * GPU uses that GPU's scratch, which keeps the last call's contents (each call
 * clears what must start at zero): calls of one process are serialized by the
 * library, so two of them never overlap on a GPU.  Blocks the calling thread
 * until the work on `stream` is done.  Other errors: BPT_EINVAL, BPT_ERANGE
 * (capacity < total; *total_out set, d_vertices untouched), BPT_EDEVICE,
 * BPT_EINTERNAL.
 */
#define BPT_NOALLOC_SCRATCH_BYTES (256ull << 20)
int bpt_sample_rrr_noalloc(bpt_graph* g, uint64_t first_sample, uint64_t n_samples,
                           uint32_t colors_per_batch, uint64_t seed, void* stream,
                           uint64_t* d_offsets, uint32_t* d_vertices, uint64_t capacity,
                           uint64_t* total_out);

/* Graph facts: vertices, edges, probability layout (BPT_PROB_*).  Any output
 * pointer may be NULL.  Returns BPT_OK or BPT_EINVAL. */
int bpt_graph_info(const bpt_graph* g, uint32_t* n, uint64_t* m, uint32_t* prob_layout);

/* Frees the device memory the graph keeps cached between calls: traversal
 * workspaces and output pools (tens of GB for graphs with millions of
 * vertices: a workspace holds a traversal slot per resident workgroup, within
 * 60% of the free device memory and 160 GB, or the share that the environment
 * variable BPT_WORKSPACE_FRACTION gives).  Calls in flight on other threads
 * keep theirs.  The next sampling call allocates again.  Returns BPT_OK or
 * BPT_EINVAL. */
int bpt_graph_release_cache(bpt_graph* g);

/* ------------------------------------------------------------------------
 * bpt_sample_rrr_jobs - many sampling requests, possibly on different graphs,
 * in one persistent fused launch (paper Section 4.1: one thread block runs a
 * group of fused traversals, and many groups are in flight).  The batches of all jobs form one list that the
 * launch's workgroups claim from a device counter, so small jobs share the GPU
 * instead of each under-filling it; then every job's CSR is written to its own
 * d_offsets / d_vertices exactly as bpt_sample_rrr_device would write it for
 * the same graph, sample range, seed and colours (the sets do not depend on
 * what else is in the launch).  A job's colors_per_batch of 0 is settled as
 * for the job alone (bpt_default_colors): a job whose samples are few, or
 * heavy, then still splits into many batches.  Jobs may use different colour
 * counts: jobs
 * whose batches need the same number of 64-bit mask words share a launch
 * (so at most five launches, widest masks first).
 *
 *   jobs, n_jobs  the requests; `total` and `status` are written back.
 *   stream        hipStream_t for all work (NULL: default stream); the call
 *                 returns after the stream has finished it.
 *   counters      if not NULL: totals over all jobs (bpt_counters above;
 *                 times summed over the launches, the launch shape the
 *                 largest).
 *
 * Returns BPT_OK; BPT_ERANGE when some job's capacity is below its total
 * (that job's d_offsets and total are valid, its d_vertices untouched; the
 * other jobs' outputs are complete); BPT_EINVAL for a bad job (nothing runs);
 * or BPT_ENOMEM, BPT_EDEVICE, BPT_EINTERNAL.
 * ---------------------------------------------------------------------- */
int bpt_sample_rrr_jobs(bpt_job* jobs, uint32_t n_jobs, void* stream, bpt_counters* counters);

/* ------------------------------------------------------------------------
 * Sampling plans: the fused path as a fixed sequence of kernels that can be
 * captured into a hipGraph and replayed (the batches of paper Section 4.1's
 * persistent launch, without a host round trip per call).
 *
 * bpt_plan_create reserves, once, everything a call of up to max_samples
 * samples at colors_per_batch colours needs on graph g: traversal slots, a
 * member pool of pool_capacity entries, per-sample arrays and a control
 * block.  colors_per_batch 0 takes bpt_default_colors(g, max_samples);
 * pool_capacity 0 takes an estimate from the graph's earlier calls (or 32
 * members per sample).  Returns NULL on error: BPT_EINVAL (NULL graph,
 * max_samples 0 or >= 2^34, bad colors_per_batch), BPT_ENOMEM, BPT_EDEVICE.
 * The graph must outlive the plan.  Free with bpt_free().
 * ---------------------------------------------------------------------- */
typedef struct bpt_plan bpt_plan;

bpt_plan* bpt_plan_create(bpt_graph* g, uint64_t max_samples, uint32_t colors_per_batch,
                          uint64_t pool_capacity);

/* bpt_plan_enqueue - enqueue the sampling of sets first_sample ..
 * first_sample + n_samples - 1 on `stream` and return at once.  The call
 * allocates nothing, launches only kernels (no memset or copy nodes) and never
 * waits on the host, so it may run inside hipStreamBeginCapture /
 * hipStreamEndCapture; each replay of the captured graph samples again.
 *
 *   n_samples    1 .. max_samples of the plan (0 writes an empty result).
 *   d_params     NULL, or device memory holding two uint64 {first_sample,
 *                seed}, read when the stream reaches the call (they override
 *                the two arguments): a captured graph then samples whatever
 *                range and seed the caller has written there, in stream order,
 *                before each replay.  Ranges past 2^34 report BPT_EINVAL.
 *   d_offsets    device array of n_samples+1 uint64 (CSR offsets).
 *   d_vertices   device array of `capacity` uint32 (members, as in
 *                bpt_sample_rrr_device); untouched when they do not fit.
 *   d_result     device (or mapped pinned host) array of two int64 written at
 *                the end: {status, members}.  status BPT_OK: members = total
 *                written.  BPT_ERANGE: capacity too small (members = the total
 *                needed, d_offsets valid) or the plan's pool too small
 *                (members = pool entries needed: create a larger plan).
 *                BPT_EINVAL: the range from d_params leaves [0, 2^34).
 *                BPT_EINTERNAL: a device consistency check failed.
 *
 * The sets equal bpt_sample_rrr_device's for the same graph, range, seed and
 * colours.  Calls on one plan must not overlap in time (one stream, or
 * ordered streams): they share its workspace.  Returns BPT_OK when enqueued;
 * BPT_EINVAL (bad handle or pointers, n_samples above the plan's maximum, a
 * host-given range past 2^34) or BPT_EDEVICE, with nothing enqueued.
 */
int bpt_plan_enqueue(bpt_plan* p, uint64_t first_sample, uint64_t n_samples, uint64_t seed,
                     const uint64_t* d_params, void* stream, uint64_t* d_offsets, uint32_t* d_vertices,
                     uint64_t capacity, int64_t* d_result);

/* ------------------------------------------------------------------------
 * Multi-job plans: bpt_sample_rrr_jobs (many graphs and sample ranges in one
 * persistent launch per mask width, paper Section 4.1) as a fixed sequence of
 * kernels that can be captured into one hipGraph and replayed.
 *
 * bpt_jobs_plan_create reserves, once, everything the n_jobs jobs need: a
 * traversal workspace per mask width sized for its largest graph, per-sample
 * arrays, member pools (pool_capacity entries in all, split over the launches
 * in proportion to the jobs' capacities; 0 takes the graphs' running
 * estimates of the set sizes) and the device
 * job tables.  Each job's graph, n_samples, colors_per_batch (0: as for the
 * job alone), d_offsets, d_vertices and capacity are fixed here, and its
 * buffers must stay valid while the plan is used; first_sample and seed are
 * taken from the job as defaults.  Returns NULL on error: BPT_EINVAL (as
 * bpt_sample_rrr_jobs), BPT_ENOMEM, BPT_EDEVICE.  Free with bpt_free(), after
 * the graphs' last use by the plan and before the graphs.
 *
 * bpt_jobs_plan_enqueue enqueues one sampling of every job on `stream` and
 * returns at once; like bpt_plan_enqueue it allocates nothing, launches only
 * kernels and never waits, so it may be captured.
 *   d_params   NULL, or device memory with 2 * n_jobs uint64: {first_sample,
 *              seed} of job i at [2i], [2i+1], read when the stream reaches the
 *              call: one captured graph then samples whatever ranges and seeds
 *              the caller writes there before each replay.
 *   d_results  device (or mapped pinned host) memory with 2 * n_jobs int64:
 *              {status, members} of job i at [2i], [2i+1], as bpt_plan_enqueue
 *              reports them (BPT_ERANGE with the pool entries needed when a
 *              launch's pool overflowed).
 * Each job's sets equal bpt_sample_rrr_device's for its graph, range, seed
 * and colours.  Calls on one plan must not overlap in time.  Returns BPT_OK
 * when enqueued; BPT_EINVAL (not a multi-job plan, d_results NULL) or
 * BPT_EDEVICE.
 * ---------------------------------------------------------------------- */
bpt_plan* bpt_jobs_plan_create(const bpt_job* jobs, uint32_t n_jobs, uint64_t pool_capacity);
int bpt_jobs_plan_enqueue(bpt_plan* p, const uint64_t* d_params, void* stream, int64_t* d_results);

/* ------------------------------------------------------------------------
 * bpt_max_cover - influence-maximization seeds from sampled RRR sets (paper
 * Section 2: with reverse influence sampling, choosing k seeds is a maximum
 * k-coverage over the sets; the greedy choice gives a 1 - 1/e approximation).
 *
 * k greedy steps on the device; each takes the vertex, among those not chosen
 * yet, that lies in the most sets not covered yet (exact integer counts; the
 * lowest vertex id on ties, also when the count is 0), then covers its sets.
 *
 *   d_offsets   device, n_sets + 1 non-decreasing entries from 0; set i is
 *               d_vertices[d_offsets[i] .. d_offsets[i+1]) (the CSR
 *               bpt_sample_rrr_device writes).
 *   d_vertices  device, d_offsets[n_sets] entries, each set ascending and
 *               without repeats, ids < n.  May be NULL when there are none.
 *   n_sets      < 2^32.   n  vertex count (>= 1).   k  seeds, k <= n.
 *   stream      hipStream_t (NULL: default); returns after it has finished.
 *   seeds       host, k entries (out): the seeds in the order chosen.
 *   gains       host, k entries (out): sets newly covered by each seed, so
 *               n * (sum of gains) / n_sets estimates the seeds' influence.
 *
 * Each step visits only the sets that hold the chosen vertex, through an
 * inverted index (vertex -> sets) built first by a counting sort.  Device
 * scratch of about 21n + n_sets + 4 x (members) bytes is allocated per call.
 * Returns
 * BPT_OK; BPT_EINVAL for bad arguments, offsets that are not a CSR of
 * d_vertices, or a member >= n (checked on the device before any set is
 * touched); BPT_ENOMEM; BPT_EDEVICE.
 * ---------------------------------------------------------------------- */
int bpt_max_cover(const uint64_t* d_offsets, const uint32_t* d_vertices, uint64_t n_sets, uint32_t n, uint32_t k,
                  void* stream, uint32_t* seeds, uint64_t* gains);

/* ------------------------------------------------------------------------
 * Serving loop with continuous batching (paper Section 2: influence
 * maximization by greedy maximum coverage over sampled RRR sets).  A server
 * owns a worker thread on the device that was current when it was created,
 * and a second thread for seed selection.  Requests submitted from any thread
 * are queued; the worker admits them in arrival order while their estimated
 * memory (the sets' expected size from a running per-graph mean, plus
 * per-sample arrays) fits the budget, always one when nothing runs, and at
 * most 64 at a time.  The GPU is fed a pipeline of bounded persistent
 * launches on two streams: each launch takes about four batches per
 * resident workgroup (at most max_jobs_per_launch requests), given out in
 * order of deadline, the submission time plus four times the request's
 * estimated service time; the next launch is enqueued while the current one
 * drains.
 * A request that arrives while others are on the GPU therefore joins the
 * next launch and shares it with them.  Each chunk's CSR
 * is appended to its request's output in sample order; a request completes
 * when its last chunk has, and seed requests then run bpt_max_cover on the
 * second thread while sampling continues.  Every request gets exactly the
 * result it would get alone.  Every request is sampled at 64 colours per
 * batch (the sets do not depend on it).
 * ---------------------------------------------------------------------- */
typedef struct bpt_server bpt_server;

#define BPT_REQ_SAMPLE 0 /* RRR sets into the request's device buffers            */
#define BPT_REQ_SEEDS 1  /* sets into server memory, then k greedy seeds (host)   */

typedef struct bpt_request {
    uint64_t tag;             /* caller's, untouched                                 */
    bpt_graph* graph;         /* in                                                  */
    uint64_t first_sample;    /* in: sample ids first_sample .. + n_samples - 1      */
    uint64_t n_samples;       /* in                                                  */
    uint64_t seed;            /* in: Philox key                                      */
    uint32_t kind;            /* in: BPT_REQ_SAMPLE or BPT_REQ_SEEDS                 */
    uint32_t k;               /* in (SEEDS): seeds wanted, 1 <= k <= n               */
    uint64_t* d_offsets;      /* in (SAMPLE): device, n_samples + 1 entries          */
    uint32_t* d_vertices;     /* in (SAMPLE): device, `capacity` entries             */
    uint64_t capacity;        /* in (SAMPLE)                                         */
    uint32_t* seeds;          /* in (SEEDS): host, k entries, written                */
    uint64_t* gains;          /* in (SEEDS): host, k entries, written                */
    uint64_t total;           /* out: members of the request's sets                  */
    int32_t status;           /* out: 1 while in flight, then BPT_OK or an error
                                 (BPT_ERANGE: SAMPLE capacity below total; offsets
                                 valid, members written only up to the capacity)    */
    uint32_t reserved;
    double t_submit;          /* out: server clock (bpt_server_now), seconds         */
    double t_start;           /* out: its launch began                               */
    double t_done;            /* out: completed                                      */
} bpt_request;

/* memory_budget: bytes of admitted work at a time (0: 8 GiB);
 * max_jobs_per_launch: requests sharing one launch at most, 0 for 256.
 * Device memory: two traversal workspaces sized for the largest graph seen
 * (about 44 bytes per vertex per resident workgroup each, within 60% of
 * the free memory) and their pools.  A workspace is made, or remade
 * larger, by the first launch that needs it: on a 4M-vertex graph that takes
 * seconds, and requests queued meanwhile wait, so a service submits one
 * request on its largest graph at start.
 * NULL on failure. */
bpt_server* bpt_server_create(uint64_t memory_budget, uint32_t max_jobs_per_launch);
/* Queues r; r must stay valid until bpt_server_wait returns it.  BPT_EINVAL
 * for a bad server or request (missing buffers, k = 0, unknown kind). */
int bpt_server_submit(bpt_server* s, bpt_request* r);
/* The next completed request, or NULL after timeout_s seconds. */
bpt_request* bpt_server_wait(bpt_server* s, double timeout_s);
/* Seconds since the server was created (the clock of t_submit / t_done). */
double bpt_server_now(bpt_server* s);
/* What the worker has done so far. */
typedef struct bpt_server_info {
    uint64_t launches; /* fused launches issued                              */
    uint64_t served;   /* requests completed                                 */
    double busy_s;     /* wall time with admitted requests, seconds          */
    double sample_s;   /* ... of which with a launch in flight               */
    double cover_s;    /* seed-selection time (second thread)                */
    double alloc_s;    /* time getting seed requests' set buffers            */
    uint64_t resampled;/* requests sampled again alone (their launch's pool
                          overflowed, or a seed request's sets outgrew the
                          server's buffer)                                   */
    double batch_s;    /* current estimate of GPU seconds per 64-sample batch
                          (orders requests by deadline)                      */
    uint32_t lane_slots;/* traversal slots of the largest lane workspace: one
                          per resident 512-thread workgroup (two per CU),
                          fewer when memory is short; 0 before the first
                          launch                                             */
} bpt_server_info;
int bpt_server_stats(bpt_server* s, bpt_server_info* out);
/* Serves what is queued, then stops the worker and frees the server. */
int bpt_server_destroy(bpt_server* s);

/* ------------------------------------------------------------------------
 * bpt_graph_set_vertex_order - a locality-preserving vertex order for sorted
 * starts (paper Section 5: reordering, e.g. reverse Cuthill-McKee, then
 * batching traversals with nearby starts).  With BPT_FLAG_SORTED_STARTS,
 * samples are batched in order of rank[start] instead of the start's id.
 * Nothing is relabelled: coins stay keyed on the original vertex and edge
 * ids, so the sets are unchanged.
 *
 *   rank  host array of n entries, a permutation of 0 .. n-1 (copied); NULL
 *         returns to id order.
 * Not to be called while a sampling call on the same graph is running.
 * Returns BPT_OK, BPT_EINVAL (bad handle, not a permutation), BPT_ENOMEM.
 * ---------------------------------------------------------------------- */
int bpt_graph_set_vertex_order(bpt_graph* g, const uint32_t* rank);

/* Colour count the library uses for colors_per_batch = 0 on this graph for a
 * job of n_samples samples: the one bpt_tune_colors measured for jobs of this
 * size range, if any; otherwise the widest of 64, 32, 16, 8 that gives every
 * workgroup the fused kernel keeps resident on this GPU at least one batch
 * (a batch runs on one workgroup, and wider batches save row scans but no
 * coin work).  0 for a bad handle. */
uint32_t bpt_default_colors(const bpt_graph* g, uint64_t n_samples);

/* ------------------------------------------------------------------------
 * bpt_tune_colors - launch-shape autotuner.  Times the fused traversal of
 * sample ids 0 .. min(n_samples, 16 x 64 x resident workgroups) - 1 under
 * `seed` (HIP events, traversal plus CSR assembly; the best of two runs for
 * trials under 4 x 64 samples per resident workgroup) at 8, 16, ..., 1024
 * colours per batch, stopping once two widths in a row are at least 10%
 * slower than the fastest so far (after an untimed pilot when the graph has
 * no set-size history: it picks the workgroup size), then, at the fastest
 * width, with the colour
 * schedule of the expansion forced to per-coin discovery and to per-edge
 * gathering of live colours instead of the kernel's per-wavefront choice
 * (kept when 3% faster).  It remembers the result for this graph and jobs of
 * the same power-of-two size range as n_samples: later calls with
 * colors_per_batch = 0 (and bpt_default_colors) take the colour count, and
 * calls at that colour count take the schedule.  Which shape is fastest
 * depends on the graph and probabilities (dense sharing favours wide batches
 * and gathering, small jobs narrow ones); the sets never do.  Trials of wide
 * masks on large graphs allocate and free tens of GB of traversal slots.
 *
 * Returns the chosen colour count, or 0 on error (bpt_last_status():
 * BPT_EINVAL for a bad handle or n_samples outside [1, 2^34), or the errors
 * of bpt_sample_rrr).  Runs traversals on the graph's device and returns no
 * sets; safe to call concurrently with sampling calls on the same graph.
 * ---------------------------------------------------------------------- */
uint32_t bpt_tune_colors(bpt_graph* g, uint64_t n_samples, uint64_t seed);

/* Host builds of the library's own arithmetic, for checks on machines
 * without a GPU: the threshold of an fp32 probability, the coin word of
 * (seed, s, e) and the start vertex of sample s on n vertices, exactly as the
 * device computes them (definitions above). */
uint32_t bpt_thr32(float p);
uint32_t bpt_coin_word(uint64_t seed, uint64_t sample, uint64_t edge);
uint32_t bpt_start_vertex(uint64_t seed, uint64_t sample, uint32_t n);

/* Library version string. */
const char* bpt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BPT_H */
