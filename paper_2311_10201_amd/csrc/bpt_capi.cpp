// C ABI of libbpt: handles, error state, workspaces and the sampling driver.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "bpt.h"
#include "bpt_host.hpp"
#include "bpt_internal.hpp"
#include "bpt_lane.hpp"
#include "bpt_rng.hpp"

#define BPT_VERSION_STRING "libbpt 0.1 (gfx950)"

namespace bpt {
namespace {

constexpr uint32_t kGraphMagic = 0x42505447u;  // "BPTG"
constexpr uint32_t kRrrMagic = 0x42505452u;    // "BPTR"
constexpr uint32_t kPlanMagic = 0x4250504Cu;   // "BPPL"
constexpr uint32_t kDeadMagic = 0xDEADBEEFu;

thread_local int t_status = BPT_OK;
thread_local std::string t_message;

void set_status(int st, const std::string& msg) {
    t_status = st;
    t_message = msg;
}
void set_ok() {
    t_status = BPT_OK;
    t_message.clear();
}

struct HipFail {
    int status;
    std::string msg;
};

#define HIP_TRY(expr)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            throw HipFail{e_ == hipErrorOutOfMemory ? BPT_ENOMEM : BPT_EDEVICE,                  \
                          std::string(#expr) + ": " + hipGetErrorString(e_)};                    \
        }                                                                                        \
    } while (0)

template <typename T>
T* dev_alloc(size_t count) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    HIP_TRY(hipMalloc(&p, bytes));
    return static_cast<T*>(p);
}

void dev_free(void* p) {
    if (p) (void)hipFree(p);
}

// What bpt_tune_colors measured fastest for one job-size range of a graph:
// colours per batch and the colour schedule of the expansion (GatherMode).
struct TunedShape {
    uint32_t colors = 0;
    uint32_t gather = kGatherAuto;
};

// One set of traversal state + output staging; a call holds one exclusively.
struct Workspace {
    int nw = 0;  // colour words per mask (fused), 0 = unfused
    int block = 0;  // threads per workgroup of the fused launches it was sized for
    uint32_t slots = 0;
    bool full = false;  // as many slots as a launch on this device can use (or memory allows)
    void* slot_mem = nullptr;
    FusedSlots fs{};
    UnfusedSlots us{};
    Control* ctl = nullptr;
    Control* ctl_host = nullptr;  // pinned
    uint32_t* pool = nullptr;
    uint64_t pool_cap = 0;
    uint32_t* counts = nullptr;
    unsigned long long* where = nullptr;
    uint64_t sample_cap = 0;
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    unsigned long long* out_offsets = nullptr;  // host-API device output
    uint64_t out_offsets_cap = 0;
    uint32_t* out_vertices = nullptr;
    uint64_t out_vertices_cap = 0;
    // job table of multi-job launches: device copy, pinned host staging, totals
    FusedJob* d_jobs = nullptr;
    FusedJob* h_jobs = nullptr;
    unsigned long long* d_totals = nullptr;
    unsigned long long* h_totals = nullptr;
    uint32_t jobs_cap = 0;
    void* order_scratch = nullptr;  // sorted starts: keys, indices and sort temporaries
    size_t order_bytes = 0;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // traversal start, traversal end, finalize end
    // When a bpt_sample_rrr_device call ends in BPT_ERANGE its sets stay in
    // counts / where / pool; the retry with a larger buffer and the same
    // arguments only re-runs the CSR assembly.  Every other launch on the
    // workspace (another sampling call, a multi-job launch, a tuning trial)
    // clears this before it overwrites those arrays.
    bool have_last = false;
    uint64_t last_first = 0, last_samples = 0, last_seed = 0;
    uint32_t last_colors = 0;
    uint32_t last_flags = 0;
    bpt_counters last_counters{};

    ~Workspace() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        dev_free(slot_mem);
        dev_free(ctl);
        if (ctl_host) (void)hipHostFree(ctl_host);
        dev_free(pool);
        dev_free(counts);
        dev_free(where);
        dev_free(scratch);
        dev_free(out_offsets);
        dev_free(out_vertices);
        dev_free(d_jobs);
        dev_free(d_totals);
        dev_free(order_scratch);
        if (h_jobs) (void)hipHostFree(h_jobs);
        if (h_totals) (void)hipHostFree(h_totals);
    }
};

}  // namespace
}  // namespace bpt

struct bpt_graph {
    uint32_t magic;
    int device;
    int cus;
    uint64_t hbm;  // device memory, bytes
    uint32_t n;
    uint64_t m;
    uint32_t layout;
    uint32_t thr_uniform;
    uint32_t* d_rowptr;
    uint32_t* d_col;
    uint32_t* d_thr_row;
    uint32_t* d_thr_edge;
    std::mutex mu;
    std::vector<bpt::Workspace*> idle;
    bpt::TunedShape tuned[64];  // measured fastest for jobs of 2^i .. 2^(i+1)-1 samples (colors 0: none)
    double mean_members = 0;  // running mean set size of this graph's calls (0: none yet), sizes pools
    uint32_t* d_rank = nullptr;  // vertex order for sorted starts (null: vertex ids)
};

// A reusable, capturable sampling setup: a private workspace with its pool and
// per-sample arrays, and a one-entry device job table that the setup kernel
// fills at run time.
namespace bpt {
namespace {
// One launch of a multi-job plan: the jobs whose batches use `nw` mask words.
// Table entries 0 .. n_fused-1 (jobs with samples) are in the fused launch;
// every entry gets a CSR assembly and a result.
struct PlanGroup {
    int nw = 1;
    bpt_graph* owner = nullptr;       // the group's graph with the most vertices
    Workspace* ws = nullptr;          // its d_jobs / d_totals hold the group's table
    std::vector<bpt_job> jobs;        // as given at creation, table order
    std::vector<uint64_t> out_base;   // position of each job's first sample in counts / where
    uint32_t n_fused = 0;
    uint64_t n_batches = 0;
    uint32_t* d_ids = nullptr;        // the caller's index of each table entry
    unsigned long long* d_caps = nullptr;
};
}  // namespace
}  // namespace bpt

struct bpt_plan {
    uint32_t magic;
    bpt_graph* graph;  // single-job plan; null for a multi-job plan
    bpt::Workspace* ws;
    bpt::FusedJob* d_job;
    uint64_t max_samples;
    uint32_t colors;
    std::vector<bpt::PlanGroup> groups;  // multi-job plan
    uint32_t n_jobs = 0;
    int device = 0;
};

struct bpt_rrr {
    uint32_t magic;
    uint64_t num_samples;
    uint64_t total;
    uint64_t* offsets;
    uint32_t* vertices;
};

namespace bpt {
namespace {

bool valid_colors(uint32_t c) { return c >= 8 && c <= 1024 && (c & (c - 1)) == 0; }

// 64-bit mask words a batch of `colors` samples needs (batches below 64
// colours use part of one word).
int mask_words(uint32_t colors) { return (int)((colors + 63) / 64); }

int env_int(const char* name, int dflt) {
    const char* v = getenv(name);
    if (!v || !*v) return dflt;
    return atoi(v);
}

// Graphs whose sets average this many members or more (running mean over the
// graph's calls) get tail helping, the visited read before discovery
// fetch-ors, and 512-thread workgroups.
constexpr double kHelpMembers = 1024.0;

size_t fused_slot_bytes(uint32_t n, int nw);

// The graph has a set-size history and its sets are small.
bool light_sets(const bpt_graph* g) {
    if (!g) return false;
    std::lock_guard<std::mutex> lk(const_cast<bpt_graph*>(g)->mu);
    return g->mean_members > 0 && g->mean_members < kHelpMembers;
}

// Fused workers, one batch per workgroup: for masks of up to four words two
// 512-thread workgroups per CU (four wavefronts per SIMD), where a heavy batch
// finishing alone on its CU keeps more lanes; four 256-thread workgroups per
// CU for graphs whose sets are small (one-word masks: twice the batches in
// flight to hide the per-level latency of light, deep traversals; R-MAT 20 WC
// 3.11 -> 2.80 ms) and for wider masks, whose LDS staging is larger.  128-
// and 1024-thread instantiations exist for tuning (BPT_FUSED_BLOCK).
int fused_block(const bpt_graph* g, int nw) {
    const int bs = env_int("BPT_FUSED_BLOCK", 0);
    if (bs == 128 || bs == 256 || (bs == 512 && nw <= 4) || (bs == 1024 && nw == 1)) return bs;
    if (nw > 4) return 256;
    // the doubled slot count must stay cheap: at most a fifth of the device's memory
    // (R-MAT 20: 1,024 slots of 46 MB, 47 GB; not R-MAT 21 or 22), so that the
    // workspaces of several cached graphs still fit side by side
    return (nw == 1 && light_sets(g) && (uint64_t)g->cus * 4 * fused_slot_bytes(g->n, 1) <= g->hbm / 5) ? 256
                                                                                                    : 512;
}

// Workgroups of `bs` threads resident per CU (1024 threads per CU).
uint64_t fused_per_cu(int bs) { return (uint64_t)(1024 / bs); }

// Colour schedule of the fused expansion: chosen by the kernel per
// wavefront, measured by the tuner, or forced (BPT_GATHER=never|always|auto,
// for tests; the sets are the same).  -1: not forced.
int gather_forced() {
    const char* v = getenv("BPT_GATHER");
    if (v && !strcmp(v, "never")) return kGatherNever;
    if (v && !strcmp(v, "always")) return kGatherAlways;
    if (v && !strcmp(v, "auto")) return kGatherAuto;
    return -1;
}
uint32_t gather_mode() {
    const int f = gather_forced();
    return f >= 0 ? (uint32_t)f : kGatherAuto;
}

// Grid of a fused launch of `bs`-thread workgroups over `slots` slots.
int fused_grid(const bpt_graph* g, int bs, uint32_t slots, uint64_t n_batches) {
    uint64_t gsz = std::min<uint64_t>({(uint64_t)slots, (uint64_t)g->cus * fused_per_cu(bs), n_batches});
    const int cap = env_int("BPT_FUSED_SLOTS", 0);
    if (cap > 0) gsz = std::min<uint64_t>(gsz, (uint64_t)cap);
    return (int)std::max<uint64_t>(1, gsz);
}

DevGraph dev_graph(const bpt_graph* g) {
    DevGraph d;
    d.rowptr = g->d_rowptr;
    d.col = g->d_col;
    d.thr_row = g->d_thr_row;
    d.thr_edge = g->d_thr_edge;
    d.thr_uniform = g->thr_uniform;
    d.prob_layout = g->layout;
    d.n = g->n;
    d.m = (uint32_t)g->m;
    return d;
}

size_t fused_slot_bytes(uint32_t n, int nw) {
    const size_t N = n;
    size_t b = 0;
    b += N * mask_record_words(nw) * 8;  // visited and frontier masks (two levels), per vertex
    b += (nw > 1) ? N * 4 : 0;  // stamp
    b += 2 * N * 4;         // queue
    b += N * 4;             // touched
    b += bitmap_words(n) * 8;  // touched bitmap
    if (nw == 1) b += sizeof(HelpRec) + (size_t)kHelpStagePos * 6 * 4;  // help record and chunk staging
    return b;
}

// Lays out `slots` fused traversal slots for graphs of up to n vertices from
// `base` (256-byte aligned pieces) and returns the bytes they take; with a
// null base it only measures.  Everything in it must be zero before the first
// launch that uses it.
size_t carve_fused_slots(char* base, uint32_t n, int nw, uint32_t slots, FusedSlots* fs) {
    const size_t S = slots, N = n;
    const size_t words = bitmap_words(n);
    size_t off = 0;
    auto take = [&](size_t sz) {
        char* q = base ? base + off : nullptr;
        off += (sz + 255) & ~(size_t)255;
        return q;
    };
    FusedSlots f{};
    f.masks = reinterpret_cast<unsigned long long*>(take(S * N * mask_record_words(nw) * 8));
    f.stamp = reinterpret_cast<uint32_t*>(take(nw > 1 ? S * N * 4 : 4));
    f.queue = reinterpret_cast<uint32_t*>(take(S * 2 * N * 4));
    f.touched = reinterpret_cast<uint32_t*>(take(S * N * 4));
    f.tbits = reinterpret_cast<unsigned long long*>(take(S * words * 8));
    f.slot_tag = reinterpret_cast<uint32_t*>(take(S * 4));
    if (nw == 1) {
        f.help = reinterpret_cast<HelpRec*>(take(S * sizeof(HelpRec)));
        f.hstage = reinterpret_cast<uint32_t*>(take(S * kHelpStagePos * 6 * 4));
    }
    f.slots = slots;
    if (fs) *fs = f;
    return off;
}

size_t unfused_slot_bytes(uint32_t n) { return bitmap_words(n) * 8 + (size_t)n * 4; }

// Device memory a new workspace may take: 60% of what is free, at most
// 160 GB (BPT_WORKSPACE_FRACTION, 0 < f <= 0.9, sets the share).  Slots of
// wide masks on large graphs are the only ones this bounds: R-MAT 22 at 128
// colours needs 138 GB for a slot per resident workgroup.
size_t memory_budget() {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return (size_t)8 << 30;
    double fraction = 0.6;
    const char* v = getenv("BPT_WORKSPACE_FRACTION");
    const double f = v ? atof(v) : 0.0;
    if (f > 0.0 && f <= 0.9) fraction = f;
    return std::min((size_t)((double)free_b * fraction), (size_t)160 << 30);
}

// Allocates and zeroes the traversal state of a new workspace.
// Diagnostics on stderr when BPT_TRACE is set: workspace and pool growth.
bool trace_on() {
    static const bool on = getenv("BPT_TRACE") != nullptr;
    return on;
}

// Traversal slots a job of `units` batches (fused, in `block`-thread
// workgroups) or samples (unfused) can keep busy at once, rounded up to a
// power of two so that workspaces are reused across jobs of similar size.
uint64_t slots_wanted(const bpt_graph* g, int nw, uint64_t units, int block) {
    const uint64_t cap = nw > 0 ? (uint64_t)g->cus * fused_per_cu(block) : (uint64_t)g->cus * 16;
    uint64_t want = 1;
    while (want < units && want < cap) want <<= 1;
    return std::min(want, cap);
}

// block: threads per workgroup of its fused launches (0: fused_block's choice).
Workspace* make_workspace(bpt_graph* g, int nw, uint64_t units, int block = 0) {
    Workspace* ws = new Workspace();
    ws->nw = nw;
    try {
        const uint32_t n = g->n;
        const size_t budget = memory_budget();
        char* p;
        if (nw > 0) {
            const size_t per = fused_slot_bytes(n, nw) + 1024;
            ws->block = block > 0 ? block : fused_block(g, nw);
            const size_t device_max = (size_t)(g->cus * fused_per_cu(ws->block));
            const size_t mem_max = std::max<size_t>(1, budget / per);
            const size_t want = std::min<size_t>(slots_wanted(g, nw, units, ws->block), mem_max);
            ws->slots = (uint32_t)std::max<size_t>(1, want);
            ws->full = want >= device_max || want >= mem_max;
            const size_t bytes = carve_fused_slots(nullptr, n, nw, ws->slots, nullptr);
            ws->slot_mem = dev_alloc<char>(bytes);
            HIP_TRY(hipMemset(ws->slot_mem, 0, bytes));
            carve_fused_slots(static_cast<char*>(ws->slot_mem), n, nw, ws->slots, &ws->fs);
        } else {
            const size_t per = unfused_slot_bytes(n) + 512;
            const size_t device_max = (size_t)g->cus * 16;  // wavefronts
            const size_t mem_max = std::max<size_t>(4, budget / per);
            size_t want = std::min<size_t>(slots_wanted(g, 0, units, 0), mem_max);
            want = std::max<size_t>(4, want / 4 * 4);  // whole workgroups of 4 waves
            ws->slots = (uint32_t)want;
            ws->full = want >= device_max || want + 4 > mem_max;
            const size_t S = ws->slots;
            const size_t words = bitmap_words(n);
            size_t bytes = S * per + 1024;
            ws->slot_mem = dev_alloc<char>(bytes);
            HIP_TRY(hipMemset(ws->slot_mem, 0, bytes));
            p = static_cast<char*>(ws->slot_mem);
            ws->us.vbits = reinterpret_cast<unsigned long long*>(p);
            p += ((S * words * 8) + 255) & ~(size_t)255;
            ws->us.log = reinterpret_cast<uint32_t*>(p);
            ws->us.slots = ws->slots;
        }
        for (hipEvent_t& e : ws->ev) HIP_TRY(hipEventCreate(&e));
        if (trace_on())
            fprintf(stderr, "[libbpt] workspace n=%u nw=%d slots=%u full=%d\n", g->n, nw, ws->slots, (int)ws->full);
        ws->ctl = dev_alloc<Control>(1);
        HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&ws->ctl_host), sizeof(Control), hipHostMallocDefault));
        HIP_TRY(hipDeviceSynchronize());
    } catch (...) {
        delete ws;
        throw;
    }
    return ws;
}

// Frees the graph's idle workspaces (all, or all but those of kind `keep_nw`).
void trim_idle(bpt_graph* g, int keep_nw) {
    std::vector<Workspace*> drop;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        std::vector<Workspace*> keep;
        for (Workspace* ws : g->idle) (ws->nw == keep_nw ? keep : drop).push_back(ws);
        g->idle.swap(keep);
    }
    for (Workspace* ws : drop) delete ws;
}

// A workspace of kind `nw` for a job of `units` batches (fused) or samples
// (unfused): an idle one with enough slots, else a new one sized to the job
// (smaller idle ones of the same kind are then dropped).
Workspace* acquire(bpt_graph* g, int nw, uint64_t units) {
    const int block = nw > 0 ? fused_block(g, nw) : 0;
    const uint64_t want = slots_wanted(g, nw, units, block);
    std::vector<Workspace*> drop;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        for (size_t i = 0; i < g->idle.size(); ++i) {
            Workspace* ws = g->idle[i];
            // a workspace that keeps a failed call's sets (BPT_ERANGE) is taken whatever
            // its shape: the retry only re-assembles them
            if (ws->nw == nw && ((ws->block == block && (ws->slots >= want || ws->full)) || ws->have_last)) {
                g->idle.erase(g->idle.begin() + i);
                return ws;
            }
        }
        std::vector<Workspace*> keep;
        for (Workspace* ws : g->idle) (ws->nw == nw ? drop : keep).push_back(ws);
        g->idle.swap(keep);
    }
    for (Workspace* ws : drop) delete ws;
    try {
        return make_workspace(g, nw, units, block);
    } catch (const HipFail& f) {
        if (f.status != BPT_ENOMEM) throw;
        trim_idle(g, -1);  // out of device memory: drop cached workspaces of other kinds, retry once
        return make_workspace(g, nw, units, block);
    }
}

void release(bpt_graph* g, Workspace* ws) {
    std::lock_guard<std::mutex> lk(g->mu);
    g->idle.push_back(ws);
}


void ensure_sample_arrays(Workspace* ws, uint64_t n_samples) {
    if (ws->sample_cap < n_samples) {
        dev_free(ws->counts);
        dev_free(ws->where);
        ws->counts = nullptr;
        ws->where = nullptr;
        ws->sample_cap = 0;
        const uint64_t cap = std::max<uint64_t>(n_samples, 1024);
        ws->counts = dev_alloc<uint32_t>(cap);
        ws->where = dev_alloc<unsigned long long>(cap);
        ws->sample_cap = cap;
    }
    const size_t need = finalize_scratch_bytes(n_samples);
    if (ws->scratch_bytes < need) {
        dev_free(ws->scratch);
        ws->scratch = nullptr;
        ws->scratch_bytes = 0;
        ws->scratch = dev_alloc<char>(need);
        ws->scratch_bytes = need;
    }
}

void ensure_pool(bpt_graph* g, Workspace* ws, uint64_t entries) {
    if (ws->pool_cap >= entries) return;
    if (trace_on()) fprintf(stderr, "[libbpt] pool n=%u %llu -> %llu entries\n", g->n,
                            (unsigned long long)ws->pool_cap, (unsigned long long)entries);
    dev_free(ws->pool);
    dev_free(ws->out_vertices);
    ws->pool = nullptr;
    ws->pool_cap = 0;
    ws->out_vertices = nullptr;
    ws->out_vertices_cap = 0;
    try {
        ws->pool = dev_alloc<uint32_t>(entries);
    } catch (const HipFail& f) {
        if (f.status != BPT_ENOMEM) throw;
        trim_idle(g, -1);
        ws->pool = dev_alloc<uint32_t>(entries);
    }
    ws->pool_cap = entries;
}

// Pool entries expected for n_samples sets of graph g: its running mean set
// size with a margin, so that a launch rarely has to run again after an
// overflow; without history, 32 per set.
uint64_t pool_estimate(bpt_graph* g, uint64_t n_samples) {
    double mean;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        mean = g->mean_members;
    }
    const double per = mean > 0 ? mean * 1.3 : 32.0;
    const double est = std::min<double>((double)n_samples * per, (double)g->n * (double)n_samples);
    return (uint64_t)est + 1024;
}

// kJobReadFirst for jobs on this graph: sets of 1,024+ members on average,
// as for tail helping (BPT_READ_FIRST=0/1 forces it).
uint32_t job_flags(bpt_graph* g) {
    const int forced = env_int("BPT_READ_FIRST", -1);
    if (forced >= 0) return forced ? kJobReadFirst : 0u;
    std::lock_guard<std::mutex> lk(g->mu);
    return g->mean_members >= kHelpMembers ? kJobReadFirst : 0u;
}

// Helping (idle workgroups joining the batches still running at the end of a
// launch) pays when sets are large: batches have few, heavy levels and the
// launch ends on a tail of them.  Deep traversals of small sets lose time to
// it, so it is used once a graph's running mean set size reaches
// kHelpMembers; BPT_HELP=0 or 1 forces it.
bool help_wanted(bpt_graph* g) {
    const int forced = env_int("BPT_HELP", -1);
    if (forced >= 0) return forced != 0;
    std::lock_guard<std::mutex> lk(g->mu);
    return g->mean_members >= kHelpMembers;
}

void note_members(bpt_graph* g, uint64_t n_samples, uint64_t total) {
    if (!n_samples) return;
    const double m = (double)total / (double)n_samples;
    std::lock_guard<std::mutex> lk(g->mu);
    g->mean_members = g->mean_members > 0 ? 0.5 * g->mean_members + 0.5 * m : m;
}

void ensure_out(Workspace* ws, uint64_t n_samples, uint64_t entries) {
    if (ws->out_offsets_cap < n_samples + 1) {
        dev_free(ws->out_offsets);
        ws->out_offsets = nullptr;
        ws->out_offsets_cap = 0;
        ws->out_offsets = dev_alloc<unsigned long long>(n_samples + 1);
        ws->out_offsets_cap = n_samples + 1;
    }
    if (ws->out_vertices_cap < entries) {
        dev_free(ws->out_vertices);
        ws->out_vertices = nullptr;
        ws->out_vertices_cap = 0;
        ws->out_vertices = dev_alloc<uint32_t>(entries);
        ws->out_vertices_cap = entries;
    }
}

void ensure_jobs(Workspace* ws, uint32_t n_jobs) {
    if (ws->jobs_cap >= n_jobs) return;
    dev_free(ws->d_jobs);
    dev_free(ws->d_totals);
    if (ws->h_jobs) (void)hipHostFree(ws->h_jobs);
    if (ws->h_totals) (void)hipHostFree(ws->h_totals);
    ws->d_jobs = nullptr;
    ws->d_totals = nullptr;
    ws->h_jobs = nullptr;
    ws->h_totals = nullptr;
    ws->jobs_cap = 0;
    const uint32_t cap = std::max<uint32_t>(n_jobs, 64);
    ws->d_jobs = dev_alloc<FusedJob>(cap);
    ws->d_totals = dev_alloc<unsigned long long>(cap);
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&ws->h_jobs), cap * sizeof(FusedJob), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&ws->h_totals), cap * sizeof(unsigned long long),
                          hipHostMallocDefault));
    ws->jobs_cap = cap;
}

uint32_t gather_for(bpt_graph* g, uint64_t n_samples, uint32_t colors);

struct CallResult {
    uint64_t total = 0;
    bpt_counters counters{};
    bool discard_workspace = false;
};

void release_or_discard(bpt_graph* g, Workspace* ws, const CallResult& r) {
    if (r.discard_workspace) delete ws;
    else release(g, ws);
}

// Runs the traversal and the CSR assembly.  When `own_output` is set the
// result goes to the workspace's own device buffers (sized to fit).
// `retry_ok`: the caller is bpt_sample_rrr_device, whose retry after
// BPT_ERANGE may reuse the sets the failed call left in the workspace.
int run_sampling(bpt_graph* g, Workspace* ws, uint64_t first, uint64_t S, uint32_t colors, uint64_t seed,
                 uint32_t flags, hipStream_t stream, unsigned long long* d_offsets, uint32_t* d_vertices,
                 uint64_t capacity, bool own_output, bool retry_ok, CallResult* res, int gather = -1) {
    const bool unfused = (flags & BPT_FLAG_UNFUSED) != 0;
    const bool sorted = (flags & BPT_FLAG_SORTED_STARTS) != 0;
    const bool reuse = retry_ok && ws->have_last && ws->last_first == first && ws->last_samples == S &&
                       ws->last_seed == seed && ws->last_colors == colors && ws->last_flags == flags;
    if (reuse) {
        if (own_output) {
            ensure_out(ws, S, ws->pool_cap);
            d_offsets = ws->out_offsets;
            d_vertices = ws->out_vertices;
            capacity = ws->out_vertices_cap;
        }
        HIP_TRY(hipEventRecord(ws->ev[1], stream));
        HIP_TRY(launch_finalize(ws->counts, ws->where, ws->pool, S, d_offsets, d_vertices, capacity, &ws->ctl->total,
                                &ws->ctl->err,
                                ws->scratch, ws->scratch_bytes, stream));
        HIP_TRY(hipEventRecord(ws->ev[2], stream));
        HIP_TRY(hipMemcpyAsync(ws->ctl_host, ws->ctl, sizeof(Control), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        float ms_fin = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms_fin, ws->ev[1], ws->ev[2]));
        res->total = ws->ctl_host->total;
        res->counters = ws->last_counters;
        res->counters.traversal_ns = 0;  // no traversal ran
        res->counters.finalize_ns = (uint64_t)((double)ms_fin * 1e6);
        if (res->total > capacity) {
            set_status(BPT_ERANGE, "output capacity " + std::to_string(capacity) + " < " +
                                       std::to_string(res->total) + " members");
            return BPT_ERANGE;
        }
        ws->have_last = false;  // delivered: the next call traverses again
        return BPT_OK;
    }
    ws->have_last = false;
    ensure_sample_arrays(ws, S);
    ensure_pool(g, ws, std::max<uint64_t>(ws->pool_cap ? 0 : (1u << 20), pool_estimate(g, S)));
    for (int attempt = 0; attempt < 8; ++attempt) {
        if (own_output) {
            ensure_out(ws, S, ws->pool_cap);
            d_offsets = ws->out_offsets;
            d_vertices = ws->out_vertices;
            capacity = ws->out_vertices_cap;
        }
        HIP_TRY(hipMemsetAsync(ws->ctl, 0, sizeof(Control), stream));
        HIP_TRY(hipEventRecord(ws->ev[0], stream));
        int block = 256, grid = 1;
        Output out;
        out.counts = ws->counts;
        out.where = ws->where;
        out.pool = ws->pool;
        out.pool_cap = ws->pool_cap;
        if (!unfused) {
            const uint32_t* order = nullptr;
            if (sorted) {  // batches of samples with neighbouring start vertices
                const size_t need = order_scratch_bytes(S, g->n);
                if (ws->order_bytes < need) {
                    dev_free(ws->order_scratch);
                    ws->order_scratch = nullptr;
                    ws->order_bytes = 0;
                    ws->order_scratch = dev_alloc<char>(need);
                    ws->order_bytes = need;
                }
                HIP_TRY(launch_sort_by_start(g->n, seed, first, S, g->d_rank, ws->order_scratch, ws->order_bytes,
                                             &order, stream));
            }
            FusedArgs a = {};
            a.job0.order = order;
            a.job0.g = dev_graph(g);
            a.job0.seed = seed;
            a.job0.first_sample = first;
            a.job0.n_samples = S;
            a.job0.batch_begin = 0;
            a.job0.out_base = 0;
            a.job0.colors = colors;
            a.job0.flags = job_flags(g);
            a.jobs = nullptr;
            a.n_jobs = 1;
            a.n_max = g->n;
            a.ws = ws->fs;
            a.out = out;
            a.ctl = ws->ctl;
            a.n_batches = (S + colors - 1) / colors;
            a.gather_mode = gather >= 0 ? (uint32_t)gather : gather_for(g, S, colors);
            block = ws->block;
            grid = fused_grid(g, block, ws->slots, a.n_batches);
            HIP_TRY(launch_fused(a, ws->nw, block, grid, help_wanted(g), stream));
        } else {
            UnfusedArgs a;
            a.g = dev_graph(g);
            a.ws = ws->us;
            a.out = out;
            a.ctl = ws->ctl;
            a.seed = seed;
            a.first_sample = first;
            a.n_samples = S;
            const uint64_t blocks_needed = (S + 3) / 4;
            block = kUnfusedBlock;
            grid = (int)std::min<uint64_t>(ws->slots / 4, blocks_needed);
            HIP_TRY(launch_unfused(a, grid, stream));
        }
        HIP_TRY(hipEventRecord(ws->ev[1], stream));
        HIP_TRY(launch_finalize(ws->counts, ws->where, ws->pool, S, d_offsets, d_vertices, capacity, &ws->ctl->total,
                                &ws->ctl->err,
                                ws->scratch, ws->scratch_bytes, stream));
        HIP_TRY(hipEventRecord(ws->ev[2], stream));
        HIP_TRY(hipMemcpyAsync(ws->ctl_host, ws->ctl, sizeof(Control), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        const Control& c = *ws->ctl_host;
        if (c.err & kErrPoolOverflow) {
            const uint64_t need = c.pool_cursor + c.pool_cursor / 8 + 1024;
            ensure_pool(g, ws, need);
            continue;
        }
        if (c.err) {
            set_status(BPT_EINTERNAL, "device consistency check failed (error bits " + std::to_string(c.err) + ")");
            res->discard_workspace = true;  // its traversal state may not be clean
            return BPT_EINTERNAL;
        }
        res->total = c.total;
        note_members(g, S, c.total);
        bpt_counters& k = res->counters;
        k.samples = S;
        k.members = c.stats[kStatMembers];
        k.sample_edges = c.stats[kStatSampleEdges];
        k.edge_accesses = c.stats[kStatEdgeAccesses];
        k.frontier_entries = c.stats[kStatEntries];
        k.philox_blocks = c.stats[kStatPhilox];
        k.live_coins = c.stats[kStatLive];
        k.levels = c.stats[kStatLevels];
        k.max_levels = c.stats[kStatMaxLevels];
        k.batches = c.stats[kStatBatches];
        float ms_trav = 0.f, ms_fin = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms_trav, ws->ev[0], ws->ev[1]));
        HIP_TRY(hipEventElapsedTime(&ms_fin, ws->ev[1], ws->ev[2]));
        k.traversal_ns = (uint64_t)((double)ms_trav * 1e6);
        k.finalize_ns = (uint64_t)((double)ms_fin * 1e6);
        k.workgroup_size = (uint64_t)block;
        k.workgroups = (uint64_t)grid;
        if (c.total > capacity) {
            ws->have_last = true;  // keep the sets for the caller's retry
            ws->last_first = first;
            ws->last_samples = S;
            ws->last_seed = seed;
            ws->last_colors = colors;
            ws->last_flags = flags;
            ws->last_counters = k;
            set_status(BPT_ERANGE, "output capacity " + std::to_string(capacity) + " < " + std::to_string(c.total) +
                                       " members");
            return BPT_ERANGE;
        }
        return BPT_OK;
    }
    set_status(BPT_ENOMEM, "output pool kept overflowing");
    return BPT_ENOMEM;
}

bpt_graph* check_graph(const void* h) {
    if (!h) return nullptr;
    const bpt_graph* g = static_cast<const bpt_graph*>(h);
    return g->magic == kGraphMagic ? const_cast<bpt_graph*>(g) : nullptr;
}

// One fused launch over several jobs (bpt_sample_rrr_jobs): the batches of
// all jobs form one list that the persistent workgroups claim from a device
// counter; each job's sets are then assembled into its own buffers.  `owner`
// is the job graph with the most vertices: its workspace's slots are large
// enough for every job.  Jobs with no samples are not in `live`.
int run_jobs(bpt_graph* owner, Workspace* ws, bpt_job* jobs, const std::vector<uint32_t>& live,
             const std::vector<uint32_t>& colors, hipStream_t stream, bpt_counters* counters) {
    const uint32_t J = (uint32_t)live.size();
    ws->have_last = false;  // counts, where and pool are overwritten below
    ensure_jobs(ws, J);
    uint64_t n_batches = 0, total_samples = 0;
    for (uint32_t i = 0; i < J; ++i) {
        const bpt_job& jb = jobs[live[i]];
        FusedJob& fj = ws->h_jobs[i];
        fj = FusedJob{};
        fj.g = dev_graph(jb.graph);
        fj.seed = jb.seed;
        fj.first_sample = jb.first_sample;
        fj.n_samples = jb.n_samples;
        fj.batch_begin = n_batches;
        fj.out_base = total_samples;
        fj.colors = colors[live[i]];
        fj.flags = job_flags(jb.graph);
        n_batches += (jb.n_samples + fj.colors - 1) / fj.colors;
        total_samples += jb.n_samples;
    }
    ensure_sample_arrays(ws, total_samples);
    {
        uint64_t est = 0;
        for (uint32_t i = 0; i < J; ++i) est += pool_estimate(jobs[live[i]].graph, jobs[live[i]].n_samples);
        ensure_pool(owner, ws, std::max<uint64_t>(ws->pool_cap ? 0 : (1u << 20), est));
    }
    for (int attempt = 0; attempt < 8; ++attempt) {
        HIP_TRY(hipMemsetAsync(ws->ctl, 0, sizeof(Control), stream));
        HIP_TRY(hipMemcpyAsync(ws->d_jobs, ws->h_jobs, J * sizeof(FusedJob), hipMemcpyHostToDevice, stream));
        HIP_TRY(hipEventRecord(ws->ev[0], stream));
        FusedArgs a = {};
        a.jobs = ws->d_jobs;
        a.n_jobs = J;
        a.n_max = owner->n;
        a.ws = ws->fs;
        a.out.counts = ws->counts;
        a.out.where = ws->where;
        a.out.pool = ws->pool;
        a.out.pool_cap = ws->pool_cap;
        a.ctl = ws->ctl;
        a.n_batches = n_batches;
        a.gather_mode = gather_mode();
        int block = 256, grid = 1;
        block = ws->block;
        grid = fused_grid(owner, block, ws->slots, n_batches);
        bool help = false;
        for (uint32_t i = 0; i < J; ++i) help = help || help_wanted(jobs[live[i]].graph);
        HIP_TRY(launch_fused(a, ws->nw, block, grid, help, stream));
        HIP_TRY(hipEventRecord(ws->ev[1], stream));
        for (uint32_t i = 0; i < J; ++i) {
            const bpt_job& jb = jobs[live[i]];
            const uint64_t base = ws->h_jobs[i].out_base;
            HIP_TRY(launch_finalize(ws->counts + base, ws->where + base, ws->pool, jb.n_samples,
                                    reinterpret_cast<unsigned long long*>(jb.d_offsets), jb.d_vertices, jb.capacity,
                                    ws->d_totals + i, &ws->ctl->err, ws->scratch, ws->scratch_bytes, stream));
        }
        HIP_TRY(hipEventRecord(ws->ev[2], stream));
        HIP_TRY(hipMemcpyAsync(ws->ctl_host, ws->ctl, sizeof(Control), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipMemcpyAsync(ws->h_totals, ws->d_totals, J * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                               stream));
        HIP_TRY(hipStreamSynchronize(stream));
        const Control& c = *ws->ctl_host;
        if (c.err & kErrPoolOverflow) {
            ensure_pool(owner, ws, c.pool_cursor + c.pool_cursor / 8 + 1024);
            continue;
        }
        if (c.err) {
            set_status(BPT_EINTERNAL, "device consistency check failed (error bits " + std::to_string(c.err) + ")");
            return BPT_EINTERNAL;
        }
        int rc = BPT_OK;
        for (uint32_t i = 0; i < J; ++i) {
            bpt_job& jb = jobs[live[i]];
            jb.total = ws->h_totals[i];
            note_members(jb.graph, jb.n_samples, jb.total);
            jb.status = jb.total > jb.capacity ? BPT_ERANGE : BPT_OK;
            if (jb.status != BPT_OK) rc = BPT_ERANGE;
        }
        if (counters) {
            bpt_counters& k = *counters;
            k = bpt_counters{};
            k.samples = total_samples;
            k.members = c.stats[kStatMembers];
            k.sample_edges = c.stats[kStatSampleEdges];
            k.edge_accesses = c.stats[kStatEdgeAccesses];
            k.frontier_entries = c.stats[kStatEntries];
            k.philox_blocks = c.stats[kStatPhilox];
            k.live_coins = c.stats[kStatLive];
            k.levels = c.stats[kStatLevels];
            k.max_levels = c.stats[kStatMaxLevels];
            k.batches = c.stats[kStatBatches];
            float ms_trav = 0.f, ms_fin = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms_trav, ws->ev[0], ws->ev[1]));
            HIP_TRY(hipEventElapsedTime(&ms_fin, ws->ev[1], ws->ev[2]));
            k.traversal_ns = (uint64_t)((double)ms_trav * 1e6);
            k.finalize_ns = (uint64_t)((double)ms_fin * 1e6);
            k.workgroup_size = (uint64_t)block;
            k.workgroups = (uint64_t)grid;
        }
        if (rc != BPT_OK) set_status(rc, "a job's output capacity is below its total (see the job's total)");
        return rc;
    }
    set_status(BPT_ENOMEM, "output pool kept overflowing");
    return BPT_ENOMEM;
}

// Colours per batch when the caller leaves the choice to the library: the
// width bpt_tune_colors measured fastest for jobs of this size, if any; else
// the widest of 64, 32, 16, 8 colours that still gives every resident
// workgroup a batch (coins are flipped per (edge, colour), so wider batches
// save row scans but no Philox work, while a batch occupies one workgroup).
int size_bucket(uint64_t n_samples) { return n_samples ? 63 - __builtin_clzll(n_samples) : 0; }

uint64_t fused_resident(const bpt_graph* g) { return (uint64_t)g->cus * fused_per_cu(fused_block(g, 1)); }

// The colour schedule of a call: forced by BPT_GATHER, else the one the tuner
// measured with these colours for this job size, else the kernel's choice.
uint32_t gather_for(bpt_graph* g, uint64_t n_samples, uint32_t colors) {
    const int f = gather_forced();
    if (f >= 0) return (uint32_t)f;
    std::lock_guard<std::mutex> lk(g->mu);
    const TunedShape& t = g->tuned[size_bucket(n_samples)];
    return t.colors == colors ? t.gather : kGatherAuto;
}

uint32_t choose_colors(bpt_graph* g, uint64_t n_samples) {
    {
        std::lock_guard<std::mutex> lk(g->mu);
        const uint32_t t = g->tuned[size_bucket(n_samples)].colors;
        if (t) return t;
    }
    const uint64_t resident = fused_resident(g);
    for (uint32_t c = 64; c > 8; c >>= 1)
        if ((n_samples + c - 1) / c >= resident) return c;
    return 8;
}

}  // namespace

// ---------------------------------------------------------------------------
// Lanes: pipelined chunk launches of the serving loop (bpt_lane.hpp).
// ---------------------------------------------------------------------------
struct Lane {
    int device = 0;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    Workspace* ws = nullptr;
    uint32_t ws_n = 0;          // vertices per slot of ws
    uint64_t pool_floor = 0;    // pool entries the last overflow showed to be needed
    bool pending = false;       // a launch was enqueued and not yet waited for
    FinSeg* h_seg = nullptr;    // CSR assembly table of the launch (pinned host, device)
    FinSeg* d_seg = nullptr;
    uint32_t seg_cap = 0;
    void* fin_scratch = nullptr;  // partial sums of the segmented assembly
    size_t fin_bytes = 0;
};

Lane* lane_create(int device, std::string* why) {
    Lane* l = new (std::nothrow) Lane();
    if (!l) {
        *why = "host allocation failed";
        return nullptr;
    }
    l->device = device;
    if (hipSetDevice(device) != hipSuccess ||
        hipStreamCreateWithFlags(&l->stream, hipStreamNonBlocking) != hipSuccess ||  // default priority
        hipEventCreateWithFlags(&l->done, hipEventDisableTiming) != hipSuccess) {
        *why = "stream or event creation failed";
        lane_destroy(l);
        return nullptr;
    }
    return l;
}

void lane_destroy(Lane* l) {
    if (!l) return;
    if (l->stream) (void)hipStreamSynchronize(l->stream);
    delete l->ws;
    if (l->h_seg) (void)hipHostFree(l->h_seg);
    dev_free(l->d_seg);
    dev_free(l->fin_scratch);
    if (l->done) (void)hipEventDestroy(l->done);
    if (l->stream) (void)hipStreamDestroy(l->stream);
    delete l;
}

hipStream_t lane_stream(Lane* l) { return l->stream; }
hipEvent_t lane_done(Lane* l) { return l->done; }

bool lane_finished(Lane* l) { return !l->pending || hipEventQuery(l->done) == hipSuccess; }

uint32_t lane_slots(const Lane* l) { return l->ws ? l->ws->slots : 0u; }

int lane_launch(Lane* l, const LaneChunk* chunks, uint32_t n, hipEvent_t after, std::string* why) {
    if (l->pending) {
        *why = "the lane's previous launch was not waited for";
        return BPT_EINVAL;
    }
    if (n == 0) return BPT_OK;
    try {
        HIP_TRY(hipSetDevice(l->device));
        bpt_graph* owner = nullptr;
        uint64_t n_batches = 0, total_samples = 0, est = 0;
        for (uint32_t i = 0; i < n; ++i) {
            const LaneChunk& c = chunks[i];
            if (!valid_colors(c.colors) || c.colors > 64 || c.n_samples == 0) {
                *why = "lane chunks take 8 to 64 colours and at least one sample";
                return BPT_EINVAL;
            }
            if (!owner || c.graph->n > owner->n) owner = c.graph;
            n_batches += (c.n_samples + c.colors - 1) / c.colors;
            total_samples += c.n_samples;
            est += pool_estimate(c.graph, c.n_samples);
        }
        if (!l->ws || l->ws_n < owner->n) {  // slots for the largest graph so far, as many as the GPU keeps resident
            delete l->ws;
            l->ws = nullptr;
            // 512-thread workgroups whatever the graphs: a lane's launches are bounded
            // chunks, and its slots are sized for the largest graph it has seen
            l->ws = make_workspace(owner, 1, ~0ull >> 1, 512);
            l->ws_n = owner->n;
        }
        Workspace* ws = l->ws;
        ensure_sample_arrays(ws, total_samples);
        ensure_jobs(ws, n);
        if (ws->pool_cap < std::max(est, l->pool_floor)) ensure_pool(owner, ws, std::max(est, l->pool_floor) * 2);
        if (l->seg_cap < n) {
            if (l->h_seg) (void)hipHostFree(l->h_seg);
            dev_free(l->d_seg);
            l->h_seg = nullptr;
            l->d_seg = nullptr;
            l->seg_cap = 0;
            const uint32_t cap = std::max<uint32_t>(n, 64);
            HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&l->h_seg), cap * sizeof(FinSeg), hipHostMallocDefault));
            l->d_seg = dev_alloc<FinSeg>(cap);
            l->seg_cap = cap;
        }
        uint64_t b = 0, base = 0, tiles = 0;
        for (uint32_t i = 0; i < n; ++i) {
            const LaneChunk& c = chunks[i];
            FinSeg& sg = l->h_seg[i];
            sg.count_base = base;
            sg.n = c.n_samples;
            sg.tile_base = tiles;
            sg.offsets = c.d_offsets;
            sg.vertices = c.d_vertices;
            sg.capacity = c.capacity;
            sg.total = c.d_total;
            tiles += finalize_tiles(c.n_samples);
            FusedJob& fj = ws->h_jobs[i];
            fj = FusedJob{};
            fj.g = dev_graph(c.graph);
            fj.seed = c.seed;
            fj.first_sample = c.first_sample;
            fj.n_samples = c.n_samples;
            fj.batch_begin = b;
            fj.out_base = base;
            fj.colors = c.colors;
            fj.flags = job_flags(c.graph);
            b += (c.n_samples + c.colors - 1) / c.colors;
            base += c.n_samples;
        }
        if (l->fin_bytes < tiles * sizeof(unsigned long long)) {
            dev_free(l->fin_scratch);
            l->fin_scratch = nullptr;
            l->fin_bytes = 0;
            const size_t bytes = std::max<size_t>(tiles * 2 * sizeof(unsigned long long), 4096);
            l->fin_scratch = dev_alloc<char>(bytes);
            l->fin_bytes = bytes;
        }
        HIP_TRY(hipMemsetAsync(ws->ctl, 0, sizeof(Control), l->stream));
        HIP_TRY(hipMemcpyAsync(ws->d_jobs, ws->h_jobs, n * sizeof(FusedJob), hipMemcpyHostToDevice, l->stream));
        HIP_TRY(hipMemcpyAsync(l->d_seg, l->h_seg, n * sizeof(FinSeg), hipMemcpyHostToDevice, l->stream));
        FusedArgs a = {};
        a.jobs = ws->d_jobs;
        a.n_jobs = n;
        a.n_max = l->ws_n;
        a.ws = ws->fs;
        a.out.counts = ws->counts;
        a.out.where = ws->where;
        a.out.pool = ws->pool;
        a.out.pool_cap = ws->pool_cap;
        a.ctl = ws->ctl;
        a.n_batches = n_batches;
        a.gather_mode = gather_mode();
        int block = 0, grid = 0;
        block = ws->block;
        grid = fused_grid(owner, block, ws->slots, n_batches);
        // no tail helping: idle workgroups leave at once, so that the next
        // launch (on the other lane) takes their place while this one drains
        HIP_TRY(launch_fused(a, 1, block, grid, false, l->stream));
        if (after) HIP_TRY(hipStreamWaitEvent(l->stream, after, 0));
        HIP_TRY(launch_finalize_segments(ws->counts, ws->where, ws->pool, total_samples, l->d_seg, n, tiles,
                                         &ws->ctl->err, l->fin_scratch, l->fin_bytes, l->stream));
        HIP_TRY(hipMemcpyAsync(ws->ctl_host, ws->ctl, sizeof(Control), hipMemcpyDeviceToHost, l->stream));
        HIP_TRY(hipEventRecord(l->done, l->stream));
        l->pending = true;
        return BPT_OK;
    } catch (const HipFail& f) {
        *why = f.msg;
        return f.status;
    } catch (const std::bad_alloc&) {
        *why = "host allocation failed";
        return BPT_ENOMEM;
    }
}

int lane_wait(Lane* l, bool* overflow, std::string* why) {
    *overflow = false;
    if (!l->pending) return BPT_OK;
    l->pending = false;
    const hipError_t e = hipEventSynchronize(l->done);
    if (e != hipSuccess) {
        *why = std::string("hipEventSynchronize: ") + hipGetErrorString(e);
        return BPT_EDEVICE;
    }
    const Control& c = *l->ws->ctl_host;
    if (c.err & kErrPoolOverflow) {
        *overflow = true;
        l->pool_floor = c.pool_cursor + c.pool_cursor / 8 + 1024;
    }
    if (c.err & ~(unsigned)kErrPoolOverflow) {
        *why = "device consistency check failed (error bits " + std::to_string(c.err) + ")";
        delete l->ws;  // its traversal state may not be clean
        l->ws = nullptr;
        l->ws_n = 0;
        return BPT_EINTERNAL;
    }
    return BPT_OK;
}

size_t max_cover_scratch(uint64_t n_sets, uint32_t n, uint32_t k, uint64_t total) {
    return max_cover_scratch_bytes(n_sets, n, k, total);
}

int max_cover_run(const uint64_t* d_offsets, const uint32_t* d_vertices, uint64_t n_sets, uint32_t n, uint32_t k,
                  hipStream_t st, uint32_t* seeds, uint64_t* gains, void* scratch, size_t scratch_bytes,
                  std::string* why) {
    if (!d_offsets || !seeds || !gains || n == 0 || k > n || n_sets >= (1ull << 32)) {
        *why = "d_offsets, seeds and gains are required; 1 <= n, k <= n, n_sets < 2^32";
        return BPT_EINVAL;
    }
    if (k == 0) return BPT_OK;
    try {
        uint64_t total = 0;
        HIP_TRY(hipMemcpyAsync(&total, d_offsets + n_sets, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (total > 0 && !d_vertices) {
            *why = "d_vertices is required when the sets have members";
            return BPT_EINVAL;
        }
        if (scratch_bytes < max_cover_scratch_bytes(n_sets, n, k, total)) {
            *why = "coverage scratch too small for " + std::to_string(total) + " members";
            return BPT_EINVAL;
        }
        uint32_t* seeds_dev = nullptr;
        unsigned long long* gains_dev = nullptr;
        unsigned int* bad_dev = nullptr;
        HIP_TRY(launch_max_cover(d_offsets, d_vertices, n_sets, total, n, k, scratch, &seeds_dev, &gains_dev,
                                 &bad_dev, st));
        unsigned int bad = 0;
        HIP_TRY(hipMemcpyAsync(seeds, seeds_dev, (size_t)k * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(gains, gains_dev, (size_t)k * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(&bad, bad_dev, sizeof(bad), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (bad) {
            *why = (bad & kCoverBadOffsets) ? "offsets are not a CSR of the vertex array" : "a set member is >= n";
            return BPT_EINVAL;
        }
    } catch (const HipFail& f) {
        *why = f.msg;
        return f.status;
    }
    return BPT_OK;
}

}  // namespace bpt

using namespace bpt;

extern "C" {

bpt_graph* bpt_create_graph(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst, const float* prob) {
    HostCsr csr;
    std::string why;
    const int st = build_host_csr(n, m, src, dst, prob, &csr, &why);
    if (st != BPT_OK) {
        set_status(st, why);
        return nullptr;
    }
    bpt_graph* g = nullptr;
    try {
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, dev));
        if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            set_status(BPT_EDEVICE, std::string("libbpt is built for gfx950; device is ") + prop.gcnArchName);
            return nullptr;
        }
        g = new bpt_graph();
        g->magic = kGraphMagic;
        g->device = dev;
        g->cus = prop.multiProcessorCount;
        g->hbm = prop.totalGlobalMem;
        g->n = n;
        g->m = m;
        g->layout = csr.layout;
        g->thr_uniform = csr.thr_uniform;
        g->d_rowptr = dev_alloc<uint32_t>(csr.rowptr.size());
        g->d_col = dev_alloc<uint32_t>(csr.col.size());
        HIP_TRY(hipMemcpy(g->d_rowptr, csr.rowptr.data(), csr.rowptr.size() * 4, hipMemcpyHostToDevice));
        if (!csr.col.empty())
            HIP_TRY(hipMemcpy(g->d_col, csr.col.data(), csr.col.size() * 4, hipMemcpyHostToDevice));
        if (csr.layout == BPT_PROB_ROW) {
            g->d_thr_row = dev_alloc<uint32_t>(csr.thr_row.size());
            HIP_TRY(hipMemcpy(g->d_thr_row, csr.thr_row.data(), csr.thr_row.size() * 4, hipMemcpyHostToDevice));
        } else if (csr.layout == BPT_PROB_EDGE) {
            g->d_thr_edge = dev_alloc<uint32_t>(csr.thr_edge.size());
            HIP_TRY(hipMemcpy(g->d_thr_edge, csr.thr_edge.data(), csr.thr_edge.size() * 4, hipMemcpyHostToDevice));
        }
    } catch (const HipFail& f) {
        if (g) {
            g->magic = kGraphMagic;
            bpt_free(g);
        }
        set_status(f.status, f.msg);
        return nullptr;
    } catch (const std::bad_alloc&) {
        if (g) bpt_free(g);
        set_status(BPT_ENOMEM, "host allocation failed");
        return nullptr;
    }
    set_ok();
    return g;
}

int bpt_sample_rrr_device(bpt_graph* g, uint64_t first_sample, uint64_t n_samples, uint32_t colors_per_batch,
                          uint64_t seed, uint32_t flags, void* stream, uint64_t* d_offsets, uint32_t* d_vertices,
                          uint64_t capacity, uint64_t* total_out, bpt_counters* counters) {
    bpt_graph* gg = check_graph(g);
    if (!gg) {
        set_status(BPT_EINVAL, "not a bpt_graph handle");
        return BPT_EINVAL;
    }
    if (!total_out || !d_offsets || (!d_vertices && capacity > 0)) {
        set_status(BPT_EINVAL, "d_offsets and total_out are required (d_vertices when capacity > 0)");
        return BPT_EINVAL;
    }
    if ((flags & ~(BPT_FLAG_UNFUSED | BPT_FLAG_SORTED_STARTS)) ||
        ((flags & BPT_FLAG_SORTED_STARTS) && ((flags & BPT_FLAG_UNFUSED) || n_samples >= (1ull << 31)))) {
        set_status(BPT_EINVAL, "unknown flag bits, or sorted starts with the unfused traversal or >= 2^31 samples");
        return BPT_EINVAL;
    }
    const bool unfused = (flags & BPT_FLAG_UNFUSED) != 0;
    uint32_t colors = colors_per_batch;
    if (!unfused) {
        if (colors == 0) colors = choose_colors(gg, n_samples);
        if (!valid_colors(colors)) {
            set_status(BPT_EINVAL, "colors_per_batch must be 0 or a power of two from 8 to 1024");
            return BPT_EINVAL;
        }
    }
    if (n_samples >= kMaxSamples || first_sample >= kMaxSamples || first_sample + n_samples > kMaxSamples) {
        set_status(BPT_EINVAL, "sample ids must stay below 2^34");
        return BPT_EINVAL;
    }
    Workspace* ws = nullptr;
    try {
        HIP_TRY(hipSetDevice(gg->device));
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (n_samples == 0) {
            HIP_TRY(hipMemsetAsync(d_offsets, 0, sizeof(uint64_t), st));
            HIP_TRY(hipStreamSynchronize(st));
            *total_out = 0;
            if (counters) memset(counters, 0, sizeof(*counters));
            set_ok();
            return BPT_OK;
        }
        ws = acquire(gg, unfused ? 0 : mask_words(colors), unfused ? n_samples : (n_samples + colors - 1) / colors);
        CallResult res;
        const int rc = run_sampling(gg, ws, first_sample, n_samples, colors, seed, flags, st,
                                    reinterpret_cast<unsigned long long*>(d_offsets), d_vertices, capacity, false,
                                    true, &res);
        release_or_discard(gg, ws, res);
        ws = nullptr;
        if (rc == BPT_OK || rc == BPT_ERANGE) {
            *total_out = res.total;
            if (counters) *counters = res.counters;
        }
        if (rc == BPT_OK) set_ok();
        return rc;
    } catch (const HipFail& f) {
        if (ws) release(gg, ws);
        set_status(f.status, f.msg);
        return f.status;
    } catch (const std::bad_alloc&) {
        if (ws) release(gg, ws);
        set_status(BPT_ENOMEM, "host allocation failed");
        return BPT_ENOMEM;
    }
}

int bpt_sample_rrr_noalloc(bpt_graph* g, uint64_t first_sample, uint64_t n_samples, uint32_t colors_per_batch,
                           uint64_t seed, void* stream, uint64_t* d_offsets, uint32_t* d_vertices, uint64_t capacity,
                           uint64_t* total_out) {
    bpt_graph* gg = check_graph(g);
    if (!gg) {
        set_status(BPT_EINVAL, "not a bpt_graph handle");
        return BPT_EINVAL;
    }
    if (!total_out || !d_offsets || (!d_vertices && capacity > 0)) {
        set_status(BPT_EINVAL, "d_offsets and total_out are required (d_vertices when capacity > 0)");
        return BPT_EINVAL;
    }
    if (n_samples >= kMaxSamples || first_sample >= kMaxSamples || first_sample + n_samples > kMaxSamples) {
        set_status(BPT_EINVAL, "sample ids must stay below 2^34");
        return BPT_EINVAL;
    }
    const uint32_t colors = colors_per_batch ? colors_per_batch : choose_colors(gg, n_samples);
    if (!valid_colors(colors)) {
        set_status(BPT_EINVAL, "colors_per_batch must be 0 or a power of two from 8 to 1024");
        return BPT_EINVAL;
    }
    // the fixed part of the scratch: control block, per-sample counts and pool
    // positions, the CSR scan's temporaries; traversal slots and the member
    // pool share the rest
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t ctl_b = up(sizeof(Control));
    const size_t counts_b = up(n_samples * 4), where_b = up(n_samples * 8);
    const size_t fin_b = up(finalize_scratch_bytes(n_samples));
    const size_t fixed = ctl_b + counts_b + where_b + fin_b;
    const int nw = mask_words(colors);
    const size_t per_slot = carve_fused_slots(nullptr, gg->n, nw, 1, nullptr);
    if (fixed + per_slot + 1024 > kNoAllocScratchBytes) {
        set_status(BPT_ENOMEM, "this call needs " + std::to_string(fixed + per_slot + 1024) +
                                   " bytes of scratch (samples, graph size and colours) but the fixed scratch holds " +
                                   std::to_string(kNoAllocScratchBytes));
        return BPT_ENOMEM;
    }
    try {
        HIP_TRY(hipSetDevice(gg->device));
        hipStream_t st = static_cast<hipStream_t>(stream);
        void* base_v = nullptr;
        HIP_TRY(noalloc_scratch(gg->device, &base_v));
        char* base = static_cast<char*>(base_v);
        // calls in this process share the device's scratch: one at a time
        static std::mutex call_mu;
        std::lock_guard<std::mutex> lk(call_mu);
        if (n_samples == 0) {
            HIP_TRY(launch_zero_fill(base, 256, st));  // offsets[0] = 0 through a kernel, no allocation
            HIP_TRY(hipMemcpyAsync(d_offsets, base, sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
            HIP_TRY(hipStreamSynchronize(st));
            *total_out = 0;
            set_ok();
            return BPT_OK;
        }
        Control* ctl = reinterpret_cast<Control*>(base);
        uint32_t* counts = reinterpret_cast<uint32_t*>(base + ctl_b);
        unsigned long long* where = reinterpret_cast<unsigned long long*>(base + ctl_b + counts_b);
        void* fin = base + ctl_b + counts_b + where_b;
        char* slot_base = base + fixed;
        const uint64_t n_batches = (n_samples + colors - 1) / colors;
        const int block_sz = fused_block(gg, nw);
        const uint64_t device_slots = (uint64_t)gg->cus * fused_per_cu(block_sz);
        uint64_t pool_want = pool_estimate(gg, n_samples);
        for (int attempt = 0; attempt < 4; ++attempt) {
            const size_t room = kNoAllocScratchBytes - fixed;
            uint64_t slots = std::min<uint64_t>(device_slots, n_batches);
            const size_t pool_bytes_want = up(pool_want * 4);
            slots = pool_bytes_want + per_slot <= room ? std::min<uint64_t>(slots, (room - pool_bytes_want) / per_slot)
                                                       : 1;
            slots = std::max<uint64_t>(slots, 1);
            const size_t slot_bytes = carve_fused_slots(nullptr, gg->n, nw, (uint32_t)slots, nullptr);
            if (slot_bytes + 1024 > room) slots = 1;
            FusedSlots fs{};
            const size_t used = carve_fused_slots(slot_base, gg->n, nw, (uint32_t)slots, &fs);
            uint32_t* pool = reinterpret_cast<uint32_t*>(slot_base + used);
            const uint64_t pool_cap = (room - used) / 4;
            if (pool_cap < pool_want && attempt > 0) {
                set_status(BPT_ENOMEM, "the sets of this call take " + std::to_string(pool_want) +
                                           " vertex ids; the fixed scratch has room for " + std::to_string(pool_cap));
                return BPT_ENOMEM;
            }
            // the control block and the traversal slots start at zero
            HIP_TRY(launch_zero_fill(ctl, ctl_b, st));
            HIP_TRY(launch_zero_fill(slot_base, used, st));
            FusedArgs a = {};
            a.job0.g = dev_graph(gg);
            a.job0.seed = seed;
            a.job0.first_sample = first_sample;
            a.job0.n_samples = n_samples;
            a.job0.colors = colors;
            a.job0.flags = job_flags(gg);
            a.n_jobs = 1;
            a.n_max = gg->n;
            a.ws = fs;
            a.out.counts = counts;
            a.out.where = where;
            a.out.pool = pool;
            a.out.pool_cap = pool_cap;
            a.ctl = ctl;
            a.n_batches = n_batches;
            a.gather_mode = gather_for(gg, n_samples, colors);
            int block = 0, grid = 0;
            block = block_sz;
            grid = fused_grid(gg, block, (uint32_t)slots, n_batches);
            HIP_TRY(launch_fused(a, nw, block, grid, help_wanted(gg), st));
            HIP_TRY(launch_finalize(counts, where, pool, n_samples, reinterpret_cast<unsigned long long*>(d_offsets),
                                    d_vertices, capacity, &ctl->total, &ctl->err, fin, fin_b, st));
            Control c;
            HIP_TRY(hipMemcpyAsync(&c, ctl, sizeof(Control), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            if (c.err & kErrPoolOverflow) {  // fewer slots, a larger pool
                pool_want = c.pool_cursor + c.pool_cursor / 16 + 1024;
                continue;
            }
            if (c.err) {
                set_status(BPT_EINTERNAL, "device consistency check failed (error bits " + std::to_string(c.err) + ")");
                return BPT_EINTERNAL;
            }
            note_members(gg, n_samples, c.total);
            *total_out = c.total;
            if (c.total > capacity) {
                set_status(BPT_ERANGE, "output capacity " + std::to_string(capacity) + " < " +
                                           std::to_string(c.total) + " members");
                return BPT_ERANGE;
            }
            set_ok();
            return BPT_OK;
        }
        set_status(BPT_ENOMEM, "the sets of this call do not fit the fixed scratch");
        return BPT_ENOMEM;
    } catch (const HipFail& f) {
        set_status(f.status, f.msg);
        return f.status;
    }
}

int bpt_sample_rrr_jobs(bpt_job* jobs, uint32_t n_jobs, void* stream, bpt_counters* counters) {
    if (n_jobs > 0 && !jobs) {
        set_status(BPT_EINVAL, "jobs is NULL");
        return BPT_EINVAL;
    }
    if (counters) memset(counters, 0, sizeof(*counters));
    bpt_graph* owner = nullptr;
    std::vector<uint32_t> live, colors(n_jobs, 0);
    int nw = 1;
    try {
        for (uint32_t i = 0; i < n_jobs; ++i) {
            bpt_job& jb = jobs[i];
            jb.total = 0;
            jb.status = BPT_EINVAL;
            bpt_graph* gg = check_graph(jb.graph);
            if (!gg) {
                set_status(BPT_EINVAL, "job " + std::to_string(i) + ": not a bpt_graph handle");
                return BPT_EINVAL;
            }
            if (owner && gg->device != owner->device) {
                set_status(BPT_EINVAL, "job " + std::to_string(i) + ": graphs of one call must share a device");
                return BPT_EINVAL;
            }
            if (!jb.d_offsets || (!jb.d_vertices && jb.capacity > 0) || jb.reserved || jb.reserved2) {
                set_status(BPT_EINVAL, "job " + std::to_string(i) +
                                           ": d_offsets required (d_vertices when capacity > 0), reserved = 0");
                return BPT_EINVAL;
            }
            if (jb.n_samples >= kMaxSamples || jb.first_sample >= kMaxSamples ||
                jb.first_sample + jb.n_samples > kMaxSamples) {
                set_status(BPT_EINVAL, "job " + std::to_string(i) + ": sample ids must stay below 2^34");
                return BPT_EINVAL;
            }
            uint32_t c = jb.colors_per_batch ? jb.colors_per_batch : choose_colors(gg, jb.n_samples);
            if (!valid_colors(c)) {
                set_status(BPT_EINVAL, "job " + std::to_string(i) +
                                           ": colors_per_batch must be 0 or a power of two from 8 to 1024");
                return BPT_EINVAL;
            }
            colors[i] = c;
            if (!owner || gg->n > owner->n) owner = gg;
            if (jb.n_samples > 0) {
                live.push_back(i);
                nw = std::max(nw, mask_words(c));
            }
        }
        if (n_jobs == 0) {
            set_ok();
            return BPT_OK;
        }
        HIP_TRY(hipSetDevice(owner->device));
        hipStream_t st = static_cast<hipStream_t>(stream);
        for (uint32_t i = 0; i < n_jobs; ++i) {
            if (jobs[i].n_samples == 0) {
                HIP_TRY(hipMemsetAsync(jobs[i].d_offsets, 0, sizeof(uint64_t), st));
                jobs[i].status = BPT_OK;
            }
        }
        if (live.empty()) {
            HIP_TRY(hipStreamSynchronize(st));
            set_ok();
            return BPT_OK;
        }
    } catch (const HipFail& f) {
        set_status(f.status, f.msg);
        return f.status;
    } catch (const std::bad_alloc&) {
        set_status(BPT_ENOMEM, "host allocation failed");
        return BPT_ENOMEM;
    }
    // one launch per mask width (1, 2, 4, 8, 16 words), widest first
    (void)nw;
    Workspace* ws = nullptr;
    bpt_graph* wowner = nullptr;
    try {
        int rc_all = BPT_OK;
        for (int w = 16; w >= 1; w >>= 1) {
            std::vector<uint32_t> group;
            wowner = nullptr;
            for (uint32_t i : live) {
                if (mask_words(colors[i]) != w) continue;
                group.push_back(i);
                bpt_graph* gg = check_graph(jobs[i].graph);
                if (!wowner || gg->n > wowner->n) wowner = gg;
            }
            if (group.empty()) continue;
            bpt_counters part{};
            uint64_t group_batches = 0;
            for (uint32_t i : group) group_batches += (jobs[i].n_samples + colors[i] - 1) / colors[i];
            ws = acquire(wowner, w, group_batches);
            const int rc = run_jobs(wowner, ws, jobs, group, colors, static_cast<hipStream_t>(stream),
                                    counters ? &part : nullptr);
            if (rc == BPT_EINTERNAL) delete ws;
            else release(wowner, ws);
            ws = nullptr;
            if (rc != BPT_OK && rc != BPT_ERANGE) return rc;
            if (rc == BPT_ERANGE) rc_all = BPT_ERANGE;
            if (counters) {
                bpt_counters& k = *counters;
                k.samples += part.samples;
                k.members += part.members;
                k.sample_edges += part.sample_edges;
                k.edge_accesses += part.edge_accesses;
                k.frontier_entries += part.frontier_entries;
                k.philox_blocks += part.philox_blocks;
                k.live_coins += part.live_coins;
                k.levels += part.levels;
                k.max_levels = std::max(k.max_levels, part.max_levels);
                k.batches += part.batches;
                k.traversal_ns += part.traversal_ns;
                k.finalize_ns += part.finalize_ns;
                k.workgroup_size = std::max(k.workgroup_size, part.workgroup_size);
                k.workgroups = std::max(k.workgroups, part.workgroups);
            }
        }
        if (rc_all == BPT_OK) set_ok();
        else set_status(BPT_ERANGE, "a job's output capacity is below its total (see the job's total)");
        return rc_all;
    } catch (const HipFail& f) {
        if (ws) release(wowner, ws);
        set_status(f.status, f.msg);
        return f.status;
    } catch (const std::bad_alloc&) {
        if (ws) release(wowner, ws);
        set_status(BPT_ENOMEM, "host allocation failed");
        return BPT_ENOMEM;
    }
}

int bpt_graph_set_vertex_order(bpt_graph* g, const uint32_t* rank) {
    bpt_graph* gg = check_graph(g);
    if (!gg) {
        set_status(BPT_EINVAL, "not a bpt_graph handle");
        return BPT_EINVAL;
    }
    uint32_t* d = nullptr;
    if (rank) {
        std::vector<uint8_t> seen(gg->n, 0);
        for (uint32_t v = 0; v < gg->n; ++v) {
            if (rank[v] >= gg->n || seen[rank[v]]) {
                set_status(BPT_EINVAL, "rank must be a permutation of 0 .. n-1");
                return BPT_EINVAL;
            }
            seen[rank[v]] = 1;
        }
        try {
            HIP_TRY(hipSetDevice(gg->device));
            d = dev_alloc<uint32_t>(gg->n);
            HIP_TRY(hipMemcpy(d, rank, (size_t)gg->n * sizeof(uint32_t), hipMemcpyHostToDevice));
        } catch (const HipFail& f) {
            dev_free(d);
            set_status(f.status, f.msg);
            return f.status;
        }
    }
    uint32_t* old = nullptr;
    {
        std::lock_guard<std::mutex> lk(gg->mu);
        old = gg->d_rank;
        gg->d_rank = d;
    }
    dev_free(old);
    set_ok();
    return BPT_OK;
}

int bpt_max_cover(const uint64_t* d_offsets, const uint32_t* d_vertices, uint64_t n_sets, uint32_t n, uint32_t k,
                  void* stream, uint32_t* seeds, uint64_t* gains) {
    if (!d_offsets || !seeds || !gains || n == 0 || k > n || n_sets >= (1ull << 32)) {
        set_status(BPT_EINVAL, "d_offsets, seeds and gains are required; 1 <= n, k <= n, n_sets < 2^32");
        return BPT_EINVAL;
    }
    if (k == 0) {
        set_ok();
        return BPT_OK;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint64_t total = 0;
    if (hipMemcpyAsync(&total, d_offsets + n_sets, sizeof(uint64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_status(BPT_EDEVICE, "reading the sets' member count");
        return BPT_EDEVICE;
    }
    void* scratch = nullptr;
    const size_t bytes = max_cover_scratch_bytes(n_sets, n, k, total);
    if (hipMalloc(&scratch, bytes) != hipSuccess) {
        set_status(BPT_ENOMEM, "device scratch of the coverage greedy");
        return BPT_ENOMEM;
    }
    std::string why;
    const int rc = max_cover_run(d_offsets, d_vertices, n_sets, n, k, st, seeds, gains, scratch, bytes, &why);
    (void)hipFree(scratch);
    if (rc != BPT_OK) {
        set_status(rc, why);
        return rc;
    }
    set_ok();
    return BPT_OK;
}

bpt_rrr* bpt_sample_rrr(bpt_graph* g, uint64_t n_samples, uint32_t colors_per_batch, uint64_t seed) {
    bpt_graph* gg = check_graph(g);
    if (!gg) {
        set_status(BPT_EINVAL, "not a bpt_graph handle");
        return nullptr;
    }
    uint32_t colors = colors_per_batch == 0 ? choose_colors(gg, n_samples) : colors_per_batch;
    if (!valid_colors(colors)) {
        set_status(BPT_EINVAL, "colors_per_batch must be 0 or a power of two from 8 to 1024");
        return nullptr;
    }
    if (n_samples >= kMaxSamples) {
        set_status(BPT_EINVAL, "n_samples must be below 2^34");
        return nullptr;
    }
    bpt_rrr* r = nullptr;
    Workspace* ws = nullptr;
    try {
        r = new bpt_rrr();
        r->magic = kRrrMagic;
        r->num_samples = n_samples;
        r->offsets = static_cast<uint64_t*>(malloc((n_samples + 1) * sizeof(uint64_t)));
        if (!r->offsets) throw std::bad_alloc();
        r->offsets[0] = 0;
        if (n_samples > 0) {
            HIP_TRY(hipSetDevice(gg->device));
            ws = acquire(gg, mask_words(colors), (n_samples + colors - 1) / colors);
            CallResult res;
            const int rc = run_sampling(gg, ws, 0, n_samples, colors, seed, 0u, nullptr, nullptr, nullptr, 0,
                                        true, false, &res);
            if (rc != BPT_OK) {
                release_or_discard(gg, ws, res);
                const int keep_status = t_status;
                const std::string keep_msg = t_message;
                bpt_free(r);
                set_status(keep_status, keep_msg);
                return nullptr;
            }
            r->total = res.total;
            r->vertices = static_cast<uint32_t*>(malloc(std::max<uint64_t>(res.total, 1) * sizeof(uint32_t)));
            if (!r->vertices) throw std::bad_alloc();
            HIP_TRY(hipMemcpy(r->offsets, ws->out_offsets, (n_samples + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost));
            if (res.total)
                HIP_TRY(hipMemcpy(r->vertices, ws->out_vertices, res.total * sizeof(uint32_t), hipMemcpyDeviceToHost));
            release(gg, ws);
            ws = nullptr;
        } else {
            r->total = 0;
            r->vertices = static_cast<uint32_t*>(malloc(sizeof(uint32_t)));
            if (!r->vertices) throw std::bad_alloc();
        }
    } catch (const HipFail& f) {
        if (ws) release(gg, ws);
        if (r) bpt_free(r);
        set_status(f.status, f.msg);
        return nullptr;
    } catch (const std::bad_alloc&) {
        if (ws) release(gg, ws);
        if (r) bpt_free(r);
        set_status(BPT_ENOMEM, "host allocation failed");
        return nullptr;
    }
    set_ok();
    return r;
}

bpt_plan* bpt_plan_create(bpt_graph* g, uint64_t max_samples, uint32_t colors_per_batch, uint64_t pool_capacity) {
    bpt_graph* gg = check_graph(g);
    if (!gg) {
        set_status(BPT_EINVAL, "not a bpt_graph handle");
        return nullptr;
    }
    if (max_samples == 0 || max_samples >= kMaxSamples) {
        set_status(BPT_EINVAL, "max_samples must be in [1, 2^34)");
        return nullptr;
    }
    const uint32_t colors = colors_per_batch ? colors_per_batch : choose_colors(gg, max_samples);
    if (!valid_colors(colors)) {
        set_status(BPT_EINVAL, "colors_per_batch must be 0 or a power of two from 8 to 1024");
        return nullptr;
    }
    bpt_plan* p = nullptr;
    try {
        HIP_TRY(hipSetDevice(gg->device));
        p = new bpt_plan();
        p->magic = kDeadMagic;  // until complete
        p->graph = gg;
        p->device = gg->device;
        p->max_samples = max_samples;
        p->colors = colors;
        const int nw = mask_words(colors);
        p->ws = make_workspace(gg, nw, (max_samples + colors - 1) / colors);
        ensure_sample_arrays(p->ws, max_samples);
        ensure_pool(gg, p->ws, pool_capacity ? pool_capacity : pool_estimate(gg, max_samples));
        p->d_job = dev_alloc<FusedJob>(1);
        FusedJob j = {};
        j.g = dev_graph(gg);
        j.colors = colors;
        j.flags = job_flags(gg);  // fixed for the plan's life, from the graph's history at creation
        HIP_TRY(hipMemcpy(p->d_job, &j, sizeof(j), hipMemcpyHostToDevice));
        HIP_TRY(hipDeviceSynchronize());
        p->magic = kPlanMagic;
    } catch (const HipFail& f) {
        if (p) {
            delete p->ws;
            dev_free(p->d_job);
            delete p;
        }
        set_status(f.status, f.msg);
        return nullptr;
    } catch (const std::bad_alloc&) {
        if (p) {
            delete p->ws;
            dev_free(p->d_job);
            delete p;
        }
        set_status(BPT_ENOMEM, "host allocation failed");
        return nullptr;
    }
    set_ok();
    return p;
}

int bpt_plan_enqueue(bpt_plan* p, uint64_t first_sample, uint64_t n_samples, uint64_t seed, const uint64_t* d_params,
                     void* stream, uint64_t* d_offsets, uint32_t* d_vertices, uint64_t capacity, int64_t* d_result) {
    if (!p || p->magic != kPlanMagic || !p->graph) {
        set_status(BPT_EINVAL, "not a single-job bpt_plan handle");
        return BPT_EINVAL;
    }
    if (!d_offsets || !d_result || (!d_vertices && capacity > 0)) {
        set_status(BPT_EINVAL, "d_offsets and d_result are required (d_vertices when capacity > 0)");
        return BPT_EINVAL;
    }
    if (n_samples > p->max_samples) {
        set_status(BPT_EINVAL, "n_samples exceeds the plan's max_samples (" + std::to_string(p->max_samples) + ")");
        return BPT_EINVAL;
    }
    if (!d_params && (first_sample >= kMaxSamples || n_samples > kMaxSamples - first_sample)) {
        set_status(BPT_EINVAL, "sample ids must stay below 2^34");
        return BPT_EINVAL;
    }
    try {
        HIP_TRY(hipSetDevice(p->graph->device));
        hipStream_t st = static_cast<hipStream_t>(stream);
        Workspace* ws = p->ws;
        HIP_TRY(launch_plan_setup(p->d_job, d_params, first_sample, seed, n_samples, kMaxSamples, ws->ctl, st));
        if (n_samples > 0) {
            FusedArgs a = {};
            a.job0.g = dev_graph(p->graph);
            a.job0.colors = p->colors;
            a.job0.n_samples = n_samples;
            a.jobs = p->d_job;  // range and seed are read from the device job the setup kernel wrote
            a.n_jobs = 1;
            a.n_max = p->graph->n;
            a.ws = ws->fs;
            a.out.counts = ws->counts;
            a.out.where = ws->where;
            a.out.pool = ws->pool;
            a.out.pool_cap = ws->pool_cap;
            a.ctl = ws->ctl;
            a.n_batches = (n_samples + p->colors - 1) / p->colors;
            a.gather_mode = gather_for(p->graph, p->max_samples, p->colors);
            int block = 0, grid = 0;
            block = ws->block;
            grid = fused_grid(p->graph, block, ws->slots, a.n_batches);
            HIP_TRY(launch_fused(a, ws->nw, block, grid, help_wanted(p->graph), st));
        }
        HIP_TRY(launch_finalize(ws->counts, ws->where, ws->pool, n_samples,
                                reinterpret_cast<unsigned long long*>(d_offsets), d_vertices, capacity,
                                &ws->ctl->total, &ws->ctl->err, ws->scratch, ws->scratch_bytes, st));
        HIP_TRY(launch_plan_report(ws->ctl, capacity, d_result, st));
    } catch (const HipFail& f) {
        set_status(f.status, f.msg);
        return f.status;
    }
    set_ok();
    return BPT_OK;
}

bpt_plan* bpt_jobs_plan_create(const bpt_job* jobs, uint32_t n_jobs, uint64_t pool_capacity) {
    if (n_jobs == 0 || !jobs) {
        set_status(BPT_EINVAL, "at least one job is required");
        return nullptr;
    }
    bpt_plan* p = nullptr;
    try {
        std::vector<uint32_t> colors(n_jobs);
        bpt_graph* first = nullptr;
        for (uint32_t i = 0; i < n_jobs; ++i) {
            const bpt_job& jb = jobs[i];
            bpt_graph* gg = check_graph(jb.graph);
            if (!gg) {
                set_status(BPT_EINVAL, "job " + std::to_string(i) + ": not a bpt_graph handle");
                return nullptr;
            }
            if (first && gg->device != first->device) {
                set_status(BPT_EINVAL, "job " + std::to_string(i) + ": graphs of one plan must share a device");
                return nullptr;
            }
            if (!first) first = gg;
            if (!jb.d_offsets || (!jb.d_vertices && jb.capacity > 0) || jb.reserved || jb.reserved2) {
                set_status(BPT_EINVAL, "job " + std::to_string(i) +
                                           ": d_offsets required (d_vertices when capacity > 0), reserved = 0");
                return nullptr;
            }
            if (jb.n_samples >= kMaxSamples || jb.first_sample >= kMaxSamples ||
                jb.first_sample + jb.n_samples > kMaxSamples) {
                set_status(BPT_EINVAL, "job " + std::to_string(i) + ": sample ids must stay below 2^34");
                return nullptr;
            }
            colors[i] = jb.colors_per_batch ? jb.colors_per_batch : choose_colors(gg, jb.n_samples);
            if (!valid_colors(colors[i])) {
                set_status(BPT_EINVAL, "job " + std::to_string(i) +
                                           ": colors_per_batch must be 0 or a power of two from 8 to 1024");
                return nullptr;
            }
        }
        HIP_TRY(hipSetDevice(first->device));
        p = new bpt_plan();
        p->magic = kDeadMagic;  // until complete
        p->graph = nullptr;
        p->ws = nullptr;
        p->d_job = nullptr;
        p->device = first->device;
        p->n_jobs = n_jobs;
        uint64_t cap_all = 0;  // pool_capacity is split over the launches by the jobs' capacities
        for (uint32_t i = 0; i < n_jobs; ++i) cap_all += jobs[i].capacity;
        std::vector<uint32_t> empty_jobs;  // no samples: only an empty CSR and a result, in the one-word group
        for (uint32_t i = 0; i < n_jobs; ++i)
            if (jobs[i].n_samples == 0) empty_jobs.push_back(i);
        for (int w = 16; w >= 1; w >>= 1) {
            std::vector<uint32_t> fused, empty;
            for (uint32_t i = 0; i < n_jobs; ++i)
                if (jobs[i].n_samples && mask_words(colors[i]) == w) fused.push_back(i);
            if (w == 1) empty = empty_jobs;
            if (fused.empty() && empty.empty()) continue;
            p->groups.emplace_back();
            PlanGroup& gr = p->groups.back();
            gr.nw = w;
            std::vector<uint32_t> ids = fused;
            ids.insert(ids.end(), empty.begin(), empty.end());
            gr.n_fused = (uint32_t)fused.size();
            uint64_t samples = 0, est = 0, cap_group = 0;
            std::vector<FusedJob> table(ids.size());
            std::vector<unsigned long long> caps(ids.size());
            for (size_t t = 0; t < ids.size(); ++t) {
                const bpt_job& jb = jobs[ids[t]];
                bpt_graph* gg = check_graph(jb.graph);
                if (!gr.owner || gg->n > gr.owner->n) gr.owner = gg;
                gr.jobs.push_back(jb);
                gr.out_base.push_back(samples);
                FusedJob& fj = table[t];
                fj = FusedJob{};
                fj.g = dev_graph(gg);
                fj.seed = jb.seed;
                fj.first_sample = jb.first_sample;
                fj.n_samples = jb.n_samples;
                fj.batch_begin = gr.n_batches;
                fj.out_base = samples;
                fj.colors = colors[ids[t]];
                fj.flags = job_flags(gg);
                gr.n_batches += (jb.n_samples + fj.colors - 1) / fj.colors;
                samples += jb.n_samples;
                est += pool_estimate(gg, jb.n_samples);
                caps[t] = jb.capacity;
                cap_group += jb.capacity;
            }
            gr.ws = make_workspace(gr.owner, w, std::max<uint64_t>(gr.n_batches, 1));
            ensure_sample_arrays(gr.ws, std::max<uint64_t>(samples, 1));
            ensure_jobs(gr.ws, (uint32_t)ids.size());
            const uint64_t pool =
                pool_capacity ? (uint64_t)((double)pool_capacity * (double)cap_group / (double)std::max<uint64_t>(cap_all, 1)) + 1024
                              : est;
            ensure_pool(gr.owner, gr.ws, std::max<uint64_t>(pool, 1024));
            gr.d_ids = dev_alloc<uint32_t>(ids.size());
            gr.d_caps = dev_alloc<unsigned long long>(ids.size());
            HIP_TRY(hipMemcpy(gr.ws->d_jobs, table.data(), table.size() * sizeof(FusedJob), hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(gr.d_ids, ids.data(), ids.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(gr.d_caps, caps.data(), caps.size() * sizeof(unsigned long long),
                              hipMemcpyHostToDevice));
        }
        HIP_TRY(hipDeviceSynchronize());
        p->magic = kPlanMagic;
    } catch (const HipFail& f) {
        if (p) {
            p->magic = kPlanMagic;
            bpt_free(p);
        }
        set_status(f.status, f.msg);
        return nullptr;
    } catch (const std::bad_alloc&) {
        if (p) {
            p->magic = kPlanMagic;
            bpt_free(p);
        }
        set_status(BPT_ENOMEM, "host allocation failed");
        return nullptr;
    }
    set_ok();
    return p;
}

int bpt_jobs_plan_enqueue(bpt_plan* p, const uint64_t* d_params, void* stream, int64_t* d_results) {
    if (!p || p->magic != kPlanMagic || p->graph || !d_results) {
        set_status(BPT_EINVAL, "a multi-job bpt_plan handle and d_results are required");
        return BPT_EINVAL;
    }
    try {
        HIP_TRY(hipSetDevice(p->device));
        hipStream_t st = static_cast<hipStream_t>(stream);
        for (PlanGroup& gr : p->groups) {
            Workspace* ws = gr.ws;
            HIP_TRY(launch_plan_setup_jobs(ws->d_jobs, gr.n_fused, d_params, gr.d_ids, kMaxSamples, ws->ctl, st));
            if (gr.n_fused > 0) {
                FusedArgs a = {};
                a.jobs = ws->d_jobs;
                a.n_jobs = gr.n_fused;
                a.n_max = gr.owner->n;
                a.ws = ws->fs;
                a.out.counts = ws->counts;
                a.out.where = ws->where;
                a.out.pool = ws->pool;
                a.out.pool_cap = ws->pool_cap;
                a.ctl = ws->ctl;
                a.n_batches = gr.n_batches;
                a.gather_mode = gather_mode();
                int block = 0, grid = 0;
                block = ws->block;
                grid = fused_grid(gr.owner, block, ws->slots, gr.n_batches);
                bool help = false;
                for (uint32_t t = 0; t < gr.n_fused; ++t) help = help || help_wanted(check_graph(gr.jobs[t].graph));
                HIP_TRY(launch_fused(a, gr.nw, block, grid, help, st));
            }
            for (size_t t = 0; t < gr.jobs.size(); ++t) {
                const bpt_job& jb = gr.jobs[t];
                HIP_TRY(launch_finalize(ws->counts + gr.out_base[t], ws->where + gr.out_base[t], ws->pool,
                                        jb.n_samples, reinterpret_cast<unsigned long long*>(jb.d_offsets),
                                        jb.d_vertices, jb.capacity, ws->d_totals + t, &ws->ctl->err, ws->scratch,
                                        ws->scratch_bytes, st));
            }
            HIP_TRY(launch_plan_report_jobs(ws->ctl, ws->d_totals, gr.d_caps, gr.d_ids, (uint32_t)gr.jobs.size(),
                                            d_results, st));
        }
    } catch (const HipFail& f) {
        set_status(f.status, f.msg);
        return f.status;
    }
    set_ok();
    return BPT_OK;
}

void bpt_free(void* handle) {
    if (!handle) {
        set_ok();
        return;
    }
    const uint32_t magic = *static_cast<const uint32_t*>(handle);
    if (magic == kGraphMagic) {
        bpt_graph* g = static_cast<bpt_graph*>(handle);
        g->magic = kDeadMagic;
        (void)hipSetDevice(g->device);
        for (Workspace* ws : g->idle) delete ws;
        g->idle.clear();
        dev_free(g->d_rowptr);
        dev_free(g->d_col);
        dev_free(g->d_thr_row);
        dev_free(g->d_thr_edge);
        dev_free(g->d_rank);
        delete g;
        set_ok();
    } else if (magic == kPlanMagic) {
        bpt_plan* p = static_cast<bpt_plan*>(handle);
        p->magic = kDeadMagic;
        (void)hipSetDevice(p->device);
        delete p->ws;
        dev_free(p->d_job);
        for (PlanGroup& gr : p->groups) {
            delete gr.ws;
            dev_free(gr.d_ids);
            dev_free(gr.d_caps);
        }
        delete p;
        set_ok();
    } else if (magic == kRrrMagic) {
        bpt_rrr* r = static_cast<bpt_rrr*>(handle);
        r->magic = kDeadMagic;
        free(r->offsets);
        free(r->vertices);
        delete r;
        set_ok();
    } else {
        set_status(BPT_EINVAL, "bpt_free: not a libbpt handle");
    }
}

uint64_t bpt_rrr_num_samples(const bpt_rrr* r) { return (r && r->magic == kRrrMagic) ? r->num_samples : 0; }
uint64_t bpt_rrr_num_members(const bpt_rrr* r) { return (r && r->magic == kRrrMagic) ? r->total : 0; }
const uint64_t* bpt_rrr_offsets(const bpt_rrr* r) { return (r && r->magic == kRrrMagic) ? r->offsets : nullptr; }
const uint32_t* bpt_rrr_vertices(const bpt_rrr* r) { return (r && r->magic == kRrrMagic) ? r->vertices : nullptr; }

int bpt_last_status(void) { return t_status; }
const char* bpt_last_error(void) { return t_message.c_str(); }

int bpt_graph_info(const bpt_graph* g, uint32_t* n, uint64_t* m, uint32_t* prob_layout) {
    const bpt_graph* gg = check_graph(g);
    if (!gg) {
        set_status(BPT_EINVAL, "not a bpt_graph handle");
        return BPT_EINVAL;
    }
    if (n) *n = gg->n;
    if (m) *m = gg->m;
    if (prob_layout) *prob_layout = gg->layout;
    set_ok();
    return BPT_OK;
}

int bpt_graph_release_cache(bpt_graph* g) {
    bpt_graph* gg = check_graph(g);
    if (!gg) {
        set_status(BPT_EINVAL, "not a bpt_graph handle");
        return BPT_EINVAL;
    }
    (void)hipSetDevice(gg->device);
    trim_idle(gg, -1);
    set_ok();
    return BPT_OK;
}

uint32_t bpt_default_colors(const bpt_graph* g, uint64_t n_samples) {
    bpt_graph* gg = check_graph(g);
    if (!gg) {
        set_status(BPT_EINVAL, "not a bpt_graph handle");
        return 0;
    }
    set_ok();
    return choose_colors(gg, n_samples);
}

uint32_t bpt_tune_colors(bpt_graph* g, uint64_t n_samples, uint64_t seed) {
    bpt_graph* gg = check_graph(g);
    if (!gg) {
        set_status(BPT_EINVAL, "not a bpt_graph handle");
        return 0;
    }
    if (n_samples == 0 || n_samples >= kMaxSamples) {
        set_status(BPT_EINVAL, "n_samples must be in [1, 2^34)");
        return 0;
    }
    // The trial is capped at sixteen 64-colour batches per resident workgroup:
    // with fewer, the launch's tail (the heaviest batches running alone) weighs
    // more than in a large job and favours narrow batches that the job would
    // not want.
    const uint64_t resident = fused_resident(gg);
    const uint64_t S = std::min<uint64_t>(n_samples, 16 * 64 * resident);
    // short trials take the best of two runs; long ones are steady in one
    const int reps = S >= 4 * 64 * resident ? 1 : 2;
    Workspace* ws = nullptr;
    // traversal + CSR assembly, in HIP events (workspace and pool sizing are outside)
    auto trial = [&](uint32_t c, int gather, uint64_t* ns_out) -> int {
        ws = acquire(gg, mask_words(c), (S + c - 1) / c);
        uint64_t ns = ~0ull;
        for (int rep = 0; rep < reps; ++rep) {
            CallResult res;
            const int rc = run_sampling(gg, ws, 0, S, c, seed, 0u, nullptr, nullptr, nullptr, 0, true, false, &res,
                                        gather);
            if (rc != BPT_OK) {
                release_or_discard(gg, ws, res);
                ws = nullptr;
                return rc;  // status set by run_sampling
            }
            ns = std::min<uint64_t>(ns, res.counters.traversal_ns + res.counters.finalize_ns);
        }
        release(gg, ws);
        ws = nullptr;
        trim_idle(gg, -1);  // one width's slots at a time: wide masks take most of the memory
        *ns_out = ns;
        return BPT_OK;
    };
    TunedShape best;
    try {
        HIP_TRY(hipSetDevice(gg->device));
        bool no_history;
        {
            std::lock_guard<std::mutex> lk(gg->mu);
            no_history = !(gg->mean_members > 0);
        }
        if (no_history) {  // an untimed pilot sets the set-size history, which picks the workgroup size
            uint64_t ns = 0;
            if (trial(64, kGatherAuto, &ns) != BPT_OK) return 0;
        }
        uint64_t best_ns = ~0ull;
        int worse = 0;  // widths in a row at least 10% slower than the best so far
        for (uint32_t c = 8; c <= 1024 && worse < 2; c <<= 1) {  // under the kernel's own schedule choice
            uint64_t ns = 0;
            if (trial(c, kGatherAuto, &ns) != BPT_OK) return 0;
            if (ns < best_ns) {
                best_ns = ns;
                best.colors = c;
                worse = 0;
            } else {
                worse = (ns * 10 >= best_ns * 11) ? worse + 1 : 0;
            }
        }
        // then the colour schedule at that width: forced either way, kept if 3% faster
        for (uint32_t mode : {(uint32_t)kGatherNever, (uint32_t)kGatherAlways}) {
            uint64_t ns = 0;
            if (trial(best.colors, (int)mode, &ns) != BPT_OK) return 0;
            if (ns * 100 < best_ns * 97) {
                best_ns = ns;
                best.gather = mode;
            }
        }
    } catch (const HipFail& f) {
        if (ws) release(gg, ws);
        set_status(f.status, f.msg);
        return 0;
    } catch (const std::bad_alloc&) {
        if (ws) release(gg, ws);
        set_status(BPT_ENOMEM, "host allocation failed");
        return 0;
    }
    {
        std::lock_guard<std::mutex> lk(gg->mu);
        gg->tuned[size_bucket(n_samples)] = best;
    }
    set_ok();
    return best.colors;
}

uint32_t bpt_thr32(float p) { return threshold_of(p); }

uint32_t bpt_coin_word(uint64_t seed, uint64_t sample, uint64_t edge) {
    const Block4 b = coin_block((uint32_t)(edge >> 2), sample, (uint32_t)seed, (uint32_t)(seed >> 32));
    return pick_word(b, (uint32_t)(edge & 3));
}

uint32_t bpt_start_vertex(uint64_t seed, uint64_t sample, uint32_t n) {
    return start_of(sample, n, (uint32_t)seed, (uint32_t)(seed >> 32));
}

const char* bpt_version(void) { return BPT_VERSION_STRING; }

}  // extern "C"
