// A serving loop over the sampling library: requests for RRR sets or for
// influence-maximization seeds (sampling followed by the greedy maximum
// coverage of paper Section 2) are queued by any thread and served by one
// worker thread that batches them continuously.  Each iteration of the worker
// admits the queued requests in arrival order while their estimated memory
// fits the budget (at least one), samples all of them with a single
// bpt_sample_rrr_jobs call (their batches share persistent launches), runs
// the seed selection of the seed requests, and hands the requests back through
// a completion queue.  A request's result is the one it would get alone: sets
// depend only on (graph, sample range, seed).
//
// The server is built on the public C ABI only (bpt.h).
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "bpt.h"

namespace {

constexpr uint32_t kServerMagic = 0x42505353u;  // "BPSS"

struct Owned {  // server-owned device output of a seed request
    uint64_t* offsets = nullptr;
    uint32_t* vertices = nullptr;
    uint64_t capacity = 0;
};

}  // namespace

struct bpt_server {
    uint32_t magic = kServerMagic;
    uint64_t budget = 0;
    uint32_t max_jobs = 0;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<bpt_request*> pending;
    std::deque<bpt_request*> done;
    std::map<const bpt_graph*, double> mean_size;  // members per sample, running estimate per graph
    uint64_t launches = 0, served = 0;
    double t_sample = 0, t_cover = 0, t_alloc = 0, t_busy = 0;  // worker time, seconds
    bool stop = false;
    std::thread worker;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

// Bytes a request is expected to occupy while it is served: the library's
// member pool and per-sample arrays, plus the server's own output for a seed
// request.
uint64_t estimate_bytes(bpt_server* sv, const bpt_request* r) {
    double mean = 32.0;
    {
        auto it = sv->mean_size.find(r->graph);
        if (it != sv->mean_size.end()) mean = it->second;
    }
    const double members = (double)r->n_samples * mean * 1.25 + 1024.0;
    double bytes = members * 4.0 + (double)r->n_samples * 12.0;
    if (r->kind == BPT_REQ_SEEDS) bytes += members * 4.0 + (double)r->n_samples * 8.0;
    return (uint64_t)bytes;
}

void free_owned(Owned& o) {
    if (o.offsets) (void)hipFree(o.offsets);
    if (o.vertices) (void)hipFree(o.vertices);
    o = Owned{};
}

bool alloc_owned(Owned& o, uint64_t n_samples, uint64_t capacity) {
    free_owned(o);
    if (hipMalloc(reinterpret_cast<void**>(&o.offsets), (n_samples + 1) * sizeof(uint64_t)) != hipSuccess) return false;
    if (hipMalloc(reinterpret_cast<void**>(&o.vertices), std::max<uint64_t>(capacity, 1) * sizeof(uint32_t)) !=
        hipSuccess) {
        free_owned(o);
        return false;
    }
    o.capacity = capacity;
    return true;
}

void finish(bpt_server* sv, bpt_request* r, int status) {
    r->status = status;
    r->t_done = sv->now();
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->done.push_back(r);
    ++sv->served;
    sv->cv_done.notify_all();
}

void add_time(bpt_server* sv, double& slot, double since) {
    const double d = sv->now() - since;
    std::lock_guard<std::mutex> lk(sv->mu);
    slot += d;
}

void serve_group(bpt_server* sv, std::vector<bpt_request*>& group, hipStream_t stream) {
    const size_t G = group.size();
    const double t_enter = sv->now();
    std::vector<Owned> owned(G);
    std::vector<bpt_job> jobs(G);
    std::vector<size_t> in_launch;  // requests whose job is in the call
    const double t_start = sv->now();
    for (size_t i = 0; i < G; ++i) {
        bpt_request* r = group[i];
        r->t_start = t_start;
        bpt_job& j = jobs[i];
        memset(&j, 0, sizeof(j));
        j.graph = r->graph;
        j.first_sample = r->first_sample;
        j.n_samples = r->n_samples;
        j.seed = r->seed;
        j.colors_per_batch = 0;
        if (r->kind == BPT_REQ_SEEDS) {
            double mean = 32.0;
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                auto it = sv->mean_size.find(r->graph);
                if (it != sv->mean_size.end()) mean = it->second;
            }
            const uint64_t cap = (uint64_t)((double)r->n_samples * mean * 1.25) + 4096;
            const double ta = sv->now();
            const bool ok = alloc_owned(owned[i], r->n_samples, cap);
            add_time(sv, sv->t_alloc, ta);
            if (!ok) continue;  // left out; fails below
            j.d_offsets = owned[i].offsets;
            j.d_vertices = owned[i].vertices;
            j.capacity = owned[i].capacity;
        } else {
            j.d_offsets = r->d_offsets;
            j.d_vertices = r->d_vertices;
            j.capacity = r->capacity;
        }
        in_launch.push_back(i);
    }
    std::vector<bpt_job> call(in_launch.size());
    for (size_t c = 0; c < in_launch.size(); ++c) call[c] = jobs[in_launch[c]];
    const double ts = sv->now();
    const int rc = call.empty() ? BPT_OK : bpt_sample_rrr_jobs(call.data(), (uint32_t)call.size(), stream, nullptr);
    add_time(sv, sv->t_sample, ts);
    for (size_t c = 0; c < in_launch.size(); ++c) jobs[in_launch[c]] = call[c];
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        ++sv->launches;
    }
    for (size_t i = 0; i < G; ++i) {
        bpt_request* r = group[i];
        bpt_job& j = jobs[i];
        if (r->kind == BPT_REQ_SEEDS && !owned[i].offsets) {
            finish(sv, r, BPT_ENOMEM);
            continue;
        }
        if (rc != BPT_OK && rc != BPT_ERANGE) {
            free_owned(owned[i]);
            finish(sv, r, rc);
            continue;
        }
        r->total = j.total;
        if (r->n_samples > 0) {
            std::lock_guard<std::mutex> lk(sv->mu);
            const double m = (double)j.total / (double)r->n_samples;
            auto it = sv->mean_size.find(r->graph);
            sv->mean_size[r->graph] = it == sv->mean_size.end() ? m : 0.5 * it->second + 0.5 * m;
        }
        if (r->kind == BPT_REQ_SAMPLE) {
            finish(sv, r, j.status);
            continue;
        }
        int st = BPT_OK;
        if (j.status == BPT_ERANGE) {  // estimate too small: sample this request again, alone
            if (!alloc_owned(owned[i], r->n_samples, j.total)) st = BPT_ENOMEM;
            else {
                uint64_t total = 0;
                st = bpt_sample_rrr_device(r->graph, r->first_sample, r->n_samples, 0, r->seed, 0, stream,
                                           owned[i].offsets, owned[i].vertices, owned[i].capacity, &total, nullptr);
            }
        }
        const double tc = sv->now();
        if (st == BPT_OK) {
            uint32_t n = 0, layout = 0;
            uint64_t m = 0;
            st = bpt_graph_info(r->graph, &n, &m, &layout);
            if (st == BPT_OK)
                st = bpt_max_cover(owned[i].offsets, owned[i].vertices, r->n_samples, n, r->k, stream, r->seeds,
                                   r->gains);
        }
        free_owned(owned[i]);
        add_time(sv, sv->t_cover, tc);
        finish(sv, r, st);
    }
    add_time(sv, sv->t_busy, t_enter);
}

void worker_main(bpt_server* sv) {
    hipStream_t stream = nullptr;
    (void)hipStreamCreate(&stream);  // default priority
    for (;;) {
        std::vector<bpt_request*> group;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_work.wait(lk, [&] { return sv->stop || !sv->pending.empty(); });
            if (sv->pending.empty() && sv->stop) break;
            uint64_t bytes = 0;
            while (!sv->pending.empty() && group.size() < sv->max_jobs) {
                bpt_request* r = sv->pending.front();
                const uint64_t b = estimate_bytes(sv, r);
                if (!group.empty() && bytes + b > sv->budget) break;
                bytes += b;
                group.push_back(r);
                sv->pending.pop_front();
            }
        }
        serve_group(sv, group, stream);
    }
    if (stream) (void)hipStreamDestroy(stream);
}

bpt_server* check_server(bpt_server* s) { return (s && s->magic == kServerMagic) ? s : nullptr; }

}  // namespace

extern "C" {

bpt_server* bpt_server_create(uint64_t memory_budget, uint32_t max_jobs_per_launch) {
    bpt_server* sv = new (std::nothrow) bpt_server();
    if (!sv) return nullptr;
    sv->budget = memory_budget ? memory_budget : (8ull << 30);
    sv->max_jobs = max_jobs_per_launch ? max_jobs_per_launch : 256;
    sv->t0 = std::chrono::steady_clock::now();
    sv->worker = std::thread(worker_main, sv);
    return sv;
}

double bpt_server_now(bpt_server* s) {
    bpt_server* sv = check_server(s);
    return sv ? sv->now() : -1.0;
}

int bpt_server_submit(bpt_server* s, bpt_request* r) {
    bpt_server* sv = check_server(s);
    if (!sv || !r || !r->graph || (r->kind != BPT_REQ_SAMPLE && r->kind != BPT_REQ_SEEDS)) return BPT_EINVAL;
    if (r->kind == BPT_REQ_SEEDS && (!r->seeds || !r->gains || r->k == 0)) return BPT_EINVAL;
    if (r->kind == BPT_REQ_SAMPLE && !r->d_offsets) return BPT_EINVAL;
    r->status = 1;  // in flight
    r->total = 0;
    r->t_submit = sv->now();
    r->t_start = r->t_done = 0.0;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stop) return BPT_EINVAL;
        sv->pending.push_back(r);
    }
    sv->cv_work.notify_one();
    return BPT_OK;
}

bpt_request* bpt_server_wait(bpt_server* s, double timeout_s) {
    bpt_server* sv = check_server(s);
    if (!sv) return nullptr;
    std::unique_lock<std::mutex> lk(sv->mu);
    if (!sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return !sv->done.empty(); }))
        return nullptr;
    bpt_request* r = sv->done.front();
    sv->done.pop_front();
    return r;
}

int bpt_server_stats(bpt_server* s, bpt_server_info* out) {
    bpt_server* sv = check_server(s);
    if (!sv || !out) return BPT_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    out->launches = sv->launches;
    out->served = sv->served;
    out->busy_s = sv->t_busy;
    out->sample_s = sv->t_sample;
    out->cover_s = sv->t_cover;
    out->alloc_s = sv->t_alloc;
    return BPT_OK;
}

int bpt_server_destroy(bpt_server* s) {
    bpt_server* sv = check_server(s);
    if (!sv) return BPT_EINVAL;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    sv->worker.join();
    sv->magic = 0;
    delete sv;
    return BPT_OK;
}

}  // extern "C"
