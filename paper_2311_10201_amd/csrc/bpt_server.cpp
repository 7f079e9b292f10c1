// A serving loop over the sampling library with continuous batching.
//
// Requests for RRR sets, or for influence-maximization seeds (sampling, then
// the greedy maximum coverage of paper Section 2), are queued by any thread.
// One worker thread keeps the GPU busy with a pipeline of bounded fused
// launches on two lanes (bpt_lane.hpp):
//  * admission: queued requests enter the running set in arrival order while
//    their estimated memory fits the budget (always one when nothing runs);
//  * a launch takes up to a fixed number of batches (four per resident
//    workgroup), filled in order of deadline: submission time plus four
//    times the request's estimated service time (its batches at the measured
//    time per batch).  A request that arrives while others are on the GPU
//    joins the very next launch, a small one finishes within it instead of
//    waiting behind large ones, and a large one moves ahead of newer small
//    ones as its deadline approaches;
//  * at most 64 requests run at a time; all chunks of a launch share one
//    CSR assembly (four kernels per launch, whatever the number of chunks);
//  * the next launch is enqueued on the other lane while the current one
//    drains, so the GPU fills with the new launch's batches during the old
//    one's tail; each chunk's CSR assembly appends to its request's output,
//    in launch order, at the request's running member count;
//  * a request is complete when the launch holding its last chunk has
//    finished; seed requests then go to a second thread that runs the
//    coverage greedy on its own stream while sampling goes on.
// Each request's sets are the ones it would get alone: they depend only on
// (graph, sample range, seed), never on chunking or on the other requests.
#include <hip/hip_runtime.h>
#include <stdlib.h>
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
#include "bpt_lane.hpp"

namespace {

constexpr uint32_t kServerMagic = 0x42505353u;  // "BPSS"
constexpr uint32_t kLanes = 2;
constexpr uint32_t kTotalsSlots = 1u << 16;  // running member counts of admitted requests (device)
constexpr size_t kMaxRunning = 64;           // admitted requests at a time
constexpr double kSlowdown = 4.0;            // deadline: submission + this many times the estimated service

double env_double(const char* name, double dflt) {
    const char* v = getenv(name);
    if (!v || !*v) return dflt;
    char* end = nullptr;
    const double x = strtod(v, &end);
    return (end && *end == 0 && x >= 0) ? x : dflt;
}

// Device buffers of seed requests' sets and of the coverage greedy, kept for
// reuse: freeing device memory would wait for every launch in flight.
class BufferCache {
   public:
    void* get(size_t bytes) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = free_.lower_bound(bytes);
        if (it != free_.end() && it->first <= 2 * bytes + (1u << 20)) {
            void* p = it->second;
            size_[p] = it->first;
            free_.erase(it);
            return p;
        }
        void* p = nullptr;
        const size_t sz = std::max<size_t>(bytes, 256);
        if (hipMalloc(&p, sz) != hipSuccess) return nullptr;
        size_[p] = sz;
        return p;
    }
    void put(void* p) {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu_);
        free_.emplace(size_[p], p);
    }
    ~BufferCache() {
        for (auto& kv : free_) (void)hipFree(kv.second);
    }

   private:
    std::mutex mu_;
    std::multimap<size_t, void*> free_;
    std::map<void*, size_t> size_;
};

// An admitted request.
struct Live {
    bpt_request* r = nullptr;
    uint32_t colors = 64;
    uint64_t n_batches = 0;
    uint64_t next_batch = 0;    // first batch not yet in a launch
    uint32_t open_chunks = 0;   // chunks in launches not yet finished
    uint64_t* d_offsets = nullptr;
    uint32_t* d_vertices = nullptr;
    uint64_t capacity = 0;
    uint32_t slot = 0;          // index of its running total
    bool broken = false;        // a launch holding one of its chunks overflowed its pool
    bool started = false;
    uint64_t bytes = 0;         // admitted estimate
};

struct InFlight {
    uint32_t lane;
    std::vector<Live*> owners;  // one entry per chunk
    uint64_t batches = 0;
    double issued = 0.0;        // server clock when enqueued
};

}  // namespace

struct bpt_server {
    uint32_t magic = kServerMagic;
    uint64_t budget = 0;
    uint32_t max_jobs = 0;
    uint64_t launch_batches = 2048;  // batches per launch: four per workgroup the fused kernel keeps resident
    double batch_s = 2e-6;           // running estimate of the GPU time per batch (deadlines)
    uint64_t resampled = 0;          // requests sampled again alone after a pool overflow
    uint32_t lane_slots = 0;         // traversal slots of the largest lane workspace
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_cover;
    std::deque<bpt_request*> pending;
    std::deque<bpt_request*> done;
    std::deque<Live*> cover_queue;
    std::map<const bpt_graph*, double> mean_size;  // members per sample, running estimate per graph
    uint64_t launches = 0, served = 0, in_use = 0;
    double t_sample = 0, t_cover = 0, t_alloc = 0, t_busy = 0;  // seconds
    double busy_since = -1.0;      // admitted work present since (open interval of t_busy)
    double sampling_since = -1.0;  // a launch in flight since (open interval of t_sample)
    bool stop = false, cover_stop = false;
    int device = 0;
    BufferCache buffers;
    unsigned long long* d_totals = nullptr;
    std::vector<uint32_t> free_slots;
    std::thread worker, coverer;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

double mean_of(bpt_server* sv, const bpt_graph* g) {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->mean_size.find(g);
    return it == sv->mean_size.end() ? 32.0 : it->second;
}

void note_mean(bpt_server* sv, const bpt_graph* g, uint64_t n_samples, uint64_t total) {
    if (!n_samples) return;
    const double m = (double)total / (double)n_samples;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->mean_size.find(g);
    sv->mean_size[g] = it == sv->mean_size.end() ? m : 0.5 * it->second + 0.5 * m;
}

// Bytes a request is expected to occupy while it is served: the server's copy
// of a seed request's sets and offsets; a sample request writes to the
// caller's buffers, so only its share of the launches' pools counts.
uint64_t estimate_bytes(bpt_server* sv, const bpt_request* r) {
    const double members = (double)r->n_samples * mean_of(sv, r->graph) * 1.25 + 1024.0;
    double bytes = members * 4.0 + (double)r->n_samples * 12.0;
    if (r->kind == BPT_REQ_SEEDS) bytes += members * 4.0 + (double)r->n_samples * 8.0;
    return (uint64_t)bytes;
}

void finish(bpt_server* sv, Live* lv, int status) {
    bpt_request* r = lv->r;
    r->status = status;
    r->t_done = sv->now();
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->in_use -= std::min(sv->in_use, lv->bytes);
    sv->free_slots.push_back(lv->slot);
    sv->done.push_back(r);
    ++sv->served;
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();  // memory and a totals slot are free again
}

void release_owned(bpt_server* sv, Live* lv) {
    if (lv->r->kind != BPT_REQ_SEEDS) return;
    sv->buffers.put(lv->d_offsets);
    sv->buffers.put(lv->d_vertices);
    lv->d_offsets = nullptr;
    lv->d_vertices = nullptr;
}

// Server-owned output of a seed request, from the buffer cache.
bool alloc_owned(bpt_server* sv, Live* lv, uint64_t capacity) {
    const double ta = sv->now();
    release_owned(sv, lv);
    lv->d_offsets = static_cast<uint64_t*>(sv->buffers.get((lv->r->n_samples + 1) * sizeof(uint64_t)));
    lv->d_vertices = static_cast<uint32_t*>(sv->buffers.get(std::max<uint64_t>(capacity, 1) * sizeof(uint32_t)));
    lv->capacity = capacity;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->t_alloc += sv->now() - ta;
    }
    return lv->d_offsets && lv->d_vertices;
}

// Samples a request alone (after a pool overflow in one of its launches, or a
// seed request whose sets outgrew the server's estimate).
int resample_alone(bpt_server* sv, Live* lv, hipStream_t stream, uint64_t* total) {
    bpt_request* r = lv->r;
    return bpt_sample_rrr_device(r->graph, r->first_sample, r->n_samples, lv->colors, r->seed, 0, stream,
                                 lv->d_offsets, lv->d_vertices, lv->capacity, total, nullptr);
}

void cover_main(bpt_server* sv) {
    hipStream_t stream = nullptr;
    (void)hipSetDevice(sv->device);
    (void)hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);  // default priority
    for (;;) {
        Live* lv = nullptr;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_cover.wait(lk, [&] { return sv->cover_stop || !sv->cover_queue.empty(); });
            if (sv->cover_queue.empty()) break;
            lv = sv->cover_queue.front();
            sv->cover_queue.pop_front();
        }
        bpt_request* r = lv->r;
        const double tc = sv->now();
        uint32_t n = 0;
        int st = bpt_graph_info(r->graph, &n, nullptr, nullptr);
        if (st == BPT_OK) {
            const size_t bytes = bpt::max_cover_scratch(r->n_samples, n, r->k, r->total);
            void* scratch = sv->buffers.get(bytes);
            std::string why;
            st = scratch ? bpt::max_cover_run(lv->d_offsets, lv->d_vertices, r->n_samples, n, r->k, stream, r->seeds,
                                              r->gains, scratch, bytes, &why)
                         : BPT_ENOMEM;
            sv->buffers.put(scratch);
        }
        release_owned(sv, lv);
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->t_cover += sv->now() - tc;
        }
        finish(sv, lv, st);
        delete lv;
    }
    if (stream) (void)hipStreamDestroy(stream);
}

// The request's last chunk has finished: check its total and hand it on.
void complete(bpt_server* sv, Live* lv, hipStream_t stream) {
    bpt_request* r = lv->r;
    unsigned long long total = 0;
    int st = hipMemcpyAsync(&total, sv->d_totals + lv->slot, sizeof(total), hipMemcpyDeviceToHost, stream) ==
                     hipSuccess &&
                     hipStreamSynchronize(stream) == hipSuccess
                 ? BPT_OK
                 : BPT_EDEVICE;
    if (st == BPT_OK) {
        note_mean(sv, r->graph, r->n_samples, total);
        if (r->kind == BPT_REQ_SEEDS && (lv->broken || total > lv->capacity)) {
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                ++sv->resampled;
            }
            if (!alloc_owned(sv, lv, total + total / 16 + 1024)) st = BPT_ENOMEM;
            else {
                uint64_t t2 = 0;
                st = resample_alone(sv, lv, stream, &t2);
                total = t2;
            }
        } else if (lv->broken) {
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                ++sv->resampled;
            }
            uint64_t t2 = 0;
            st = resample_alone(sv, lv, stream, &t2);
            total = t2;
        } else if (total > lv->capacity) {
            st = BPT_ERANGE;
        }
    }
    r->total = total;
    if (r->kind == BPT_REQ_SEEDS && st == BPT_OK) {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->cover_queue.push_back(lv);
        sv->cv_cover.notify_one();
        return;
    }
    release_owned(sv, lv);
    finish(sv, lv, st);
    delete lv;
}

void worker_main(bpt_server* sv) {
    (void)hipSetDevice(sv->device);
    hipStream_t stream = nullptr;
    (void)hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);  // default priority
    std::string why;
    bpt::Lane* lanes[kLanes] = {};
    for (uint32_t i = 0; i < kLanes; ++i) lanes[i] = bpt::lane_create(sv->device, &why);
    std::vector<Live*> running;        // admitted, with batches not yet launched or chunks in flight
    std::deque<InFlight> inflight;     // launches in issue order
    uint32_t next_lane = 0;
    double last_fin = 0.0;             // when the last waited-for launch finished
    for (;;) {
        // 1. admission
        std::vector<uint32_t> lv_slots;
        std::vector<std::pair<bpt_request*, uint64_t>> admitted;  // with its estimated bytes
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            const bool idle = running.empty() && inflight.empty();
            if (idle && sv->pending.empty()) {
                if (sv->busy_since >= 0) {
                    sv->t_busy += sv->now() - sv->busy_since;
                    sv->busy_since = -1.0;
                }
                if (sv->stop) break;
                sv->cv_work.wait(lk, [&] { return sv->stop || !sv->pending.empty(); });
                if (sv->pending.empty()) continue;
            }
            while (!sv->pending.empty() && !sv->free_slots.empty() && running.size() + admitted.size() < kMaxRunning) {
                bpt_request* r = sv->pending.front();
                lk.unlock();
                const uint64_t b = estimate_bytes(sv, r);
                lk.lock();
                const bool none = running.empty() && admitted.empty();
                if (!none && sv->in_use + b > sv->budget) break;
                sv->in_use += b;
                sv->pending.pop_front();
                admitted.emplace_back(r, b);
                lv_slots.push_back(sv->free_slots.back());
                sv->free_slots.pop_back();
                if (sv->busy_since < 0) sv->busy_since = sv->now();
            }
        }
        for (size_t ai = 0; ai < admitted.size(); ++ai) {
            bpt_request* r = admitted[ai].first;
            Live* lv = new Live();
            lv->r = r;
            lv->bytes = admitted[ai].second;
            lv->slot = lv_slots[ai];
            // 64 colours (one mask word, what the lanes run): alone, a small request would
            // take fewer colours to give every workgroup a batch, but here other requests
            // fill the launch, and wider batches mean fewer batches for the same samples
            lv->colors = 64;
            lv->n_batches = (r->n_samples + lv->colors - 1) / lv->colors;
            if (r->kind == BPT_REQ_SEEDS) {
                const uint64_t cap = (uint64_t)((double)r->n_samples * mean_of(sv, r->graph) * 1.25) + 4096;
                if (!alloc_owned(sv, lv, cap)) {
                    release_owned(sv, lv);
                    finish(sv, lv, BPT_ENOMEM);
                    delete lv;
                    continue;
                }
            } else {
                lv->d_offsets = r->d_offsets;
                lv->d_vertices = r->d_vertices;
                lv->capacity = r->capacity;
            }
            if (r->n_samples == 0) {  // an empty CSR, no launch
                const bool ok = hipMemsetAsync(lv->d_offsets, 0, sizeof(uint64_t), stream) == hipSuccess &&
                                hipStreamSynchronize(stream) == hipSuccess;
                r->t_start = sv->now();
                r->total = 0;
                if (r->kind == BPT_REQ_SEEDS && ok) {
                    memset(r->seeds, 0, r->k * sizeof(uint32_t));
                    memset(r->gains, 0, r->k * sizeof(uint64_t));
                }
                release_owned(sv, lv);
                finish(sv, lv, ok ? BPT_OK : BPT_EDEVICE);
                delete lv;
                continue;
            }
            const bool ok = hipMemsetAsync(sv->d_totals + lv->slot, 0, sizeof(unsigned long long), stream) ==
                                hipSuccess &&
                            hipStreamSynchronize(stream) == hipSuccess;
            if (!ok) {
                release_owned(sv, lv);
                finish(sv, lv, BPT_EDEVICE);
                delete lv;
                continue;
            }
            running.push_back(lv);
        }

        // 2. a launch on a free lane: the next batches of every running request
        std::vector<Live*> want;
        for (Live* lv : running)
            if (lv->next_batch < lv->n_batches) want.push_back(lv);
        bpt::Lane* lane = lanes[next_lane];
        if (!want.empty() && lane && inflight.size() < kLanes && bpt::lane_finished(lane)) {
            // Earliest deadline first: a request's deadline is its submission time plus
            // kSlowdown times its estimated service time (its batches at the measured
            // time per batch), so small requests go ahead of large ones, and a large one
            // moves ahead of newer small ones as its deadline approaches.
            std::vector<std::pair<Live*, uint64_t>> plan;
            uint64_t room = sv->launch_batches;
            {
                std::vector<Live*> order(want.begin(), want.end());
                double tb;
                {
                    std::lock_guard<std::mutex> lk(sv->mu);
                    tb = sv->batch_s;
                }
                std::stable_sort(order.begin(), order.end(), [tb](const Live* x, const Live* y) {
                    return x->r->t_submit + kSlowdown * tb * (double)x->n_batches <
                           y->r->t_submit + kSlowdown * tb * (double)y->n_batches;
                });
                for (Live* lv : order) {
                    if (room == 0 || plan.size() >= sv->max_jobs) break;
                    const uint64_t t = std::min(room, lv->n_batches - lv->next_batch);
                    plan.emplace_back(lv, t);
                    room -= t;
                }
            }
            std::vector<bpt::LaneChunk> chunks;
            InFlight fl;
            fl.lane = next_lane;
            for (auto& pt : plan) {
                Live* lv = pt.first;
                const uint64_t take = pt.second;
                if (take == 0) continue;
                bpt_request* r = lv->r;
                const uint64_t s0 = lv->next_batch * lv->colors;
                const uint64_t ns = std::min<uint64_t>(take * lv->colors, r->n_samples - s0);
                bpt::LaneChunk c;
                c.graph = r->graph;
                c.first_sample = r->first_sample + s0;
                c.n_samples = ns;
                c.seed = r->seed;
                c.colors = lv->colors;
                c.d_offsets = reinterpret_cast<unsigned long long*>(lv->d_offsets) + s0;
                c.d_vertices = lv->d_vertices;
                c.capacity = lv->capacity;
                c.d_total = sv->d_totals + lv->slot;
                chunks.push_back(c);
                fl.owners.push_back(lv);
                lv->next_batch += take;
                fl.batches += take;
                ++lv->open_chunks;
                if (!lv->started) {
                    lv->started = true;
                    r->t_start = sv->now();
                }
            }
            fl.issued = sv->now();
            hipEvent_t after = inflight.empty() ? nullptr : bpt::lane_done(lanes[inflight.back().lane]);
            const int rc = bpt::lane_launch(lane, chunks.data(), (uint32_t)chunks.size(), after, &why);
            if (rc != BPT_OK) {  // nothing of it ran: its requests fail
                for (Live* lv : fl.owners) lv->broken = true, lv->next_batch = lv->n_batches, --lv->open_chunks;
                for (auto it = running.begin(); it != running.end();) {
                    Live* lv = *it;
                    if (lv->broken && lv->open_chunks == 0) {
                        it = running.erase(it);
                        release_owned(sv, lv);
                        finish(sv, lv, rc);
                        delete lv;
                    } else {
                        ++it;
                    }
                }
            } else {
                {
                    std::lock_guard<std::mutex> lk(sv->mu);
                    if (sv->sampling_since < 0) sv->sampling_since = sv->now();
                    ++sv->launches;
                    sv->lane_slots = std::max(sv->lane_slots, bpt::lane_slots(lane));
                }
                inflight.push_back(std::move(fl));
                next_lane = (next_lane + 1) % kLanes;
            }
            continue;  // admit and launch again before waiting
        }

        // 3. the oldest launch: with both lanes busy, wait for it; with a lane free,
        // poll it and look for arrivals, which go to the free lane at once
        if (inflight.empty()) continue;
        InFlight& fl = inflight.front();
        bpt::Lane* fl_lane = lanes[fl.lane];
        if (inflight.size() < kLanes && !bpt::lane_finished(fl_lane)) {
            std::unique_lock<std::mutex> lk(sv->mu);
            if (sv->cv_work.wait_for(lk, std::chrono::microseconds(50), [&] {
                    return !sv->pending.empty() && !sv->free_slots.empty() && running.size() < kMaxRunning;
                }))
                continue;
            if (!bpt::lane_finished(fl_lane)) continue;
        }
        bool overflow = false;
        const int rc = bpt::lane_wait(fl_lane, &overflow, &why);
        const double t_fin = sv->now();
        if (2 * fl.batches >= sv->launch_batches) {
            // GPU time per batch from a well-filled launch, counted from when the one
            // before it finished (the two overlap).  Small launches are left out: their
            // fixed cost would make every batch look slow and push large requests'
            // deadlines far out.
            const double per = (t_fin - std::max(fl.issued, last_fin)) / (double)fl.batches;
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->batch_s = 0.8 * sv->batch_s + 0.2 * per;
        }
        last_fin = t_fin;
        for (Live* lv : fl.owners) {
            --lv->open_chunks;
            if (overflow || rc != BPT_OK) lv->broken = true;
        }
        std::vector<Live*> owners = std::move(fl.owners);
        inflight.pop_front();
        if (inflight.empty()) {
            std::lock_guard<std::mutex> lk(sv->mu);
            if (sv->sampling_since >= 0) sv->t_sample += sv->now() - sv->sampling_since;
            sv->sampling_since = -1.0;
        }
        std::sort(owners.begin(), owners.end());
        owners.erase(std::unique(owners.begin(), owners.end()), owners.end());
        for (Live* lv : owners) {
            if (lv->open_chunks != 0 || lv->next_batch < lv->n_batches) continue;
            running.erase(std::find(running.begin(), running.end(), lv));
            complete(sv, lv, stream);
        }
    }
    for (uint32_t i = 0; i < kLanes; ++i) bpt::lane_destroy(lanes[i]);
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
    int cus = 0;
    if (hipGetDevice(&sv->device) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, sv->device) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&sv->d_totals), kTotalsSlots * sizeof(unsigned long long)) !=
            hipSuccess) {
        delete sv;
        return nullptr;
    }
    // four batches per resident 512-thread workgroup (BPT_SERVE_LAUNCH_BATCHES overrides it)
    sv->launch_batches = (uint64_t)env_double("BPT_SERVE_LAUNCH_BATCHES", (double)std::max(cus, 1) * 8);
    if (sv->launch_batches == 0) sv->launch_batches = 1;
    sv->free_slots.reserve(kTotalsSlots);
    for (uint32_t i = kTotalsSlots; i > 0; --i) sv->free_slots.push_back(i - 1);
    sv->worker = std::thread(worker_main, sv);
    sv->coverer = std::thread(cover_main, sv);
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
    if (r->kind == BPT_REQ_SAMPLE && (!r->d_offsets || (!r->d_vertices && r->capacity > 0))) return BPT_EINVAL;
    if (r->n_samples >= (1ull << 34) || r->first_sample >= (1ull << 34) ||
        r->first_sample + r->n_samples > (1ull << 34))
        return BPT_EINVAL;
    r->status = 1;  // in flight
    r->total = 0;
    r->reserved = 0;
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
    const double t = sv->now();
    out->busy_s = sv->t_busy + (sv->busy_since >= 0 ? t - sv->busy_since : 0.0);
    out->sample_s = sv->t_sample + (sv->sampling_since >= 0 ? t - sv->sampling_since : 0.0);
    out->cover_s = sv->t_cover;
    out->alloc_s = sv->t_alloc;
    out->resampled = sv->resampled;
    out->batch_s = sv->batch_s;
    out->lane_slots = sv->lane_slots;
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
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->cover_stop = true;
    }
    sv->cv_cover.notify_all();
    sv->coverer.join();
    sv->magic = 0;
    (void)hipFree(sv->d_totals);
    delete sv;
    return BPT_OK;
}

}  // extern "C"
