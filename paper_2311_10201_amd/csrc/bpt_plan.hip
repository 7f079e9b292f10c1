// The two small kernels around a plan's call (bpt_plan_enqueue): a call is
// setup -> fused traversal -> CSR assembly -> report, all kernels, so that a
// stream capture records it as a graph of kernel nodes only.  The control
// block is cleared by a kernel rather than a memset node, and the sample range
// and seed can come from device memory, so one captured graph serves any
// range the caller writes before a replay.
#include "bpt.h"
#include "bpt_internal.hpp"

namespace bpt {

namespace {

constexpr int kSetupBlock = 256;

__global__ __launch_bounds__(kSetupBlock) void plan_setup(FusedJob* job, const uint64_t* params, uint64_t first,
                                                          uint64_t seed, uint64_t n_samples, uint64_t max_ids,
                                                          Control* ctl) {
    static_assert(sizeof(Control) % sizeof(uint32_t) == 0, "the control block is cleared word by word");
    uint32_t* w = reinterpret_cast<uint32_t*>(ctl);
    for (uint32_t i = threadIdx.x; i < sizeof(Control) / sizeof(uint32_t); i += kSetupBlock) w[i] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        if (params) {
            first = params[0];
            seed = params[1];
        }
        job->first_sample = first;
        job->seed = seed;
        job->n_samples = n_samples;
        // ids past the limit still give well-defined sets; the caller is told
        if (first >= max_ids || n_samples > max_ids - first) ctl->err = kErrBadRange;
    }
}

__global__ void plan_report(const Control* ctl, unsigned long long capacity, int64_t* result) {
    const unsigned int err = ctl->err;
    int64_t status = BPT_OK;
    unsigned long long members = ctl->total;
    if (err & kErrBadRange) {
        status = BPT_EINVAL;
    } else if (err & kErrPoolOverflow) {
        status = BPT_ERANGE;
        members = ctl->pool_cursor;  // pool entries the call needed
    } else if (err) {
        status = BPT_EINTERNAL;
    } else if (members > capacity) {
        status = BPT_ERANGE;
    }
    result[0] = status;
    result[1] = (int64_t)members;
}

// Multi-job plans: clears the control block and writes every job's sample
// range and seed, from params[2 * ids[i]] (first_sample, seed) when params is
// not null (else the values the table already holds).
__global__ __launch_bounds__(kSetupBlock) void plan_setup_jobs(FusedJob* jobs, uint32_t n_jobs,
                                                               const uint64_t* params, const uint32_t* ids,
                                                               uint64_t max_ids, Control* ctl) {
    uint32_t* w = reinterpret_cast<uint32_t*>(ctl);
    for (uint32_t i = threadIdx.x; i < sizeof(Control) / sizeof(uint32_t); i += kSetupBlock) w[i] = 0u;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n_jobs; i += kSetupBlock) {
        FusedJob& j = jobs[i];
        if (params) {
            j.first_sample = params[2 * (size_t)ids[i]];
            j.seed = params[2 * (size_t)ids[i] + 1];
        }
        if (j.first_sample >= max_ids || j.n_samples > max_ids - j.first_sample) atomicOr(&ctl->err, kErrBadRange);
    }
}

// {status, members} of each job of a multi-job plan's launch, at
// result[2 * ids[i]]: as plan_report, with the job's own total and capacity.
__global__ __launch_bounds__(kSetupBlock) void plan_report_jobs(const Control* ctl,
                                                                const unsigned long long* totals,
                                                                const unsigned long long* capacities,
                                                                const uint32_t* ids, uint32_t n_jobs,
                                                                int64_t* result) {
    const unsigned int err = ctl->err;
    for (uint32_t i = threadIdx.x; i < n_jobs; i += kSetupBlock) {
        int64_t status = BPT_OK;
        unsigned long long members = totals[i];
        if (err & kErrBadRange) {
            status = BPT_EINVAL;
        } else if (err & kErrPoolOverflow) {
            status = BPT_ERANGE;
            members = ctl->pool_cursor;  // pool entries the launch needed
        } else if (err) {
            status = BPT_EINTERNAL;
        } else if (members > capacities[i]) {
            status = BPT_ERANGE;
        }
        result[2 * (size_t)ids[i]] = status;
        result[2 * (size_t)ids[i] + 1] = (int64_t)members;
    }
}

}  // namespace

hipError_t launch_plan_setup_jobs(FusedJob* jobs, uint32_t n_jobs, const uint64_t* params, const uint32_t* ids,
                                  uint64_t max_ids, Control* ctl, hipStream_t stream) {
    hipLaunchKernelGGL(plan_setup_jobs, dim3(1), dim3(kSetupBlock), 0, stream, jobs, n_jobs, params, ids, max_ids,
                       ctl);
    return hipGetLastError();
}

hipError_t launch_plan_report_jobs(const Control* ctl, const unsigned long long* totals,
                                   const unsigned long long* capacities, const uint32_t* ids, uint32_t n_jobs,
                                   int64_t* result, hipStream_t stream) {
    hipLaunchKernelGGL(plan_report_jobs, dim3(1), dim3(kSetupBlock), 0, stream, ctl, totals, capacities, ids,
                       n_jobs, result);
    return hipGetLastError();
}

hipError_t launch_plan_setup(FusedJob* job, const uint64_t* params, uint64_t first, uint64_t seed,
                             uint64_t n_samples, uint64_t max_ids, Control* ctl, hipStream_t stream) {
    hipLaunchKernelGGL(plan_setup, dim3(1), dim3(kSetupBlock), 0, stream, job, params, first, seed, n_samples,
                       max_ids, ctl);
    return hipGetLastError();
}

hipError_t launch_plan_report(const Control* ctl, unsigned long long capacity, int64_t* result, hipStream_t stream) {
    hipLaunchKernelGGL(plan_report, dim3(1), dim3(1), 0, stream, ctl, capacity, result);
    return hipGetLastError();
}

}  // namespace bpt
