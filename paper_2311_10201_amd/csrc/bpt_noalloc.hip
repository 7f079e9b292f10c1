// Fixed device scratch of the allocation-free sampling call
// (bpt_sample_rrr_noalloc in bpt_capi.cpp).
//
// The scratch is one file-scope device array.  Every GPU the library runs on
// holds its own copy, at its own address, from the time the code object is
// loaded until the process ends.  Host code never passes the array's name to
// a kernel or a copy: in host code that name is only a stand-in for the device
// symbol.  noalloc_scratch() resolves the address once per device, with that
// device current, and every later use goes through the address it returns.
#include <algorithm>
#include <mutex>

#include "bpt.h"
#include "bpt_internal.hpp"

namespace bpt {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

constexpr int kFillBlock = 256;

__global__ __launch_bounds__(kFillBlock) void zero_fill(uint4* p, size_t n16) {
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    const size_t stride = (size_t)gridDim.x * kFillBlock;
    for (size_t i = (size_t)blockIdx.x * kFillBlock + threadIdx.x; i < n16; i += stride) p[i] = z;
}

}  // namespace

hipError_t noalloc_scratch(int device, void** addr) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_addr[device] = p;
    }
    *addr = g_addr[device];
    return hipSuccess;
}

hipError_t launch_zero_fill(void* p, size_t bytes, hipStream_t stream) {
    if (bytes == 0) return hipSuccess;
    if ((reinterpret_cast<uintptr_t>(p) & 15u) || (bytes & 15u)) return hipErrorInvalidValue;
    const size_t n16 = bytes / 16;
    const size_t blocks = std::min<size_t>((n16 + kFillBlock - 1) / kFillBlock, 4096);
    hipLaunchKernelGGL(zero_fill, dim3((unsigned)blocks), dim3(kFillBlock), 0, stream, static_cast<uint4*>(p), n16);
    return hipGetLastError();
}

}  // namespace bpt
