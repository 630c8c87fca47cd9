// Device scratch of the allocation-free simulate entry point, and the small
// kernel that writes a scanner's subray table into it.
//
// `scratch` is a file-scope device array: every GPU the library runs on holds
// its own copy, at its own address, until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is a stand-in, not a
// device address); it looks the address up once per device with
// hipGetSymbolAddress and uses that.
#include <hip/hip_runtime.h>

#include <mutex>

#include "vls_internal.h"

namespace vls {
namespace {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
hipError_t g_status[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};

// A scanner's subray table, passed by value as the kernel's argument.
struct PatternArg {
    double v[5 * kWave];
};

__global__ void k_store_pattern(PatternArg a, int n, double* __restrict__ dst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = a.v[i];
}

}  // namespace

hipError_t noalloc_scratch(int device, void** ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_done[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != device) e = hipSetDevice(device);
        void* p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e == hipSuccess) g_ptr[device] = p;
        g_status[device] = e;
        g_done[device] = true;
        if (cur != device) (void)hipSetDevice(cur);
    }
    *ptr = g_ptr[device];
    return g_status[device];
}

hipError_t launch_store_pattern(const double* table, int n, double* dst, hipStream_t stream)
{
    if (n <= 0 || n > 5 * kWave) return hipErrorInvalidValue;
    PatternArg a;
    for (int i = 0; i < 5 * kWave; ++i) a.v[i] = i < n ? table[i] : 0.0;
    hipLaunchKernelGGL(k_store_pattern, dim3((n + 255) / 256), dim3(256), 0, stream, a, n, dst);
    return hipGetLastError();
}

}  // namespace vls
