// Device scratch of the allocation-free step (dgidp_step_noalloc in
// include/dgidp.h): one fixed array per GPU, in the code object's static
// device memory, so that the entry point never calls the allocator.  Each GPU
// the library runs on holds the array until the process ends.
//
// In host code the array's name stands for a host-side shadow, not a device
// address: the device address comes from hipGetSymbolAddress, taken once per
// device (with that device current) and kept per device; host code uses only
// that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dgidp_internal.h"

namespace dgidp {

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_lock;
void* g_ptr[kMaxDevices] = {};

}  // namespace

__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

int noalloc_scratch_setup()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return -1;
    std::lock_guard<std::mutex> g(g_lock);
    if (g_ptr[dev]) return 0;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return -1;
    }
    g_ptr[dev] = p;
    return 0;
}

void* noalloc_scratch(size_t* bytes)
{
    int dev = -1;
    if (bytes) *bytes = kNoallocScratchBytes;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_lock);
    return g_ptr[dev];
}

// a fill kernel rather than a memset, so that the clearing is also safe in a
// captured graph
int launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t s)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_fill_u64, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace dgidp
