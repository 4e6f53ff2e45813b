// The allocation-free entry point, abft_stencil_run_noalloc: an online or plain run whose whole
// workspace (checksum planes, constant-term checksums, flag slots, counters, event log, fault
// plan) lies in one static device array of ABFT_NOALLOC_SCRATCH_BYTES per GPU instead of
// memory from hipMalloc.  Every call on a GPU shares that GPU's array, which keeps the last
// call's contents (the run clears what must start at zero); calls that overlap on one GPU race.
#include <mutex>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "abft_internal.h"

// The workspace.  In host code its name is only a stand-in for the symbol: its device address
// on the current GPU comes from hipGetSymbolAddress (scratch_address below), and only that
// address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[ABFT_NOALLOC_SCRATCH_BYTES];

namespace abft {

// One thread per sweep index t: a binary search of the sweep-sorted plan.
__global__ void fault_index_kernel(const abft_fault* f, int32_t n, int32_t* first, int64_t tmax)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > tmax) return;
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (f[mid].sweep < t) lo = mid + 1;
        else hi = mid;
    }
    first[t] = lo;
}

hipError_t launch_fault_index(const abft_fault* faults, int32_t n, int32_t* first, int64_t tmax,
                              hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (tmax + 1 + 255) / 256;
    hipLaunchKernelGGL(fault_index_kernel, dim3((unsigned)blocks), dim3(256), 0, st, faults, n,
                       first, tmax);
    return hipGetLastError();
}

}  // namespace abft

namespace {

std::mutex g_scratch_mu;
unsigned char* g_scratch[abft::kMaxDevices];  // device address of `scratch` per GPU, or null

// The array's address on the current device, looked up once per device with that device
// current (each GPU holds its own copy at its own address).
abft_status scratch_address(unsigned char** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return abft::run_error(ABFT_E_HIP, "no current device");
    if (dev < 0 || dev >= abft::kMaxDevices)
        return abft::run_error(ABFT_E_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev] == nullptr) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) {
            (void)hipGetLastError();
            return abft::run_error(ABFT_E_HIP, "hipGetSymbolAddress of the scratch array failed");
        }
        g_scratch[dev] = static_cast<unsigned char*>(ptr);
    }
    *out = g_scratch[dev];
    return ABFT_OK;
}

}  // namespace

extern "C" abft_status abft_stencil_run_noalloc(const abft_problem* p, const abft_options* o,
                                                const abft_fault* faults, int32_t nfaults,
                                                int64_t nsweeps, void* hip_stream,
                                                abft_report* out)
{
    roctxRangePushA("abft_stencil_run_noalloc");
    struct Pop {
        ~Pop() { roctxRangePop(); }
    } pop;
    try {
        abft::NoAllocLayout L{};
        abft_status s = abft::noalloc_layout(p, o, faults, nfaults,
                                             (size_t)ABFT_NOALLOC_SCRATCH_BYTES, &L);
        if (s) return s;
        unsigned char* ws = nullptr;
        if ((s = scratch_address(&ws))) return s;
        return abft::run_in_workspace(p, o, faults, nfaults, nsweeps, hip_stream, ws, L, out);
    } catch (...) {
        return abft::run_error(ABFT_E_NOMEM, "host allocation failed");
    }
}
