// Device-resident scratch for the allocation-free entry point tp_bin_noalloc:
// one file-scope array per device holds the launch's sample descriptor, its
// edge table, the exact tier's counters and its deferral list, so a call
// needs no device allocation (graph capture, fixed-memory serving loops).
//
// In host code ``scratch`` names a host-side stand-in, not a device address:
// the device address is taken once per device with hipGetSymbolAddress and
// only that pointer is handed to kernels.  Every call on one device shares the
// array, which keeps the last call's contents; the set-up kernel rewrites the
// descriptor, the edges and the counters at the start of every call.  Calls
// that overlap on one device race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tp_kernel.h"
#include "tp_noalloc.h"

namespace tpk {

namespace {

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

struct SetupArgs {
    KSample k;
    int32_t nedges;
    double edges[NA_EDGES];
};
static_assert(sizeof(SetupArgs) <= 3584, "set-up kernel arguments beyond 3.5 KiB");

// Writes the descriptor and the edges into the scratch array and clears the
// list counters (a kernel, not a memset, so that callers may capture it).
__global__ __launch_bounds__(256) void tp_noalloc_setup(const SetupArgs a, unsigned char *base)
{
    KSample *k = reinterpret_cast<KSample *>(base + NA_SAMPLE_OFF);
    double *e = reinterpret_cast<double *>(base + NA_EDGES_OFF);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(base + NA_COUNT_OFF);
    if (threadIdx.x == 0) {
        *k = a.k;
        cnt[0] = 0u;
        cnt[1] = 0u;
    }
    for (int i = threadIdx.x; i < a.nedges; i += blockDim.x) e[i] = a.edges[i];
}

constexpr int MAX_DEVICES = 64;
std::mutex g_na_mu;
unsigned char *g_na_ptr[MAX_DEVICES] = {};

}  // namespace

hipError_t noalloc_scratch(int device, unsigned char **out)
{
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[device]) {
        // the current device is ``device``: its own copy of the array
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_na_ptr[device] = static_cast<unsigned char *>(p);
    }
    *out = g_na_ptr[device];
    return hipSuccess;
}

hipError_t launch_noalloc_setup(const KSample &k, const double *edges, int nedges, unsigned char *base,
                                hipStream_t st)
{
    SetupArgs a;
    a.k = k;
    a.nedges = nedges;
    for (int i = 0; i < nedges; ++i) a.edges[i] = edges[i];
    hipLaunchKernelGGL(tp_noalloc_setup, dim3(1), dim3(256), 0, st, a, base);
    return hipGetLastError();
}

}  // namespace tpk
