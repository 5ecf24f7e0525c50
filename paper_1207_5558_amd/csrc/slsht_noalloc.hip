// Allocation-free forward entry point: the coupling scratch of slsht_forward lives in
// a file-scope device array instead of the plan's own buffer, so a call allocates
// nothing.  Each GPU holds its own copy of the array for the life of the process.
#include <hip/hip_runtime.h>

#include <mutex>

#include "slsht_internal.h"

namespace {

// The array's name is a host-side stand-in in host code; the device address of each
// GPU's copy comes from hipGetSymbolAddress (scratch_ptr below) and is the only form
// passed to kernels.
__device__ __align__(256) unsigned char scratch[SLSHT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

namespace slsht {

// Resolves (once per device, with `device` current) the device address of this GPU's
// copy of the scratch array.  Returns SLSHT_OK and the address, or an error status.
int noalloc_scratch(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices)
        return set_error(SLSHT_EINVAL, "device %d beyond the %d devices the allocation-free "
                                       "entry point tracks", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(SLSHT_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s",
                             device, hipGetErrorString(e));
        g_ptr[device] = p;
    }
    *out = g_ptr[device];
    return SLSHT_OK;
}

}  // namespace slsht

extern "C" int slsht_forward_noalloc(slsht_plan_t plan, const void* f, const void* h, void* g,
                                     void* stream) {
    if (!plan || !f || !h || !g) return slsht::set_error(SLSHT_EINVAL, "NULL argument");
    const slsht::DevPlan& P = plan->P;
    const size_t need = slsht::coupling_bytes(P.d);
    if (need > (size_t)SLSHT_NOALLOC_SCRATCH_BYTES)
        return slsht::set_error(SLSHT_ETOOBIG,
                                "coupling scratch of %zu bytes exceeds the %zu-byte static "
                                "scratch of slsht_forward_noalloc", need,
                                (size_t)SLSHT_NOALLOC_SCRATCH_BYTES);
    slsht::DeviceGuard guard(plan->device);
    if (!guard.ok) return slsht::set_error(SLSHT_EDEVICE, "hipSetDevice failed");
    void* A = nullptr;
    const int rc = slsht::noalloc_scratch(plan->device, &A);
    if (rc) return rc;
    const hipError_t e = slsht::enqueue_forward(P, (const double2*)f, (const double2*)h, g,
                                                (double2*)A, (hipStream_t)stream);
    if (e != hipSuccess)
        return slsht::set_error(SLSHT_EDEVICE, "forward launch: %s", hipGetErrorString(e));
    return SLSHT_OK;
}
