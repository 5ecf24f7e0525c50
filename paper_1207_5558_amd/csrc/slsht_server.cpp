// Serving loop of the directional SLSHT library (continuous batching).
#include <hip/hip_runtime.h>

#include "slsht_internal.h"

extern "C" {
int slsht_server_create(int, size_t, int, slsht_server_t* out) {
    if (out) *out = nullptr;
    return SLSHT_EINVAL;
}
int slsht_server_destroy(slsht_server_t) { return SLSHT_EINVAL; }
int slsht_submit(slsht_server_t, const slsht_desc*, const void*, const void*, uint64_t*) { return SLSHT_EINVAL; }
int slsht_poll(slsht_server_t, uint64_t, int*, const void**, size_t*, int*) { return SLSHT_EINVAL; }
int slsht_wait(slsht_server_t, uint64_t, int) { return SLSHT_EINVAL; }
int slsht_release(slsht_server_t, uint64_t) { return SLSHT_EINVAL; }
int slsht_request_times(slsht_server_t, uint64_t, double*, double*, double*) { return SLSHT_EINVAL; }
double slsht_server_clock(slsht_server_t) { return 0.0; }
}
