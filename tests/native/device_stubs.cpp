// Stand-ins for the device-side launchers of libslsht, so that the host core
// (slsht_api.cpp, slsht_server.cpp, slsht_geom.cpp) links into a sanitizer build with g++
// and runs on a machine without a GPU: every launcher reports that there is no device.
#include <hip/hip_runtime.h>

#include "../../paper_1207_5558_amd/csrc/slsht_internal.h"

namespace slsht {

bool choose_synthesis_shape(DevPlan& P, size_t) {
    P.tb = 1;
    P.block = 256;
    P.lds_bytes = 0;
    return true;
}
const void* synthesis_kernel_key(const DevPlan& P) { return &P; }
size_t factored_workspace_bytes(const slsht_desc&) { return 0; }
size_t modulated_workspace_bytes(const slsht_desc&) { return 0; }
int noalloc_scratch(int, void** out) {
    *out = nullptr;
    return set_error(SLSHT_EDEVICE, "no device");
}
int slepian_window(int, double, double, double2*, double*) {
    return set_error(SLSHT_EDEVICE, "no device");
}
hipError_t launch_wigner_table(const DevPlan&, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_coupling(const DevPlan&, const double2*, double2*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_coupling_modulated(const DevPlan&, const double2*, double2*, void*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_delta_trapani(int, double*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_factored(const DevPlan&, const double2*, const double2*, double2*, void*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_synthesis(const DevPlan&, const double2*, const double2*, void*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_synthesis_batch(const DevPlan* const*, const double2* const*, const double2* const*,
                                  void* const*, int, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_energy(const DevPlan&, const double2*, const double2*, float*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_inverse(const DevPlan&, const void*, double, const double2*, double2*, hipStream_t) {
    return hipErrorNoDevice;
}

}  // namespace slsht
