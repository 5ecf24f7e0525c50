// Internal interface between the host core (slsht_api.cpp, slsht_server.cpp)
// and the gfx950 kernels (slsht_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/slsht.h"

namespace slsht {

// Number of Wigner-d entries d^p_{q,q'} with p < L, |q|,|q'| <= p:
// sum_{p<L} (2p+1)^2 = L(4L^2-1)/3.
inline int64_t dtab_row_len(int L) { return (int64_t)L * (4LL * L * L - 1) / 3; }
// Offset of degree p inside one theta row of the table.
__host__ __device__ inline int dtab_off(int p) { return p * (4 * p * p - 1) / 3; }

// Work item of the synthesis kernels: output slot lm, degree l, order m, and
// the slot of order -m that is filled by conjugate symmetry (-1 if none).
struct Item {
    int lm, l, m, mirror;
};

// Device-resident plan data, shared by the launchers.
struct DevPlan {
    slsht_desc d;
    int n_theta_out;     // theta_hi - theta_lo
    int nslot_phi;       // (n_phi + 1) / 2 phi "slots": a and n_phi - a share one
    int ncp_omega;       // n_omega / 2 + 1 omega slots
    void* dtab;          // [n_theta_out][dtab_row_len(L_h)] double or float
    void* tw_phi;        // [L_h-1][nslot_phi] (cos, sin) double2 or float2
    void* tw_omega;      // [L_h-1][ncp_omega] (cos, sin) double2 or float2
    void* tw_full;       // ENERGY: [n_phi] float2 (cos, sin)(2 pi j / n_phi)
    double* qw;          // [n_theta] beta weights (FULL plans)
    Item* items;         // synthesis work items
    int n_items;
    Item* items_l;       // ENERGY: one item per degree (lm = l - l_lo)
    double2* A;          // coupling scratch [n_lm][L_h^2]
    int tb;              // theta rows per synthesis block
    int block;           // threads per synthesis block
    size_t lds_bytes;    // dynamic LDS of the synthesis kernel
};

// Launchers; each returns hipSuccess or the launch error.
hipError_t launch_wigner_table(const DevPlan& P, hipStream_t s);
hipError_t launch_coupling(const DevPlan& P, const double2* f, double2* A, hipStream_t s);
hipError_t launch_synthesis(const DevPlan& P, const double2* A, const double2* h, void* g,
                            hipStream_t s);
hipError_t launch_energy(const DevPlan& P, const double2* A, const double2* h, float* E,
                         hipStream_t s);
// ENERGY output limits of the MFMA kernel (checked on the host).
constexpr int kEnergyMaxOmega = 64;
constexpr int kEnergyMaxTiles = 136;   // (slot tiles x omega tiles) over 8 waves, 17 each
size_t energy_lds_for(const DevPlan& P);
hipError_t launch_inverse(const DevPlan& P, const void* g, double2 scale, double2* f_out,
                          hipStream_t s);
// Chooses tb / block / lds_bytes for a plan (host only; uses the LDS limit).
bool choose_synthesis_shape(DevPlan& P, size_t lds_limit);

}  // namespace slsht
