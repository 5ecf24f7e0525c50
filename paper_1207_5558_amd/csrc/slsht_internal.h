// Internal interface between the host core (slsht_api.cpp, slsht_server.cpp)
// and the gfx950 kernels (slsht_kernels.hip, slsht_synth.hip, slsht_energy.hip).  Not part
// of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/slsht.h"

namespace slsht {

// Wigner-d table rows hold the canonical entries d^p_{Q,Q'}(theta_b), p < L,
// 0 <= Q <= p, -Q <= Q' <= Q, at dtab_off(p) + Q^2 + Q + Q'; every other (q, q')
// follows from d_{q,q'} = (-1)^{q-q'} d_{q',q} = d_{-q',-q} (Section IV-B).
// Entries per row: sum_{p<L} (p+1)^2 = L(L+1)(2L+1)/6, a quarter of the full set.
__host__ __device__ inline int64_t dtab_row_len(int L) { return (int64_t)L * (L + 1) * (2 * L + 1) / 6; }
// Offset of degree p inside one theta row of the table.
__host__ __device__ inline int dtab_off(int p) { return p * (p + 1) * (2 * p + 1) / 6; }

// Azimuthal band-limit of the window: h_s^r = 0 for |r| >= n_az (n_az = L_h if unset).
inline int n_az_of(const slsht_desc& d) { return d.n_az > 0 ? d.n_az : d.L_h; }

// Device tables shared by every descriptor with the same window band-limit, grid,
// theta rows, precision and output kind: Wigner-d(theta_b), phi/omega twiddles,
// beta weights.  Freed when the last plan using them goes away.
struct Tables {
    int device = 0;
    int L_h = 0, n_phi = 0, n_theta = 0, n_omega = 0, theta_lo = 0, theta_hi = 0, precision = 0;
    bool energy = false;
    void* dtab = nullptr;       // [n_theta_out][dtab_row_len(L_h)] canonical; double for FP64
                                // and ENERGY plans, float for FP32 FULL plans
    void* tw_phi = nullptr;     // [L_h-1][(n_phi+1)/2] (cos, sin) double2 or float2
    void* tw_omega = nullptr;   // [L_h-1][n_omega/2+1] (cos, sin) double2 or float2
    void* tw_full = nullptr;    // ENERGY: phi twiddle fragments, float2 [nst][nkk][64]
    double* qw = nullptr;       // [n_theta] beta weights of the inverse
    size_t bytes = 0;
    ~Tables();
};

// Geometry of the ENERGY path (slsht_energy.hip): MFMA tiles, order chunks and workspace
// offsets, computed on the host from the descriptor and passed to the kernels by value.
struct EnergyGeom {
    int L, K, KP, nkk, N;            // window band-limit, 2L-1, L rounded up to 4, KP/4, n_az
    int n_phi, n_omega, ncw, nctp;   // grid; omega columns padded to nctp tiles of 16
    int nslot, nst, nsplit, nstb;    // phi slots, their 16-slot tiles, blocks per row, tiles each
    int per, tpw;                    // waves per omega tile, slot tiles per wave (kernel bucket)
    int n_theta_out, theta_lo, l_lo, n_l, real_pair;
    int mc, nchunks, rows, ntiles;   // orders per chunk, chunks, (l, m) rows and 16-row tiles
    int afrag_tile;                  // floats of A fragments per 16-row tile
    int64_t slab;                    // floats of P/M fragments per ((l, m), theta row)
    size_t off_w, off_af, off_pm, off_ep, total;   // workspace byte offsets and size
};

// Geometry of the staged FULL synthesis (slsht_staged.hip; window band-limits above 16,
// n_omega <= 64): U GEMM over chunks of items, then the phi stage from the P/M rows.
struct StagedGeom {
    int L, N, n_omega;               // band-limit, n_az, omega samples
    int n_theta_out, l_lo, real_pair, f64;
    int n_cols, ncol;                // (omega, theta row) columns n_omega * n_theta_out; to 16s
    int n_items, ntiles;             // items, 16-item tiles of the A fragments
    int afrag_tile;                  // elements of A fragments per 16-item tile
    int it;                          // items per block of the W/U kernel (16 or 8)
    int n_itiles, n_ctiles;          // item tiles (rounded up to 8s), 16-column tiles
    int cchunk, n_cchunks;           // column tiles per block, column chunks
    int threads;                     // threads per block
    size_t lds;                      // LDS bytes per block
    size_t off_w, off_af, total;     // workspace byte offsets and size
};

// Everything a launch needs for one descriptor.
struct DevPlan {
    slsht_desc d{};                 // theta_hi resolved
    std::shared_ptr<Tables> T;
    int n_theta_out = 0;            // theta_hi - theta_lo
    int nslot_phi = 0;              // (n_phi + 1) / 2 phi slots: a and n_phi - a share one
    int ncp_omega = 0;              // n_omega / 2 + 1 omega slots
    int64_t n_lm = 0;
    int n_items = 0;                // synthesis items: n_lm, or the m >= 0 pairs with REAL_PAIR
    double2* A = nullptr;           // coupling scratch owned by a public plan
    int tb = 1;                     // theta rows per synthesis block
    int block = 256;                // threads per synthesis block
    size_t lds_bytes = 0;           // dynamic LDS of the synthesis kernel
    EnergyGeom eg{};                // ENERGY plans: tiles, chunks, workspace layout
    bool staged = false;            // FULL plans synthesised by the W/U path (slsht_staged.hip)
    StagedGeom sg{};                // staged FULL plans: chunks, workspace layout
    void* ework = nullptr;          // ENERGY / staged plans: workspace of
                                    // workspace_bytes(*this) bytes
};

// Saves and restores the caller's current device around a library call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
    DeviceGuard(const DeviceGuard&) = delete;
    DeviceGuard& operator=(const DeviceGuard&) = delete;
};

// Thread-local error message (slsht_last_error), shared by the host files.
int set_error(int code, const char* fmt, ...);

// Host-only checks and sizes.
int check_desc(const slsht_desc* d);
size_t tables_bytes(const slsht_desc& d);
size_t coupling_bytes(const slsht_desc& d);
size_t output_bytes(const slsht_desc& d);
// Workspace of an ENERGY plan (the largest over device LDS sizes) or of a staged FULL
// plan; 0 for other FULL plans.
size_t workspace_bytes(const slsht_desc& d);
// Tables are keyed by the fields they depend on.
std::string tables_key(const slsht_desc& d);
// Builds the device tables for d on `device` (which must be current); synchronises
// only its own stream.  Returns SLSHT_OK or an error status (message set).
int build_tables(const slsht_desc& d, int device, std::shared_ptr<Tables>& out);
// Fills a DevPlan for d over existing tables (host only, no allocation).
int make_view(const slsht_desc& d, const std::shared_ptr<Tables>& T, size_t lds_limit,
              DevPlan& P);
// Enqueues coupling + synthesis (FULL or ENERGY) of one forward transform on s,
// with A as the coupling scratch (coupling_bytes(d)).
hipError_t enqueue_forward(const DevPlan& P, const double2* f, const double2* h, void* g,
                           double2* A, hipStream_t s);
size_t device_lds_limit(int device);
// Device address of this GPU's copy of the static scratch array of the allocation-free
// entry point (slsht_noalloc.hip), resolved once per device with that device current.
int noalloc_scratch(int device, void** out);

// Launchers; each returns hipSuccess or the launch error.
hipError_t launch_wigner_table(const DevPlan& P, hipStream_t s);
hipError_t launch_coupling(const DevPlan& P, const double2* f, double2* A, hipStream_t s);
// Coupling through the modulated-signal transform (slsht_modsht.hip); work holds
// modulated_workspace_bytes(d).
size_t modulated_workspace_bytes(const slsht_desc& d);
hipError_t launch_coupling_modulated(const DevPlan& P, const double2* f, double2* A, void* work,
                                     hipStream_t s);
// Factoring-of-rotations route on the minimal grid (slsht_factored.hip).
// Delta^p = d^p(pi/2), p < L, canonical layout (dtab_row_len(L) doubles).
hipError_t launch_delta_trapani(int L, double* out, hipStream_t s);
size_t factored_workspace_bytes(const slsht_desc& d);
hipError_t launch_factored(const DevPlan& P, const double2* A, const double2* h, double2* g,
                           void* work, hipStream_t s);
// Slepian window on R_(theta_c, a) (current device); h_out host complex128[L*L].
int slepian_window(int L, double theta_c, double a, double2* h_out, double* concentration);
hipError_t launch_synthesis(const DevPlan& P, const double2* A, const double2* h, void* g,
                            hipStream_t s);
// Up to kSynthBatchMax FULL transforms in one grid; they must share one synthesis
// kernel (equal synthesis_kernel_key) and block size.
constexpr int kSynthBatchMax = 16;
const void* synthesis_kernel_key(const DevPlan& P);
hipError_t launch_synthesis_batch(const DevPlan* const* P, const double2* const* A,
                                  const double2* const* h, void* const* g, int n, hipStream_t s);
// ENERGY path: W table, A fragments, P/M slabs and partial energies in P.ework.
hipError_t launch_energy(const DevPlan& P, const double2* A, const double2* h, float* E,
                         hipStream_t s);
// Where the W table puts entry (theta row t, row r = wq_off(q) + p - |q|, omega column c):
//   tiled = 0: W[t * tstride + r * rstride + c]; each theta row writes columns c < cw, those
//              with c >= n_omega as zeros;
//   tiled = 1: by tiles of 16 of the columns col = c * n_theta_out + t (theta fastest), each
//              tile holding all L_h^2 rows: W[((col / 16) * L_h^2 + r) * 16 + col % 16]; the
//              columns from n_omega * n_theta_out up to ncol (a multiple of 16) are zeros.
struct WtableLayout {
    int tiled;
    int64_t tstride, rstride;
    int cw, ncol;
};
// W^p_q(theta_b, omega_c) = sum_{q'} h_p^{q'} d^p_{q,q'}(theta_b) e^{-i q' omega_c} for every
// theta row of the table (slsht_staged.hip): d in FP64 (d64) or FP32, W stored complex128
// (w64) or complex64 in layout `lay`.
hipError_t launch_wtable(const void* dtab, bool d64, const double2* h, void* W, bool w64, int L,
                         int N, int n_omega, int n_theta_out, const WtableLayout& lay,
                         hipStream_t s);
// FULL synthesis through the W table and the U GEMM (W/U kernel): geometry (false if the
// plan does not qualify) and launch.
bool staged_geom(const slsht_desc& d, int n_theta_out, int n_items, StagedGeom& g);
hipError_t launch_synthesis_staged(const DevPlan& P, const double2* A, const double2* h, void* g,
                                   hipStream_t s);
// Workspace bytes of a plan view (ENERGY or staged FULL; 0 otherwise).
size_t plan_workspace_bytes(const DevPlan& P);
// Host-only: geometry of the ENERGY path for d (false if no tiling fits lds_limit).
bool energy_geom(const slsht_desc& d, int n_theta_out, size_t lds_limit, EnergyGeom& g);
// Twiddle fragments (cos, sin)(k phi_a) of the ENERGY phi stage, float pairs.
void energy_twiddles(const EnergyGeom& g, std::vector<float>& out);
size_t energy_twiddle_bytes(const EnergyGeom& g);
// f_out = k * (beta-weighted sum of g) / h[0], h_0^0 read on the device.
hipError_t launch_inverse(const DevPlan& P, const void* g, double k, const double2* h,
                          double2* f_out, hipStream_t s);
// Chooses tb / block / lds_bytes of the FULL synthesis (host only).
bool choose_synthesis_shape(DevPlan& P, size_t lds_limit);
size_t energy_lds_for(const DevPlan& P);

// ENERGY output limits of the MFMA kernels (checked on the host).
constexpr int kEnergyMaxOmega = 64;
// omega samples of the W table (its twiddles sit in 16 KB of LDS beside the h d rows)
constexpr int kWuThreads = 768;     // threads per block of the W/U kernel (12 waves)
constexpr int kWuMaxWaves = 16;     // waves per block of the W/U kernel, at most
constexpr int kWtableMaxOmega = 1024;
// LDS of one W/U block's P|M rows (the CU has 160 KB; a few hundred bytes stay static)
constexpr size_t kWuMaxLds = (size_t)156 << 10;
constexpr int kEnergyMaxTiles = 136;   // (slot tiles x omega tiles) over 8 waves, 17 each
constexpr int kEnergyMaxTpw = 17;
constexpr int kEnergyPhiWaves = 8;    // waves of one phi-stage block
// Workspace budget of the P/M slabs of one chunk of orders.
constexpr size_t kEnergyChunkBudget = (size_t)16 << 30;

}  // namespace slsht

// A public plan: the launch view and its device.
struct slsht_plan_s {
    slsht::DevPlan P;
    int device;
};
