// Host-side geometry of the MFMA paths: tiles, chunks and workspace layouts of the ENERGY
// kernels (slsht_energy.hip) and of the staged FULL synthesis (slsht_staged.hip), and the
// ENERGY twiddle table.  Host code only, so that it builds and runs under the host
// sanitizers without a GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "slsht_internal.h"

namespace slsht {

namespace {

// MFMA k-steps (2 complex degrees each) of the p-sum of U_{+-k}.
int u_steps(int L, int k) { return (L - k + 1) / 2; }

}  // namespace

bool energy_geom(const slsht_desc& d, int n_theta_out, size_t lds_limit, EnergyGeom& g) {
    g = EnergyGeom{};
    g.L = d.L_h;
    g.K = 2 * d.L_h - 1;
    g.KP = (d.L_h + 3) / 4 * 4;
    g.nkk = g.KP / 4;
    g.N = n_az_of(d);
    g.n_phi = d.n_phi;
    g.n_omega = d.n_omega;
    const int nct = (d.n_omega + 15) / 16;
    g.nctp = nct == 3 ? 4 : nct;                       // omega tiles padded to divide 8 waves
    g.ncw = g.nctp * 16;
    g.nslot = (d.n_phi + 1) / 2;
    g.nst = (g.nslot + 15) / 16;
    g.n_theta_out = n_theta_out;
    g.theta_lo = d.theta_lo;
    g.l_lo = d.l_lo;
    g.n_l = d.l_hi - d.l_lo;
    g.real_pair = (d.flags & SLSHT_REAL_PAIR) ? 1 : 0;
    // E3: the block's twiddle fragments live in LDS; split the slot tiles over several
    // blocks when one (l, theta) row's table does not fit
    const size_t per_tile = (size_t)g.nkk * 64 * sizeof(float2);
    const int fit = (int)std::min<size_t>(lds_limit / per_tile, (size_t)g.nst);
    if (fit < 1) return false;
    g.nsplit = (g.nst + fit - 1) / fit;
    g.nstb = (g.nst + g.nsplit - 1) / g.nsplit;
    g.per = kEnergyPhiWaves / g.nctp;
    const int tpw = (g.nstb + g.per - 1) / g.per;
    if (tpw > kEnergyMaxTpw) return false;
    g.tpw = tpw <= 4 ? 4 : (tpw <= 8 ? 8 : (tpw <= 12 ? 12 : kEnergyMaxTpw));   // kernel bucket
    g.slab = (int64_t)g.nctp * g.nkk * 64 * 4;
    // orders per chunk: the P/M slabs of one chunk within the workspace budget
    const int max_orders = g.real_pair ? d.l_hi : 2 * d.l_hi - 1;
    const size_t per_order = (size_t)g.n_l * n_theta_out * g.slab * sizeof(float);
    int mc = (int)std::max<size_t>(1, std::min<size_t>(kEnergyChunkBudget / per_order,
                                                       (size_t)max_orders));
    g.nchunks = (max_orders + mc - 1) / mc;
    g.mc = (max_orders + g.nchunks - 1) / g.nchunks;
    g.rows = g.n_l * g.mc;
    g.ntiles = (g.rows + 15) / 16;
    int steps = 0;
    for (int k = 0; k < g.L; ++k) steps += (k ? 2 : 1) * u_steps(g.L, k);
    g.afrag_tile = steps * 64;
    auto al = [](size_t n) { return (n + 255) / 256 * 256; };
    size_t off = 0;
    g.off_w = off;
    off += al((size_t)n_theta_out * g.L * g.L * g.ncw * sizeof(float2));
    g.off_af = off;
    off += al((size_t)g.ntiles * g.afrag_tile * sizeof(float));
    g.off_pm = off;
    off += al((size_t)g.rows * n_theta_out * g.slab * sizeof(float));
    g.off_ep = off;
    if (g.nchunks > 1)
        off += al((size_t)g.n_l * n_theta_out * g.nsplit * kEnergyPhiWaves * g.tpw * 8 * 64 *
                  sizeof(float));
    g.total = off;
    return true;
}

// Twiddle fragments of E3 (host): entry (st, kk, lane) = (cos, sin)(2 pi (k a mod n_phi) / n_phi),
// k = 4 kk + lane / 16, a = 16 st + lane % 16; zero for a >= nslot.  Phases reduced in integers.
void energy_twiddles(const EnergyGeom& g, std::vector<float>& out) {
    out.assign((size_t)g.nst * g.nkk * 64 * 2, 0.0f);
    for (int st = 0; st < g.nst; ++st)
        for (int kk = 0; kk < g.nkk; ++kk)
            for (int lane = 0; lane < 64; ++lane) {
                const int k = 4 * kk + lane / 16, a = 16 * st + lane % 16;
                if (a >= g.nslot) continue;
                const long long r = ((long long)k * a) % g.n_phi;
                const double ang = 2.0 * M_PI * (double)r / (double)g.n_phi;
                const size_t i = (((size_t)st * g.nkk + kk) * 64 + lane) * 2;
                out[i] = (float)std::cos(ang);
                out[i + 1] = (float)std::sin(ang);
            }
}

size_t energy_twiddle_bytes(const EnergyGeom& g) { return (size_t)g.nst * g.nkk * 64 * sizeof(float2); }

size_t energy_lds_for(const DevPlan& P) {
    return (size_t)P.eg.nstb * P.eg.nkk * 64 * sizeof(float2);
}

bool staged_geom(const slsht_desc& d, int n_theta_out, int n_items, StagedGeom& g) {
    g = StagedGeom{};
    // At window band-limits up to 16 the fused kernel of slsht_synth.hip (theta stage on the
    // VALU, beside other blocks' phi stages on the matrix cores) is faster (measured at
    // L_h = 16, L_f = 128 and 192: by 5-24%, FP64 and FP32).  Above 16 its theta stage
    // (sum_p (2p+1)^2 complex MACs per theta row and item) outweighs the rest, and this path
    // is ahead (the minimal grid of L_h = 18: 9.6 against 13.4 ms FP64).
    if (d.output_mode != SLSHT_OUT_FULL || d.L_h <= 16 || d.n_omega > kWtableMaxOmega) return false;
    g.L = d.L_h;
    g.N = n_az_of(d);
    g.n_omega = d.n_omega;
    g.n_theta_out = n_theta_out;
    g.n_cols = n_theta_out * d.n_omega;
    g.ncol = (g.n_cols + 15) / 16 * 16;
    g.l_lo = d.l_lo;
    g.real_pair = (d.flags & SLSHT_REAL_PAIR) ? 1 : 0;
    g.f64 = d.precision == SLSHT_FP64 ? 1 : 0;
    g.n_items = n_items;
    g.ntiles = (n_items + 15) / 16;
    int steps = 0;
    for (int k = 0; k < g.L; ++k) steps += (k ? 2 : 1) * u_steps(g.L, k);
    g.afrag_tile = steps * 64;
    const size_t vb = g.f64 ? 16 : 8, rb = g.f64 ? 8 : 4;
    // block: `it` items x 16 (omega, theta row) columns at a time; its P|M rows (2L + 1
    // complex each) sit in LDS.  The columns run over omega and theta rows together, so only
    // the last of the n_omega * n_theta_out columns' tiles carries padding.
    g.it = (size_t)16 * 16 * (2 * g.L + 1) * vb <= kWuMaxLds ? 16 : 8;
    g.lds = (size_t)g.it * 16 * (2 * g.L + 1) * vb;
    g.threads = kWuThreads;
    g.n_itiles = ((n_items + g.it - 1) / g.it + 7) / 8 * 8;
    g.n_ctiles = g.ncol / 16;
    // column tiles per block: as many as keep >= 8192 blocks in the grid (32 rounds of one
    // block per CU; measured 2-4% ahead of 4096 and of 16384 at L_h = 18 and 24)
    int cc = (int)std::max<int64_t>(1, (int64_t)g.n_itiles * g.n_ctiles / 8192);
    cc = std::min(cc, std::max(1, g.n_ctiles));
    g.n_cchunks = (g.n_ctiles + cc - 1) / cc;
    g.cchunk = (g.n_ctiles + g.n_cchunks - 1) / g.n_cchunks;
    auto al = [](size_t n) { return (n + 255) / 256 * 256; };
    size_t off = 0;
    g.off_w = off;
    off += al((size_t)g.L * g.L * g.ncol * vb);
    g.off_af = off;
    off += al((size_t)g.ntiles * g.afrag_tile * rb);
    g.total = off;
    return true;
}

}  // namespace slsht
