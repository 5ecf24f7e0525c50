// gfx950 kernels of the ENERGY output of the directional SLSHT forward path:
// E(rho; l) = sum_m |g(rho; l, m)|^2, FP32-mixed, reduced over the orders m so that g is
// never written.
//
// The separated form (eq. Eq:alternative_harmonic_formulation_wigner with the separation
// of variables of Section IV-B) is summed in this order:
//
//   W^p_q(theta_b, omega_c) = sum_{|q'| <= p} h_p^{q'} d^p_{q,q'}(theta_b) e^{-i q' omega_c}
//                                                        (FP64, once per call; no (l, m))
//   U_q(theta_b, omega_c; l, m) = sum_{p >= |q|} A^p_q(l, m) W^p_q(theta_b, omega_c)
//                                  (per (theta_b, q) a GEMM over the (l, m) rows, on MFMA)
//   P_k = U_k + U_{-k},  M_k = -i (U_k - U_{-k})          (k >= 0; P_0 = U_0, M_0 = 0)
//   g(phi_a) = sum_k cos(k phi_a) P_k + sin(k phi_a) M_k,  g(phi_{n-a}) = same with - sin
//                           (per (l, theta_b) a GEMM over the phi slots, on MFMA)
//   E(phi_a) += |g(phi_a)|^2,  E(phi_{n-a}) += |g(phi_{n-a})|^2.
//
// The p- and q'-sums are the theta and omega stages of the FULL kernels taken in the other
// order: the q'-sum no longer depends on (l, m), so it is done once per theta row, and the
// p-sum becomes a dense contraction shared by all orders.  Kernels per call:
//   E0 wtable_kernel        W for every theta row (slsht_staged.hip)    -> workspace
// and per chunk of orders (mc orders of every degree; the P/M slabs of a chunk sit in the
// workspace, and E is carried across chunks in a partial buffer in register-tile order):
//   E1 energy_afrag_kernel  A^p_{+-k} of the chunk's (l, m) rows in MFMA fragment order, FP32,
//                           scaled by sqrt(2) for m > 0 on the real-pair path
//   E2 energy_u_kernel      U, the fold into P_k, M_k, stored as B fragments of E3
//   E3 energy_phi_kernel    phi synthesis + |g|^2 accumulation, the bulk of the work
// MFMA lane layout (v_mfma_f32_16x16x4f32, verified on gfx950): lane l supplies A[l%16][l/16]
// and B[l/16][l%16] and receives D rows 4*(l/16)+r, column l%16.
#include "slsht_device.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

namespace slsht {

namespace {

constexpr int kUWaves = 8;        // E2: one 16-row tile per wave

// MFMA k-steps (2 complex degrees each) of the p-sum of U_{+-k}.
__host__ __device__ inline int u_steps(int L, int k) { return (L - k + 1) / 2; }

__device__ inline int orders_of(const EnergyGeom& g, int l) { return g.real_pair ? l + 1 : 2 * l + 1; }

__device__ inline f4v mfma4(float a, float b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

}  // namespace

// ------------------------------------------------------------------------------
// E1: the chunk's coupling rows in A-fragment order.  Row r of the chunk is degree
// l_lo + r / mc, order index chunk*mc + r % mc (m = that index - l, or the index itself on the
// real-pair path); rows past a degree's last order are zero.  Step s of U_{+-k} holds, in lane
// (i, j4), component (j4 & 1) of A^p_{+-k} with p = k + 2s + (j4 >> 1) for row 16*tile + i.
__global__ void __launch_bounds__(64) energy_afrag_kernel(const double2* __restrict__ A,
                                                          float* __restrict__ af,
                                                          const EnergyGeom g, int chunk) {
    const int tile = blockIdx.x, lane = threadIdx.x;
    const int row = tile * 16 + (lane & 15), j4 = lane >> 4;
    const int L = g.L;
    const int li = row / g.mc, mj = row - li * g.mc;
    bool valid = li < g.n_l;
    int64_t lm = 0;
    double w = 1.0;
    if (valid) {
        const int l = g.l_lo + li;
        const int mi = chunk * g.mc + mj;
        valid = mi < orders_of(g, l);
        const int m = g.real_pair ? mi : mi - l;
        lm = (int64_t)l * l + l + m - (int64_t)g.l_lo * g.l_lo;
        // real pair: E = |g_0|^2 + 2 sum_{m>0} |g_m|^2, the weight folded into A
        if (g.real_pair && m > 0) w = 1.4142135623730951;
    }
    float* out = af + (int64_t)tile * g.afrag_tile + lane;
    int off = 0;
    for (int k = 0; k < L; ++k) {
        const int steps = u_steps(L, k);
        for (int sg = 0; sg < (k ? 2 : 1); ++sg) {
            const int q = sg ? -k : k;
            for (int s = 0; s < steps; ++s) {
                const int p = k + 2 * s + (j4 >> 1);
                float v = 0.0f;
                if (valid && p < L) {
                    const double2 a = A[lm * L * L + p * p + p + q];
                    v = (float)(w * ((j4 & 1) ? a.y : a.x));
                }
                out[(int64_t)(off + s) * 64] = v;
            }
            off += steps;
        }
    }
}

// ------------------------------------------------------------------------------
// E2: U_{+-k}(theta_b, omega_c) for 16 rows per wave as complex GEMMs on real MFMAs
// (complex inner index p expanded to (Re, Im), B = [[W_re, W_im], [-W_im, W_re]] row pairs),
// then P_k, M_k stored as the B fragments of E3: slab (row, theta), entry
// ((ct * nkk + k / 4) * 64 + (k % 4) * 16 + c % 16) holds float4 (P.re, P.im, M.re, M.im)
// of omega column c = 16 ct + c % 16.  W_{+-k} of the block's theta row is staged in LDS.
__global__ void __launch_bounds__(64 * kUWaves) energy_u_kernel(const float2* __restrict__ W,
                                                                const float* __restrict__ af,
                                                                float* __restrict__ pm,
                                                                const EnergyGeom g, int chunk) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* Ws = reinterpret_cast<float2*>(smem_raw);   // [<= 2 (L-1) or L rows][ncw]
    const int L = g.L, ncw = g.ncw;
    const int t = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = blockIdx.y * kUWaves + wave;
    const bool active = tile < g.ntiles;
    const int j4 = lane >> 4, col = lane & 15;
    const float2* Wt = W + (int64_t)t * L * L * ncw;
    const float* aft = af + (int64_t)(active ? tile : 0) * g.afrag_tile + lane;

    // the four output rows of this lane: 16 * tile + 4 * j4 + r
    int64_t base[4];
    bool rv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = tile * 16 + 4 * j4 + r;
        const int li = row / g.mc, mj = row - li * g.mc;
        rv[r] = active && li < g.n_l && chunk * g.mc + mj < orders_of(g, g.l_lo + li);
        base[r] = (((int64_t)li * g.n_theta_out + t) * g.mc + mj) * g.slab + (int64_t)col * 4;
    }

    // W_{+-k} of the next k is loaded into registers while the MFMAs of this k run
    // (at most (2L-2) * 64 / 2 float4 over the block's threads: 4 each)
    constexpr int kWPer = (2 * SLSHT_MAX_LH - 2) * kEnergyMaxOmega / 2 / (64 * kUWaves) + 1;
    float4 wr[kWPer];
    auto load_w = [&](int k) {
        const int n4 = (k ? 2 * (L - k) : L) * ncw / 2;
        const float4* src = reinterpret_cast<const float4*>(Wt + (int64_t)wq_off(L, k) * ncw);
#pragma unroll
        for (int i = 0; i < kWPer; ++i) {
            const int idx = threadIdx.x + i * 64 * kUWaves;
            wr[i] = idx < n4 ? src[idx] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
    };
    // the A fragments of the next k likewise (steps <= 16 per sign; L2-resident)
    float apn[16], amn[16];
    auto load_a = [&](int k, int off) {
        const int steps = u_steps(L, k);
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            apn[s] = (active && s < steps) ? aft[(int64_t)(off + s) * 64] : 0.0f;
            amn[s] = (active && k && s < steps) ? aft[(int64_t)(off + steps + s) * 64] : 0.0f;
        }
    };
    load_w(0);
    load_a(0, 0);
    int aoff = 0;
    for (int k = 0; k < L; ++k) {
        const int steps = u_steps(L, k);
        __syncthreads();
        {
            const int n4 = (k ? 2 * (L - k) : L) * ncw / 2;
            float4* dst = reinterpret_cast<float4*>(Ws);
#pragma unroll
            for (int i = 0; i < kWPer; ++i) {
                const int idx = threadIdx.x + i * 64 * kUWaves;
                if (idx < n4) dst[idx] = wr[i];
            }
        }
        __syncthreads();
        float ap[16], am[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            ap[s] = apn[s];
            am[s] = amn[s];
        }
        const int aoff_next = aoff + (k ? 2 : 1) * steps;
        if (k + 1 < L) {
            load_w(k + 1);
            load_a(k + 1, aoff_next);
        }
        if (active) {
            const int lastp = L - k - 1;                    // last row of W_{+k}
            for (int ct = 0; ct < g.nctp; ++ct) {
                f4v upr = {0, 0, 0, 0}, upi = {0, 0, 0, 0}, umr = {0, 0, 0, 0}, umi = {0, 0, 0, 0};
                const float2* wcol = Ws + ct * 16 + col;
#pragma unroll
                for (int s = 0; s < 16; ++s) {
                    if (s >= steps) break;
                    // rows past the last degree meet a zero A fragment; clamp them in range
                    const int rp = min(2 * s + (j4 >> 1), lastp);
                    const float2 wp = wcol[rp * ncw];
                    upr = mfma4(ap[s], (j4 & 1) ? -wp.y : wp.x, upr);
                    upi = mfma4(ap[s], (j4 & 1) ? wp.x : wp.y, upi);
                    if (k) {
                        const float2 wm = wcol[(L - k + rp) * ncw];
                        umr = mfma4(am[s], (j4 & 1) ? -wm.y : wm.x, umr);
                        umi = mfma4(am[s], (j4 & 1) ? wm.x : wm.y, umi);
                    }
                }
                const int64_t e = ((int64_t)(ct * g.nkk + (k >> 2)) * 64 + (k & 3) * 16) * 4;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (!rv[r]) continue;
                    float4 v;
                    v.x = upr[r] + umr[r];
                    v.y = upi[r] + umi[r];
                    v.z = k ? upi[r] - umi[r] : 0.0f;                // M_0 = 0
                    v.w = k ? umr[r] - upr[r] : 0.0f;
                    *reinterpret_cast<float4*>(pm + base[r] + e) = v;
                }
            }
        }
        aoff = aoff_next;
    }
    // rows k = L .. KP-1 of the last k-step are zero (the phi kernel reads whole steps)
    for (int k = L; k < g.KP; ++k)
        for (int ct = 0; ct < g.nctp; ++ct) {
            const int64_t e = ((int64_t)(ct * g.nkk + (k >> 2)) * 64 + (k & 3) * 16) * 4;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (rv[r])
                    *reinterpret_cast<float4*>(pm + base[r] + e) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
}

// ------------------------------------------------------------------------------
// E3: phi synthesis and energy.  One block = one degree l x one theta row x one slot range
// (all of the row's slots unless the twiddle table must be split), the chunk's orders in a
// loop.  Wave w owns omega tile ct = w % nctp and slot tiles st = st0 + j * per; per order
// it loads its B fragments (P_k, M_k of that omega tile, float4 per k-step) from the slab
// and, per slot tile, runs four real GEMMs [16 slots x k] . [k x 16 omega] with A fragments
// (cos, sin)(k phi_a) from the LDS table in fragment order (one contiguous 512-B read per
// k-step), then E(a) += |C + S|^2, E(n - a) += |C - S|^2.  The energies stay in registers
// over the chunk; between chunks they go to the partial buffer in register order.
template <int TPW, int NKK>
__global__ void __launch_bounds__(64 * kEnergyPhiWaves) energy_phi_kernel(
    const float* __restrict__ pm, const float2* __restrict__ twf, float* __restrict__ ep,
    float* __restrict__ E, const EnergyGeom g, int chunk) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* tws = reinterpret_cast<float2*>(smem_raw);   // [nstb][NKK][64], NKK == g.nkk
    const int row_blk = blockIdx.x / g.nsplit, sp = blockIdx.x - row_blk * g.nsplit;
    const int li = row_blk / g.n_theta_out, t = row_blk - li * g.n_theta_out;
    const int l = g.l_lo + li;
    const int nm = orders_of(g, l);
    const int m0 = chunk * g.mc;
    if (m0 >= nm) return;
    const int cnt = min(g.mc, nm - m0);
    const bool first = chunk == 0, last = m0 + cnt >= nm;
    const int st_lo = sp * g.nstb, st_hi = min(g.nst, st_lo + g.nstb);
    const int nkk = g.nkk;
    {
        const float4* src = reinterpret_cast<const float4*>(twf + (int64_t)st_lo * nkk * 64);
        float4* dst = reinterpret_cast<float4*>(tws);
        for (int i = threadIdx.x; i < (st_hi - st_lo) * nkk * 32; i += blockDim.x) dst[i] = src[i];
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kq = lane >> 4, col = lane & 15;
    const int ct = wave % g.nctp, st0 = wave / g.nctp, per = g.per;

    float Ep[TPW][4], Em[TPW][4];
    float4* epb = reinterpret_cast<float4*>(ep) +
                  ((int64_t)blockIdx.x * kEnergyPhiWaves + wave) * TPW * 2 * 64 + lane;
    if (first) {
#pragma unroll
        for (int j = 0; j < TPW; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) { Ep[j][r] = 0.0f; Em[j][r] = 0.0f; }
    } else {
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
            const float4 a = epb[(2 * j) * 64], b = epb[(2 * j + 1) * 64];
            Ep[j][0] = a.x; Ep[j][1] = a.y; Ep[j][2] = a.z; Ep[j][3] = a.w;
            Em[j][0] = b.x; Em[j][1] = b.y; Em[j][2] = b.z; Em[j][3] = b.w;
        }
    }
    __syncthreads();

    const float4* slab0 = reinterpret_cast<const float4*>(pm + (int64_t)row_blk * g.mc * g.slab) +
                          (int64_t)ct * nkk * 64 + lane;
    const int64_t slab4 = g.slab / 4;
    // B fragments (rows k >= L of a slab hold zeros, so they are used as loaded)
    float4 b[NKK];
    auto load_b = [&](int mj) {
        const float4* sb = slab0 + (int64_t)mj * slab4;
#pragma unroll
        for (int kk = 0; kk < NKK; ++kk) b[kk] = sb[kk * 64];
    };
    // One float per 128-B line of this wave's part of an order's slab: pulls the order after
    // next into L2; the value is consumed an order later, so the load never stalls.
    auto touch_b = [&](int mj) {
        return reinterpret_cast<const float*>(slab0 - lane + (int64_t)mj * slab4)
            [(lane % (NKK * 8)) * 32];
    };
    // Software pipeline over the tiles of all orders: the MFMAs of tile j are issued first;
    // then the A fragments of the next tile are loaded and the energy of the previous tile
    // is updated from its accumulators while tile j's MFMAs occupy the matrix core.  After
    // the last tile's MFMAs the next order's B fragments are loaded the same way.
    auto energy_update = [&](int j, const f4v& cre, const f4v& cim, const f4v& sre,
                             const f4v& sim) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float pr = cre[r] + sre[r], pi = cim[r] + sim[r];
            const float mr = cre[r] - sre[r], mi = cim[r] - sim[r];
            Ep[j][r] = fmaf(pi, pi, fmaf(pr, pr, Ep[j][r]));
            Em[j][r] = fmaf(mi, mi, fmaf(mr, mr, Em[j][r]));
        }
        // Materialise this tile's energy here, so that its MFMA accumulators die now
        // (otherwise the updates sink to the end of the unrolled loop and every tile's
        // accumulators stay live at once).
        asm volatile("" : "+v"(Ep[j][0]), "+v"(Ep[j][1]), "+v"(Ep[j][2]), "+v"(Ep[j][3]),
                     "+v"(Em[j][0]), "+v"(Em[j][1]), "+v"(Em[j][2]), "+v"(Em[j][3]));
    };
    load_b(0);
    float touch = touch_b(min(1, cnt - 1));
    f4v pcre = {0, 0, 0, 0}, pcim = {0, 0, 0, 0}, psre = {0, 0, 0, 0}, psim = {0, 0, 0, 0};
    for (int mj = 0; mj < cnt; ++mj) {
        // The LDS offset is made opaque per order so that the twiddle loads (invariant
        // over the orders) are not hoisted out of this loop into registers.
        int tw_lane = lane;
        asm volatile("" : "+v"(tw_lane));
        // tiles past the block's range repeat its last tile (never stored)
        auto tile_tw = [&](int j) {
            const int st = min(st_lo + st0 + j * per, st_hi - 1);
            return tws + (st - st_lo) * NKK * 64 + tw_lane;
        };
        float2 z[NKK];
#pragma unroll
        for (int kk = 0; kk < NKK; ++kk) z[kk] = tile_tw(0)[kk * 64];
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
            f4v cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0}, sre = {0, 0, 0, 0}, sim = {0, 0, 0, 0};
#pragma unroll
            for (int kk = 0; kk < NKK; ++kk) {
                cre = mfma4(z[kk].x, b[kk].x, cre);
                cim = mfma4(z[kk].x, b[kk].y, cim);
                sre = mfma4(z[kk].y, b[kk].z, sre);
                sim = mfma4(z[kk].y, b[kk].w, sim);
            }
            __builtin_amdgcn_sched_barrier(0);
            if (j + 1 < TPW) {
#pragma unroll
                for (int kk = 0; kk < NKK; ++kk) z[kk] = tile_tw(j + 1)[kk * 64];
            } else {
                // next order (the last order reloads itself: clamped, branch-free)
                asm volatile("" ::"v"(touch));
                load_b(min(mj + 1, cnt - 1));
                touch = touch_b(min(mj + 2, cnt - 1));
            }
            // previous tile (at j = 0 the last tile of the previous order; before the first
            // order its accumulators are zero and add nothing)
            energy_update(j > 0 ? j - 1 : TPW - 1, pcre, pcim, psre, psim);
            __builtin_amdgcn_sched_barrier(0);
            pcre = cre;
            pcim = cim;
            psre = sre;
            psim = sim;
        }
    }
    energy_update(TPW - 1, pcre, pcim, psre, psim);
    asm volatile("" ::"v"(touch));

    if (!last) {
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
            epb[(2 * j) * 64] = make_float4(Ep[j][0], Ep[j][1], Ep[j][2], Ep[j][3]);
            epb[(2 * j + 1) * 64] = make_float4(Em[j][0], Em[j][1], Em[j][2], Em[j][3]);
        }
        return;
    }
    // final store: lane holds slots 16 st + 4 kq + r of omega column 16 ct + col
    const int c = ct * 16 + col;
    if (c >= g.n_omega) return;
    float* row = E + (((int64_t)li * g.n_omega + c) * g.n_theta_out + t) * g.n_phi;
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
        const int st = st_lo + st0 + j * per;
        if (st >= st_hi) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int s = st * 16 + 4 * kq + r;
            if (s >= g.nslot) continue;
            row[s] = Ep[j][r];
            if (s > 0) row[g.n_phi - s] = Em[j][r];
        }
    }
}

hipError_t launch_energy(const DevPlan& P, const double2* A, const double2* h, float* E,
                         hipStream_t s) {
    const EnergyGeom& g = P.eg;
    char* ws = static_cast<char*>(P.ework);
    if (!ws) return hipErrorInvalidValue;
    float2* W = reinterpret_cast<float2*>(ws + g.off_w);
    float* af = reinterpret_cast<float*>(ws + g.off_af);
    float* pm = reinterpret_cast<float*>(ws + g.off_pm);
    float* ep = reinterpret_cast<float*>(ws + g.off_ep);
    const WtableLayout lay{0, (int64_t)g.L * g.L * g.ncw, g.ncw, g.ncw, 0};
    hipError_t e = launch_wtable(P.T->dtab, true, h, W, false, g.L, g.N, g.n_omega,
                                 g.n_theta_out, lay, s);
    if (e != hipSuccess) return e;

    const int ti = g.tpw == 4 ? 0 : (g.tpw == 8 ? 1 : (g.tpw == 12 ? 2 : 3));
#define SLSHT_PHI_ROW(T)                                                                    \
    {(const void*)energy_phi_kernel<T, 1>, (const void*)energy_phi_kernel<T, 2>,          \
     (const void*)energy_phi_kernel<T, 3>, (const void*)energy_phi_kernel<T, 4>,          \
     (const void*)energy_phi_kernel<T, 5>, (const void*)energy_phi_kernel<T, 6>,          \
     (const void*)energy_phi_kernel<T, 7>, (const void*)energy_phi_kernel<T, 8>}
    const void* fns[4][8] = {SLSHT_PHI_ROW(4), SLSHT_PHI_ROW(8), SLSHT_PHI_ROW(12),
                             SLSHT_PHI_ROW(kEnergyMaxTpw)};
#undef SLSHT_PHI_ROW
    const int ki = g.nkk - 1;
    const void* phi = fns[ti][ki];
    const size_t lds_phi = energy_lds_for(P);
    if (lds_phi > 64 * 1024)
        (void)hipFuncSetAttribute(phi, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_phi);
    const size_t lds_u = (size_t)std::max(g.L, 2 * (g.L - 1)) * g.ncw * sizeof(float2);
    const float2* twf = reinterpret_cast<const float2*>(P.T->tw_full);
    const dim3 ugrid(g.n_theta_out, (g.ntiles + kUWaves - 1) / kUWaves);
    const dim3 pgrid(g.n_l * g.n_theta_out * g.nsplit);
    for (int c = 0; c < g.nchunks; ++c) {
        hipLaunchKernelGGL(energy_afrag_kernel, dim3(g.ntiles), dim3(64), 0, s, A, af, g, c);
        hipLaunchKernelGGL(energy_u_kernel, ugrid, dim3(64 * kUWaves), lds_u, s,
                           (const float2*)W, (const float*)af, pm, g, c);
        const float* pmc = pm;
        void* args[] = {(void*)&pmc, (void*)&twf, (void*)&ep, (void*)&E, (void*)&g, (void*)&c};
        e = hipLaunchKernel(phi, pgrid, dim3(64 * kEnergyPhiWaves), args, lds_phi, s);
        if (e != hipSuccess) return e;
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace slsht
