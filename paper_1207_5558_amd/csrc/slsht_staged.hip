// gfx950 kernels of the staged FULL synthesis (window band-limits above 16, n_omega <= 64),
// and the W table it shares with the ENERGY path.
//
// The separated form (eq. Eq:alternative_harmonic_formulation_wigner, separation of
// variables of Section IV-B) is summed with the q'-sum first:
//   W^p_q(theta_b, omega_c) = sum_{|q'| <= p, |q'| < N} h_p^{q'} d^p_{q,q'}(theta_b) e^{-i q' omega_c}
//   U_q(theta_b, omega_c; l, m) = sum_{p >= |q|} A^p_q(l, m) W^p_q(theta_b, omega_c)
//   P_k = U_k + U_{-k},  M_k = -i (U_k - U_{-k})
// W depends on neither l nor m, so the p-sum is a dense product over the (l, m) items for
// each (theta_b, q): a GEMM on the matrix cores (v_mfma_f64_16x16x4f64 for FP64 plans,
// v_mfma_f32_16x16x4f32 for FP32-mixed).  Kernels:
//   wtable_kernel      W of every theta row (FP64 sums; stored in the plan precision)
//   staged_afrag_kernel A^p_{+-k} of a chunk of items in MFMA A-fragment order
//   staged_u_kernel    U, the fold into P_k, M_k, stored per (item, theta row) as rows
//                      [P_0 .. P_{PW-1}, M_0 .. M_{PW-1}] x omega
// and the phi synthesis + store of the FULL kernel reads those rows (synth_pm_kernel in
// slsht_synth.hip) in place of its own theta and omega stages.
// MFMA lane layouts (gfx950): lane l supplies A[l%16][l/16] and B[l/16][l%16]; the FP32 form
// returns D rows 4(l/16)+r, the FP64 form rows (l/16)+4r, of column l%16.
#include "slsht_device.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

namespace slsht {

namespace {

constexpr int kStagedWaves = 8;        // u kernel: one 16-item tile per wave
constexpr int kStagedCols = 64;        // u kernel: omega columns per block (4 tiles of 16)

// MFMA step and D-row map per precision.
template <typename T> struct StagedMfma;
template <> struct StagedMfma<float> {
    using acc = f4v;
    static __device__ __forceinline__ acc step(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int j4, int r) { return 4 * j4 + r; }
};
template <> struct StagedMfma<double> {
    using acc = d4v;
    static __device__ __forceinline__ acc step(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int j4, int r) { return j4 + 4 * r; }
};

__host__ __device__ inline int u_steps(int L, int k) { return (L - k + 1) / 2; }

}  // namespace

// ------------------------------------------------------------------------------
// W^p_q(theta_b, omega_c), one block per (theta row, q), q ordered 0, +1, -1, +2, -2, ...
// (row offset wq_off).  h_p^{q'} d^p_{q,q'}(theta_b) is staged in LDS (canonical table entries
// through the symmetries of Section IV-B); each thread sums one (p, c) over q' against
// cos/sin(2 pi j / n_omega) at j = q' c mod n_omega, in FP64.  Columns c >= n_omega (padding
// to ncw) are written as zeros.
template <typename DT, typename OV>
__global__ void __launch_bounds__(256) wtable_kernel(const double2* __restrict__ h,
                                                     const DT* __restrict__ dtab,
                                                     OV* __restrict__ W, int L, int N,
                                                     int n_omega, int ncw) {
    __shared__ double2 hd[SLSHT_MAX_LH * (2 * SLSHT_MAX_LH - 1)];
    __shared__ double2 tw[kEnergyMaxOmega];
    const int K = 2 * L - 1;
    const int t = blockIdx.x, qi = blockIdx.y;
    const int k = (qi + 1) / 2;
    const int q = (qi & 1) ? k : -k;
    const DT* drow = dtab + (int64_t)t * dtab_row_len(L);
    for (int i = threadIdx.x; i < L * K; i += blockDim.x) {
        const int p = i / K, qp = i - p * K - (L - 1);
        const int aqp = qp < 0 ? -qp : qp;
        double2 v = vmk<double2>(0.0, 0.0);
        if (p >= k && aqp <= p && aqp < N) {
            int Q, Qp;
            bool neg;
            d_canonical(q, qp, Q, Qp, neg);
            const double e = (double)drow[dtab_off(p) + Q * Q + Q + Qp];
            const double dv = neg ? -e : e;
            const double2 hv = h[p * p + p + qp];
            v = vmk<double2>(hv.x * dv, hv.y * dv);
        }
        hd[i] = v;
    }
    for (int j = threadIdx.x; j < n_omega; j += blockDim.x) {
        double s, c;
        sincospi(2.0 * (double)j / (double)n_omega, &s, &c);
        tw[j] = vmk<double2>(c, s);
    }
    __syncthreads();
    OV* out = W + ((int64_t)t * L * L + wq_off(L, q)) * ncw;
    for (int i = threadIdx.x; i < (L - k) * ncw; i += blockDim.x) {
        const int pr = i / ncw, c = i - pr * ncw, p = k + pr;
        double sr = 0.0, si = 0.0;
        if (c < n_omega) {
            const int P = min(p, N - 1);
            int idx = (int)(((int64_t)(n_omega - c) * P) % n_omega);     // (-P c) mod n
            const double2* row = hd + p * K + (L - 1);
            for (int qp = -P; qp <= P; ++qp) {
                const double2 hv = row[qp];
                const double2 e = tw[idx];                                 // e^{-i q' w} = c - i s
                sr += hv.x * e.x + hv.y * e.y;
                si += hv.y * e.x - hv.x * e.y;
                idx += c;
                if (idx >= n_omega) idx -= n_omega;
            }
        }
        out[i] = vmk<OV>((decltype(OV::x))sr, (decltype(OV::x))si);
    }
}

hipError_t launch_wtable(const void* dtab, bool d64, const double2* h, void* W, bool w64, int L,
                         int N, int n_omega, int ncw, int n_theta_out, hipStream_t s) {
    const dim3 grid(n_theta_out, 2 * L - 1), block(256);
    if (d64 && w64)
        hipLaunchKernelGGL((wtable_kernel<double, double2>), grid, block, 0, s, h,
                           (const double*)dtab, (double2*)W, L, N, n_omega, ncw);
    else if (d64)
        hipLaunchKernelGGL((wtable_kernel<double, float2>), grid, block, 0, s, h,
                           (const double*)dtab, (float2*)W, L, N, n_omega, ncw);
    else
        hipLaunchKernelGGL((wtable_kernel<float, float2>), grid, block, 0, s, h,
                           (const float*)dtab, (float2*)W, L, N, n_omega, ncw);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------
// A fragments of one chunk of items: tile `tile` covers items item0 + 16 tile + i; step s of
// U_{+-k} holds, in lane (i, j4), component (j4 & 1) of A^p_{+-k} with p = k + 2s + (j4 >> 1).
// Items past the chunk are zero.
template <typename T>
__global__ void __launch_bounds__(64) staged_afrag_kernel(const double2* __restrict__ A,
                                                          T* __restrict__ af, const StagedGeom g,
                                                          int item0, int n_chunk) {
    const int tile = blockIdx.x, lane = threadIdx.x;
    const int row = tile * 16 + (lane & 15), j4 = lane >> 4;
    const int L = g.L;
    const bool valid = row < n_chunk;
    int64_t lm = 0;
    if (valid) lm = item_decode(item0 + row, g.l_lo, g.real_pair).lm;
    T* out = af + (int64_t)tile * g.afrag_tile + lane;
    int off = 0;
    for (int k = 0; k < L; ++k) {
        const int steps = u_steps(L, k);
        for (int sg = 0; sg < (k ? 2 : 1); ++sg) {
            const int q = sg ? -k : k;
            for (int s = 0; s < steps; ++s) {
                const int p = k + 2 * s + (j4 >> 1);
                T v = 0;
                if (valid && p < L) {
                    const double2 a = A[lm * L * L + p * p + p + q];
                    v = (T)((j4 & 1) ? a.y : a.x);
                }
                out[(int64_t)(off + s) * 64] = v;
            }
            off += steps;
        }
    }
}

// ------------------------------------------------------------------------------
// U_{+-k}(theta_b, omega_c) for 16 items per wave and 64 omega columns per block, as complex
// GEMMs on real MFMAs (complex inner index p expanded to (Re, Im), B = [[W_re, W_im],
// [-W_im, W_re]] row pairs), folded in registers and stored to the P/M rows of the chunk:
//   pm[((item - item0) n_theta_out + theta) 2PW ncw + kslot ncw + c],  kslot = k (P_k) or
//   PW + k (M_k); rows k = L .. PW-1 are zero.
// W_{+-k} of the block's theta row and column range is staged in LDS; the next k's W rows
// and A fragments are loaded into registers while this k's MFMAs run.
template <typename T>
__global__ void __launch_bounds__(64 * kStagedWaves) staged_u_kernel(
    const typename VecOf<T>::type* __restrict__ W, const T* __restrict__ af,
    typename VecOf<T>::type* __restrict__ pm, const StagedGeom g, int n_chunk) {
    using V = typename VecOf<T>::type;
    using MF = StagedMfma<T>;
    using Acc = typename MF::acc;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* Ws = reinterpret_cast<V*>(smem_raw);               // [<= max(L, 2L-2) rows][64]
    const int L = g.L, ncw = g.ncw;
    const int t = blockIdx.x, c0 = blockIdx.z * kStagedCols;
    const int ncols = min(kStagedCols, ncw - c0);          // a multiple of 16
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = blockIdx.y * kStagedWaves + wave;
    const int ntiles = (n_chunk + 15) / 16;
    const bool active = tile < ntiles;
    const int j4 = lane >> 4, col = lane & 15;
    const V* Wt = W + (int64_t)t * L * L * ncw + c0;
    const T* aft = af + (int64_t)(active ? tile : 0) * g.afrag_tile + lane;
    const int64_t rowlen = (int64_t)2 * g.PW * ncw;        // V elements per (item, theta)

    int64_t base[4];
    bool rv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = tile * 16 + MF::drow(j4, r);
        rv[r] = active && row < n_chunk;
        base[r] = ((int64_t)row * g.n_theta_out + t) * rowlen + c0 + col;
    }

    // W rows of the next k in registers (at most (2L-2) x 64 elements over the block)
    constexpr int kWPer = ((2 * SLSHT_MAX_LH - 2) * kStagedCols + 64 * kStagedWaves - 1) /
                          (64 * kStagedWaves);
    V wr[kWPer];
    auto load_w = [&](int k) {
        const int n = (k ? 2 * (L - k) : L) * ncols;
        const V* src = Wt + (int64_t)wq_off(L, k) * ncw;
#pragma unroll
        for (int i = 0; i < kWPer; ++i) {
            const int idx = threadIdx.x + i * 64 * kStagedWaves;
            const int r = idx / ncols, c = idx - r * ncols;
            wr[i] = idx < n ? src[(int64_t)r * ncw + c] : vmk<V>(0, 0);
        }
    };
    // FP64: the A fragments are loaded at their own k (register budget)
    constexpr bool kPrefetchA = sizeof(T) == 4;
    T apn[16], amn[16];
    auto load_a = [&](int k, int off) {
        const int steps = u_steps(L, k);
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            apn[s] = (active && s < steps) ? aft[(int64_t)(off + s) * 64] : T(0);
            amn[s] = (active && k && s < steps) ? aft[(int64_t)(off + steps + s) * 64] : T(0);
        }
    };
    load_w(0);
    if (kPrefetchA) load_a(0, 0);
    int aoff = 0;
    for (int k = 0; k < L; ++k) {
        const int steps = u_steps(L, k);
        __syncthreads();
        {
            const int n = (k ? 2 * (L - k) : L) * ncols;
#pragma unroll
            for (int i = 0; i < kWPer; ++i) {
                const int idx = threadIdx.x + i * 64 * kStagedWaves;
                const int r = idx / ncols, c = idx - r * ncols;
                if (idx < n) Ws[r * kStagedCols + c] = wr[i];
            }
        }
        __syncthreads();
        if (!kPrefetchA) load_a(k, aoff);
        T ap[16], am[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            ap[s] = apn[s];
            am[s] = amn[s];
        }
        const int aoff_next = aoff + (k ? 2 : 1) * steps;
        if (k + 1 < L) {
            load_w(k + 1);
            if (kPrefetchA) load_a(k + 1, aoff_next);
        }
        if (active) {
            const int lastp = L - k - 1;
            for (int ct = 0; ct < ncols / 16; ++ct) {
                Acc upr = {0, 0, 0, 0}, upi = {0, 0, 0, 0}, umr = {0, 0, 0, 0}, umi = {0, 0, 0, 0};
                const V* wcol = Ws + ct * 16 + col;
#pragma unroll
                for (int s = 0; s < 16; ++s) {
                    if (s >= steps) break;
                    // rows past the last degree meet a zero A fragment; clamp them in range
                    const int rp = min(2 * s + (j4 >> 1), lastp);
                    const V wp = wcol[rp * kStagedCols];
                    upr = MF::step(ap[s], (j4 & 1) ? -wp.y : wp.x, upr);
                    upi = MF::step(ap[s], (j4 & 1) ? wp.x : wp.y, upi);
                    if (k) {
                        const V wm = wcol[(L - k + rp) * kStagedCols];
                        umr = MF::step(am[s], (j4 & 1) ? -wm.y : wm.x, umr);
                        umi = MF::step(am[s], (j4 & 1) ? wm.x : wm.y, umi);
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (!rv[r]) continue;
                    V* o = pm + base[r] + ct * 16;
                    o[(int64_t)k * ncw] = vmk<V>(upr[r] + umr[r], upi[r] + umi[r]);
                    o[(int64_t)(g.PW + k) * ncw] =
                        k ? vmk<V>(upi[r] - umi[r], umr[r] - upr[r]) : vmk<V>(0, 0);   // M_0 = 0
                }
            }
        }
        aoff = aoff_next;
    }
    // rows k = L .. PW-1 of P and M are zero (the phi stage runs whole k-steps)
    for (int k = L; k < g.PW; ++k)
        for (int ct = 0; ct < ncols / 16; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (rv[r]) {
                    V* o = pm + base[r] + ct * 16;
                    o[(int64_t)k * ncw] = vmk<V>(0, 0);
                    o[(int64_t)(g.PW + k) * ncw] = vmk<V>(0, 0);
                }
}

// ------------------------------------------------------------------------------
// Host: geometry and launches.

hipError_t launch_synthesis_staged(const DevPlan& P, const double2* A, const double2* h, void* g,
                                   hipStream_t s) {
    const StagedGeom& sg = P.sg;
    char* ws = static_cast<char*>(P.ework);
    if (!ws) return hipErrorInvalidValue;
    void* W = ws + sg.off_w;
    void* af = ws + sg.off_af;
    void* pm = ws + sg.off_pm;
    hipError_t e = launch_wtable(P.T->dtab, sg.f64 != 0, h, W, sg.f64 != 0, sg.L, sg.N,
                                 sg.n_omega, sg.ncw, sg.n_theta_out, s);
    if (e != hipSuccess) return e;
    const size_t lds_u = (size_t)std::max(sg.L, 2 * (sg.L - 1)) * kStagedCols *
                         (sg.f64 ? sizeof(double2) : sizeof(float2));
    for (int c = 0; c < sg.nchunks; ++c) {
        const int item0 = c * sg.ichunk;
        const int n = std::min(sg.ichunk, sg.n_items - item0);
        const int ntiles = (n + 15) / 16;
        const dim3 ugrid(sg.n_theta_out, (ntiles + kStagedWaves - 1) / kStagedWaves,
                         (sg.ncw + kStagedCols - 1) / kStagedCols);
        if (sg.f64) {
            hipLaunchKernelGGL(staged_afrag_kernel<double>, dim3(ntiles), dim3(64), 0, s, A,
                               (double*)af, sg, item0, n);
            hipLaunchKernelGGL(staged_u_kernel<double>, ugrid, dim3(64 * kStagedWaves), lds_u, s,
                               (const double2*)W, (const double*)af, (double2*)pm, sg, n);
        } else {
            hipLaunchKernelGGL(staged_afrag_kernel<float>, dim3(ntiles), dim3(64), 0, s, A,
                               (float*)af, sg, item0, n);
            hipLaunchKernelGGL(staged_u_kernel<float>, ugrid, dim3(64 * kStagedWaves), lds_u, s,
                               (const float2*)W, (const float*)af, (float2*)pm, sg, n);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = launch_synthesis_pm(P, pm, item0, n, g, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace slsht
