// gfx950 kernels of the W/U FULL synthesis (window band-limits above 8), and the W table it
// shares with the ENERGY path.
//
// The separated form (eq. Eq:alternative_harmonic_formulation_wigner, separation of
// variables of Section IV-B) is summed with the q'-sum first:
//   W^p_q(theta_b, omega_c) = sum_{|q'| <= p, |q'| < N} h_p^{q'} d^p_{q,q'}(theta_b) e^{-i q' omega_c}
//   U_q(theta_b, omega_c; l, m) = sum_{p >= |q|} A^p_q(l, m) W^p_q(theta_b, omega_c)
//   P_k = U_k + U_{-k},  M_k = -i (U_k - U_{-k})
// W depends on neither l nor m, so the p-sum is a dense product over the (l, m) items for
// each (theta_b, q): a GEMM on the matrix cores (v_mfma_f64_16x16x4f64 for FP64 plans,
// v_mfma_f32_16x16x4f32 for FP32-mixed).  Kernels:
//   wtable_kernel       W of every theta row (FP64 sums; stored in the plan precision)
//   staged_afrag_kernel A^p_{+-k} of the items in MFMA A-fragment order
//   wu_phi_kernel       per block of items and a run of (theta row, omega) column tiles:
//                       U, the fold into P_k, M_k in LDS, then the phi stage and store
//                       (slsht_phi.h)
// MFMA lane layouts (gfx950): lane l supplies A[l%16][l/16] and B[l/16][l%16]; the FP32 form
// returns D rows 4(l/16)+r, the FP64 form rows (l/16)+4r, of column l%16.
#include "slsht_device.h"
#include "slsht_phi.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

namespace slsht {

namespace {

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
// cos/sin(2 pi j / n_omega) at j = q' c mod n_omega, in FP64.  Where entry (theta row t,
// row r, column c) sits, and which padding columns are written as zeros: WtableLayout.
template <typename DT, typename OV>
__global__ void __launch_bounds__(256) wtable_kernel(const double2* __restrict__ h,
                                                     const DT* __restrict__ dtab,
                                                     OV* __restrict__ W, int L, int N,
                                                     int n_omega, const WtableLayout lay) {
    __shared__ double2 hd[SLSHT_MAX_LH * (2 * SLSHT_MAX_LH - 1)];
    extern __shared__ double2 tw[];                      // [n_omega] (dynamic)
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
    const int r0 = wq_off(L, q), n_theta = gridDim.x;
    const int cw = lay.tiled ? n_omega : lay.cw;
    for (int i = threadIdx.x; i < (L - k) * cw; i += blockDim.x) {
        const int pr = i / cw, c = i - pr * cw, p = k + pr;
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
        int64_t at;
        if (lay.tiled) {
            const int64_t col = (int64_t)c * n_theta + t;
            at = ((col >> 4) * L * L + r0 + pr) * 16 + (col & 15);
        } else {
            at = (int64_t)t * lay.tstride + (int64_t)(r0 + pr) * lay.rstride + c;
        }
        W[at] = vmk<OV>((decltype(OV::x))sr, (decltype(OV::x))si);
    }
    if (lay.tiled && t == 0) {                           // the last tile's padding columns
        const int64_t c0 = (int64_t)n_omega * n_theta;
        const int pad = (int)(lay.ncol - c0);
        for (int i = threadIdx.x; i < (L - k) * pad; i += blockDim.x) {
            const int pr = i / pad;
            const int64_t col = c0 + (i - pr * pad);
            W[((col >> 4) * L * L + r0 + pr) * 16 + (col & 15)] = vmk<OV>(0, 0);
        }
    }
}

hipError_t launch_wtable(const void* dtab, bool d64, const double2* h, void* W, bool w64, int L,
                         int N, int n_omega, int n_theta_out, const WtableLayout& lay,
                         hipStream_t s) {
    if (n_omega < 1 || n_omega > kWtableMaxOmega || n_theta_out < 1) return hipErrorInvalidValue;
    const dim3 grid(n_theta_out, 2 * L - 1), block(256);
    const size_t lds = (size_t)n_omega * sizeof(double2);
    if (d64 && w64)
        hipLaunchKernelGGL((wtable_kernel<double, double2>), grid, block, lds, s, h,
                           (const double*)dtab, (double2*)W, L, N, n_omega, lay);
    else if (d64)
        hipLaunchKernelGGL((wtable_kernel<double, float2>), grid, block, lds, s, h,
                           (const double*)dtab, (float2*)W, L, N, n_omega, lay);
    else
        hipLaunchKernelGGL((wtable_kernel<float, float2>), grid, block, lds, s, h,
                           (const float*)dtab, (float2*)W, L, N, n_omega, lay);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------
// offset (in 64-lane fragment steps) of U_{+k}'s A fragments within a 16-item tile
__device__ __forceinline__ int afrag_off(int L, int k) {
    int off = 0;
    for (int j = 0; j < k; ++j) off += (j ? 2 : 1) * u_steps(L, j);
    return off;
}

// A fragments of one chunk of items: tile `tile` covers items item0 + 16 tile + i; step s of
// U_{+-k} holds, in lane (i, j4), component (j4 & 1) of A^p_{+-k} with p = k + 2s + (j4 >> 1).
// Items past the chunk are zero.  kAfragWaves waves per tile take the k in turn.
constexpr int kAfragWaves = 4;
template <typename T>
__global__ void __launch_bounds__(64 * kAfragWaves) staged_afrag_kernel(
    const double2* __restrict__ A, T* __restrict__ af, const StagedGeom g, int item0, int n_chunk) {
    const int tile = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = tile * 16 + (lane & 15), j4 = lane >> 4;
    const int L = g.L;
    const bool valid = row < n_chunk;
    int64_t lm = 0;
    if (valid) lm = item_decode(item0 + row, g.l_lo, g.real_pair).lm;
    T* out = af + (int64_t)tile * g.afrag_tile + lane;
    for (int k = wave; k < L; k += kAfragWaves) {
        const int steps = u_steps(L, k);
        int off = afrag_off(L, k);
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
// The W/U kernel: one block = `IT` items x a run of tiles of 16 columns, a column being an
// (omega, theta row) pair: col = c n_theta_out + t over all n_omega * n_theta_out of them, the
// order of the output rows (A depends on neither, so a tile may span omega values, and only
// the last tile is padded).  Per column tile:
//   1. U_{+-k}(theta_t, omega_c) for the block's items and columns, as complex GEMMs on real
//      MFMAs (the complex inner index p expanded to (Re, Im), B = [[W_re, W_im],
//      [-W_im, W_re]] row pairs); the waves split the k, and each folds its U_{+-k} into
//      P_k = U_k + U_{-k}, M_k = -i (U_k - U_{-k}) and writes them to the block's P|M rows
//      in LDS (row = item * 16 + column: P_0..P_{L-1} at 0, M_0..M_{L-1} at L);
//   2. the phi stage over those rows on the matrix cores (phi_stage_mfma), stored to g.
// IT = 16 where the block's P|M rows fit in LDS (FP64 up to L_h = 19); else IT = 8: the A
// operand's rows 8..15 are zero and the D rows past 8 are dropped.  A block runs 12 waves
// (one block per CU): the register cap of 168 VGPRs this sets costs the band-limit bucket 32
// a few spilled registers, and still runs faster than 8 waves with none.
// Blocks are laid out so that those sharing an item tile (the same A fragments) run on one
// XCD: block b goes to XCD b mod 8 under round-robin dispatch.
struct WUArgs {
    int L, n_omega, n_cols, ncol, n_theta_out, n_phi, nslot, l_lo, real_pair, n_items;
    int afrag_tile, n_itiles, n_ctiles, cchunk, n_cchunks;
    uint32_t kmask[kWuMaxWaves];  // k of U_{+-k} taken by each wave (bit k)
};

static_assert(kWuThreads % 64 == 0 && kWuThreads / 64 <= kWuMaxWaves,
              "W/U block: whole waves, kmask sized");

// Splits the k of U_{+-k} over `nw` waves: costliest first (MFMA steps, four GEMMs, two
// for k = 0), each to the wave with the least work so far.
static void wu_kmasks(int L, int nw, uint32_t* mask) {
    auto cost = [&](int k) { return u_steps(L, k) * (k ? 4 : 2); };
    int load[kWuMaxWaves] = {0};
    bool used[SLSHT_MAX_LH] = {false};
    for (int w = 0; w < kWuMaxWaves; ++w) mask[w] = 0;
    for (int n = 0; n < L; ++n) {
        int k = -1;
        for (int c = 0; c < L; ++c)
            if (!used[c] && (k < 0 || cost(c) > cost(k))) k = c;
        used[k] = true;
        int best = 0;
        for (int w = 1; w < nw; ++w)
            if (load[w] < load[best]) best = w;
        load[best] += cost(k);
        mask[best] |= 1u << k;
    }
}

template <typename T, int LH, int IT, int NT>
__global__ void __launch_bounds__(NT) wu_phi_kernel(
    const typename VecOf<T>::type* __restrict__ W, const T* __restrict__ af,
    const typename VecOf<T>::type* __restrict__ twphi, typename VecOf<T>::type* __restrict__ g,
    const WUArgs a) {
    using V = typename VecOf<T>::type;
    using MF = StagedMfma<T>;
    using Acc = typename MF::acc;
    constexpr int SB = 4;                            // MFMA steps per load group of the U GEMM
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* PM_s = reinterpret_cast<V*>(smem_raw);        // [IT * 16 rows][2L + 1]
    __shared__ int64_t s_lm[IT], s_mir[IT];
    __shared__ int64_t s_roff[16];                   // output row offset of each column of the tile
    __shared__ T s_sign[IT];

    const int b = blockIdx.x;
    const int xcd = b & 7, j = b >> 3;
    const int grp = j / a.n_cchunks;
    const int itile = xcd * (a.n_itiles >> 3) + grp;
    const int cch = j - grp * a.n_cchunks;
    const int item0 = itile * IT;
    if (item0 >= a.n_items) return;                  // whole block: uniform
    const int L = a.L, pms = 2 * L + 1;
    const int ct_begin = cch * a.cchunk, ct_end = min(a.n_ctiles, ct_begin + a.cchunk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const int i16 = lane & 15, j4 = lane >> 4;

    const int64_t lm_stride = (int64_t)a.n_omega * a.n_theta_out * a.n_phi;
    if (tid < IT) {
        const int item = item0 + tid;
        if (item < a.n_items) {
            const Item it = item_decode(item, a.l_lo, a.real_pair);
            s_lm[tid] = (int64_t)it.lm * lm_stride;
            s_mir[tid] = it.mirror >= 0 ? (int64_t)it.mirror * lm_stride : -1;
            s_sign[tid] = (it.m & 1) ? T(-1) : T(1);
        } else {
            s_lm[tid] = -1;
            s_mir[tid] = -1;
            s_sign[tid] = T(1);
        }
    }
    // this lane's A-operand row: item (item0 % 16) + i16 of its 16-item fragment tile
    const bool arow = i16 < IT && item0 + i16 < a.n_items;
    const T* aft = af + (int64_t)(item0 / 16) * a.afrag_tile + j4 * 16 + (item0 % 16) + i16;
    __syncthreads();

    const uint32_t kmask = a.kmask[wave];                  // this wave's k of U_{+-k}

    // column tiles: 16 consecutive columns col = c * n_theta_out + t, which is also the
    // output row (omega_c, theta_t) of every item
    for (int ct = ct_begin; ct < ct_end; ++ct) {
        if (tid < 16) {
            const int col = ct * 16 + tid;
            s_roff[tid] = col < a.n_cols ? (int64_t)col * a.n_phi : -1;
        }
        const V* Wt = W + (int64_t)ct * L * L * 16 + i16;     // the tile's rows, 16 columns each
        for (uint32_t km = kmask; km; km &= km - 1) {
            const int k = __builtin_ctz(km);
            const int steps = u_steps(L, k);
            const int off = afrag_off(L, k);
            const int lastp = L - k - 1;
            const V* wpk = Wt + wq_off(L, k) * 16;
            const V* wmk = wpk + (L - k) * 16;
            Acc upr = {0, 0, 0, 0}, upi = {0, 0, 0, 0}, umr = {0, 0, 0, 0}, umi = {0, 0, 0, 0};
            // the p-sum in groups of SB MFMA steps: loads of a group first, then its MFMAs
            for (int s0 = 0; s0 < steps; s0 += SB) {
                T ap[SB], am[SB];
                V wp[SB], wm[SB];
#pragma unroll
                for (int u = 0; u < SB; ++u) {
                    const int s = s0 + u;
                    // rows past the last degree meet a zero A fragment; clamp them in range
                    const int rp = min(2 * s + (j4 >> 1), lastp);
                    const bool in = s < steps;
                    ap[u] = (in && arow) ? aft[(int64_t)(off + s) * 64] : T(0);
                    am[u] = (in && arow && k) ? aft[(int64_t)(off + steps + s) * 64] : T(0);
                    wp[u] = in ? wpk[rp * 16] : vmk<V>(0, 0);
                    wm[u] = (in && k) ? wmk[rp * 16] : vmk<V>(0, 0);
                }
#pragma unroll
                for (int u = 0; u < SB; ++u) {
                    if (s0 + u >= steps) break;          // the last group's padding (uniform)
                    upr = MF::step(ap[u], (j4 & 1) ? -wp[u].y : wp[u].x, upr);
                    upi = MF::step(ap[u], (j4 & 1) ? wp[u].x : wp[u].y, upi);
                    if (k) {
                        umr = MF::step(am[u], (j4 & 1) ? -wm[u].y : wm[u].x, umr);
                        umi = MF::step(am[u], (j4 & 1) ? wm[u].x : wm[u].y, umi);
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int item = MF::drow(j4, r);
                if (item >= IT) continue;
                V* row = PM_s + (item * 16 + i16) * pms;
                row[k] = vmk<V>(upr[r] + umr[r], upi[r] + umi[r]);
                row[L + k] = k ? vmk<V>(upi[r] - umi[r], umr[r] - upr[r]) : vmk<V>(0, 0);  // M_0 = 0
            }
        }
        __syncthreads();
        phi_stage_mfma<T, LH>(PM_s, pms, L, IT * 16, L, twphi, a.nslot, a.n_phi,
                              [&](int rr, V*& out, V*& mout, T& ms) {
                                  const int item = rr >> 4;
                                  const int64_t base = s_lm[item];
                                  const int64_t rowoff = s_roff[rr & 15];
                                  if (base < 0 || rowoff < 0) {
                                      out = nullptr;
                                      mout = nullptr;
                                      ms = T(1);
                                      return;
                                  }
                                  out = g + base + rowoff;
                                  const int64_t mb = s_mir[item];
                                  mout = mb >= 0 ? g + mb + rowoff : nullptr;
                                  ms = s_sign[item];
                              });
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------
// Host: launches.

template <typename T, int LH, int IT, int NT>
static hipError_t launch_wu(const StagedGeom& sg, const DevPlan& P, const void* W, const void* af,
                            void* g, hipStream_t s) {
    if (sg.threads != NT) return hipErrorInvalidConfiguration;
    using V = typename VecOf<T>::type;
    WUArgs a;
    a.L = sg.L;
    a.n_omega = sg.n_omega;
    a.n_cols = sg.n_cols;
    a.ncol = sg.ncol;
    a.n_theta_out = sg.n_theta_out;
    a.n_phi = P.d.n_phi;
    a.nslot = P.nslot_phi;
    a.l_lo = sg.l_lo;
    a.real_pair = sg.real_pair;
    a.n_items = sg.n_items;
    a.afrag_tile = sg.afrag_tile;
    a.n_itiles = sg.n_itiles;
    a.n_ctiles = sg.n_ctiles;
    a.cchunk = sg.cchunk;
    a.n_cchunks = sg.n_cchunks;
    wu_kmasks(sg.L, NT / 64, a.kmask);
    const int64_t nblk = (int64_t)sg.n_itiles * sg.n_cchunks;
    if (nblk > 0x7fffffff) return hipErrorInvalidConfiguration;
    const void* fn = (const void*)wu_phi_kernel<T, LH, IT, NT>;
    if (sg.lds > 64 * 1024)
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sg.lds);
    const V* Wv = static_cast<const V*>(W);
    const T* afv = static_cast<const T*>(af);
    const V* tw = static_cast<const V*>(P.T->tw_phi);
    V* gv = static_cast<V*>(g);
    void* args[] = {(void*)&Wv, (void*)&afv, (void*)&tw, (void*)&gv, (void*)&a};
    return hipLaunchKernel(fn, dim3((unsigned)nblk), dim3(NT), args, sg.lds, s);
}

hipError_t launch_synthesis_staged(const DevPlan& P, const double2* A, const double2* h, void* g,
                                   hipStream_t s) {
    const StagedGeom& sg = P.sg;
    char* ws = static_cast<char*>(P.ework);
    if (!ws) return hipErrorInvalidValue;
    void* W = ws + sg.off_w;
    void* af = ws + sg.off_af;
    // W by tiles of 16 (omega, theta row) columns
    const WtableLayout lay{1, 0, 0, 0, sg.ncol};
    hipError_t e = launch_wtable(P.T->dtab, sg.f64 != 0, h, W, sg.f64 != 0, sg.L, sg.N,
                                 sg.n_omega, sg.n_theta_out, lay, s);
    if (e != hipSuccess) return e;
    const dim3 ablk(64 * kAfragWaves);
    if (sg.f64)
        hipLaunchKernelGGL(staged_afrag_kernel<double>, dim3(sg.ntiles), ablk, 0, s, A,
                           (double*)af, sg, 0, sg.n_items);
    else
        hipLaunchKernelGGL(staged_afrag_kernel<float>, dim3(sg.ntiles), ablk, 0, s, A,
                           (float*)af, sg, 0, sg.n_items);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // window band-limits 17..32 (staged_geom): buckets 24 and 32, blocks of kWuThreads
    const bool b24 = sg.L <= 24;
    if (sg.f64) {
        if (sg.it == 16) return launch_wu<double, 24, 16, kWuThreads>(sg, P, W, af, g, s);   // L_h <= 19
        return b24 ? launch_wu<double, 24, 8, kWuThreads>(sg, P, W, af, g, s)
                   : launch_wu<double, 32, 8, kWuThreads>(sg, P, W, af, g, s);
    }
    return b24 ? launch_wu<float, 24, 16, kWuThreads>(sg, P, W, af, g, s)
               : launch_wu<float, 32, 16, kWuThreads>(sg, P, W, af, g, s);
}

}  // namespace slsht
