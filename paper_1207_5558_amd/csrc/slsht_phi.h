// The phi stage of the FULL synthesis on the matrix cores, shared by the fused kernel of
// slsht_synth.hip (theta and omega stages in the block) and the W/U kernel of
// slsht_staged.hip (U GEMM in the block):
//   g(phi_a) = P_0 + sum_{k>0} P_k cos(k phi_a) + M_k sin(k phi_a),
//   g(phi_{n-a}) = the same with the sine part negated,
// as a pair of real GEMMs, one row per (complex output row, Re|Im) and one column per slot:
//   C = Pmat (rows x k) * cos(k phi_a) (k x a),   S = Mmat * sin(k phi_a),
// with P_0 carried by cos(0) = 1 (M_0 = 0).  16x16x4 MFMA (FP32 or FP64): lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; the FP32 form returns D rows 4(l/16)+r, the FP64 form
// rows (l/16)+4r, of column l%16.  A-operand rows are permuted per precision so that every
// lane receives Re and Im of two complex rows.
#pragma once

#include "slsht_device.h"

#include <hip/hip_runtime.h>

namespace slsht {

template <typename T> struct MfmaOf;
template <> struct MfmaOf<float> {
    using acc = f4v;
    static __device__ __forceinline__ acc step(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // A-operand row i -> complex row (of the 8 in a tile) and part; D rows 4j+r hold
    // Re, Im of complex rows 2j and 2j+1
    static __device__ __forceinline__ int row_of(int i) { return i >> 1; }
    static __device__ __forceinline__ int part_of(int i) { return i & 1; }
    static __device__ __forceinline__ int first_row(int j) { return 2 * j; }
    static __device__ __forceinline__ int second_row(int j) { return 2 * j + 1; }
};
template <> struct MfmaOf<double> {
    using acc = d4v;
    static __device__ __forceinline__ acc step(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // D rows j+4r: r = 0, 1 are Re, Im of complex row j, r = 2, 3 of row j + 4
    static __device__ __forceinline__ int row_of(int i) { return (i & 3) + 4 * (i >> 3); }
    static __device__ __forceinline__ int part_of(int i) { return (i >> 2) & 1; }
    static __device__ __forceinline__ int first_row(int j) { return j; }
    static __device__ __forceinline__ int second_row(int j) { return j + 4; }
};

// 4x4 transpose between lane groups (16 lanes each) and four registers: on entry
// lane group j of register x holds M[j][x]; on exit lane group x of register j does.
// v_permlane32_swap exchanges the upper half-wave of its first operand with the lower
// half-wave of its second; v_permlane16_swap exchanges the odd 16-lane rows of its
// first operand with the even rows of its second.
__device__ __forceinline__ void transpose4_u32(unsigned& r0, unsigned& r1, unsigned& r2,
                                               unsigned& r3) {
    auto p = __builtin_amdgcn_permlane32_swap(r0, r2, false, false);
    r0 = p[0]; r2 = p[1];
    p = __builtin_amdgcn_permlane32_swap(r1, r3, false, false);
    r1 = p[0]; r3 = p[1];
    p = __builtin_amdgcn_permlane16_swap(r0, r1, false, false);
    r0 = p[0]; r1 = p[1];
    p = __builtin_amdgcn_permlane16_swap(r2, r3, false, false);
    r2 = p[0]; r3 = p[1];
}

__device__ __forceinline__ void transpose4(float& a, float& b, float& c, float& d) {
    unsigned x0 = __float_as_uint(a), x1 = __float_as_uint(b), x2 = __float_as_uint(c),
             x3 = __float_as_uint(d);
    transpose4_u32(x0, x1, x2, x3);
    a = __uint_as_float(x0); b = __uint_as_float(x1); c = __uint_as_float(x2); d = __uint_as_float(x3);
}

__device__ __forceinline__ void transpose4(double& a, double& b, double& c, double& d) {
    unsigned long long x0 = __double_as_longlong(a), x1 = __double_as_longlong(b),
                       x2 = __double_as_longlong(c), x3 = __double_as_longlong(d);
    unsigned l0 = (unsigned)x0, l1 = (unsigned)x1, l2 = (unsigned)x2, l3 = (unsigned)x3;
    unsigned h0 = (unsigned)(x0 >> 32), h1 = (unsigned)(x1 >> 32), h2 = (unsigned)(x2 >> 32),
             h3 = (unsigned)(x3 >> 32);
    transpose4_u32(l0, l1, l2, l3);
    transpose4_u32(h0, h1, h2, h3);
    a = __longlong_as_double((long long)(((unsigned long long)h0 << 32) | l0));
    b = __longlong_as_double((long long)(((unsigned long long)h1 << 32) | l1));
    c = __longlong_as_double((long long)(((unsigned long long)h2 << 32) | l2));
    d = __longlong_as_double((long long)(((unsigned long long)h3 << 32) | l3));
}

// B fragments of one 16-slot tile of the phi GEMMs: lane (li, lj) supplies row
// k = 4 kk + lj, column s of cos(k phi_s) and sin(k phi_s); zero past L or nslot.
template <typename T, int KQ>
__device__ __forceinline__ void load_phi_b(const typename VecOf<T>::type* __restrict__ twp,
                                           int nslot, int L, int kq, int s, int lj, T* bc, T* bs) {
#pragma unroll
    for (int kk = 0; kk < KQ; ++kk) {
        const int k = 4 * kk + lj;
        T cv = 0, sv = 0;
        if (kk < kq && s < nslot) {
            if (k == 0) {
                cv = 1;
            } else if (k < L) {
                const auto tw = twp[(k - 1) * nslot + s];
                cv = tw.x;
                sv = tw.y;
            }
        }
        bc[kk] = cv;
        bs[kk] = sv;
    }
}

// Phi stage over `nrows` complex P|M rows held in LDS (row r at PM + r * pms: P_0..P_{L-1}
// at 0.., M_0..M_{L-1} at moff..).  Work unit = (8 complex rows, 64 slots): four 16-slot
// GEMM tiles share the unit's A fragments (tiles wholly past nslot are skipped); their
// results are transposed across lane groups so that lane l holds slot 64 unit + l of each
// row and every store instruction writes consecutive outputs of one row.  Rows of at most
// 32 slots (short rows: n_phi <= 63) take two 8-row groups per unit instead, tiles 0-1 for
// the first and 2-3 for the second, so that after the transpose lanes 0-31 hold slots 0-31
// of the first group and lanes 32-63 those of the second, and one store instruction writes
// two rows.  The waves of the block split the units, slot-range-major, so that a wave's B
// fragments (cos/sin(k phi_s)) stay in registers while it walks the rows of one slot range.
//   row_out(r, out, mirror, msign): destination of row r (out = nullptr skips it) and, with
//   conjugate symmetry, the row of order -m (g(l,-m) = (-1)^m conj(g(l,m))) or nullptr.
template <typename T, int LH, typename RowOut>
__device__ __forceinline__ void phi_stage_mfma(const typename VecOf<T>::type* PM, int pms,
                                               int moff, int nrows, int L,
                                               const typename VecOf<T>::type* __restrict__ twp,
                                               int nslot, int n_phi, RowOut row_out) {
    using V = typename VecOf<T>::type;
    using MF = MfmaOf<T>;
    using Acc = typename MF::acc;
    constexpr int KQ = LH / 4;                   // MFMA k-steps of the phi GEMM
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
    const int li = lane & 15, lj = lane >> 4;
    const int n_rt = (nrows + 7) / 8;
    const bool pair = nslot <= 32;               // two 8-row groups per unit
    const int n_st = (nslot + 63) / 64;
    const int kq = (L + 3) / 4;
    const int arow = MF::row_of(li), apart = MF::part_of(li);
    // FP64 with L_h > 16 reloads the B fragments per unit instead (register budget)
    constexpr bool kKeepB = !(sizeof(T) == 8 && LH > 16);
    constexpr int NB = kKeepB ? 4 : 1;
    T bcr[NB][KQ], bsr[NB][KQ];
    int cur_st = -1;
    const int nu = pair ? (n_rt + 1) / 2 : n_rt * n_st;
    const int u_end = ((wave + 1) * nu) / nwaves;
    for (int u = (wave * nu) / nwaves; u < u_end; ++u) {
        const int st = pair ? 0 : u / n_rt;
        const int rt = pair ? 2 * u : u - st * n_rt;          // the (first) 8-row group
        // tiles holding slots: of the 64-slot range, or of each 32-slot half in pair mode
        const int ntile = pair ? (nslot + 15) / 16 : min(4, (nslot - st * 64 + 15) / 16);
        if (kKeepB && st != cur_st) {
            cur_st = st;
#pragma unroll
            for (int x = 0; x < NB; ++x) load_phi_b<T, KQ>(twp, nslot, L, kq, st * 64 + x * 16 + li, lj,
                                                         bcr[x], bsr[x]);
        }
        T pa[KQ], ma[KQ];
        // w[x][e]: x = 16-slot tile of the unit, e = (row h, value): Re/Im of C+S, C-S
        T w[4][8];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            // pair mode: tiles 2-3 repeat the slots of tiles 0-1 for the second row group
            const int tx = pair ? (x & 1) : x;
            const int rg = pair ? rt + (x >> 1) : rt;
            if (x == 0 || (pair && x == 2)) {
                const int ra = rg * 8 + arow;
                const T* prow = reinterpret_cast<const T*>(PM + (ra < nrows ? ra : 0) * pms) + apart;
#pragma unroll
                for (int kk = 0; kk < KQ; ++kk) {
                    const int k = 4 * kk + lj;
                    const bool ok = kk < kq && k < L && ra < nrows;
                    pa[kk] = ok ? prow[2 * k] : T(0);
                    ma[kk] = ok ? prow[2 * (moff + k)] : T(0);
                }
            }
            const int xb = kKeepB ? tx : 0;
            Acc C = {0, 0, 0, 0}, Sg = {0, 0, 0, 0};
            if (tx < ntile && rg < n_rt) {
                if (!kKeepB)
                    load_phi_b<T, KQ>(twp, nslot, L, kq, st * 64 + tx * 16 + li, lj, bcr[0], bsr[0]);
                const T* bc = bcr[xb];
                const T* bs = bsr[xb];
#pragma unroll
                for (int kk = 0; kk < KQ; ++kk) {
                    if (kk < kq) {
                        C = MF::step(pa[kk], bc[kk], C);
                        Sg = MF::step(ma[kk], bs[kk], Sg);
                    }
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                w[x][4 * h + 0] = C[2 * h] + Sg[2 * h];
                w[x][4 * h + 1] = C[2 * h + 1] + Sg[2 * h + 1];
                w[x][4 * h + 2] = C[2 * h] - Sg[2 * h];
                w[x][4 * h + 3] = C[2 * h + 1] - Sg[2 * h + 1];
            }
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) transpose4(w[0][e], w[1][e], w[2][e], w[3][e]);
        // now w[j][e] of lane l belongs to row group j and slot 64*st + l, or in pair mode
        // to row group j of 8-row group rt + (l >> 5) and slot l & 31
        const int s = pair ? (lane & 31) : st * 64 + lane;
        const int rbase = (pair ? rt + (lane >> 5) : rt) * 8;
        if (s >= nslot) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int rr = rbase + (h ? MF::second_row(j) : MF::first_row(j));
                if (rr >= nrows) continue;
                V* out;
                V* mout;
                T msign;
                row_out(rr, out, mout, msign);
                if (!out) continue;
                const V v1 = vmk<V>(w[j][4 * h + 0], w[j][4 * h + 1]);
                const V v2 = vmk<V>(w[j][4 * h + 2], w[j][4 * h + 3]);
                out[s] = v1;
                if (s > 0) out[n_phi - s] = v2;
                if (mout) {
                    mout[s] = vmk<V>(msign * v1.x, -msign * v1.y);
                    if (s > 0) mout[n_phi - s] = vmk<V>(msign * v2.x, -msign * v2.y);
                }
            }
        }
    }
}

}  // namespace slsht
