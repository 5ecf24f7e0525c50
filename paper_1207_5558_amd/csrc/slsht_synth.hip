// gfx950 kernel K3 of the directional SLSHT forward path: the fused synthesis of
// g(phi_a, theta_b, omega_c; l, m) from the coupling coefficients A^p_q(l, m), the
// window h and the Wigner-d table, in the separated form of
// eq. Eq:alternative_harmonic_formulation_wigner (Section IV-B).
#include "slsht_device.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

namespace slsht {

// ------------------------------------------------------------------------------
// K3: fused synthesis.  One block = one (l, m) item x a tile of tb theta rows.
//   stage 1 (theta): S_{q,q'}(theta_b) = sum_p A^p_q h_p^{q'} d^p_{q,q'}(theta_b)   -> LDS
//   stage 2 (omega): U_q(theta_b, omega_c) = sum_{q'} S_{q,q'} e^{-i q' omega_c}, folded
//                    into P_q = U_q + U_{-q}, M_q = -i (U_q - U_{-q})             -> LDS
//   stage 3 (phi):   g(phi_a) = U_0 + sum_{q>0} P_q cos(q phi_a) + M_q sin(q phi_a),
//                    g(phi_{n-a}) = same with the sine part negated                -> HBM
// The cosine/sine folding uses phi_{n-a} = -phi_a (mod 2 pi), so one product makes
// two outputs; stage 2 folds omega the same way.  For L_h <= 8 stage 3 runs on the
// VALU: a lane keeps cos/sin(q phi_a) of its slots in registers and reads U_0, P_q, M_q
// as LDS broadcasts.  For L_h > 8 those broadcasts would bound it, and stage 3 is a
// pair of real GEMMs on the matrix cores, one row per (omega_c, theta_b, Re|Im) and
// one column per slot a:
//   C = Pmat (rows x k) * cos(k phi_a) (k x a),   S = Mmat * sin(k phi_a),
// with P_0 = U_0 carried by cos(0) = 1.  16x16x4 MFMA (FP32 or FP64): lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; the FP32 form returns D rows 4(l/16)+r, the FP64
// form rows (l/16)+4r, of column l%16.  A-operand rows are permuted per precision so
// that every lane receives Re and Im of two complex rows.

struct SynthArgs {
    const double2* A;
    const double2* h;
    const void* dtab;
    const void* twphi;
    const void* twom;
    void* g;
    int64_t dstride;
    int L, K, n_phi, n_omega, n_theta_out, tb, n_tiles, nslot, ncp, l_lo, real_pair;
    int N;        // azimuthal band-limit of the window (|q'| < N)
    int xsize;    // elements of the A/h | P/M union region in LDS
    int item0;    // first item of this launch (chunks of the staged path)
    const void* pm;     // staged path: P/M rows [item - item0][theta][2 PW][pm_ncw]
    int pm_ncw;
};

struct SynthBatch {
    SynthArgs r[kSynthBatchMax];
    int first[kSynthBatchMax + 1];
    int n;
};

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

// One block of one transform: block `bid` of the grid that a.n_items x a.n_tiles blocks form.
// PMIN: the P/M rows come from the staged path's U GEMM (a.pm) instead of stages 1-2.
template <typename T, int LH, int NS, bool PMIN = false>
__device__ __forceinline__ void synth_block(const SynthArgs& a, const int bid) {
    using V = typename VecOf<T>::type;
    using MF = MfmaOf<T>;
    using Acc = typename MF::acc;
    constexpr int KQ = LH / 4;                   // MFMA k-steps of the phi GEMM
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* S_s = reinterpret_cast<V*>(smem_raw);
    const int L = a.L, K = a.K;
    // P|M row: P_0..P_{PW-1} M_0..M_{PW-1}; the VALU phi stage reads LH entries, the MFMA
    // stage the k-steps that cover L
    const int PW = LH <= 8 ? LH : (L + 3) / 4 * 4;
    const int PMS = 2 * PW + 1;                  // complex stride of one P|M row
    V* X_s = PMIN ? S_s : S_s + a.tb * K * K;
    V* A_s = X_s;
    V* h_s = X_s + L * L;
    V* PM_s = X_s;                               // [c*tb + t][P_0..P_{PW-1} M_0..M_{PW-1}]
    V* TW_s = X_s + a.xsize;                     // [L-1][ncp] omega twiddles

    const int item_rel = bid / a.n_tiles;
    const int tile = bid - item_rel * a.n_tiles;
    const Item it = item_decode(a.item0 + item_rel, a.l_lo, a.real_pair);
    const int t0 = tile * a.tb;
    const int tb = min(a.tb, a.n_theta_out - t0);
    const int tid = threadIdx.x, nth = blockDim.x;

    if constexpr (PMIN) {
        // P/M rows of the tile's theta rows: global [theta][kslot][c] -> LDS [(c, theta)][kslot]
        const V* src = reinterpret_cast<const V*>(a.pm) +
                       ((int64_t)item_rel * a.n_theta_out + t0) * 2 * PW * a.pm_ncw;
        const int per_t = 2 * PW * a.n_omega;
        for (int i = tid; i < tb * per_t; i += nth) {
            const int t = i / per_t, r = i - t * per_t;
            const int ks = r / a.n_omega, c = r - ks * a.n_omega;
            PM_s[(c * tb + t) * PMS + ks] = src[((int64_t)t * 2 * PW + ks) * a.pm_ncw + c];
        }
        __syncthreads();
    } else {
        const V* twg = reinterpret_cast<const V*>(a.twom);
        for (int i = tid; i < L * L; i += nth) {
            A_s[i] = vcast<V>(a.A[(int64_t)it.lm * L * L + i]);
            h_s[i] = vcast<V>(a.h[i]);
        }
        for (int i = tid; i < (L - 1) * a.ncp; i += nth) TW_s[i] = twg[i];
        __syncthreads();

        // stage 1: theta contraction over |q'| < N (see theta_item / theta_pair)
        const T* dt = reinterpret_cast<const T*>(a.dtab);
        const int KK = K * K;
        const int nrep = theta_items(L, a.N);
        for (int j = 0; j * nth < tb * nrep; ++j) {
            if (tid >= tb * nrep - j * nth) break;
            const int idx = snake_item(j, tid, nth, tb * nrep);
            const int t = idx / nrep;
            int s_, q, qp;
            theta_item(idx - t * nrep, L, a.N, s_, q, qp);
            V v, vm;
            theta_pair<T, V, (sizeof(T) == 8 ? 4 : 8)>(dt + (int64_t)(t0 + t) * a.dstride, A_s, h_s, L, s_, q, qp, v, vm);
            S_s[t * KK + (q + L - 1) * K + (qp + L - 1)] = v;
            if (s_ > 0) S_s[t * KK + (L - 1 - q) * K + (L - 1 - qp)] = vm;
        }
        __syncthreads();

        // stage 2: omega synthesis, folded into P/M
        const V* twom = TW_s;
        const int per_t = a.ncp * L;
        for (int idx = tid; idx < tb * per_t; idx += nth) {
            const int t = idx / per_t;
            const int r = idx - t * per_t;
            const int cs = r / L;
            const int qa = r - cs * L;
            const V* Sp = S_s + t * KK + (qa + L - 1) * K;
            const V* Sm = S_s + t * KK + (L - 1 - qa) * K;
            V Xp = Sp[L - 1], Xm = Sm[L - 1];
            V Yp = vmk<V>(0, 0), Ym = vmk<V>(0, 0);
            for (int k = 1; k < a.N; ++k) {
                const V tw = twom[(k - 1) * a.ncp + cs];
                const V a1 = Sp[L - 1 + k], a2 = Sp[L - 1 - k];
                const V b1 = Sm[L - 1 + k], b2 = Sm[L - 1 - k];
                Xp.x += (a1.x + a2.x) * tw.x; Xp.y += (a1.y + a2.y) * tw.x;
                Yp.x += (a1.x - a2.x) * tw.y; Yp.y += (a1.y - a2.y) * tw.y;
                Xm.x += (b1.x + b2.x) * tw.x; Xm.y += (b1.y + b2.y) * tw.x;
                Ym.x += (b1.x - b2.x) * tw.y; Ym.y += (b1.y - b2.y) * tw.y;
            }
            Yp = vmul_mi(Yp);
            Ym = vmul_mi(Ym);
            const int c1 = cs;
            int c2 = a.n_omega - cs;
            if (cs == 0 || c2 == cs) c2 = -1;
            for (int side = 0; side < 2; ++side) {
                const int c = side == 0 ? c1 : c2;
                if (c < 0) break;
                const V Up = side == 0 ? vadd(Xp, Yp) : vsub(Xp, Yp);
                V* P = PM_s + (c * tb + t) * PMS;
                V* M = P + PW;
                if (qa == 0) {
                    P[0] = Up;
                    M[0] = vmk<V>(0, 0);
                    for (int k = L; k < PW; ++k) { P[k] = vmk<V>(0, 0); M[k] = vmk<V>(0, 0); }
                } else {
                    const V Um = side == 0 ? vadd(Xm, Ym) : vsub(Xm, Ym);
                    P[qa] = vadd(Up, Um);
                    M[qa] = vmul_mi(vsub(Up, Um));
                }
            }
        }
        __syncthreads();
    }

    if constexpr (LH <= 8) {
        // stage 3: phi synthesis and store.  Wave w takes rows w, w + nwaves, ...; a lane
        // owns NS phi slots of each chunk of 64*NS slots and keeps their cos/sin(q phi_a) in
        // registers, so every U_0/P_q/M_q broadcast from LDS feeds NS slots (2*NS outputs).
        const int lane = tid & 63, wave = tid >> 6, nwaves = nth >> 6;
        const V* twp = reinterpret_cast<const V*>(a.twphi);
        V* g = reinterpret_cast<V*>(a.g);
        const int nrows = a.n_omega * tb;
        const T msign = (it.m & 1) ? T(-1) : T(1);
        const int64_t lm_stride = (int64_t)a.n_omega * a.n_theta_out * a.n_phi;
        for (int cb = 0; cb < a.nslot; cb += 64 * NS) {
            T cw[NS][LH], sw[NS][LH];
    #pragma unroll
            for (int j = 0; j < NS; ++j) {
                const int s = cb + j * 64 + lane;
    #pragma unroll
                for (int k = 1; k < LH; ++k) {
                    if (k < L && s < a.nslot) {
                        const V tw = twp[(k - 1) * a.nslot + s];
                        cw[j][k] = tw.x;
                        sw[j][k] = tw.y;
                    } else {
                        cw[j][k] = 0;
                        sw[j][k] = 0;
                    }
                }
            }
            for (int row = wave; row < nrows; row += nwaves) {
                const int c = row / tb;
                const int t = row - c * tb;
                const V* P = PM_s + (c * tb + t) * PMS;
                const V* M = P + LH;
                V C[NS], Sv[NS];
                const V p0 = P[0];
    #pragma unroll
                for (int j = 0; j < NS; ++j) { C[j] = p0; Sv[j] = vmk<V>(0, 0); }
    #pragma unroll
                for (int k = 1; k < LH; ++k) {
                    const V pk = P[k], mk = M[k];
    #pragma unroll
                    for (int j = 0; j < NS; ++j) {
                        C[j].x += pk.x * cw[j][k];
                        C[j].y += pk.y * cw[j][k];
                        Sv[j].x += mk.x * sw[j][k];
                        Sv[j].y += mk.y * sw[j][k];
                    }
                }
                const int64_t rowoff = ((int64_t)c * a.n_theta_out + (t0 + t)) * a.n_phi;
                V* out = g + (int64_t)it.lm * lm_stride + rowoff;
                V* mout = it.mirror >= 0 ? g + (int64_t)it.mirror * lm_stride + rowoff : nullptr;
    #pragma unroll
                for (int j = 0; j < NS; ++j) {
                    const int s = cb + j * 64 + lane;
                    if (s < a.nslot) {
                        const V v1 = vadd(C[j], Sv[j]), v2 = vsub(C[j], Sv[j]);
                        out[s] = v1;
                        if (s > 0) out[a.n_phi - s] = v2;
                        if (mout) {
                            // g(l,-m) = (-1)^m conj(g(l,m))
                            mout[s] = vmk<V>(msign * v1.x, -msign * v1.y);
                            if (s > 0) mout[a.n_phi - s] = vmk<V>(msign * v2.x, -msign * v2.y);
                        }
                    }
                }
            }
        }
    } else {
        // stage 3: phi synthesis on the matrix cores.  Work unit = (8 complex rows, 64 slots):
        // four 16-slot GEMM tiles share the unit's A fragments; their results are then
        // transposed across lane groups so that lane l holds slot 64*unit + l of each row
        // and every store instruction writes 64 consecutive outputs of one row.
        const int lane = tid & 63, wave = tid >> 6, nwaves = nth >> 6;
        const int li = lane & 15, lj = lane >> 4;
        const V* twp = reinterpret_cast<const V*>(a.twphi);
        V* g = reinterpret_cast<V*>(a.g);
        const int nrows = a.n_omega * tb;
        const int n_rt = (nrows + 7) / 8;
        const int n_st = (a.nslot + 63) / 64;
        const int kq = (L + 3) / 4;
        const T msign = (it.m & 1) ? T(-1) : T(1);
        const int64_t lm_stride = (int64_t)a.n_omega * a.n_theta_out * a.n_phi;
        V* gl = g + (int64_t)it.lm * lm_stride;
        V* gm = it.mirror >= 0 ? g + (int64_t)it.mirror * lm_stride : nullptr;
        const int arow = MF::row_of(li), apart = MF::part_of(li);
        // B fragments (cos/sin(k phi_s)) of the unit's four slot tiles stay in registers
        // while consecutive units share the slot range: a wave takes a contiguous run of
        // units ordered slot-range-major.  FP64 with L_h > 16 reloads them per unit instead
        // (register budget).
        constexpr bool kKeepB = !(sizeof(T) == 8 && LH > 16);
        constexpr int NB = kKeepB ? 4 : 1;
        T bcr[NB][KQ], bsr[NB][KQ];
        int cur_st = -1;
        const int nu = n_rt * n_st;
        const int u_end = ((wave + 1) * nu) / nwaves;
        for (int u = (wave * nu) / nwaves; u < u_end; ++u) {
            const int st = u / n_rt;
            const int rt = u - st * n_rt;
            if (kKeepB && st != cur_st) {
                cur_st = st;
    #pragma unroll
                for (int x = 0; x < NB; ++x) load_phi_b<T, KQ>(twp, a.nslot, L, kq, st * 64 + x * 16 + li, lj,
                                                             bcr[x], bsr[x]);
            }
            const int ra = rt * 8 + arow;
            const T* prow = reinterpret_cast<const T*>(PM_s + (ra < nrows ? ra : 0) * PMS) + apart;
            T pa[KQ], ma[KQ];
    #pragma unroll
            for (int kk = 0; kk < KQ; ++kk) {
                const int k = 4 * kk + lj;
                pa[kk] = (kk < kq && ra < nrows) ? prow[2 * k] : T(0);
                ma[kk] = (kk < kq && ra < nrows) ? prow[2 * (PW + k)] : T(0);
            }
            // w[x][e]: x = 16-slot tile of the unit, e = (row h, value): Re/Im of C+S, C-S
            T w[4][8];
    #pragma unroll
            for (int x = 0; x < 4; ++x) {
                const int xb = kKeepB ? x : 0;
                if (!kKeepB)
                    load_phi_b<T, KQ>(twp, a.nslot, L, kq, st * 64 + x * 16 + li, lj, bcr[0], bsr[0]);
                const T* bc = bcr[xb];
                const T* bs = bsr[xb];
                Acc C = {0, 0, 0, 0}, Sg = {0, 0, 0, 0};
    #pragma unroll
                for (int kk = 0; kk < KQ; ++kk) {
                    if (kk < kq) {
                        C = MF::step(pa[kk], bc[kk], C);
                        Sg = MF::step(ma[kk], bs[kk], Sg);
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
            // now w[j][e] of lane l belongs to row group j, slot 64*st + l
            const int s = st * 64 + lane;
            if (s >= a.nslot) continue;
    #pragma unroll
            for (int j = 0; j < 4; ++j) {
    #pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int rr = rt * 8 + (h ? MF::second_row(j) : MF::first_row(j));
                    if (rr >= nrows) continue;
                    const int c = rr / tb;
                    const int t = rr - c * tb;
                    const V v1 = vmk<V>(w[j][4 * h + 0], w[j][4 * h + 1]);
                    const V v2 = vmk<V>(w[j][4 * h + 2], w[j][4 * h + 3]);
                    const int64_t rowoff = ((int64_t)c * a.n_theta_out + (t0 + t)) * a.n_phi;
                    V* out = gl + rowoff;
                    out[s] = v1;
                    if (s > 0) out[a.n_phi - s] = v2;
                    if (gm) {
                        // g(l,-m) = (-1)^m conj(g(l,m))
                        V* mout = gm + rowoff;
                        mout[s] = vmk<V>(msign * v1.x, -msign * v1.y);
                        if (s > 0) mout[a.n_phi - s] = vmk<V>(msign * v2.x, -msign * v2.y);
                    }
                }
            }
        }
    }
}

template <typename T, int LH, int NS>
__global__ void __launch_bounds__(256) synth_full_kernel(const SynthArgs a) {
    synth_block<T, LH, NS>(a, (int)blockIdx.x);
}

// The phi stage and store alone, from the staged path's P/M rows (L_h above 16).
template <typename T, int LH>
__global__ void __launch_bounds__(256) synth_pm_kernel(const SynthArgs a) {
    synth_block<T, LH, 1, true>(a, (int)blockIdx.x);
}

// Several transforms that share one kernel instance in one grid (a tile list across
// requests): transform r owns blocks [first[r], first[r+1]).  The per-transform arguments
// travel in the kernel-argument block, so a launch needs no device allocation or copy.
template <typename T, int LH, int NS>
__global__ void __launch_bounds__(256) synth_batch_kernel(const SynthBatch b) {
    int r = 0;
    while (r + 1 < b.n && (int)blockIdx.x >= b.first[r + 1]) ++r;
    synth_block<T, LH, NS>(b.r[r], (int)blockIdx.x - b.first[r]);
}

static int lh_bucket(int L) { return L <= 4 ? 4 : (L <= 8 ? 8 : (L <= 16 ? 16 : (L <= 24 ? 24 : 32))); }

static size_t synth_xsize(const DevPlan& P, int tb) {
    const int LH = lh_bucket(P.d.L_h);
    const int PW = LH <= 8 ? LH : (P.d.L_h + 3) / 4 * 4;
    const size_t rows = ((size_t)tb * P.d.n_omega + 7) / 8 * 8;
    if (P.staged) return rows * (2 * PW + 1);             // P/M rows only
    return std::max((size_t)2 * P.d.L_h * P.d.L_h, rows * (2 * PW + 1));
}

static size_t synth_lds_bytes(const DevPlan& P, int tb) {
    const int L = P.d.L_h, K = 2 * L - 1;
    const size_t v = P.d.precision == SLSHT_FP64 ? 16 : 8;
    if (P.staged) return synth_xsize(P, tb) * v;
    const size_t s = (size_t)tb * K * K;
    const size_t tw = (size_t)(L > 1 ? L - 1 : 0) * (P.d.n_omega / 2 + 1);
    return (s + synth_xsize(P, tb) + tw) * v;
}

// Phi slots per lane of the VALU phi stage (L_h <= 8): the most that the row needs and
// the register budget allows.
static int ns_max(bool f64, int LH) {
    if (f64) return LH == 4 ? 4 : 3;
    return 4;
}

template <typename T, int LH, int NS>
static const void* synth_pick(bool batch) {
    return batch ? (const void*)synth_batch_kernel<T, LH, NS> : (const void*)synth_full_kernel<T, LH, NS>;
}

template <typename T, int LH>
static const void* synth_fn_t(int nslot, bool batch) {
    if constexpr (LH >= 16) {
        return synth_pick<T, LH, 1>(batch);
    } else {
        const int ns = std::min((nslot + 63) / 64, ns_max(sizeof(T) == 8, LH));
        if constexpr (sizeof(T) == 8 && LH == 8) {
            return ns <= 1 ? synth_pick<T, LH, 1>(batch)
                 : ns == 2 ? synth_pick<T, LH, 2>(batch)
                           : synth_pick<T, LH, 3>(batch);
        } else {
            return ns <= 1 ? synth_pick<T, LH, 1>(batch)
                 : ns == 2 ? synth_pick<T, LH, 2>(batch)
                 : ns == 3 ? synth_pick<T, LH, 3>(batch)
                           : synth_pick<T, LH, 4>(batch);
        }
    }
}

static const void* synth_pm_fn(const DevPlan& P) {
    const bool f64 = P.d.precision == SLSHT_FP64;
    switch (lh_bucket(P.d.L_h)) {
        case 24: return f64 ? (const void*)synth_pm_kernel<double, 24> : (const void*)synth_pm_kernel<float, 24>;
        default: return f64 ? (const void*)synth_pm_kernel<double, 32> : (const void*)synth_pm_kernel<float, 32>;
    }
}

static const void* synth_fn(const DevPlan& P, bool batch = false) {
    if (P.staged) return synth_pm_fn(P);
    const bool f64 = P.d.precision == SLSHT_FP64;
    const int ns = P.nslot_phi;
    switch (lh_bucket(P.d.L_h)) {
        case 4: return f64 ? synth_fn_t<double, 4>(ns, batch) : synth_fn_t<float, 4>(ns, batch);
        case 8: return f64 ? synth_fn_t<double, 8>(ns, batch) : synth_fn_t<float, 8>(ns, batch);
        case 16: return f64 ? synth_fn_t<double, 16>(ns, batch) : synth_fn_t<float, 16>(ns, batch);
        case 24: return f64 ? synth_fn_t<double, 24>(ns, batch) : synth_fn_t<float, 24>(ns, batch);
        default: return f64 ? synth_fn_t<double, 32>(ns, batch) : synth_fn_t<float, 32>(ns, batch);
    }
}

// Staged plans run their own launches (W table, U GEMM, phi stage per chunk), so each one
// gets a key of its own and is never grouped with other transforms.
const void* synthesis_kernel_key(const DevPlan& P) { return P.staged ? (const void*)&P : synth_fn(P); }

// Theta rows per block: stages 1-2 run between barriers with no stores in flight, so
// the store stream is kept busy by other resident blocks.  The tile is the largest one
// (at most 8 rows) among those that reach the highest resident block count the kernel's
// registers and the LDS allow.
bool choose_synthesis_shape(DevPlan& P, size_t lds_limit) {
    P.block = 256;
    const void* fn = synth_fn(P);
    int best_occ = 0, best_tb = 0;
    for (int tb = std::min(8, P.n_theta_out); tb >= 1; --tb) {
        const size_t lds = synth_lds_bytes(P, tb);
        if (lds > lds_limit) continue;
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, P.block, lds) != hipSuccess)
            occ = lds <= 64 * 1024 ? 2 : 1;
        if (occ > best_occ) {
            best_occ = occ;
            best_tb = tb;
        }
    }
    if (best_tb == 0) return false;
    P.tb = best_tb;
    P.lds_bytes = synth_lds_bytes(P, best_tb);
    return true;
}

static SynthArgs synth_args(const DevPlan& P, const double2* A, const double2* h, void* g) {
    SynthArgs a;
    a.A = A;
    a.h = h;
    a.dtab = P.T->dtab;
    a.twphi = P.T->tw_phi;
    a.twom = P.T->tw_omega;
    a.g = g;
    a.dstride = dtab_row_len(P.d.L_h);
    a.L = P.d.L_h;
    a.K = 2 * P.d.L_h - 1;
    a.n_phi = P.d.n_phi;
    a.n_omega = P.d.n_omega;
    a.n_theta_out = P.n_theta_out;
    a.tb = P.tb;
    a.n_tiles = (P.n_theta_out + P.tb - 1) / P.tb;
    a.nslot = P.nslot_phi;
    a.ncp = P.ncp_omega;
    a.l_lo = P.d.l_lo;
    a.real_pair = (P.d.flags & SLSHT_REAL_PAIR) ? 1 : 0;
    a.xsize = (int)synth_xsize(P, P.tb);
    a.N = n_az_of(P.d);
    a.item0 = 0;
    a.pm = nullptr;
    a.pm_ncw = 0;
    return a;
}

hipError_t launch_synthesis_pm(const DevPlan& P, const void* pm, int item0, int n, void* g,
                               hipStream_t s) {
    SynthArgs a = synth_args(P, nullptr, nullptr, g);
    a.item0 = item0;
    a.pm = pm;
    a.pm_ncw = P.sg.ncw;
    const int64_t nblk = (int64_t)n * a.n_tiles;
    if (nblk > 0x7fffffff) return hipErrorInvalidConfiguration;
    const void* fn = synth_pm_fn(P);
    if (P.lds_bytes > 64 * 1024)
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.lds_bytes);
    void* args[] = {&a};
    return hipLaunchKernel(fn, dim3((unsigned)nblk), dim3(P.block), args, P.lds_bytes, s);
}

hipError_t launch_synthesis(const DevPlan& P, const double2* A, const double2* h, void* g,
                            hipStream_t s) {
    if (P.staged) return launch_synthesis_staged(P, A, h, g, s);
    SynthArgs a = synth_args(P, A, h, g);
    const int64_t nblk = (int64_t)P.n_items * a.n_tiles;
    if (nblk > 0x7fffffff) return hipErrorInvalidConfiguration;   // grid.x limit
    void* args[] = {&a};
    return hipLaunchKernel(synth_fn(P), dim3((unsigned)nblk), dim3(P.block), args, P.lds_bytes, s);
}

hipError_t launch_synthesis_batch(const DevPlan* const* P, const double2* const* A,
                                  const double2* const* h, void* const* g, int n, hipStream_t s) {
    if (n < 1 || n > kSynthBatchMax) return hipErrorInvalidValue;
    if (P[0]->staged) {
        // staged plans are grouped alone (their key is unique)
        if (n != 1) return hipErrorInvalidValue;
        return launch_synthesis_staged(*P[0], A[0], h[0], g[0], s);
    }
    const void* fn = synth_fn(*P[0], true);
    SynthBatch b;
    std::memset(&b, 0, sizeof(b));
    b.n = n;
    int64_t nblk = 0;
    size_t lds = 0;
    for (int i = 0; i < n; ++i) {
        if (synth_fn(*P[i], true) != fn || P[i]->block != P[0]->block)
            return hipErrorInvalidValue;                               // one kernel per launch
        b.r[i] = synth_args(*P[i], A[i], h[i], g[i]);
        b.first[i] = (int)nblk;
        nblk += (int64_t)P[i]->n_items * b.r[i].n_tiles;
        if (nblk > 0x7fffffff) return hipErrorInvalidConfiguration;
        lds = std::max(lds, P[i]->lds_bytes);
    }
    b.first[n] = (int)nblk;
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    void* args[] = {&b};
    return hipLaunchKernel(fn, dim3((unsigned)nblk), dim3(P[0]->block), args, lds, s);
}

}  // namespace slsht
