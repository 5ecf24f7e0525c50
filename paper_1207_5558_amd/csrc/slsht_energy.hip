// gfx950 kernel K3e of the directional SLSHT forward path: the ENERGY output
// E(rho; l) = sum_m |g(rho; l, m)|^2, reduced over the orders m on the fly.
#include "slsht_device.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

namespace slsht {

// ------------------------------------------------------------------------------
// K3e: energy epilogue, FP32.  One block = one degree l x one theta row; the order m
// runs inside the block and E(phi_a, theta_b, omega_c; l) = sum_m |g|^2 stays in
// registers until all orders are done, so g is never written.  The block's canonical
// Wigner-d row is staged in LDS once.  Per m:
//   stage 1 (VALU): S_{q,q'}(theta_b) as in K3, d read from LDS          -> LDS
//   stage 2 (MFMA + VALU): omega synthesis as folded real GEMMs
//                   X[q][c] = S[q][0] + sum_k (S[q][k] + S[q][-k]) cos(k omega_c),
//                   Y[q][c] = sum_k (S[q][k] - S[q][-k]) sin(k omega_c), then the fold
//                   into P_k, M_k, stored k-major with omega contiguous (the B operand
//                   layout of stage 3)                                        -> LDS
//   stage 3 (MFMA): the phi synthesis is a real GEMM per part (Re, Im) and per
//                   cos/sin half:  C[a][c] = sum_k cos(k phi_a) P_k(c),
//                   S[a][c] = sum_k sin(k phi_a) M_k(c)   (16x16x4 FP32 MFMA),
//                   then E(a) += |C+S|^2 and E(n-a) += |C-S|^2 elementwise.
// A fragments (cos/sin(k phi_a)) come from an n_phi-entry cos/sin table in LDS at
// index k*a mod n_phi, advanced incrementally.  Lane l of a 16x16x4 FP32 MFMA
// supplies A[l%16][l/16] and B[l/16][l%16] and receives D rows 4*(l/16)+r, column l%16.

struct EnergyArgs {
    const double2* A;
    const double2* h;
    const float* dtab;
    const float2* twom;
    const float2* twfull;
    float* E;
    int64_t dstride;
    int L, K, KP, l_lo, n_l, n_phi, n_omega, n_theta_out, nslot, ncp, nst, nct, nctp, cstride;
    int real_pair, nblk;
    int N;        // azimuthal band-limit of the window (|q'| < N)
};

constexpr int kEnergyWaves = 8;

// TPW: slot tiles per wave; NKK >= KP/4: k-steps of the MFMA loops, a compile-time bound
// so that the loops unroll and every A fragment of a tile is loaded before its MFMAs.
template <int TPW, int NKK>
__global__ void __launch_bounds__(64 * kEnergyWaves) energy_kernel(const EnergyArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int L = a.L, K = a.K, KK = K * K, KP = a.KP, cs_ = a.cstride;
    const int ncw = (a.ncp + 15) / 16 * 16;                      // omega slots, padded
    const int nqt = (K + 15) / 16;                               // q tiles of the omega GEMM
    float4* XY = reinterpret_cast<float4*>(smem_raw);            // [nqt*16][ncw] X, Y parts
    float2* A_s = reinterpret_cast<float2*>(XY + nqt * 16 * ncw);
    float2* h_s = A_s + L * L;
    float2* S_s = h_s + L * L;                                   // [K][K], stages 1-2
    float* PMt = reinterpret_cast<float*>(S_s);                  // [4][KP][cstride], fold and
                                                                 // stage 3 (S_s is dead by then)
    float2* tw = S_s + max(KK, 2 * KP * cs_);                    // [n_phi] cos/sin(2 pi j/n_phi)
    float2* twW = tw + a.n_phi;                                  // [KP][ncw] cos/sin(k omega_cs)
    float* D_s = reinterpret_cast<float*>(twW + KP * ncw);       // canonical d row of this block
    const int tid = threadIdx.x, nth = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;

    // XCD-aware order: consecutive logical blocks (same theta row, other degrees) land
    // on one XCD and share its L2 copy of the Wigner-d row.
    int bid = blockIdx.x;
    if ((a.nblk & 7) == 0) bid = (blockIdx.x & 7) * (a.nblk >> 3) + (blockIdx.x >> 3);
    const int t = bid / a.n_l;
    const int lidx = bid - t * a.n_l;
    const int l = a.l_lo + lidx;

    for (int i = tid; i < a.n_phi; i += nth) tw[i] = a.twfull[i];
    {
        const float* drow = a.dtab + (int64_t)t * a.dstride;
        for (int i = tid; i < a.dstride; i += nth) D_s[i] = drow[i];
    }
    for (int i = tid; i < KP * ncw; i += nth) {
        const int k = i / ncw, cs = i - k * ncw;
        float2 v = vmk<float2>(0.0f, 0.0f);
        if (cs < a.ncp && k < L) v = k == 0 ? vmk<float2>(1.0f, 0.0f) : a.twom[(k - 1) * a.ncp + cs];
        twW[i] = v;
    }
    for (int i = tid; i < L * L; i += nth) h_s[i] = vcast<float2>(a.h[i]);

    // energy of this wave's tiles (omega tile w % nctp, slot tiles w / nctp + j * 8 / nctp)
    float Ep[TPW][4], Em[TPW][4];
#pragma unroll
    for (int j = 0; j < TPW; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) { Ep[j][r] = 0.0f; Em[j][r] = 0.0f; }

    const int nrep = theta_items(L, a.N);
    const int nm = a.real_pair ? l + 1 : 2 * l + 1;
    for (int mi = 0; mi < nm; ++mi) {
        const int m = a.real_pair ? mi : mi - l;
        // real pair: E = 2 (|g_0|^2 / 2 + sum_{m>0} |g_m|^2); the m = 0 half-weight is
        // applied by scaling that order's B fragments by sqrt(1/2), the factor 2 at the store
        const float bscale = (a.real_pair && m == 0) ? 0.70710678118654752f : 1.0f;
        const int64_t lm = (int64_t)l * l + l + m - (int64_t)a.l_lo * a.l_lo;
        for (int i = tid; i < L * L; i += nth) A_s[i] = vcast<float2>(a.A[lm * L * L + i]);
        __syncthreads();

        // stage 1: theta contraction over |q'| < N (see theta_item / theta_pair)
        for (int j = 0; j * nth < nrep; ++j) {
            if (tid >= nrep - j * nth) break;
            int s_, q, qp;
            theta_item(snake_item(j, tid, nth, nrep), L, a.N, s_, q, qp);
            float2 v, vm;
            theta_pair<float, float2, 4>(D_s, A_s, h_s, L, s_, q, qp, v, vm);
            S_s[(q + L - 1) * K + (qp + L - 1)] = v;
            if (s_ > 0) S_s[(L - 1 - q) * K + (L - 1 - qp)] = vm;
        }
        __syncthreads();

        // stage 2: omega synthesis as folded real GEMMs on the MFMA units,
        //   X[q][c] = S[q][0] + sum_{k>0} (S[q][k] + S[q][-k]) cos(k omega_c)
        //   Y[q][c] =           sum_{k>0} (S[q][k] - S[q][-k]) sin(k omega_c)
        // (Re and Im separately), one 16x16 (q, omega-slot) tile per wave and step.
        for (int it = wave; it < nqt * (ncw / 16); it += kEnergyWaves) {
            const int qt = it % nqt, ct2 = it / nqt;
            const int kq2 = lane >> 4, c16 = lane & 15;
            const int qi = qt * 16 + c16;
            f4v xr = {0, 0, 0, 0}, xi = {0, 0, 0, 0}, yr = {0, 0, 0, 0}, yi = {0, 0, 0, 0};
#pragma unroll
            for (int kk = 0; kk < NKK; ++kk) {
                const int k = kk * 4 + kq2;
                float2 ap = vmk<float2>(0.0f, 0.0f), am = vmk<float2>(0.0f, 0.0f);
                if (qi < K && k < a.N) {
                    const float2* row = S_s + qi * K + (L - 1);
                    if (k == 0) {
                        ap = row[0];
                    } else {
                        const float2 s1 = row[k], s2 = row[-k];
                        ap = vadd(s1, s2);
                        am = vsub(s1, s2);
                    }
                }
                const float2 w = k < KP ? twW[k * ncw + ct2 * 16 + c16] : vmk<float2>(0.0f, 0.0f);
                xr = __builtin_amdgcn_mfma_f32_16x16x4f32(ap.x, w.x, xr, 0, 0, 0);
                xi = __builtin_amdgcn_mfma_f32_16x16x4f32(ap.y, w.x, xi, 0, 0, 0);
                yr = __builtin_amdgcn_mfma_f32_16x16x4f32(am.x, w.y, yr, 0, 0, 0);
                yi = __builtin_amdgcn_mfma_f32_16x16x4f32(am.y, w.y, yi, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float4 v;
                v.x = xr[r]; v.y = xi[r]; v.z = yr[r]; v.w = yi[r];
                XY[(qt * 16 + 4 * kq2 + r) * ncw + ct2 * 16 + c16] = v;
            }
        }
        __syncthreads();

        // fold q = +-k: U_q(omega_c) = X + Y', U_q(omega_{n-c}) = X - Y' with Y' = -i Y, then
        // P_k = U_k + U_{-k}, M_k = -i (U_k - U_{-k}); stored k-major, omega contiguous
        for (int idx = tid; idx < L * a.ncp; idx += nth) {
            const int qa = idx / a.ncp, cs = idx - qa * a.ncp;
            const float4 vp = XY[(L - 1 + qa) * ncw + cs];
            const float4 vm = XY[(L - 1 - qa) * ncw + cs];
            int c2 = a.n_omega - cs;
            if (cs == 0 || c2 == cs) c2 = -1;
            for (int side = 0; side < 2; ++side) {
                const int c = side == 0 ? cs : c2;
                if (c < 0) break;
                const float sg = side == 0 ? 1.0f : -1.0f;
                const float2 Up = vmk<float2>(vp.x + sg * vp.w, vp.y - sg * vp.z);
                float2 P, M;
                if (qa == 0) {
                    P = Up;
                    M = vmk<float2>(0, 0);
                } else {
                    const float2 Um = vmk<float2>(vm.x + sg * vm.w, vm.y - sg * vm.z);
                    P = vadd(Up, Um);
                    M = vmul_mi(vsub(Up, Um));
                }
                PMt[(0 * KP + qa) * cs_ + c] = P.x;
                PMt[(1 * KP + qa) * cs_ + c] = P.y;
                PMt[(2 * KP + qa) * cs_ + c] = M.x;
                PMt[(3 * KP + qa) * cs_ + c] = M.y;
            }
        }
        // rows L..KP-1 of the B table are read as zeros by stage 3
        for (int idx = tid; idx < 4 * (KP - L) * cs_; idx += nth) {
            const int part = idx / ((KP - L) * cs_);
            const int rem = idx - part * (KP - L) * cs_;
            PMt[(part * KP + L) * cs_ + rem] = 0.0f;
        }
        __syncthreads();

        // stage 3: MFMA phi synthesis and energy accumulation.  Wave w owns omega tile
        // ct = w % nctp and slot tiles st = w / nctp + j * (waves / nctp), so its B fragments
        // (P_k, M_k of that omega tile) are loaded once per m and stay in registers across
        // all its slot tiles.  The lane index is made opaque so that the per-tile index
        // arithmetic is redone for every m instead of being hoisted out of the m loop.
        int lane_o = lane;
        asm volatile("" : "+v"(lane_o));
        const int kq = lane_o >> 4, col = lane_o & 15;
        const int nkk = KP / 4;
        const int ct = wave % a.nctp, st0 = wave / a.nctp, sstep = kEnergyWaves / a.nctp;
        float breg[4][NKK];
        {
            const int bcol = ct * 16 + col;
#pragma unroll
            for (int kk = 0; kk < NKK; ++kk) {
                const int k = kk * 4 + kq;
#pragma unroll
                for (int part = 0; part < 4; ++part)
                    breg[part][kk] = kk < nkk ? bscale * PMt[(part * KP + k) * cs_ + bcol] : 0.0f;
            }
        }
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
            const int st = st0 + j * sstep;
            if (st >= a.nst) break;
            const int as = st * 16 + col;                      // slot of this lane's A rows
            int step4 = 4 * as;                                // (4 as) mod n_phi, as < n_phi
            while (step4 >= a.n_phi) step4 -= a.n_phi;
            int idx = kq * as;                                 // (kq as) mod n_phi, kq < 4
            while (idx >= a.n_phi) idx -= a.n_phi;
            // A fragments of all k-steps first (k beyond L meets a zero B row)
            float2 cz[NKK];
#pragma unroll
            for (int kk = 0; kk < NKK; ++kk) {
                cz[kk] = tw[idx];
                idx += step4;
                if (idx >= a.n_phi) idx -= a.n_phi;
            }
            f4v cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0}, sre = {0, 0, 0, 0}, sim = {0, 0, 0, 0};
#pragma unroll
            for (int kk = 0; kk < NKK; ++kk) {
                cre = __builtin_amdgcn_mfma_f32_16x16x4f32(cz[kk].x, breg[0][kk], cre, 0, 0, 0);
                cim = __builtin_amdgcn_mfma_f32_16x16x4f32(cz[kk].x, breg[1][kk], cim, 0, 0, 0);
                sre = __builtin_amdgcn_mfma_f32_16x16x4f32(cz[kk].y, breg[2][kk], sre, 0, 0, 0);
                sim = __builtin_amdgcn_mfma_f32_16x16x4f32(cz[kk].y, breg[3][kk], sim, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float pr = cre[r] + sre[r], pi = cim[r] + sim[r];
                const float mr = cre[r] - sre[r], mi2 = cim[r] - sim[r];
                Ep[j][r] = fmaf(pi, pi, fmaf(pr, pr, Ep[j][r]));
                Em[j][r] = fmaf(mi2, mi2, fmaf(mr, mr, Em[j][r]));
            }
            // Materialise this tile's energy here, so that its four MFMA accumulators die
            // before the next tile starts (otherwise the updates sink to the end of the
            // unrolled loop and every tile's accumulators stay live at once).
            asm volatile("" : "+v"(Ep[j][0]), "+v"(Ep[j][1]), "+v"(Ep[j][2]), "+v"(Ep[j][3]),
                         "+v"(Em[j][0]), "+v"(Em[j][1]), "+v"(Em[j][2]), "+v"(Em[j][3]));
        }
        __syncthreads();
    }

    // store: lane holds slots st*16 + 4*(lane/16) + r of omega column ct*16 + lane%16
    const float escale = a.real_pair ? 2.0f : 1.0f;
    const int kq = lane >> 4, col = lane & 15;
    const int ct = wave % a.nctp, st0 = wave / a.nctp, sstep = kEnergyWaves / a.nctp;
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
        const int st = st0 + j * sstep;
        if (st >= a.nst) break;
        const int c = ct * 16 + col;
        if (c >= a.n_omega) continue;
        float* row = a.E + (((int64_t)lidx * a.n_omega + c) * a.n_theta_out + t) * a.n_phi;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int s = st * 16 + 4 * kq + r;
            if (s >= a.nslot) continue;
            row[s] = escale * Ep[j][r];
            if (s > 0) row[a.n_phi - s] = escale * Em[j][r];
        }
    }
}

// Row stride (floats) of the k-major B table: at least nctp*16 columns, and
// congruent to 16 mod 32 so that the 4 k rows a wave reads land on different banks.
static int energy_cstride(int nctp) {
    const int c = nctp * 16;
    return c % 32 == 0 ? c + 16 : c;
}

static size_t energy_lds_bytes(const DevPlan& P, int KP, int cstride) {
    const int L = P.d.L_h, K = 2 * L - 1;
    const int ncw = (P.d.n_omega / 2 + 1 + 15) / 16 * 16, nqt = (K + 15) / 16;
    const size_t sp = std::max((size_t)K * K, (size_t)2 * KP * cstride);   // S_s | PMt
    return (size_t)nqt * 16 * ncw * sizeof(float4) + (size_t)2 * L * L * sizeof(float2) +
           sp * sizeof(float2) + (size_t)P.d.n_phi * sizeof(float2) +
           (size_t)KP * ncw * sizeof(float2) + (size_t)dtab_row_len(L) * sizeof(float);
}

hipError_t launch_energy(const DevPlan& P, const double2* A, const double2* h, float* E,
                         hipStream_t s) {
    EnergyArgs a;
    a.A = A;
    a.h = h;
    a.dtab = reinterpret_cast<const float*>(P.T->dtab);
    a.twom = reinterpret_cast<const float2*>(P.T->tw_omega);
    a.twfull = reinterpret_cast<const float2*>(P.T->tw_full);
    a.E = E;
    a.dstride = dtab_row_len(P.d.L_h);
    a.L = P.d.L_h;
    a.K = 2 * P.d.L_h - 1;
    a.KP = (P.d.L_h + 3) / 4 * 4;
    a.l_lo = P.d.l_lo;
    a.n_l = P.d.l_hi - P.d.l_lo;
    a.n_phi = P.d.n_phi;
    a.n_omega = P.d.n_omega;
    a.n_theta_out = P.n_theta_out;
    a.nslot = P.nslot_phi;
    a.ncp = P.ncp_omega;
    a.nst = (P.nslot_phi + 15) / 16;
    a.nct = (P.d.n_omega + 15) / 16;
    a.nctp = a.nct == 3 ? 4 : a.nct;                  // omega tiles padded to divide 8 waves
    a.cstride = energy_cstride(a.nctp);
    a.real_pair = (P.d.flags & SLSHT_REAL_PAIR) ? 1 : 0;
    a.nblk = a.n_l * P.n_theta_out;
    a.N = n_az_of(P.d);
    const size_t lds = energy_lds_bytes(P, a.KP, a.cstride);
    const int per = kEnergyWaves / a.nctp;           // waves sharing one omega tile
    const int tpw = (a.nst + per - 1) / per;
    const int nkk = a.KP / 4;
    const int ki = nkk <= 2 ? 0 : (nkk <= 4 ? 1 : 2);
    const int ti = tpw <= 4 ? 0 : (tpw <= 8 ? 1 : (tpw <= 12 ? 2 : (tpw <= 17 ? 3 : -1)));
    if (ti < 0) return hipErrorInvalidValue;
    const void* fns[4][3] = {
        {(const void*)energy_kernel<4, 2>, (const void*)energy_kernel<4, 4>, (const void*)energy_kernel<4, 8>},
        {(const void*)energy_kernel<8, 2>, (const void*)energy_kernel<8, 4>, (const void*)energy_kernel<8, 8>},
        {(const void*)energy_kernel<12, 2>, (const void*)energy_kernel<12, 4>, (const void*)energy_kernel<12, 8>},
        {(const void*)energy_kernel<17, 2>, (const void*)energy_kernel<17, 4>, (const void*)energy_kernel<17, 8>}};
    const void* fn = fns[ti][ki];
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    void* args[] = {&a};
    const hipError_t e = hipLaunchKernel(fn, dim3(a.nblk), dim3(64 * kEnergyWaves), args, lds, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

size_t energy_lds_for(const DevPlan& P) {
    const int KP = (P.d.L_h + 3) / 4 * 4;
    const int nct = (P.d.n_omega + 15) / 16;
    return energy_lds_bytes(P, KP, energy_cstride(nct == 3 ? 4 : nct));
}

}  // namespace slsht
