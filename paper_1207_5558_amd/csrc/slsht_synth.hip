// gfx950 kernel K3 of the directional SLSHT forward path: the fused synthesis of
// g(phi_a, theta_b, omega_c; l, m) from the coupling coefficients A^p_q(l, m), the
// window h and the Wigner-d table, in the separated form of
// eq. Eq:alternative_harmonic_formulation_wigner (Section IV-B).
#include "slsht_device.h"
#include "slsht_phi.h"

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
// pair of real GEMMs on the matrix cores (phi_stage_mfma, slsht_phi.h).

struct SynthArgs {
    const double2* A;
    const double2* h;
    const void* dtab;
    const void* twphi;
    const void* twom;
    void* g;
    int64_t dstride;
    int L, K, n_phi, n_omega, n_theta_out, tb, n_tiles, nslot, ncp, l_lo, real_pair;
    int nblk;     // blocks of the transform (n_items x n_tiles)
    int N;        // azimuthal band-limit of the window (|q'| < N)
    int xsize;    // elements of the A/h | P/M union region in LDS
};

struct SynthBatch {
    SynthArgs r[kSynthBatchMax];
    int first[kSynthBatchMax + 1];
    int n;
};

// One block of one transform: block `bid` of the grid that a.n_items x a.n_tiles blocks form.
template <typename T, int LH, int NS>
__device__ __forceinline__ void synth_block(const SynthArgs& a, const int bid) {
    using V = typename VecOf<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* S_s = reinterpret_cast<V*>(smem_raw);
    const int L = a.L, K = a.K;
    // P|M row: P_0..P_{PW-1} M_0..M_{PW-1}; the VALU phi stage reads LH entries, the MFMA
    // stage the k-steps that cover L
    const int PW = LH <= 8 ? LH : (L + 3) / 4 * 4;
    const int PMS = 2 * PW + 1;                  // complex stride of one P|M row
    V* X_s = S_s + a.tb * K * K;
    V* A_s = X_s;
    V* h_s = X_s + L * L;
    V* PM_s = X_s;                               // [c*tb + t][P_0..P_{PW-1} M_0..M_{PW-1}]
    V* TW_s = X_s + a.xsize;                     // [L-1][ncp] omega twiddles

    const int item_rel = bid / a.n_tiles;
    const int tile = bid - item_rel * a.n_tiles;
    const Item it = item_decode(item_rel, a.l_lo, a.real_pair);
    const int t0 = tile * a.tb;
    const int tb = min(a.tb, a.n_theta_out - t0);
    const int tid = threadIdx.x, nth = blockDim.x;

    {
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
        // stage 3: phi synthesis on the matrix cores (slsht_phi.h); row c * tb + t of the
        // tile is output row (omega_c, theta_{t0 + t})
        const T msign = (it.m & 1) ? T(-1) : T(1);
        const int64_t lm_stride = (int64_t)a.n_omega * a.n_theta_out * a.n_phi;
        V* gl = reinterpret_cast<V*>(a.g) + (int64_t)it.lm * lm_stride;
        V* gm = it.mirror >= 0 ? reinterpret_cast<V*>(a.g) + (int64_t)it.mirror * lm_stride : nullptr;
        const int n_theta = a.n_theta_out, n_phi = a.n_phi;
        phi_stage_mfma<T, LH>(PM_s, PMS, PW, a.n_omega * tb, L, reinterpret_cast<const V*>(a.twphi),
                              a.nslot, n_phi, [&](int rr, V*& out, V*& mout, T& ms) {
                                  const int c = rr / tb;
                                  const int t = rr - c * tb;
                                  const int64_t rowoff = ((int64_t)c * n_theta + (t0 + t)) * n_phi;
                                  out = gl + rowoff;
                                  mout = gm ? gm + rowoff : nullptr;
                                  ms = msign;
                              });
    }
}

// Round-robin dispatch sends block b to XCD b mod 8.  For the VALU phi form the blocks are
// renumbered so that each XCD runs one contiguous run of (item, theta tile) blocks:
// neighbouring tiles of an item, which share the output lines at their boundaries, then go
// through the same L2 (mid workload: 2.10 -> 1.97 ms FP64, 1.18 -> 1.04 ms FP32).  The MFMA
// form keeps dispatch order (the same renumbering cost it 7% at L_h = 16, L_f = 192).  The
// grid is a multiple of 8 blocks; those past the transform exit.
template <int LH>
__device__ __forceinline__ int xcd_block(int nblk_grid) {
    if constexpr (LH <= 8) {
        const int per = nblk_grid >> 3;
        return (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    } else {
        return (int)blockIdx.x;
    }
}

template <typename T, int LH, int NS>
__global__ void __launch_bounds__(256) synth_full_kernel(const SynthArgs a) {
    const int bid = xcd_block<LH>((int)gridDim.x);
    if (bid >= a.nblk) return;
    synth_block<T, LH, NS>(a, bid);
}

// Several transforms that share one kernel instance in one grid (a tile list across
// requests): transform r owns blocks [first[r], first[r+1]).  The per-transform arguments
// travel in the kernel-argument block, so a launch needs no device allocation or copy.
template <typename T, int LH, int NS>
__global__ void __launch_bounds__(256) synth_batch_kernel(const SynthBatch b) {
    const int bid = xcd_block<LH>((int)gridDim.x);
    if (bid >= b.first[b.n]) return;
    int r = 0;
    while (r + 1 < b.n && bid >= b.first[r + 1]) ++r;
    synth_block<T, LH, NS>(b.r[r], bid - b.first[r]);
}

static int lh_bucket(int L) { return L <= 4 ? 4 : (L <= 8 ? 8 : (L <= 16 ? 16 : (L <= 24 ? 24 : 32))); }

static size_t synth_xsize(const DevPlan& P, int tb) {
    const int LH = lh_bucket(P.d.L_h);
    const int PW = LH <= 8 ? LH : (P.d.L_h + 3) / 4 * 4;
    const size_t rows = ((size_t)tb * P.d.n_omega + 7) / 8 * 8;
    return std::max((size_t)2 * P.d.L_h * P.d.L_h, rows * (2 * PW + 1));
}

static size_t synth_lds_bytes(const DevPlan& P, int tb) {
    const int L = P.d.L_h, K = 2 * L - 1;
    const size_t v = P.d.precision == SLSHT_FP64 ? 16 : 8;
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

static const void* synth_fn(const DevPlan& P, bool batch = false) {
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

// Plans on the W/U path (L_h > 16, slsht_staged.hip) run their own launches (W table, A
// fragments, the W/U kernel), so each one gets a key of its own and is never grouped with
// other transforms.
const void* synthesis_kernel_key(const DevPlan& P) { return P.staged ? (const void*)&P : synth_fn(P); }

// Theta rows per block: stages 1-2 run between barriers with no stores in flight, so
// the store stream is kept busy by other resident blocks.  The tile is the largest one
// (at most 8 rows) among those that reach the highest resident block count the kernel's
// registers and the LDS allow.
bool choose_synthesis_shape(DevPlan& P, size_t lds_limit) {
    if (P.staged) {                       // the W/U kernel's shape is fixed by its geometry
        P.block = P.sg.threads;
        P.tb = 1;
        P.lds_bytes = P.sg.lds;
        return P.lds_bytes <= lds_limit;
    }
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
    a.nblk = (int)std::min<int64_t>((int64_t)P.n_items * a.n_tiles, 0x7fffffff);
    return a;
}

hipError_t launch_synthesis(const DevPlan& P, const double2* A, const double2* h, void* g,
                            hipStream_t s) {
    if (P.staged) return launch_synthesis_staged(P, A, h, g, s);
    SynthArgs a = synth_args(P, A, h, g);
    const int64_t nblk = (int64_t)P.n_items * a.n_tiles;
    const int64_t grid = (nblk + 7) / 8 * 8;                         // 8 XCDs
    if (grid > 0x7fffffff) return hipErrorInvalidConfiguration;   // grid.x limit
    a.nblk = (int)nblk;
    void* args[] = {&a};
    return hipLaunchKernel(synth_fn(P), dim3((unsigned)grid), dim3(P.block), args, P.lds_bytes, s);
}

hipError_t launch_synthesis_batch(const DevPlan* const* P, const double2* const* A,
                                  const double2* const* h, void* const* g, int n, hipStream_t s) {
    if (n < 1 || n > kSynthBatchMax) return hipErrorInvalidValue;
    if (P[0]->staged) {
        // W/U plans are grouped alone (their key is unique)
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
    const int64_t grid = (nblk + 7) / 8 * 8;                         // 8 XCDs
    if (grid > 0x7fffffff) return hipErrorInvalidConfiguration;
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    void* args[] = {&b};
    return hipLaunchKernel(fn, dim3((unsigned)grid), dim3(P[0]->block), args, lds, s);
}

}  // namespace slsht
