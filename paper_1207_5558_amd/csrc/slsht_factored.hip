// The paper's own route for the distribution on its minimal grid E_{L_h}
// (n_phi = n_omega = K = 2 L_h - 1, n_theta = L_h): factoring of rotations
// (Section IV-B).  With Delta^p = d^p(pi/2) and
//   d^p_{q,q'}(beta) = i^{q-q'} sum_{q''} Delta^p_{q'',q} Delta^p_{q'',q'} e^{-i q'' beta}
// (eq. Eq:WignerD_expansion_new), the separated form becomes a 3-D Fourier sum
//   g(alpha_a, beta_b, gamma_c; l, m) = sum_{q, q'', q'} C_{q,q'',q'}(l, m) e^{-i (q alpha_a + q'' beta_b + q' gamma_c)},
//   C_{q,q'',q'}(l, m) = i^{q-q'} sum_{p >= max(|q|,|q''|,|q'|)} A^p_q(l, m) h_p^{q'} Delta^p_{q'',q} Delta^p_{q'',q'}.
// FP64, in three launches after Delta:
//   * HD[p][q''][q'] = i^{-q'} h_p^{q'} Delta^p_{q'',q'}, the window's half of C (once per call);
//   * one block per (l, m), looping over q: the slice C_q[q''][q'] =
//     sum_p (i^q A^p_q Delta^p_{q'',q}) HD[p][q''][q'] in LDS, its gamma sum over q', then its
//     beta sum over q'' for b < L_h, written as U[lm][q][b][c];
//   * one block per (l, m, b): the alpha sum over q into g's FULL layout.
// Each 1-D sum over k in (-L_h, L_h) with K outputs is folded: with
// S_k^{+-} = X_k +- X_{-k}, sum_k X_k e^{-i k 2 pi j / K} = X_0 + sum_{k>0} S_k^+ cos(k 2 pi j/K)
// - i sum_{k>0} S_k^- sin(k 2 pi j/K), and outputs j and K - j differ only in the sign of
// the sine part; cos/sin come from a K-entry table at index k j mod K.  C is O(L_h^4)
// per (l, m), as the paper states; the sums are direct, not FFTs (K <= 63).
#include "slsht_device.h"

#include <hip/hip_runtime.h>

namespace slsht {

// Delta^p_{Q,Q'} = d^p_{Q,Q'}(pi/2) in the canonical layout (0 <= Q <= p, |Q'| <= Q), by
// the recursion of Trapani and Navaza that the paper uses (Section IV-B): one thread per
// column (p, Q'), seeded on the edge Q = p by
//   Delta^p_{p,Q'} = (-1)^{p-Q'} 2^{-p} sqrt(C(2p, p+Q'))
// (Wigner's formula at beta = pi/2, where only one term survives), then down the column
// by the first-index three-term relation of d at beta = pi/2,
//   sqrt((p+Q)(p-Q+1)) Delta_{Q-1,Q'} = 2 Q' Delta_{Q,Q'} - sqrt((p-Q)(p+Q+1)) Delta_{Q+1,Q'},
// down to Q = |Q'|.  O(p) work per column, O(L^3) in all.
__global__ void delta_trapani_kernel(int L, double* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= L * L) return;
    int p = (int)sqrt((double)t);
    while (p * p > t) --p;
    while ((p + 1) * (p + 1) <= t) ++p;
    const int qp = t - p * p - p, aqp = qp < 0 ? -qp : qp;
    // C(2p, p - |Q'|) by the multiplicative formula; every partial product is the
    // integer C(p + |Q'| + i, i), exact while below 2^53
    const int k = p - aqp;
    double c = 1.0;
    for (int i = 1; i <= k; ++i) c = c * (double)(p + aqp + i) / (double)i;
    double cur = ldexp(sqrt(c), -p);
    if ((p - qp) & 1) cur = -cur;
    double up = 0.0;   // Delta_{Q+1,Q'}
    double* row = out + dtab_off(p);
    row[p * p + p + qp] = cur;
    for (int Q = p; Q > aqp; --Q) {
        const double nxt = (2.0 * qp * cur - sqrt((double)(p - Q) * (p + Q + 1)) * up) /
                           sqrt((double)(p + Q) * (p - Q + 1));
        up = cur;
        cur = nxt;
        row[(Q - 1) * (Q - 1) + (Q - 1) + qp] = cur;
    }
}

hipError_t launch_delta_trapani(int L, double* out, hipStream_t s) {
    hipLaunchKernelGGL(delta_trapani_kernel, dim3((L * L + 127) / 128), dim3(128), 0, s, L, out);
    return hipGetLastError();
}

// HD[p][q''+L-1][q'+L-1] = i^{-q'} h_p^{q'} Delta^p_{q'',q'} for p >= max(|q''|,|q'|), else 0.
__global__ void factored_hd_kernel(const double2* __restrict__ h, const double* __restrict__ delta,
                                   int L, double2* __restrict__ HD) {
    const int K = 2 * L - 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= L * K * K) return;
    const int p = idx / (K * K), rem = idx - p * K * K;
    const int q2 = rem / K - (L - 1), q1 = rem % K - (L - 1);
    const int a2 = q2 < 0 ? -q2 : q2, a1 = q1 < 0 ? -q1 : q1;
    double2 v = make_double2(0.0, 0.0);
    if (p >= a2 && p >= a1) {
        int Q, Qp;
        bool neg;
        d_canonical(q2, q1, Q, Qp, neg);
        double d = delta[dtab_off(p) + Q * Q + Q + Qp];
        if (neg) d = -d;
        const double2 hv = h[p * p + p + q1];
        const double2 t = make_double2(hv.x * d, hv.y * d);
        // times i^{-q'}
        const int e = ((-q1) % 4 + 4) % 4;
        v = e == 0 ? t : e == 1 ? make_double2(-t.y, t.x) : e == 2 ? make_double2(-t.x, -t.y)
                                                               : make_double2(t.y, -t.x);
    }
    HD[idx] = v;
}

namespace {

// X_0 + sum_{k=1}^{L-1} (X_k + X_{-k}) cos(2 pi k j / K) and sum_k (X_k - X_{-k}) sin(...),
// X_k at x[k * stride] (x centred on k = 0).
__device__ __forceinline__ void folded_sum(const double2* x, int stride, int L, int K, int j,
                                           const double2* __restrict__ tw, double2& P, double2& S) {
    P = x[0];
    S = make_double2(0.0, 0.0);
    int r = 0;
    for (int k = 1; k < L; ++k) {
        r += j;
        if (r >= K) r -= K;
        const double2 a = x[k * stride], b = x[-k * stride];
        const double2 cs = tw[r];
        P.x = fma(a.x + b.x, cs.x, P.x);
        P.y = fma(a.y + b.y, cs.x, P.y);
        S.x = fma(a.x - b.x, cs.y, S.x);
        S.y = fma(a.y - b.y, cs.y, S.y);
    }
}

}  // namespace

// U[lm][q+L-1][b][c] = sum_{q''} e^{-i q'' beta_b} sum_{q'} C_{q,q'',q'} e^{-i q' gamma_c}, b < L.
__global__ void __launch_bounds__(256) factored_slab_kernel(const double2* __restrict__ A,
                                                           const double2* __restrict__ HD,
                                                           const double* __restrict__ delta, int L,
                                                           double2* __restrict__ U) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int K = 2 * L - 1, KK = K * K;
    double2* AD = reinterpret_cast<double2*>(smem_raw);      // [L][K]
    double2* C_s = AD + L * K;                               // [K][K]  (q'', q')
    double2* T_s = C_s + KK;                                 // [K][K]  (q'', c)
    double2* tw = T_s + KK;                                  // [K] (cos, sin)(2 pi r / K)
    const int64_t lm = blockIdx.x;
    const int tid = threadIdx.x, nth = blockDim.x;
    const double2* Alm = A + lm * L * L;
    for (int r = tid; r < K; r += nth) {
        double sn, cs;
        sincospi(2.0 * (double)r / (double)K, &sn, &cs);
        tw[r] = make_double2(cs, sn);
    }
    __syncthreads();
    double2* Ulm = U + lm * (int64_t)K * L * K;
    for (int q = -(L - 1); q < L; ++q) {
        const int aq = q < 0 ? -q : q;
        // AD[p][q''] = i^q A^p_q Delta^p_{q'',q}
        for (int i = tid; i < L * K; i += nth) {
            const int p = i / K, q2 = i - p * K - (L - 1);
            const int a2 = q2 < 0 ? -q2 : q2;
            double2 v = make_double2(0.0, 0.0);
            if (p >= aq && p >= a2) {
                int Q, Qp;
                bool neg;
                d_canonical(q2, q, Q, Qp, neg);
                double d = delta[dtab_off(p) + Q * Q + Q + Qp];
                if (neg) d = -d;
                const double2 a = Alm[p * p + p + q];
                const double2 t = make_double2(a.x * d, a.y * d);
                const int e = ((q % 4) + 4) % 4;
                v = e == 0 ? t : e == 1 ? make_double2(-t.y, t.x) : e == 2 ? make_double2(-t.x, -t.y)
                                                                       : make_double2(t.y, -t.x);
            }
            AD[i] = v;
        }
        __syncthreads();
        // C_q[q''][q'] = sum_{p >= max(|q|, |q''|, |q'|)} AD[p][q''] HD[p][q''][q']
        for (int i = tid; i < KK; i += nth) {
            const int q2 = i / K - (L - 1), q1 = i % K - (L - 1);
            const int a2 = q2 < 0 ? -q2 : q2, a1 = q1 < 0 ? -q1 : q1;
            int p0 = aq > a2 ? aq : a2;
            p0 = p0 > a1 ? p0 : a1;
            double sr = 0.0, si = 0.0;
            const double2* hd = HD + i;
            const double2* ad = AD + (q2 + L - 1);
            for (int p = p0; p < L; ++p) {
                const double2 x = ad[p * K], y = hd[(int64_t)p * KK];
                sr = fma(x.x, y.x, fma(-x.y, y.y, sr));
                si = fma(x.x, y.y, fma(x.y, y.x, si));
            }
            C_s[i] = make_double2(sr, si);
        }
        __syncthreads();
        // gamma: T[q''][c] = sum_{q'} C_q[q''][q'] e^{-i q' gamma_c}
        for (int i = tid; i < K * L; i += nth) {
            const int r2 = i / L, j = i - r2 * L;
            double2 P, S;
            folded_sum(C_s + r2 * K + (L - 1), 1, L, K, j, tw, P, S);
            // P - i S and, for K - j, P + i S
            T_s[r2 * K + j] = make_double2(P.x + S.y, P.y - S.x);
            if (j > 0) T_s[r2 * K + (K - j)] = make_double2(P.x - S.y, P.y + S.x);
        }
        __syncthreads();
        // beta, b < L: U[q][b][c] = sum_{q''} T[q''][c] e^{-i q'' beta_b}
        double2* Uq = Ulm + (int64_t)(q + L - 1) * L * K;
        for (int i = tid; i < L * K; i += nth) {
            const int b = i / K, c = i - b * K;
            double2 P, S;
            folded_sum(T_s + (L - 1) * K + c, K, L, K, b, tw, P, S);
            Uq[i] = make_double2(P.x + S.y, P.y - S.x);
        }
        // the next q writes AD (read before the second barrier above) and C_s, T_s (read
        // before the barriers that follow the next AD stage), so no barrier is needed here
    }
}

// g[lm][c][b][a] = sum_q U[lm][q][b][c] e^{-i q alpha_a}; one block per (lm, b).
__global__ void __launch_bounds__(256) factored_alpha_kernel(const double2* __restrict__ U, int L,
                                                            double2* __restrict__ g) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int K = 2 * L - 1;
    double2* U_s = reinterpret_cast<double2*>(smem_raw);     // [K][K] (q, c)
    double2* tw = U_s + K * K;
    const int64_t blk = blockIdx.x;
    const int64_t lm = blk / L;
    const int b = (int)(blk - lm * L);
    const int tid = threadIdx.x, nth = blockDim.x;
    const double2* Ulm = U + lm * (int64_t)K * L * K;
    for (int i = tid; i < K * K; i += nth) {
        const int q = i / K, c = i - q * K;
        U_s[i] = Ulm[((int64_t)q * L + b) * K + c];
    }
    for (int r = tid; r < K; r += nth) {
        double sn, cs;
        sincospi(2.0 * (double)r / (double)K, &sn, &cs);
        tw[r] = make_double2(cs, sn);
    }
    __syncthreads();
    double2* glm = g + lm * (int64_t)K * L * K;
    for (int i = tid; i < K * L; i += nth) {
        const int c = i / L, j = i - c * L;
        double2 P, S;
        folded_sum(U_s + (L - 1) * K + c, K, L, K, j, tw, P, S);
        double2* row = glm + ((int64_t)c * L + b) * K;
        row[j] = make_double2(P.x + S.y, P.y - S.x);
        if (j > 0) row[K - j] = make_double2(P.x - S.y, P.y + S.x);
    }
}

namespace {
size_t up256(size_t b) { return (b + 255) / 256 * 256; }
}  // namespace

size_t factored_workspace_bytes(const slsht_desc& d) {
    const int64_t L = d.L_h, K = 2 * L - 1;
    const int64_t n_lm = (int64_t)d.l_hi * d.l_hi - (int64_t)d.l_lo * d.l_lo;
    return up256((size_t)dtab_row_len(d.L_h) * sizeof(double)) +
           up256((size_t)L * K * K * sizeof(double2)) + (size_t)n_lm * K * L * K * sizeof(double2);
}

hipError_t launch_factored(const DevPlan& P, const double2* A, const double2* h, double2* g,
                           void* work, hipStream_t s) {
    const int L = P.d.L_h, K = 2 * L - 1;
    const int64_t n_lm = P.n_lm;
    char* base = static_cast<char*>(work);
    double* delta = reinterpret_cast<double*>(base);
    const size_t dbytes = up256((size_t)dtab_row_len(L) * sizeof(double));
    double2* HD = reinterpret_cast<double2*>(base + dbytes);
    double2* U = reinterpret_cast<double2*>(base + dbytes + up256((size_t)L * K * K * sizeof(double2)));
    hipError_t e = launch_delta_trapani(L, delta, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(factored_hd_kernel, dim3((L * K * K + 255) / 256), dim3(256), 0, s, h, delta,
                       L, HD);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const size_t lds1 = (size_t)(L * K + 2 * K * K + K) * sizeof(double2);   // <= 160 KiB at L = 32
    if (lds1 > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)factored_slab_kernel,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds1);
    hipLaunchKernelGGL(factored_slab_kernel, dim3((unsigned)n_lm), dim3(256), lds1, s, A, HD, delta,
                       L, U);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const size_t lds2 = (size_t)(K * K + K) * sizeof(double2);
    if (lds2 > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)factored_alpha_kernel,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2);
    hipLaunchKernelGGL(factored_alpha_kernel, dim3((unsigned)(n_lm * L)), dim3(256), lds2, s, U, L, g);
    return hipGetLastError();
}

}  // namespace slsht
