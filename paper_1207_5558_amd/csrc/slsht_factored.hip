// The paper's own route for the distribution on its minimal grid E_{L_h}
// (n_phi = n_omega = K = 2 L_h - 1, n_theta = L_h): factoring of rotations
// (Section IV-B).  With Delta^p = d^p(pi/2) and
//   d^p_{q,q'}(beta) = i^{q-q'} sum_{q''} Delta^p_{q'',q} Delta^p_{q'',q'} e^{-i q'' beta}
// (eq. Eq:WignerD_expansion_new), the separated form becomes a 3-D Fourier sum
//   g(alpha_a, beta_b, gamma_c; l, m) = sum_{q, q'', q'} C_{q,q'',q'}(l, m) e^{-i (q alpha_a + q'' beta_b + q' gamma_c)},
//   C_{q,q'',q'}(l, m) = i^{q-q'} sum_{p >= max(|q|,|q''|,|q'|)} A^p_q(l, m) h_p^{q'} Delta^p_{q'',q} Delta^p_{q'',q'},
// evaluated here in FP64 as four plain passes over a per-(l, m) workspace: C, then the
// gamma, beta (b < L_h only) and alpha sums, one thread per output value.  It is the
// paper's CPU-era design kept as a second route: the separated-form kernel K3 computes
// the same g on this grid (and on any other) with less work.
#include "slsht_device.h"

#include <hip/hip_runtime.h>

namespace slsht {

namespace {

// e^{-i k 2 pi j / K} for integer k, j: exact phase reduction, then one sincospi.
__device__ __forceinline__ double2 phase(int k, int j, int K) {
    int r = (int)(((int64_t)k * j) % K);
    if (r < 0) r += K;
    double s, c;
    sincospi(2.0 * (double)r / (double)K, &s, &c);
    return make_double2(c, -s);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

}  // namespace

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

// C[lm][q][q''][q'] (indices shifted by L-1); one thread per (q, q'', q'), block per lm.
__global__ void factored_c_kernel(const double2* __restrict__ A, const double2* __restrict__ h,
                                  const double* __restrict__ delta, int L, double2* __restrict__ C) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int K = 2 * L - 1, KKK = K * K * K;
    double2* A_s = reinterpret_cast<double2*>(smem_raw);
    double2* h_s = A_s + L * L;
    double* D_s = reinterpret_cast<double*>(h_s + L * L);
    const int lm = blockIdx.x;
    for (int i = threadIdx.x; i < L * L; i += blockDim.x) {
        A_s[i] = A[(int64_t)lm * L * L + i];
        h_s[i] = h[i];
    }
    for (int i = threadIdx.x; i < (int)dtab_row_len(L); i += blockDim.x) D_s[i] = delta[i];
    __syncthreads();
    double2* out = C + (int64_t)lm * KKK;
    for (int idx = threadIdx.x; idx < KKK; idx += blockDim.x) {
        const int q = idx / (K * K) - (L - 1);
        const int rem = idx % (K * K);
        const int q2 = rem / K - (L - 1), qp = rem % K - (L - 1);
        const int aq = q < 0 ? -q : q, a2 = q2 < 0 ? -q2 : q2, ap = qp < 0 ? -qp : qp;
        int p0 = aq > a2 ? aq : a2;
        p0 = p0 > ap ? p0 : ap;
        // canonical positions of Delta^p_{q'',q} and Delta^p_{q'',q'}
        int Q1, Q1p, Q2, Q2p;
        bool n1, n2;
        d_canonical(q2, q, Q1, Q1p, n1);
        d_canonical(q2, qp, Q2, Q2p, n2);
        double sr = 0.0, si = 0.0;
        for (int p = p0; p < L; ++p) {
            const double d1 = D_s[dtab_off(p) + Q1 * Q1 + Q1 + Q1p];
            const double d2 = D_s[dtab_off(p) + Q2 * Q2 + Q2 + Q2p];
            const double2 a = A_s[p * p + p + q], hv = h_s[p * p + p + qp];
            const double w = d1 * d2;
            sr += (a.x * hv.x - a.y * hv.y) * w;
            si += (a.x * hv.y + a.y * hv.x) * w;
        }
        if (n1 != n2) { sr = -sr; si = -si; }
        // times i^{q - q'}
        const int e = ((q - qp) % 4 + 4) % 4;
        double2 v = make_double2(sr, si);
        if (e == 1) v = make_double2(-si, sr);
        else if (e == 2) v = make_double2(-sr, -si);
        else if (e == 3) v = make_double2(si, -sr);
        out[idx] = v;
    }
}

// gamma sum: T[lm][q][q''][c] = sum_{q'} C[lm][q][q''][q'] e^{-i q' gamma_c}
__global__ void factored_gamma_kernel(const double2* __restrict__ C, int L, double2* __restrict__ T) {
    const int K = 2 * L - 1;
    const int64_t KKK = (int64_t)K * K * K;
    const int lm = blockIdx.y;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= KKK) return;
    const int row = idx / K, c = idx % K;
    const double2* in = C + lm * KKK + (int64_t)row * K;
    double2 acc = make_double2(0.0, 0.0);
    for (int j = 0; j < K; ++j) {
        const double2 t = cmul(in[j], phase(j - (L - 1), c, K));
        acc.x += t.x;
        acc.y += t.y;
    }
    T[lm * KKK + idx] = acc;
}

// beta sum, b < L: U[lm][q][b][c] = sum_{q''} T[lm][q][q''][c] e^{-i q'' beta_b}
__global__ void factored_beta_kernel(const double2* __restrict__ T, int L, double2* __restrict__ U) {
    const int K = 2 * L - 1;
    const int64_t KKK = (int64_t)K * K * K, KLK = (int64_t)K * L * K;
    const int lm = blockIdx.y;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= KLK) return;
    const int q = idx / (L * K), rem = idx % (L * K);
    const int b = rem / K, c = rem % K;
    const double2* in = T + lm * KKK + (int64_t)q * K * K + c;
    double2 acc = make_double2(0.0, 0.0);
    for (int j = 0; j < K; ++j) {
        const double2 t = cmul(in[(int64_t)j * K], phase(j - (L - 1), b, K));
        acc.x += t.x;
        acc.y += t.y;
    }
    U[lm * KLK + idx] = acc;
}

// alpha sum into the FULL layout: g[lm][c][b][a] = sum_q U[lm][q][b][c] e^{-i q alpha_a}
__global__ void factored_alpha_kernel(const double2* __restrict__ U, int L, double2* __restrict__ g) {
    const int K = 2 * L - 1;
    const int64_t KLK = (int64_t)K * L * K;
    const int lm = blockIdx.y;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= KLK) return;
    const int c = idx / (L * K), rem = idx % (L * K);
    const int b = rem / K, a = rem % K;
    const double2* in = U + lm * KLK + (int64_t)b * K + c;
    double2 acc = make_double2(0.0, 0.0);
    for (int j = 0; j < K; ++j) {
        const double2 t = cmul(in[(int64_t)j * L * K], phase(j - (L - 1), a, K));
        acc.x += t.x;
        acc.y += t.y;
    }
    g[lm * KLK + idx] = acc;
}

size_t factored_workspace_bytes(const slsht_desc& d) {
    const int64_t K = 2 * d.L_h - 1;
    const int64_t n_lm = (int64_t)d.l_hi * d.l_hi - (int64_t)d.l_lo * d.l_lo;
    const size_t delta = ((size_t)dtab_row_len(d.L_h) * sizeof(double) + 255) / 256 * 256;
    return delta + (size_t)2 * n_lm * K * K * K * sizeof(double2);
}

hipError_t launch_factored(const DevPlan& P, const double2* A, const double2* h, double2* g,
                           void* work, hipStream_t s) {
    const int L = P.d.L_h, K = 2 * L - 1;
    const int64_t n_lm = P.n_lm;
    double* delta = static_cast<double*>(work);
    const size_t dbytes = ((size_t)dtab_row_len(L) * sizeof(double) + 255) / 256 * 256;
    double2* C = reinterpret_cast<double2*>(static_cast<char*>(work) + dbytes);
    double2* T = C + n_lm * K * K * K;
    hipError_t e = launch_delta_trapani(L, delta, s);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)2 * L * L * sizeof(double2) + (size_t)dtab_row_len(L) * sizeof(double);
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)factored_c_kernel,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(factored_c_kernel, dim3((unsigned)n_lm), dim3(256), lds, s, A, h, delta, L, C);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t KKK = (int64_t)K * K * K, KLK = (int64_t)K * L * K;
    hipLaunchKernelGGL(factored_gamma_kernel, dim3((unsigned)((KKK + 255) / 256), (unsigned)n_lm),
                       dim3(256), 0, s, C, L, T);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(factored_beta_kernel, dim3((unsigned)((KLK + 255) / 256), (unsigned)n_lm),
                       dim3(256), 0, s, T, L, C);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(factored_alpha_kernel, dim3((unsigned)((KLK + 255) / 256), (unsigned)n_lm),
                       dim3(256), 0, s, C, L, g);
    return hipGetLastError();
}

}  // namespace slsht
