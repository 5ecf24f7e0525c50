// Coupling through the spherical harmonic transform of the modulated signal
// (Appendix A, eq. Eq:sht_sep_variable): the paper's own way to obtain
//   A^p_q(l, m) = conj((conj(f) Y_l^m)_p^q) = int f conj(Y_l^m) Y_p^q ds.
// With Y_l^m(theta, phi) = lam_l^m(theta) e^{i m phi} the phi integral separates:
//   int_0^{2 pi} f(theta, phi) e^{-i (m-q) phi} dphi = 2 pi F_{m-q}(theta),
//   F_mu(theta) = sum_{l' >= |mu|} f_{l'}^mu lam_{l'}^mu(theta)
// (the conjugate of the paper's I(theta, m-q)), and the theta integral is a quadrature
//   A^p_q(l, m) = 2 pi sum_j w_j lam_l^m(theta_j) lam_p^q(theta_j) F_{m-q}(theta_j).
// The paper samples f on an equiangular grid and uses that grid's exact weights; here
// the nodes are Gauss-Legendre in cos(theta), also exact: after the phi integral the
// integrand is a polynomial in cos(theta) of degree <= (L_f-1) + (l_hi-1) + (L_h-1), so
// n_theta = that degree / 2 + 1 nodes suffice.  Since f arrives as coefficients, F is
// synthesised from them directly (O(L_f^3) over all nodes) rather than by sampling f
// and transforming back.  Four FP64 passes over a caller-provided workspace: nodes and
// weights, F, the normalised Legendre values of the l-window and of p < L_h, then one
// block per (l, m) contracting over the nodes (O(n_lm L_h^2 L_f), the paper's
// O(L_f^3 L_h^2)).
#include "slsht_device.h"

#include <hip/hip_runtime.h>

namespace slsht {

namespace {

constexpr double kTwoPi = 6.28318530717958647692;

// lam_l^m(x) for l = m, m+1, ... at fixed m and x by the three-term recursion in l
// from the sectoral value lam_m^m = (-1)^m sqrt((2m+1)!! / (4 pi (2m)!!)) sin^m theta.
// The running values are kept as cur = lam * 2^E: the sectoral value underflows for
// large m near the poles, and the recursion must still grow it back to full size at
// higher l, so it is rescaled by 2^600 while small and the scale removed as it grows.
struct LegendreRun {
    double x = 0.0, prev = 0.0, cur = 0.0;
    int l = 0, m = 0, E = 0;

    __device__ void start(int m_, double x_) {
        m = m_;
        l = m_;
        x = x_;
        const double sx = sqrt(fmax(0.0, 1.0 - x * x));
        double v = 0.28209479177387814347;   // 1 / sqrt(4 pi)
        E = 0;
        for (int k = 1; k <= m; ++k) {
            v *= -sqrt((2.0 * k + 1.0) / (2.0 * k)) * sx;
            if (v != 0.0 && fabs(v) < 0x1p-600) {
                v *= 0x1p600;
                E += 600;
            }
        }
        prev = 0.0;
        cur = v;
    }
    __device__ double value() const { return E == 0 ? cur : ldexp(cur, -E); }
    // advance to l + 1
    __device__ void step() {
        const double dl = l + 1, dm = m;
        double nxt;
        if (l == m) {
            nxt = sqrt(2.0 * dm + 3.0) * x * cur;
        } else {
            const double a = sqrt((4.0 * dl * dl - 1.0) / (dl * dl - dm * dm));
            const double b = sqrt(((dl - 1.0) * (dl - 1.0) - dm * dm) / (4.0 * (dl - 1.0) * (dl - 1.0) - 1.0));
            nxt = a * (x * cur - b * prev);
        }
        prev = cur;
        cur = nxt;
        ++l;
        if (E > 0 && fabs(cur) > 0x1p600) {
            cur *= 0x1p-600;
            prev *= 0x1p-600;
            E -= 600;
        }
    }
};

}  // namespace

// Gauss-Legendre nodes x_j (descending, so theta ascends) and weights w_j on [-1, 1]:
// Newton's method on P_n from the asymptotic guess, one thread per node.
__global__ void gl_nodes_kernel(int n, double* __restrict__ x, double* __restrict__ w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double z = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        const double dz = p1 / dp;
        z -= dz;
        if (fabs(dz) <= 1e-16 * fabs(z) + 1e-300) break;
    }
    // one more evaluation of P_n' at the converged node for the weight
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
}

// F[j][mu + L_f - 1] = sum_{l'=|mu|}^{L_f-1} f_{l'}^mu lam_{l'}^mu(theta_j); one thread per
// (node, |mu|) computes both signs (lam^{-mu} = (-1)^mu lam^mu).
__global__ void modsht_fsynth_kernel(const double2* __restrict__ f, int L_f,
                                     const double* __restrict__ x, int n_nodes,
                                     double2* __restrict__ F) {
    const int mu = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (mu >= L_f || j >= n_nodes) return;
    LegendreRun r;
    r.start(mu, x[j]);
    double2 fp = make_double2(0.0, 0.0), fm = make_double2(0.0, 0.0);
    for (int l = mu; l < L_f; ++l) {
        if (l > mu) r.step();
        const double v = r.value();
        const double2 cp = f[l * l + l + mu], cm = f[l * l + l - mu];
        fp.x += cp.x * v;
        fp.y += cp.y * v;
        fm.x += cm.x * v;
        fm.y += cm.y * v;
    }
    const double sg = (mu & 1) ? -1.0 : 1.0;
    double2* row = F + (int64_t)j * (2 * L_f - 1) + (L_f - 1);
    row[mu] = fp;
    if (mu > 0) row[-mu] = make_double2(sg * fm.x, sg * fm.y);
}

// lam[j][(l(l+1) - lo(lo+1))/2 + m] = lam_l^m(theta_j) for lo <= l < hi, 0 <= m <= l; one
// thread per (node, m).  The threads of a block walk the same l at each step (those with
// m > l idle), so the stores of one l are contiguous.
__global__ void modsht_legendre_kernel(const double* __restrict__ x, int n_nodes, int lo, int hi,
                                       double* __restrict__ lam) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (j >= n_nodes) return;
    const int64_t row = (int64_t)hi * (hi + 1) / 2 - (int64_t)lo * (lo + 1) / 2;
    double* out = lam + (int64_t)j * row - (int64_t)lo * (lo + 1) / 2;
    const double xj = x[j];
    LegendreRun r;
    for (int l = blockIdx.x * blockDim.x; l < hi; ++l) {
        if (l < m) continue;
        if (l == m) r.start(m, xj);
        else r.step();
        if (l >= lo) out[(int64_t)l * (l + 1) / 2 + m] = r.value();
    }
}

struct ModArgs {
    const double* w;        // [n] quadrature weights
    const double2* F;       // [n][2 L_f - 1]
    const double* lamW;     // [n][nW] window degrees
    const double* lamP;     // [n][L_h (L_h+1)/2] window band p < L_h
    double2* A;             // [n_lm][L_h^2]
    int n, L_f, L_h, l_lo, nW;
};

// A[lm][p^2+p+q] = 2 pi sum_j w_j lam_l^m(theta_j) lam_p^q(theta_j) F_{m-q}(theta_j); one
// block per (l, m), one thread per (p, q); the (l, m) factor of each node is staged in LDS.
__global__ void modsht_coupling_kernel(const ModArgs a) {
    extern __shared__ double Wj[];
    const int64_t lm = blockIdx.x;
    const int64_t flat = lm + (int64_t)a.l_lo * a.l_lo;
    int l = (int)sqrt((double)flat);
    while ((int64_t)l * l > flat) --l;
    while ((int64_t)(l + 1) * (l + 1) <= flat) ++l;
    const int m = (int)(flat - (int64_t)l * l - l);
    const int am = m < 0 ? -m : m;
    const double sm = (m < 0 && (am & 1)) ? -kTwoPi : kTwoPi;
    const int64_t wofs = (int64_t)l * (l + 1) / 2 - (int64_t)a.l_lo * (a.l_lo + 1) / 2 + am;
    for (int j = threadIdx.x; j < a.n; j += blockDim.x)
        Wj[j] = sm * a.w[j] * a.lamW[(int64_t)j * a.nW + wofs];
    __syncthreads();
    const int LL = a.L_h * a.L_h;
    const int nP = a.L_h * (a.L_h + 1) / 2;
    const int KF = 2 * a.L_f - 1;
    for (int t = threadIdx.x; t < LL; t += blockDim.x) {
        int p = (int)sqrt((double)t);
        while (p * p > t) --p;
        while ((p + 1) * (p + 1) <= t) ++p;
        const int q = t - p * p - p, aq = q < 0 ? -q : q;
        const int mu = m - q;
        double sr = 0.0, si = 0.0;
        if (mu > -a.L_f && mu < a.L_f) {
            const double* lp = a.lamP + p * (p + 1) / 2 + aq;
            const double2* Fm = a.F + (mu + a.L_f - 1);
            for (int j = 0; j < a.n; ++j) {
                const double c = Wj[j] * lp[(int64_t)j * nP];
                const double2 v = Fm[(int64_t)j * KF];
                sr += c * v.x;
                si += c * v.y;
            }
            if (q < 0 && (aq & 1)) {
                sr = -sr;
                si = -si;
            }
        }
        a.A[lm * LL + t] = make_double2(sr, si);
    }
}

namespace {

struct ModLayout {
    int n = 0, nW = 0, nP = 0;
    size_t off_x = 0, off_w = 0, off_F = 0, off_lamW = 0, off_lamP = 0, bytes = 0;
};

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

ModLayout mod_layout(const slsht_desc& d) {
    ModLayout Lo;
    const int deg = (d.L_f - 1) + (d.l_hi - 1) + (d.L_h - 1);
    Lo.n = deg / 2 + 1;
    Lo.nW = (int)((int64_t)d.l_hi * (d.l_hi + 1) / 2 - (int64_t)d.l_lo * (d.l_lo + 1) / 2);
    Lo.nP = d.L_h * (d.L_h + 1) / 2;
    size_t o = 0;
    Lo.off_x = o;    o += up256((size_t)Lo.n * sizeof(double));
    Lo.off_w = o;    o += up256((size_t)Lo.n * sizeof(double));
    Lo.off_F = o;    o += up256((size_t)Lo.n * (2 * d.L_f - 1) * sizeof(double2));
    Lo.off_lamW = o; o += up256((size_t)Lo.n * Lo.nW * sizeof(double));
    Lo.off_lamP = o; o += up256((size_t)Lo.n * Lo.nP * sizeof(double));
    Lo.bytes = o;
    return Lo;
}

}  // namespace

size_t modulated_workspace_bytes(const slsht_desc& d) { return mod_layout(d).bytes; }

hipError_t launch_coupling_modulated(const DevPlan& P, const double2* f, double2* A, void* work,
                                     hipStream_t s) {
    const slsht_desc& d = P.d;
    const ModLayout Lo = mod_layout(d);
    char* base = static_cast<char*>(work);
    double* x = reinterpret_cast<double*>(base + Lo.off_x);
    double* w = reinterpret_cast<double*>(base + Lo.off_w);
    double2* F = reinterpret_cast<double2*>(base + Lo.off_F);
    double* lamW = reinterpret_cast<double*>(base + Lo.off_lamW);
    double* lamP = reinterpret_cast<double*>(base + Lo.off_lamP);
    hipError_t e;
    hipLaunchKernelGGL(gl_nodes_kernel, dim3((Lo.n + 63) / 64), dim3(64), 0, s, Lo.n, x, w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(modsht_fsynth_kernel, dim3((d.L_f + 63) / 64, Lo.n), dim3(64), 0, s, f,
                       d.L_f, x, Lo.n, F);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(modsht_legendre_kernel, dim3((d.l_hi + 63) / 64, Lo.n), dim3(64), 0, s, x,
                       Lo.n, d.l_lo, d.l_hi, lamW);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(modsht_legendre_kernel, dim3((d.L_h + 63) / 64, Lo.n), dim3(64), 0, s, x,
                       Lo.n, 0, d.L_h, lamP);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    ModArgs a{w, F, lamW, lamP, A, Lo.n, d.L_f, d.L_h, d.l_lo, Lo.nW};
    const int LL = d.L_h * d.L_h;
    const int threads = LL <= 64 ? 64 : (LL <= 256 ? 256 : 512);
    hipLaunchKernelGGL(modsht_coupling_kernel, dim3((unsigned)P.n_lm), dim3(threads),
                       (size_t)Lo.n * sizeof(double), s, a);
    return hipGetLastError();
}

}  // namespace slsht
