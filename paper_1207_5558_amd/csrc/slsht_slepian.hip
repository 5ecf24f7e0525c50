// Slepian eigenfunction window on an elliptical region (Section III-D): the function
// band-limited to s < L_h with the largest energy concentration in
//   R_(theta_c, a) = {x : dist(x, F1) + dist(x, F2) <= 2a},  F1 = (theta_c, 0), F2 = (theta_c, pi)
// (eq. Eq:region_def).  The region is symmetric under phi -> -phi and phi -> pi - phi, so
// in the real harmonic basis X_s^r = c_r lam_s^r(theta) cos(r phi) (r >= 0) and
// Z_s^r = sqrt(2) lam_s^r(theta) sin(r phi) (r >= 1), c_0 = 1, c_r = sqrt(2), the
// concentration matrix splits into four real symmetric blocks: cos/sin class x parity
// of r.  Its entries
//   D = c_r c_r' sum_j w_j lam_s^r(theta_j) lam_s'^r'(theta_j) (J_{|r-r'|}(theta_j) +- J_{r+r'}(theta_j)) / 2,
// with J_k(theta) = int over the region's phi set at theta of cos(k phi), are summed on
// the GPU in FP64 (one thread per entry); the top eigenpair of each block is found on the
// host (Lanczos with complete reorthogonalisation, Sturm bisection and inverse iteration,
// eig_top.h), and the best of the four is the window.
//
// Quadrature in theta: [0, b] (cos b = cos a / cos theta_c) is the part where the whole
// circle lies in R, so J_k = 2 pi delta_k0 and the integrand is a polynomial in
// cos(theta) of degree <= 2 L_h - 2: Gauss-Legendre in cos(theta) with L_h + 8 nodes is
// exact.  On [b, a] the phi set is |phi| <= phi*, |phi - pi| <= phi*, with phi* ~ the
// square root of the distance to either end; theta = b + (a - b)(1 - cos(pi t))/2 makes
// the integrand smooth in t, and Gauss-Legendre in t converges spectrally.
#include "eig_top.h"
#include "slsht_device.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

namespace slsht {

// lam[j][s(s+1)/2 + r] = N_s^r P_s^r(x_j), r >= 0, Condon-Shortley phase; one thread
// per (node, r), three-term recursion in s from the sectoral value.
__global__ void slepian_legendre_kernel(const double* __restrict__ x, int n_nodes, int L,
                                        double* __restrict__ lam) {
    const int j = blockIdx.x;
    const int r = threadIdx.x;
    if (j >= n_nodes || r >= L) return;
    const int nl = L * (L + 1) / 2;
    const double xx = x[j], sx = sqrt(fmax(0.0, 1.0 - xx * xx));
    double* out = lam + (int64_t)j * nl;
    double v = 0.28209479177387814347;   // 1 / sqrt(4 pi)
    for (int m = 1; m <= r; ++m) v *= -sqrt((2.0 * m + 1.0) / (2.0 * m)) * sx;
    out[r * (r + 1) / 2 + r] = v;
    if (r + 1 >= L) return;
    double prev = v, cur = sqrt(2.0 * r + 3.0) * xx * v;
    out[(r + 1) * (r + 2) / 2 + r] = cur;
    for (int s = r + 2; s < L; ++s) {
        const double A = sqrt((4.0 * s * s - 1.0) / ((double)s * s - (double)r * r));
        const double B = sqrt((((double)s - 1) * (s - 1) - (double)r * r) / (4.0 * (s - 1.0) * (s - 1.0) - 1.0));
        const double nxt = A * (xx * cur - B * prev);
        out[s * (s + 1) / 2 + r] = nxt;
        prev = cur;
        cur = nxt;
    }
}

// One block of the concentration matrix: rows/columns are the (s, r) of that block
// (idx_s, idx_r), cls = +1 for the cos class, -1 for the sin class.
__global__ void slepian_matrix_kernel(const double* __restrict__ lam, const double* __restrict__ w,
                                      const double* __restrict__ J, int n_nodes, int L, int nk,
                                      const int* __restrict__ bs, const int* __restrict__ br,
                                      int nb, double cls, double* __restrict__ D) {
    const int i = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb || k >= nb || k < i) return;
    const int nl = L * (L + 1) / 2;
    const int s1 = bs[i], r1 = br[i], s2 = bs[k], r2 = br[k];
    const int o1 = s1 * (s1 + 1) / 2 + r1, o2 = s2 * (s2 + 1) / 2 + r2;
    const int km = r1 > r2 ? r1 - r2 : r2 - r1, kp = r1 + r2;
    double acc = 0.0;
    for (int j = 0; j < n_nodes; ++j) {
        const double* lj = lam + (int64_t)j * nl;
        const double* Jj = J + (int64_t)j * nk;
        acc += w[j] * lj[o1] * lj[o2] * (Jj[km] + cls * Jj[kp]);
    }
    const double c1 = r1 == 0 ? 1.0 : 1.41421356237309504880;
    const double c2 = r2 == 0 ? 1.0 : 1.41421356237309504880;
    const double v = 0.5 * c1 * c2 * acc;
    D[(int64_t)i * nb + k] = v;
    D[(int64_t)k * nb + i] = v;
}

namespace {

// Gauss-Legendre nodes/weights on [-1, 1] by Newton's method on P_n.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
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
            if (fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

double dist(double t1, double p1, double t2, double p2) {
    const double c = sin(t1) * sin(t2) * cos(p1 - p2) + cos(t1) * cos(t2);
    return acos(std::min(1.0, std::max(-1.0, c)));
}

// phi* in [0, pi/2]: the region's boundary at colatitude theta (distance sum = 2a).
double phi_half_width(double theta, double tc, double a) {
    auto f = [&](double p) { return dist(theta, p, tc, 0.0) + dist(theta, p, tc, M_PI) - 2.0 * a; };
    if (f(0.0) >= 0.0) return 0.0;
    if (f(0.5 * M_PI) <= 0.0) return 0.5 * M_PI;
    double lo = 0.0, hi = 0.5 * M_PI;
    for (int it = 0; it < 200 && hi - lo > 1e-17; ++it) {
        const double mid = 0.5 * (lo + hi);
        (f(mid) <= 0.0 ? lo : hi) = mid;
    }
    return 0.5 * (lo + hi);
}

}  // namespace

int slepian_window(int L, double tc, double a, double2* h_out, double* conc) {
    const double b = acos(cos(a) / cos(tc));
    // theta nodes: x = cos(theta), weight including sin(theta) dtheta
    std::vector<double> xg, wg, xs, ws, ph;
    const int n1 = L + 8;
    gauss_legendre(n1, xg, wg);
    for (int i = 0; i < n1; ++i) {
        xs.push_back(0.5 * (1.0 + cos(b)) + 0.5 * (1.0 - cos(b)) * xg[i]);
        ws.push_back(0.5 * (1.0 - cos(b)) * wg[i]);
        ph.push_back(-1.0);                       // whole circle
    }
    if (a > b) {
        const int n2 = 8 * L + 64;
        gauss_legendre(n2, xg, wg);
        for (int i = 0; i < n2; ++i) {
            const double t = 0.5 * (1.0 + xg[i]);
            const double th = b + 0.5 * (a - b) * (1.0 - cos(M_PI * t));
            const double dth = 0.5 * (a - b) * M_PI * sin(M_PI * t) * 0.5 * wg[i];
            xs.push_back(cos(th));
            ws.push_back(dth * sin(th));
            ph.push_back(phi_half_width(th, tc, a));
        }
    }
    const int nn = (int)xs.size(), nk = 2 * L - 1;
    std::vector<double> J((size_t)nn * nk, 0.0);
    for (int j = 0; j < nn; ++j)
        for (int k = 0; k < nk; ++k) {
            double v;
            if (ph[j] < 0.0) v = k == 0 ? 2.0 * M_PI : 0.0;
            else if (k == 0) v = 4.0 * ph[j];
            else v = (k % 2 == 0) ? 4.0 * sin(k * ph[j]) / k : 0.0;
            J[(size_t)j * nk + k] = v;
        }
    // the four blocks: (class, parity of r)
    struct Block { double cls; int par; std::vector<int> s, r; };
    Block blocks[4] = {{1.0, 0, {}, {}}, {1.0, 1, {}, {}}, {-1.0, 0, {}, {}}, {-1.0, 1, {}, {}}};
    for (Block& B : blocks)
        for (int s = 0; s < L; ++s)
            for (int r = (B.cls > 0 ? 0 : 1); r <= s; ++r)
                if ((r & 1) == B.par) { B.s.push_back(s); B.r.push_back(r); }
    size_t maxnb = 0;
    for (Block& B : blocks) maxnb = std::max(maxnb, B.s.size());

    const int nl = L * (L + 1) / 2;
    double *dx = nullptr, *dw = nullptr, *dJ = nullptr, *dlam = nullptr, *dD = nullptr;
    int *dbs = nullptr, *dbr = nullptr;
    hipError_t e = hipSuccess;
    auto ok = [&](hipError_t x) { if (e == hipSuccess) e = x; return e == hipSuccess; };
    ok(hipMalloc(&dx, nn * sizeof(double)));
    ok(hipMalloc(&dw, nn * sizeof(double)));
    ok(hipMalloc(&dJ, J.size() * sizeof(double)));
    ok(hipMalloc(&dlam, (size_t)nn * nl * sizeof(double)));
    ok(hipMalloc(&dD, maxnb * maxnb * sizeof(double)));
    ok(hipMalloc(&dbs, maxnb * sizeof(int)));
    ok(hipMalloc(&dbr, maxnb * sizeof(int)));
    ok(hipMemcpy(dx, xs.data(), nn * sizeof(double), hipMemcpyHostToDevice));
    ok(hipMemcpy(dw, ws.data(), nn * sizeof(double), hipMemcpyHostToDevice));
    ok(hipMemcpy(dJ, J.data(), J.size() * sizeof(double), hipMemcpyHostToDevice));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(slepian_legendre_kernel, dim3(nn), dim3(64 * ((L + 63) / 64)), 0, 0,
                           dx, nn, L, dlam);
        ok(hipGetLastError());
    }
    double best = -1.0;
    std::vector<double> bestvec;
    int bestb = 0, eig_failed = -1;
    for (int bi = 0; bi < 4 && e == hipSuccess; ++bi) {
        Block& B = blocks[bi];
        const int nb = (int)B.s.size();
        if (nb == 0) continue;
        ok(hipMemcpy(dbs, B.s.data(), nb * sizeof(int), hipMemcpyHostToDevice));
        ok(hipMemcpy(dbr, B.r.data(), nb * sizeof(int), hipMemcpyHostToDevice));
        if (e != hipSuccess) break;
        dim3 blk(16, 16), grd((nb + 15) / 16, (nb + 15) / 16);
        hipLaunchKernelGGL(slepian_matrix_kernel, grd, blk, 0, 0, dlam, dw, dJ, nn, L, nk, dbs,
                           dbr, nb, B.cls, dD);
        ok(hipGetLastError());
        std::vector<double> A((size_t)nb * nb);
        ok(hipMemcpy(A.data(), dD, A.size() * sizeof(double), hipMemcpyDeviceToHost));
        if (e != hipSuccess) break;
        std::vector<double> v;
        double lam = 0.0;
        if (sym_top_eigenpair(A, nb, &lam, v) != 0) {
            eig_failed = bi;
            break;
        }
        if (lam > best) { best = lam; bestvec = v; bestb = bi; }
    }
    for (void* p : {(void*)dx, (void*)dw, (void*)dJ, (void*)dlam, (void*)dD, (void*)dbs, (void*)dbr})
        if (p) (void)hipFree(p);
    if (e != hipSuccess) return set_error(SLSHT_EDEVICE, "slepian window: %s", hipGetErrorString(e));
    if (eig_failed >= 0)
        return set_error(SLSHT_EDEVICE, "slepian window: the eigenpair of concentration block %d "
                         "failed its residual check (non-finite or unconverged)", eig_failed);
    // real basis -> complex coefficients; sign: the largest coefficient positive
    const Block& B = blocks[bestb];
    int imax = 0;
    for (size_t i = 1; i < bestvec.size(); ++i)
        if (fabs(bestvec[i]) > fabs(bestvec[imax]) + 1e-12) imax = (int)i;
    const double sg = bestvec[imax] < 0 ? -1.0 : 1.0;
    for (int i = 0; i < L * L; ++i) h_out[i] = make_double2(0.0, 0.0);
    const double rs2 = 0.70710678118654752440;
    for (size_t i = 0; i < bestvec.size(); ++i) {
        const int s = B.s[i], r = B.r[i];
        const double c = sg * bestvec[i];
        const double par = (r & 1) ? -1.0 : 1.0;
        if (B.cls > 0) {
            if (r == 0) {
                h_out[s * s + s] = make_double2(c, 0.0);
            } else {            // X = (Y^r + (-1)^r Y^{-r}) / sqrt(2)
                h_out[s * s + s + r] = make_double2(c * rs2, 0.0);
                h_out[s * s + s - r] = make_double2(par * c * rs2, 0.0);
            }
        } else {                // Z = (Y^r - (-1)^r Y^{-r}) / (sqrt(2) i)
            h_out[s * s + s + r] = make_double2(0.0, -c * rs2);
            h_out[s * s + s - r] = make_double2(0.0, par * c * rs2);
        }
    }
    if (conc) *conc = best;
    return SLSHT_OK;
}

}  // namespace slsht
