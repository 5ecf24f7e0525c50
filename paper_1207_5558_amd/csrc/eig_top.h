// Largest eigenpair of a dense real symmetric matrix (host code, header-only).
//
// Used for the Slepian concentration problem of Section III-D, whose blocks have at most a
// few hundred rows and whose top eigenvector is the window.  Method:
//  1. the Lanczos process (Lanczos 1950) from a fixed generic start vector, with complete
//     reorthogonalisation of every new direction against the whole basis, applied twice
//     (the "twice is enough" rule of Kahan and Parlett); when the Krylov space becomes
//     invariant before it has n directions the process restarts from a fresh direction
//     orthogonal to the basis, so the tridiagonal T (block diagonal at restarts) carries
//     every eigenvalue of the matrix;
//  2. the largest eigenvalue of T by bisection on the Sturm count of its LDL^T pivots
//     (Givens' method, as in Barth, Martin and Wilkinson 1967);
//  3. its eigenvector by inverse iteration on T - lambda I, solved by Gaussian elimination
//     with row interchanges (Wilkinson), mapped back through the Lanczos basis;
//  4. the Rayleigh quotient of that vector and a residual check on the full matrix: a
//     residual above tolerance is reported as failure, never returned as a result.
#pragma once

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <vector>

namespace slsht {
namespace eig {

// Number of eigenvalues of the symmetric tridiagonal (a, b) strictly below x
// (pivots of the LDL^T factorisation of T - x I; a pivot too close to zero is
// nudged to -pivmin, which keeps the count monotone in x).
inline int sturm_below(const std::vector<double>& a, const std::vector<double>& b, double x,
                       double pivmin) {
    int count = 0;
    double piv = 1.0;
    for (size_t i = 0; i < a.size(); ++i) {
        double t = a[i] - x;
        if (i > 0) t -= b[i - 1] * b[i - 1] / piv;
        if (std::fabs(t) < pivmin) t = -pivmin;
        if (t < 0.0) ++count;
        piv = t;
    }
    return count;
}

// Largest eigenvalue of the tridiagonal (a, b) by bisection of a Gershgorin interval.
inline double tridiag_top(const std::vector<double>& a, const std::vector<double>& b) {
    const size_t k = a.size();
    double lo = a[0], hi = a[0], bmax = 0.0;
    for (size_t i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
        if (i + 1 < k) bmax = std::max(bmax, b[i] * b[i]);
    }
    const double pivmin = DBL_MIN * std::max(1.0, bmax);
    const double span = std::max(std::fabs(lo), std::fabs(hi));
    lo -= 2.0 * DBL_EPSILON * span + pivmin;
    hi += 2.0 * DBL_EPSILON * span + pivmin;
    for (int it = 0; it < 4096; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;                 // interval at one ulp
        if (hi - lo <= 2.0 * DBL_EPSILON * std::max(std::fabs(lo), std::fabs(hi)) + pivmin) break;
        if (sturm_below(a, b, mid, pivmin) == (int)k) hi = mid;   // every eigenvalue below mid
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// Solves (T - s I) y = rhs in place for the symmetric tridiagonal (a, b): elimination
// with row interchanges leaves an upper factor with two superdiagonals (u0, u1, u2).
// Zero pivots are replaced by `tiny` (inverse iteration wants the near-singular solve).
inline void tridiag_shifted_solve(const std::vector<double>& a, const std::vector<double>& b,
                                  double s, double tiny, std::vector<double>& y) {
    const size_t k = a.size();
    std::vector<double> u0(k), u1(k, 0.0), u2(k, 0.0);
    for (size_t i = 0; i < k; ++i) {
        u0[i] = a[i] - s;
        if (i + 1 < k) u1[i] = b[i];
    }
    for (size_t i = 0; i + 1 < k; ++i) {
        const double sub = b[i];               // entry (i+1, i) of the current system
        if (std::fabs(u0[i]) >= std::fabs(sub)) {
            if (u0[i] == 0.0) u0[i] = tiny;
            const double f = sub / u0[i];
            u0[i + 1] -= f * u1[i];
            u1[i + 1] -= f * u2[i];
            y[i + 1] -= f * y[i];
        } else {
            // swap row i (u0[i], u1[i], u2[i]) with row i+1 (sub, u0[i+1], u1[i+1], 0)
            const double r0 = u0[i], r1 = u1[i], r2 = u2[i];
            u0[i] = sub;
            u1[i] = u0[i + 1];
            u2[i] = (i + 1 < k) ? u1[i + 1] : 0.0;
            std::swap(y[i], y[i + 1]);
            const double f = r0 / sub;
            u0[i + 1] = r1 - f * u1[i];
            u1[i + 1] = r2 - f * u2[i];
            y[i + 1] -= f * y[i];
        }
    }
    if (u0[k - 1] == 0.0) u0[k - 1] = tiny;
    for (size_t ii = k; ii-- > 0;) {
        double t = y[ii];
        if (ii + 1 < k) t -= u1[ii] * y[ii + 1];
        if (ii + 2 < k) t -= u2[ii] * y[ii + 2];
        y[ii] = t / u0[ii];
    }
}

}  // namespace eig

// Largest eigenvalue *lambda and unit eigenvector x of the n x n symmetric matrix A
// (row-major, not modified).  Returns 0, or -1 when the input is empty or not finite or
// the final residual |A x - lambda x| exceeds 1e-10 of the matrix norm.
inline int sym_top_eigenpair(const std::vector<double>& A, int n, double* lambda,
                             std::vector<double>& x) {
    if (n <= 0 || (long)A.size() < (long)n * n) return -1;
    double fro = 0.0;
    for (long i = 0; i < (long)n * n; ++i) fro += A[i] * A[i];
    fro = std::sqrt(fro);
    if (!std::isfinite(fro)) return -1;
    x.assign(n, 0.0);
    if (fro == 0.0) {
        x[0] = 1.0;
        *lambda = 0.0;
        return 0;
    }
    auto matvec = [&](const double* v, double* w) {
        for (int i = 0; i < n; ++i) {
            const double* row = &A[(size_t)i * n];
            double acc = 0.0;
            for (int j = 0; j < n; ++j) acc += row[j] * v[j];
            w[i] = acc;
        }
    };
    auto dot = [&](const double* u, const double* v) {
        double acc = 0.0;
        for (int i = 0; i < n; ++i) acc += u[i] * v[i];
        return acc;
    };
    std::vector<double> Q((size_t)n * n);        // Lanczos basis, direction j at Q[j*n]
    std::vector<double> alpha, beta;             // T: diagonal, off-diagonal (0 at restarts)
    std::vector<double> w(n);
    // orthogonalise w against directions 0..cnt-1, twice; returns the norm left
    auto orthogonalise = [&](int cnt) {
        for (int pass = 0; pass < 2; ++pass)
            for (int k = 0; k < cnt; ++k) {
                const double* q = &Q[(size_t)k * n];
                const double c = dot(q, w.data());
                for (int i = 0; i < n; ++i) w[i] -= c * q[i];
            }
        return std::sqrt(dot(w.data(), w.data()));
    };
    // a fresh direction orthogonal to the first cnt ones (start vector when cnt == 0):
    // a fixed vector with all components nonzero, then unit vectors in turn
    int next_unit = 0;
    auto fresh = [&](int cnt) {
        for (int attempt = 0; attempt <= n; ++attempt) {
            if (cnt == 0 && attempt == 0) {
                for (int i = 0; i < n; ++i) w[i] = 1.0 + 0.5 * std::sin(1.0 + 2.3 * i);
            } else {
                std::fill(w.begin(), w.end(), 0.0);
                w[(next_unit++) % n] = 1.0;
            }
            const double nrm = orthogonalise(cnt);
            if (nrm > 1e-3) {
                for (int i = 0; i < n; ++i) Q[(size_t)cnt * n + i] = w[i] / nrm;
                return true;
            }
        }
        return false;
    };
    if (!fresh(0)) return -1;
    const double small = 1e-12 * fro;
    for (int j = 0; j < n; ++j) {
        const double* q = &Q[(size_t)j * n];
        matvec(q, w.data());
        const double a = dot(q, w.data());
        alpha.push_back(a);
        if (j == n - 1) break;
        const double nrm = orthogonalise(j + 1);
        if (nrm > small) {
            beta.push_back(nrm);
            for (int i = 0; i < n; ++i) Q[(size_t)(j + 1) * n + i] = w[i] / nrm;
        } else {                                  // invariant subspace: restart
            beta.push_back(0.0);
            if (!fresh(j + 1)) return -1;
        }
    }
    const double lam_t = eig::tridiag_top(alpha, beta);
    // inverse iteration on T - lam_t I
    std::vector<double> y(n, 1.0);
    const double tiny = DBL_EPSILON * fro;
    for (int it = 0; it < 3; ++it) {
        eig::tridiag_shifted_solve(alpha, beta, lam_t, tiny, y);
        double ny = 0.0;
        for (double v : y) ny += v * v;
        ny = std::sqrt(ny);
        if (!(ny > 0.0) || !std::isfinite(ny)) return -1;
        for (double& v : y) v /= ny;
    }
    for (int k = 0; k < n; ++k) {
        const double* qk = &Q[(size_t)k * n];
        for (int i = 0; i < n; ++i) x[i] += y[k] * qk[i];
    }
    double nx = std::sqrt(dot(x.data(), x.data()));
    for (double& v : x) v /= nx;
    matvec(x.data(), w.data());
    const double rq = dot(x.data(), w.data());
    double res = 0.0;
    for (int i = 0; i < n; ++i) res += (w[i] - rq * x[i]) * (w[i] - rq * x[i]);
    res = std::sqrt(res);
    if (!(res <= 1e-10 * fro)) return -1;
    *lambda = rq;
    return 0;
}

}  // namespace slsht
