// gfx950 kernels of the directional SLSHT forward path and its inverse.
//
// Separated form of the distribution (eq. Eq:alternative_harmonic_formulation_wigner,
// evaluated by separation of variables as noted in Section IV-B):
//
//   g(phi_a, theta_b, omega_c; l, m)
//     = sum_q e^{-i q phi_a} sum_{q'} e^{-i q' omega_c}
//       sum_{p >= max(|q|,|q'|)} A^p_q(l,m) h_p^{q'} d^p_{q,q'}(theta_b)
//
// with A^p_q(l,m) = sum_{l'} f_{l'}^{m-q} T(l', m-q; p, q; l, m) the Wigner-3j
// coupling of f (Eq:harmonic_formulation).  Kernels:
//   K1 wigner_table_kernel  d^p_{q,q'}(theta_b), FP64 recursion in p
//   K2 coupling_kernel      A^p_q(l,m), FP64 two-sided 3j recursions
//   K3 synth_full_kernel    theta-contraction, omega- and phi-synthesis, store
//                           (slsht_synth.hip); K3e energy_kernel (slsht_energy.hip)
//   K4 inverse_kernel       weighted sum over the grid (Section IV-A)
#include "slsht_device.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

namespace slsht {

// ------------------------------------------------------------------------------
// K1: Wigner-d table.  One thread per (theta row, canonical pair Q >= |Q'|); the thread seeds
// d^{p0}_{q,q'} at p0 = max(|q|,|q'|) from the one-term form of Wigner's sum
// and climbs in p with the three-term recursion
//   p sqrt(((p+1)^2-q^2)((p+1)^2-q'^2)) d^{p+1}
//     = (2p+1)(p(p+1) cos(beta) - q q') d^p - (p+1) sqrt((p^2-q^2)(p^2-q'^2)) d^{p-1},
// all in FP64; consecutive threads hold consecutive canonical pairs, so each degree's
// row segment is written contiguously.  beta = 2 pi b / n_phi (grid E_L, Section II-D).

__device__ __forceinline__ double ipow(double x, int n) {
    double r = 1.0;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
}

template <typename OutT>
__global__ void wigner_table_kernel(OutT* __restrict__ tab, int L, int n_phi, int theta_lo,
                                    int n_rows, int64_t row_len) {
    const int pair = blockIdx.x * blockDim.x + threadIdx.x;   // = q^2 + q + q'
    const int row = blockIdx.y;
    if (pair >= L * L || row >= n_rows) return;
    int q = (int)sqrtf((float)pair);
    while (q * q > pair) --q;
    while ((q + 1) * (q + 1) <= pair) ++q;
    const int qp = pair - q * q - q;
    const int b = theta_lo + row;
    double sh, ch;                       // sin(beta/2), cos(beta/2), beta/2 = pi b / n_phi
    sincospi((double)b / (double)n_phi, &sh, &ch);
    const double cb = cospi(2.0 * (double)b / (double)n_phi);

    const int aq = q < 0 ? -q : q, aqp = qp < 0 ? -qp : qp;
    const int j0 = aq > aqp ? aq : aqp;
    // Seed: d^j_{r,cc}(beta) for r = +-j, by the single surviving term of
    // Wigner's sum; d^j_{q,q'} = (-1)^{q-q'} d^j_{q',q} covers |q'| > |q|.
    int r, cc;
    double sg = 1.0;
    if (aq >= aqp) { r = q; cc = qp; }
    else { r = qp; cc = q; sg = ((q - qp) & 1) ? -1.0 : 1.0; }
    double bin = 1.0;                    // C(2j, j - cc)
    for (int i = 1; i <= j0 - cc; ++i) bin *= (double)(j0 + cc + i) / (double)i;
    double d = sqrt(bin) * sg;
    if (r == j0) d *= ipow(ch, j0 + cc) * ipow(-sh, j0 - cc);
    else         d *= ipow(ch, j0 - cc) * ipow(sh, j0 + cc);

    OutT* out = tab + (int64_t)row * row_len;
    double dprev = 0.0;
    const double qq = (double)q * (double)qp;
    for (int p = j0; p < L; ++p) {
        out[dtab_off(p) + pair] = (OutT)d;
        if (p + 1 >= L) break;
        double dn;
        if (p == 0) {
            dn = cb;                     // d^1_{00} = cos(beta); the recursion divides by p
        } else {
            const double dp = (double)p;
            const double up = sqrt(((dp + 1) * (dp + 1) - (double)q * q) * ((dp + 1) * (dp + 1) - (double)qp * qp));
            const double dn_ = sqrt((dp * dp - (double)q * q) * (dp * dp - (double)qp * qp));
            dn = ((2 * dp + 1) * (dp * (dp + 1) * cb - qq) * d - (dp + 1) * dn_ * dprev) / (dp * up);
        }
        dprev = d;
        d = dn;
    }
}

hipError_t launch_wigner_table(const DevPlan& P, hipStream_t s) {
    const int L = P.d.L_h;
    dim3 block(128), grid((L * L + 127) / 128, P.n_theta_out);
    const int64_t rl = dtab_row_len(L);
    if (P.d.precision == SLSHT_FP64 || P.d.output_mode == SLSHT_OUT_ENERGY)
        hipLaunchKernelGGL(wigner_table_kernel<double>, grid, block, 0, s, (double*)P.T->dtab, L,
                           P.d.n_phi, P.d.theta_lo, P.n_theta_out, rl);
    else
        hipLaunchKernelGGL(wigner_table_kernel<float>, grid, block, 0, s, (float*)P.T->dtab, L,
                           P.d.n_phi, P.d.theta_lo, P.n_theta_out, rl);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------
// K2: coupling A^p_q(l,m) = (-1)^m sqrt((2p+1)(2l+1)/(4 pi))
//        * sum_{l'} sqrt(2l'+1) (l' p l; 0 0 0) (l' p l; m-q q -m) f_{l'}^{m-q}
// (Gaunt form of the triple product T of Eq:harmonic_formulation).
//
// The 3j symbols (j j2 j3; m1 m2 m3), m1 = -m2-m3, are generated over
// j in [jmin, jmax] by the Schulten-Gordon three-term recursion
//   j A(j+1) F(j+1) + B(j) F(j) + (j+1) A(j) F(j-1) = 0,
//   A(j) = sqrt((j^2-(j2-j3)^2)((j2+j3+1)^2-j^2)(j^2-m1^2)),
//   B(j) = -(2j+1)((j2(j2+1)-j3(j3+1)) m1 - j(j+1)(m3-m2)),
// run forward from jmin while |F| grows and backward from jmax down to the
// meeting point (each direction is stable where the true solution grows), then
// matched, normalised by sum (2j+1) F^2 = 1 and signed so that F(jmax) has the
// sign (-1)^(j2-j3-m1).  Nothing is stored per j: the caller's sink consumes
// the unnormalised values and the returned factors finish the job.
// Inside the two loops each step needs A(j) and a division by j A(j): A and 1/A come from
// one reciprocal square root refined by Goldschmidt's iteration, 1/j from a table `invj`
// (invj[j - jbase] = 1/j), so no step runs a full-precision square root or division.

// sqrt(t) and 1/sqrt(t) for t >= 1 (0 and 0 for t <= 0): v_rsq_f64's estimate y, then two
// steps of Goldschmidt's coupled iteration g -> sqrt(t), h -> 1/(2 sqrt(t)) (each squares
// the relative error), and a last Newton correction of g.
__device__ __forceinline__ void sqrt_and_rsqrt(double t, double& sq, double& rs) {
    const double y = __builtin_amdgcn_rsq(t > 0.0 ? t : 1.0);
    double g = t * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, t);
    sq = t > 0.0 ? fma(d, h, g) : 0.0;
    rs = t > 0.0 ? 2.0 * h : 0.0;
}

struct ThreeJ {
    int jmin, jmax, jm;
    double c;       // backward values are multiplied by c to join the forward ones
    double scale;   // final factor: sign / sqrt(norm)
};

template <class Sink>
__device__ ThreeJ threej_two_sided(int j2, int j3, int m2, int m3, const double* invj, int jbase,
                                   Sink& sink) {
    const int m1 = -m2 - m3;
    const double dj2 = j2, dj3 = j3, dm1 = m1, dm2 = m2, dm3 = m3;
    const double dd = dj2 - dj3, ss = (dj2 + dj3 + 1) * (dj2 + dj3 + 1);
    const double bc = (dj2 * (dj2 + 1) - dj3 * (dj3 + 1)) * dm1, dm = dm3 - dm2;
    auto At = [&](double j) { return (j * j - dd * dd) * (ss - j * j) * (j * j - dm1 * dm1); };
    auto Af = [&](double j) {
        const double t = At(j);
        return t > 0.0 ? sqrt(t) : 0.0;
    };
    auto Bf = [&](double j) { return -(2 * j + 1) * (bc - j * (j + 1) * dm); };

    ThreeJ r;
    const int ad = j2 > j3 ? j2 - j3 : j3 - j2;
    const int am1 = m1 < 0 ? -m1 : m1;
    r.jmin = ad > am1 ? ad : am1;
    r.jmax = j2 + j3;
    int jm = r.jmin;
    double Fprev = 0.0, Fcur = 1.0;
    double norm_f = (2.0 * jm + 1.0);
    sink.fwd(jm, 1.0);
    if (r.jmax > r.jmin) {
        double F1;
        if (r.jmin == 0) F1 = (j2 > 0) ? dm2 / sqrt(dj2 * (dj2 + 1)) : 0.0;   // (1 j j; 0 m -m)/(0 j j; 0 m -m)
        else F1 = -Bf((double)r.jmin) / ((double)r.jmin * Af((double)r.jmin + 1));
        if (fabs(F1) > 1.0) {
            jm = r.jmin + 1;
            Fprev = 1.0;
            Fcur = F1;
            norm_f += (2.0 * jm + 1.0) * F1 * F1;
            sink.fwd(jm, F1);
            double Aj = Af((double)jm);
            while (jm < r.jmax) {
                const double j = jm;
                double Aj1, rAj1;
                sqrt_and_rsqrt(At(j + 1), Aj1, rAj1);
                const double Fn = -(Bf(j) * Fcur + (j + 1) * Aj * Fprev) * (invj[jm - jbase] * rAj1);
                if (fabs(Fn) <= fabs(Fcur)) break;
                ++jm;
                Fprev = Fcur;
                Fcur = Fn;
                Aj = Aj1;
                norm_f += (2.0 * jm + 1.0) * Fn * Fn;
                sink.fwd(jm, Fn);
                if (fabs(Fcur) > 1e120) {
                    Fcur *= 1e-120; Fprev *= 1e-120; norm_f *= 1e-240;
                    sink.rescale_fwd(1e-120);
                }
            }
        }
    }
    r.jm = jm;
    double norm, top;
    if (jm < r.jmax) {
        int j = r.jmax;
        double Bc = 1.0, Bn = 0.0, topb = 1.0, norm_b = (2.0 * j + 1.0);
        sink.bwd(j, 1.0);
        double Aj, rAj, Aj1 = 0.0;
        sqrt_and_rsqrt(At((double)j), Aj, rAj);
        for (;;) {
            const double dj = j;
            const double Bp = -(Bf(dj) * Bc + dj * Aj1 * Bn) * (invj[j + 1 - jbase] * rAj);
            --j;
            Bn = Bc; Bc = Bp; Aj1 = Aj;
            if (j == jm) break;
            sqrt_and_rsqrt(At((double)j), Aj, rAj);
            norm_b += (2.0 * j + 1.0) * Bc * Bc;
            sink.bwd(j, Bc);
            if (fabs(Bc) > 1e120) {
                Bc *= 1e-120; Bn *= 1e-120; norm_b *= 1e-240; topb *= 1e-120;
                sink.rescale_bwd(1e-120);
            }
        }
        r.c = Fcur / Bc;
        norm = norm_f + r.c * r.c * norm_b;
        top = r.c * topb;
    } else {
        r.c = 1.0;
        norm = norm_f;
        top = Fcur;
    }
    const double sigma = ((j2 - j3 - m1) & 1) ? -1.0 : 1.0;
    r.scale = ((top * sigma) > 0.0 ? 1.0 : -1.0) / sqrt(norm);
    return r;
}

// Accumulates sum_j w_j F(j) f_j^{mp} and sum_j w_j F(j) f_j^{-mp} (the mirrored orders) with
// w_j = sqrt(2j+1) Z(j) for j < L_f.  Z(j) vanishes where j + p + l is odd (the parity rule of
// (j p l; 0 0 0)); those terms are skipped.
struct DotSink {
    const double2* f;
    const double* z;     // Z row for this p: sqrt(2j+1) (j p l; 0 0 0) at index j - zlo
    int zlo, L_f, mp, par;
    double fr, fi, br, bi;   // order mp: forward and backward sums
    double gr, gi, cr, ci;   // order -mp
    __device__ void add(int j, double v, double& ar, double& ai, double& xr, double& xi) {
        if (j >= L_f || ((j ^ par) & 1)) return;
        const double w = z[j - zlo] * v;
        const int64_t c0 = (int64_t)j * j + j;
        const double2 c = f[c0 + mp];
        const double2 d = f[c0 - mp];
        ar += w * c.x;
        ai += w * c.y;
        xr += w * d.x;
        xi += w * d.y;
    }
    __device__ void fwd(int j, double v) { add(j, v, fr, fi, gr, gi); }
    __device__ void bwd(int j, double v) { add(j, v, br, bi, cr, ci); }
    __device__ void rescale_fwd(double s) { fr *= s; fi *= s; gr *= s; gi *= s; }
    __device__ void rescale_bwd(double s) { br *= s; bi *= s; cr *= s; ci *= s; }
};

// One block per (l, m >= 0).  (j p l; m-q q -m) and (j p l; q-m -q m) differ by (-1)^(j+p+l),
// which is 1 wherever (j p l; 0 0 0) is nonzero, so A^p_q(l, m) and A^p_{-q}(l, -m) share
// their 3j recursion and differ only in the f_j^{+-(m-q)} they sum.  For m = 0 the pairs
// (p, q), (p, -q) share one recursion in the same way.
__global__ void coupling_kernel(const double2* __restrict__ f, double2* __restrict__ A, int L_f,
                                int L_h, int l_lo) {
    __shared__ double Z[SLSHT_MAX_LH * SLSHT_MAX_LH];
    __shared__ double invj[2 * SLSHT_MAX_LH + 1];
    const Item it = item_decode(blockIdx.x, l_lo, 1);
    const int l = it.l, m = it.m, L2 = L_h * L_h;
    // every recursion below runs over j in [|l - p|, l + p], p < L_h
    const int jbase = l - L_h + 1 > 1 ? l - L_h + 1 : 1;
    for (int i = threadIdx.x; i < 2 * L_h + 1; i += blockDim.x) invj[i] = 1.0 / (double)(jbase + i);
    __syncthreads();
    // Z rows: sqrt(2j+1) (j p l; 0 0 0) for j in [|l-p|, l+p], row p at offset p*p.  The
    // symbol vanishes unless j + p + l is even; its closed form (the Racah formula with zero
    // orders) gives the ratio of consecutive nonzero entries, at a = p + l - j,
    // b = j + l - p, c = j + p - l, J = j + p + l:
    //   Z(j + 2) / Z(j) = -sqrt(2 (b+1)(c+1)(J/2+1) a / ((b+2)(c+2)(J+3)(a-1))).
    // One 32-lane group per row: lane i takes j = |l-p| + 2i, the ratios are multiplied
    // along the lanes, then normalised by sum_j (2j+1) Z^2 = 1 and signed by Z(|l-p|)'s sign
    // (-1)^max(l, p).
    {
        const int grp = threadIdx.x >> 5, gl = threadIdx.x & 31, ngrp = blockDim.x >> 5;
        for (int p = grp; p < L_h; p += ngrp) {
            const int n = (l < p ? l : p) + 1;                 // nonzero entries (<= 32)
            const int j0 = l > p ? l - p : p - l;
            const int j = j0 + 2 * gl;
            double R = 1.0;
            if (gl >= 1 && gl < n) {
                const double jp = j - 2;
                const double a = p + l - jp, b = jp + l - p, c = jp + p - l, J = jp + p + l;
                R = -sqrt(2.0 * (b + 1) * (c + 1) * (0.5 * J + 1) * a /
                          ((b + 2) * (c + 2) * (J + 3) * (a - 1)));
            }
            for (int d = 1; d < 32; d <<= 1) {                 // inclusive prefix product
                const double o = __shfl_up(R, d, 32);
                if (gl >= d) R *= o;
            }
            double w = gl < n ? (2.0 * j + 1.0) * R * R : 0.0;
            for (int d = 16; d > 0; d >>= 1) w += __shfl_xor(w, d, 32);
            const double scale = (((l > p ? l : p) & 1) ? -1.0 : 1.0) / sqrt(w);
            double* row = Z + p * p;
            if (gl < n) {
                row[2 * gl] = scale * R * sqrt(2.0 * j + 1.0);
                if (gl + 1 < n) row[2 * gl + 1] = 0.0;
            }
        }
    }
    __syncthreads();
    const double sm = (m & 1) ? -1.0 : 1.0;
    const double pref = sm * sqrt((2.0 * l + 1.0) / (4.0 * M_PI));
    // tasks: every (p, q) for m > 0; (p, q >= 0) for m = 0, task p(p+1)/2 + q
    const int ntask = m > 0 ? L2 : L_h * (L_h + 1) / 2;
    for (int task = threadIdx.x; task < ntask; task += blockDim.x) {
        int p, q;
        if (m > 0) {
            lm_of(task, p, q);
        } else {
            p = (int)((sqrt(8.0 * task + 1.0) - 1.0) * 0.5);
            while ((p + 1) * (p + 2) / 2 <= task) ++p;
            while (p * (p + 1) / 2 > task) --p;
            q = task - p * (p + 1) / 2;
        }
        DotSink ds;
        ds.f = f;
        ds.z = Z + p * p;
        ds.zlo = l > p ? l - p : p - l;
        ds.L_f = L_f;
        ds.mp = m - q;
        ds.par = (p + l) & 1;
        ds.fr = ds.fi = ds.br = ds.bi = 0.0;
        ds.gr = ds.gi = ds.cr = ds.ci = 0.0;
        const ThreeJ t = threej_two_sided(p, l, q, -m, invj, jbase, ds);
        const double k = pref * sqrt(2.0 * p + 1.0) * t.scale;
        const double2 out = vmk<double2>(k * (ds.fr + t.c * ds.br), k * (ds.fi + t.c * ds.bi));
        const double2 mir = vmk<double2>(k * (ds.gr + t.c * ds.cr), k * (ds.gi + t.c * ds.ci));
        A[(int64_t)it.lm * L2 + p * p + p + q] = out;
        if (m > 0)
            A[(int64_t)it.mirror * L2 + p * p + p - q] = mir;        // A^p_{-q}(l, -m)
        else if (q > 0)
            A[(int64_t)it.lm * L2 + p * p + p - q] = mir;            // A^p_{-q}(l, 0)
    }
}

hipError_t launch_coupling(const DevPlan& P, const double2* f, double2* A, hipStream_t s) {
    // blocks: the (l, m >= 0)
    const int n_blk = P.d.l_hi * (P.d.l_hi + 1) / 2 - P.d.l_lo * (P.d.l_lo + 1) / 2;
    const int L2 = P.d.L_h * P.d.L_h;
    // whole waves only: the (p, q) past the block (the largest p, the longest recursions)
    // go to its first lanes, which hold the smallest p
    const int block = std::max(64, std::min(512, L2 / 64 * 64));
    hipLaunchKernelGGL(coupling_kernel, dim3(n_blk), dim3(block), 0, s, f, A, P.d.L_f, P.d.L_h,
                       P.d.l_lo);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------
// K4: inverse.  f_out[lm] = scale * sum_{c,b,a} q(theta_b) g[lm][c][b][a], one block per lm,
// FP64 accumulation, wavefront shuffle + LDS reduction.

template <typename V>
__global__ void __launch_bounds__(256) inverse_kernel(const V* __restrict__ g,
                                                      const double* __restrict__ qw, int n_phi,
                                                      int n_theta, int n_omega, double k,
                                                      const double2* __restrict__ h,
                                                      double2* __restrict__ f_out, int n_lm) {
    // each XCD (block b runs on XCD b mod 8) takes a contiguous run of the (l, m) slabs
    const int lm = (int)(blockIdx.x & 7) * (int)(gridDim.x >> 3) + (int)(blockIdx.x >> 3);
    if (lm >= n_lm) return;
    __shared__ double qs[(SLSHT_MAX_NPHI + 1) / 2];
    __shared__ double red[2][8];
    for (int i = threadIdx.x; i < n_theta; i += blockDim.x) qs[i] = qw[i];
    __syncthreads();
    const int64_t n = (int64_t)n_omega * n_theta * n_phi;
    const V* gp = g + (int64_t)lm * n;
    // element i sits at phi index a of a row whose theta index is b; both advance with the
    // block stride (sa, sb, with a carry from a into b), so the loop divides nothing
    const int stride = blockDim.x;
    const int sa = stride % n_phi, sb = (stride / n_phi) % n_theta;
    int a = threadIdx.x % n_phi, b = (threadIdx.x / n_phi) % n_theta;
    auto advance = [&]() {
        a += sa;
        b += sb;
        if (a >= n_phi) {
            a -= n_phi;
            ++b;
        }
        if (b >= n_theta) b -= n_theta;
    };
    double ar = 0.0, ai = 0.0;
    int64_t i = threadIdx.x;
    for (; i + 3 * (int64_t)stride < n; i += 4 * (int64_t)stride) {   // four loads in flight
        V v[4];
        int bb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            v[u] = gp[i + u * (int64_t)stride];
            bb[u] = b;
            advance();
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ar += qs[bb[u]] * (double)v[u].x;
            ai += qs[bb[u]] * (double)v[u].y;
        }
    }
    for (; i < n; i += stride) {
        const V v = gp[i];
        ar += qs[b] * (double)v.x;
        ai += qs[b] * (double)v.y;
        advance();
    }
    for (int o = 32; o > 0; o >>= 1) {
        ar += __shfl_xor(ar, o);
        ai += __shfl_xor(ai, o);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[0][w] = ar; red[1][w] = ai; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sr = 0.0, si = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) { sr += red[0][k]; si += red[1][k]; }
        // f = k * sum / h_0^0 (read here, so that no host synchronisation is needed)
        const double2 h00 = h[0];
        const double mag2 = h00.x * h00.x + h00.y * h00.y;
        const double scx = k * h00.x / mag2, scy = -k * h00.y / mag2;
        double2 o;
        o.x = scx * sr - scy * si;
        o.y = scx * si + scy * sr;
        f_out[lm] = o;
    }
}

hipError_t launch_inverse(const DevPlan& P, const void* g, double k, const double2* h,
                          double2* f_out, hipStream_t s) {
    const int n_lm = P.d.l_hi * P.d.l_hi - P.d.l_lo * P.d.l_lo;
    const int grid = (n_lm + 7) / 8 * 8;
    if (P.d.precision == SLSHT_FP64)
        hipLaunchKernelGGL(inverse_kernel<double2>, dim3(grid), dim3(256), 0, s,
                           (const double2*)g, P.T->qw, P.d.n_phi, P.d.n_theta, P.d.n_omega, k, h,
                           f_out, n_lm);
    else
        hipLaunchKernelGGL(inverse_kernel<float2>, dim3(grid), dim3(256), 0, s,
                           (const float2*)g, P.T->qw, P.d.n_phi, P.d.n_theta, P.d.n_omega, k, h,
                           f_out, n_lm);
    return hipGetLastError();
}

}  // namespace slsht
