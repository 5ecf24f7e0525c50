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
//   K4 inverse_kernel       weighted sum over the grid (Section IV-A)
#include "slsht_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

namespace slsht {

// ------------------------------------------------------------------------------
// small complex helpers (interleaved re, im in HIP vector types)

template <typename T> struct VecOf;
template <> struct VecOf<double> { using type = double2; };
template <> struct VecOf<float> { using type = float2; };

template <typename V> __device__ __forceinline__ V vmk(decltype(V::x) x, decltype(V::x) y) {
    V v; v.x = x; v.y = y; return v;
}
template <typename V> __device__ __forceinline__ V vadd(V a, V b) { return vmk<V>(a.x + b.x, a.y + b.y); }
template <typename V> __device__ __forceinline__ V vsub(V a, V b) { return vmk<V>(a.x - b.x, a.y - b.y); }
// -i * v
template <typename V> __device__ __forceinline__ V vmul_mi(V v) { return vmk<V>(v.y, -v.x); }
template <typename V> __device__ __forceinline__ V vcast(double2 a) {
    return vmk<V>((decltype(V::x))a.x, (decltype(V::x))a.y);
}

// ------------------------------------------------------------------------------
// K1: Wigner-d table.  One thread per (theta row, q, q'); the thread seeds
// d^{p0}_{q,q'} at p0 = max(|q|,|q'|) from the one-term form of Wigner's sum
// and climbs in p with the three-term recursion
//   p sqrt(((p+1)^2-q^2)((p+1)^2-q'^2)) d^{p+1}
//     = (2p+1)(p(p+1) cos(beta) - q q') d^p - (p+1) sqrt((p^2-q^2)(p^2-q'^2)) d^{p-1},
// all in FP64; consecutive threads hold consecutive q', so each degree's row
// segment is written contiguously.  beta = 2 pi b / n_phi (grid E_L, Section II-D).

__device__ __forceinline__ double ipow(double x, int n) {
    double r = 1.0;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
}

template <typename OutT>
__global__ void wigner_table_kernel(OutT* __restrict__ tab, int L, int n_phi, int theta_lo,
                                    int n_rows, int64_t row_len) {
    const int K = 2 * L - 1;
    const int pair = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (pair >= K * K || row >= n_rows) return;
    const int q = pair / K - (L - 1);
    const int qp = pair % K - (L - 1);
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
        out[dtab_off(p) + (q + p) * (2 * p + 1) + (qp + p)] = (OutT)d;
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
    const int L = P.d.L_h, K = 2 * L - 1;
    dim3 block(128), grid((K * K + 127) / 128, P.n_theta_out);
    const int64_t rl = dtab_row_len(L);
    if (P.d.precision == SLSHT_FP64)
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

struct ThreeJ {
    int jmin, jmax, jm;
    double c;       // backward values are multiplied by c to join the forward ones
    double scale;   // final factor: sign / sqrt(norm)
};

template <class Sink>
__device__ ThreeJ threej_two_sided(int j2, int j3, int m2, int m3, Sink& sink) {
    const int m1 = -m2 - m3;
    const double dj2 = j2, dj3 = j3, dm1 = m1, dm2 = m2, dm3 = m3;
    const double dd = dj2 - dj3, ss = (dj2 + dj3 + 1) * (dj2 + dj3 + 1);
    const double bc = (dj2 * (dj2 + 1) - dj3 * (dj3 + 1)) * dm1, dm = dm3 - dm2;
    auto Af = [&](double j) {
        const double t = (j * j - dd * dd) * (ss - j * j) * (j * j - dm1 * dm1);
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
                const double Aj1 = Af(j + 1);
                const double Fn = -(Bf(j) * Fcur + (j + 1) * Aj * Fprev) / (j * Aj1);
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
        double Aj = Af((double)j), Aj1 = 0.0;
        for (;;) {
            const double dj = j;
            const double Bp = -(Bf(dj) * Bc + dj * Aj1 * Bn) / ((dj + 1) * Aj);
            --j;
            Bn = Bc; Bc = Bp; Aj1 = Aj;
            if (j == jm) break;
            Aj = Af((double)j);
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

// Writes the unnormalised sequence into an LDS row; the caller rescales it.
struct RowSink {
    double* row;
    int jmin, jmax, jm_hi, jb_lo;
    __device__ void fwd(int j, double v) { row[j - jmin] = v; jm_hi = j; }
    __device__ void bwd(int j, double v) { row[j - jmin] = v; jb_lo = j; }
    __device__ void rescale_fwd(double s) { for (int j = jmin; j <= jm_hi; ++j) row[j - jmin] *= s; }
    __device__ void rescale_bwd(double s) { for (int j = jb_lo; j <= jmax; ++j) row[j - jmin] *= s; }
};

// Accumulates sum_j w_j F(j) with w_j = sqrt(2j+1) Z(j) f_j^{mp} for j < L_f.
struct DotSink {
    const double2* f;
    const double* z;     // Z row for this p: (j p l; 0 0 0) at index j - zlo
    int zlo, L_f, mp;
    double fr, fi, br, bi;
    __device__ void add(int j, double v, double& ar, double& ai) {
        if (j >= L_f) return;
        const double w = sqrt(2.0 * j + 1.0) * z[j - zlo] * v;
        const double2 c = f[(int64_t)j * j + j + mp];
        ar += w * c.x;
        ai += w * c.y;
    }
    __device__ void fwd(int j, double v) { add(j, v, fr, fi); }
    __device__ void bwd(int j, double v) { add(j, v, br, bi); }
    __device__ void rescale_fwd(double s) { fr *= s; fi *= s; }
    __device__ void rescale_bwd(double s) { br *= s; bi *= s; }
};

__device__ __forceinline__ void lm_of(int lm_abs, int& l, int& m) {
    int ll = (int)sqrt((double)lm_abs);
    while (ll * ll > lm_abs) --ll;
    while ((ll + 1) * (ll + 1) <= lm_abs) ++ll;
    l = ll;
    m = lm_abs - ll * ll - ll;
}

__global__ void coupling_kernel(const double2* __restrict__ f, double2* __restrict__ A, int L_f,
                                int L_h, int l_lo) {
    __shared__ double Z[SLSHT_MAX_LH * SLSHT_MAX_LH];
    const int lm = blockIdx.x;
    int l, m;
    lm_of(lm + l_lo * l_lo, l, m);
    // Z rows: (j p l; 0 0 0) for j in [|l-p|, l+p], row p at offset p*p.
    for (int p = threadIdx.x; p < L_h; p += blockDim.x) {
        RowSink rs;
        rs.row = Z + p * p;
        rs.jmin = l > p ? l - p : p - l;
        rs.jmax = l + p;
        rs.jm_hi = rs.jmin;
        rs.jb_lo = rs.jmax;
        const ThreeJ t = threej_two_sided(p, l, 0, 0, rs);
        for (int j = t.jmin; j <= t.jmax; ++j)
            rs.row[j - t.jmin] *= (j <= t.jm ? t.scale : t.c * t.scale);
    }
    __syncthreads();
    const double sm = (m & 1) ? -1.0 : 1.0;
    const double pref = sm * sqrt((2.0 * l + 1.0) / (4.0 * M_PI));
    for (int pq = threadIdx.x; pq < L_h * L_h; pq += blockDim.x) {
        int p, q;
        lm_of(pq, p, q);
        DotSink ds;
        ds.f = f;
        ds.z = Z + p * p;
        ds.zlo = l > p ? l - p : p - l;
        ds.L_f = L_f;
        ds.mp = m - q;
        ds.fr = ds.fi = ds.br = ds.bi = 0.0;
        const ThreeJ t = threej_two_sided(p, l, q, -m, ds);
        const double k = pref * sqrt(2.0 * p + 1.0) * t.scale;
        double2 out;
        out.x = k * (ds.fr + t.c * ds.br);
        out.y = k * (ds.fi + t.c * ds.bi);
        A[(int64_t)lm * L_h * L_h + pq] = out;
    }
}

hipError_t launch_coupling(const DevPlan& P, const double2* f, double2* A, hipStream_t s) {
    const int n_lm = P.d.l_hi * P.d.l_hi - P.d.l_lo * P.d.l_lo;
    const int L2 = P.d.L_h * P.d.L_h;
    const int block = L2 <= 64 ? 64 : (L2 <= 256 ? 256 : 512);
    hipLaunchKernelGGL(coupling_kernel, dim3(n_lm), dim3(block), 0, s, f, A, P.d.L_f, P.d.L_h,
                       P.d.l_lo);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------
// K3: fused synthesis.  One block = one (l, m) item x a tile of tb theta rows.
//   stage 1 (theta): S_{q,q'}(theta_b) = sum_p A^p_q h_p^{q'} d^p_{q,q'}(theta_b)   -> LDS
//   stage 2 (omega): U_q(theta_b, omega_c) = sum_{q'} S_{q,q'} e^{-i q' omega_c}, folded
//                    into P_q = U_q + U_{-q}, M_q = -i (U_q - U_{-q})             -> LDS
//   stage 3 (phi):   g(phi_a) = U_0 + sum_{q>0} P_q cos(q phi_a) + M_q sin(q phi_a),
//                    g(phi_{n-a}) = same with the sine part negated                -> HBM
// The cosine/sine folding uses phi_{n-a} = -phi_a (mod 2 pi), so one product makes
// two outputs; stage 2 folds omega the same way.  Stage 3 is a pair of real GEMMs on
// the matrix cores, one row per (omega_c, theta_b, Re|Im) and one column per slot a:
//   C = Pmat (rows x k) * cos(k phi_a) (k x a),   S = Mmat * sin(k phi_a),
// with P_0 = U_0 carried by cos(0) = 1.  16x16x4 MFMA (FP32 or FP64): lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; the FP32 form returns D rows 4(l/16)+r, the FP64
// form rows (l/16)+4r, of column l%16.  A-operand rows are permuted per precision so
// that every lane receives Re and Im of two complex rows.

// Theta-stage work items.  The K x K entries (q, q') of S are visited ring by ring,
// s = max(|q|,|q'|) (every entry of ring s sums L - s degrees p, so lanes of a wave share
// trip counts), and one item covers (q, q') and its mirror (-q, -q'), which reuses the
// same d values: d^p_{-q,-q'} = (-1)^{q-q'} d^p_{q,q'} (symmetry in Section IV-B).
// Ring s >= 1 has 4s items: q = -s (q' = -s..s), then q' = s (q = -s+1..s-1); rings are
// stored from s = L-1 down to 1, and the last item is (0, 0) alone.
__device__ __forceinline__ int ring_items(int L) { return 2 * L * (L - 1) + 1; }

__device__ __forceinline__ void ring_item(int r, int L, int& s, int& q, int& qp) {
    int j;
    if (r == ring_items(L) - 1) {
        s = 0;
        j = 0;
    } else {
        const int x = 2 * (L - 1) * L - r;          // = 2 s (s+1) + (4s - j), 0 <= j < 4s
        s = (int)((sqrtf(2.0f * (float)x + 1.0f) - 1.0f) * 0.5f);
        while (2 * s * (s + 1) < x) ++s;
        while (s > 0 && 2 * (s - 1) * s >= x) --s;
        j = 2 * s * (s + 1) - x;
    }
    if (j <= 2 * s) { q = -s; qp = -s + j; }
    else { qp = s; q = -s + (j - 2 * s); }
}

// S_{q,q'} and S_{-q,-q'} of one theta row for the ring item (s, q, q').  Offsets into
// the Wigner-d row advance by additions; the d values of PF consecutive degrees are
// loaded together before they are used, so an item waits for memory ceil((L-s)/PF)
// times rather than L-s times.
template <typename T, typename V, int PF>
__device__ __forceinline__ void theta_pair(const T* __restrict__ drow, const V* A_s, const V* h_s,
                                           int L, int s, int q, int qp, V& out, V& mirror) {
    int off = dtab_off(s) + (q + s) * (2 * s + 1) + (qp + s);
    int ia = s * s + s;                              // p^2 + p
    T sr = 0, si = 0, tr = 0, ti = 0;
    for (int p0 = s; p0 < L; p0 += PF) {
        T dv[PF];
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int p = p0 + i;
            dv[i] = 0;
            if (p < L) {
                dv[i] = drow[off];
                off += (2 * p + 1) * (2 * p + 1) + 2 * q + 4 * p + 4;
            }
        }
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int p = p0 + i;
            if (p < L) {
                const V a1 = A_s[ia + q], h1 = h_s[ia + qp];
                const V a2 = A_s[ia - q], h2 = h_s[ia - qp];
                sr += (a1.x * h1.x - a1.y * h1.y) * dv[i];
                si += (a1.x * h1.y + a1.y * h1.x) * dv[i];
                tr += (a2.x * h2.x - a2.y * h2.y) * dv[i];
                ti += (a2.x * h2.y + a2.y * h2.x) * dv[i];
                ia += 2 * p + 2;
            }
        }
    }
    const T sgn = ((q - qp) & 1) ? T(-1) : T(1);
    out = vmk<V>(sr, si);
    mirror = vmk<V>(sgn * tr, sgn * ti);
}

struct SynthArgs {
    const double2* A;
    const double2* h;
    const void* dtab;
    const void* twphi;
    const void* twom;
    void* g;
    int64_t dstride;
    int L, K, n_phi, n_omega, n_theta_out, tb, n_tiles, nslot, ncp, l_lo, real_pair;
    int xsize;    // elements of the A/h | P/M union region in LDS
};

// Synthesis item -> output slot lm, degree l, order m and the slot of order -m that is
// filled by conjugate symmetry (-1 if none).  Without REAL_PAIR the items are the lm
// slots themselves; with it they enumerate (l, m), l_lo <= l, 0 <= m <= l, in order.
struct Item {
    int lm, l, m, mirror;
};

__device__ __forceinline__ Item item_decode(int item, int l_lo, int real_pair) {
    Item it;
    if (!real_pair) {
        lm_of(item + l_lo * l_lo, it.l, it.m);
        it.lm = item;
        it.mirror = -1;
        return it;
    }
    const int64_t x = item + (int64_t)l_lo * (l_lo + 1) / 2;   // = l(l+1)/2 + m
    int l = (int)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
    while ((int64_t)(l + 1) * (l + 2) / 2 <= x) ++l;
    while ((int64_t)l * (l + 1) / 2 > x) --l;
    it.l = l;
    it.m = (int)(x - (int64_t)l * (l + 1) / 2);
    it.lm = l * l + l + it.m - l_lo * l_lo;
    it.mirror = it.m > 0 ? l * l + l - it.m - l_lo * l_lo : -1;
    return it;
}

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

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

template <typename T, int LH, int NS>
__global__ void __launch_bounds__(256) synth_full_kernel(const SynthArgs a) {
    using V = typename VecOf<T>::type;
    using MF = MfmaOf<T>;
    using Acc = typename MF::acc;
    constexpr int KQ = LH / 4;                   // MFMA k-steps of the phi GEMM
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* S_s = reinterpret_cast<V*>(smem_raw);
    const int L = a.L, K = a.K;
    const int PMS = 2 * LH + 1;                  // complex stride of one P|M row
    V* X_s = S_s + a.tb * K * K;
    V* A_s = X_s;
    V* h_s = X_s + LH * LH;
    V* PM_s = X_s;                               // [c*tb + t][P_0..P_{LH-1} M_0..M_{LH-1}]
    V* TW_s = X_s + a.xsize;                     // [L-1][ncp] omega twiddles

    const int item = blockIdx.x / a.n_tiles;
    const int tile = blockIdx.x - item * a.n_tiles;
    const Item it = item_decode(item, a.l_lo, a.real_pair);
    const int t0 = tile * a.tb;
    const int tb = min(a.tb, a.n_theta_out - t0);
    const int tid = threadIdx.x, nth = blockDim.x;

    const V* twg = reinterpret_cast<const V*>(a.twom);
    for (int i = tid; i < L * L; i += nth) {
        A_s[i] = vcast<V>(a.A[(int64_t)it.lm * L * L + i]);
        h_s[i] = vcast<V>(a.h[i]);
    }
    for (int i = tid; i < (L - 1) * a.ncp; i += nth) TW_s[i] = twg[i];
    __syncthreads();

    // stage 1: theta contraction, ring-ordered items (see ring_item / theta_pair)
    const T* dt = reinterpret_cast<const T*>(a.dtab);
    const int KK = K * K;
    const int nrep = ring_items(L);
    for (int idx = tid; idx < tb * nrep; idx += nth) {
        const int t = idx / nrep;
        int s_, q, qp;
        ring_item(idx - t * nrep, L, s_, q, qp);
        V v, vm;
        theta_pair<T, V, (LH < 16 ? LH : 16)>(dt + (int64_t)(t0 + t) * a.dstride, A_s, h_s, L, s_, q, qp, v, vm);
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
        for (int k = 1; k < L; ++k) {
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
            V* M = P + LH;
            if (qa == 0) {
                P[0] = Up;
                M[0] = vmk<V>(0, 0);
                for (int k = L; k < LH; ++k) { P[k] = vmk<V>(0, 0); M[k] = vmk<V>(0, 0); }
            } else {
                const V Um = side == 0 ? vadd(Xm, Ym) : vsub(Xm, Ym);
                P[qa] = vadd(Up, Um);
                M[qa] = vmul_mi(vsub(Up, Um));
            }
        }
    }
    __syncthreads();

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
                ma[kk] = (kk < kq && ra < nrows) ? prow[2 * (LH + k)] : T(0);
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

static int lh_bucket(int L) { return L <= 4 ? 4 : (L <= 8 ? 8 : (L <= 16 ? 16 : 32)); }

static size_t synth_xsize(const DevPlan& P, int tb) {
    const int LH = lh_bucket(P.d.L_h);
    const size_t rows = ((size_t)tb * P.d.n_omega + 7) / 8 * 8;
    return std::max((size_t)2 * LH * LH, rows * (2 * LH + 1));
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

template <typename T, int LH>
static const void* synth_fn_t(int nslot) {
    if constexpr (LH >= 16) {
        return (const void*)synth_full_kernel<T, LH, 1>;
    } else {
        const int ns = std::min((nslot + 63) / 64, ns_max(sizeof(T) == 8, LH));
        if constexpr (sizeof(T) == 8 && LH == 8) {
            return ns <= 1 ? (const void*)synth_full_kernel<T, LH, 1>
                 : ns == 2 ? (const void*)synth_full_kernel<T, LH, 2>
                           : (const void*)synth_full_kernel<T, LH, 3>;
        } else {
            return ns <= 1 ? (const void*)synth_full_kernel<T, LH, 1>
                 : ns == 2 ? (const void*)synth_full_kernel<T, LH, 2>
                 : ns == 3 ? (const void*)synth_full_kernel<T, LH, 3>
                           : (const void*)synth_full_kernel<T, LH, 4>;
        }
    }
}

static const void* synth_fn(const DevPlan& P) {
    const bool f64 = P.d.precision == SLSHT_FP64;
    const int ns = P.nslot_phi;
    switch (lh_bucket(P.d.L_h)) {
        case 4: return f64 ? synth_fn_t<double, 4>(ns) : synth_fn_t<float, 4>(ns);
        case 8: return f64 ? synth_fn_t<double, 8>(ns) : synth_fn_t<float, 8>(ns);
        case 16: return f64 ? synth_fn_t<double, 16>(ns) : synth_fn_t<float, 16>(ns);
        default: return f64 ? synth_fn_t<double, 32>(ns) : synth_fn_t<float, 32>(ns);
    }
}

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

hipError_t launch_synthesis(const DevPlan& P, const double2* A, const double2* h, void* g,
                            hipStream_t s) {
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
    const int64_t nblk = (int64_t)P.n_items * a.n_tiles;
    void* args[] = {&a};
    return hipLaunchKernel(synth_fn(P), dim3((unsigned)nblk), dim3(P.block), args, P.lds_bytes, s);
}

// ------------------------------------------------------------------------------
// K3e: energy epilogue, FP32.  One block = one degree l x one theta row; the order m
// runs inside the block and E(phi_a, theta_b, omega_c; l) = sum_m |g|^2 stays in
// registers until all orders are done, so g is never written.  Per m:
//   stage 1 (VALU): S_{q,q'}(theta_b) as in K3                              -> LDS
//   stage 2 (VALU): omega synthesis folded into P_k, M_k, stored k-major with
//                   omega contiguous (the B operand layout of the MFMA below)  -> LDS
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
};

constexpr int kEnergyWaves = 8;

template <int TPW>
__global__ void __launch_bounds__(64 * kEnergyWaves) energy_kernel(const EnergyArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int L = a.L, K = a.K, KK = K * K, KP = a.KP, cs_ = a.cstride;
    float2* A_s = reinterpret_cast<float2*>(smem_raw);
    float2* h_s = A_s + L * L;
    float2* S_s = h_s + L * L;
    float* PMt = reinterpret_cast<float*>(S_s + KK);          // [4][KP][cstride]
    float2* tw = reinterpret_cast<float2*>(PMt + 4 * KP * cs_);  // [n_phi] cos/sin(2 pi j/n_phi)
    const int ncw = (a.ncp + 15) / 16 * 16;                      // omega slots, padded
    const int nqt = (K + 15) / 16;                               // q tiles of the omega GEMM
    float2* twW = tw + a.n_phi;                                  // [KP][ncw] cos/sin(k omega_cs)
    float4* XY = reinterpret_cast<float4*>(twW + KP * ncw);      // [nqt*16][ncw] X, Y parts
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
    for (int i = tid; i < 4 * KP * cs_; i += nth) PMt[i] = 0.0f;
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

    const float* drow = a.dtab + (int64_t)t * a.dstride;
    const int nrep = ring_items(L);
    const int nm = a.real_pair ? l + 1 : 2 * l + 1;
    for (int mi = 0; mi < nm; ++mi) {
        const int m = a.real_pair ? mi : mi - l;
        const float wgt = (a.real_pair && m > 0) ? 2.0f : 1.0f;
        const int64_t lm = (int64_t)l * l + l + m - (int64_t)a.l_lo * a.l_lo;
        for (int i = tid; i < L * L; i += nth) A_s[i] = vcast<float2>(a.A[lm * L * L + i]);
        __syncthreads();

        // stage 1: theta contraction, ring-ordered items (see ring_item / theta_pair)
        for (int r = tid; r < nrep; r += nth) {
            int s_, q, qp;
            ring_item(r, L, s_, q, qp);
            float2 v, vm;
            theta_pair<float, float2, 8>(drow, A_s, h_s, L, s_, q, qp, v, vm);
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
            for (int kk = 0; kk < KP / 4; ++kk) {
                const int k = kk * 4 + kq2;
                float2 ap = vmk<float2>(0.0f, 0.0f), am = vmk<float2>(0.0f, 0.0f);
                if (qi < K && k < L) {
                    const float2* row = S_s + qi * K + (L - 1);
                    if (k == 0) {
                        ap = row[0];
                    } else {
                        const float2 s1 = row[k], s2 = row[-k];
                        ap = vadd(s1, s2);
                        am = vsub(s1, s2);
                    }
                }
                const float2 w = twW[k * ncw + ct2 * 16 + c16];
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
        float breg[4][8];
        {
            const int bcol = ct * 16 + col;
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                const int k = kk * 4 + kq;
#pragma unroll
                for (int part = 0; part < 4; ++part)
                    breg[part][kk] = kk < nkk ? PMt[(part * KP + k) * cs_ + bcol] : 0.0f;
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
            f4v cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0}, sre = {0, 0, 0, 0}, sim = {0, 0, 0, 0};
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                if (kk >= nkk) break;
                const float2 cz = tw[idx];
                cre = __builtin_amdgcn_mfma_f32_16x16x4f32(cz.x, breg[0][kk], cre, 0, 0, 0);
                cim = __builtin_amdgcn_mfma_f32_16x16x4f32(cz.x, breg[1][kk], cim, 0, 0, 0);
                sre = __builtin_amdgcn_mfma_f32_16x16x4f32(cz.y, breg[2][kk], sre, 0, 0, 0);
                sim = __builtin_amdgcn_mfma_f32_16x16x4f32(cz.y, breg[3][kk], sim, 0, 0, 0);
                idx += step4;
                if (idx >= a.n_phi) idx -= a.n_phi;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float pr = cre[r] + sre[r], pi = cim[r] + sim[r];
                const float mr = cre[r] - sre[r], mi2 = cim[r] - sim[r];
                Ep[j][r] += wgt * (pr * pr + pi * pi);
                Em[j][r] += wgt * (mr * mr + mi2 * mi2);
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
            row[s] = Ep[j][r];
            if (s > 0) row[a.n_phi - s] = Em[j][r];
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
    return (size_t)(2 * L * L + K * K) * sizeof(float2) + (size_t)4 * KP * cstride * sizeof(float) +
           (size_t)P.d.n_phi * sizeof(float2) + (size_t)KP * ncw * sizeof(float2) +
           (size_t)nqt * 16 * ncw * sizeof(float4);
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
    const size_t lds = energy_lds_bytes(P, a.KP, a.cstride);
    const int per = kEnergyWaves / a.nctp;           // waves sharing one omega tile
    const int tpw = (a.nst + per - 1) / per;
    dim3 grid(a.nblk), block(64 * kEnergyWaves);
    if (lds > 64 * 1024) {
        const void* fns[] = {(const void*)energy_kernel<4>, (const void*)energy_kernel<8>,
                             (const void*)energy_kernel<12>, (const void*)energy_kernel<17>};
        for (const void* fn : fns)
            (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    }
    if (tpw <= 4) hipLaunchKernelGGL(energy_kernel<4>, grid, block, lds, s, a);
    else if (tpw <= 8) hipLaunchKernelGGL(energy_kernel<8>, grid, block, lds, s, a);
    else if (tpw <= 12) hipLaunchKernelGGL(energy_kernel<12>, grid, block, lds, s, a);
    else if (tpw <= 17) hipLaunchKernelGGL(energy_kernel<17>, grid, block, lds, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

size_t energy_lds_for(const DevPlan& P) {
    const int KP = (P.d.L_h + 3) / 4 * 4;
    const int nct = (P.d.n_omega + 15) / 16;
    return energy_lds_bytes(P, KP, energy_cstride(nct == 3 ? 4 : nct));
}

// ------------------------------------------------------------------------------
// K4: inverse.  f_out[lm] = scale * sum_{c,b,a} q(theta_b) g[lm][c][b][a], one block per lm,
// FP64 accumulation, wavefront shuffle + LDS reduction.

template <typename V>
__global__ void __launch_bounds__(256) inverse_kernel(const V* __restrict__ g,
                                                      const double* __restrict__ qw, int n_phi,
                                                      int n_theta, int n_omega, double2 scale,
                                                      double2* __restrict__ f_out) {
    __shared__ double qs[(SLSHT_MAX_NPHI + 1) / 2];
    __shared__ double red[2][8];
    for (int i = threadIdx.x; i < n_theta; i += blockDim.x) qs[i] = qw[i];
    __syncthreads();
    const int64_t n = (int64_t)n_omega * n_theta * n_phi;
    const V* gp = g + (int64_t)blockIdx.x * n;
    double ar = 0.0, ai = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int b = (int)((i / n_phi) % n_theta);
        const V v = gp[i];
        ar += qs[b] * (double)v.x;
        ai += qs[b] * (double)v.y;
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
        double2 o;
        o.x = scale.x * sr - scale.y * si;
        o.y = scale.x * si + scale.y * sr;
        f_out[blockIdx.x] = o;
    }
}

hipError_t launch_inverse(const DevPlan& P, const void* g, double2 scale, double2* f_out,
                          hipStream_t s) {
    const int n_lm = P.d.l_hi * P.d.l_hi - P.d.l_lo * P.d.l_lo;
    if (P.d.precision == SLSHT_FP64)
        hipLaunchKernelGGL(inverse_kernel<double2>, dim3(n_lm), dim3(256), 0, s,
                           (const double2*)g, P.T->qw, P.d.n_phi, P.d.n_theta, P.d.n_omega, scale, f_out);
    else
        hipLaunchKernelGGL(inverse_kernel<float2>, dim3(n_lm), dim3(256), 0, s,
                           (const float2*)g, P.T->qw, P.d.n_phi, P.d.n_theta, P.d.n_omega, scale, f_out);
    return hipGetLastError();
}

}  // namespace slsht
