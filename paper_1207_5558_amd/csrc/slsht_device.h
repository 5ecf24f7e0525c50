// Device helpers shared by the gfx950 kernels: interleaved complex arithmetic, the
// (l, m) index map and the ring-ordered theta contraction of the synthesis kernels.
#pragma once

#include "slsht_internal.h"

#include <hip/hip_runtime.h>

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

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

// Flat coefficient index l^2 + l + m -> (l, m).
__device__ __forceinline__ void lm_of(int lm_abs, int& l, int& m) {
    int ll = (int)sqrt((double)lm_abs);
    while (ll * ll > lm_abs) --ll;
    while ((ll + 1) * (ll + 1) <= lm_abs) ++ll;
    l = ll;
    m = lm_abs - ll * ll - ll;
}

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

}  // namespace slsht
