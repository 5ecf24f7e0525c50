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

// Row offset of W_q (rows p = |q| .. L-1) inside one theta row of the W table of the
// ENERGY and staged FULL paths, with q ordered 0, +1, -1, +2, -2, ...; W_{+k} and W_{-k} are
// adjacent (2 (L-k) rows for k >= 1), and a theta row holds L^2 rows in all.
__host__ __device__ inline int wq_off(int L, int q) {
    if (q == 0) return 0;
    const int k = q > 0 ? q : -q;
    const int base = L + (k - 1) * (2 * L - k);
    return q > 0 ? base : base + (L - k);
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

// Theta-stage items for a window with azimuthal band-limit N (S_{q,q'} = 0 for
// |q'| >= N, so only |q'| < N is computed).  N = L: the ring order above.  N < L
// (steerable window): q' = 0 with q = 0..L-1 first, then q' = 1..N-1 with every q; each
// item again covers (q, q') and (-q, -q').
__device__ __forceinline__ int theta_items(int L, int N) {
    return N >= L ? ring_items(L) : L + (N - 1) * (2 * L - 1);
}

__device__ __forceinline__ void theta_item(int r, int L, int N, int& s, int& q, int& qp) {
    if (N >= L) {
        ring_item(r, L, s, q, qp);
        return;
    }
    if (r < L) {
        q = r;
        qp = 0;
    } else {
        const int K = 2 * L - 1, x = r - L;
        qp = 1 + x / K;
        q = x - (qp - 1) * K - (L - 1);
    }
    const int aq = q < 0 ? -q : q;
    s = aq > qp ? aq : qp;
}

// Item of thread `tid` in round j of a block-wide loop over `total` items (valid when
// tid < min(nth, total - j*nth)).  Rounds alternate direction: with items sorted by trip
// count, a thread's long items pair with short ones and the per-thread totals even out.
__device__ __forceinline__ int snake_item(int j, int tid, int nth, int total) {
    const int base = j * nth;
    const int cnt = total - base < nth ? total - base : nth;
    return base + ((j & 1) ? cnt - 1 - tid : tid);
}

// Canonical table entry of d^p_{q,q'}: d_{q,q'} = sign * d_{Q,Q'} with Q = max(|q|,|q'|)
// >= |Q'|, from d_{q,q'} = (-1)^{q-q'} d_{q',q} = d_{-q',-q} (symmetries of Section IV-B).
__device__ __forceinline__ void d_canonical(int q, int qp, int& Q, int& Qp, bool& neg) {
    const int aq = q < 0 ? -q : q, aqp = qp < 0 ? -qp : qp;
    const bool odd = ((q - qp) & 1) != 0;
    if (aq >= aqp) {
        if (q >= 0) { Q = q; Qp = qp; neg = false; }
        else { Q = -q; Qp = -qp; neg = odd; }
    } else {
        if (qp > 0) { Q = qp; Qp = q; neg = odd; }
        else { Q = -qp; Qp = -q; neg = false; }
    }
}

// S_{q,q'} and S_{-q,-q'} of one theta row for the ring item (s, q, q'), from the
// canonical Wigner-d row (global memory or LDS).  Offsets into the row advance by
// additions; the d, A and h values of PF consecutive degrees are loaded together before
// they are used, so an item waits for memory ceil((L-s)/PF) times rather than L-s times.
template <typename T, typename V, int PF>
__device__ __forceinline__ void theta_pair(const T* __restrict__ drow, const V* A_s, const V* h_s,
                                           int L, int s, int q, int qp, V& out, V& mirror) {
    int Q, Qp;
    bool neg;
    d_canonical(q, qp, Q, Qp, neg);                  // Q == s
    int off = dtab_off(s) + Q * Q + Q + Qp;
    T sr = 0, si = 0, tr = 0, ti = 0;
    for (int p0 = s; p0 < L; p0 += PF) {
        // all loads of PF degrees first, branch-free: degrees past L read valid entries
        // (of degree L-1) and are weighted by zero
        T dv[PF];
        V a1[PF], h1[PF], a2[PF], h2[PF];
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int p = p0 + i;
            const bool ok = p < L;
            const int pe = ok ? p : L - 1;
            const int ia = pe * pe + pe;
            const T x = drow[ok ? off : 0];
            dv[i] = ok ? x : T(0);
            a1[i] = A_s[ia + q];
            h1[i] = h_s[ia + qp];
            a2[i] = A_s[ia - q];
            h2[i] = h_s[ia - qp];
            off += (p + 1) * (p + 1);
        }
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            sr += (a1[i].x * h1[i].x - a1[i].y * h1[i].y) * dv[i];
            si += (a1[i].x * h1[i].y + a1[i].y * h1[i].x) * dv[i];
            tr += (a2[i].x * h2[i].x - a2[i].y * h2[i].y) * dv[i];
            ti += (a2[i].x * h2[i].y + a2[i].y * h2[i].x) * dv[i];
        }
    }
    const T sg = neg ? T(-1) : T(1);
    const T sgm = ((q - qp) & 1) ? -sg : sg;
    out = vmk<V>(sg * sr, sg * si);
    mirror = vmk<V>(sgm * tr, sgm * ti);
}

}  // namespace slsht
