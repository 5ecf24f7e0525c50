// Host core of the directional SLSHT library: descriptor checks, footprints,
// device tables, plans, and the forward / coupling / inverse entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "slsht_internal.h"

namespace {

thread_local std::string g_err;

int hip_fail(hipError_t e, const char* what) {
    return slsht::set_error(SLSHT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool mul_ok(size_t a, size_t b, size_t& r) {
    if (a != 0 && b > std::numeric_limits<size_t>::max() / a) return false;
    r = a * b;
    return true;
}

int theta_hi_of(const slsht_desc& d) { return d.theta_hi == 0 ? d.n_theta : d.theta_hi; }

// Beta weights q(beta_b), Section IV-A (definitions of q(beta) and w(m) after
// eq. Eq:sig_reconstruction_discrete), with L = (n_phi - 1) / 2.  Only even m
// contribute for beta != 0 (the m = +-1 terms cancel in the cosine sum).
void beta_weights(int n_phi, int n_theta, std::vector<double>& q) {
    const int L = (n_phi - 1) / 2;
    q.assign(n_theta, 0.0);
    const double pi = M_PI;
    for (int b = 0; b < n_theta; ++b) {
        if (b == 0) {
            q[b] = 4.0 * pi * pi / (std::floor(L / 2.0) + 0.5);
            continue;
        }
        double sum = 0.0;
        for (int m = -L; m <= L; ++m) {
            if (m & 1) continue;
            // cos(m beta) with beta = 2 pi b / n_phi, phase reduced exactly in integers
            const long long k = ((long long)m * b) % n_phi;
            sum += 2.0 / (1.0 - (double)m * m) * std::cos(2.0 * pi * (double)k / n_phi);
        }
        q[b] = 8.0 * pi * pi * sum;
    }
}

template <typename T>
void twiddles(int L, int n, int nslot, std::vector<T>& out) {
    // out[(k-1)*nslot + s] = (cos, sin)(2 pi k s / n), k = 1..L-1; phase reduced in integers
    const int rows = L > 1 ? L - 1 : 1;
    out.assign((size_t)rows * nslot * 2, T(0));
    for (int k = 1; k < L; ++k)
        for (int s = 0; s < nslot; ++s) {
            const long long r = ((long long)k * s) % n;
            const double ang = 2.0 * M_PI * (double)r / (double)n;
            out[((size_t)(k - 1) * nslot + s) * 2 + 0] = (T)std::cos(ang);
            out[((size_t)(k - 1) * nslot + s) * 2 + 1] = (T)std::sin(ang);
        }
}

struct TableSizes {
    size_t dtab, twphi, twom, twfull, qw;
    size_t total() const { return dtab + twphi + twom + twfull + qw; }
};

// ENERGY tiles for table sizes: independent of the LDS split.
slsht::EnergyGeom energy_tiles(const slsht_desc& d) {
    slsht::EnergyGeom g{};
    (void)slsht::energy_geom(d, theta_hi_of(d) - d.theta_lo, (size_t)1 << 30, g);
    return g;
}

TableSizes table_sizes(const slsht_desc& d) {
    TableSizes t;
    const bool energy = d.output_mode == SLSHT_OUT_ENERGY;
    const bool f64 = d.precision == SLSHT_FP64;
    const size_t rb = (f64 || energy) ? 8 : 4, vb = f64 ? 16 : 8;
    const int L = d.L_h;
    const size_t nslot = (size_t)(d.n_phi + 1) / 2, ncp = (size_t)d.n_omega / 2 + 1;
    const size_t rows = (size_t)(L > 1 ? L - 1 : 1);
    t.dtab = (size_t)(theta_hi_of(d) - d.theta_lo) * (size_t)slsht::dtab_row_len(L) * rb;
    t.twphi = energy ? 0 : rows * nslot * vb;
    t.twom = energy ? 0 : rows * ncp * vb;
    t.twfull = energy ? slsht::energy_twiddle_bytes(energy_tiles(d)) : 0;
    t.qw = (size_t)d.n_theta * sizeof(double);
    return t;
}

}  // namespace

namespace slsht {

int set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

Tables::~Tables() {
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != device) (void)hipSetDevice(device);
    void* ptrs[] = {dtab, tw_phi, tw_omega, tw_full, qw};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
}

int check_desc(const slsht_desc* d) {
    if (!d) return set_error(SLSHT_EINVAL, "desc is NULL");
    if (d->L_f < 1 || d->L_f > SLSHT_MAX_LF)
        return set_error(SLSHT_EINVAL, "L_f=%d outside [1, %d]", d->L_f, SLSHT_MAX_LF);
    if (d->L_h < 1 || d->L_h > SLSHT_MAX_LH)
        return set_error(SLSHT_EINVAL, "L_h=%d outside [1, %d]", d->L_h, SLSHT_MAX_LH);
    if (d->l_lo < 0 || d->l_hi <= d->l_lo || d->l_hi > d->L_f + d->L_h - 1)
        return set_error(SLSHT_EINVAL,
                         "need 0 <= l_lo < l_hi <= L_f + L_h - 1 (got l_lo=%d l_hi=%d)", d->l_lo,
                         d->l_hi);
    if (d->n_phi < 1 || d->n_phi > SLSHT_MAX_NPHI || (d->n_phi % 2) == 0)
        return set_error(SLSHT_EINVAL, "n_phi=%d must be odd and in [1, %d]", d->n_phi,
                         SLSHT_MAX_NPHI);
    if (d->n_theta != (d->n_phi + 1) / 2)
        return set_error(SLSHT_EINVAL, "n_theta=%d must equal (n_phi + 1) / 2 = %d", d->n_theta,
                         (d->n_phi + 1) / 2);
    if (d->n_omega < 1 || d->n_omega > 4096)
        return set_error(SLSHT_EINVAL, "n_omega=%d outside [1, 4096]", d->n_omega);
    if (d->precision != SLSHT_FP64 && d->precision != SLSHT_FP32_MIXED)
        return set_error(SLSHT_EINVAL, "unknown precision %d", d->precision);
    if (d->output_mode != SLSHT_OUT_FULL && d->output_mode != SLSHT_OUT_ENERGY)
        return set_error(SLSHT_EINVAL, "unknown output_mode %d", d->output_mode);
    if (d->flags & ~(uint32_t)SLSHT_REAL_PAIR)
        return set_error(SLSHT_EINVAL, "unknown flags 0x%x", d->flags);
    if (d->n_az < 0 || d->n_az > d->L_h)
        return set_error(SLSHT_EINVAL, "n_az=%d outside [0, L_h=%d]", d->n_az, d->L_h);
    const int thi = theta_hi_of(*d);
    if (d->theta_lo < 0 || thi <= d->theta_lo || thi > d->n_theta)
        return set_error(SLSHT_EINVAL, "need 0 <= theta_lo < theta_hi <= n_theta (got %d, %d)",
                         d->theta_lo, d->theta_hi);
    if (d->output_mode == SLSHT_OUT_ENERGY) {
        if (d->precision != SLSHT_FP32_MIXED)
            return set_error(SLSHT_EINVAL, "ENERGY output needs precision SLSHT_FP32_MIXED");
        if (d->n_omega > kEnergyMaxOmega)
            return set_error(SLSHT_EINVAL, "ENERGY output needs n_omega <= %d", kEnergyMaxOmega);
        const int nst = ((d->n_phi + 1) / 2 + 15) / 16, nct = (d->n_omega + 15) / 16;
        const int nctp = nct == 3 ? 4 : nct;      // omega tiles padded to divide the 8 waves
        if (nst * nctp > kEnergyMaxTiles)
            return set_error(SLSHT_EINVAL,
                             "ENERGY output needs ceil(((n_phi+1)/2)/16) * T <= %d with T = "
                             "ceil(n_omega/16) rounded up to 1, 2 or 4 (n_phi <= 1087 at "
                             "n_omega > 32)", kEnergyMaxTiles);
    }
    size_t out;
    const int64_t n_lm = (int64_t)d->l_hi * d->l_hi - (int64_t)d->l_lo * d->l_lo;
    const int64_t n_l = d->l_hi - d->l_lo;
    const size_t per = d->output_mode == SLSHT_OUT_FULL
                           ? (size_t)n_lm * (d->precision == SLSHT_FP64 ? 16 : 8)
                           : (size_t)n_l * (d->precision == SLSHT_FP64 ? 8 : 4);
    const size_t n_rho = (size_t)d->n_phi * (thi - d->theta_lo) * d->n_omega;
    if (!mul_ok(per, n_rho, out)) return set_error(SLSHT_EINVAL, "output size overflows size_t");
    return SLSHT_OK;
}

size_t tables_bytes(const slsht_desc& d) { return table_sizes(d).total(); }

size_t workspace_bytes(const slsht_desc& d) {
    const int n_theta_out = theta_hi_of(d) - d.theta_lo;
    if (d.output_mode == SLSHT_OUT_FULL) {
        const int64_t n_items = (d.flags & SLSHT_REAL_PAIR)
                                    ? (int64_t)d.l_hi * (d.l_hi + 1) / 2 - (int64_t)d.l_lo * (d.l_lo + 1) / 2
                                    : (int64_t)d.l_hi * d.l_hi - (int64_t)d.l_lo * d.l_lo;
        StagedGeom g{};
        return staged_geom(d, n_theta_out, (int)n_items, g) ? g.total : 0;
    }
    // ENERGY: the largest over the LDS sizes a device may report (64 KiB to 160 KiB)
    size_t best = 0;
    for (size_t lds : {(size_t)64 << 10, (size_t)160 << 10}) {
        EnergyGeom g{};
        if (energy_geom(d, n_theta_out, lds, g)) best = std::max(best, g.total);
    }
    return best;
}

size_t plan_workspace_bytes(const DevPlan& P) {
    if (P.d.output_mode == SLSHT_OUT_ENERGY) return P.eg.total;
    return P.staged ? P.sg.total : 0;
}

size_t coupling_bytes(const slsht_desc& d) {
    const size_t n_lm = (size_t)d.l_hi * d.l_hi - (size_t)d.l_lo * d.l_lo;
    return n_lm * d.L_h * d.L_h * sizeof(double2);
}

size_t output_bytes(const slsht_desc& d) {
    const size_t n_rho = (size_t)d.n_phi * (theta_hi_of(d) - d.theta_lo) * d.n_omega;
    if (d.output_mode == SLSHT_OUT_FULL) {
        const size_t n_lm = (size_t)d.l_hi * d.l_hi - (size_t)d.l_lo * d.l_lo;
        return n_lm * n_rho * (d.precision == SLSHT_FP64 ? 16 : 8);
    }
    return (size_t)(d.l_hi - d.l_lo) * n_rho * (d.precision == SLSHT_FP64 ? 8 : 4);
}

std::string tables_key(const slsht_desc& d) {
    char buf[160];
    snprintf(buf, sizeof buf, "%d/%d/%d/%d/%d/%d/%d", d.L_h, d.n_phi, d.n_omega, d.theta_lo,
             theta_hi_of(d), d.precision, d.output_mode);
    return buf;
}

size_t device_lds_limit(int device) {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
            hipSuccess || lds <= 0)
        lds = 64 * 1024;
    return (size_t)lds;
}

int make_view(const slsht_desc& d, const std::shared_ptr<Tables>& T, size_t lds_limit,
              DevPlan& P) {
    P.d = d;
    P.d.theta_hi = theta_hi_of(d);
    P.T = T;
    P.n_theta_out = P.d.theta_hi - P.d.theta_lo;
    P.nslot_phi = (P.d.n_phi + 1) / 2;
    P.ncp_omega = P.d.n_omega / 2 + 1;
    P.n_lm = (int64_t)P.d.l_hi * P.d.l_hi - (int64_t)P.d.l_lo * P.d.l_lo;
    if (P.d.flags & SLSHT_REAL_PAIR) {
        const int64_t a = (int64_t)P.d.l_hi * (P.d.l_hi + 1) / 2;
        const int64_t b = (int64_t)P.d.l_lo * (P.d.l_lo + 1) / 2;
        P.n_items = (int)(a - b);
    } else {
        P.n_items = (int)P.n_lm;
    }
    P.staged = P.d.output_mode == SLSHT_OUT_FULL &&
               staged_geom(P.d, P.n_theta_out, P.n_items, P.sg);
    if (P.d.output_mode == SLSHT_OUT_FULL && !choose_synthesis_shape(P, lds_limit))
        return set_error(SLSHT_EINVAL, "no synthesis tiling fits %zu bytes of LDS", lds_limit);
    if (P.d.output_mode == SLSHT_OUT_ENERGY &&
        (!energy_geom(P.d, P.n_theta_out, lds_limit, P.eg) || energy_lds_for(P) > lds_limit))
        return set_error(SLSHT_EINVAL, "no ENERGY tiling fits %zu bytes of LDS", lds_limit);
    return SLSHT_OK;
}

int build_tables(const slsht_desc& d, int device, std::shared_ptr<Tables>& out) {
    const TableSizes ts = table_sizes(d);
    auto T = std::make_shared<Tables>();
    T->device = device;
    T->L_h = d.L_h;
    T->n_phi = d.n_phi;
    T->n_theta = d.n_theta;
    T->n_omega = d.n_omega;
    T->theta_lo = d.theta_lo;
    T->theta_hi = theta_hi_of(d);
    T->precision = d.precision;
    T->energy = d.output_mode == SLSHT_OUT_ENERGY;
    T->bytes = ts.total();
    hipError_t e = hipSuccess;
    auto alloc = [&](void** p, size_t n) {
        if (e == hipSuccess && n) e = hipMalloc(p, n);
    };
    alloc(&T->dtab, ts.dtab);
    alloc(&T->tw_phi, ts.twphi);
    alloc(&T->tw_omega, ts.twom);
    alloc(&T->tw_full, ts.twfull);
    alloc((void**)&T->qw, ts.qw);
    if (e != hipSuccess)
        return set_error(SLSHT_ENOMEM, "table allocation failed: %s", hipGetErrorString(e));

    const int nslot = (d.n_phi + 1) / 2, ncp = d.n_omega / 2 + 1;
    if (T->energy) {
        // (cos, sin)(k phi_a) in the fragment order of the ENERGY phi stage
        std::vector<float> tf;
        energy_twiddles(energy_tiles(d), tf);
        e = hipMemcpy(T->tw_full, tf.data(), ts.twfull, hipMemcpyHostToDevice);
    } else if (d.precision == SLSHT_FP64) {
        std::vector<double> tp, to;
        twiddles(d.L_h, d.n_phi, nslot, tp);
        twiddles(d.L_h, d.n_omega, ncp, to);
        e = hipMemcpy(T->tw_phi, tp.data(), ts.twphi, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(T->tw_omega, to.data(), ts.twom, hipMemcpyHostToDevice);
    } else {
        std::vector<float> tp, to;
        twiddles(d.L_h, d.n_phi, nslot, tp);
        twiddles(d.L_h, d.n_omega, ncp, to);
        e = hipMemcpy(T->tw_phi, tp.data(), ts.twphi, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(T->tw_omega, to.data(), ts.twom, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) {
        std::vector<double> qw;
        beta_weights(d.n_phi, d.n_theta, qw);
        e = hipMemcpy(T->qw, qw.data(), ts.qw, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return hip_fail(e, "table upload");
    // Wigner-d table on the device, on a private stream
    DevPlan P;
    P.d = d;
    P.d.theta_hi = theta_hi_of(d);
    P.T = T;
    P.n_theta_out = P.d.theta_hi - P.d.theta_lo;
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = launch_wigner_table(P, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (s) (void)hipStreamDestroy(s);
    if (e != hipSuccess) return hip_fail(e, "Wigner-d table build");
    out = T;
    return SLSHT_OK;
}

hipError_t enqueue_forward(const DevPlan& P, const double2* f, const double2* h, void* g,
                           double2* A, hipStream_t s) {
    hipError_t e = launch_coupling(P, f, A, s);
    if (e != hipSuccess) return e;
    if (P.d.output_mode == SLSHT_OUT_FULL) return launch_synthesis(P, A, h, g, s);
    return launch_energy(P, A, h, (float*)g, s);
}

}  // namespace slsht

using slsht::DeviceGuard;

extern "C" {

const char* slsht_last_error(void) { return g_err.c_str(); }

int slsht_validate(const slsht_desc* desc) { return slsht::check_desc(desc); }

int slsht_footprint(const slsht_desc* desc, size_t* plan_bytes, size_t* out_bytes,
                    size_t* scratch_bytes) {
    int rc = slsht::check_desc(desc);
    if (rc) return rc;
    if (plan_bytes)
        *plan_bytes = slsht::tables_bytes(*desc) + slsht::coupling_bytes(*desc) +
                      slsht::workspace_bytes(*desc);
    if (out_bytes) *out_bytes = slsht::output_bytes(*desc);
    if (scratch_bytes) *scratch_bytes = 0;
    return SLSHT_OK;
}

int64_t slsht_coupling_size(const slsht_desc* desc) {
    if (slsht::check_desc(desc)) return -1;
    return (int64_t)(slsht::coupling_bytes(*desc) / sizeof(double2));
}

int slsht_plan(const slsht_desc* desc, int device, slsht_plan_t* out) {
    if (!out) return slsht::set_error(SLSHT_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = slsht::check_desc(desc);
    if (rc) return rc;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
        return slsht::set_error(SLSHT_EDEVICE, "no HIP device available");
    if (device < 0 || device >= ndev)
        return slsht::set_error(SLSHT_EINVAL, "device %d out of range", device);
    DeviceGuard guard(device);
    if (!guard.ok) return slsht::set_error(SLSHT_EDEVICE, "hipSetDevice(%d) failed", device);
    void* noalloc_ptr = nullptr;      // set-up of slsht_forward_noalloc's scratch address
    rc = slsht::noalloc_scratch(device, &noalloc_ptr);
    if (rc) return rc;

    std::shared_ptr<slsht::Tables> T;
    rc = slsht::build_tables(*desc, device, T);
    if (rc) return rc;
    slsht_plan_s* pl = new slsht_plan_s();
    pl->device = device;
    rc = slsht::make_view(*desc, T, slsht::device_lds_limit(device), pl->P);
    if (rc) {
        delete pl;
        return rc;
    }
    hipError_t e = hipMalloc((void**)&pl->P.A, slsht::coupling_bytes(*desc));
    const size_t wsb = slsht::plan_workspace_bytes(pl->P);
    if (e == hipSuccess && wsb) e = hipMalloc(&pl->P.ework, wsb);
    if (e != hipSuccess) {
        if (pl->P.A) (void)hipFree(pl->P.A);
        delete pl;
        return slsht::set_error(SLSHT_ENOMEM, "coupling scratch / workspace: %s",
                                hipGetErrorString(e));
    }
    *out = pl;
    return SLSHT_OK;
}

int slsht_plan_destroy(slsht_plan_t plan) {
    if (!plan) return slsht::set_error(SLSHT_EINVAL, "plan is NULL");
    {
        DeviceGuard guard(plan->device);
        (void)hipDeviceSynchronize();
        if (plan->P.A) (void)hipFree(plan->P.A);
        if (plan->P.ework) (void)hipFree(plan->P.ework);
    }
    delete plan;
    return SLSHT_OK;
}

int slsht_plan_desc(slsht_plan_t plan, slsht_desc* out) {
    if (!plan || !out) return slsht::set_error(SLSHT_EINVAL, "NULL argument");
    *out = plan->P.d;
    return SLSHT_OK;
}

int slsht_coupling(slsht_plan_t plan, const void* f, void* A, void* stream) {
    if (!plan || !f || !A) return slsht::set_error(SLSHT_EINVAL, "NULL argument");
    DeviceGuard guard(plan->device);
    if (!guard.ok) return slsht::set_error(SLSHT_EDEVICE, "hipSetDevice failed");
    hipError_t e = slsht::launch_coupling(plan->P, (const double2*)f, (double2*)A,
                                          (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "coupling launch");
    return SLSHT_OK;
}

int slsht_synthesize(slsht_plan_t plan, const void* A, const void* h, void* g, void* stream) {
    if (!plan || !A || !h || !g) return slsht::set_error(SLSHT_EINVAL, "NULL argument");
    DeviceGuard guard(plan->device);
    if (!guard.ok) return slsht::set_error(SLSHT_EDEVICE, "hipSetDevice failed");
    const slsht::DevPlan& P = plan->P;
    hipStream_t s = (hipStream_t)stream;
    const hipError_t e =
        P.d.output_mode == SLSHT_OUT_FULL
            ? slsht::launch_synthesis(P, (const double2*)A, (const double2*)h, g, s)
            : slsht::launch_energy(P, (const double2*)A, (const double2*)h, (float*)g, s);
    if (e != hipSuccess) return hip_fail(e, "synthesis launch");
    return SLSHT_OK;
}

int slsht_forward(slsht_plan_t plan, const void* f, const void* h, void* g, void* stream) {
    if (!plan || !f || !h || !g) return slsht::set_error(SLSHT_EINVAL, "NULL argument");
    DeviceGuard guard(plan->device);
    if (!guard.ok) return slsht::set_error(SLSHT_EDEVICE, "hipSetDevice failed");
    hipError_t e = slsht::enqueue_forward(plan->P, (const double2*)f, (const double2*)h, g,
                                          plan->P.A, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    return SLSHT_OK;
}

int slsht_forward_batch(int n, const slsht_plan_t* plans, const void* const* f,
                        const void* const* h, void* const* g, void* stream) {
    if (n < 1) return slsht::set_error(SLSHT_EINVAL, "n=%d < 1", n);
    if (!plans || !f || !h || !g) return slsht::set_error(SLSHT_EINVAL, "NULL argument");
    for (int i = 0; i < n; ++i) {
        if (!plans[i] || !f[i] || !h[i] || !g[i])
            return slsht::set_error(SLSHT_EINVAL, "NULL entry %d", i);
        if (plans[i]->device != plans[0]->device)
            return slsht::set_error(SLSHT_EINVAL, "plan %d is on device %d, plan 0 on %d", i,
                                    plans[i]->device, plans[0]->device);
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i])
                return slsht::set_error(SLSHT_EINVAL, "plan %d repeats plan %d (one coupling "
                                        "scratch per plan)", i, j);
    }
    DeviceGuard guard(plans[0]->device);
    if (!guard.ok) return slsht::set_error(SLSHT_EDEVICE, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    for (int i = 0; i < n && e == hipSuccess; ++i)
        e = slsht::launch_coupling(plans[i]->P, (const double2*)f[i], plans[i]->P.A, s);
    // FULL transforms grouped by synthesis kernel, up to kSynthBatchMax per grid
    std::vector<char> done(n, 0);
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        if (done[i]) continue;
        const slsht::DevPlan& Pi = plans[i]->P;
        if (Pi.d.output_mode != SLSHT_OUT_FULL) {
            e = slsht::launch_energy(Pi, Pi.A, (const double2*)h[i], (float*)g[i], s);
            done[i] = 1;
            continue;
        }
        const void* key = slsht::synthesis_kernel_key(Pi);
        std::vector<const slsht::DevPlan*> P;
        std::vector<const double2*> A, H;
        std::vector<void*> G;
        for (int j = i; j < n && (int)P.size() < slsht::kSynthBatchMax; ++j) {
            const slsht::DevPlan& Pj = plans[j]->P;
            if (done[j] || Pj.d.output_mode != SLSHT_OUT_FULL ||
                slsht::synthesis_kernel_key(Pj) != key || Pj.block != Pi.block)
                continue;
            P.push_back(&Pj);
            A.push_back(Pj.A);
            H.push_back((const double2*)h[j]);
            G.push_back(g[j]);
            done[j] = 1;
        }
        e = slsht::launch_synthesis_batch(P.data(), A.data(), H.data(), G.data(), (int)P.size(), s);
    }
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    return SLSHT_OK;
}

int slsht_forward_windows(slsht_plan_t plan, const void* f, const void* h, int n_windows,
                          void* g, void* stream) {
    if (!plan || !f || !h || !g) return slsht::set_error(SLSHT_EINVAL, "NULL argument");
    if (n_windows < 1) return slsht::set_error(SLSHT_EINVAL, "n_windows=%d < 1", n_windows);
    DeviceGuard guard(plan->device);
    if (!guard.ok) return slsht::set_error(SLSHT_EDEVICE, "hipSetDevice failed");
    const slsht::DevPlan& P = plan->P;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = slsht::launch_coupling(P, (const double2*)f, P.A, s);
    if (e != hipSuccess) return hip_fail(e, "coupling launch");
    const size_t hn = (size_t)P.d.L_h * P.d.L_h;
    const size_t ob = slsht::output_bytes(P.d);
    for (int w = 0; w < n_windows; ++w) {
        const double2* hw = (const double2*)h + w * hn;
        void* gw = (char*)g + w * ob;
        e = P.d.output_mode == SLSHT_OUT_FULL ? slsht::launch_synthesis(P, P.A, hw, gw, s)
                                              : slsht::launch_energy(P, P.A, hw, (float*)gw, s);
        if (e != hipSuccess) return hip_fail(e, "synthesis launch");
    }
    return SLSHT_OK;
}

static bool factored_eligible(const slsht_desc& d) {
    return d.output_mode == SLSHT_OUT_FULL && d.precision == SLSHT_FP64 && d.flags == 0 &&
           (d.n_az == 0 || d.n_az == d.L_h) && d.n_phi == 2 * d.L_h - 1 &&
           d.n_omega == 2 * d.L_h - 1 && d.theta_lo == 0 && theta_hi_of(d) == d.n_theta &&
           ((int64_t)d.l_hi * d.l_hi - (int64_t)d.l_lo * d.l_lo) * d.L_h <= 0x7fffffff;
}

int64_t slsht_factored_workspace(const slsht_desc* desc) {
    if (slsht::check_desc(desc) != SLSHT_OK) return -1;
    if (!factored_eligible(*desc)) {
        slsht::set_error(SLSHT_EINVAL, "the factored route needs a FULL FP64 plan on the minimal "
                                       "grid n_phi = n_omega = 2 L_h - 1, all theta rows, no flags, "
                                       "at most 2^31 - 1 (l, m, theta) rows");
        return -1;
    }
    return (int64_t)slsht::factored_workspace_bytes(*desc);
}

int slsht_forward_factored(slsht_plan_t plan, const void* f, const void* h, void* g, void* work,
                           size_t work_bytes, void* stream) {
    if (!plan || !f || !h || !g || !work) return slsht::set_error(SLSHT_EINVAL, "NULL argument");
    const slsht::DevPlan& P = plan->P;
    const int64_t need = slsht_factored_workspace(&P.d);
    if (need < 0) return SLSHT_EINVAL;
    if (work_bytes < (size_t)need)
        return slsht::set_error(SLSHT_EINVAL, "workspace of %zu bytes, needs %lld", work_bytes,
                                (long long)need);
    DeviceGuard guard(plan->device);
    if (!guard.ok) return slsht::set_error(SLSHT_EDEVICE, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = slsht::launch_coupling(P, (const double2*)f, P.A, s);
    if (e == hipSuccess) e = slsht::launch_factored(P, P.A, (const double2*)h, (double2*)g, work, s);
    if (e != hipSuccess) return hip_fail(e, "factored route launch");
    return SLSHT_OK;
}

int slsht_synthesize_factored(slsht_plan_t plan, const void* A, const void* h, void* g,
                              void* work, size_t work_bytes, void* stream) {
    if (!plan || !A || !h || !g || !work) return slsht::set_error(SLSHT_EINVAL, "NULL argument");
    const slsht::DevPlan& P = plan->P;
    const int64_t need = slsht_factored_workspace(&P.d);
    if (need < 0) return SLSHT_EINVAL;
    if (work_bytes < (size_t)need)
        return slsht::set_error(SLSHT_EINVAL, "workspace of %zu bytes, needs %lld", work_bytes,
                                (long long)need);
    DeviceGuard guard(plan->device);
    if (!guard.ok) return slsht::set_error(SLSHT_EDEVICE, "hipSetDevice failed");
    hipError_t e = slsht::launch_factored(P, (const double2*)A, (const double2*)h, (double2*)g,
                                          work, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "factored synthesis launch");
    return SLSHT_OK;
}

int slsht_wigner_delta(int L_h, int device, void* delta, void* stream) {
    if (!delta) return slsht::set_error(SLSHT_EINVAL, "delta is NULL");
    if (L_h < 1 || L_h > SLSHT_MAX_LH)
        return slsht::set_error(SLSHT_EINVAL, "L_h=%d outside [1, %d]", L_h, SLSHT_MAX_LH);
    DeviceGuard guard(device);
    if (!guard.ok) return slsht::set_error(SLSHT_EDEVICE, "hipSetDevice(%d) failed", device);
    hipError_t e = slsht::launch_delta_trapani(L_h, (double*)delta, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "Delta launch");
    return SLSHT_OK;
}

int64_t slsht_modulated_workspace(const slsht_desc* desc) {
    if (slsht::check_desc(desc) != SLSHT_OK) return -1;
    return (int64_t)slsht::modulated_workspace_bytes(*desc);
}

int slsht_coupling_modulated(slsht_plan_t plan, const void* f, void* A, void* work,
                             size_t work_bytes, void* stream) {
    if (!plan || !f || !A || !work) return slsht::set_error(SLSHT_EINVAL, "NULL argument");
    const slsht::DevPlan& P = plan->P;
    const size_t need = slsht::modulated_workspace_bytes(P.d);
    if (work_bytes < need)
        return slsht::set_error(SLSHT_EINVAL, "workspace of %zu bytes, needs %zu", work_bytes,
                                need);
    DeviceGuard guard(plan->device);
    if (!guard.ok) return slsht::set_error(SLSHT_EDEVICE, "hipSetDevice failed");
    hipError_t e = slsht::launch_coupling_modulated(P, (const double2*)f, (double2*)A, work,
                                                    (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "modulated coupling launch");
    return SLSHT_OK;
}

int slsht_slepian_window(int L_h, double theta_c, double a, int device, void* h_out,
                         double* concentration) {
    if (!h_out) return slsht::set_error(SLSHT_EINVAL, "h_out is NULL");
    if (L_h < 1 || L_h > SLSHT_MAX_LH)
        return slsht::set_error(SLSHT_EINVAL, "L_h=%d outside [1, %d]", L_h, SLSHT_MAX_LH);
    if (!(theta_c >= 0.0) || !(a > theta_c) || !(a <= 0.5 * M_PI + 1e-12))
        return slsht::set_error(SLSHT_EINVAL, "need 0 <= theta_c < a <= pi/2 (got %g, %g)",
                                theta_c, a);
    DeviceGuard guard(device);
    if (!guard.ok) return slsht::set_error(SLSHT_EDEVICE, "hipSetDevice(%d) failed", device);
    return slsht::slepian_window(L_h, theta_c, std::min(a, 0.5 * M_PI), (double2*)h_out,
                                 concentration);
}

int slsht_inverse(slsht_plan_t plan, const void* g, const void* h, void* f_out, void* stream) {
    if (!plan || !g || !h || !f_out) return slsht::set_error(SLSHT_EINVAL, "NULL argument");
    const slsht::DevPlan& P = plan->P;
    if (P.d.output_mode != SLSHT_OUT_FULL)
        return slsht::set_error(SLSHT_EINVAL, "inverse needs a FULL plan");
    if (P.d.theta_lo != 0 || P.d.theta_hi != P.d.n_theta)
        return slsht::set_error(SLSHT_EINVAL,
                                "inverse needs every theta row (theta_lo=0, theta_hi=n_theta)");
    if (P.d.n_phi < 2 * P.d.L_h - 1 || P.d.n_omega < 2 * slsht::n_az_of(P.d) - 1)
        return slsht::set_error(SLSHT_EINVAL,
                                "inverse needs n_phi >= 2 L_h - 1 and n_omega >= 2 n_az - 1");
    DeviceGuard guard(plan->device);
    if (!guard.ok) return slsht::set_error(SLSHT_EDEVICE, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)stream;
    // f = f_hat / (sqrt(16 pi^3) h00) with f_hat = (1 / (n_phi^2 n_omega)) x the weighted sum
    const double k = 1.0 / ((double)P.d.n_phi * P.d.n_phi * P.d.n_omega *
                            std::sqrt(16.0 * M_PI * M_PI * M_PI));
    hipError_t e = slsht::launch_inverse(P, g, k, (const double2*)h, (double2*)f_out, s);
    if (e != hipSuccess) return hip_fail(e, "inverse launch");
    return SLSHT_OK;
}

}  // extern "C"
