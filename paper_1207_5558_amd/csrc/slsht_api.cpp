// Host core of the directional SLSHT library: descriptor checks, footprints,
// plans (device tables), and the forward / coupling / inverse entry points.
#include <hip/hip_runtime.h>

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

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(SLSHT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Saves and restores the caller's current device around a library call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

struct Sizes {
    int n_theta_out;
    int64_t n_lm, n_l, n_rho_out;
    size_t vbytes;     // complex output element
    size_t rbytes;     // real (energy) output element
    size_t dtab, twphi, twom, twfull, qw, items, items_l, coupling, out;
};

bool mul_ok(size_t a, size_t b, size_t& r) {
    if (a != 0 && b > std::numeric_limits<size_t>::max() / a) return false;
    r = a * b;
    return true;
}

int check_desc(const slsht_desc* d) {
    if (!d) return fail(SLSHT_EINVAL, "desc is NULL");
    if (d->L_f < 1 || d->L_f > SLSHT_MAX_LF)
        return fail(SLSHT_EINVAL, "L_f=%d outside [1, %d]", d->L_f, SLSHT_MAX_LF);
    if (d->L_h < 1 || d->L_h > SLSHT_MAX_LH)
        return fail(SLSHT_EINVAL, "L_h=%d outside [1, %d]", d->L_h, SLSHT_MAX_LH);
    if (d->l_lo < 0 || d->l_hi <= d->l_lo || d->l_hi > d->L_f + d->L_h - 1)
        return fail(SLSHT_EINVAL, "need 0 <= l_lo < l_hi <= L_f + L_h - 1 (got l_lo=%d l_hi=%d)",
                    d->l_lo, d->l_hi);
    if (d->n_phi < 1 || d->n_phi > SLSHT_MAX_NPHI || (d->n_phi % 2) == 0)
        return fail(SLSHT_EINVAL, "n_phi=%d must be odd and in [1, %d]", d->n_phi, SLSHT_MAX_NPHI);
    if (d->n_theta != (d->n_phi + 1) / 2)
        return fail(SLSHT_EINVAL, "n_theta=%d must equal (n_phi + 1) / 2 = %d", d->n_theta,
                    (d->n_phi + 1) / 2);
    if (d->n_omega < 1 || d->n_omega > 4096)
        return fail(SLSHT_EINVAL, "n_omega=%d outside [1, 4096]", d->n_omega);
    if (d->precision != SLSHT_FP64 && d->precision != SLSHT_FP32_MIXED)
        return fail(SLSHT_EINVAL, "unknown precision %d", d->precision);
    if (d->output_mode != SLSHT_OUT_FULL && d->output_mode != SLSHT_OUT_ENERGY)
        return fail(SLSHT_EINVAL, "unknown output_mode %d", d->output_mode);
    if (d->flags & ~(uint32_t)SLSHT_REAL_PAIR)
        return fail(SLSHT_EINVAL, "unknown flags 0x%x", d->flags);
    const int thi = d->theta_hi == 0 ? d->n_theta : d->theta_hi;
    if (d->theta_lo < 0 || thi <= d->theta_lo || thi > d->n_theta)
        return fail(SLSHT_EINVAL, "need 0 <= theta_lo < theta_hi <= n_theta (got %d, %d)",
                    d->theta_lo, d->theta_hi);
    if (d->output_mode == SLSHT_OUT_ENERGY) {
        if (d->precision != SLSHT_FP32_MIXED)
            return fail(SLSHT_EINVAL, "ENERGY output needs precision SLSHT_FP32_MIXED");
        if (d->n_omega > slsht::kEnergyMaxOmega)
            return fail(SLSHT_EINVAL, "ENERGY output needs n_omega <= %d", slsht::kEnergyMaxOmega);
        const int nst = ((d->n_phi + 1) / 2 + 15) / 16, nct = (d->n_omega + 15) / 16;
        if (nst * nct > slsht::kEnergyMaxTiles)
            return fail(SLSHT_EINVAL,
                        "ENERGY output needs ceil(((n_phi+1)/2)/16) * ceil(n_omega/16) <= %d "
                        "(n_phi <= 1087 at n_omega = 64)", slsht::kEnergyMaxTiles);
    }
    return SLSHT_OK;
}

int compute_sizes(const slsht_desc* d, Sizes& s) {
    int rc = check_desc(d);
    if (rc) return rc;
    const int thi = d->theta_hi == 0 ? d->n_theta : d->theta_hi;
    s.n_theta_out = thi - d->theta_lo;
    s.n_lm = (int64_t)d->l_hi * d->l_hi - (int64_t)d->l_lo * d->l_lo;
    s.n_l = d->l_hi - d->l_lo;
    s.n_rho_out = (int64_t)d->n_phi * s.n_theta_out * d->n_omega;
    const bool f64 = d->precision == SLSHT_FP64;
    s.vbytes = f64 ? 16 : 8;
    s.rbytes = f64 ? 8 : 4;
    const int L = d->L_h;
    const size_t nslot = (size_t)(d->n_phi + 1) / 2, ncp = (size_t)d->n_omega / 2 + 1;
    s.dtab = (size_t)s.n_theta_out * (size_t)slsht::dtab_row_len(L) * s.rbytes;
    s.twphi = (size_t)(L > 1 ? L - 1 : 1) * nslot * s.vbytes;
    s.twom = (size_t)(L > 1 ? L - 1 : 1) * ncp * s.vbytes;
    s.twfull = d->output_mode == SLSHT_OUT_ENERGY ? (size_t)d->n_phi * sizeof(float2) : 0;
    s.qw = (size_t)d->n_theta * sizeof(double);
    s.items = (size_t)s.n_lm * sizeof(slsht::Item);
    s.items_l = (size_t)s.n_l * sizeof(slsht::Item);
    s.coupling = (size_t)s.n_lm * L * L * sizeof(double2);
    size_t per = d->output_mode == SLSHT_OUT_FULL ? (size_t)s.n_lm * s.vbytes : (size_t)s.n_l * s.rbytes;
    if (!mul_ok(per, (size_t)s.n_rho_out, s.out))
        return fail(SLSHT_EINVAL, "output size overflows size_t");
    return SLSHT_OK;
}

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

void free_plan_mem(slsht::DevPlan& P) {
    void* ptrs[] = {P.dtab, P.tw_phi, P.tw_omega, P.tw_full, P.qw, P.items, P.items_l, P.A};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    P.dtab = P.tw_phi = P.tw_omega = P.tw_full = nullptr;
    P.qw = nullptr;
    P.items = P.items_l = nullptr;
    P.A = nullptr;
}

}  // namespace

struct slsht_plan_s {
    slsht::DevPlan P;
    int device;
};

extern "C" {

const char* slsht_last_error(void) { return g_err.c_str(); }

int slsht_validate(const slsht_desc* desc) {
    Sizes s;
    return compute_sizes(desc, s);
}

int slsht_footprint(const slsht_desc* desc, size_t* plan_bytes, size_t* out_bytes,
                    size_t* scratch_bytes) {
    Sizes s;
    int rc = compute_sizes(desc, s);
    if (rc) return rc;
    if (plan_bytes)
        *plan_bytes = s.dtab + s.twphi + s.twom + s.twfull + s.qw + s.items + s.items_l + s.coupling;
    if (out_bytes) *out_bytes = s.out;
    if (scratch_bytes) *scratch_bytes = 0;
    return SLSHT_OK;
}

int64_t slsht_coupling_size(const slsht_desc* desc) {
    Sizes s;
    if (compute_sizes(desc, s)) return -1;
    return s.n_lm * desc->L_h * desc->L_h;
}

int slsht_plan(const slsht_desc* desc, int device, slsht_plan_t* out) {
    if (!out) return fail(SLSHT_EINVAL, "out is NULL");
    *out = nullptr;
    Sizes s;
    int rc = compute_sizes(desc, s);
    if (rc) return rc;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
        return fail(SLSHT_EDEVICE, "no HIP device available");
    if (device < 0 || device >= ndev) return fail(SLSHT_EINVAL, "device %d out of range", device);
    DeviceGuard guard(device);
    if (!guard.ok) return fail(SLSHT_EDEVICE, "hipSetDevice(%d) failed", device);

    slsht_plan_s* pl = new slsht_plan_s();
    pl->device = device;
    slsht::DevPlan& P = pl->P;
    P.d = *desc;
    if (P.d.theta_hi == 0) P.d.theta_hi = P.d.n_theta;
    P.n_theta_out = s.n_theta_out;
    P.nslot_phi = (P.d.n_phi + 1) / 2;
    P.ncp_omega = P.d.n_omega / 2 + 1;

    int lds_limit = 0;
    if (hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
        hipSuccess)
        lds_limit = 64 * 1024;
    if (P.d.output_mode == SLSHT_OUT_FULL && !slsht::choose_synthesis_shape(P, (size_t)lds_limit)) {
        delete pl;
        return fail(SLSHT_EINVAL, "no synthesis tiling fits %d bytes of LDS for this descriptor",
                    lds_limit);
    }
    if (P.d.output_mode == SLSHT_OUT_ENERGY && slsht::energy_lds_for(P) > (size_t)lds_limit) {
        const size_t need = slsht::energy_lds_for(P);
        delete pl;
        return fail(SLSHT_EINVAL, "ENERGY kernel needs %zu bytes of LDS, device allows %d", need,
                    lds_limit);
    }

    // items: output slot, degree, order, mirrored slot
    std::vector<slsht::Item> items;
    const bool pair = (P.d.flags & SLSHT_REAL_PAIR) != 0;
    for (int l = P.d.l_lo; l < P.d.l_hi; ++l)
        for (int m = pair ? 0 : -l; m <= l; ++m) {
            const int base = l * l + l - P.d.l_lo * P.d.l_lo;
            items.push_back({base + m, l, m, (pair && m > 0) ? base - m : -1});
        }
    P.n_items = (int)items.size();
    std::vector<slsht::Item> items_l;
    for (int l = P.d.l_lo; l < P.d.l_hi; ++l) items_l.push_back({l - P.d.l_lo, l, 0, -1});

    std::vector<double> qw;
    beta_weights(P.d.n_phi, P.d.n_theta, qw);

    hipError_t e = hipSuccess;
    auto alloc = [&](void** p, size_t n) {
        if (e == hipSuccess) e = hipMalloc(p, n ? n : 16);
    };
    alloc(&P.dtab, s.dtab);
    alloc(&P.tw_phi, s.twphi);
    alloc(&P.tw_omega, s.twom);
    alloc((void**)&P.qw, s.qw);
    alloc((void**)&P.items, s.items);
    alloc((void**)&P.items_l, s.items_l);
    alloc((void**)&P.A, s.coupling);
    if (s.twfull) alloc(&P.tw_full, s.twfull);
    if (e != hipSuccess) {
        free_plan_mem(P);
        delete pl;
        return fail(SLSHT_ENOMEM, "plan allocation failed: %s", hipGetErrorString(e));
    }
    if (P.d.precision == SLSHT_FP64) {
        std::vector<double> tp, to;
        twiddles(P.d.L_h, P.d.n_phi, P.nslot_phi, tp);
        twiddles(P.d.L_h, P.d.n_omega, P.ncp_omega, to);
        e = hipMemcpy(P.tw_phi, tp.data(), tp.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(P.tw_omega, to.data(), to.size() * sizeof(double), hipMemcpyHostToDevice);
    } else {
        std::vector<float> tp, to;
        twiddles(P.d.L_h, P.d.n_phi, P.nslot_phi, tp);
        twiddles(P.d.L_h, P.d.n_omega, P.ncp_omega, to);
        e = hipMemcpy(P.tw_phi, tp.data(), tp.size() * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(P.tw_omega, to.data(), to.size() * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && s.twfull) {
        // cos/sin(2 pi j / n_phi), j < n_phi, for the ENERGY kernel's phi synthesis
        std::vector<float> tf((size_t)P.d.n_phi * 2);
        for (int j = 0; j < P.d.n_phi; ++j) {
            const double ang = 2.0 * M_PI * (double)j / (double)P.d.n_phi;
            tf[2 * j] = (float)std::cos(ang);
            tf[2 * j + 1] = (float)std::sin(ang);
        }
        e = hipMemcpy(P.tw_full, tf.data(), s.twfull, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemcpy(P.qw, qw.data(), s.qw, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(P.items, items.data(), items.size() * sizeof(slsht::Item), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(P.items_l, items_l.data(), items_l.size() * sizeof(slsht::Item),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = slsht::launch_wigner_table(P, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_plan_mem(P);
        delete pl;
        return hip_fail(e, "plan build");
    }
    *out = pl;
    return SLSHT_OK;
}

int slsht_plan_destroy(slsht_plan_t plan) {
    if (!plan) return fail(SLSHT_EINVAL, "plan is NULL");
    DeviceGuard guard(plan->device);
    (void)hipDeviceSynchronize();
    free_plan_mem(plan->P);
    delete plan;
    return SLSHT_OK;
}

int slsht_plan_desc(slsht_plan_t plan, slsht_desc* out) {
    if (!plan || !out) return fail(SLSHT_EINVAL, "NULL argument");
    *out = plan->P.d;
    return SLSHT_OK;
}

int slsht_coupling(slsht_plan_t plan, const void* f, void* A, void* stream) {
    if (!plan || !f || !A) return fail(SLSHT_EINVAL, "NULL argument");
    DeviceGuard guard(plan->device);
    if (!guard.ok) return fail(SLSHT_EDEVICE, "hipSetDevice failed");
    hipError_t e = slsht::launch_coupling(plan->P, (const double2*)f, (double2*)A, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "coupling launch");
    return SLSHT_OK;
}

int slsht_forward(slsht_plan_t plan, const void* f, const void* h, void* g, void* stream) {
    if (!plan || !f || !h || !g) return fail(SLSHT_EINVAL, "NULL argument");
    const slsht::DevPlan& P = plan->P;
    DeviceGuard guard(plan->device);
    if (!guard.ok) return fail(SLSHT_EDEVICE, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = slsht::launch_coupling(P, (const double2*)f, P.A, s);
    if (e != hipSuccess) return hip_fail(e, "coupling launch");
    if (P.d.output_mode == SLSHT_OUT_FULL)
        e = slsht::launch_synthesis(P, P.A, (const double2*)h, g, s);
    else
        e = slsht::launch_energy(P, P.A, (const double2*)h, (float*)g, s);
    if (e != hipSuccess) return hip_fail(e, "synthesis launch");
    return SLSHT_OK;
}

int slsht_inverse(slsht_plan_t plan, const void* g, const void* h, void* f_out, void* stream) {
    if (!plan || !g || !h || !f_out) return fail(SLSHT_EINVAL, "NULL argument");
    const slsht::DevPlan& P = plan->P;
    if (P.d.output_mode != SLSHT_OUT_FULL)
        return fail(SLSHT_EINVAL, "inverse needs a FULL plan");
    if (P.d.theta_lo != 0 || P.d.theta_hi != P.d.n_theta)
        return fail(SLSHT_EINVAL, "inverse needs every theta row (theta_lo=0, theta_hi=n_theta)");
    if (P.d.n_phi < 2 * P.d.L_h - 1 || P.d.n_omega < 2 * P.d.L_h - 1)
        return fail(SLSHT_EINVAL, "inverse needs n_phi, n_omega >= 2 L_h - 1");
    DeviceGuard guard(plan->device);
    if (!guard.ok) return fail(SLSHT_EDEVICE, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)stream;
    double2 h00;
    hipError_t e = hipMemcpyAsync(&h00, h, sizeof(double2), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading h_0^0");
    const double mag2 = h00.x * h00.x + h00.y * h00.y;
    if (!(mag2 > 0.0)) return fail(SLSHT_EINVAL, "h_0^0 is zero: the inverse divides by it");
    // scale = 1 / (n_phi^2 n_omega sqrt(16 pi^3) h00)
    const double k = 1.0 / ((double)P.d.n_phi * P.d.n_phi * P.d.n_omega * std::sqrt(16.0 * M_PI * M_PI * M_PI));
    double2 scale;
    scale.x = k * h00.x / mag2;
    scale.y = -k * h00.y / mag2;
    e = slsht::launch_inverse(P, g, scale, (double2*)f_out, s);
    if (e != hipSuccess) return hip_fail(e, "inverse launch");
    return SLSHT_OK;
}

}  // extern "C"
