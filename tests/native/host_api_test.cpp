// Host paths of the C ABI under the address and undefined-behaviour sanitizers, without a
// GPU: descriptor checks, footprints and workspace sizes of random descriptors (valid and
// not), and the error returns of the entry points that need a device.
#include <cassert>
#include <cstdio>
#include <cstring>
#include <random>

#include "slsht.h"

int main() {
    std::mt19937 rng(2024);
    int valid = 0, invalid = 0;
    for (int it = 0; it < 20000; ++it) {
        slsht_desc d{};
        d.L_f = (int)(rng() % 300) - 2;
        d.L_h = (int)(rng() % 36) - 1;
        d.l_lo = (int)(rng() % 80) - 1;
        d.l_hi = d.l_lo + (int)(rng() % 20) - 2;
        d.n_phi = (int)(rng() % 1200) - 2;
        d.n_theta = rng() % 8 ? (d.n_phi + 1) / 2 : (int)(rng() % 600);
        d.n_omega = (int)(rng() % 80);
        d.precision = (int)(rng() % 3);
        d.output_mode = (int)(rng() % 3);
        d.flags = rng() % 5 == 0 ? 2u : (uint32_t)(rng() % 2);
        d.theta_lo = rng() % 4 ? 0 : (int)(rng() % 20);
        d.theta_hi = rng() % 4 ? 0 : d.theta_lo + (int)(rng() % 20) - 1;
        d.n_az = rng() % 3 ? 0 : (int)(rng() % 36) - 1;
        const int v = slsht_validate(&d);
        size_t plan = 0, out = 0, scratch = 1;
        const int f = slsht_footprint(&d, &plan, &out, &scratch);
        assert(v == f);
        const long long n = slsht_coupling_size(&d);
        if (v == SLSHT_OK) {
            ++valid;
            assert(out > 0 && plan > 0 && scratch == 0);
            assert(n == ((long long)d.l_hi * d.l_hi - (long long)d.l_lo * d.l_lo) * d.L_h * d.L_h);
        } else {
            ++invalid;
            assert(n == -1);
            assert(std::strlen(slsht_last_error()) > 0);
        }
    }
    // the ENERGY workload and a staged FULL plan hold workspaces
    slsht_desc e{};
    e.L_f = 512; e.L_h = 32; e.l_lo = 100; e.l_hi = 116; e.n_phi = 1087; e.n_theta = 544;
    e.n_omega = 63; e.precision = SLSHT_FP32_MIXED; e.output_mode = SLSHT_OUT_ENERGY;
    size_t pe = 0, oe = 0;
    assert(slsht_footprint(&e, &pe, &oe, nullptr) == SLSHT_OK);
    assert(oe == (size_t)16 * 1087 * 544 * 63 * 4 && pe > ((size_t)16 << 30));
    slsht_desc s{};
    s.L_f = 40; s.L_h = 20; s.l_lo = 0; s.l_hi = 9; s.n_phi = 119; s.n_theta = 60; s.n_omega = 39;
    size_t ps = 0;
    assert(slsht_footprint(&s, &ps, nullptr, nullptr) == SLSHT_OK);
    s.L_h = 16;
    size_t p16 = 0;
    assert(slsht_footprint(&s, &p16, nullptr, nullptr) == SLSHT_OK && ps > p16);
    // device entry points fail cleanly without a GPU
    slsht_plan_t plan = nullptr;
    const int pr = slsht_plan(&s, 0, &plan);
    assert(pr != SLSHT_OK && plan == nullptr && std::strlen(slsht_last_error()) > 0);
    slsht_server_t srv = nullptr;
    assert(slsht_server_create(0, (size_t)1 << 30, 2, &srv) != SLSHT_OK && srv == nullptr);
    assert(slsht_forward(nullptr, nullptr, nullptr, nullptr, nullptr) == SLSHT_EINVAL);
    assert(slsht_submit(nullptr, &s, nullptr, nullptr, nullptr) == SLSHT_EINVAL);
    int st = 0;
    assert(slsht_poll(nullptr, 1, &st, nullptr, nullptr, nullptr) == SLSHT_EINVAL);
    printf("host api ok: %d valid, %d invalid descriptors\n", valid, invalid);
    return 0;
}
