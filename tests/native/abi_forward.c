/* A plain C consumer of the library: plans the tiny FP64 transform through
 * include/slsht.h, runs slsht_forward and slsht_inverse with device buffers from the
 * HIP runtime, and writes g and the recovered coefficients for the Python test to
 * compare with the oracle.  Usage: abi_forward <in.bin> <g.bin> <f_out.bin>, where in.bin
 * holds f (complex128[L_f^2]) then h (complex128[L_h^2]). */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "slsht.h"

#define CHECK_HIP(x)                                                            \
    do {                                                                        \
        hipError_t e_ = (x);                                                    \
        if (e_ != hipSuccess) {                                                 \
            fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));     \
            return 2;                                                           \
        }                                                                       \
    } while (0)
#define CHECK_SL(x)                                                             \
    do {                                                                        \
        int s_ = (x);                                                           \
        if (s_ != SLSHT_OK) {                                                   \
            fprintf(stderr, "%s failed (%d): %s\n", #x, s_, slsht_last_error()); \
            return 3;                                                           \
        }                                                                       \
    } while (0)

static int read_all(const char* path, void* buf, size_t n) {
    FILE* fp = fopen(path, "rb");
    if (!fp) return 0;
    size_t got = fread(buf, 1, n, fp);
    fclose(fp);
    return got == n;
}

static int write_all(const char* path, const void* buf, size_t n) {
    FILE* fp = fopen(path, "wb");
    if (!fp) return 0;
    size_t put = fwrite(buf, 1, n, fp);
    fclose(fp);
    return put == n;
}

int main(int argc, char** argv) {
    if (argc != 4) {
        fprintf(stderr, "usage: %s in.bin g.bin f_out.bin\n", argv[0]);
        return 1;
    }
    slsht_desc d = {0};
    d.L_f = 8;
    d.L_h = 3;
    d.l_lo = 0;
    d.l_hi = 8;
    d.n_phi = 21;
    d.n_theta = 11;
    d.n_omega = 5;
    d.precision = SLSHT_FP64;
    d.output_mode = SLSHT_OUT_FULL;
    CHECK_SL(slsht_validate(&d));
    size_t plan_bytes = 0, out_bytes = 0, scratch = 0;
    CHECK_SL(slsht_footprint(&d, &plan_bytes, &out_bytes, &scratch));
    const size_t nf = (size_t)d.L_f * d.L_f * 16, nh = (size_t)d.L_h * d.L_h * 16;
    const size_t n_lm = (size_t)d.l_hi * d.l_hi - (size_t)d.l_lo * d.l_lo;
    char* host = (char*)malloc(nf + nh + out_bytes + n_lm * 16);
    if (!host || !read_all(argv[1], host, nf + nh)) {
        fprintf(stderr, "cannot read %s\n", argv[1]);
        return 1;
    }
    void *f_dev = NULL, *h_dev = NULL, *g_dev = NULL, *fo_dev = NULL;
    CHECK_HIP(hipMalloc(&f_dev, nf));
    CHECK_HIP(hipMalloc(&h_dev, nh));
    CHECK_HIP(hipMalloc(&g_dev, out_bytes));
    CHECK_HIP(hipMalloc(&fo_dev, n_lm * 16));
    CHECK_HIP(hipMemcpy(f_dev, host, nf, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(h_dev, host + nf, nh, hipMemcpyHostToDevice));
    slsht_plan_t plan = NULL;
    CHECK_SL(slsht_plan(&d, 0, &plan));
    CHECK_SL(slsht_forward(plan, f_dev, h_dev, g_dev, NULL));
    CHECK_SL(slsht_inverse(plan, g_dev, h_dev, fo_dev, NULL));
    CHECK_HIP(hipDeviceSynchronize());
    char* g_host = host + nf + nh;
    char* fo_host = g_host + out_bytes;
    CHECK_HIP(hipMemcpy(g_host, g_dev, out_bytes, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(fo_host, fo_dev, n_lm * 16, hipMemcpyDeviceToHost));
    CHECK_SL(slsht_plan_destroy(plan));
    CHECK_HIP(hipFree(f_dev));
    CHECK_HIP(hipFree(h_dev));
    CHECK_HIP(hipFree(g_dev));
    CHECK_HIP(hipFree(fo_dev));
    if (!write_all(argv[2], g_host, out_bytes) || !write_all(argv[3], fo_host, n_lm * 16)) {
        fprintf(stderr, "cannot write outputs\n");
        return 1;
    }
    free(host);
    printf("abi_forward ok: %zu output bytes\n", out_bytes);
    return 0;
}
