/*
 * Host-side paths of the C-ABI under AddressSanitizer and
 * UndefinedBehaviorSanitizer, for tests/test_abi_sanitized.py (the library's
 * host code instrumented, its device code as always; no GPU needed): the
 * parameter validation and state layout of every precision and rounding
 * mode, the batch head size, the error strings, and every entry point's
 * rejection of null, misaligned or undersized arguments.  Exit status 0 when
 * every call returns the expected code.
 */
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "../include/lbm_axi.h"

static int failures = 0;

#define EXPECT(cond)                                                     \
    do {                                                                 \
        if (!(cond)) {                                                   \
            fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                  \
        }                                                                \
    } while (0)

static lbm_axi_params base(int nr, int nz, int precision)
{
    lbm_axi_params p;
    memset(&p, 0, sizeof p);
    p.nr = nr;
    p.nz = nz;
    p.z_periodic = 1;
    p.precision = precision;
    p.collision = LBM_AXI_MRT;
    p.W = 4.0;
    p.mobility = 0.1;
    p.sigma = 1e-3;
    p.rho_l = 1000.0;
    p.rho_g = 1.0;
    p.nu_l = 0.1;
    p.nu_g = 0.1;
    for (int a = 0; a < 9; ++a) {
        p.s_f[a] = 1.0;
        p.s_g[a] = 1.0;
    }
    return p;
}

int main(void)
{
    const int precisions[3] = {LBM_AXI_FP64, LBM_AXI_FP32, LBM_AXI_FP16D};
    const int sizes[6][2] = {{4, 4}, {5, 7}, {33, 130}, {256, 512}, {4096, 8192}, {1, 1 << 25}};
    size_t last[3] = {0, 0, 0};
    for (int q = 0; q < 3; ++q) {
        for (int s = 0; s < 6; ++s) {
            lbm_axi_params p = base(sizes[s][0], sizes[s][1], precisions[q]);
            size_t b = lbm_axi_state_bytes(&p);
            if (sizes[s][0] < 4) {
                EXPECT(b == 0);
            } else {
                EXPECT(b > 0 && b % 256 == 0);
                EXPECT(b >= last[q]);
                last[q] = b;
            }
        }
        // every collision form, both z modes, the free energy rate
        for (int form = 0; form < 3; ++form)
            for (int zper = 0; zper < 2; ++zper) {
                lbm_axi_params p = base(16, 32, precisions[q]);
                p.collision = form;
                p.z_periodic = zper;
                EXPECT(lbm_axi_state_bytes(&p) > 0);
                p.free_s1 = 1;
                p.s_g[1] = 1.2;
                const size_t fb = lbm_axi_state_bytes(&p);
                EXPECT(form == LBM_AXI_SRT ? fb == 0 : fb > 0);    /* not with SRT */
            }
        // the g rounding option: FP16-deviation storage only
        lbm_axi_params p = base(16, 32, precisions[q]);
        p.fp16_rounding = LBM_AXI_ROUND_STOCHASTIC;
        EXPECT((lbm_axi_state_bytes(&p) > 0) == (precisions[q] == LBM_AXI_FP16D));
        p.fp16_rounding = 2;
        EXPECT(lbm_axi_state_bytes(&p) == 0);
    }
    EXPECT(last[2] < last[1] && last[1] < last[0]);
    // grid limit and invalid values
    {
        lbm_axi_params p = base(8192, 8192, LBM_AXI_FP32);
        EXPECT(lbm_axi_state_bytes(&p) == 0);            /* nr*nz > 2^25 */
        p = base(16, 32, LBM_AXI_FP32);
        p.W = NAN;
        EXPECT(lbm_axi_state_bytes(&p) == 0);
        p = base(16, 32, LBM_AXI_FP32);
        p.g_z = INFINITY;
        EXPECT(lbm_axi_state_bytes(&p) == 0);
        p = base(16, 32, LBM_AXI_FP32);
        p.s_g[2] = 0.0;
        EXPECT(lbm_axi_state_bytes(&p) == 0);
        p = base(16, 32, 7);
        EXPECT(lbm_axi_state_bytes(&p) == 0);
        p = base(16, 32, LBM_AXI_FP32);
        p.g_ramp = -1.0;
        EXPECT(lbm_axi_state_bytes(&p) == 0);
        EXPECT(lbm_axi_state_bytes(NULL) == 0);
    }
    // batch head
    for (int q = 0; q < 3; ++q) {
        size_t h1 = lbm_axi_batch_reserved_bytes(1, precisions[q]);
        size_t h64 = lbm_axi_batch_reserved_bytes(64, precisions[q]);
        EXPECT(h1 > 0 && h1 % 256 == 0 && h64 > h1);
    }
    EXPECT(lbm_axi_batch_reserved_bytes(0, LBM_AXI_FP32) == 0);
    EXPECT(lbm_axi_batch_reserved_bytes(4, 7) == 0);
    // error strings
    for (int code = -10; code <= 1; ++code) {
        const char *m = lbm_axi_strerror(code);
        EXPECT(m != NULL && strlen(m) > 0);
    }
    // rejections before any device work
    {
        static double phi0[16 * 32];
        lbm_axi_params p = base(16, 32, LBM_AXI_FP32);
        lbm_axi_case *c = (lbm_axi_case *)(uintptr_t)1;
        EXPECT(lbm_axi_init(&p, (void *)(uintptr_t)4096, 1 << 20, phi0, NULL, NULL) == LBM_AXI_EINVAL);
        EXPECT(lbm_axi_init(&p, NULL, 1 << 20, phi0, NULL, &c) == LBM_AXI_EINVAL && c == NULL);
        EXPECT(lbm_axi_init(&p, (void *)(uintptr_t)4100, 1 << 20, phi0, NULL, &c) == LBM_AXI_EINVAL);
        EXPECT(lbm_axi_init(&p, (void *)(uintptr_t)4096, 1 << 20, NULL, NULL, &c) == LBM_AXI_EINVAL);
        EXPECT(lbm_axi_init(&p, (void *)(uintptr_t)4096, 256, phi0, NULL, &c) == LBM_AXI_ENOMEM);
        p.nr = 2;
        EXPECT(lbm_axi_init(&p, (void *)(uintptr_t)4096, 1 << 20, phi0, NULL, &c) == LBM_AXI_EINVAL);
        EXPECT(lbm_axi_step(NULL, 1) != LBM_AXI_OK);
        EXPECT(lbm_axi_moments(NULL, NULL, NULL, NULL, NULL, NULL, NULL) != LBM_AXI_OK);
        EXPECT(lbm_axi_get_state(NULL, NULL, NULL, NULL, NULL) != LBM_AXI_OK);
        EXPECT(lbm_axi_set_state(NULL, NULL, NULL, NULL, 0) != LBM_AXI_OK);
        int64_t t = -1;
        EXPECT(lbm_axi_time(NULL, &t) != LBM_AXI_OK);
        EXPECT(lbm_axi_set_tile(NULL, 8) != LBM_AXI_OK);
        EXPECT(lbm_axi_destroy(NULL) == LBM_AXI_OK);     /* NULL is accepted */
    }
    {
        lbm_axi_batch *b = (lbm_axi_batch *)(uintptr_t)1;
        EXPECT(lbm_axi_batch_create(NULL, 1 << 30, 4, LBM_AXI_FP32, NULL, &b) == LBM_AXI_EINVAL && b == NULL);
        EXPECT(lbm_axi_batch_create((void *)(uintptr_t)4100, 1 << 30, 4, LBM_AXI_FP32, NULL, &b) == LBM_AXI_EINVAL);
        EXPECT(lbm_axi_batch_create((void *)(uintptr_t)4096, 1024, 4, LBM_AXI_FP32, NULL, &b) == LBM_AXI_ENOMEM);
        EXPECT(lbm_axi_batch_create((void *)(uintptr_t)4096, 1 << 30, 0, LBM_AXI_FP32, NULL, &b) == LBM_AXI_EINVAL);
        EXPECT(lbm_axi_batch_create((void *)(uintptr_t)4096, 1 << 30, 4, LBM_AXI_FP32, NULL, NULL) == LBM_AXI_EINVAL);
        int32_t n = 0;
        EXPECT(lbm_axi_batch_run(NULL, 10) != LBM_AXI_OK);
        EXPECT(lbm_axi_batch_prepare(NULL, 10) != LBM_AXI_OK);
        EXPECT(lbm_axi_batch_poll(NULL, NULL, 0, &n) != LBM_AXI_OK);
        EXPECT(lbm_axi_batch_release(NULL, 0) != LBM_AXI_OK);
        EXPECT(lbm_axi_batch_set_config(NULL, 8, 0, 1, 16) != LBM_AXI_OK);
        EXPECT(lbm_axi_batch_sync(NULL) != LBM_AXI_OK);
        EXPECT(lbm_axi_batch_destroy(NULL) == LBM_AXI_OK);
    }
    {
        EXPECT(lbm_axi_device_copy((void *)(uintptr_t)4096, (void *)(uintptr_t)8192, 24, NULL) == LBM_AXI_EINVAL);
        EXPECT(lbm_axi_device_copy((void *)(uintptr_t)4100, (void *)(uintptr_t)8192, 32, NULL) == LBM_AXI_EINVAL);
        EXPECT(lbm_axi_device_copy(NULL, (void *)(uintptr_t)8192, 32, NULL) == LBM_AXI_EINVAL);
        EXPECT(lbm_axi_device_copy((void *)(uintptr_t)4096, (void *)(uintptr_t)4112, 32, NULL) == LBM_AXI_EINVAL);
    }
    printf("%d failing checks\n", failures);
    return failures ? 1 : 0;
}
