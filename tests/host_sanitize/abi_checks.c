/* Host-side checks of the C ABI, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host code of the library (see
 * tests/test_host_sanitizers.py).  Every call here is answered by the host
 * code alone: geometry and flag validation, workspace planning for single
 * and batched reductions (including sizes near the limits, where an integer
 * overflow would show), the minimum-rotation query, status strings, and the
 * rejection of missing contexts and pointers.  No GPU is needed; when one is
 * present the context is created and destroyed once as well.
 *
 * Exit status 0 when every expectation holds; the sanitizers abort on the
 * first error they find. */

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "graphic.h"

static int failures = 0;

#define EXPECT(cond)                                                      \
    do {                                                                  \
        if (!(cond)) {                                                    \
            fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, \
                    __LINE__, #cond);                                     \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

static graphic_geom geom(int64_t t, int32_t n, int32_t p, uint32_t flags) {
    graphic_geom g;
    g.n_frames = t;
    g.n = n;
    g.pad = p;
    g.flags = flags;
    return g;
}

static void check_status_strings(void) {
    for (int s = -3; s < 12; ++s) {
        const char* str = graphic_status_string((graphic_status)s);
        EXPECT(str != NULL && strlen(str) > 0);
    }
    EXPECT(strstr(graphic_version(), "gfx950") != NULL);
}

static void check_resolved_pad(void) {
    static const int32_t ns[] = {-4, 0, 2, 4, 6, 7, 8, 100, 128, 1000, 1024, 2048, 2050, 4096, 4098, 1 << 30};
    static const int32_t ps[] = {-1, 0, 1, 8, 16, 64, 96, 256, 2048, 4096, 8192, 1 << 30};
    for (size_t i = 0; i < sizeof ns / sizeof ns[0]; ++i)
        for (size_t j = 0; j < sizeof ps / sizeof ps[0]; ++j) {
            graphic_geom g = geom(3, ns[i], ps[j], 0);
            const int32_t p = graphic_resolved_pad(&g);
            if (p > 0) {
                EXPECT((p & (p - 1)) == 0 && p >= ns[i] && p <= 4096 && p >= 16);
            }
        }
    graphic_geom g = geom(3, 1024, 0, 0);
    EXPECT(graphic_resolved_pad(&g) == 2048);
    EXPECT(graphic_resolved_pad(NULL) < 0);
}

static void check_workspace_sizes(void) {
    static const int64_t ts[] = {-1, 0, 1, 2, 4095, 4096, 4097, 100000, (int64_t)1 << 24, ((int64_t)1 << 24) + 1,
                                 (int64_t)1 << 40, INT64_MAX};
    static const int32_t ns[] = {4, 6, 8, 128, 1024, 2048, 4096};
    static const uint32_t fl[] = {0u, GRAPHIC_KEEP_PADDED, GRAPHIC_CHECK_FINITE,
                                  GRAPHIC_KEEP_PADDED | GRAPHIC_CHECK_FINITE, 4u, 0x80000000u};
    size_t bytes = 0;
    for (int op = -1; op <= 8; ++op)
        for (size_t i = 0; i < sizeof ts / sizeof ts[0]; ++i)
            for (size_t j = 0; j < sizeof ns / sizeof ns[0]; ++j)
                for (size_t k = 0; k < sizeof fl / sizeof fl[0]; ++k) {
                    graphic_geom g = geom(ts[i], ns[j], 0, fl[k]);
                    bytes = 0;
                    const graphic_status s = graphic_workspace_size(NULL, op, &g, &bytes);
                    EXPECT(s == GRAPHIC_OK || s == GRAPHIC_ERR_ARG || s == GRAPHIC_ERR_UNSUPPORTED);
                    if (s == GRAPHIC_OK && op == GRAPHIC_OP_ROTATE) {
                        /* the rotation's scratch holds at least one x-sheared frame */
                        const int32_t p = graphic_resolved_pad(&g);
                        EXPECT(bytes >= (size_t)ns[j] * (size_t)p * 4u);
                    }
                }
    graphic_geom g = geom(16, 128, 0, 0);
    EXPECT(graphic_workspace_size(NULL, GRAPHIC_OP_SHIFT, &g, NULL) == GRAPHIC_ERR_ARG);
    EXPECT(graphic_workspace_size(NULL, GRAPHIC_OP_SHIFT, NULL, &bytes) == GRAPHIC_ERR_ARG);
}

static void check_batch_plans(void) {
    static float dummy_f[16];
    static double dummy_d[16];
    graphic_cube_desc d[20];
    memset(d, 0, sizeof d);
    static const int32_t ns[] = {128, 256, 512, 1024, 2048};
    for (int i = 0; i < 20; ++i) {
        d[i].cube = dummy_f;
        d[i].n_frames = 1 + 37 * i;
        d[i].n = ns[i % 5];
        d[i].pad = 0;
        d[i].dx = dummy_d;
        d[i].dy = dummy_d;
        d[i].parang_deg = dummy_d;
        d[i].final_img = dummy_f;
    }
    size_t bytes = 0;
    EXPECT(graphic_batch_workspace_size(NULL, d, 20, 0, &bytes) == GRAPHIC_OK && bytes > 0);
    size_t in_place = 0;
    EXPECT(graphic_batch_workspace_size(NULL, d, 20, GRAPHIC_BATCH_INPLACE, &in_place) == GRAPHIC_OK);
    EXPECT(in_place > 0 && in_place < bytes);
    EXPECT(graphic_batch_workspace_size(NULL, d, 0, 0, &bytes) != GRAPHIC_OK);
    EXPECT(graphic_batch_workspace_size(NULL, NULL, 3, 0, &bytes) != GRAPHIC_OK);
    EXPECT(graphic_batch_workspace_size(NULL, d, 20, 0, NULL) == GRAPHIC_ERR_ARG);
    EXPECT(graphic_batch_workspace_size(NULL, d, -1, 0, &bytes) != GRAPHIC_OK);
    /* frame counts and sizes at and beyond the limits */
    graphic_cube_desc big = d[3];
    big.n_frames = (int64_t)1 << 24;
    big.n = 4096;
    big.pad = 4096;
    EXPECT(graphic_batch_workspace_size(NULL, &big, 1, 0, &bytes) == GRAPHIC_OK);
    big.n_frames = INT64_MAX;
    EXPECT(graphic_batch_workspace_size(NULL, &big, 1, 0, &bytes) != GRAPHIC_OK);
    big.n_frames = 10;
    big.n = 7;
    EXPECT(graphic_batch_workspace_size(NULL, &big, 1, 0, &bytes) != GRAPHIC_OK);
    big.n = 1024;
    big.final_img = NULL;
    EXPECT(graphic_batch_workspace_size(NULL, &big, 1, 0, &bytes) != GRAPHIC_OK);
}

static void check_alpha_min(void) {
    double a = -1.0;
    EXPECT(graphic_alpha_min_deg(1.0, 4.0, 10.0, &a) == GRAPHIC_OK);
    EXPECT(fabs(2.0 * 10.0 * sin(a * M_PI / 360.0) - 4.0) < 1e-12);
    EXPECT(graphic_alpha_min_deg(0.0, 4.0, 10.0, &a) == GRAPHIC_OK && a == 0.0);
    EXPECT(graphic_alpha_min_deg(5.0, 4.0, 10.0, &a) == GRAPHIC_OK && fabs(a - 180.0) < 1e-9);
    EXPECT(graphic_alpha_min_deg(6.0, 4.0, 10.0, &a) == GRAPHIC_ERR_ARG);
    EXPECT(graphic_alpha_min_deg(NAN, 4.0, 10.0, &a) == GRAPHIC_ERR_ARG);
    EXPECT(graphic_alpha_min_deg(1.0, INFINITY, 10.0, &a) == GRAPHIC_ERR_ARG);
    EXPECT(graphic_alpha_min_deg(1.0, 4.0, -1.0, &a) == GRAPHIC_ERR_ARG);
    EXPECT(graphic_alpha_min_deg(1.0, 4.0, 10.0, NULL) == GRAPHIC_ERR_ARG);
}

static void check_null_context(void) {
    graphic_geom g = geom(1, 8, 0, 0);
    float f[64];
    double d[4] = {0, 0, 0, 0};
    EXPECT(graphic_shift(NULL, &g, f, f, d, d, NULL, NULL, 0, NULL) == GRAPHIC_ERR_ARG);
    EXPECT(graphic_rotate(NULL, &g, f, f, d, NULL, NULL, 0, NULL) == GRAPHIC_ERR_ARG);
    EXPECT(graphic_rotate_noalloc(NULL, &g, f, f, d, NULL, NULL) == GRAPHIC_ERR_ARG);
    EXPECT(graphic_median(NULL, &g, f, f, NULL, 0, NULL) == GRAPHIC_ERR_ARG);
    EXPECT(graphic_adi_reduce(NULL, &g, f, d, d, d, f, NULL, NULL, NULL, 0, NULL) == GRAPHIC_ERR_ARG);
    EXPECT(graphic_median_nan(NULL, &g, f, f, NULL) == GRAPHIC_ERR_ARG);
    EXPECT(graphic_parallactic_angles(NULL, d, 1, 0.0, 0.0, 0.0, d, NULL) == GRAPHIC_ERR_ARG);
    EXPECT(graphic_autotune(NULL, &g, NULL, 0, NULL) == GRAPHIC_ERR_ARG);
    EXPECT(graphic_tuning_import(NULL, "col 1024 0 1") == GRAPHIC_ERR_ARG);
    size_t need = 0;
    char buf[16];
    EXPECT(graphic_tuning_export(NULL, buf, sizeof buf, &need) == GRAPHIC_ERR_ARG);
    EXPECT(graphic_timing_enable(NULL, 1) == GRAPHIC_ERR_ARG);
    EXPECT(graphic_graph_launch(NULL, NULL) == GRAPHIC_ERR_ARG);
    graphic_graph_destroy(NULL);
    graphic_destroy(NULL);
}

static void check_context(void) {
    graphic_ctx ctx = NULL;
    const graphic_status s = graphic_create(&ctx, 0);
    if (s != GRAPHIC_OK) {
        /* no GPU on this host: the error is reported, nothing is returned */
        EXPECT(ctx == NULL);
        EXPECT(graphic_create(NULL, 0) == GRAPHIC_ERR_ARG);
        return;
    }
    /* a GPU is present: host-only queries through a live context */
    EXPECT(graphic_tuning_import(ctx, "col 1024 0 1\nnot a line\nmed 3 1\n") != GRAPHIC_OK ||
           graphic_tuning_import(ctx, "col 1024 0 1\n") == GRAPHIC_OK);
    size_t need = 0;
    EXPECT(graphic_tuning_export(ctx, NULL, 0, &need) == GRAPHIC_OK || need > 0);
    graphic_destroy(ctx);
}

int main(void) {
    check_status_strings();
    check_resolved_pad();
    check_workspace_sizes();
    check_batch_plans();
    check_alpha_min();
    check_null_context();
    check_context();
    if (failures) {
        fprintf(stderr, "%d expectation(s) failed\n", failures);
        return 1;
    }
    printf("abi host checks passed\n");
    return 0;
}
