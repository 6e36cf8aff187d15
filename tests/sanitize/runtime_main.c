/* Drives the host-side entry points of the runtime library that need no
 * GPU -- argument checks and their error messages, the shape table, the bin
 * table, the model file format (round trip, truncated, foreign and missing
 * files) -- for a build whose host code runs under AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers_cpu.py).  argv[1]: a
 * scratch directory.  Exit status 0 when every call returned what it
 * should; any sanitizer report fails the test. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ssgpu.h"

static int failures = 0;
#define EXPECT(cond)                                                        \
    do {                                                                    \
        if (!(cond)) {                                                      \
            fprintf(stderr, "line %d: expectation failed: %s\n", __LINE__, \
                    #cond);                                                 \
            ++failures;                                                     \
        }                                                                   \
    } while (0)

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    char path[4096], bad[4096];
    snprintf(path, sizeof(path), "%s/model.ssm", argv[1]);
    snprintf(bad, sizeof(bad), "%s/truncated.ssm", argv[1]);

    EXPECT(ss_version() > 0);
    ss_params p;
    ss_params_default(&p);
    EXPECT(p.span_min == 0.05 && p.span_mid == 0.2 && p.span_max == 0.5 && p.flags == 0);
    const int ns = ss_num_shapes();
    EXPECT(ns > 0);
    for (int i = -1; i <= ns; ++i) {
        int32_t nw = 0, ppl = 0;
        int rc = ss_shape_info(i, &nw, &ppl);
        EXPECT((i >= 0 && i < ns) ? (rc == SS_OK && nw > 0 && ppl > 0) : rc == SS_ERR_INVALID_ARG);
    }
    EXPECT(ss_shape_info(0, NULL, NULL) == SS_ERR_INVALID_ARG);

    /* the bin table of a few grids, and refused grids */
    const ss_grid grids[3] = {{0.05, 20.0, 50000}, {0.1, 10.0, 20000}, {1.0, 1.5, 3}};
    int64_t *first = malloc(sizeof(int64_t) * 1025);
    for (int g = 0; g < 3; ++g) {
        EXPECT(ss_bin_table(&grids[g], first) == SS_OK);
        EXPECT(first[0] == 0 && first[1024] == grids[g].n_freq);
        for (int b = 0; b < 1024; ++b) EXPECT(first[b] <= first[b + 1]);
    }
    const ss_grid bad_grid = {2.0, 1.0, 10};
    EXPECT(ss_bin_table(&bad_grid, first) == SS_ERR_INVALID_ARG);
    EXPECT(strlen(ss_last_error()) > 0);
    EXPECT(ss_bin_table(NULL, first) == SS_ERR_INVALID_ARG);

    /* calls that fail on their arguments before touching a device */
    ss_catalog cat = {1, 5, NULL, NULL, NULL, NULL};
    EXPECT(ss_periodogram(NULL, &cat, &grids[1], &p, NULL, NULL, NULL) == SS_ERR_INVALID_ARG);
    EXPECT(ss_best_period(NULL, 0, &cat, &grids[1], &p, NULL, NULL, NULL, NULL, NULL) ==
           SS_ERR_INVALID_ARG);
    int64_t per = 0, nb = 0;
    EXPECT(ss_plan_batches(NULL, 10, 100, &grids[1], SS_FP64, 1, 0.75, 1 << 20, &per, &nb) ==
           SS_ERR_INVALID_ARG);
    EXPECT(ss_ctx_check_counts(NULL, NULL) == SS_ERR_INVALID_ARG);

    /* the model file: round trip, then a truncated copy, a foreign file and a
     * missing one */
    const int np = ss_enc_num_params();
    EXPECT(np > 0);
    float *a = malloc(sizeof(float) * np * 6);
    float *m = a + np, *v = a + 2 * np, *a2 = a + 3 * np, *m2 = a + 4 * np, *v2 = a + 5 * np;
    for (int i = 0; i < np; ++i) {
        a[i] = (float)i * 1e-3f - 7.0f;
        m[i] = (float)(i % 13) * 0.25f;
        v[i] = (float)(i % 7) * 0.5f;
    }
    EXPECT(ss_model_file_write(path, &grids[0], 42, a, m, v) == SS_OK);
    ss_grid g2;
    int32_t step = 0;
    EXPECT(ss_model_file_read(path, &g2, &step, a2, m2, v2) == SS_OK);
    EXPECT(step == 42 && g2.f_min == grids[0].f_min && g2.f_max == grids[0].f_max &&
           g2.n_freq == grids[0].n_freq);
    EXPECT(memcmp(a, a2, sizeof(float) * np) == 0 && memcmp(m, m2, sizeof(float) * np) == 0 &&
           memcmp(v, v2, sizeof(float) * np) == 0);
    FILE *in = fopen(path, "rb");
    FILE *out = fopen(bad, "wb");
    EXPECT(in && out);
    if (in && out) {
        char buf[4096];
        size_t want = 3000, got = fread(buf, 1, want, in);
        fwrite(buf, 1, got, out);
    }
    if (in) fclose(in);
    if (out) fclose(out);
    EXPECT(ss_model_file_read(bad, &g2, &step, a2, m2, v2) == SS_ERR_INVALID_ARG);
    out = fopen(bad, "wb");
    if (out) {
        fputs("not a model file at all", out);
        fclose(out);
    }
    EXPECT(ss_model_file_read(bad, &g2, &step, a2, m2, v2) == SS_ERR_INVALID_ARG);
    EXPECT(ss_model_file_read("/nonexistent/dir/model.ssm", &g2, &step, a2, m2, v2) ==
           SS_ERR_INVALID_ARG);
    EXPECT(ss_model_file_write(path, NULL, 0, a, m, v) == SS_ERR_INVALID_ARG);
    free(a);
    free(first);
    printf("runtime checks: %d failure(s)\n", failures);
    return failures == 0 ? 0 : 1;
}
