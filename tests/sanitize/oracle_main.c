/* Drives the CPU oracle through all of its entry points on seeded synthetic
 * light curves and edge cases, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers_cpu.py).  Prints one
 * checksum line; any sanitizer report fails the test. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void ora_periodogram(int method, int64_t n_obj, const int64_t *offsets, const double *t,
                     const double *y, const double *e, double fmin, double fmax,
                     int64_t n_freq, const int64_t *ks, int64_t nk, const double *spans,
                     double alpha, double fixed_span, double *pgram, int32_t *status);
int64_t ora_best(int64_t nk, const double *p);
void ora_smooth(int n, const double *x, const double *v, const double *w, double span,
                int periodic, int cv, double vsmlsq, double *s, double *r, double *lev);
double ora_pdm(int n, const double *tt, const double *y, const double *w, double ybar,
               double chi0, double f, int B);

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double uni(void)
{
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rng_state >> 11) * 0x1p-53;
}

int main(void)
{
    /* objects: lengths (with a too-short one), one with a bad error bar, one
     * with a NaN magnitude, one of constant magnitude, one with repeated
     * times (ties), a dense one */
    const int lens[] = {5, 4, 37, 60, 8, 9, 120, 300};
    const int n_obj = (int)(sizeof(lens) / sizeof(lens[0]));
    int64_t offsets[sizeof(lens) / sizeof(lens[0]) + 1];
    offsets[0] = 0;
    for (int o = 0; o < n_obj; ++o) offsets[o + 1] = offsets[o] + lens[o];
    const int64_t total = offsets[n_obj];
    double *t = malloc(total * sizeof(double)), *y = malloc(total * sizeof(double)),
           *e = malloc(total * sizeof(double));
    for (int o = 0; o < n_obj; ++o) {
        double tc = 0.0;
        for (int64_t i = offsets[o]; i < offsets[o + 1]; ++i) {
            if (o == 6 && (i - offsets[o]) % 2 == 1)
                t[i] = t[i - 1];  /* repeated times */
            else
                t[i] = (tc += 0.5 + 20.0 * uni());
            y[i] = 15.0 + 0.3 * sin(6.283185307179586 * t[i] / 1.7) + 0.05 * (uni() - 0.5);
            e[i] = 0.02 + 0.05 * uni();
        }
    }
    e[offsets[3] + 2] = 0.0;            /* bad error bar */
    y[offsets[4] + 1] = NAN;            /* non-finite magnitude */
    for (int64_t i = offsets[5]; i < offsets[6]; ++i) y[i] = 14.0;  /* constant */
    const double spans[3] = {0.05, 0.2, 0.5};
    const int64_t n_freq = 41;
    double *pg = malloc(n_obj * n_freq * sizeof(double));
    int32_t status[sizeof(lens) / sizeof(lens[0])];
    double check = 0.0;
    const double alphas[3] = {0.0, 4.5, 9.0};
    for (int method = 0; method < 3; ++method) {
        for (int a = 0; a < 3; ++a) {
            for (int fixed = 0; fixed < 2; ++fixed) {
                ora_periodogram(method, n_obj, offsets, t, y, e, 0.05, 3.0, n_freq, NULL, 0,
                                spans, alphas[a], fixed ? 0.3 : 0.0, pg, status);
                for (int o = 0; o < n_obj; ++o) {
                    int64_t b = ora_best(n_freq, pg + o * n_freq);
                    check += (double)(b + 1) + (b >= 0 ? pg[o * n_freq + b] : 0.0) + status[o];
                }
            }
        }
    }
    /* selected indices */
    const int64_t ks[4] = {0, 7, 7, 40};
    ora_periodogram(0, n_obj, offsets, t, y, e, 0.05, 3.0, n_freq, ks, 4, spans, 9.0, 0.0, pg,
                    status);
    check += pg[6 * 4 + 3];
    /* the smoother alone: periodic and not, with leverage, on tied abscissae */
    enum { N = 11 };
    double x[N], v[N], w[N], s[N], r[N], lev[N];
    for (int j = 0; j < N; ++j) {
        x[j] = (double)(j / 2) / 6.0;
        v[j] = sin(6.0 * x[j]);
        w[j] = 1.0 + j;
    }
    for (int per = 0; per < 2; ++per) {
        ora_smooth(N, x, v, w, 0.3, per, 1, 1e-9, s, r, lev);
        for (int j = 0; j < N; ++j) check += s[j] + r[j] + lev[j];
    }
    /* the phase-dispersion score */
    check += ora_pdm(lens[7], t + offsets[7], y + offsets[7], e + offsets[7], 15.0, 1.0, 0.59, 8);
    printf("oracle checksum %.17g\n", check);
    free(t);
    free(y);
    free(e);
    free(pg);
    return isfinite(check) ? 0 : 1;
}
