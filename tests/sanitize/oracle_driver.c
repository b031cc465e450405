/*
 * Runs every routine of the FP64 oracle (oracle/oracle.c, linked in) once on
 * small seeded inputs, for builds with the host sanitizers (AddressSanitizer
 * + UndefinedBehaviorSanitizer, or ThreadSanitizer over the OpenMP loops).
 * Test infrastructure: tests/test_oracle_sanitizers.py builds and runs it.
 * It checks only a few invariants that hold whatever the inputs; the results
 * themselves are pinned by the Python tests.  Exit status 0 = clean.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    double L[3];
    double tilt[3];
    int32_t dim;
} orc_box;

void orc_minimum_image(const orc_box* b, double* d, int64_t n);
int orc_ball_count(const orc_box*, const float*, int64_t, const float*, int64_t, double, int32_t,
                   int64_t*);
int orc_ball_fill(const orc_box*, const float*, int64_t, const float*, int64_t, double, int32_t,
                  const int64_t*, int32_t*, double*);
int orc_rdf(const orc_box*, const float*, int64_t, const float*, int64_t, int64_t, double, double,
            int32_t, double, uint64_t*, uint64_t*, uint64_t*);
int orc_ball_rdf_rows(const orc_box*, const float*, int64_t, const float*, int64_t, int64_t, double,
                      int32_t, int64_t, int32_t*, double*, int64_t*, int64_t, double, double,
                      double, uint64_t*, uint64_t*, uint64_t*);
int orc_correlation(const orc_box*, const float*, const float*, int64_t, const float*,
                    const float*, int64_t, int64_t, double, double, int32_t, double, double*,
                    double*, uint64_t*, uint64_t*, uint64_t*);
int orc_knn(const orc_box*, const float*, int64_t, const float*, int64_t, int32_t, int32_t,
            int32_t, double, int32_t*, double*, int32_t*);
int orc_pmft2d(const orc_box*, const float*, int64_t, const float*, const float*, int64_t, int64_t,
               int64_t, double, double, double, int32_t, double, double, uint64_t*, uint64_t*,
               uint64_t*);
int orc_pmft_xyt(const orc_box*, const float*, const float*, int64_t, const float*, const float*,
                 int64_t, int64_t, int64_t, int64_t, double, double, double, int32_t, double,
                 double, double, uint64_t*, uint64_t*, uint64_t*);
int orc_pmft_xyz(const orc_box*, const float*, int64_t, const float*, const float*, int64_t,
                 int64_t, int64_t, int64_t, double, double, double, double, int32_t, double,
                 double, uint64_t*, uint64_t*, uint64_t*);
int orc_smooth_rdf(const orc_box*, const float*, int64_t, int64_t, double, double, double*);
int orc_smooth_rdf_row(const orc_box*, const float*, int64_t, int64_t, const double*, int64_t,
                       double, double, double*);
int orc_smooth_rdf_grad(const orc_box*, const float*, int64_t, int64_t, double, double,
                        const double*, const int64_t*, int64_t, double*);

static uint64_t rng_state = 88172645463325252ull;
static double urand(void) /* xorshift64, uniform [0, 1) */
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) / 9007199254740992.0;
}

static int fail(const char* what)
{
    fprintf(stderr, "invariant failed: %s\n", what);
    return 1;
}

int main(void)
{
    const int64_t n = 400, nq = 150;
    orc_box b3 = {{7.5, 8.0, 8.5}, {0.2, -0.1, 0.15}, 3};
    orc_box b2 = {{9.0, 8.0, 1.0}, {0.25, 0.0, 0.0}, 2};
    float* p = malloc(sizeof(float) * 3 * n);
    float* q = malloc(sizeof(float) * 3 * nq);
    float* th = malloc(sizeof(float) * n);
    float* quat = malloc(sizeof(float) * 4 * nq);
    float* val = malloc(sizeof(float) * 2 * n);
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 3; ++k) p[3 * i + k] = (float)(8.0 * (urand() - 0.5));
        th[i] = (float)(7.0 * urand());
        val[2 * i] = (float)(urand() - 0.5);
        val[2 * i + 1] = (float)(urand() - 0.5);
    }
    for (int64_t i = 0; i < nq; ++i) {
        for (int k = 0; k < 3; ++k) q[3 * i + k] = (float)(8.0 * (urand() - 0.5));
        double s = 0.0;
        for (int k = 0; k < 4; ++k) {
            quat[4 * i + k] = (float)(urand() - 0.5);
            s += quat[4 * i + k] * quat[4 * i + k];
        }
        if (s < 1e-6) quat[4 * i] = 1.0f;
    }
    int bad = 0;
    double d[6] = {5.0, -9.0, 3.3, -0.1, 0.2, 40.0};
    orc_minimum_image(&b3, d, 2);
    if (!(fabs(d[2]) <= 4.25 + 1e-12 && fabs(d[5]) <= 4.25 + 1e-12)) bad |= fail("minimum image");

    const double rmax = 2.9, r2 = rmax * rmax * (1.0 + 1e-5);
    int64_t* cnt = calloc(n, sizeof(int64_t));
    orc_ball_count(&b3, p, n, p, n, r2, 1, cnt);
    int64_t* off = calloc(n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + cnt[i];
    int32_t* idx = malloc(sizeof(int32_t) * (off[n] + 1));
    double* rr = malloc(sizeof(double) * (off[n] + 1));
    orc_ball_fill(&b3, p, n, p, n, r2, 1, off, idx, rr);
    for (int64_t e = 0; e < off[n]; ++e)
        if (!(idx[e] >= 0 && idx[e] < n && rr[e] < r2)) bad |= fail("ball fill");

    uint64_t lo[64], hi[64], amb = 0, lo2[64] = {0}, hi2[64] = {0}, amb2[1] = {0};
    orc_rdf(&b3, p, n, p, n, 40, 0.0, rmax, 1, 1e-5, lo, hi, &amb);
    const int64_t cap = 256;
    int64_t* rc = malloc(sizeof(int64_t) * n);
    int32_t* ri = malloc(sizeof(int32_t) * n * cap);
    double* rr2 = malloc(sizeof(double) * n * cap);
    orc_ball_rdf_rows(&b3, p, n, p, n, 0, r2, 1, cap, ri, rr2, rc, 40, 0.0, rmax, 1e-5, lo2, hi2,
                      amb2);
    for (int k = 0; k < 40; ++k)
        if (lo[k] != lo2[k] || hi[k] != hi2[k] || lo[k] > hi[k]) bad |= fail("rdf rows");
    for (int64_t i = 0; i < n; ++i)
        if (rc[i] != cnt[i]) bad |= fail("row counts");

    double sc[2 * 30], am[30];
    uint64_t clo[30], chi[30], camb;
    orc_correlation(&b3, p, val, n, q, val, nq, 30, 0.2, rmax, 0, 1e-5, sc, am, clo, chi, &camb);

    int32_t ki[150 * 14], kl[150];
    double kr[150 * 14];
    orc_knn(&b3, p, n, q, nq, 12, 2, 0, 0.0, ki, kr, kl);
    for (int64_t i = 0; i < nq; ++i)
        for (int t = 1; t < kl[i]; ++t)
            if (kr[i * 14 + t] < kr[i * 14 + t - 1]) bad |= fail("knn order");

    uint64_t plo[20 * 24], phi[20 * 24], pamb;
    orc_pmft2d(&b2, p, n, q, th, nq, 20, 24, 2.5, 2.5, 2.5, 0, 1e-5, 2.5e-5, plo, phi, &pamb);
    uint64_t tlo[10 * 10 * 6], thi[10 * 10 * 6], tamb;
    orc_pmft_xyt(&b2, p, th, n, p, th, n, 10, 10, 6, 2.0, 2.0, 2.0, 1, 1e-5, 2e-5, 6.3e-5, tlo, thi,
                 &tamb);
    uint64_t zlo[8 * 8 * 8], zhi[8 * 8 * 8], zamb;
    orc_pmft_xyz(&b3, p, n, q, quat, nq, 8, 8, 8, 2.0, 2.0, 2.0, 2.0, 0, 1e-5, 2e-5, zlo, zhi, &zamb);

    double h[60], hrow[60], gh[60], grad[3 * 5];
    orc_smooth_rdf(&b3, p, n, 60, 3.0, 0.05, h);
    double pk[3] = {p[0], p[1], p[2]};
    orc_smooth_rdf_row(&b3, p, n, 0, pk, 60, 3.0, 0.05, hrow);
    for (int k = 0; k < 60; ++k) gh[k] = urand() - 0.5;
    const int64_t rows[5] = {0, 3, 77, 150, 399};
    orc_smooth_rdf_grad(&b3, p, n, 60, 3.0, 0.05, gh, rows, 5, grad);
    for (int k = 0; k < 15; ++k)
        if (!isfinite(grad[k])) bad |= fail("smoothed gradient");

    free(p); free(q); free(th); free(quat); free(val); free(cnt); free(off); free(idx); free(rr);
    free(rc); free(ri); free(rr2);
    if (!bad) printf("oracle driver: clean\n");
    return bad;
}
