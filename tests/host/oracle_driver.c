/*
 * A plain C driver of the CPU oracle (oracle/oracle.c), built with the
 * address and undefined-behaviour sanitizers: every exported entry point runs
 * on small shapes of each kind (sigma = 2, 3, 4; d = 2, 3), including the
 * float, sampled and two-array variants, and a few results are checked
 * against closed forms (the l = 1 limits 2/(sigma+1) and 2/3).  Exits
 * non-zero on a failed check; the sanitizers abort on a memory or
 * undefined-behaviour error.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    double R, maxW, E, bound, rho;
    uint64_t argmax_W, nonfinite;
} cert_t;
typedef struct {
    double r, bound;
    uint64_t argmin, nonfinite;
} cert_opt_t;

uint64_t or_num_entries(int, int, int);
int or_decode(int, int, int, uint64_t, int *);
uint64_t or_encode(int, int, int, const int *);
int or_sweep(int, int, int, const double *const *, double *);
int or_sweep_at(int, int, int, const double *const *, const uint64_t *, uint64_t, double *);
int or_sweep_at_f32(int, int, int, const float *const *, const uint64_t *, uint64_t, double *);
int or_certify(int, int, int, const double *, const double *, cert_t *);
int or_certify_W_at(int, int, int, const double *, double, const uint64_t *, uint64_t, double *);
int or_certify_W_at_f32(int, int, int, const float *, double, const uint64_t *, uint64_t,
                        double *);
int or_certify_optimal(int, int, int, const double *, cert_opt_t *);
int or_certify_optimal_f32(int, int, int, const float *, cert_opt_t *);
int or_optimal_ratio_at(int, int, int, const double *, const uint64_t *, uint64_t, double *);
int or_two_array_step(int, int, int, const double *, double, double *);
int or_two_array_step_at(int, int, int, const double *, double, const uint64_t *, uint64_t,
                         double *);
int or_sample_growth(int, int, int, const double *, const double *, double *);
int or_sample_coordinates(int, int, int, uint64_t *);
int or_max_diff(const double *, const double *, uint64_t, double *, uint64_t *);
int or_max_diff_f32(const float *, const float *, uint64_t, double *, uint64_t *);
int or_feasible_triplet(int, int, int, int64_t, int64_t, double *, double *, double *);
int or_brute_W(int, int, int, int, const int *, uint64_t *);

static int failures = 0;
#define CHECK(c, ...)                               \
    do {                                            \
        if (!(c)) {                                 \
            ++failures;                             \
            printf("FAIL line %d: ", __LINE__);     \
            printf(__VA_ARGS__);                    \
            printf("\n");                           \
        }                                           \
    } while (0)

static void shape(int sigma, int d, int h)
{
    const uint64_t n = or_num_entries(sigma, d, h);
    CHECK(n > 0, "num_entries %d %d %d", sigma, d, h);
    double *u = malloc(n * sizeof *u), *p = malloc(n * sizeof *p), *o = malloc(n * sizeof *o);
    float *uf = malloc(n * sizeof *uf), *pf = malloc(n * sizeof *pf);
    int *sym = malloc(sizeof(int) * (size_t)(d * h));
    uint64_t idx[5] = {0, 1, n / 3, n / 2, n - 1};
    double at[5];
    for (uint64_t i = 0; i < n; ++i) {
        u[i] = (double)((i * 2654435761u) % 1000) / 125.0;
        p[i] = u[i] - 0.4 - (double)(i % 7) / 64.0;
        uf[i] = (float)u[i];
        pf[i] = (float)p[i];
    }
    for (int k = 0; k < 5; ++k) {
        CHECK(or_decode(sigma, d, h, idx[k], sym) == 0, "decode");
        CHECK(or_encode(sigma, d, h, sym) == idx[k], "encode(decode(i)) != i");
    }
    const double *lags[3] = {u, p, p};
    const float *lagsf[3] = {uf, pf, pf};
    CHECK(or_sweep(sigma, d, h, lags, o) == 0, "sweep");
    CHECK(or_sweep_at(sigma, d, h, lags, idx, 5, at) == 0, "sweep_at");
    for (int k = 0; k < 5; ++k) CHECK(at[k] == o[idx[k]], "sweep_at != sweep");
    CHECK(or_sweep_at_f32(sigma, d, h, lagsf, idx, 5, at) == 0, "sweep_at_f32");
    cert_t c;
    CHECK(or_certify(sigma, d, h, u, p, &c) == 0, "certify");
    CHECK(or_certify_W_at(sigma, d, h, u, c.R, idx, 5, at) == 0, "W_at");
    for (int k = 0; k < 5; ++k) CHECK(at[k] <= c.maxW, "W_at above maxW");
    CHECK(or_certify_W_at_f32(sigma, d, h, uf, c.R, idx, 5, at) == 0, "W_at_f32");
    cert_opt_t q;
    CHECK(or_certify_optimal(sigma, d, h, u, &q) == 0, "optimal");
    CHECK(or_optimal_ratio_at(sigma, d, h, u, idx, 5, at) == 0, "ratio_at");
    for (int k = 0; k < 5; ++k) CHECK(at[k] >= q.r, "ratio below r");
    CHECK(or_certify_optimal_f32(sigma, d, h, uf, &q) == 0, "optimal_f32");
    double R;
    uint64_t arg;
    CHECK(or_max_diff(u, p, n, &R, &arg) == 0 && R == c.R, "max_diff");
    CHECK(or_max_diff_f32(uf, pf, n, &R, &arg) == 0, "max_diff_f32");
    CHECK(or_two_array_step(sigma, d, h, u, 0.37, o) == 0, "two_array_step");
    CHECK(or_two_array_step_at(sigma, d, h, u, 0.37, idx, 5, at) == 0, "two_array_step_at");
    for (int k = 0; k < 5; ++k) CHECK(at[k] == o[idx[k]], "two_array_step_at != step");
    CHECK(or_sample_growth(sigma, d, h, o, u, &R) == 0 && isfinite(R), "sample_growth");
    uint64_t *cs = malloc(4096 * sizeof *cs);
    CHECK(or_sample_coordinates(sigma, d, h, cs) == 0, "sample_coordinates");
    for (int k = 0; k < 4096; ++k) CHECK(cs[k] < n / (uint64_t)sigma, "sample outside the half");
    free(cs); free(u); free(p); free(o); free(uf); free(pf); free(sym);
}

int main(void)
{
    shape(2, 2, 1); shape(2, 2, 3); shape(2, 2, 6);
    shape(4, 2, 1); shape(4, 2, 2);
    shape(2, 3, 1); shape(2, 3, 3);
    shape(3, 2, 2);
    /* closed forms at l = 1 */
    double best[4];
    CHECK(or_feasible_triplet(2, 2, 1, 80, 1, NULL, best, NULL) == 0, "triplet");
    CHECK(fabs(best[3] - 2.0 / 3.0) < 1e-9, "sigma = d = 2, l = 1: %.12f", best[3]);
    CHECK(or_feasible_triplet(4, 2, 1, 80, 1, NULL, best, NULL) == 0, "triplet");
    CHECK(fabs(best[3] - 0.4) < 1e-9, "sigma = 4, d = 2, l = 1: %.12f", best[3]);
    CHECK(or_feasible_triplet(2, 3, 1, 120, 1, NULL, best, NULL) == 0, "triplet");
    CHECK(fabs(best[3] - 2.0 / 3.0) < 1e-9, "sigma = 2, d = 3, l = 1: %.12f", best[3]);
    double hist[4 * 20], ring[2 * 16];
    CHECK(or_feasible_triplet(2, 2, 2, 20, 1, hist, best, ring) == 0, "triplet with history");
    int heads[4] = {0, 1, 1, 0};
    uint64_t sum;
    CHECK(or_brute_W(2, 2, 2, 3, heads, &sum) == 0 && sum > 0, "brute_W");
    printf("%s (%d failed checks)\n", failures ? "FAIL" : "ok", failures);
    return failures != 0;
}
