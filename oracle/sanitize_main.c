/*
 * sanitize_main.c -- TEST INFRASTRUCTURE ONLY.  A driver that calls every
 * entry point of oracle.c on small grids (including the smallest, n = 3,
 * zero steps, windows at both ends and a final cotangent) and on invalid
 * arguments, so that tests/test_oracle_sanitizers.py can run the oracle
 * under AddressSanitizer and UndefinedBehaviorSanitizer.  It checks return
 * codes and that the results are finite; the values themselves are pinned
 * by the other oracle tests.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_max_threads(void);
int oracle_heat_f64(double *u, int64_t n, int64_t nsteps, double r, int nthreads);
int oracle_heat_f32(float *u, int64_t n, int64_t nsteps, float r, int nthreads);
int oracle_ks_f64(double *u, int64_t n, int64_t nsteps, double dt, double dx, int nthreads);
int oracle_heat_fma_f64(double *u, int64_t n, int64_t nsteps, double r, int nthreads);
int oracle_heat_fma_f32(float *u, int64_t n, int64_t nsteps, float r, int nthreads);
int oracle_ks_fma_f64(double *u, int64_t n, int64_t nsteps, double dt, double dx, int nthreads);
int oracle_heat_f64_points(const double *u0, int64_t n, int64_t nsteps, double r,
                           const int64_t *idx, int64_t count, double *out);
int oracle_heat_f32_points(const float *u0, int64_t n, int64_t nsteps, float r,
                           const int64_t *idx, int64_t count, float *out);
int oracle_ks_f64_points(const double *u0, int64_t n, int64_t nsteps, double dt, double dx,
                         const int64_t *idx, int64_t count, double *out);
int oracle_heat_f64_adjoint(const double *u0, int64_t n, int64_t nsteps, double r, int64_t n0,
                            double wgt, const double *cot_final, double *grad, int nthreads);
int oracle_ks_f64_adjoint(const double *u0, int64_t n, int64_t nsteps, double dt, double dx,
                          int64_t n0, double wgt, const double *cot_final, double *grad,
                          int nthreads);
int oracle_ks_f64_tlm(const double *u0, int64_t n, int64_t nsteps, double dt, double dx,
                      int64_t n0, double wgt, const double *cot_final, const double *dirs,
                      int64_t ndirs, double *dJ, int nthreads);
int oracle_euler_f64(double *q, int64_t n, int64_t nsteps, double dt, double dx, double gamma,
                     int nthreads);

static int failures = 0;

static void expect(int cond, const char *what)
{
    if (!cond) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

static void fill(double *u, int64_t n, unsigned seed)
{
    for (int64_t i = 0; i < n; ++i) {
        seed = seed * 1103515245u + 12345u;
        u[i] = ((double)(seed >> 8) / 16777216.0) - 0.5;
    }
}

static int finite_all(const double *u, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(u[i]))
            return 0;
    return 1;
}

int main(void)
{
    const int64_t sizes[] = {3, 4, 7, 64, 129};
    expect(oracle_max_threads() >= 1, "max_threads");
    for (unsigned si = 0; si < sizeof sizes / sizeof sizes[0]; ++si) {
        const int64_t n = sizes[si];
        double *u = malloc((size_t)n * sizeof *u), *g = malloc((size_t)n * sizeof *g);
        double *c = malloc((size_t)n * sizeof *c), *d = malloc((size_t)(3 * n) * sizeof *d);
        float *f = malloc((size_t)n * sizeof *f);
        double *q = malloc((size_t)(3 * n) * sizeof *q);
        int64_t idx[3] = {0, n / 2, n - 1};
        double out[3], dJ[3];
        float outf[3];
        for (int64_t steps = 0; steps <= 5; steps += 5) {
            fill(u, n, 1u + (unsigned)n);
            for (int64_t i = 0; i < n; ++i)
                f[i] = (float)u[i];
            expect(oracle_heat_f64(u, n, steps, 0.3, 2) == 0, "heat_f64");
            expect(oracle_heat_f32(f, n, steps, 0.3f, 2) == 0, "heat_f32");
            expect(oracle_heat_fma_f64(u, n, steps, 0.3, 2) == 0, "heat_fma_f64");
            expect(oracle_heat_fma_f32(f, n, steps, 0.3f, 2) == 0, "heat_fma_f32");
            expect(oracle_ks_f64(u, n, steps, 0.005, 0.5, 2) == 0, "ks_f64");
            expect(oracle_ks_fma_f64(u, n, steps, 0.005, 0.5, 2) == 0, "ks_fma_f64");
            expect(finite_all(u, n), "finite forward results");
            expect(oracle_heat_f64_points(u, n, steps, 0.3, idx, 3, out) == 0, "heat points");
            expect(oracle_heat_f32_points(f, n, steps, 0.3f, idx, 3, outf) == 0, "heat f32 points");
            expect(oracle_ks_f64_points(u, n, steps, 0.005, 0.5, idx, 3, out) == 0, "ks points");
            fill(c, n, 7u);
            fill(d, 3 * n, 9u);
            for (int64_t n0 = -1; n0 <= steps + 1; n0 += (steps + 2)) {
                expect(oracle_heat_f64_adjoint(u, n, steps, 0.3, n0, 0.1, c, g, 2) == 0,
                       "heat adjoint");
                expect(oracle_ks_f64_adjoint(u, n, steps, 0.005, 0.5, n0, 0.1, c, g, 2) == 0,
                       "ks adjoint");
                expect(oracle_ks_f64_adjoint(u, n, steps, 0.005, 0.5, n0, 0.1, NULL, g, 2) == 0,
                       "ks adjoint without cotangent");
                expect(finite_all(g, n), "finite gradients");
                expect(oracle_ks_f64_tlm(u, n, steps, 0.005, 0.5, n0, 0.1, c, d, 3, dJ, 2) == 0,
                       "ks tlm");
                expect(finite_all(dJ, 3), "finite tangent-linear derivatives");
            }
            for (int64_t i = 0; i < n; ++i) {
                const double rho = 1.0 + 0.2 * u[i], m = 0.1 * u[i], p = 1.0;
                q[3 * i] = rho;
                q[3 * i + 1] = m;
                q[3 * i + 2] = p / 0.4 + 0.5 * m * m / rho;
            }
            expect(oracle_euler_f64(q, n, steps, 0.2 / (double)n, 1.0 / (double)n, 1.4, 2) == 0,
                   "euler");
            expect(finite_all(q, 3 * n), "finite Euler results");
        }
        /* invalid arguments are rejected, not run */
        expect(oracle_heat_f64(u, 2, 1, 0.3, 1) != 0, "heat rejects n < 3");
        expect(oracle_ks_f64(u, n, -1, 0.005, 0.5, 1) != 0, "ks rejects negative steps");
        expect(oracle_ks_f64(u, n, 1, 0.005, 0.0, 1) != 0, "ks rejects dx = 0");
        expect(oracle_ks_f64_tlm(u, n, 1, 0.005, 0.5, 0, 0.1, NULL, d, 0, dJ, 1) != 0,
               "tlm rejects zero directions");
        expect(oracle_euler_f64(NULL, n, 1, 0.1, 0.1, 1.4, 1) != 0, "euler rejects NULL");
        free(u); free(g); free(c); free(d); free(f); free(q);
    }
    if (failures)
        return 1;
    printf("oracle sanitizer driver: all entry points ran clean\n");
    return 0;
}
