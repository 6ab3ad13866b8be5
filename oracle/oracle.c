/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.  A plain, slow, obviously correct CPU
 * implementation of what the swept rule computes.  Only tests, the smoke
 * check and the benchmark's CPU-baseline leg may load this code; the product
 * path never calls it.  It shares no source with the HIP library.
 *
 * What is computed.  The swept rule (paper, Sections 2-3) does not change the
 * numbers a time-stepper produces: it only reorders the per-point sub-timestep
 * updates in space-time so that nodes communicate once per many sub-timesteps,
 * with no redundant work.  So the oracle is the plain definition: apply the
 * sub-timestep update to every point of the periodic 1D grid (Section 3: the
 * domain is periodic, every point has a left and a right neighbour), one
 * sub-timestep after the other, from two full-grid buffers.
 *
 * Schemes (the paper fixes their structure, not every rounding; the readings
 * below are the oracle's definition and every GPU path must reproduce them
 * bit for bit):
 *
 *  Heat, 3-point finite difference with forward Euler (Section 4 names this
 *  scheme as the cheapest sub-timestep, "3 FLOPs"); one sub-timestep per step:
 *      u'[i] = u[i] + r * ((u[i-1] + u[i+1]) - 2*u[i])
 *  evaluated in exactly that association, in the storage precision
 *  (binary64 or binary32), with no fused multiply-add.
 *
 *  Kuramoto-Sivashinsky u_t = -u u_x - u_xx - u_xxxx (Section 6: finite
 *  differences in space, explicit second-order Runge-Kutta in time).  The RK2
 *  midpoint rule is split into four radius-1 sub-timesteps that forward the
 *  variables the next one needs (Section 2: a sub-timestep reads the inputs
 *  of a point and of its two neighbours and forwards unused variables):
 *      D2(a)[i]  = ((a[i-1] + a[i+1]) - 2*a[i]) * c2          c2 = 1/(dx*dx)
 *      D1(a)[i]  = (a[i+1] - a[i-1]) * c1                     c1 = 1/(2*dx)
 *      F(a,b)[i] = -(((a[i]*D1(a)[i]) + b[i]) + D2(b)[i])
 *      sub0: (u)      -> (u, w),    w  = D2(u)
 *      sub1: (u,w)    -> (u, v),    v  = u + h*F(u,w)          h  = dt/2
 *      sub2: (u,v)    -> (u, v, z), z  = D2(v)
 *      sub3: (u,v,z)  -> (u'),      u' = u + dt*F(v,z)
 *  F(u,w) is the right-hand side with u_xxxx = D2(D2 u); the midpoint stage
 *  follows the two-stage Runge-Kutta example of Section 2.  The constants
 *  c1, c2, h are rounded once, here, exactly as written above.
 *
 *  Euler equations of gas dynamics (Section 7: second-order finite volume,
 *  minmod limiter, interface flux with scalar dissipation proportional to the
 *  spectral radius of the Roe matrix, midpoint Runge-Kutta; Section 2: a
 *  second-order finite-volume step is one slope sub-timestep plus one
 *  flux-difference sub-timestep, so the midpoint rule takes four).  A cell
 *  holds q = (rho, m = rho*u, E); gamma is a parameter, gm1 = gamma - 1:
 *      u = m/rho,  p = gm1*(E - 0.5*(m*u)),  f(q) = (m, m*u + p, (E + p)*u)
 *      minmod(a,b) = min(a,b) if a,b > 0;  max(a,b) if a,b < 0;  else 0
 *      slope(q)[i] = minmod(q[i] - q[i-1], q[i+1] - q[i])  (per component)
 *      face i+1/2: qL = q[i] + 0.5*s[i],  qR = q[i+1] - 0.5*s[i+1]
 *        Roe average with a = sqrt(rhoL), b = sqrt(rhoR), H = (E + p)/rho:
 *        ur = (a*uL + b*uR)/(a + b),  Hr = (a*HL + b*HR)/(a + b),
 *        cr2 = gm1*(Hr - 0.5*(ur*ur)),  lam = |ur| + sqrt(cr2)  (0 if cr2 <= 0)
 *        F = 0.5*(f(qL) + f(qR)) - (0.5*lam)*(qR - qL)
 *      sub0: (q)       -> (q, s),    s  = slope(q)
 *      sub1: (q, s)    -> (q, r),    r  = q - ch*(F[i+1/2] - F[i-1/2])   ch = (0.5*dt)/dx
 *      sub2: (q, r)    -> (q, r, s), s  = slope(r)
 *      sub3: (q, r, s) -> (q'),      q' = q - cf*(F[i+1/2] - F[i-1/2])   cf = dt/dx
 *  with the fluxes of sub1 from (q, s) and those of sub3 from (r, s).  Each
 *  cell evaluates both of its faces (the face i+1/2 of cell i and the face
 *  i-1/2 of cell i+1 are the same function of the same inputs, so they are
 *  equal bit for bit and the scheme stays conservative).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 * -ffp-contract=off is required so that no multiply-add is fused.  OpenMP
 * only splits the independent per-point loop of a sub-timestep, so results do
 * not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-3)

static int64_t wrap(int64_t i, int64_t n)
{
    int64_t m = i % n;
    return m < 0 ? m + n : m;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ heat */

/* One forward-Euler heat sub-timestep on the whole periodic grid. */
static void heat_step_f64(const double *a, double *b, int64_t n, double r)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        double left = a[wrap(i - 1, n)];
        double mid = a[i];
        double right = a[wrap(i + 1, n)];
        double lap = (left + right) - 2.0 * mid;
        b[i] = mid + r * lap;
    }
}

static void heat_step_f32(const float *a, float *b, int64_t n, float r)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        float left = a[wrap(i - 1, n)];
        float mid = a[i];
        float right = a[wrap(i + 1, n)];
        float lap = (left + right) - 2.0f * mid;
        b[i] = mid + r * lap;
    }
}

/* Advance u (n points, in place) by nsteps heat steps with coefficient r. */
int oracle_heat_f64(double *u, int64_t n, int64_t nsteps, double r, int nthreads)
{
    double *a, *b, *t;
    int64_t s;
    if (!u || n < 3 || nsteps < 0)
        return ORACLE_EINVAL;
    set_threads(nthreads);
    b = (double *)malloc((size_t)n * sizeof(double));
    if (!b)
        return ORACLE_ENOMEM;
    a = u;
    for (s = 0; s < nsteps; ++s) {
        heat_step_f64(a, b, n, r);
        t = a; a = b; b = t;
    }
    if (a != u) {
        memcpy(u, a, (size_t)n * sizeof(double));
        free(a);
    } else {
        free(b);
    }
    return ORACLE_OK;
}

int oracle_heat_f32(float *u, int64_t n, int64_t nsteps, float r, int nthreads)
{
    float *a, *b, *t;
    int64_t s;
    if (!u || n < 3 || nsteps < 0)
        return ORACLE_EINVAL;
    set_threads(nthreads);
    b = (float *)malloc((size_t)n * sizeof(float));
    if (!b)
        return ORACLE_ENOMEM;
    a = u;
    for (s = 0; s < nsteps; ++s) {
        heat_step_f32(a, b, n, r);
        t = a; a = b; b = t;
    }
    if (a != u) {
        memcpy(u, a, (size_t)n * sizeof(float));
        free(a);
    } else {
        free(b);
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------ Kuramoto-Sivashinsky */

typedef struct {
    double dt, h, c1, c2;
} ks_consts;

static ks_consts ks_make(double dt, double dx)
{
    ks_consts k;
    k.dt = dt;
    k.h = 0.5 * dt;
    k.c1 = 1.0 / (2.0 * dx);
    k.c2 = 1.0 / (dx * dx);
    return k;
}

/* -( (a_i * D1(a)_i + b_i) + D2(b)_i ), from the three neighbours of a and b */
static double ks_rhs(double al, double am, double ar,
                     double bl, double bm, double br, const ks_consts *k)
{
    double d1a = (ar - al) * k->c1;
    double d2b = ((bl + br) - 2.0 * bm) * k->c2;
    return -(((am * d1a) + bm) + d2b);
}

static double ks_d2(double l, double m, double r, const ks_consts *k)
{
    return ((l + r) - 2.0 * m) * k->c2;
}

/* Advance u (n points, in place) by nsteps RK2 steps = 4*nsteps sub-timesteps. */
int oracle_ks_f64(double *u, int64_t n, int64_t nsteps, double dt, double dx,
                  int nthreads)
{
    ks_consts k;
    double *un, *w, *v, *z;
    int64_t s, i;
    if (!u || n < 3 || nsteps < 0 || !(dx > 0.0))
        return ORACLE_EINVAL;
    set_threads(nthreads);
    k = ks_make(dt, dx);
    un = (double *)malloc((size_t)n * sizeof(double));
    w = (double *)malloc((size_t)n * sizeof(double));
    v = (double *)malloc((size_t)n * sizeof(double));
    z = (double *)malloc((size_t)n * sizeof(double));
    if (!un || !w || !v || !z) {
        free(un); free(w); free(v); free(z);
        return ORACLE_ENOMEM;
    }
    for (s = 0; s < nsteps; ++s) {
        /* sub0: w = D2(u) */
#pragma omp parallel for schedule(static)
        for (i = 0; i < n; ++i)
            w[i] = ks_d2(u[wrap(i - 1, n)], u[i], u[wrap(i + 1, n)], &k);
        /* sub1: v = u + h * F(u, w) */
#pragma omp parallel for schedule(static)
        for (i = 0; i < n; ++i) {
            int64_t l = wrap(i - 1, n), r = wrap(i + 1, n);
            v[i] = u[i] + k.h * ks_rhs(u[l], u[i], u[r], w[l], w[i], w[r], &k);
        }
        /* sub2: z = D2(v) */
#pragma omp parallel for schedule(static)
        for (i = 0; i < n; ++i)
            z[i] = ks_d2(v[wrap(i - 1, n)], v[i], v[wrap(i + 1, n)], &k);
        /* sub3: u' = u + dt * F(v, z) */
#pragma omp parallel for schedule(static)
        for (i = 0; i < n; ++i) {
            int64_t l = wrap(i - 1, n), r = wrap(i + 1, n);
            un[i] = u[i] + k.dt * ks_rhs(v[l], v[i], v[r], z[l], z[i], z[r], &k);
        }
        memcpy(u, un, (size_t)n * sizeof(double));
    }
    free(un); free(w); free(v); free(z);
    return ORACLE_OK;
}

/* ------------------------------------------------- contraction-on forms */
/*
 * The same schemes with each multiply-add fused, as the paper's Section 4
 * counts the heat sub-timestep ("3 FLOPs": an add and two multiply-adds).
 * fma() is the correctly rounded a*b + c of C99, so these definitions fix
 * every bit too:
 *   heat:  u'[i] = fma(r, fma(-2, u[i], u[i-1] + u[i+1]), u[i])
 *   KS:    D2(a)[i]  = fma(-2, a[i], a[i-1] + a[i+1]) * c2
 *          F(a,b)[i] = -(fma(a[i], D1(a)[i], b[i]) + D2(b)[i])
 *          v = fma(h, F(u,w), u),  u' = fma(dt, F(v,z), u)
 */
static void heat_fma_step_f64(const double *a, double *b, int64_t n, double r)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        double lap = fma(-2.0, a[i], a[wrap(i - 1, n)] + a[wrap(i + 1, n)]);
        b[i] = fma(r, lap, a[i]);
    }
}

static void heat_fma_step_f32(const float *a, float *b, int64_t n, float r)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        float lap = fmaf(-2.0f, a[i], a[wrap(i - 1, n)] + a[wrap(i + 1, n)]);
        b[i] = fmaf(r, lap, a[i]);
    }
}

int oracle_heat_fma_f64(double *u, int64_t n, int64_t nsteps, double r, int nthreads)
{
    double *a, *b, *t;
    int64_t s;
    if (!u || n < 3 || nsteps < 0)
        return ORACLE_EINVAL;
    set_threads(nthreads);
    b = (double *)malloc((size_t)n * sizeof(double));
    if (!b)
        return ORACLE_ENOMEM;
    a = u;
    for (s = 0; s < nsteps; ++s) {
        heat_fma_step_f64(a, b, n, r);
        t = a; a = b; b = t;
    }
    if (a != u) {
        memcpy(u, a, (size_t)n * sizeof(double));
        free(a);
    } else {
        free(b);
    }
    return ORACLE_OK;
}

int oracle_heat_fma_f32(float *u, int64_t n, int64_t nsteps, float r, int nthreads)
{
    float *a, *b, *t;
    int64_t s;
    if (!u || n < 3 || nsteps < 0)
        return ORACLE_EINVAL;
    set_threads(nthreads);
    b = (float *)malloc((size_t)n * sizeof(float));
    if (!b)
        return ORACLE_ENOMEM;
    a = u;
    for (s = 0; s < nsteps; ++s) {
        heat_fma_step_f32(a, b, n, r);
        t = a; a = b; b = t;
    }
    if (a != u) {
        memcpy(u, a, (size_t)n * sizeof(float));
        free(a);
    } else {
        free(b);
    }
    return ORACLE_OK;
}

static double ks_fma_d2(double l, double m, double r, const ks_consts *k)
{
    return fma(-2.0, m, l + r) * k->c2;
}

static double ks_fma_rhs(double al, double am, double ar,
                         double bl, double bm, double br, const ks_consts *k)
{
    double d1a = (ar - al) * k->c1;
    return -(fma(am, d1a, bm) + ks_fma_d2(bl, bm, br, k));
}

int oracle_ks_fma_f64(double *u, int64_t n, int64_t nsteps, double dt, double dx,
                      int nthreads)
{
    ks_consts k;
    double *un, *w, *v, *z;
    int64_t s, i;
    if (!u || n < 3 || nsteps < 0 || !(dx > 0.0))
        return ORACLE_EINVAL;
    set_threads(nthreads);
    k = ks_make(dt, dx);
    un = (double *)malloc((size_t)n * sizeof(double));
    w = (double *)malloc((size_t)n * sizeof(double));
    v = (double *)malloc((size_t)n * sizeof(double));
    z = (double *)malloc((size_t)n * sizeof(double));
    if (!un || !w || !v || !z) {
        free(un); free(w); free(v); free(z);
        return ORACLE_ENOMEM;
    }
    for (s = 0; s < nsteps; ++s) {
#pragma omp parallel for schedule(static)
        for (i = 0; i < n; ++i)
            w[i] = ks_fma_d2(u[wrap(i - 1, n)], u[i], u[wrap(i + 1, n)], &k);
#pragma omp parallel for schedule(static)
        for (i = 0; i < n; ++i) {
            int64_t l = wrap(i - 1, n), r = wrap(i + 1, n);
            v[i] = fma(k.h, ks_fma_rhs(u[l], u[i], u[r], w[l], w[i], w[r], &k), u[i]);
        }
#pragma omp parallel for schedule(static)
        for (i = 0; i < n; ++i)
            z[i] = ks_fma_d2(v[wrap(i - 1, n)], v[i], v[wrap(i + 1, n)], &k);
#pragma omp parallel for schedule(static)
        for (i = 0; i < n; ++i) {
            int64_t l = wrap(i - 1, n), r = wrap(i + 1, n);
            un[i] = fma(k.dt, ks_fma_rhs(v[l], v[i], v[r], z[l], z[i], z[r], &k), u[i]);
        }
        memcpy(u, un, (size_t)n * sizeof(double));
    }
    free(un); free(w); free(v); free(z);
    return ORACLE_OK;
}

/* ------------------------------------------------ single outputs by cone */
/*
 * The value of point i after L sub-timesteps depends only on the inputs
 * within L points of i (paper, Section 2: over n sub-timesteps the domain of
 * dependence grows to the points within n edges).  These functions evaluate
 * a few outputs of a large run one at a time: they apply the same update as
 * above, level by level, on the shrinking window [i-L+l, i+L-l] of the
 * periodic grid.  Used when the full grid is too large for the full run.
 */

int oracle_heat_f64_points(const double *u0, int64_t n, int64_t nsteps, double r,
                           const int64_t *idx, int64_t count, double *out)
{
    int64_t q;
    if (!u0 || !idx || !out || n < 3 || nsteps < 0 || count < 0)
        return ORACLE_EINVAL;
    for (q = 0; q < count; ++q) {
        int64_t width = 2 * nsteps + 1, l, j;
        double *a = (double *)malloc((size_t)width * sizeof(double));
        double *b = (double *)malloc((size_t)width * sizeof(double));
        if (!a || !b) {
            free(a); free(b);
            return ORACLE_ENOMEM;
        }
        for (j = 0; j < width; ++j)
            a[j] = u0[wrap(idx[q] - nsteps + j, n)];
        for (l = 1; l <= nsteps; ++l) {
            int64_t wnew = width - 2 * l;
            for (j = 0; j < wnew; ++j) {
                double lap = (a[j] + a[j + 2]) - 2.0 * a[j + 1];
                b[j] = a[j + 1] + r * lap;
            }
            { double *t = a; a = b; b = t; }
        }
        out[q] = a[0];
        free(a); free(b);
    }
    return ORACLE_OK;
}

int oracle_heat_f32_points(const float *u0, int64_t n, int64_t nsteps, float r,
                           const int64_t *idx, int64_t count, float *out)
{
    int64_t q;
    if (!u0 || !idx || !out || n < 3 || nsteps < 0 || count < 0)
        return ORACLE_EINVAL;
    for (q = 0; q < count; ++q) {
        int64_t width = 2 * nsteps + 1, l, j;
        float *a = (float *)malloc((size_t)width * sizeof(float));
        float *b = (float *)malloc((size_t)width * sizeof(float));
        if (!a || !b) {
            free(a); free(b);
            return ORACLE_ENOMEM;
        }
        for (j = 0; j < width; ++j)
            a[j] = u0[wrap(idx[q] - nsteps + j, n)];
        for (l = 1; l <= nsteps; ++l) {
            int64_t wnew = width - 2 * l;
            for (j = 0; j < wnew; ++j) {
                float lap = (a[j] + a[j + 2]) - 2.0f * a[j + 1];
                b[j] = a[j + 1] + r * lap;
            }
            { float *t = a; a = b; b = t; }
        }
        out[q] = a[0];
        free(a); free(b);
    }
    return ORACLE_OK;
}

int oracle_ks_f64_points(const double *u0, int64_t n, int64_t nsteps, double dt,
                         double dx, const int64_t *idx, int64_t count, double *out)
{
    ks_consts k;
    int64_t q;
    if (!u0 || !idx || !out || n < 3 || nsteps < 0 || count < 0 || !(dx > 0.0))
        return ORACLE_EINVAL;
    k = ks_make(dt, dx);
    for (q = 0; q < count; ++q) {
        /* 4 sub-timesteps per step, each of radius 1 */
        int64_t rad = 4 * nsteps, width = 2 * rad + 1, s, j;
        double *u = (double *)malloc((size_t)width * sizeof(double));
        double *w = (double *)malloc((size_t)width * sizeof(double));
        double *v = (double *)malloc((size_t)width * sizeof(double));
        double *z = (double *)malloc((size_t)width * sizeof(double));
        double *un = (double *)malloc((size_t)width * sizeof(double));
        int64_t lo = 0; /* live window is [lo, width-lo) of the index frame */
        if (!u || !w || !v || !z || !un) {
            free(u); free(w); free(v); free(z); free(un);
            return ORACLE_ENOMEM;
        }
        for (j = 0; j < width; ++j)
            u[j] = u0[wrap(idx[q] - rad + j, n)];
        for (s = 0; s < nsteps; ++s) {
            for (j = lo + 1; j < width - lo - 1; ++j)
                w[j] = ks_d2(u[j - 1], u[j], u[j + 1], &k);
            for (j = lo + 2; j < width - lo - 2; ++j)
                v[j] = u[j] + k.h * ks_rhs(u[j - 1], u[j], u[j + 1],
                                            w[j - 1], w[j], w[j + 1], &k);
            for (j = lo + 3; j < width - lo - 3; ++j)
                z[j] = ks_d2(v[j - 1], v[j], v[j + 1], &k);
            for (j = lo + 4; j < width - lo - 4; ++j)
                un[j] = u[j] + k.dt * ks_rhs(v[j - 1], v[j], v[j + 1],
                                              z[j - 1], z[j], z[j + 1], &k);
            lo += 4;
            for (j = lo; j < width - lo; ++j)
                u[j] = un[j];
        }
        out[q] = u[rad];
        free(u); free(w); free(v); free(z); free(un);
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------- discrete adjoints */
/*
 * Gradient of a scalar objective with respect to the initial field, by the
 * discrete adjoint of the schemes above: the transpose of each sub-timestep's
 * Jacobian, applied in reverse order (in real arithmetic; the operations are
 * evaluated in the order written below).  Objective:
 *
 *   J(u0) = wgt * sum_{j = n0}^{nsteps} sum_i (u_i^j)^2  +  sum_i c_i u_i^nsteps
 *
 * where u^j is the field after j time steps and c = cot_final (NULL: 0).
 * With d2(x)_i = ((x[i-1] + x[i+1]) - 2 x[i]) * c2 and a bar for cotangents:
 *
 *   heat (the step matrix is symmetric):  ub = ub' + r*((ub'[i-1] + ub'[i+1]) - 2 ub')
 *
 *   KS, reverse of sub3 (u' = u + dt*F(v,z)), g = dt*ub':
 *     vb = (c1*((g[i+1]*v[i+1]) - (g[i-1]*v[i-1]))) - (g*((v[i+1] - v[i-1])*c1))
 *     zb = -(g + d2(g))                       ub = ub'
 *   reverse of sub2 (z = D2(v)):  vb = vb + d2(zb)
 *   reverse of sub1 (v = u + h*F(u,w)), q = h*vb:
 *     ub = (ub + vb) + ((c1*((q[i+1]*u[i+1]) - (q[i-1]*u[i-1]))) - (q*((u[i+1] - u[i-1])*c1)))
 *     wb = -(q + d2(q))
 *   reverse of sub0 (w = D2(u)):  ub = ub + d2(wb)
 *
 * u and v are the forward fields of the same step (u^{j-1} and the midpoint
 * value).  After the cotangent of u^j is formed, for j >= n0:
 * ub = ub + (2 wgt) * u^j.  The forward fields are recomputed block by block
 * from stored copies of u every ADJ_BLOCK steps.
 */
#define ADJ_BLOCK 64

static void add_source(double *ub, const double *u, int64_t n, double two_w)
{
    int64_t i;
    for (i = 0; i < n; ++i)
        ub[i] = ub[i] + two_w * u[i];
}

/* forward to the end, keeping u^j for j = 0, B, 2B, ... ; returns u^nsteps in fin */
static int checkpoints(const double *u0, int64_t n, int64_t nsteps, int ks, double r,
                       double dt, double dx, double **ck_out, double *fin)
{
    int64_t nb = nsteps / ADJ_BLOCK + 1, s;
    double *ck = (double *)malloc((size_t)(nb * n) * sizeof(double));
    double *cur = (double *)malloc((size_t)n * sizeof(double));
    if (!ck || !cur) {
        free(ck); free(cur);
        return ORACLE_ENOMEM;
    }
    memcpy(cur, u0, (size_t)n * sizeof(double));
    for (s = 0; s < nsteps; ++s) {
        if (s % ADJ_BLOCK == 0)
            memcpy(ck + (s / ADJ_BLOCK) * n, cur, (size_t)n * sizeof(double));
        if (ks)
            oracle_ks_f64(cur, n, 1, dt, dx, 0);
        else
            oracle_heat_f64(cur, n, 1, r, 0);
    }
    memcpy(fin, cur, (size_t)n * sizeof(double));
    free(cur);
    *ck_out = ck;
    return ORACLE_OK;
}

int oracle_heat_f64_adjoint(const double *u0, int64_t n, int64_t nsteps, double r, int64_t n0,
                            double wgt, const double *cot_final, double *grad, int nthreads)
{
    double *ck = NULL, *lev, *ub, *tmp, *fin;
    const double two_w = 2.0 * wgt;
    int64_t s, i;
    int rc;
    if (!u0 || !grad || n < 3 || nsteps < 0)
        return ORACLE_EINVAL;
    set_threads(nthreads);
    lev = (double *)malloc((size_t)((ADJ_BLOCK + 1) * n) * sizeof(double));
    ub = (double *)malloc((size_t)n * sizeof(double));
    tmp = (double *)malloc((size_t)n * sizeof(double));
    fin = (double *)malloc((size_t)n * sizeof(double));
    if (!lev || !ub || !tmp || !fin) {
        free(lev); free(ub); free(tmp); free(fin);
        return ORACLE_ENOMEM;
    }
    rc = checkpoints(u0, n, nsteps, 0, r, 0.0, 1.0, &ck, fin);
    if (rc) {
        free(lev); free(ub); free(tmp); free(fin);
        return rc;
    }
    for (i = 0; i < n; ++i)
        ub[i] = cot_final ? cot_final[i] : 0.0;
    if (nsteps >= n0)
        add_source(ub, fin, n, two_w);
    for (s = nsteps; s > 0;) {
        const int64_t bs = ((s - 1) / ADJ_BLOCK) * ADJ_BLOCK;
        int64_t j;
        memcpy(lev, ck + (bs / ADJ_BLOCK) * n, (size_t)n * sizeof(double));
        for (j = bs; j < s; ++j)           /* lev[j - bs] = u^j */
            heat_step_f64(lev + (j - bs) * n, lev + (j - bs + 1) * n, n, r);
        for (j = s; j > bs; --j) {         /* ub: cotangent of u^j -> of u^{j-1} */
#pragma omp parallel for schedule(static)
            for (i = 0; i < n; ++i) {
                double l = ub[wrap(i - 1, n)], m = ub[i], rr = ub[wrap(i + 1, n)];
                tmp[i] = m + r * ((l + rr) - 2.0 * m);
            }
            memcpy(ub, tmp, (size_t)n * sizeof(double));
            if (j - 1 >= n0)
                add_source(ub, lev + (j - 1 - bs) * n, n, two_w);
        }
        s = bs;
    }
    memcpy(grad, ub, (size_t)n * sizeof(double));
    free(ck); free(lev); free(ub); free(tmp); free(fin);
    return ORACLE_OK;
}

int oracle_ks_f64_adjoint(const double *u0, int64_t n, int64_t nsteps, double dt, double dx,
                          int64_t n0, double wgt, const double *cot_final, double *grad,
                          int nthreads)
{
    ks_consts k;
    double *ck = NULL, *U, *V, *ub, *vb, *zb, *wb, *tmp, *fin, *w, *z;
    const double two_w = 2.0 * wgt;
    int64_t s, i;
    int rc;
    if (!u0 || !grad || n < 3 || nsteps < 0 || !(dx > 0.0))
        return ORACLE_EINVAL;
    set_threads(nthreads);
    k = ks_make(dt, dx);
    U = (double *)malloc((size_t)((ADJ_BLOCK + 1) * n) * sizeof(double));  /* u^j */
    V = (double *)malloc((size_t)(ADJ_BLOCK * n) * sizeof(double));        /* midpoint v */
    ub = (double *)malloc((size_t)n * sizeof(double));
    vb = (double *)malloc((size_t)n * sizeof(double));
    zb = (double *)malloc((size_t)n * sizeof(double));
    wb = (double *)malloc((size_t)n * sizeof(double));
    tmp = (double *)malloc((size_t)n * sizeof(double));
    fin = (double *)malloc((size_t)n * sizeof(double));
    w = (double *)malloc((size_t)n * sizeof(double));
    z = (double *)malloc((size_t)n * sizeof(double));
    if (!U || !V || !ub || !vb || !zb || !wb || !tmp || !fin || !w || !z) {
        free(U); free(V); free(ub); free(vb); free(zb); free(wb); free(tmp); free(fin);
        free(w); free(z);
        return ORACLE_ENOMEM;
    }
    rc = checkpoints(u0, n, nsteps, 1, 0.0, dt, dx, &ck, fin);
    if (rc) {
        free(U); free(V); free(ub); free(vb); free(zb); free(wb); free(tmp); free(fin);
        free(w); free(z);
        return rc;
    }
    for (i = 0; i < n; ++i)
        ub[i] = cot_final ? cot_final[i] : 0.0;
    if (nsteps >= n0)
        add_source(ub, fin, n, two_w);
    for (s = nsteps; s > 0;) {
        const int64_t bs = ((s - 1) / ADJ_BLOCK) * ADJ_BLOCK;
        int64_t j;
        memcpy(U, ck + (bs / ADJ_BLOCK) * n, (size_t)n * sizeof(double));
        for (j = bs; j < s; ++j) {         /* one RK2 step, keeping u^j and v */
            const double *u = U + (j - bs) * n;
            double *v = V + (j - bs) * n, *un = U + (j - bs + 1) * n;
#pragma omp parallel for schedule(static)
            for (i = 0; i < n; ++i)
                w[i] = ks_d2(u[wrap(i - 1, n)], u[i], u[wrap(i + 1, n)], &k);
#pragma omp parallel for schedule(static)
            for (i = 0; i < n; ++i) {
                int64_t l = wrap(i - 1, n), r = wrap(i + 1, n);
                v[i] = u[i] + k.h * ks_rhs(u[l], u[i], u[r], w[l], w[i], w[r], &k);
            }
#pragma omp parallel for schedule(static)
            for (i = 0; i < n; ++i)
                z[i] = ks_d2(v[wrap(i - 1, n)], v[i], v[wrap(i + 1, n)], &k);
#pragma omp parallel for schedule(static)
            for (i = 0; i < n; ++i) {
                int64_t l = wrap(i - 1, n), r = wrap(i + 1, n);
                un[i] = u[i] + k.dt * ks_rhs(v[l], v[i], v[r], z[l], z[i], z[r], &k);
            }
        }
        for (j = s; j > bs; --j) {         /* ub: cotangent of u^j -> of u^{j-1} */
            const double *u = U + (j - 1 - bs) * n, *v = V + (j - 1 - bs) * n;
            /* reverse of sub3: g = dt*ub */
#pragma omp parallel for schedule(static)
            for (i = 0; i < n; ++i) {
                int64_t l = wrap(i - 1, n), r = wrap(i + 1, n);
                double gl = k.dt * ub[l], gm = k.dt * ub[i], gr = k.dt * ub[r];
                vb[i] = (k.c1 * ((gr * v[r]) - (gl * v[l]))) - (gm * ((v[r] - v[l]) * k.c1));
                zb[i] = -(gm + ks_d2(gl, gm, gr, &k));
            }
            /* reverse of sub2 */
#pragma omp parallel for schedule(static)
            for (i = 0; i < n; ++i)
                tmp[i] = vb[i] + ks_d2(zb[wrap(i - 1, n)], zb[i], zb[wrap(i + 1, n)], &k);
            memcpy(vb, tmp, (size_t)n * sizeof(double));
            /* reverse of sub1: q = h*vb */
#pragma omp parallel for schedule(static)
            for (i = 0; i < n; ++i) {
                int64_t l = wrap(i - 1, n), r = wrap(i + 1, n);
                double ql = k.h * vb[l], qm = k.h * vb[i], qr = k.h * vb[r];
                tmp[i] = (ub[i] + vb[i]) +
                         ((k.c1 * ((qr * u[r]) - (ql * u[l]))) - (qm * ((u[r] - u[l]) * k.c1)));
                wb[i] = -(qm + ks_d2(ql, qm, qr, &k));
            }
            memcpy(ub, tmp, (size_t)n * sizeof(double));
            /* reverse of sub0 */
#pragma omp parallel for schedule(static)
            for (i = 0; i < n; ++i)
                tmp[i] = ub[i] + ks_d2(wb[wrap(i - 1, n)], wb[i], wb[wrap(i + 1, n)], &k);
            memcpy(ub, tmp, (size_t)n * sizeof(double));
            if (j - 1 >= n0)
                add_source(ub, U + (j - 1 - bs) * n, n, two_w);
        }
        s = bs;
    }
    memcpy(grad, ub, (size_t)n * sizeof(double));
    free(ck); free(U); free(V); free(ub); free(vb); free(zb); free(wb); free(tmp); free(fin);
    free(w); free(z);
    return ORACLE_OK;
}

/* ------------------------------------------------- KS tangent-linear model */
/*
 * Forward-mode derivative of the same objective as the adjoints above along
 * given directions: each sub-timestep of the KS scheme and its derivative
 * (the tangent-linear model, no truncation error) are stepped together,
 *   dw = D2(du)
 *   dF(a,b; da,db) = -(((da*D1(a) + a*D1(da)) + db) + D2(db))
 *   dv = du + h*dF(u,w; du,dw),   dz = D2(dv),   du' = du + dt*dF(v,z; dv,dz)
 * with D1, D2 as in the forward scheme, and
 *   dJ[q] = sum_{j=n0}^{nsteps} 2*wgt*<u^j, du^j> + <cot_final, du^nsteps>.
 * The forward values are computed exactly as oracle_ks_f64 computes them.
 * dirs holds ndirs directions of n points each (row q = direction q).  The
 * dot products are summed serially with a compensated (Neumaier) sum, so the
 * result does not depend on the thread count.
 */
typedef struct {
    double s, c;
} nsum;

static void nsum_add(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double nsum_val(const nsum *a) { return a->s + a->c; }

/* acc[q] += scale * <x, d[., q]> for every direction q */
static void tlm_dot(nsum *acc, const double *x, const double *d, int64_t n, int64_t nd,
                    double scale)
{
    int64_t q, i;
    for (q = 0; q < nd; ++q) {
        nsum s = {0.0, 0.0};
        for (i = 0; i < n; ++i)
            nsum_add(&s, x[i] * d[i * nd + q]);
        nsum_add(&acc[q], scale * nsum_val(&s));
    }
}

/* dF(a,b; da,db) at every point and direction (linear in b, so b is not read) */
static void tlm_rhs(const double *a, const double *da, const double *db,
                    int64_t n, int64_t nd, const ks_consts *k, double *out)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        const int64_t l = wrap(i - 1, n), r = wrap(i + 1, n);
        const double d1a = (a[r] - a[l]) * k->c1;
        int64_t q;
        for (q = 0; q < nd; ++q) {
            const double d1da = (da[r * nd + q] - da[l * nd + q]) * k->c1;
            const double d2db = ((db[l * nd + q] + db[r * nd + q]) - 2.0 * db[i * nd + q]) * k->c2;
            out[i * nd + q] = -((((da[i * nd + q] * d1a) + (a[i] * d1da)) + db[i * nd + q]) + d2db);
        }
    }
}

static void tlm_d2(const double *a, int64_t n, int64_t nd, const ks_consts *k, double *out)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        const int64_t l = wrap(i - 1, n), r = wrap(i + 1, n);
        int64_t q;
        for (q = 0; q < nd; ++q)
            out[i * nd + q] = ((a[l * nd + q] + a[r * nd + q]) - 2.0 * a[i * nd + q]) * k->c2;
    }
}

int oracle_ks_f64_tlm(const double *u0, int64_t n, int64_t nsteps, double dt, double dx,
                      int64_t n0, double wgt, const double *cot_final, const double *dirs,
                      int64_t ndirs, double *dJ, int nthreads)
{
    ks_consts k;
    double *u, *w, *v, *z, *un, *du, *dw, *dv, *dz, *df;
    nsum *acc;
    const double two_w = 2.0 * wgt;
    int64_t s, i, q;
    const int64_t nd = ndirs;
    if (!u0 || !dirs || !dJ || n < 3 || nsteps < 0 || ndirs < 1 || !(dx > 0.0))
        return ORACLE_EINVAL;
    set_threads(nthreads);
    k = ks_make(dt, dx);
    u = (double *)malloc((size_t)n * sizeof(double));
    w = (double *)malloc((size_t)n * sizeof(double));
    v = (double *)malloc((size_t)n * sizeof(double));
    z = (double *)malloc((size_t)n * sizeof(double));
    un = (double *)malloc((size_t)n * sizeof(double));
    du = (double *)malloc((size_t)(n * nd) * sizeof(double));
    dw = (double *)malloc((size_t)(n * nd) * sizeof(double));
    dv = (double *)malloc((size_t)(n * nd) * sizeof(double));
    dz = (double *)malloc((size_t)(n * nd) * sizeof(double));
    df = (double *)malloc((size_t)(n * nd) * sizeof(double));
    acc = (nsum *)calloc((size_t)nd, sizeof(nsum));
    if (!u || !w || !v || !z || !un || !du || !dw || !dv || !dz || !df || !acc) {
        free(u); free(w); free(v); free(z); free(un);
        free(du); free(dw); free(dv); free(dz); free(df); free(acc);
        return ORACLE_ENOMEM;
    }
    memcpy(u, u0, (size_t)n * sizeof(double));
    for (i = 0; i < n; ++i)
        for (q = 0; q < nd; ++q)
            du[i * nd + q] = dirs[q * n + i];
    if (n0 <= 0)
        tlm_dot(acc, u, du, n, nd, two_w);
    for (s = 1; s <= nsteps; ++s) {
        /* sub0: w = D2(u), dw = D2(du) */
#pragma omp parallel for schedule(static)
        for (i = 0; i < n; ++i)
            w[i] = ks_d2(u[wrap(i - 1, n)], u[i], u[wrap(i + 1, n)], &k);
        tlm_d2(du, n, nd, &k, dw);
        /* sub1: v = u + h*F(u,w), dv = du + h*dF */
#pragma omp parallel for schedule(static)
        for (i = 0; i < n; ++i) {
            int64_t l = wrap(i - 1, n), r = wrap(i + 1, n);
            v[i] = u[i] + k.h * ks_rhs(u[l], u[i], u[r], w[l], w[i], w[r], &k);
        }
        tlm_rhs(u, du, dw, n, nd, &k, df);
#pragma omp parallel for schedule(static)
        for (i = 0; i < n * nd; ++i)
            dv[i] = du[i] + k.h * df[i];
        /* sub2: z = D2(v), dz = D2(dv) */
#pragma omp parallel for schedule(static)
        for (i = 0; i < n; ++i)
            z[i] = ks_d2(v[wrap(i - 1, n)], v[i], v[wrap(i + 1, n)], &k);
        tlm_d2(dv, n, nd, &k, dz);
        /* sub3: u' = u + dt*F(v,z), du' = du + dt*dF */
#pragma omp parallel for schedule(static)
        for (i = 0; i < n; ++i) {
            int64_t l = wrap(i - 1, n), r = wrap(i + 1, n);
            un[i] = u[i] + k.dt * ks_rhs(v[l], v[i], v[r], z[l], z[i], z[r], &k);
        }
        tlm_rhs(v, dv, dz, n, nd, &k, df);
#pragma omp parallel for schedule(static)
        for (i = 0; i < n * nd; ++i)
            du[i] = du[i] + k.dt * df[i];
        memcpy(u, un, (size_t)n * sizeof(double));
        if (s >= n0)
            tlm_dot(acc, u, du, n, nd, two_w);
    }
    if (cot_final)
        tlm_dot(acc, cot_final, du, n, nd, 1.0);
    for (q = 0; q < nd; ++q)
        dJ[q] = nsum_val(&acc[q]);
    free(u); free(w); free(v); free(z); free(un);
    free(du); free(dw); free(dv); free(dz); free(df); free(acc);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ Euler */

typedef struct {
    double gm1, ch, cf;
} euler_consts;

static double minmod(double a, double b)
{
    if (a > 0.0 && b > 0.0)
        return a < b ? a : b;
    if (a < 0.0 && b < 0.0)
        return a > b ? a : b;
    return 0.0;
}

/* physical flux of the state q into f, and the total enthalpy (E + p)/rho */
static double euler_flux(const double q[3], double gm1, double f[3])
{
    const double u = q[1] / q[0];
    const double p = gm1 * (q[2] - (0.5 * (q[1] * u)));
    f[0] = q[1];
    f[1] = (q[1] * u) + p;
    f[2] = (q[2] + p) * u;
    return (q[2] + p) / q[0];
}

/* interface flux between the reconstructed states qL and qR */
static void euler_face(const double qL[3], const double qR[3], double gm1, double F[3])
{
    double fL[3], fR[3];
    const double HL = euler_flux(qL, gm1, fL);
    const double HR = euler_flux(qR, gm1, fR);
    const double a = sqrt(qL[0]), b = sqrt(qR[0]);
    const double uL = qL[1] / qL[0], uR = qR[1] / qR[0];
    const double ur = ((a * uL) + (b * uR)) / (a + b);
    const double Hr = ((a * HL) + (b * HR)) / (a + b);
    const double cr2 = gm1 * (Hr - (0.5 * (ur * ur)));
    const double lam = fabs(ur) + (cr2 > 0.0 ? sqrt(cr2) : 0.0);
    const double hl = 0.5 * lam;
    for (int c = 0; c < 3; ++c)
        F[c] = (0.5 * (fL[c] + fR[c])) - (hl * (qR[c] - qL[c]));
}

/* the flux difference F[i+1/2] - F[i-1/2] of cell i from the values v and
 * slopes s of cells l = i-1, i, r = i+1 */
static void euler_dflux(const double *v, const double *s, int64_t l, int64_t i, int64_t r,
                        double gm1, double d[3])
{
    double qL[3], qR[3], FL[3], FR[3];
    for (int c = 0; c < 3; ++c) {                 /* face i-1/2 */
        qL[c] = v[3 * l + c] + (0.5 * s[3 * l + c]);
        qR[c] = v[3 * i + c] - (0.5 * s[3 * i + c]);
    }
    euler_face(qL, qR, gm1, FL);
    for (int c = 0; c < 3; ++c) {                 /* face i+1/2 */
        qL[c] = v[3 * i + c] + (0.5 * s[3 * i + c]);
        qR[c] = v[3 * r + c] - (0.5 * s[3 * r + c]);
    }
    euler_face(qL, qR, gm1, FR);
    for (int c = 0; c < 3; ++c)
        d[c] = FR[c] - FL[c];
}

static void euler_slopes(const double *v, double *s, int64_t n)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        const int64_t l = wrap(i - 1, n), r = wrap(i + 1, n);
        for (int c = 0; c < 3; ++c)
            s[3 * i + c] = minmod(v[3 * i + c] - v[3 * l + c], v[3 * r + c] - v[3 * i + c]);
    }
}

/* out = base - coef * (flux difference of (v, s)) */
static void euler_update(const double *base, const double *v, const double *s, double *out,
                         int64_t n, double gm1, double coef)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        double d[3];
        euler_dflux(v, s, wrap(i - 1, n), i, wrap(i + 1, n), gm1, d);
        for (int c = 0; c < 3; ++c)
            out[3 * i + c] = base[3 * i + c] - (coef * d[c]);
    }
}

/* q: n cells of (rho, m, E), advanced in place by nsteps midpoint steps */
int oracle_euler_f64(double *q, int64_t n, int64_t nsteps, double dt, double dx, double gamma,
                     int nthreads)
{
    if (!q || n < 3 || nsteps < 0 || !(dx > 0.0))
        return ORACLE_EINVAL;
    set_threads(nthreads);
    double *s = (double *)malloc((size_t)n * 3 * sizeof(double));
    double *r = (double *)malloc((size_t)n * 3 * sizeof(double));
    double *qn = (double *)malloc((size_t)n * 3 * sizeof(double));
    if (!s || !r || !qn) {
        free(s);
        free(r);
        free(qn);
        return ORACLE_ENOMEM;
    }
    euler_consts k;
    k.gm1 = gamma - 1.0;
    k.ch = (0.5 * dt) / dx;
    k.cf = dt / dx;
    for (int64_t t = 0; t < nsteps; ++t) {
        euler_slopes(q, s, n);                         /* sub0 */
        euler_update(q, q, s, r, n, k.gm1, k.ch);      /* sub1: r = q - ch*dF(q, s) */
        euler_slopes(r, s, n);                         /* sub2 */
        euler_update(q, r, s, qn, n, k.gm1, k.cf);     /* sub3: q' = q - cf*dF(r, s) */
        memcpy(q, qn, (size_t)n * 3 * sizeof(double));
    }
    free(s);
    free(r);
    free(qn);
    return ORACLE_OK;
}
