/*
 * fabm_oracle.c -- reference implementation of the fractional
 * Adams-Bashforth-Moulton predictor-corrector (Diethelm's method) as stated in
 * Section 2 ("Preliminaries") of Baban, Bonchis, Fikl, Rosu, "Parallel
 * simulations for Fractional-Order Systems", arXiv:1611.08678.
 *
 * TEST INFRASTRUCTURE. This file is the oracle the GPU library is checked
 * against. Only the test suite, the package smoke check and the CPU-baseline
 * leg of the benchmark may load it. It shares no code, header, table or
 * constant with the GPU library, and the GPU library never calls it.
 *
 * Everything is written for clarity, not speed:
 *   - weights b_m, a_m, c_m are evaluated straight from their defining
 *     formulas (Section 2, the predictor weights after eq. (2) and the
 *     corrector weights a_n, c_n) in IEEE binary128 (__float128) and rounded
 *     once to double, so the catastrophic cancellation of the power
 *     differences at large m costs nothing;
 *   - history sums run in ascending source index with x87 long double
 *     accumulators, no blocking, no reordering;
 *   - one predictor and one corrector per step (PECE), in the order the
 *     paper gives them.
 *
 * Readings of the paper used here (the paper is garbled or silent on them):
 *   - the predictor weight is b_m = ((m+1)^a - m^a)/Gamma(a+1), with a minus
 *     sign; the printed "+" would not reproduce a constant right-hand side
 *     and gives b_m = 2m+1 at a = 1;
 *   - alpha lies in (0, 2]; the ceil(alpha) initial values y(0) and, for
 *     alpha > 1, y'(0) enter every step through the Taylor polynomial
 *     sum_{k < ceil(alpha)} t^k / k! y^(k)(0) of eq. (1) (y0 + t y'(0)); the
 *     weights keep their formulas, which hold for any alpha > 0;
 *   - history values f_k are evaluated at the corrected y_k; t_n = n*h;
 *   - a non-finite state freezes the trajectory: the step index where it
 *     first appears is returned and every later row is NaN.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#ifdef _OPENMP
#include <omp.h>
#endif
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* System identifiers (own numbering; kept equal to the library's public
 * enumeration by a test, not by a shared header). */
enum {
    ORC_LINEAR = 0,    /* f = A y + b0 + b1 t, theta = (A row-major, b0, b1) */
    ORC_CHEN = 1,      /* (a(y-x), (c-a)x - xz + cy, xy - bz),  theta = (a,b,c) */
    ORC_ROSSLER = 2,   /* (-y-z, x + a y, b + z(x-c)),          theta = (a,b,c) */
    ORC_VDP = 3,       /* (v, mu(1-x^2)v - x),                  theta = (mu)    */
    ORC_FINANCIAL = 4, /* (z + (y-a)x, 1 - b y - x^2, -x - c z), theta = (a,b,c) */
    ORC_HINDMARSH_ROSE = 5, /* (y - a x^3 + b x^2 - z + I, c - d x^2 - y, r (s (x - xr) - z)),
                               theta = (a, b, c, d, r, s, xr, I) */
    ORC_CALLBACK = 99  /* user function pointer (oracle-only test problems) */
};

typedef void (*orc_rhs_cb)(double t, const double *y, double *f, void *user);

typedef struct {
    int system;
    int d;
    const double *theta;
    orc_rhs_cb cb;
    void *user;
} orc_rhs;

/* ------------------------------------------------------------------------ */
/* Right-hand sides f(t, y; theta). Textbook forms of the systems the paper   */
/* names in its introduction; the paper itself prints no equations for them. */
/* ------------------------------------------------------------------------ */
static void rhs_eval(const orc_rhs *r, double t, const double *y, double *f)
{
    const double *p = r->theta;
    switch (r->system) {
    case ORC_LINEAR: {
        int d = r->d;
        const double *A = p, *b0 = p + d * d, *b1 = p + d * d + d;
        for (int i = 0; i < d; ++i) {
            long double s = 0.0L;
            for (int j = 0; j < d; ++j) s += (long double)A[i * d + j] * y[j];
            f[i] = (double)(s + b0[i] + (long double)b1[i] * t);
        }
        break;
    }
    case ORC_CHEN:
        f[0] = p[0] * (y[1] - y[0]);
        f[1] = (p[2] - p[0]) * y[0] - y[0] * y[2] + p[2] * y[1];
        f[2] = y[0] * y[1] - p[1] * y[2];
        break;
    case ORC_ROSSLER:
        f[0] = -y[1] - y[2];
        f[1] = y[0] + p[0] * y[1];
        f[2] = p[1] + y[2] * (y[0] - p[2]);
        break;
    case ORC_VDP:
        f[0] = y[1];
        f[1] = p[0] * (1.0 - y[0] * y[0]) * y[1] - y[0];
        break;
    case ORC_FINANCIAL:
        f[0] = y[2] + (y[1] - p[0]) * y[0];
        f[1] = 1.0 - p[1] * y[1] - y[0] * y[0];
        f[2] = -y[0] - p[2] * y[2];
        break;
    case ORC_HINDMARSH_ROSE: {
        const double x = y[0];
        f[0] = y[1] - p[0] * x * x * x + p[1] * x * x - y[2] + p[7];
        f[1] = p[2] - p[3] * x * x - y[1];
        f[2] = p[4] * (p[5] * (x - p[6]) - y[2]);
        break;
    }
    case ORC_CALLBACK:
        r->cb(t, y, f, r->user);
        break;
    default:
        for (int i = 0; i < r->d; ++i) f[i] = NAN;
    }
}

/* Number of parameters of each system (LINEAR: d*d + 2d). */
int oracle_n_params(int system, int d)
{
    switch (system) {
    case ORC_LINEAR: return d * d + 2 * d;
    case ORC_CHEN: case ORC_ROSSLER: case ORC_FINANCIAL: return 3;
    case ORC_VDP: return 1;
    case ORC_HINDMARSH_ROSE: return 8;
    default: return 0;
    }
}

int oracle_dim(int system, int d_linear)
{
    switch (system) {
    case ORC_LINEAR: return d_linear;
    case ORC_CHEN: case ORC_ROSSLER: case ORC_FINANCIAL: case ORC_HINDMARSH_ROSE: return 3;
    case ORC_VDP: return 2;
    default: return -1;
    }
}

/* Transposed Jacobian products used by the discrete adjoint:
 *   gy[j]     += sum_i fbar[i] * df_i/dy_j
 *   gtheta[q] += sum_i fbar[i] * df_i/dtheta_q
 * Derivatives of the forms in rhs_eval, written out by hand. */
static void rhs_vjp(const orc_rhs *r, double t, const double *y,
                    const long double *fbar, long double *gy, long double *gth)
{
    const double *p = r->theta;
    switch (r->system) {
    case ORC_LINEAR: {
        int d = r->d;
        const double *A = p;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                gy[j] += fbar[i] * A[i * d + j];
                gth[i * d + j] += fbar[i] * y[j];
            }
        for (int i = 0; i < d; ++i) {
            gth[d * d + i] += fbar[i];
            gth[d * d + d + i] += fbar[i] * t;
        }
        break;
    }
    case ORC_CHEN: {
        double a = p[0], b = p[1], c = p[2], x = y[0], yy = y[1], z = y[2];
        gy[0] += fbar[0] * (-a) + fbar[1] * (c - a - z) + fbar[2] * yy;
        gy[1] += fbar[0] * a + fbar[1] * c + fbar[2] * x;
        gy[2] += fbar[1] * (-x) + fbar[2] * (-b);
        gth[0] += fbar[0] * (yy - x) + fbar[1] * (-x);
        gth[1] += fbar[2] * (-z);
        gth[2] += fbar[1] * (x + yy);
        break;
    }
    case ORC_ROSSLER: {
        double a = p[0], c = p[2], x = y[0], yy = y[1], z = y[2];
        gy[0] += fbar[1] + fbar[2] * z;
        gy[1] += -fbar[0] + fbar[1] * a;
        gy[2] += -fbar[0] + fbar[2] * (x - c);
        gth[0] += fbar[1] * yy;
        gth[1] += fbar[2];
        gth[2] += fbar[2] * (-z);
        break;
    }
    case ORC_VDP: {
        double mu = p[0], x = y[0], v = y[1];
        gy[0] += fbar[1] * (-2.0 * mu * x * v - 1.0);
        gy[1] += fbar[0] + fbar[1] * mu * (1.0 - x * x);
        gth[0] += fbar[1] * (1.0 - x * x) * v;
        break;
    }
    case ORC_FINANCIAL: {
        double a = p[0], b = p[1], c = p[2], x = y[0], yy = y[1], z = y[2];
        gy[0] += fbar[0] * (yy - a) + fbar[1] * (-2.0 * x) - fbar[2];
        gy[1] += fbar[0] * x + fbar[1] * (-b);
        gy[2] += fbar[0] + fbar[2] * (-c);
        gth[0] += fbar[0] * (-x);
        gth[1] += fbar[1] * (-yy);
        gth[2] += fbar[2] * (-z);
        break;
    }
    case ORC_HINDMARSH_ROSE: {
        double a = p[0], b = p[1], d = p[3], r = p[4], sg = p[5], xr = p[6];
        double x = y[0], z = y[2];
        gy[0] += fbar[0] * (-3.0 * a * x * x + 2.0 * b * x) + fbar[1] * (-2.0 * d * x) +
                 fbar[2] * (r * sg);
        gy[1] += fbar[0] - fbar[1];
        gy[2] += -fbar[0] - fbar[2] * r;
        gth[0] += fbar[0] * (-x * x * x);
        gth[1] += fbar[0] * (x * x);
        gth[2] += fbar[1];
        gth[3] += fbar[1] * (-x * x);
        gth[4] += fbar[2] * (sg * (x - xr) - z);
        gth[5] += fbar[2] * (r * (x - xr));
        gth[6] += fbar[2] * (-r * sg);
        gth[7] += fbar[0];
        break;
    }
    default:
        break;
    }
}

/* ------------------------------------------------------------------------ */
/* Weights (Section 2): for lag m = 0..n-1                                   */
/*   b_m = ((m+1)^a - m^a) / Gamma(a+1)                                      */
/*   a_m = ((m+2)^(a+1) - 2 (m+1)^(a+1) + m^(a+1)) / Gamma(a+2)              */
/*   c_m = (m^(a+1) - (m-a)(m+1)^a) / Gamma(a+2)                             */
/* evaluated in binary128 from P(j) = j^a and Q(j) = j * P(j) = j^(a+1).     */
/* ------------------------------------------------------------------------ */
void oracle_weights(double alpha, int64_t n, double *b, double *a, double *c)
{
    __float128 al = alpha;
    __float128 g1 = tgammaq(al + 1), g2 = tgammaq(al + 2);
    __float128 P0 = 0, P1 = 1, P2 = powq((__float128)2, al); /* P(m), P(m+1), P(m+2) */
    for (int64_t m = 0; m < n; ++m) {
        __float128 fm = (__float128)m;
        __float128 Q0 = fm * P0, Q1 = (fm + 1) * P1, Q2 = (fm + 2) * P2;
        if (b) b[m] = (double)((P1 - P0) / g1);
        if (a) a[m] = (double)((Q2 - 2 * Q1 + Q0) / g2);
        if (c) c[m] = (double)((Q0 - (fm - al) * P1) / g2);
        P0 = P1;
        P1 = P2;
        P2 = powq(fm + 3, al);
    }
}

/* h^alpha, 1/Gamma(alpha+2) in double, from binary128. */
static void step_scalars(double alpha, double h, double *ha, double *ig2)
{
    *ha = (double)powq((__float128)h, (__float128)alpha);
    *ig2 = (double)(1 / tgammaq((__float128)alpha + 2));
}

static int all_finite(const double *v, int d)
{
    for (int i = 0; i < d; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* Number of initial values eq. (1) needs: ceil(alpha) (1 or 2 here). */
static int n_init_of(double alpha) { return alpha > 1.0 ? 2 : 1; }

/* The Taylor polynomial of the initial values at t (the term that stands
 * before the history integral in eq. (1)): T(t) = y(0) + t y'(0) for
 * 1 < alpha <= 2, y(0) otherwise. init is [ceil(alpha)][d]. */
static void taylor_base(double alpha, double t, const double *init, int d, double *out)
{
    for (int i = 0; i < d; ++i) out[i] = init[i];
    if (n_init_of(alpha) == 2)
        for (int i = 0; i < d; ++i) out[i] += t * init[d + i];
}

/* ------------------------------------------------------------------------ */
/* One trajectory of the PECE scheme, Section 2 (eq. (2) and the corrector). */
/* For n = 0 .. N-1:                                                         */
/*   P    = sum_{k=0}^{n}  b_{n-k} f_k                                       */
/*   C    = c_n f_0 + sum_{k=1}^{n} a_{n-k} f_k                              */
/*   yP   = T(t_{n+1}) + h^a P,       fP = f(t_{n+1}, yP)                    */
/*   y    = T(t_{n+1}) + h^a (C + fP / Gamma(a+2)),  f_{n+1} = f(t_{n+1}, y) */
/* with T the Taylor polynomial of the initial values y0 ([ceil(a)][d]).     */
/* Outputs (row-major [N+1][d]): y (required), yP (row 0 = y0), f.           */
/* b, a, c: caller-provided weight tables of length >= N (may be NULL, then  */
/* they are computed here). Returns 0, or the first step with a non-finite   */
/* state (rows from there on are NaN).                                       */
/* ------------------------------------------------------------------------ */
static int64_t solve_one(const orc_rhs *r, double alpha, double h, int64_t N,
                         const double *y0, const double *wb, const double *wa,
                         const double *wc, double *y, double *yp, double *f)
{
    int d = r->d;
    double ha, ig2;
    step_scalars(alpha, h, &ha, &ig2);
    double *bb = (double *)wb, *aa = (double *)wa, *cc = (double *)wc;
    int own = 0;
    if (!bb || !aa || !cc) {
        own = 1;
        bb = malloc(sizeof(double) * (N + 1));
        aa = malloc(sizeof(double) * (N + 1));
        cc = malloc(sizeof(double) * (N + 1));
        oracle_weights(alpha, N, bb, aa, cc);
    }
    double *F = f ? f : malloc(sizeof(double) * (N + 1) * d);
    double *ypr = malloc(sizeof(double) * d), *fp = malloc(sizeof(double) * d);
    double *T = malloc(sizeof(double) * d);
    long double *SP = malloc(sizeof(long double) * d), *SC = malloc(sizeof(long double) * d);

    memcpy(y, y0, sizeof(double) * d);
    if (yp) memcpy(yp, y0, sizeof(double) * d);
    rhs_eval(r, 0.0, y0, F);
    int64_t status = 0;

    for (int64_t n = 0; n < N; ++n) {
        double *yn1 = y + (n + 1) * d;
        if (status) {
            for (int i = 0; i < d; ++i) {
                yn1[i] = NAN;
                F[(n + 1) * d + i] = NAN;
                if (yp) yp[(n + 1) * d + i] = NAN;
            }
            continue;
        }
        double t1 = (double)(n + 1) * h;
        for (int i = 0; i < d; ++i) {
            SP[i] = 0.0L;
            SC[i] = (long double)cc[n] * F[i];
        }
        for (int64_t k = 0; k <= n; ++k) {
            const double *fk = F + k * d;
            long double wbk = bb[n - k];
            for (int i = 0; i < d; ++i) SP[i] += wbk * fk[i];
            if (k >= 1) {
                long double wak = aa[n - k];
                for (int i = 0; i < d; ++i) SC[i] += wak * fk[i];
            }
        }
        taylor_base(alpha, t1, y0, d, T);
        for (int i = 0; i < d; ++i) ypr[i] = T[i] + ha * (double)SP[i];
        rhs_eval(r, t1, ypr, fp);
        for (int i = 0; i < d; ++i) yn1[i] = T[i] + ha * ((double)SC[i] + fp[i] * ig2);
        rhs_eval(r, t1, yn1, F + (n + 1) * d);
        if (yp) memcpy(yp + (n + 1) * d, ypr, sizeof(double) * d);
        if (!all_finite(yn1, d) || !all_finite(F + (n + 1) * d, d)) {
            status = n + 1;
            for (int i = 0; i < d; ++i) {
                yn1[i] = NAN;
                F[(n + 1) * d + i] = NAN;
            }
        }
    }
    if (own) {
        free(bb);
        free(aa);
        free(cc);
    }
    if (!f) free(F);
    free(ypr);
    free(fp);
    free(T);
    free(SP);
    free(SC);
    return status;
}

int64_t oracle_solve(int system, int d, const double *theta, double alpha, double h,
                     int64_t N, const double *y0, const double *wb, const double *wa,
                     const double *wc, double *y, double *yp, double *f)
{
    orc_rhs r = {system, d, theta, 0, 0};
    return solve_one(&r, alpha, h, N, y0, wb, wa, wc, y, yp, f);
}

/* ------------------------------------------------------------------------ */
/* Non-commensurate orders: eq. (1) with its own order alpha_i for each     */
/* state component. Component i takes the Section 2 scheme with its own     */
/* weights b^(i), a^(i), c^(i), h^alpha_i and Gamma(alpha_i + 2), and its    */
/* own ceil(alpha_i) initial values; the components meet only through f.    */
/* alpha is [d]; init is [n_init][d] (y(0), then y'(0), which components    */
/* with alpha_i > 1 need). Outputs and status as in solve_one.              */
/* ------------------------------------------------------------------------ */
static int64_t solve_orders(const orc_rhs *r, const double *alpha, double h, int64_t N,
                            const double *init, int n_init, double *y, double *yp, double *f)
{
    int d = r->d;
    size_t L = (size_t)N + 1;
    double *W = malloc(sizeof(double) * 3 * L * d); /* component i: b, a, c at 3 i L */
    double *ha = malloc(sizeof(double) * d), *ig2 = malloc(sizeof(double) * d);
    for (int i = 0; i < d; ++i) {
        oracle_weights(alpha[i], N, W + 3 * i * L, W + (3 * i + 1) * L, W + (3 * i + 2) * L);
        step_scalars(alpha[i], h, &ha[i], &ig2[i]);
    }
    double *F = f ? f : malloc(sizeof(double) * L * d);
    double *ypr = malloc(sizeof(double) * d), *fp = malloc(sizeof(double) * d);
    double *T = malloc(sizeof(double) * d);
    long double *SP = malloc(sizeof(long double) * d), *SC = malloc(sizeof(long double) * d);

    memcpy(y, init, sizeof(double) * d);
    if (yp) memcpy(yp, init, sizeof(double) * d);
    rhs_eval(r, 0.0, init, F);
    int64_t status = 0;

    for (int64_t n = 0; n < N; ++n) {
        double *yn1 = y + (n + 1) * d;
        if (status) {
            for (int i = 0; i < d; ++i) {
                yn1[i] = NAN;
                F[(n + 1) * d + i] = NAN;
                if (yp) yp[(n + 1) * d + i] = NAN;
            }
            continue;
        }
        double t1 = (double)(n + 1) * h;
        for (int i = 0; i < d; ++i) {
            const double *bb = W + 3 * i * L, *aa = bb + L, *cc = aa + L;
            SP[i] = 0.0L;
            SC[i] = (long double)cc[n] * F[i];
            for (int64_t k = 0; k <= n; ++k) {
                long double wbk = bb[n - k];
                SP[i] += wbk * F[k * d + i];
                if (k >= 1) {
                    long double wak = aa[n - k];
                    SC[i] += wak * F[k * d + i];
                }
            }
            T[i] = init[i];
            if (n_init_of(alpha[i]) == 2 && n_init == 2) T[i] += t1 * init[d + i];
        }
        for (int i = 0; i < d; ++i) ypr[i] = T[i] + ha[i] * (double)SP[i];
        rhs_eval(r, t1, ypr, fp);
        for (int i = 0; i < d; ++i) yn1[i] = T[i] + ha[i] * ((double)SC[i] + fp[i] * ig2[i]);
        rhs_eval(r, t1, yn1, F + (n + 1) * d);
        if (yp) memcpy(yp + (n + 1) * d, ypr, sizeof(double) * d);
        if (!all_finite(yn1, d) || !all_finite(F + (n + 1) * d, d)) {
            status = n + 1;
            for (int i = 0; i < d; ++i) {
                yn1[i] = NAN;
                F[(n + 1) * d + i] = NAN;
            }
        }
    }
    if (!f) free(F);
    free(W); free(ha); free(ig2); free(ypr); free(fp); free(T); free(SP); free(SC);
    return status;
}

int64_t oracle_solve_orders(int system, int d, const double *theta, const double *alpha,
                            double h, int64_t N, const double *init, int n_init, double *y,
                            double *yp, double *f)
{
    orc_rhs r = {system, d, theta, 0, 0};
    return solve_orders(&r, alpha, h, N, init, n_init, y, yp, f);
}

int64_t oracle_solve_orders_cb(orc_rhs_cb cb, void *user, int d, const double *alpha, double h,
                               int64_t N, const double *init, int n_init, double *y, double *yp,
                               double *f)
{
    orc_rhs r = {ORC_CALLBACK, d, 0, cb, user};
    return solve_orders(&r, alpha, h, N, init, n_init, y, yp, f);
}

/* Batch of non-commensurate trajectories: alpha [batch][d], init
 * [batch][n_init][d], theta [batch][n_theta]; rows at row_off[i]. */
void oracle_solve_orders_batch(int system, int d, int n_theta, int n_init, int64_t batch,
                               const double *alpha, const double *h, const int64_t *N,
                               const double *init, const double *theta, const int64_t *row_off,
                               double *y, int64_t *status)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < batch; ++i) {
        orc_rhs r = {system, d, theta + i * n_theta, 0, 0};
        status[i] = solve_orders(&r, alpha + i * d, h[i], N[i], init + i * n_init * d, n_init,
                                 y + row_off[i] * d, 0, 0);
    }
}

/* One step of the same scheme from a given history (teacher forcing), to
 * check single rows of trajectories too long to re-solve: with f_0..f_{t-1}
 * read from f_hist (row-major [t][d]), the step n = t-1 of solve_one, with
 * the same arithmetic, writes y_t to y_out. mag_out[i] receives
 * h^a (sum_k |b_{n-k} f_k| + |c_n f_0| + sum_{k>=1} |a_{n-k} f_k|), the size
 * of the terms whose rounding the result carries. Weight tables of length
 * >= t are required. */
void oracle_step_from_history(int system, int d, const double *theta, double alpha, double h,
                              int64_t t, const double *y0, const double *f_hist,
                              const double *wb, const double *wa, const double *wc,
                              double *y_out, double *mag_out)
{
    orc_rhs r = {system, d, theta, 0, 0};
    double ha, ig2;
    step_scalars(alpha, h, &ha, &ig2);
    const int64_t n = t - 1;
    long double *SP = malloc(sizeof(long double) * d), *SC = malloc(sizeof(long double) * d);
    long double *MG = malloc(sizeof(long double) * d);
    double *ypr = malloc(sizeof(double) * d), *fp = malloc(sizeof(double) * d);
    double *T = malloc(sizeof(double) * d);
    taylor_base(alpha, (double)t * h, y0, d, T);
    for (int i = 0; i < d; ++i) {
        SP[i] = 0.0L;
        SC[i] = (long double)wc[n] * f_hist[i];
        MG[i] = fabsl(SC[i]);
    }
    for (int64_t k = 0; k <= n; ++k) {
        const double *fk = f_hist + k * d;
        long double wbk = wb[n - k];
        for (int i = 0; i < d; ++i) {
            SP[i] += wbk * fk[i];
            MG[i] += fabsl(wbk * fk[i]);
        }
        if (k >= 1) {
            long double wak = wa[n - k];
            for (int i = 0; i < d; ++i) {
                SC[i] += wak * fk[i];
                MG[i] += fabsl(wak * fk[i]);
            }
        }
    }
    for (int i = 0; i < d; ++i) ypr[i] = T[i] + ha * (double)SP[i];
    rhs_eval(&r, (double)t * h, ypr, fp);
    for (int i = 0; i < d; ++i) {
        y_out[i] = T[i] + ha * ((double)SC[i] + fp[i] * ig2);
        mag_out[i] = ha * (double)MG[i];
    }
    free(T);
    free(SP);
    free(SC);
    free(MG);
    free(ypr);
    free(fp);
}

/* f(t_k, y_k) for rows k = 0..n-1 of y (row-major [n][d]), t_k = k h. */
void oracle_rhs_rows(int system, int d, const double *theta, double h, int64_t n,
                     const double *y, double *f)
{
    orc_rhs r = {system, d, theta, 0, 0};
    for (int64_t k = 0; k < n; ++k) rhs_eval(&r, (double)k * h, y + k * d, f + k * d);
}

/* Same scheme with a caller-supplied right-hand side (oracle-only problems
 * such as manufactured solutions). */
int64_t oracle_solve_cb(orc_rhs_cb cb, void *user, int d, double alpha, double h,
                        int64_t N, const double *y0, double *y, double *yp, double *f)
{
    orc_rhs r = {ORC_CALLBACK, d, 0, cb, user};
    return solve_one(&r, alpha, h, N, y0, 0, 0, 0, y, yp, f);
}

/* A batch of independent trajectories: instance i has its own alpha, h, N,
 * initial values (block i of [batch][n_init][d]; an instance uses the first
 * ceil(alpha_i) rows of its block) and theta (row i of [batch][n_theta]); its rows
 * start at row_off[i] of y (and of yp / f when given). Instances run in
 * parallel over OpenMP threads; each instance's arithmetic is the
 * single-trajectory scheme above, so results do not depend on the thread
 * count. status[i] receives the per-instance status. */
void oracle_solve_batch(int system, int d, int n_theta, int n_init, int64_t batch,
                        const double *alpha, const double *h, const int64_t *N,
                        const double *y0, const double *theta, const int64_t *row_off,
                        double *y, double *yp, double *f, int64_t *status)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < batch; ++i) {
        orc_rhs r = {system, d, theta + i * n_theta, 0, 0};
        int64_t o = row_off[i] * d;
        status[i] = solve_one(&r, alpha[i], h[i], N[i], y0 + i * n_init * d, 0, 0, 0, y + o,
                              yp ? yp + o : 0, f ? f + o : 0);
    }
}

/* ------------------------------------------------------------------------ */
/* History sums alone, for a given history f_0..f_{N-1} (teacher forcing):   */
/*   P_t = sum_{k=0}^{t-1} b_{t-1-k} f_k                                     */
/*   C_t = c_{t-1} f_0 + sum_{k=1}^{t-1} a_{t-1-k} f_k,   t = 1..N           */
/* and the magnitudes sum |w| |f| of both (rounding-error scale).            */
/* Outputs are [N][d] (row t-1 holds target t). OpenMP over targets.         */
/* ------------------------------------------------------------------------ */
void oracle_history_sums(double alpha, int64_t N, int d, const double *f, double *P,
                         double *C, double *Pabs, double *Cabs)
{
    double *bb = malloc(sizeof(double) * (N + 1));
    double *aa = malloc(sizeof(double) * (N + 1));
    double *cc = malloc(sizeof(double) * (N + 1));
    oracle_weights(alpha, N, bb, aa, cc);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 1; t <= N; ++t) {
        for (int i = 0; i < d; ++i) {
            long double sp = 0, sc = (long double)cc[t - 1] * f[i];
            long double ap = 0, ac = fabsl((long double)cc[t - 1] * f[i]);
            for (int64_t k = 0; k < t; ++k) {
                long double fk = f[k * d + i];
                sp += bb[t - 1 - k] * fk;
                ap += fabsl(bb[t - 1 - k] * fk);
                if (k >= 1) {
                    sc += aa[t - 1 - k] * fk;
                    ac += fabsl(aa[t - 1 - k] * fk);
                }
            }
            P[(t - 1) * d + i] = (double)sp;
            C[(t - 1) * d + i] = (double)sc;
            if (Pabs) Pabs[(t - 1) * d + i] = (double)ap;
            if (Cabs) Cabs[(t - 1) * d + i] = (double)ac;
        }
    }
    free(bb);
    free(aa);
    free(cc);
}

/* The same sums for selected targets only: rows[j] (1 <= rows[j] <= N) is a  */
/* target t, and row j of P, C, Pabs, Cabs receives its P_t, C_t and          */
/* magnitude sums. Weights come from oracle_weights, the sums run over the    */
/* whole history in ascending source order exactly as above. OpenMP over the  */
/* selected targets.                                                          */
void oracle_history_sums_rows(double alpha, int64_t N, int d, const double *f, int64_t n_rows,
                              const int64_t *rows, double *P, double *C, double *Pabs,
                              double *Cabs)
{
    double *bb = malloc(sizeof(double) * (N + 1));
    double *aa = malloc(sizeof(double) * (N + 1));
    double *cc = malloc(sizeof(double) * (N + 1));
    oracle_weights(alpha, N, bb, aa, cc);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n_rows; ++j) {
        const int64_t t = rows[j];
        for (int i = 0; i < d; ++i) {
            long double sp = 0, sc = (long double)cc[t - 1] * f[i];
            long double ap = 0, ac = fabsl((long double)cc[t - 1] * f[i]);
            for (int64_t k = 0; k < t; ++k) {
                long double fk = f[k * d + i];
                sp += bb[t - 1 - k] * fk;
                ap += fabsl(bb[t - 1 - k] * fk);
                if (k >= 1) {
                    sc += aa[t - 1 - k] * fk;
                    ac += fabsl(aa[t - 1 - k] * fk);
                }
            }
            P[j * d + i] = (double)sp;
            C[j * d + i] = (double)sc;
            if (Pabs) Pabs[j * d + i] = (double)ap;
            if (Cabs) Cabs[j * d + i] = (double)ac;
        }
    }
    free(bb);
    free(aa);
    free(cc);
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint of the PECE scheme above (reverse mode, derived by hand  */
/* from the forward recursion). For L = sum_{n=0}^{N} <g_n, y_n>:            */
/*   ybar_0 starts at g_0, thetabar at 0, fbar_k at 0. For n = N .. 1:       */
/*     ybar_n   = g_n + J_y(t_n, y_n)^T fbar_n;  thetabar += J_th^T fbar_n   */
/*     ybar_0  += ybar_n;  u = h^a ybar_n                                    */
/*     (for 1 < a <= 2 also y'bar_0 += t_n (ybar_n + ypbar_n): both y_n and  */
/*      yP_n contain t_n y'(0) through the Taylor polynomial)                */
/*     ypbar    = J_y(t_n, yP_n)^T (u / Gamma(a+2)); thetabar likewise       */
/*     ybar_0  += ypbar;   v = h^a ypbar                                     */
/*     fbar_0  += c_{n-1} u;  fbar_k += a_{n-1-k} u  (1 <= k <= n-1)         */
/*     fbar_k  += b_{n-1-k} v                        (0 <= k <= n-1)         */
/*   finally ybar_0 += J_y(0, y0)^T fbar_0 and thetabar += J_th^T fbar_0.    */
/* gy is [N+1][d]; outputs gy0 [ceil(a)][d] (the gradient with respect to   */
/* y(0), then y'(0) for a > 1) and gtheta [n_theta]. Returns the forward     */
/* status (gradients are NaN when the forward blew up).                      */
/* ------------------------------------------------------------------------ */
int64_t oracle_adjoint(int system, int d, const double *theta, double alpha, double h,
                       int64_t N, const double *y0, const double *gy, double *gy0,
                       double *gtheta)
{
    orc_rhs r = {system, d, theta, 0, 0};
    int nth = oracle_n_params(system, d);
    double *bb = malloc(sizeof(double) * (N + 1));
    double *aa = malloc(sizeof(double) * (N + 1));
    double *cc = malloc(sizeof(double) * (N + 1));
    oracle_weights(alpha, N, bb, aa, cc);
    double *Y = malloc(sizeof(double) * (N + 1) * d);
    double *YP = malloc(sizeof(double) * (N + 1) * d);
    int64_t st = solve_one(&r, alpha, h, N, y0, bb, aa, cc, Y, YP, 0);
    double ha, ig2;
    step_scalars(alpha, h, &ha, &ig2);

    long double *fbar = calloc((size_t)(N + 1) * d, sizeof(long double));
    const int ni = n_init_of(alpha);
    long double *gy0l = calloc(d, sizeof(long double));
    long double *gy1l = calloc(d, sizeof(long double));
    long double *gthl = calloc(nth > 0 ? nth : 1, sizeof(long double));
    long double *ybar = calloc(d, sizeof(long double));
    long double *u = calloc(d, sizeof(long double)), *v = calloc(d, sizeof(long double));
    long double *tmp = calloc(d, sizeof(long double));
    long double *ypbar = calloc(d, sizeof(long double));

    for (int i = 0; i < d; ++i) gy0l[i] = gy[i];
    for (int64_t n = N; n >= 1; --n) {
        double tn = (double)n * h;
        for (int i = 0; i < d; ++i) ybar[i] = gy[n * d + i];
        rhs_vjp(&r, tn, Y + n * d, fbar + n * d, ybar, gthl);
        for (int i = 0; i < d; ++i) {
            gy0l[i] += ybar[i];
            u[i] = (long double)ha * ybar[i];
            tmp[i] = u[i] * ig2;
        }
        for (int i = 0; i < d; ++i) ypbar[i] = 0;
        rhs_vjp(&r, tn, YP + n * d, tmp, ypbar, gthl);
        for (int i = 0; i < d; ++i) {
            gy0l[i] += ypbar[i];
            if (ni == 2) gy1l[i] += (long double)tn * (ybar[i] + ypbar[i]);
            v[i] = (long double)ha * ypbar[i];
        }
        for (int i = 0; i < d; ++i) fbar[i] += (long double)cc[n - 1] * u[i];
        for (int64_t k = 1; k <= n - 1; ++k)
            for (int i = 0; i < d; ++i) fbar[k * d + i] += (long double)aa[n - 1 - k] * u[i];
        for (int64_t k = 0; k <= n - 1; ++k)
            for (int i = 0; i < d; ++i) fbar[k * d + i] += (long double)bb[n - 1 - k] * v[i];
    }
    rhs_vjp(&r, 0.0, y0, fbar, gy0l, gthl);
    for (int i = 0; i < d; ++i) gy0[i] = (double)gy0l[i];
    if (ni == 2)
        for (int i = 0; i < d; ++i) gy0[d + i] = (double)gy1l[i];
    for (int q = 0; q < nth; ++q) gtheta[q] = (double)gthl[q];
    if (st) {
        for (int i = 0; i < ni * d; ++i) gy0[i] = NAN;
        for (int q = 0; q < nth; ++q) gtheta[q] = NAN;
    }
    free(bb); free(aa); free(cc); free(Y); free(YP); free(fbar); free(gy0l); free(gy1l);
    free(gthl); free(ybar); free(u); free(v); free(tmp); free(ypbar);
    return st;
}

/* Discrete adjoint of solve_orders (non-commensurate orders), the recursion
 * of oracle_adjoint with component i's own weights, h^alpha_i and
 * Gamma(alpha_i + 2) wherever component i's sums and updates appear. init is
 * [n_init][d]; gy0 receives [n_init][d] (dL/dy(0), then dL/dy'(0) for
 * components with alpha_i > 1, zero for the others). */
int64_t oracle_adjoint_orders(int system, int d, const double *theta, const double *alpha,
                              double h, int64_t N, const double *init, int n_init,
                              const double *gy, double *gy0, double *gtheta)
{
    orc_rhs r = {system, d, theta, 0, 0};
    int nth = oracle_n_params(system, d);
    size_t L = (size_t)N + 1;
    double *W = malloc(sizeof(double) * 3 * L * d);
    double *ha = malloc(sizeof(double) * d), *ig2 = malloc(sizeof(double) * d);
    for (int i = 0; i < d; ++i) {
        oracle_weights(alpha[i], N, W + 3 * i * L, W + (3 * i + 1) * L, W + (3 * i + 2) * L);
        step_scalars(alpha[i], h, &ha[i], &ig2[i]);
    }
    double *Y = malloc(sizeof(double) * L * d);
    double *YP = malloc(sizeof(double) * L * d);
    int64_t st = solve_orders(&r, alpha, h, N, init, n_init, Y, YP, 0);

    long double *fbar = calloc(L * d, sizeof(long double));
    long double *gy0l = calloc(d, sizeof(long double));
    long double *gy1l = calloc(d, sizeof(long double));
    long double *gthl = calloc(nth > 0 ? nth : 1, sizeof(long double));
    long double *ybar = calloc(d, sizeof(long double));
    long double *u = calloc(d, sizeof(long double)), *v = calloc(d, sizeof(long double));
    long double *tmp = calloc(d, sizeof(long double));
    long double *ypbar = calloc(d, sizeof(long double));

    for (int i = 0; i < d; ++i) gy0l[i] = gy[i];
    for (int64_t n = N; n >= 1; --n) {
        double tn = (double)n * h;
        for (int i = 0; i < d; ++i) ybar[i] = gy[n * d + i];
        rhs_vjp(&r, tn, Y + n * d, fbar + n * d, ybar, gthl);
        for (int i = 0; i < d; ++i) {
            gy0l[i] += ybar[i];
            u[i] = (long double)ha[i] * ybar[i];
            tmp[i] = u[i] * ig2[i];
        }
        for (int i = 0; i < d; ++i) ypbar[i] = 0;
        rhs_vjp(&r, tn, YP + n * d, tmp, ypbar, gthl);
        for (int i = 0; i < d; ++i) {
            gy0l[i] += ypbar[i];
            if (n_init_of(alpha[i]) == 2) gy1l[i] += (long double)tn * (ybar[i] + ypbar[i]);
            v[i] = (long double)ha[i] * ypbar[i];
        }
        for (int i = 0; i < d; ++i) {
            const double *bb = W + 3 * i * L, *aa = bb + L, *cc = aa + L;
            fbar[i] += (long double)cc[n - 1] * u[i];
            for (int64_t k = 1; k <= n - 1; ++k) fbar[k * d + i] += (long double)aa[n - 1 - k] * u[i];
            for (int64_t k = 0; k <= n - 1; ++k) fbar[k * d + i] += (long double)bb[n - 1 - k] * v[i];
        }
    }
    rhs_vjp(&r, 0.0, init, fbar, gy0l, gthl);
    for (int i = 0; i < d; ++i) gy0[i] = (double)gy0l[i];
    if (n_init == 2)
        for (int i = 0; i < d; ++i) gy0[d + i] = (double)gy1l[i];
    for (int q = 0; q < nth; ++q) gtheta[q] = (double)gthl[q];
    if (st) {
        for (int i = 0; i < n_init * d; ++i) gy0[i] = NAN;
        for (int q = 0; q < nth; ++q) gtheta[q] = NAN;
    }
    free(W); free(ha); free(ig2); free(Y); free(YP); free(fbar); free(gy0l); free(gy1l);
    free(gthl); free(ybar); free(u); free(v); free(tmp); free(ypbar);
    return st;
}

/* Right-hand side alone, for tests of the system definitions. */
void oracle_rhs(int system, int d, const double *theta, double t, const double *y, double *f)
{
    orc_rhs r = {system, d, theta, 0, 0};
    rhs_eval(&r, t, y, f);
}

/* Threads the OpenMP loops above use (for reporting the cores of a timing). */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
