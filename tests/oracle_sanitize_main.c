/*
 * Driver for the sanitizer build of the CPU oracle (test infrastructure).
 *
 * Built together with oracle/pdf_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitizers.py and run as a
 * plain executable.  It calls every exported oracle function on grids and
 * points that reach the edge cases (axes of 2 knots, subgrids of 2, knots,
 * thresholds, the last knot, outside points, NaN, absent pids, several
 * threads, empty batches) and checks a few facts that hold at any size:
 * knot reproduction, a constant grid reproduced, NaN outside in mode 0.
 * Exit status 0 means every call was clean and every check held.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void ora_hermite_basis(double t, double h[4]);
double ora_hermite_eval(double z0, double z1, double y0, double y1, double m0, double m1, double z);
double ora_hermite_1d(const double *z, const double *y, long ys, int n, int i, double zq);
int ora_xfx(int n_flav, const int32_t *pids, int n_x, const double *x_knots, int n_sub,
            const int32_t *q_off, const double *q2_knots, const double *xf, int n_req,
            const int32_t *req_pids, long n, const double *x, const double *q2, double *out,
            int mode, int nthreads);
int ora_locate(int n_x, const double *x_knots, int n_sub, const int32_t *q_off,
               const double *q2_knots, long n, const double *x, const double *q2, int32_t *ix,
               int32_t *s, int32_t *iq, int32_t *inside);
int ora_stencil_absmax(int n_flav, const int32_t *pids, int n_x, const double *x_knots,
                       int n_sub, const int32_t *q_off, const double *q2_knots,
                       const double *xf, int n_req, const int32_t *req_pids, long n,
                       const double *x, const double *q2, double *out);
int ora_alphas(int n_as, const double *as_q2, const double *as_val, long n, const double *q2,
               double *out, int mode, int nthreads);
int ora_dy(int n_flav, const int32_t *pids, int n_x, const double *x_knots, int n_sub,
           const int32_t *q_off, const double *q2_knots, const double *xf, int n_as,
           const double *as_q2, const double *as_val, long n, const double *u1,
           const double *u2, double xmin, double s, double *out, int nthreads);

static int failures = 0;

static void check(int cond, const char *what)
{
    if (!cond) {
        fprintf(stderr, "check failed: %s\n", what);
        ++failures;
    }
}

/* Runs every call on one grid: nx x knots, subgrids given by counts. */
static void exercise(int nx, int n_sub, const int *counts, int nthreads)
{
    int nq = 0;
    int32_t q_off[8];
    q_off[0] = 0;
    for (int s = 0; s < n_sub; ++s) {
        nq += counts[s];
        q_off[s + 1] = nq;
    }
    double *xk = malloc(sizeof(double) * nx);
    double *qk = malloc(sizeof(double) * nq);
    for (int i = 0; i < nx; ++i)
        xk[i] = exp(log(1e-5) * (1.0 - (double)i / (nx - 1)));
    double lo = 1.0;
    for (int s = 0; s < n_sub; ++s) {
        double hi = lo * 5.0;
        for (int k = 0; k < counts[s]; ++k)
            qk[q_off[s] + k] = k == counts[s] - 1 ? hi : lo * pow(5.0, (double)k / (counts[s] - 1));
        lo = hi;
    }
    const int nf = 11;
    int32_t pids[11] = {-5, -4, -3, -2, -1, 21, 1, 2, 3, 4, 5};
    double *xf = malloc(sizeof(double) * nf * nx * nq);
    double *cst = malloc(sizeof(double) * nf * nx * nq);
    for (long e = 0; e < (long)nf * nx * nq; ++e) {
        xf[e] = sin(0.37 * (double)e) + 0.1 * (double)(e % 7);
        cst[e] = 1.25;
    }
    /* points: every knot pair, then outside points, NaN and random points */
    long n = (long)nx * nq + 6 + 200;
    double *x = malloc(sizeof(double) * n), *q2 = malloc(sizeof(double) * n);
    long p = 0;
    for (int i = 0; i < nx; ++i)
        for (int k = 0; k < nq; ++k, ++p) {
            x[p] = xk[i];
            q2[p] = qk[k];
        }
    long nk = p;
    double outside_x[6] = {xk[0] * 0.5, 2.0, 0.1, 0.1, NAN, 0.1};
    double outside_q[6] = {2.0, 2.0, 0.5, qk[nq - 1] * 2.0, 2.0, NAN};
    for (int j = 0; j < 6; ++j, ++p) {
        x[p] = outside_x[j];
        q2[p] = outside_q[j];
    }
    unsigned long long r = 12345;
    for (; p < n; ++p) {
        r = r * 6364136223846793005ull + 1442695040888963407ull;
        double a = (double)(r >> 11) / 9007199254740992.0;
        r = r * 6364136223846793005ull + 1442695040888963407ull;
        double b = (double)(r >> 11) / 9007199254740992.0;
        x[p] = exp(log(xk[0]) * (1.0 - a));
        q2[p] = exp(log(qk[nq - 1]) * b);
    }
    int32_t req[13] = {21, 0, 7, -5, 5, 1, 2, 3, -1, -2, 4, -3, -4};
    int n_req = 13;
    double *out = malloc(sizeof(double) * n * n_req);
    double *out1 = malloc(sizeof(double) * n * n_req);
    for (int mode = 0; mode < 2; ++mode) {
        ora_xfx(nf, pids, nx, xk, n_sub, q_off, qk, xf, n_req, req, n, x, q2, out, mode, nthreads);
        for (long e = 0; e < nk; ++e) {
            int i = (int)(e / nq), k = (int)(e % nq);
            int kk = (k + 1 < nq && qk[k + 1] == qk[k]) ? k + 1 : k;   /* upper copy on a tie */
            check(out[e * n_req + 0] == xf[((long)5 * nx + i) * nq + kk], "knot reproduction");
            check(out[e * n_req + 1] == out[e * n_req + 0], "pid 0 is the gluon");
            check(out[e * n_req + 2] == 0.0, "absent pid gives 0");
        }
        for (int j = 0; j < 6; ++j) {
            double v = out[(nk + j) * n_req];
            if (mode == 0 || j >= 4)
                check(isnan(v), "outside or NaN gives NaN");
            else
                check(isfinite(v), "clamped point is finite");
        }
    }
    ora_xfx(nf, pids, nx, xk, n_sub, q_off, qk, cst, n_req, req, n, x, q2, out1, 1, nthreads);
    for (long e = 0; e < n; ++e) {
        if (e >= nk + 4 && e < nk + 6)
            continue;
        check(fabs(out1[e * n_req] - 1.25) <= 1e-14, "constant grid reproduced");
    }
    int32_t *ix = malloc(sizeof(int32_t) * n), *s = malloc(sizeof(int32_t) * n);
    int32_t *iq = malloc(sizeof(int32_t) * n), *ins = malloc(sizeof(int32_t) * n);
    ora_locate(nx, xk, n_sub, q_off, qk, n, x, q2, ix, s, iq, ins);
    for (long e = 0; e < n; ++e) {
        if (!ins[e])
            continue;
        check(ix[e] >= 0 && ix[e] <= nx - 2, "x bin in range");
        check(s[e] >= 0 && s[e] < n_sub, "subgrid in range");
        check(iq[e] >= 0 && iq[e] <= counts[s[e]] - 2, "Q^2 bin in range");
    }
    ora_stencil_absmax(nf, pids, nx, xk, n_sub, q_off, qk, xf, n_req, req, n, x, q2, out);
    for (long e = 0; e < n; ++e)
        check(out[e * n_req + 2] == 0.0, "absent pid has no stencil");
    /* alpha_s on the Q^2 knots (repeated at thresholds) */
    double *as_val = malloc(sizeof(double) * nq);
    for (int k = 0; k < nq; ++k)
        as_val[k] = 0.3 / (1.0 + 0.1 * log(qk[k]));
    double *as_out = malloc(sizeof(double) * n);
    for (int mode = 0; mode < 2; ++mode)
        ora_alphas(nq, qk, as_val, n, q2, as_out, mode, nthreads);
    ora_alphas(nq, qk, as_val, nq, qk, as_out, 0, nthreads);
    for (int k = 0; k < nq; ++k)
        check(as_out[k] == as_val[k], "alpha_s knot reproduction");
    /* integrand */
    double *u1 = malloc(sizeof(double) * 300), *u2 = malloc(sizeof(double) * 300);
    double *dy_out = malloc(sizeof(double) * 300);
    for (int j = 0; j < 300; ++j) {
        u1[j] = (double)j / 300.0;
        u2[j] = (double)((j * 7) % 300) / 300.0;
    }
    ora_dy(nf, pids, nx, xk, n_sub, q_off, qk, xf, nq, qk, as_val, 300, u1, u2, 1e-5,
           13000.0 * 13000.0, dy_out, nthreads);
    for (int j = 0; j < 300; ++j)
        check(isfinite(dy_out[j]), "integrand finite");
    /* empty batches */
    ora_xfx(nf, pids, nx, xk, n_sub, q_off, qk, xf, n_req, req, 0, x, q2, out, 0, nthreads);
    ora_alphas(nq, qk, as_val, 0, q2, as_out, 0, nthreads);
    free(u1), free(u2), free(dy_out), free(as_out), free(as_val);
    free(ix), free(s), free(iq), free(ins);
    free(out), free(out1), free(x), free(q2), free(xf), free(cst), free(xk), free(qk);
}

int main(void)
{
    double h[4];
    ora_hermite_basis(0.5, h);
    check(h[1] == 0.125, "basis");
    double z[2] = {0.0, 1.0}, y[2] = {1.0, 3.0};
    check(ora_hermite_1d(z, y, 1, 2, 0, 0.5) == 2.0, "two-knot axis is linear");
    check(ora_hermite_eval(0.0, 1.0, 0.0, 1.0, 1.0, 1.0, 0.25) == 0.25, "line");
    const int c1[3] = {4, 6, 40};
    const int c2[1] = {2};
    const int c3[4] = {2, 3, 2, 5};
    exercise(100, 3, c1, 4);
    exercise(2, 1, c2, 1);
    exercise(3, 4, c3, 3);
    if (failures)
        fprintf(stderr, "%d checks failed\n", failures);
    else
        printf("oracle sanitizer run clean\n");
    return failures ? 1 : 0;
}
