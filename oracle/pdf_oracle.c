/*
 * Plain CPU FP64 oracle for batched parton-density and alpha_s interpolation.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the package smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library: it recomputes every knot
 * logarithm, slope and weight itself, per query, in the order the method
 * states them.
 *
 * The method (PDFFlow, arXiv:2012.08221, Sec. 2.1) evaluates the LHAPDF
 * interpolation for a batch of independent points: a set of flavours {a} and
 * equal-length arrays x_i, Q_i in, an array of interpolated values out.  The
 * interpolation is log-bicubic: cubic Hermite along ln x, then cubic Hermite
 * along ln Q^2 over the rows so obtained, inside the Q^2 subgrid that holds the
 * point.  alpha_s(Q^2) uses the same 1-D cubic Hermite along ln Q^2 (Sec. 2.1,
 * alpha_s paragraph).  The paper gives no formulas; the readings used are:
 *   - slopes: one-sided divided difference at the ends of an axis (or of a
 *     subgrid), mean of the left and right divided differences inside;
 *   - bins: the largest knot <= the query, compared on raw x and Q^2, clamped so
 *     that a query on the last knot falls in the last interval; a Q^2 equal to a
 *     subgrid threshold belongs to the upper subgrid;
 *   - out of the grid: NaN (mode 0) or the value at the clamped point (mode 1);
 *   - a pid not present in the grid evaluates to 0; 0 and 21 both mean gluon;
 *   - the returned quantity is x f(x, Q^2), as the Sec. 3.2 luminosity divides
 *     the returned values by x1 and x2.
 *
 * Nothing here is blocked, fused or reordered for speed; a thread pool only
 * splits the list of points into contiguous ranges.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* 1-D cubic Hermite                                                          */
/* ------------------------------------------------------------------------ */

/* Cubic Hermite basis on t in [0,1]: h00, h10, h01, h11. */
void ora_hermite_basis(double t, double h[4])
{
    double t2 = t * t, t3 = t2 * t;
    h[0] = 2.0 * t3 - 3.0 * t2 + 1.0;
    h[1] = t3 - 2.0 * t2 + t;
    h[2] = -2.0 * t3 + 3.0 * t2;
    h[3] = t3 - t2;
}

/* Cubic Hermite on [z0, z1] with end values y0, y1 and end slopes m0, m1
 * (slopes are dy/dz), evaluated at z. */
double ora_hermite_eval(double z0, double z1, double y0, double y1,
                        double m0, double m1, double z)
{
    double dz = z1 - z0;
    double t = (z - z0) / dz;
    double h[4];
    ora_hermite_basis(t, h);
    return h[0] * y0 + h[1] * dz * m0 + h[2] * y1 + h[3] * dz * m1;
}

/* Slope at knot j of an axis with n knots z[], values y[j*ys]:
 * one-sided difference at either end, mean of the two neighbouring divided
 * differences inside. */
static double knot_slope(const double *z, const double *y, long ys, int n, int j)
{
    if (j == 0)
        return (y[ys] - y[0]) / (z[1] - z[0]);
    if (j == n - 1)
        return (y[(long)(n - 1) * ys] - y[(long)(n - 2) * ys]) / (z[n - 1] - z[n - 2]);
    double dl = (y[(long)j * ys] - y[(long)(j - 1) * ys]) / (z[j] - z[j - 1]);
    double dr = (y[(long)(j + 1) * ys] - y[(long)j * ys]) / (z[j + 1] - z[j]);
    return 0.5 * (dl + dr);
}

/* 1-D interpolant of the knots (z[j], y[j*ys]), j < n, on interval i, at zq. */
double ora_hermite_1d(const double *z, const double *y, long ys, int n, int i, double zq)
{
    double m0 = knot_slope(z, y, ys, n, i);
    double m1 = knot_slope(z, y, ys, n, i + 1);
    return ora_hermite_eval(z[i], z[i + 1], y[(long)i * ys], y[(long)(i + 1) * ys], m0, m1, zq);
}

/* Largest index j in [0, n) with z[j] <= v (caller guarantees z[0] <= v),
 * clamped to n-2 so that the interval [j, j+1] exists. */
static int bin_of(const double *z, int n, double v)
{
    int j = 0;
    for (int k = 0; k < n; ++k)
        if (z[k] <= v)
            j = k;
    if (j > n - 2)
        j = n - 2;
    return j;
}

/* ------------------------------------------------------------------------ */
/* PDF grid                                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n_flav;
    const int32_t *pids;
    int n_x;
    const double *x;       /* x knots, strictly increasing */
    int n_sub;
    const int32_t *q_off;  /* n_sub+1 offsets into q2[] */
    const double *q2;      /* concatenated subgrid knots */
    const double *xf;      /* [n_flav][n_x][n_q] */
} grid_t;

static int grid_nq(const grid_t *g) { return g->q_off[g->n_sub]; }

/* Row of the grid holding a PDG id: 0 is read as the gluon, 21. */
static int flavour_row(const grid_t *g, int pid)
{
    if (pid == 0)
        pid = 21;
    for (int f = 0; f < g->n_flav; ++f) {
        int p = g->pids[f] == 0 ? 21 : g->pids[f];
        if (p == pid)
            return f;
    }
    return -1;
}

/* Where a point falls: subgrid s, x interval ix, subgrid-local Q^2 interval iq.
 * Returns 0 if in the grid (after clamping in mode 1), -1 if outside in mode 0.
 * *xv and *q2v receive the (possibly clamped) coordinates. */
static int locate(const grid_t *g, double x, double q2, int mode,
                  int *ix, int *s, int *iq, double *xv, double *q2v)
{
    int nq = grid_nq(g);
    double xlo = g->x[0], xhi = g->x[g->n_x - 1];
    double qlo = g->q2[0], qhi = g->q2[nq - 1];
    int inside = (x >= xlo && x <= xhi && q2 >= qlo && q2 <= qhi);
    if (!inside) {
        if (mode == 0 || isnan(x) || isnan(q2))
            return -1;
        x = x < xlo ? xlo : (x > xhi ? xhi : x);
        q2 = q2 < qlo ? qlo : (q2 > qhi ? qhi : q2);
    }
    /* subgrid: largest s whose first knot is <= Q^2; a tie at a threshold
     * therefore selects the upper subgrid. */
    int sub = 0;
    for (int k = 0; k < g->n_sub; ++k)
        if (g->q2[g->q_off[k]] <= q2)
            sub = k;
    *s = sub;
    *ix = bin_of(g->x, g->n_x, x);
    *iq = bin_of(g->q2 + g->q_off[sub], g->q_off[sub + 1] - g->q_off[sub], q2);
    *xv = x;
    *q2v = q2;
    return 0;
}

/* xf of grid row f at one point: Hermite along ln x on each Q^2 row that the
 * Q-direction stencil needs, then Hermite along ln Q^2 over those rows. */
static double interp_2d(const grid_t *g, const double *lnx, const double *lnq2,
                        int f, int ix, int s, int iq, double x, double q2)
{
    int nq = grid_nq(g);
    int off = g->q_off[s];
    int ns = g->q_off[s + 1] - off;
    int k_lo = iq - 1 < 0 ? 0 : iq - 1;
    int k_hi = iq + 2 > ns - 1 ? ns - 1 : iq + 2;
    double u = log(x), w = log(q2);
    double rows[4];
    for (int k = k_lo; k <= k_hi; ++k) {
        const double *col = g->xf + (long)f * g->n_x * nq + off + k;   /* stride nq along x */
        rows[k - k_lo] = ora_hermite_1d(lnx, col, nq, g->n_x, ix, u);
    }
    /* The Q^2 window [k_lo, k_hi] holds exactly the knots whose existence
     * decides the one-sided vs centred slope at iq and iq+1. */
    return ora_hermite_1d(lnq2 + off + k_lo, rows, 1, k_hi - k_lo + 1, iq - k_lo, w);
}

typedef struct {
    const grid_t *g;
    const double *lnx, *lnq2;
    const int32_t *rows;   /* per requested column: grid row or -1 */
    int n_req;
    const double *x, *q2;
    double *out;
    int mode;
    long lo, hi;
} xfx_job;

static void *xfx_worker(void *arg)
{
    xfx_job *j = (xfx_job *)arg;
    for (long p = j->lo; p < j->hi; ++p) {
        int ix, s, iq;
        double xv, q2v;
        int rc = locate(j->g, j->x[p], j->q2[p], j->mode, &ix, &s, &iq, &xv, &q2v);
        for (int r = 0; r < j->n_req; ++r) {
            double v;
            if (j->rows[r] < 0)
                v = 0.0;
            else if (rc != 0)
                v = NAN;
            else
                v = interp_2d(j->g, j->lnx, j->lnq2, j->rows[r], ix, s, iq, xv, q2v);
            j->out[p * j->n_req + r] = v;
        }
    }
    return NULL;
}

typedef void *(*worker_fn)(void *);

static void run_parallel(void *jobs, size_t job_size, long n, int nthreads,
                         void (*set_range)(void *, long, long), worker_fn fn)
{
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    pthread_t th[256];
    long chunk = (n + nthreads - 1) / nthreads;
    int started = 0;
    for (int t = 0; t < nthreads; ++t) {
        long lo = t * chunk, hi = lo + chunk > n ? n : lo + chunk;
        if (lo >= hi && t > 0)
            break;
        void *job = (char *)jobs + (size_t)t * job_size;
        set_range(job, lo < n ? lo : n, hi > lo ? hi : lo);
        if (nthreads == 1) {
            fn(job);
            return;
        }
        pthread_create(&th[t], NULL, fn, job);
        ++started;
    }
    for (int t = 0; t < started; ++t)
        pthread_join(th[t], NULL);
}

static void xfx_set_range(void *job, long lo, long hi)
{
    ((xfx_job *)job)->lo = lo;
    ((xfx_job *)job)->hi = hi;
}

/* Batched xf for the requested pids at points (x[p], q2[p]); out[n][n_req]. */
int ora_xfx(int n_flav, const int32_t *pids, int n_x, const double *x_knots,
            int n_sub, const int32_t *q_off, const double *q2_knots, const double *xf,
            int n_req, const int32_t *req_pids,
            long n, const double *x, const double *q2, double *out,
            int mode, int nthreads)
{
    grid_t g = {n_flav, pids, n_x, x_knots, n_sub, q_off, q2_knots, xf};
    int nq = grid_nq(&g);
    double *lnx = (double *)malloc(sizeof(double) * n_x);
    double *lnq2 = (double *)malloc(sizeof(double) * nq);
    int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (n_req > 0 ? n_req : 1));
    for (int i = 0; i < n_x; ++i)
        lnx[i] = log(x_knots[i]);
    for (int k = 0; k < nq; ++k)
        lnq2[k] = log(q2_knots[k]);
    for (int r = 0; r < n_req; ++r)
        rows[r] = flavour_row(&g, req_pids[r]);
    if (nthreads < 1)
        nthreads = 1;
    xfx_job *jobs = (xfx_job *)calloc((size_t)nthreads, sizeof(xfx_job));
    for (int t = 0; t < nthreads; ++t) {
        xfx_job j = {&g, lnx, lnq2, rows, n_req, x, q2, out, mode, 0, 0};
        jobs[t] = j;
    }
    run_parallel(jobs, sizeof(xfx_job), n, nthreads, xfx_set_range, xfx_worker);
    free(jobs);
    free(rows);
    free(lnq2);
    free(lnx);
    return 0;
}

/* Bins of each point: ix, subgrid s, subgrid-local iq; inside[p] = 1 if the
 * point is in the grid (mode 0 semantics). */
int ora_locate(int n_x, const double *x_knots, int n_sub, const int32_t *q_off,
               const double *q2_knots, long n, const double *x, const double *q2,
               int32_t *ix, int32_t *s, int32_t *iq, int32_t *inside)
{
    grid_t g = {0, NULL, n_x, x_knots, n_sub, q_off, q2_knots, NULL};
    for (long p = 0; p < n; ++p) {
        int a = 0, b = 0, c = 0;
        double xv, q2v;
        int rc = locate(&g, x[p], q2[p], 0, &a, &b, &c, &xv, &q2v);
        ix[p] = a;
        s[p] = b;
        iq[p] = c;
        inside[p] = rc == 0;
    }
    return 0;
}

/* Largest |knot value| over the stencil a point touches for one pid (0 if the
 * pid is absent or the point outside the grid); the error metric's scale. */
int ora_stencil_absmax(int n_flav, const int32_t *pids, int n_x, const double *x_knots,
                       int n_sub, const int32_t *q_off, const double *q2_knots,
                       const double *xf, int n_req, const int32_t *req_pids,
                       long n, const double *x, const double *q2, double *out)
{
    grid_t g = {n_flav, pids, n_x, x_knots, n_sub, q_off, q2_knots, xf};
    int nq = grid_nq(&g);
    for (long p = 0; p < n; ++p) {
        int ix, s, iq;
        double xv, q2v;
        int rc = locate(&g, x[p], q2[p], 0, &ix, &s, &iq, &xv, &q2v);
        for (int r = 0; r < n_req; ++r) {
            int f = flavour_row(&g, req_pids[r]);
            double m = 0.0;
            if (f >= 0 && rc == 0) {
                int off = q_off[s], ns = q_off[s + 1] - off;
                for (int i = ix - 1; i <= ix + 2; ++i) {
                    if (i < 0 || i >= n_x)
                        continue;
                    for (int k = iq - 1; k <= iq + 2; ++k) {
                        if (k < 0 || k >= ns)
                            continue;
                        double v = fabs(xf[((long)f * n_x + i) * nq + off + k]);
                        if (v > m)
                            m = v;
                    }
                }
            }
            out[p * n_req + r] = m;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* alpha_s(Q^2)                                                               */
/* ------------------------------------------------------------------------ */

/* The alpha_s knots split into subgrids wherever a Q^2 knot repeats. */
static double alphas_one(int n, const double *q2k, const double *lnq2k, const double *val,
                         double q2, int mode)
{
    if (!(q2 >= q2k[0] && q2 <= q2k[n - 1])) {
        if (mode == 0 || isnan(q2))
            return NAN;
        q2 = q2 < q2k[0] ? q2k[0] : q2k[n - 1];
    }
    /* subgrid: the last start (index 0 or just after a repeat) whose knot <= q2 */
    int start = 0;
    for (int j = 0; j + 1 < n; ++j)
        if (q2k[j] == q2k[j + 1] && q2k[j + 1] <= q2)
            start = j + 1;
    int end = start;                  /* last index of the subgrid */
    while (end + 1 < n && q2k[end + 1] != q2k[end])
        ++end;
    int ns = end - start + 1;
    int iq = bin_of(q2k + start, ns, q2);
    int k_lo = iq - 1 < 0 ? 0 : iq - 1;
    int k_hi = iq + 2 > ns - 1 ? ns - 1 : iq + 2;
    return ora_hermite_1d(lnq2k + start + k_lo, val + start + k_lo, 1,
                          k_hi - k_lo + 1, iq - k_lo, log(q2));
}

typedef struct {
    int n_as;
    const double *as_q2, *ln_as_q2, *as_val;
    const double *q2;
    double *out;
    int mode;
    long lo, hi;
} as_job;

static void *as_worker(void *arg)
{
    as_job *j = (as_job *)arg;
    for (long p = j->lo; p < j->hi; ++p)
        j->out[p] = alphas_one(j->n_as, j->as_q2, j->ln_as_q2, j->as_val, j->q2[p], j->mode);
    return NULL;
}

static void as_set_range(void *job, long lo, long hi)
{
    ((as_job *)job)->lo = lo;
    ((as_job *)job)->hi = hi;
}

int ora_alphas(int n_as, const double *as_q2, const double *as_val,
               long n, const double *q2, double *out, int mode, int nthreads)
{
    double *ln = (double *)malloc(sizeof(double) * n_as);
    for (int j = 0; j < n_as; ++j)
        ln[j] = log(as_q2[j]);
    if (nthreads < 1)
        nthreads = 1;
    as_job *jobs = (as_job *)calloc((size_t)nthreads, sizeof(as_job));
    for (int t = 0; t < nthreads; ++t) {
        as_job j = {n_as, as_q2, ln, as_val, q2, out, mode, 0, 0};
        jobs[t] = j;
    }
    run_parallel(jobs, sizeof(as_job), n, nthreads, as_set_range, as_worker);
    free(jobs);
    free(ln);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* LO Drell-Yan-like integrand (Sec. 3.1, Eq. 1 luminosity with a unit        */
/* matrix element)                                                            */
/* ------------------------------------------------------------------------ */
/*
 * x_j = exp(ln xmin + u_j * ln(1/xmin)), Q^2 = x1 x2 s clipped to the grid, and
 * I = (ln(1/xmin))^2 alpha_s(Q^2) sum_{q=1..5} xf_q(x1) xf_{-q}(x2).
 * The Jacobian of the log map, x1 x2 (ln(1/xmin))^2, cancels the 1/(x1 x2)
 * that turns xf into f.
 */
typedef struct {
    const grid_t *g;
    const double *lnx, *lnq2;
    int n_as;
    const double *as_q2, *ln_as_q2, *as_val;
    const double *u1, *u2;
    double xmin, s;
    double *out;
    long lo, hi;
} dy_job;

static void *dy_worker(void *arg)
{
    dy_job *j = (dy_job *)arg;
    const grid_t *g = j->g;
    int nq = grid_nq(g);
    double lnmin = log(j->xmin), lnrange = log(1.0 / j->xmin);
    for (long p = j->lo; p < j->hi; ++p) {
        double x1 = exp(lnmin + j->u1[p] * lnrange);
        double x2 = exp(lnmin + j->u2[p] * lnrange);
        double q2 = x1 * x2 * j->s;
        if (q2 < g->q2[0])
            q2 = g->q2[0];
        if (q2 > g->q2[nq - 1])
            q2 = g->q2[nq - 1];
        int ix1, ix2, s1, s2, iq1, iq2;
        double xv1, xv2, qv1, qv2;
        int rc1 = locate(g, x1, q2, 0, &ix1, &s1, &iq1, &xv1, &qv1);
        int rc2 = locate(g, x2, q2, 0, &ix2, &s2, &iq2, &xv2, &qv2);
        double lum = 0.0;
        for (int q = 1; q <= 5; ++q) {
            int fq = flavour_row(g, q), fqb = flavour_row(g, -q);
            double a = (fq < 0) ? 0.0 : (rc1 ? NAN : interp_2d(g, j->lnx, j->lnq2, fq, ix1, s1, iq1, xv1, qv1));
            double b = (fqb < 0) ? 0.0 : (rc2 ? NAN : interp_2d(g, j->lnx, j->lnq2, fqb, ix2, s2, iq2, xv2, qv2));
            lum += a * b;
        }
        double as = alphas_one(j->n_as, j->as_q2, j->ln_as_q2, j->as_val, q2, 0);
        j->out[p] = lnrange * lnrange * as * lum;
    }
    return NULL;
}

static void dy_set_range(void *job, long lo, long hi)
{
    ((dy_job *)job)->lo = lo;
    ((dy_job *)job)->hi = hi;
}

int ora_dy(int n_flav, const int32_t *pids, int n_x, const double *x_knots,
           int n_sub, const int32_t *q_off, const double *q2_knots, const double *xf,
           int n_as, const double *as_q2, const double *as_val,
           long n, const double *u1, const double *u2, double xmin, double s,
           double *out, int nthreads)
{
    grid_t g = {n_flav, pids, n_x, x_knots, n_sub, q_off, q2_knots, xf};
    int nq = grid_nq(&g);
    double *lnx = (double *)malloc(sizeof(double) * n_x);
    double *lnq2 = (double *)malloc(sizeof(double) * nq);
    double *lnas = (double *)malloc(sizeof(double) * n_as);
    for (int i = 0; i < n_x; ++i)
        lnx[i] = log(x_knots[i]);
    for (int k = 0; k < nq; ++k)
        lnq2[k] = log(q2_knots[k]);
    for (int k = 0; k < n_as; ++k)
        lnas[k] = log(as_q2[k]);
    if (nthreads < 1)
        nthreads = 1;
    dy_job *jobs = (dy_job *)calloc((size_t)nthreads, sizeof(dy_job));
    for (int t = 0; t < nthreads; ++t) {
        dy_job j = {&g, lnx, lnq2, n_as, as_q2, lnas, as_val, u1, u2, xmin, s, out, 0, 0};
        jobs[t] = j;
    }
    run_parallel(jobs, sizeof(dy_job), n, nthreads, dy_set_range, dy_worker);
    free(jobs);
    free(lnas);
    free(lnq2);
    free(lnx);
    return 0;
}
