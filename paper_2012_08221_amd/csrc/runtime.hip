// Host runtime behind the pdfx C-ABI: descriptor validation, FP64 derivation
// of the per-interval tables, device upload, launch-shape selection and the
// eval entry points.  Kernels live in the other .hip files of this directory.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pdfx.h"
#include "pdfx_internal.h"
#include "runtime_internal.h"
#include "lumi_internal.h"
#include "extrap_internal.h"
#include "bwd_internal.h"
#include "set_internal.h"

using namespace pdfx;

namespace pdfx {

static thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int fail_hip(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? PDFX_ENOMEM : PDFX_EHIP, "%s: %s", what,
                hipGetErrorString(e));
}

void clear_error() { g_last_error.clear(); }

namespace {
__global__ void zero_counter(unsigned long long *c) { *c = 0ull; }
}  // namespace

int error_mode_begin(void *counter, hipStream_t s)
{
    hipLaunchKernelGGL(zero_counter, dim3(1), dim3(1), 0, s, (unsigned long long *)counter);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? PDFX_OK : fail_hip(e, "counter reset launch");
}

int error_mode_end(void *counter, hipStream_t s, int64_t *total)
{
    unsigned long long v = 0;
    hipError_t e = hipMemcpyAsync(&v, counter, sizeof v, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return fail_hip(e, "read the call's domain count");
    *total += (int64_t)v;
    if (v)
        return fail(PDFX_EDOMAIN, "%llu point(s) outside the grid", v);
    return PDFX_OK;
}

DeviceBuf::~DeviceBuf()
{
    if (ptr)
        (void)hipFree(ptr);
}

hipError_t DeviceBuf::upload(const void *src, size_t n)
{
    if (ptr) {
        (void)hipFree(ptr);
        ptr = nullptr;
    }
    bytes = n;
    if (n == 0)
        return hipSuccess;
    hipError_t e = hipMalloc(&ptr, n);
    if (e != hipSuccess) {
        ptr = nullptr;
        return e;
    }
    if (src)
        e = hipMemcpy(ptr, src, n, hipMemcpyHostToDevice);
    else
        e = hipMemset(ptr, 0, n);
    return e;
}

static int canonical_pid(int p) { return p == 0 ? 21 : p; }

// Checks a knot axis made of subgrids [off[s], off[s+1]): raw knots finite and
// > 0, strictly increasing inside a subgrid, neighbouring subgrids sharing the
// boundary knot value.
static int check_axis(const double *z, const int32_t *off, int n_sub, const char *name)
{
    for (int s = 0; s < n_sub; ++s) {
        if (off[s + 1] - off[s] < 2)
            return fail(PDFX_EINVAL, "%s: subgrid %d has fewer than 2 knots", name, s);
        for (int k = off[s]; k < off[s + 1]; ++k) {
            if (!std::isfinite(z[k]) || !(z[k] > 0.0))
                return fail(PDFX_EINVAL, "%s: knot %d is not finite and positive", name, k);
            if (k > off[s] && !(z[k] > z[k - 1]))
                return fail(PDFX_EINVAL, "%s: knots not strictly increasing at %d", name, k);
        }
        if (s + 1 < n_sub && z[off[s + 1] - 1] != z[off[s + 1]])
            return fail(PDFX_EINVAL, "%s: boundary knot of subgrids %d/%d not repeated", name, s,
                        s + 1);
    }
    return PDFX_OK;
}

// Builds the host tables of one axis (see IntervalRec) and uploads them.
int AxisHost::build(const double *z, const int32_t *off, int n_sub)
{
    n = off[n_sub];
    knots.assign(z, z + n);
    std::vector<double> ln(n);
    for (int k = 0; k < n; ++k)
        ln[k] = std::log(z[k]);
    rec64.assign(n > 1 ? n - 1 : 1, IntervalRec<double>{});
    rec32.assign(n > 1 ? n - 1 : 1, IntervalRec<float>{});
    for (int s = 0; s < n_sub; ++s) {
        const int a = off[s], b = off[s + 1];  // knots a..b-1
        for (int i = a; i + 1 < b; ++i) {
            const double d = ln[i + 1] - ln[i];
            const bool left = i > a, right = i + 1 < b - 1;
            const double cl = left ? 0.5 : 0.0, cr = right ? 0.5 : 0.0;
            const double rm = left ? d / (ln[i] - ln[i - 1]) : 0.0;
            const double rp = right ? d / (ln[i + 2] - ln[i + 1]) : 0.0;
            IntervalRec<double> r;
            r.z = ln[i];
            r.inv_d = 1.0 / d;
            r.pl = cl * rm;
            r.ql = 1.0 - cl;
            r.plql = r.pl - r.ql;
            r.pr = cr * rp;
            r.qr = 1.0 - cr;
            r.qrpr = r.qr - r.pr;
            rec64[i] = r;
            IntervalRec<float> f;
            f.z = 0.f;
            f.inv_d = 0.f;
            f.pl = (float)r.pl;
            f.plql = (float)r.plql;
            f.ql = (float)r.ql;
            f.qr = (float)r.qr;
            f.qrpr = (float)r.qrpr;
            f.pr = (float)r.pr;
            rec32[i] = f;
        }
    }
    // Bucket seeds over [ln z_0, ln z_{n-1}]: seed[b] = largest interval whose
    // start is <= the bucket's lower edge (clamped to n-2).
    nbuckets = std::min(4096, std::max(64, 4 * n));
    ln_lo = ln[0];
    const double span = ln[n - 1] - ln[0];
    inv_hb = nbuckets / span;
    seed.assign(nbuckets, 0);
    int i = 0;
    for (int b = 0; b < nbuckets; ++b) {
        const double edge = ln_lo + b * (span / nbuckets);
        while (i + 1 < n - 1 && ln[i + 1] <= edge)
            ++i;
        seed[b] = (uint16_t)i;
    }
    hipError_t e;
    if ((e = d_knots.upload(knots.data(), sizeof(double) * n)) != hipSuccess)
        return fail_hip(e, "upload knots");
    if ((e = d_rec64.upload(rec64.data(), sizeof(rec64[0]) * rec64.size())) != hipSuccess)
        return fail_hip(e, "upload interval table");
    if ((e = d_rec32.upload(rec32.data(), sizeof(rec32[0]) * rec32.size())) != hipSuccess)
        return fail_hip(e, "upload interval table");
    if ((e = d_seed.upload(seed.data(), sizeof(uint16_t) * nbuckets)) != hipSuccess)
        return fail_hip(e, "upload seeds");
    return PDFX_OK;
}

AxisDev AxisHost::dev() const
{
    AxisDev a;
    a.knots = (const double *)d_knots.ptr;
    a.rec64 = (const IntervalRec<double> *)d_rec64.ptr;
    a.rec32 = (const IntervalRec<float> *)d_rec32.ptr;
    a.seed = (const uint16_t *)d_seed.ptr;
    a.n = n;
    a.nbuckets = nbuckets;
    a.lo = knots.front();
    a.hi = knots.back();
    a.ln_lo = ln_lo;
    a.inv_hb = inv_hb;
    return a;
}

int device_cu_count()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 256;
    return cus;
}

int validate_desc(const pdfx_grid_desc *d, bool need_values)
{
    if (!d)
        return fail(PDFX_EINVAL, "descriptor is NULL");
    if (d->n_flav < 1 || d->n_flav > kMaxReq)
        return fail(PDFX_EINVAL, "n_flav = %d outside [1, %d]", d->n_flav, kMaxReq);
    if (!d->pids)
        return fail(PDFX_EINVAL, "pids is NULL");
    for (int f = 0; f < d->n_flav; ++f)
        for (int g = 0; g < f; ++g)
            if (canonical_pid(d->pids[f]) == canonical_pid(d->pids[g]))
                return fail(PDFX_EINVAL, "pid %d appears twice", d->pids[f]);
    if (d->n_x < 2 || d->n_x > 4096)
        return fail(PDFX_EINVAL, "n_x = %d outside [2, 4096]", d->n_x);
    if (!d->x)
        return fail(PDFX_EINVAL, "x knots are NULL");
    if (d->n_sub < 1 || d->n_sub > 16)
        return fail(PDFX_EINVAL, "n_sub = %d outside [1, 16]", d->n_sub);
    if (!d->q_off || !d->q2)
        return fail(PDFX_EINVAL, "q_off or q2 is NULL");
    if (d->q_off[0] != 0)
        return fail(PDFX_EINVAL, "q_off[0] must be 0");
    for (int s = 0; s < d->n_sub; ++s)
        if (d->q_off[s + 1] <= d->q_off[s])
            return fail(PDFX_EINVAL, "q_off not increasing at %d", s);
    if (d->q_off[d->n_sub] > 4096)
        return fail(PDFX_EINVAL, "n_q = %d above 4096", d->q_off[d->n_sub]);
    const int32_t xoff[2] = {0, d->n_x};
    int rc;
    if ((rc = check_axis(d->x, xoff, 1, "x")) != PDFX_OK)
        return rc;
    if ((rc = check_axis(d->q2, d->q_off, d->n_sub, "q2")) != PDFX_OK)
        return rc;
    if (!grid_fits_lds(d->n_x, d->q_off[d->n_sub], d->n_as, true))
        return fail(PDFX_EINVAL, "grid %dx%d too large for one LDS slab", d->n_x,
                    d->q_off[d->n_sub]);
    if (need_values && !d->xf)
        return fail(PDFX_EINVAL, "values (xf) are required here");
    if (d->xf) {
        const size_t nv = (size_t)d->n_flav * d->n_x * d->q_off[d->n_sub];
        for (size_t i = 0; i < nv; ++i)
            if (!std::isfinite(d->xf[i]))
                return fail(PDFX_EINVAL, "value %zu is not finite", i);
    }
    if (d->n_as < 0)
        return fail(PDFX_EINVAL, "n_as < 0");
    if (d->n_as > 0) {
        if (!d->as_q2 || !d->as_val)
            return fail(PDFX_EINVAL, "alpha_s arrays are NULL");
        std::vector<int32_t> off{0};
        for (int j = 0; j + 1 < d->n_as; ++j)
            if (d->as_q2[j] == d->as_q2[j + 1])
                off.push_back(j + 1);
        off.push_back(d->n_as);
        if ((rc = check_axis(d->as_q2, off.data(), (int)off.size() - 1, "alpha_s q2")) != PDFX_OK)
            return rc;
        for (int j = 0; j < d->n_as; ++j)
            if (!std::isfinite(d->as_val[j]))
                return fail(PDFX_EINVAL, "alpha_s value %d is not finite", j);
    }
    return PDFX_OK;
}


}  // namespace pdfx

int pdfx_grid::row_of(int pid) const
{
    const int p = pdfx::canonical_pid(pid);
    for (int f = 0; f < nf; ++f)
        if (pdfx::canonical_pid(pids[f]) == p)
            return f;
    return -1;
}

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------

extern "C" {

const char *pdfx_last_error(void) { return pdfx::g_last_error.c_str(); }

const char *pdfx_version(void) { return "pdfx 0.1 (gfx950)"; }

int pdfx_load_grid(const pdfx_grid_desc *d, pdfx_grid **out)
{
    clear_error();
    if (!out)
        return fail(PDFX_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_desc(d, false);
    if (rc != PDFX_OK)
        return rc;
    pdfx_grid *g = new pdfx_grid();
    rc = grid_init(g, d);
    if (rc != PDFX_OK) {
        delete g;
        return rc;
    }
    *out = g;
    return PDFX_OK;
}

void pdfx_free_grid(pdfx_grid *g) { delete g; }

int pdfx_grid_shape(const pdfx_grid *g, int32_t *n_flav, int32_t *n_x, int32_t *n_q,
                    int32_t *n_sub, int32_t *n_as)
{
    clear_error();
    if (!g)
        return fail(PDFX_EINVAL, "grid is NULL");
    if (n_flav)
        *n_flav = g->nf;
    if (n_x)
        *n_x = g->ax.n;
    if (n_q)
        *n_q = g->aq.n;
    if (n_sub)
        *n_sub = g->n_sub;
    if (n_as)
        *n_as = g->has_alphas ? g->aa.n : 0;
    return PDFX_OK;
}

static int eval_xfx_common(const pdfx_grid *g, const void *xf_dev, int prec, const int32_t *pids,
                           int32_t n_req, const double *x, const double *q, int64_t n_pts,
                           void *out, int domain_mode, void *stream, int q_is_q)
{
    clear_error();
    // EXTRAPOLATE: the forward pass in clamp mode, then the continuation
    // rewrites the rows of the points outside the grid
    const bool extrap = domain_mode == PDFX_DOMAIN_EXTRAPOLATE;
    const bool err = domain_mode == PDFX_DOMAIN_ERROR;
    XfxArgs a;
    int rc = prepare_xfx_args(g, xf_dev, prec, pids, n_req, x, q, n_pts, out,
                              extrap ? PDFX_DOMAIN_CLAMP : err ? PDFX_DOMAIN_NAN : domain_mode,
                              &a);
    if (rc != PDFX_OK || n_pts == 0)
        return rc;
    if (extrap && ((uintptr_t)out & (prec == PDFX_F64 ? 7 : 3)))
        return fail(PDFX_EINVAL, "misaligned device pointer");
    a.q_is_q = q_is_q;
    if (err) {
        a.dom_count = (unsigned long long *)g->call_count.ptr;
        if ((rc = error_mode_begin(g->call_count.ptr, (hipStream_t)stream)) != PDFX_OK)
            return rc;
    }
    rc = run_xfx(g, a, xf_dev, prec, (hipStream_t)stream);
    if (rc == PDFX_OK && err)
        return error_mode_end(g->call_count.ptr, (hipStream_t)stream, &g->host_count);
    if (rc != PDFX_OK || !extrap)
        return rc;
    ExtrapArgs e{};
    e.ax = g->ax.dev();
    e.aq = g->aq.dev();
    e.vals = g->vals[prec].ptr;
    e.nx = g->ax.n;
    e.nq = g->aq.n;
    e.slab_elems = g->slab_elems[prec];
    e.n_req = n_req;
    for (int r = 0; r < n_req; ++r)
        e.row[r] = g->row_of(pids[r]);
    // knot index evaluated at a knot value: the bin rule of the forward
    // kernels (largest i <= n-2 with k[i] <= v; a repeated knot's upper copy),
    // then the knot itself
    auto knot_at = [](const std::vector<double> &k, double v) {
        const int n = (int)k.size();
        int i = 0;
        while (i < n - 2 && k[i + 1] <= v)
            ++i;
        return k[i] == v ? i : i + 1;
    };
    const std::vector<double> &kx = g->ax.knots, &kq = g->aq.knots;
    const int nxk = (int)kx.size(), nqk = (int)kq.size();
    e.kx[0] = knot_at(kx, kx[0]);
    e.kx[1] = knot_at(kx, kx[1]);
    e.kx[2] = knot_at(kx, kx[nxk - 1]);
    e.kx[3] = knot_at(kx, kx[nxk - 2]);
    e.kq[0] = knot_at(kq, kq[0]);
    e.kq[1] = knot_at(kq, kq[1]);
    e.kq[2] = knot_at(kq, kq[nqk - 1]);
    e.kq[3] = knot_at(kq, kq[nqk - 2]);
    e.x = x;
    e.q = q;
    e.q_is_q = q_is_q;
    e.out = out;
    e.n = n_pts;
    hipError_t he;
    if (xf_dev) {
        RepackArgs r{xf_dev, g->scratch_vals[prec].ptr, g->nf, e.nx, e.nq, e.slab_elems};
        if ((he = launch_repack(r, prec == PDFX_F32S, (hipStream_t)stream)) != hipSuccess)
            return fail_hip(he, "repack launch");
        e.vals = g->scratch_vals[prec].ptr;
    }
    if ((he = launch_extrap(e, prec == PDFX_F32S, g->cus, (hipStream_t)stream)) != hipSuccess)
        return fail_hip(he, "continuation launch");
    return PDFX_OK;
}

int pdfx_eval_xfx(const pdfx_grid *g, const void *xf_dev, int prec, const int32_t *pids,
                  int32_t n_req, const double *x, const double *q2, int64_t n_pts, void *out,
                  int domain_mode, void *stream)
{
    return eval_xfx_common(g, xf_dev, prec, pids, n_req, x, q2, n_pts, out, domain_mode, stream,
                           0);
}

int pdfx_eval_xfxQ(const pdfx_grid *g, const void *xf_dev, int prec, const int32_t *pids,
                   int32_t n_req, const double *x, const double *q, int64_t n_pts, void *out,
                   int domain_mode, void *stream)
{
    return eval_xfx_common(g, xf_dev, prec, pids, n_req, x, q, n_pts, out, domain_mode, stream, 1);
}

// alpha_s launch after the argument checks; domain_mode NAN or CLAMP, outside
// points counted in *counter.
static int run_alphas(const pdfx_grid *g, const double *q, int64_t n, void *out, int prec,
                      int domain_mode, hipStream_t stream, int q_is_q, void *counter)
{
    AlphasArgs a;
    a.a = g->aa.dev();
    a.vals = prec == PDFX_F64 ? g->as_vals64.ptr : g->as_vals32.ptr;
    a.q2 = q;
    a.out = out;
    a.n = n;
    a.domain_mode = domain_mode;
    a.q_is_q = q_is_q;
    a.dom_count = (unsigned long long *)counter;
    hipError_t e = launch_alphas(a, prec == PDFX_F32S, stream);
    if (e != hipSuccess)
        return fail_hip(e, "alpha_s launch");
    return PDFX_OK;
}

int pdfx_eval_xfx_alphas(const pdfx_grid *g, const void *xf_dev, int prec, const int32_t *pids,
                         int32_t n_req, const double *x, const double *q2, int64_t n_pts,
                         void *out, void *as_out, int domain_mode, void *stream)
{
    clear_error();
    if (!g)
        return fail(PDFX_EINVAL, "grid is NULL");
    if (!g->has_alphas)
        return fail(PDFX_ENOALPHAS, "grid has no alpha_s knots");
    if (domain_mode != PDFX_DOMAIN_NAN && domain_mode != PDFX_DOMAIN_CLAMP &&
        domain_mode != PDFX_DOMAIN_ERROR)
        return fail(PDFX_EINVAL, "domain mode %d: alpha_s takes NAN, CLAMP or ERROR",
                    domain_mode);
    const bool err = domain_mode == PDFX_DOMAIN_ERROR;
    const int mode = err ? PDFX_DOMAIN_NAN : domain_mode;
    XfxArgs a;
    int rc = prepare_xfx_args(g, xf_dev, prec, pids, n_req, x, q2, n_pts, out, mode, &a);
    if (rc != PDFX_OK || n_pts == 0)
        return rc;
    if (!as_out)
        return fail(PDFX_EINVAL, "as_out is NULL");
    if ((uintptr_t)as_out & (prec == PDFX_F64 ? 7 : 3))
        return fail(PDFX_EINVAL, "misaligned device pointer");
    hipStream_t st = (hipStream_t)stream;
    if (err) {
        a.dom_count = (unsigned long long *)g->call_count.ptr;
        if ((rc = error_mode_begin(g->call_count.ptr, st)) != PDFX_OK)
            return rc;
    }
    bool as_done = false;
    if (g->alphas_on_q) {
        a.as_vals = prec == PDFX_F64 ? g->as_vals64.ptr : g->as_vals32.ptr;   // padded
        a.as_out = as_out;
    }
    rc = run_xfx(g, a, xf_dev, prec, st, &as_done);
    if (rc == PDFX_OK && !as_done)
        rc = run_alphas(g, q2, n_pts, as_out, prec, mode, st, 0, a.dom_count);
    if (rc == PDFX_OK && err)
        return error_mode_end(g->call_count.ptr, st, &g->host_count);
    return rc;
}

static int eval_alphas_common(const pdfx_grid *g, const double *q, int64_t n, void *out,
                              int prec, int domain_mode, void *stream, int q_is_q)
{
    clear_error();
    if (!g)
        return fail(PDFX_EINVAL, "grid is NULL");
    if (!g->has_alphas)
        return fail(PDFX_ENOALPHAS, "grid has no alpha_s knots");
    if (prec != PDFX_F64 && prec != PDFX_F32S)
        return fail(PDFX_EINVAL, "unknown precision %d", prec);
    if (domain_mode != PDFX_DOMAIN_NAN && domain_mode != PDFX_DOMAIN_CLAMP &&
        domain_mode != PDFX_DOMAIN_ERROR)
        return fail(PDFX_EINVAL, "unknown domain mode %d", domain_mode);
    if (n < 0)
        return fail(PDFX_EINVAL, "n < 0");
    if (n == 0)
        return PDFX_OK;
    if (!q || !out)
        return fail(PDFX_EINVAL, "q2 or out is NULL");
    if (((uintptr_t)q & 7) || ((uintptr_t)out & (prec == PDFX_F64 ? 7 : 3)))
        return fail(PDFX_EINVAL, "misaligned device pointer");
    hipStream_t st = (hipStream_t)stream;
    if (domain_mode != PDFX_DOMAIN_ERROR)
        return run_alphas(g, q, n, out, prec, domain_mode, st, q_is_q, g->dom_count.ptr);
    int rc = error_mode_begin(g->call_count.ptr, st);
    if (rc == PDFX_OK)
        rc = run_alphas(g, q, n, out, prec, PDFX_DOMAIN_NAN, st, q_is_q, g->call_count.ptr);
    if (rc == PDFX_OK)
        rc = error_mode_end(g->call_count.ptr, st, &g->host_count);
    return rc;
}

int pdfx_eval_alphas(const pdfx_grid *g, const double *q2, int64_t n, void *out, int prec,
                     int domain_mode, void *stream)
{
    return eval_alphas_common(g, q2, n, out, prec, domain_mode, stream, 0);
}

int pdfx_eval_alphasQ(const pdfx_grid *g, const double *q, int64_t n, void *out, int prec,
                      int domain_mode, void *stream)
{
    return eval_alphas_common(g, q, n, out, prec, domain_mode, stream, 1);
}

int pdfx_domain_errors(const pdfx_grid *g, int64_t *count)
{
    clear_error();
    if (!g || !count)
        return fail(PDFX_EINVAL, "grid or count is NULL");
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess)
        return fail_hip(e, "synchronize");
    unsigned long long v = 0;
    e = hipMemcpy(&v, g->dom_count.ptr, sizeof v, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return fail_hip(e, "read domain counter");
    e = hipMemset(g->dom_count.ptr, 0, sizeof v);
    if (e != hipSuccess)
        return fail_hip(e, "reset domain counter");
    *count = (int64_t)v + g->host_count;
    g->host_count = 0;
    return PDFX_OK;
}

int pdfx_set_domain_errors(const pdfx_set *s, int64_t *count)
{
    clear_error();
    if (!s || !count)
        return fail(PDFX_EINVAL, "set or count is NULL");
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess)
        return fail_hip(e, "synchronize");
    unsigned long long v = 0;
    e = hipMemcpy(&v, s->dom_count.ptr, sizeof v, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return fail_hip(e, "read domain counter");
    e = hipMemset(s->dom_count.ptr, 0, sizeof v);
    if (e != hipSuccess)
        return fail_hip(e, "reset domain counter");
    *count = (int64_t)v + s->host_count;
    s->host_count = 0;
    return PDFX_OK;
}

int pdfx_check_points(const pdfx_grid_desc *d, const double *x, const double *q2, int64_t n,
                      int64_t *n_outside)
{
    clear_error();
    if (n_outside)
        *n_outside = 0;
    int rc = validate_desc(d, false);
    if (rc != PDFX_OK)
        return rc;
    if (n < 0)
        return fail(PDFX_EINVAL, "n < 0");
    if (n > 0 && (!x || !q2))
        return fail(PDFX_EINVAL, "x or q2 is NULL");
    const double xlo = d->x[0], xhi = d->x[d->n_x - 1];
    const double qlo = d->q2[0], qhi = d->q2[d->q_off[d->n_sub] - 1];
    int64_t bad = 0;
    for (int64_t p = 0; p < n; ++p)
        bad += !(x[p] >= xlo && x[p] <= xhi && q2[p] >= qlo && q2[p] <= qhi);   // NaN: outside
    if (n_outside)
        *n_outside = bad;
    if (bad)
        return fail(PDFX_EDOMAIN, "%lld of %lld points outside the grid", (long long)bad,
                    (long long)n);
    return PDFX_OK;
}

int pdfx_get_launch(const pdfx_grid *g, int prec, int32_t *block, int32_t *ppt)
{
    clear_error();
    if (!g || !block || !ppt)
        return fail(PDFX_EINVAL, "NULL argument");
    if (prec != PDFX_F64 && prec != PDFX_F32S)
        return fail(PDFX_EINVAL, "unknown precision %d", prec);
    *block = g->shape[prec].block;
    *ppt = g->shape[prec].ppt;
    return PDFX_OK;
}

int pdfx_set_launch(pdfx_grid *g, int prec, int32_t block, int32_t ppt)
{
    clear_error();
    if (!g)
        return fail(PDFX_EINVAL, "grid is NULL");
    if (prec != PDFX_F64 && prec != PDFX_F32S)
        return fail(PDFX_EINVAL, "unknown precision %d", prec);
    LaunchShape ls{block, ppt};
    if (!launch_shape_supported(ls) && !(prec == PDFX_F32S && launch_shape_f32_only(ls)))
        return fail(PDFX_EINVAL, "launch shape (%d, %d) not compiled for this precision", block,
                    ppt);
    g->shape[prec] = ls;
    g->shape_pinned[prec] = true;
    return PDFX_OK;
}

int pdfx_get_dy_launch(const pdfx_grid *g, int prec, int32_t *block, int32_t *ppt)
{
    clear_error();
    if (!g || !block || !ppt)
        return fail(PDFX_EINVAL, "NULL argument");
    if (prec != PDFX_F64 && prec != PDFX_F32S)
        return fail(PDFX_EINVAL, "unknown precision %d", prec);
    *block = g->dy_shape[prec].block;
    *ppt = g->dy_shape[prec].ppt;
    return PDFX_OK;
}

int pdfx_set_dy_launch(pdfx_grid *g, int prec, int32_t block, int32_t ppt)
{
    clear_error();
    if (!g)
        return fail(PDFX_EINVAL, "grid is NULL");
    if (prec != PDFX_F64 && prec != PDFX_F32S)
        return fail(PDFX_EINVAL, "unknown precision %d", prec);
    LaunchShape ls{block, ppt};
    if (!dy_shape_supported(ls, prec == PDFX_F32S))
        return fail(PDFX_EINVAL, "integrand launch shape (%d, %d) not compiled", block, ppt);
    g->dy_shape[prec] = ls;
    return PDFX_OK;
}

int pdfx_get_lumi_launch(const pdfx_grid *g, int prec, int32_t *block, int32_t *ppt)
{
    clear_error();
    if (!g || !block || !ppt)
        return fail(PDFX_EINVAL, "NULL argument");
    if (prec != PDFX_F64 && prec != PDFX_F32S)
        return fail(PDFX_EINVAL, "unknown precision %d", prec);
    *block = g->lumi_shape[prec].block;
    *ppt = g->lumi_shape[prec].ppt;
    return PDFX_OK;
}

int pdfx_set_lumi_launch(pdfx_grid *g, int prec, int32_t block, int32_t ppt)
{
    clear_error();
    if (!g)
        return fail(PDFX_EINVAL, "grid is NULL");
    if (prec != PDFX_F64 && prec != PDFX_F32S)
        return fail(PDFX_EINVAL, "unknown precision %d", prec);
    LaunchShape ls{block, ppt};
    if (!lumi_shape_supported(ls, prec == PDFX_F32S))
        return fail(PDFX_EINVAL, "luminosity launch shape (%d, %d) not compiled", block, ppt);
    g->lumi_shape[prec] = ls;
    g->lumi_pinned[prec] = true;
    return PDFX_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// grid construction and the forward launch
// ---------------------------------------------------------------------------

namespace pdfx {

int slab_elems_for(int nx, int nq, bool f32)
{
    const int per16 = f32 ? 4 : 2;
    const int e = (nx + 2) * (nq + 2);
    return (e + per16 - 1) / per16 * per16;
}

// LDS layout of the forward kernel: x tables, Q^2 tables, then one or two slabs.
size_t xfx_lds_layout(XfxArgs &a, bool f32, bool *double_buffer)
{
    size_t off = 0;
    auto take = [&](size_t bytes, size_t align) {
        off = (off + align - 1) / align * align;
        const size_t r = off;
        off += bytes;
        return (int)r;
    };
    const AxisDev *axes[2] = {&a.ax, &a.aq};
    AxisLds *lds[2] = {&a.lx, &a.lq};
    for (int i = 0; i < 2; ++i) {
        lds[i]->knots = take((size_t)axes[i]->n * 8, 16);
        lds[i]->seed = take((size_t)axes[i]->nbuckets * 2, 16);
        lds[i]->rec64 = take((size_t)(axes[i]->n - 1) * 64, 64);
        lds[i]->rec32 = take(f32 ? (size_t)(axes[i]->n - 1) * 32 : 0, 64);
    }
    const size_t slab = (size_t)a.slab_elems * (f32 ? 4 : 8);
    a.lds_slab0 = take(slab, 16);
    if (off > kLdsLimit)
        return 0;
    if (off + slab <= kLdsLimit) {
        a.lds_slab1 = take(slab, 16);
        *double_buffer = true;
    } else {
        a.lds_slab1 = a.lds_slab0;
        *double_buffer = false;
    }
    return off;
}

// A grid is usable if the tables plus one slab of the given precision fit LDS.
bool grid_fits_lds(int nx, int nq, int n_as, bool f32)
{
    (void)n_as;
    XfxArgs a{};
    a.ax.n = nx;
    a.ax.nbuckets = std::min(4096, std::max(64, 4 * nx));
    a.aq.n = nq;
    a.aq.nbuckets = std::min(4096, std::max(64, 4 * nq));
    a.slab_elems = slab_elems_for(nx, nq, f32);
    bool db = false;
    return xfx_lds_layout(a, f32, &db) != 0;
}

template <typename V>
static std::vector<V> bordered_slabs(const double *xf, int nf, int nx, int nq, int slab_elems)
{
    std::vector<V> out((size_t)nf * slab_elems, V(0));
    const int nqp = nq + 2;
    for (int f = 0; f < nf; ++f)
        for (int i = 0; i < nx; ++i)
            for (int k = 0; k < nq; ++k)
                out[(size_t)f * slab_elems + (size_t)(i + 1) * nqp + (k + 1)] =
                    (V)xf[((size_t)f * nx + i) * nq + k];
    return out;
}

// Flavour-group node slabs: rows G at a time (G = 16 / sizeof(V)), each knot
// of the (nx+2) x (nq+2) slab with a border one knot wide (or of the nx x nq
// slab without) holding its G row values side by side, one group every
// gstride nodes; rows past nf, the border and the padding are 0.
template <typename V>
static std::vector<V> group_slabs(const double *xf, int nf, int nx, int nq, int n_groups,
                                  int gstride, int border)
{
    constexpr int G = 16 / (int)sizeof(V);
    const int w = nq + 2 * border;          // nodes per slab row
    const size_t nodes = (size_t)gstride;   // group stride in nodes (slab + zero padding)
    std::vector<V> out((size_t)n_groups * nodes * G, V(0));
    for (int f = 0; f < nf; ++f)
        for (int i = 0; i < nx; ++i)
            for (int k = 0; k < nq; ++k)
                out[((size_t)(f / G) * nodes + (size_t)(i + border) * w + (k + border)) * G +
                    f % G] = (V)xf[((size_t)f * nx + i) * nq + k];
    return out;
}

int grid_init(pdfx_grid *g, const pdfx_grid_desc *d)
{
    g->nf = d->n_flav;
    g->n_sub = d->n_sub;
    g->pids.assign(d->pids, d->pids + d->n_flav);
    g->q_off.assign(d->q_off, d->q_off + d->n_sub + 1);
    const int32_t xoff[2] = {0, d->n_x};
    int rc;
    if ((rc = g->ax.build(d->x, xoff, 1)) != PDFX_OK)
        return rc;
    if ((rc = g->aq.build(d->q2, d->q_off, d->n_sub)) != PDFX_OK)
        return rc;
    const int nx = g->ax.n, nq = g->aq.n;
    g->slab_elems[PDFX_F64] = slab_elems_for(nx, nq, false);
    g->slab_elems[PDFX_F32S] = slab_elems_for(nx, nq, true);
    g->n_groups[PDFX_F64] = (g->nf + 1) / 2;
    g->n_groups[PDFX_F32S] = (g->nf + 3) / 4;
    g->gstride = grp_slab_stride(nx, nq);
    g->dma_grid = dma_supported(LaunchShape{512, 1}, nx, nq, g->ax.nbuckets, g->aq.nbuckets);
    const size_t node_bytes = (size_t)g->gstride * 16;
    hipError_t e;
    if (d->xf) {
        auto v64 = bordered_slabs<double>(d->xf, g->nf, nx, nq, g->slab_elems[PDFX_F64]);
        auto v32 = bordered_slabs<float>(d->xf, g->nf, nx, nq, g->slab_elems[PDFX_F32S]);
        if ((e = g->vals[PDFX_F64].upload(v64.data(), v64.size() * sizeof(double))) != hipSuccess)
            return fail_hip(e, "upload values");
        if ((e = g->vals[PDFX_F32S].upload(v32.data(), v32.size() * sizeof(float))) != hipSuccess)
            return fail_hip(e, "upload values");
        auto g64 = group_slabs<double>(d->xf, g->nf, nx, nq, g->n_groups[PDFX_F64], g->gstride, 1);
        auto g32 = group_slabs<float>(d->xf, g->nf, nx, nq, g->n_groups[PDFX_F32S], g->gstride, 1);
        if ((e = g->gvals[PDFX_F64].upload(g64.data(), g64.size() * sizeof(double))) != hipSuccess)
            return fail_hip(e, "upload values");
        if ((e = g->gvals[PDFX_F32S].upload(g32.data(), g32.size() * sizeof(float))) != hipSuccess)
            return fail_hip(e, "upload values");
        if (g->dma_grid) {
            auto d64 = group_slabs<double>(d->xf, g->nf, nx, nq, g->n_groups[PDFX_F64], nx * nq, 0);
            auto d32 = group_slabs<float>(d->xf, g->nf, nx, nq, g->n_groups[PDFX_F32S], nx * nq, 0);
            if ((e = g->dvals[PDFX_F64].upload(d64.data(), d64.size() * sizeof(double))) != hipSuccess)
                return fail_hip(e, "upload values");
            if ((e = g->dvals[PDFX_F32S].upload(d32.data(), d32.size() * sizeof(float))) != hipSuccess)
                return fail_hip(e, "upload values");
        }
        g->has_values = true;
    }
    // repacked copies of caller-provided values land here
    for (int p = 0; p < 2; ++p) {
        const size_t bytes = (size_t)g->nf * g->slab_elems[p] * (p == PDFX_F64 ? 8 : 4);
        if ((e = g->scratch_vals[p].upload(nullptr, bytes)) != hipSuccess)
            return fail_hip(e, "allocate value scratch");
        if ((e = g->scratch_gvals[p].upload(nullptr, g->n_groups[p] * node_bytes)) != hipSuccess)
            return fail_hip(e, "allocate value scratch");
        if (g->dma_grid && (e = g->scratch_dvals[p].upload(nullptr, (size_t)g->n_groups[p] * nx *
                                                                        nq * 16)) != hipSuccess)
            return fail_hip(e, "allocate value scratch");
    }
    if (d->n_as > 0) {
        std::vector<int32_t> off{0};
        for (int j = 0; j + 1 < d->n_as; ++j)
            if (d->as_q2[j] == d->as_q2[j + 1])
                off.push_back(j + 1);
        off.push_back(d->n_as);
        if ((rc = g->aa.build(d->as_q2, off.data(), (int)off.size() - 1)) != PDFX_OK)
            return rc;
        // padded: [0, a_0 .. a_{n-1}, 0], FP32 copy rounded up to an even length
        std::vector<double> p64(d->n_as + 2, 0.0);
        std::vector<float> p32((d->n_as + 3) / 2 * 2, 0.f);
        for (int j = 0; j < d->n_as; ++j) {
            p64[j + 1] = d->as_val[j];
            p32[j + 1] = (float)d->as_val[j];
        }
        if ((e = g->as_vals64.upload(p64.data(), p64.size() * sizeof(double))) != hipSuccess)
            return fail_hip(e, "upload alpha_s");
        if ((e = g->as_vals32.upload(p32.data(), p32.size() * sizeof(float))) != hipSuccess)
            return fail_hip(e, "upload alpha_s");
        g->has_alphas = true;
        const AxisHost &aa = g->aa, &aq = g->aq;
        g->alphas_on_q = aa.n == aq.n && aa.nbuckets == aq.nbuckets && aa.ln_lo == aq.ln_lo &&
                         aa.inv_hb == aq.inv_hb && aa.knots == aq.knots && aa.seed == aq.seed &&
                         aa.rec64.size() == aq.rec64.size() &&
                         std::memcmp(aa.rec64.data(), aq.rec64.data(),
                                     aa.rec64.size() * sizeof(aa.rec64[0])) == 0 &&
                         aa.rec32.size() == aq.rec32.size() &&
                         std::memcmp(aa.rec32.data(), aq.rec32.data(),
                                     aa.rec32.size() * sizeof(aa.rec32[0])) == 0;
    }
    if ((e = g->dom_count.upload(nullptr, sizeof(unsigned long long))) != hipSuccess ||
        (e = g->call_count.upload(nullptr, sizeof(unsigned long long))) != hipSuccess)
        return fail_hip(e, "allocate domain counter");
    g->shape[PDFX_F64] = default_shape(false);
    g->shape[PDFX_F32S] = default_shape(true);
    g->cus = device_cu_count();
    return PDFX_OK;
}

LaunchShape default_shape(bool f32) { return f32 ? LaunchShape{512, 1} : LaunchShape{512, 1}; }

// Request columns -> distinct grid rows (each staged once per tile) plus the
// columns of absent pids.
static void plan_columns(const pdfx_grid *g, const int32_t *pids, int n_req, XfxArgs *a)
{
    int rows[kMaxReq];
    for (int r = 0; r < n_req; ++r)
        rows[r] = g->row_of(pids[r]);
    a->n_u = 0;
    a->n_zero = 0;
    int ncols = 0;
    a->ucol_off[0] = 0;
    bool used[kMaxReq] = {false};
    for (int r = 0; r < n_req; ++r) {
        if (rows[r] < 0) {
            a->zcols[a->n_zero++] = r;
            continue;
        }
        if (used[r])
            continue;
        const int u = a->n_u++;
        a->urow[u] = rows[r];
        for (int c = r; c < n_req; ++c)
            if (rows[c] == rows[r]) {
                a->ucols[ncols++] = c;
                used[c] = true;
            }
        a->ucol_off[u + 1] = ncols;
    }
}

int prepare_xfx_args(const pdfx_grid *g, const void *xf_dev, int prec, const int32_t *pids,
                     int32_t n_req, const double *x, const double *q, int64_t n_pts, void *out,
                     int domain_mode, XfxArgs *a)
{
    if (!g)
        return fail(PDFX_EINVAL, "grid is NULL");
    if (prec != PDFX_F64 && prec != PDFX_F32S)
        return fail(PDFX_EINVAL, "unknown precision %d", prec);
    if (domain_mode == PDFX_DOMAIN_EXTRAPOLATE)
        return fail(PDFX_EINVAL, "domain mode EXTRAPOLATE applies to pdfx_eval_xfx and "
                                 "pdfx_eval_xfxQ only");
    if (domain_mode != PDFX_DOMAIN_NAN && domain_mode != PDFX_DOMAIN_CLAMP)
        return fail(PDFX_EINVAL, "unknown domain mode %d", domain_mode);
    if (n_req < 1 || n_req > PDFX_MAX_REQ)
        return fail(PDFX_EINVAL, "n_req = %d outside [1, %d]", n_req, PDFX_MAX_REQ);
    if (!pids)
        return fail(PDFX_EINVAL, "pids is NULL");
    if (n_pts < 0)
        return fail(PDFX_EINVAL, "n_pts < 0");
    if (!xf_dev && !g->has_values)
        return fail(PDFX_ENOVALUES, "grid has no owned values and xf_dev is NULL");
    if (n_pts > 0 && (!x || !q || !out))
        return fail(PDFX_EINVAL, "x, q2 or out is NULL");
    const uintptr_t a8 = (uintptr_t)7, a4 = (uintptr_t)3;
    if (((uintptr_t)x & a8) || ((uintptr_t)q & a8) || ((uintptr_t)out & a4) ||
        ((uintptr_t)xf_dev & (prec == PDFX_F64 ? a8 : a4)))
        return fail(PDFX_EINVAL, "misaligned device pointer");
    *a = XfxArgs{};
    a->ax = g->ax.dev();
    a->aq = g->aq.dev();
    a->vals = g->vals[prec].ptr;
    a->nf = g->nf;
    a->nx = g->ax.n;
    a->nq = g->aq.n;
    a->slab_elems = g->slab_elems[prec];
    bool db = false;
    if (xfx_lds_layout(*a, prec == PDFX_F32S, &db) == 0)
        return fail(PDFX_EINVAL, "grid too large for an LDS slab in this precision");
    a->n_req = n_req;
    plan_columns(g, pids, n_req, a);
    a->x = x;
    a->q = q;
    a->q_is_q = 0;
    a->out = out;
    a->n = n_pts;
    a->domain_mode = domain_mode;
    a->dom_count = (unsigned long long *)g->dom_count.ptr;
    return PDFX_OK;
}

// Stages of the flavour-group kernel for the request in a: the groups holding
// its distinct rows, in order of first use, and where each result slot goes.
// False if more groups are touched than the kernel holds results for.
static bool plan_stages(XfxArgs &a, int G)
{
    a.n_stage = 0;
    for (int k = 0; k < kGrpMaxSlots; ++k)
        a.slot_u[k] = -1;
    for (int u = 0; u < a.n_u; ++u) {
        const int gi = a.urow[u] / G;
        int st = 0;
        while (st < a.n_stage && a.sgrp[st] != gi)
            ++st;
        if (st == a.n_stage) {
            if ((a.n_stage + 1) * G > kGrpMaxSlots)
                return false;
            a.sgrp[a.n_stage++] = gi;
        }
        a.slot_u[st * G + a.urow[u] % G] = u;
    }
    a.n_dup = 0;
    for (int k = 0; k < kGrpMaxSlots; ++k) {
        const int u = a.slot_u[k];
        a.slot_col[k] = u >= 0 ? a.ucols[a.ucol_off[u]] : -1;
        for (int c = u >= 0 ? a.ucol_off[u] + 1 : 0; u >= 0 && c < a.ucol_off[u + 1]; ++c) {
            a.dup_src[a.n_dup] = a.slot_col[k];
            a.dup_dst[a.n_dup++] = a.ucols[c];
        }
    }
    return true;
}

// Repack caller values (if any) and launch the forward kernel.  Shapes with
// results held in registers (ppt > 0) use the flavour-group kernels when the
// request's groups fit them: the double-buffered one when the grid fits its
// LDS and `out` is 16-byte aligned, else the single-buffer one when its slab
// fits; everything else uses the per-flavour kernel.
int run_xfx(const pdfx_grid *g, XfxArgs &a, const void *xf_dev, int prec, hipStream_t s,
            bool *as_done)
{
    hipError_t e;
    const bool f32 = prec == PDFX_F32S;
    if (as_done)
        *as_done = false;
    LaunchShape ls = g->shape[prec];
    if (!g->shape_pinned[prec] && ls.ppt > 1) {
        // a small call: (512, 1) gives twice or more the workgroups
        const int64_t tile = (int64_t)ls.block * ls.ppt;
        if ((a.n + tile - 1) / tile < g->cus / 2)
            ls = LaunchShape{512, 1};
    }
    const bool staged = ls.ppt > 0 && plan_stages(a, f32 ? 4 : 2);
    if (staged && g->dma_grid && (uintptr_t)a.out % 16 == 0 &&
        dma_supported(ls, a.nx, a.nq, a.ax.nbuckets, a.aq.nbuckets, f32)) {
        a.gvals = g->dvals[prec].ptr;
        a.gstride = a.nx * a.nq;
        if (xf_dev) {
            if ((e = launch_grp_repack(xf_dev, g->scratch_dvals[prec].ptr, g->nf, a.nx, a.nq,
                                       g->n_groups[prec], a.gstride, false, f32, s)) != hipSuccess)
                return fail_hip(e, "repack launch");
            a.gvals = g->scratch_dvals[prec].ptr;
        }
        if (a.as_out && !dma_alphas_fit(a.nx, a.nq, f32)) {
            a.as_out = nullptr;
            a.as_vals = nullptr;
        }
        const int maxb = g->max_blocks(prec, a, 2, ls);
        e = f32 ? launch_xfx_dma_f32s(a, ls, maxb, s) : launch_xfx_dma_f64(a, ls, maxb, s);
        if (e != hipSuccess)
            return fail_hip(e, "xfx launch");
        if (as_done)
            *as_done = a.as_out != nullptr;
        return PDFX_OK;
    }
    a.as_out = nullptr;
    a.as_vals = nullptr;
    if (launch_shape_f32_only(ls))
        ls = LaunchShape{512, 2};   // the other kernels' nearest shape
    bool grouped = staged && grp_shape_supported(ls, a.nx, a.nq);
    if (grouped) {
        XfxArgs probe = a;
        grouped = grp_lds_layout(probe, f32, ls.block) != 0;
    }
    if (grouped) {
        a.gvals = g->gvals[prec].ptr;
        a.gstride = g->gstride;
        if (xf_dev) {
            if ((e = launch_grp_repack(xf_dev, g->scratch_gvals[prec].ptr, g->nf, a.nx, a.nq,
                                       g->n_groups[prec], g->gstride, true, f32, s)) != hipSuccess)
                return fail_hip(e, "repack launch");
            a.gvals = g->scratch_gvals[prec].ptr;
        }
        const int maxb = g->max_blocks(prec, a, 1, ls);
        e = f32 ? launch_xfx_grp_f32s(a, ls, maxb, s) : launch_xfx_grp_f64(a, ls, maxb, s);
        if (e != hipSuccess)
            return fail_hip(e, "xfx launch");
        return PDFX_OK;
    }
    if (xf_dev) {
        RepackArgs r{xf_dev, g->scratch_vals[prec].ptr, g->nf, a.nx, a.nq, a.slab_elems};
        if ((e = launch_repack(r, f32, s)) != hipSuccess)
            return fail_hip(e, "repack launch");
        a.vals = g->scratch_vals[prec].ptr;
    }
    const int maxb = g->max_blocks(prec, a, 0, ls);
    e = f32 ? launch_xfx_f32s(a, ls, maxb, s) : launch_xfx_f64(a, ls, maxb, s);
    if (e != hipSuccess)
        return fail_hip(e, "xfx launch");
    return PDFX_OK;
}

}  // namespace pdfx

// Resident workgroups of launch shape ls over the whole device (cached per
// precision, kernel and shape; the persistent kernels never launch more).
int pdfx_grid::max_blocks(int prec, const pdfx::XfxArgs &a, int kernel,
                          pdfx::LaunchShape ls) const
{
    for (int c = 0; c < 2; ++c)
        if (occ_shape[prec][kernel][c].block == ls.block &&
            occ_shape[prec][kernel][c].ppt == ls.ppt && occ_blocks[prec][kernel][c] > 0)
            return occ_blocks[prec][kernel][c];
    int per_cu = 0;
    hipError_t e;
    if (kernel == 2)
        e = prec == PDFX_F32S ? pdfx::xfx_dma_occupancy_f32s(ls, &per_cu)
                              : pdfx::xfx_dma_occupancy_f64(ls, &per_cu);
    else if (kernel == 1)
        e = prec == PDFX_F32S ? pdfx::xfx_grp_occupancy_f32s(a, ls, &per_cu)
                              : pdfx::xfx_grp_occupancy_f64(a, ls, &per_cu);
    else
        e = prec == PDFX_F32S ? pdfx::xfx_occupancy_f32s(a, ls, &per_cu)
                              : pdfx::xfx_occupancy_f64(a, ls, &per_cu);
    if (e != hipSuccess || per_cu < 1)
        per_cu = 1;
    const int c = occ_next[prec][kernel];
    occ_next[prec][kernel] = c ^ 1;
    occ_shape[prec][kernel][c] = ls;
    occ_blocks[prec][kernel][c] = per_cu * cus;
    return occ_blocks[prec][kernel][c];
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------

namespace pdfx {

// The adjoint with its workspace either grown in the grid (fixed_ws NULL) or
// taken from fixed_ws, fixed_cap bytes, which a call that needs more rejects
// before enqueuing anything.
int eval_xfx_backward(const pdfx_grid *g, const void *xf_dev, int prec, const int32_t *pids,
                      int32_t n_req, const double *x, const double *q2, int64_t n_pts,
                      const void *grad_out, void *grad_xf, double *grad_x, double *grad_q2,
                      int domain_mode, void *stream, void *fixed_ws, size_t fixed_cap)
{
    XfxArgs fa;
    // grad_out takes the place of `out` in the argument checks
    int rc = prepare_xfx_args(g, xf_dev, prec, pids, n_req, x, q2, n_pts,
                              const_cast<void *>(grad_out), domain_mode, &fa);
    if (rc != PDFX_OK)
        return rc;
    const uintptr_t a8 = 7, a4 = 3;
    if (((uintptr_t)grad_x & a8) || ((uintptr_t)grad_q2 & a8) ||
        ((uintptr_t)grad_xf & (prec == PDFX_F64 ? a8 : a4)))
        return fail(PDFX_EINVAL, "misaligned device pointer");
    if (!grad_xf && !grad_x && !grad_q2)
        return PDFX_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    const bool want_coord = grad_x || grad_q2;
    // coordinate sums by the forward-style kernel when the grid and the
    // request fit the double-buffered layout
    CoordArgs ca{};
    bool coord_fwd = false;
    if (want_coord && n_pts > 0 && g->dma_grid) {
        ca.x = fa;
        coord_fwd = plan_stages(ca.x, prec == PDFX_F32S ? 4 : 2) &&
                    dma_supported(LaunchShape{512, 1}, fa.nx, fa.nq, fa.ax.nbuckets,
                                  fa.aq.nbuckets);
    }
    // workspace: idx, flag, tx, tq, accx, accw per point, the FP64 knot
    // accumulator and the per-workgroup maxima of |dL/dout|
    const int64_t n = n_pts;
    const size_t nv = (size_t)g->nf * fa.nx * fa.nq;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t o_idx = 0, o_flag = o_idx + al(4 * n), o_tx = o_flag + al(n),
                 o_tq = o_tx + al(8 * n), o_ax = o_tq + al(8 * n), o_aw = o_ax + al(8 * n),
                 o_g = o_aw + al(8 * n), o_m = o_g + al(8 * nv),
                 total = o_m + al((size_t)8 * kMaxPart * fa.n_u);
    char *ws;
    if (fixed_ws) {
        if (total > fixed_cap)
            return fail(PDFX_EINVAL,
                        "%lld points on a %zu-value grid need %zu bytes of adjoint workspace; "
                        "the allocation-free call has %zu",
                        (long long)n, nv, total, fixed_cap);
        ws = (char *)fixed_ws;
    } else {
        if (g->bwd_ws.bytes < total) {
            if ((e = g->bwd_ws.upload(nullptr, total)) != hipSuccess)
                return fail_hip(e, "allocate adjoint workspace");
        }
        ws = (char *)g->bwd_ws.ptr;
    }
    if (xf_dev && want_coord && !coord_fwd) {
        RepackArgs r{xf_dev, g->scratch_vals[prec].ptr, g->nf, fa.nx, fa.nq, fa.slab_elems};
        if ((e = launch_repack(r, prec == PDFX_F32S, s)) != hipSuccess)
            return fail_hip(e, "repack launch");
        fa.vals = g->scratch_vals[prec].ptr;
    }
    BwdArgs a{};
    a.ax = fa.ax;
    a.aq = fa.aq;
    a.vals = fa.vals;
    a.nf = g->nf;
    a.nx = fa.nx;
    a.nq = fa.nq;
    a.slab_elems = fa.slab_elems;
    a.n_req = n_req;
    a.n_u = fa.n_u;
    for (int i = 0; i < kMaxReq; ++i) {
        a.urow[i] = fa.urow[i];
        a.ucols[i] = fa.ucols[i];
    }
    for (int i = 0; i <= kMaxReq; ++i)
        a.ucol_off[i] = fa.ucol_off[i];
    a.x = x;
    a.q = q2;
    a.n = n;
    a.domain_mode = domain_mode;
    a.gout = grad_out;
    a.st_idx = (int32_t *)(ws + o_idx);
    a.st_flag = (uint8_t *)(ws + o_flag);
    a.st_tx = (double *)(ws + o_tx);
    a.st_tq = (double *)(ws + o_tq);
    a.accx = want_coord ? (double *)(ws + o_ax) : nullptr;
    a.accw = want_coord ? (double *)(ws + o_aw) : nullptr;
    a.gacc = grad_xf ? (double *)(ws + o_g) : nullptr;
    a.gmax = grad_xf ? (double *)(ws + o_m) : nullptr;
    a.gout_f32 = prec == PDFX_F32S;
    if (coord_fwd) {
        ca.x.gvals = g->dvals[prec].ptr;
        ca.x.gstride = fa.nx * fa.nq;
        if (xf_dev) {
            if ((e = launch_grp_repack(xf_dev, g->scratch_dvals[prec].ptr, g->nf, fa.nx, fa.nq,
                                       g->n_groups[prec], ca.x.gstride, false, prec == PDFX_F32S,
                                       s)) != hipSuccess)
                return fail_hip(e, "repack launch");
            ca.x.gvals = g->scratch_dvals[prec].ptr;
        }
        ca.gout = grad_out;
        ca.grad_x = grad_x;
        ca.grad_q2 = grad_q2;
        if (a.gacc) {
            ca.st_idx = a.st_idx;
            ca.st_flag = a.st_flag;
            ca.st_tx = a.st_tx;
            ca.st_tq = a.st_tq;
            ca.gacc = a.gacc;
            ca.n_gacc = (int64_t)nv;
            ca.gmax = a.gmax;
            a.n_part = coord_grad_blocks(n, g->cus);
        }
        if ((e = launch_coord_grad(ca, prec == PDFX_F32S, g->cus, s)) != hipSuccess)
            return fail_hip(e, "adjoint launch");
    }
    e = launch_backward_ex(a, prec == PDFX_F32S, grad_xf, grad_x, grad_q2, g->cus, s, coord_fwd);
    if (e != hipSuccess)
        return fail_hip(e, "adjoint launch");
    return PDFX_OK;
}

}  // namespace pdfx

extern "C" int pdfx_eval_xfx_backward(const pdfx_grid *g, const void *xf_dev, int prec,
                                      const int32_t *pids, int32_t n_req, const double *x,
                                      const double *q2, int64_t n_pts, const void *grad_out,
                                      void *grad_xf, double *grad_x, double *grad_q2,
                                      int domain_mode, void *stream)
{
    pdfx::clear_error();
    return pdfx::eval_xfx_backward(g, xf_dev, prec, pids, n_req, x, q2, n_pts, grad_out, grad_xf,
                                   grad_x, grad_q2, domain_mode, stream, nullptr, 0);
}

// ---------------------------------------------------------------------------
// sets of members
// ---------------------------------------------------------------------------

pdfx_set::~pdfx_set()
{
    for (auto *g : members)
        delete g;
    for (auto *b : dma_vals)
        delete b;
}

namespace pdfx {

// Borderless group slabs with G values of V per node: group gi holds rows
// gi*G .. gi*G+G-1 (0 past n_flav), one every gstride nodes.
template <typename V>
static std::vector<V> group_slabs_g(const double *xf, int nf, int nx, int nq, int G, int gstride)
{
    const int n_groups = (nf + G - 1) / G;
    std::vector<V> out((size_t)n_groups * gstride * G, V(0));
    for (int f = 0; f < nf; ++f)
        for (int i = 0; i < nx; ++i)
            for (int k = 0; k < nq; ++k)
                out[((size_t)(f / G) * gstride + (size_t)i * nq + k) * G + f % G] =
                    (V)xf[((size_t)f * nx + i) * nq + k];
    return out;
}

// Node-width classes of a set for the double-buffered set kernel: per member
// and precision the widest node (16, 8, 4 bytes) whose slab fits, else (FP64)
// 8-byte nodes with the slab split over both LDS slabs; the group slabs in that
// width, and the member lists per class.
static int set_build_classes(pdfx_set *s, const pdfx_grid_desc *members, int n_mem)
{
    std::vector<SetMemberDev> md(n_mem);
    hipError_t e;
    for (int m = 0; m < n_mem; ++m) {
        const pdfx_grid *g = s->members[m];
        md[m].ax = g->ax.dev();
        md[m].aq = g->aq.dev();
        md[m].nx = g->ax.n;
        md[m].nq = g->aq.n;
        md[m].split_rows[0] = md[m].split_rows[1] = 0;
        for (int p = 0; p < 2; ++p) {
            const bool f32 = p == PDFX_F32S;
            int nb = set_node_bytes(g->ax.n, g->aq.n, g->ax.nbuckets, g->aq.nbuckets, f32);
            int cls = -1;
            for (int c = 0; c < 3; ++c)
                if (kSetClassWidth[c] == nb)
                    cls = c;
            // Wider nodes split over both slabs before narrower nodes in one
            // (fewer stages): 16-byte nodes over both, then 8-byte nodes over
            // both when even 8-byte nodes do not fit one slab (FP64) or only
            // 4-byte ones do (FP32).
            const int nbx = g->ax.nbuckets, nbq = g->aq.nbuckets;
            if (nb != 16) {
                const int r16 = set_split_rows(g->ax.n, g->aq.n, nbx, nbq, 16);
                if (r16 > 0) {
                    md[m].split_rows[p] = r16;
                    nb = 16;
                    cls = 4;
                }
            }
            if (cls < 0 || (f32 && nb == 4)) {
                const int r8 = set_split_rows(g->ax.n, g->aq.n, nbx, nbq, 8);
                if (r8 > 0) {
                    md[m].split_rows[p] = r8;
                    nb = 8;
                    cls = 3;
                }
            }
            md[m].nb[p] = nb;
            md[m].gvals[p] = nullptr;
            md[m].gstride[p] = 0;
            if (cls < 0) {
                s->rest_ids[p].push_back(m);
                continue;
            }
            const int vsize = f32 ? 4 : 8;
            const int G = nb / vsize;
            const int per16 = 16 / nb;   // nodes per 16 bytes
            const int gstride = (g->ax.n * g->aq.n + per16 - 1) / per16 * per16;
            auto *buf = new DeviceBuf();
            s->dma_vals.push_back(buf);
            if (f32) {
                auto v = group_slabs_g<float>(members[m].xf, g->nf, g->ax.n, g->aq.n, G, gstride);
                e = buf->upload(v.data(), v.size() * sizeof(float));
            } else {
                auto v = group_slabs_g<double>(members[m].xf, g->nf, g->ax.n, g->aq.n, G, gstride);
                e = buf->upload(v.data(), v.size() * sizeof(double));
            }
            if (e != hipSuccess)
                return fail_hip(e, "upload member values");
            md[m].gvals[p] = buf->ptr;
            md[m].gstride[p] = gstride;
            s->cls_ids[p][cls].push_back(m);
        }
    }
    if ((e = s->dma_mem.upload(md.data(), md.size() * sizeof(SetMemberDev))) != hipSuccess)
        return fail_hip(e, "upload set descriptors");
    for (int p = 0; p < 2; ++p) {
        // one work list for every class: dearest classes first, and inside a
        // class the largest grids first
        std::vector<int> order;
        for (int o = 0; o < kSetClasses; ++o) {
            const int c = kSetClassOrder[o];
            std::vector<int> ids = s->cls_ids[p][c];
            std::stable_sort(ids.begin(), ids.end(), [&](int u, int v) {
                return md[u].nx * md[u].nq > md[v].nx * md[v].nq;
            });
            for (int m : ids) {
                order.push_back(m);
                order.push_back(c);
            }
        }
        s->n_order[p] = (int)order.size() / 2;
        if (!order.empty() &&
            (e = s->order_dev[p].upload(order.data(), order.size() * sizeof(int))) != hipSuccess)
            return fail_hip(e, "upload set work list");
        if (!s->rest_ids[p].empty() &&
            (e = s->rest_dev[p].upload(s->rest_ids[p].data(),
                                       s->rest_ids[p].size() * sizeof(int))) != hipSuccess)
            return fail_hip(e, "upload set work list");
    }
    return PDFX_OK;
}

// LDS layout of the single-slab set kernel for the largest of the members ids
// (all members if ids is null); 0 if it does not fit.
static size_t set_lds_layout(const pdfx_set *s, bool f32, const std::vector<int> *ids,
                             SetArgs *a)
{
    int max_nx = 0, max_nq = 0, max_nbx = 0, max_nbq = 0;
    size_t max_slab = 0;
    const int n = ids ? (int)ids->size() : (int)s->members.size();
    if (n == 0)
        return 0;
    for (int i = 0; i < n; ++i) {
        const pdfx_grid *g = s->members[ids ? (*ids)[i] : i];
        max_nx = std::max(max_nx, g->ax.n);
        max_nq = std::max(max_nq, g->aq.n);
        max_nbx = std::max(max_nbx, g->ax.nbuckets);
        max_nbq = std::max(max_nbq, g->aq.nbuckets);
        const int p = f32 ? PDFX_F32S : PDFX_F64;
        max_slab = std::max(max_slab, (size_t)g->slab_elems[p] * (f32 ? 4 : 8));
    }
    size_t off = 0;
    auto take = [&](size_t bytes, size_t align) {
        off = (off + align - 1) / align * align;
        const size_t r = off;
        off += bytes;
        return (int)r;
    };
    a->lx.knots = take((size_t)max_nx * 8, 16);
    a->lx.seed = take((size_t)max_nbx * 2, 16);
    a->lx.rec64 = take((size_t)(max_nx - 1) * 64, 64);
    a->lx.rec32 = take(f32 ? (size_t)(max_nx - 1) * 32 : 0, 64);
    a->lq.knots = take((size_t)max_nq * 8, 16);
    a->lq.seed = take((size_t)max_nbq * 2, 16);
    a->lq.rec64 = take((size_t)(max_nq - 1) * 64, 64);
    a->lq.rec32 = take(f32 ? (size_t)(max_nq - 1) * 32 : 0, 64);
    a->lds_slab = take(max_slab, 16);
    // the kernel's own static __shared__ word sits beside the dynamic region
    return off + 16 <= kLdsLimit ? off : 0;
}

}  // namespace pdfx

extern "C" {

int pdfx_load_set(const pdfx_grid_desc *members, int32_t n_mem, pdfx_set **out)
{
    using namespace pdfx;
    clear_error();
    if (!out)
        return fail(PDFX_EINVAL, "out is NULL");
    *out = nullptr;
    if (!members || n_mem < 1 || n_mem > 100000)
        return fail(PDFX_EINVAL, "need 1..100000 member descriptors");
    for (int m = 0; m < n_mem; ++m) {
        int rc = validate_desc(&members[m], true);
        if (rc != PDFX_OK)
            return fail(rc, "member %d: %s", m, pdfx_last_error());
        if (members[m].n_flav != members[0].n_flav)
            return fail(PDFX_EINVAL, "member %d: flavour count differs from member 0", m);
        for (int f = 0; f < members[0].n_flav; ++f)
            if (members[m].pids[f] != members[0].pids[f])
                return fail(PDFX_EINVAL, "member %d: pid list differs from member 0", m);
    }
    pdfx_set *s = new pdfx_set();
    s->pids.assign(members[0].pids, members[0].pids + members[0].n_flav);
    std::vector<MemberDev> md(n_mem);
    for (int m = 0; m < n_mem; ++m) {
        pdfx_grid *g = new pdfx_grid();
        s->members.push_back(g);
        pdfx_grid_desc d = members[m];
        d.n_as = 0;  // alpha_s is not part of a set evaluation
        int rc = grid_init(g, &d);
        if (rc != PDFX_OK) {
            delete s;
            return rc;
        }
        md[m].ax = g->ax.dev();
        md[m].aq = g->aq.dev();
        md[m].vals64 = g->vals[PDFX_F64].ptr;
        md[m].vals32 = g->vals[PDFX_F32S].ptr;
        md[m].nx = g->ax.n;
        md[m].nq = g->aq.n;
        md[m].slab64 = g->slab_elems[PDFX_F64];
        md[m].slab32 = g->slab_elems[PDFX_F32S];
        s->max_nx = std::max(s->max_nx, g->ax.n);
        s->max_nq = std::max(s->max_nq, g->aq.n);
    }
    SetArgs probe{};
    if (set_lds_layout(s, true, nullptr, &probe) == 0) {
        delete s;
        return fail(PDFX_EINVAL, "the largest member does not fit one LDS slab");
    }
    int rc = set_build_classes(s, members, n_mem);
    if (rc != PDFX_OK) {
        delete s;
        return rc;
    }
    hipError_t e;
    if ((e = s->mem_desc.upload(md.data(), md.size() * sizeof(MemberDev))) != hipSuccess ||
        (e = s->counter.upload(nullptr, 256)) != hipSuccess ||
        (e = s->dom_count.upload(nullptr, sizeof(unsigned long long))) != hipSuccess ||
        (e = s->call_count.upload(nullptr, sizeof(unsigned long long))) != hipSuccess) {
        delete s;
        return fail_hip(e, "upload set descriptors");
    }
    s->cus = device_cu_count();
    *out = s;
    return PDFX_OK;
}

void pdfx_free_set(pdfx_set *s) { delete s; }

int pdfx_eval_set_xfx(const pdfx_set *s, int prec, const int32_t *pids, int32_t n_req,
                      const double *x, const double *q2, int64_t n_pts, void *out,
                      int domain_mode, void *stream)
{
    using namespace pdfx;
    clear_error();
    if (!s)
        return fail(PDFX_EINVAL, "set is NULL");
    // argument checks and the column plan, as for one member
    XfxArgs fa;
    const pdfx_grid *g0 = s->members[0];
    const bool err = domain_mode == PDFX_DOMAIN_ERROR;
    if (err)
        domain_mode = PDFX_DOMAIN_NAN;
    int rc = prepare_xfx_args(g0, nullptr, prec == PDFX_F64 ? PDFX_F32S : prec, pids, n_req, x,
                              q2, n_pts, out, domain_mode, &fa);
    if (rc != PDFX_OK)
        return rc;
    if (prec != PDFX_F64 && prec != PDFX_F32S)
        return fail(PDFX_EINVAL, "unknown precision %d", prec);
    if (n_pts == 0)
        return PDFX_OK;
    SetArgs a{};
    a.mem = (const MemberDev *)s->mem_desc.ptr;
    a.n_mem = (int)s->members.size();
    a.n_req = n_req;
    a.n_u = fa.n_u;
    a.n_zero = fa.n_zero;
    for (int i = 0; i < kMaxReq; ++i) {
        a.urow[i] = fa.urow[i];
        a.ucols[i] = fa.ucols[i];
        a.zcols[i] = fa.zcols[i];
    }
    for (int i = 0; i <= kMaxReq; ++i)
        a.ucol_off[i] = fa.ucol_off[i];
    a.x = x;
    a.q = q2;
    a.n = n_pts;
    a.out = out;
    a.domain_mode = domain_mode;
    a.dom_count = (unsigned long long *)(err ? s->call_count.ptr : s->dom_count.ptr);
    a.counter = (unsigned int *)s->counter.ptr;
    const LaunchShape ls = s->shape[prec];
    const int64_t tile_pts = (int64_t)ls.block * ls.ppt;
    const int64_t ntiles = (n_pts + tile_pts - 1) / tile_pts;
    int64_t tpi = s->tiles_per_item[prec];
    if (tpi < 1)
        tpi = 1;
    const int64_t ipm = (ntiles + tpi - 1) / tpi;
    if ((int64_t)a.n_mem * ipm > 0x7fffffff)
        return fail(PDFX_EINVAL, "work list too long");
    a.tiles_per_item = (int)tpi;
    a.items_per_member = (int)ipm;
    a.n_items = (int)(a.n_mem * ipm);
    const bool f32 = prec == PDFX_F32S;
    hipError_t e;
    // Double-buffered classes, all in one launch: a launch shape the kernel
    // is compiled for, 16-byte aligned member blocks, and a request whose
    // groups fit the result slots of every group width G its classes use.
    // The other members (or all, otherwise) go through the single-slab kernel.
    SetDmaArgs d{};
    const int vs = f32 ? 4 : 8;
    bool dma = set_dma_shape_supported(ls, f32) && (uintptr_t)out % 16 == 0 &&
               (n_pts * n_req * vs) % 16 == 0 && s->n_order[prec] > 0;
    bool have_dup = false;
    for (int c = 0; c < kSetClasses && dma; ++c) {
        if (s->cls_ids[prec][c].empty())
            continue;
        const int G = kSetClassWidth[c] / vs;
        const int gi = G == 1 ? 0 : G == 2 ? 1 : 2;
        XfxArgs plan = fa;
        if (!plan_stages(plan, G)) {
            dma = false;
            break;
        }
        d.plan[gi].n_stage = plan.n_stage;
        for (int k = 0; k < kGrpMaxSlots; ++k) {
            d.plan[gi].sgrp[k] = plan.sgrp[k];
            d.plan[gi].slot_col[k] = plan.slot_col[k];
        }
        if (!have_dup) {   // the repeated columns do not depend on G
            have_dup = true;
            d.n_zero = plan.n_zero;
            d.n_dup = plan.n_dup;
            for (int k = 0; k < kMaxReq; ++k) {
                d.zcols[k] = plan.zcols[k];
                d.dup_src[k] = plan.dup_src[k];
                d.dup_dst[k] = plan.dup_dst[k];
            }
        }
    }
    if (dma) {
        d.mem = (const SetMemberDev *)s->dma_mem.ptr;
        d.ids = (const int2 *)s->order_dev[prec].ptr;
        d.n_ids = s->n_order[prec];
        d.items_per_member = (int)ipm;
        d.tiles_per_item = (int)tpi;
        d.n_items = (int)(d.n_ids * ipm);
        d.counter = a.counter;
        d.n_req = n_req;
        d.x = x;
        d.q = q2;
        d.n = n_pts;
        d.out = out;
        d.domain_mode = domain_mode;
        d.dom_count = a.dom_count;
        int64_t pass = (int64_t)kSetSlabBytes / ((int64_t)n_req * vs) / 16 * 16;
        if (pass > tile_pts)
            pass = tile_pts;
        d.out_pass_pts = (int)pass;
    }
    // the single-slab kernel takes the members outside the classes (all of
    // them without the classes) and needs each one's slab in LDS
    const size_t lds = set_lds_layout(s, f32, dma ? &s->rest_ids[prec] : nullptr, &a);
    if (lds == 0 && (!dma || !s->rest_ids[prec].empty()))
        return fail(PDFX_EINVAL, "a member does not fit LDS in this precision%s",
                    dma ? "" : " (members beyond one slab need the double-buffered classes: "
                               "16-byte aligned output blocks and a set launch shape they "
                               "are compiled for)");
    if (err && (rc = error_mode_begin(s->call_count.ptr, (hipStream_t)stream)) != PDFX_OK)
        return rc;
    auto done = [&]() {
        return err ? error_mode_end(s->call_count.ptr, (hipStream_t)stream, &s->host_count)
                   : PDFX_OK;
    };
    if (dma) {
        if ((e = launch_set_dma(d, f32, ls, s->cus, (hipStream_t)stream)) != hipSuccess)
            return fail_hip(e, "set launch");
        if (s->rest_ids[prec].empty())
            return done();
        a.mem_ids = (const int *)s->rest_dev[prec].ptr;
        a.n_items = (int)(s->rest_ids[prec].size() * ipm);
    }
    // the single-slab kernel runs the FP32-only class shape as (512, 2): tiles
    // of half the points, twice as many per work item (same points per item)
    LaunchShape ls_set = ls;
    if (launch_shape_f32_only(ls)) {
        ls_set = LaunchShape{512, 2};
        a.tiles_per_item *= 2;
    }
    e = launch_set(a, f32, ls_set, lds, s->cus, (hipStream_t)stream);
    if (e != hipSuccess)
        return fail_hip(e, "set launch");
    return done();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Drell-Yan-like integrand
// ---------------------------------------------------------------------------

namespace pdfx {

// True if the integrand can use the double-buffered kernel: the grid fits
// it and holds the 11 partons in the standard order -5 .. -1, g, 1 .. 5.
static bool dy_dma_ok(const pdfx_grid *g)
{
    if (!g->dma_grid || g->nf != 11 ||
        !dy_dma_supported(g->ax.n, g->aq.n, g->aa.n, g->ax.nbuckets, g->aq.nbuckets))
        return false;
    for (int q = 1; q <= 5; ++q)
        if (g->row_of(q) != 5 + q || g->row_of(-q) != 5 - q)
            return false;
    return true;
}

static int prepare_dy(const pdfx_grid *g, const void *xf_dev, int prec, const double *u1,
                      const double *u2, int64_t n, double xmin, double s, DyArgs *a,
                      hipStream_t stream)
{
    if (!g)
        return fail(PDFX_EINVAL, "grid is NULL");
    if (prec != PDFX_F64 && prec != PDFX_F32S)
        return fail(PDFX_EINVAL, "unknown precision %d", prec);
    if (!g->has_alphas)
        return fail(PDFX_ENOALPHAS, "the integrand needs alpha_s knots");
    if (!xf_dev && !g->has_values)
        return fail(PDFX_ENOVALUES, "grid has no owned values and xf_dev is NULL");
    if (n < 0)
        return fail(PDFX_EINVAL, "n < 0");
    if (n > 0 && (!u1 || !u2))
        return fail(PDFX_EINVAL, "u1 or u2 is NULL");
    if (((uintptr_t)u1 & 7) || ((uintptr_t)u2 & 7))
        return fail(PDFX_EINVAL, "misaligned device pointer");
    if (!(xmin > 0.0 && xmin < 1.0) || !(s > 0.0) || !std::isfinite(s))
        return fail(PDFX_EINVAL, "need 0 < xmin < 1 and s > 0");
    *a = DyArgs{};
    a->ax = g->ax.dev();
    a->aq = g->aq.dev();
    a->aa = g->aa.dev();
    a->as_vals = prec == PDFX_F64 ? g->as_vals64.ptr : g->as_vals32.ptr;
    a->as_vals64 = (const double *)g->as_vals64.ptr;
    a->vals = g->vals[prec].ptr;
    a->nf = g->nf;
    a->nx = g->ax.n;
    a->nq = g->aq.n;
    a->slab_elems = g->slab_elems[prec];
    bool db = false;
    if (dy_lds_layout(*a, prec == PDFX_F32S, &db) == 0)
        return fail(PDFX_EINVAL, "grid too large for an LDS slab in this precision");
    a->n_seq = 0;
    for (int q = 1; q <= 5; ++q) {
        const int rq = g->row_of(q), rqb = g->row_of(-q);
        if (rq < 0 || rqb < 0)
            continue;   // an absent parton contributes 0
        a->seq_row[a->n_seq++] = rq;
        a->seq_row[a->n_seq++] = rqb;
    }
    a->u1 = u1;
    a->u2 = u2;
    a->n = n;
    a->lnxmin = std::log(xmin);
    a->lnrange = std::log(1.0 / xmin);
    a->s = s;
    a->L2 = a->lnrange * a->lnrange;
    a->dom_count = (unsigned long long *)g->dom_count.ptr;
    if (xf_dev && n > 0) {
        RepackArgs r{xf_dev, g->scratch_vals[prec].ptr, g->nf, a->nx, a->nq, a->slab_elems};
        hipError_t e = launch_repack(r, prec == PDFX_F32S, stream);
        if (e != hipSuccess)
            return fail_hip(e, "repack launch");
        a->vals = g->scratch_vals[prec].ptr;
    }
    return PDFX_OK;
}

}  // namespace pdfx

extern "C" {

int32_t pdfx_dy_max_blocks(void) { return pdfx::kDyMaxBlocks; }

int pdfx_eval_dy(const pdfx_grid *g, const void *xf_dev, int prec, const double *u1,
                 const double *u2, int64_t n, double xmin, double s, void *out,
                 double *block_sums, int32_t *n_blocks, void *stream)
{
    using namespace pdfx;
    clear_error();
    if (n_blocks)
        *n_blocks = 0;
    DyArgs a;
    int rc = prepare_dy(g, xf_dev, prec, u1, u2, n, xmin, s, &a, (hipStream_t)stream);
    if (rc != PDFX_OK || n == 0)
        return rc;
    if (((uintptr_t)out & 3) || ((uintptr_t)block_sums & 7))
        return fail(PDFX_EINVAL, "misaligned device pointer");
    a.out = out;
    a.block_sums = block_sums;
    int nb = 0;
    hipError_t e;
    const bool f32 = prec == PDFX_F32S;
    if (dy_dma_ok(g)) {
        // double-buffered kernel over the flavour groups of the grid
        a.gvals = g->dvals[prec].ptr;
        a.gstride = a.nx * a.nq;
        if (xf_dev) {
            if ((e = launch_grp_repack(xf_dev, g->scratch_dvals[prec].ptr, g->nf, a.nx, a.nq,
                                       g->n_groups[prec], a.gstride, false, f32,
                                       (hipStream_t)stream)) != hipSuccess)
                return fail_hip(e, "repack launch");
            a.gvals = g->scratch_dvals[prec].ptr;
        }
        e = launch_dy_dma_forward(a, f32, g->dy_shape[prec], g->cus, (hipStream_t)stream, &nb);
    } else {
        e = launch_dy_forward(a, f32, g->cus, (hipStream_t)stream, &nb);
    }
    if (e != hipSuccess)
        return fail_hip(e, "integrand launch");
    if (n_blocks)
        *n_blocks = nb;
    return PDFX_OK;
}

int pdfx_eval_dy_backward(const pdfx_grid *g, const void *xf_dev, int prec, const double *u1,
                          const double *u2, int64_t n, double xmin, double s, double scale,
                          void *grad_xf, void *stream)
{
    using namespace pdfx;
    clear_error();
    DyArgs a;
    int rc = prepare_dy(g, xf_dev, prec, u1, u2, n, xmin, s, &a, (hipStream_t)stream);
    if (rc != PDFX_OK)
        return rc;
    if (!grad_xf)
        return fail(PDFX_EINVAL, "grad_xf is NULL");
    if ((uintptr_t)grad_xf & (prec == PDFX_F64 ? 7 : 3))
        return fail(PDFX_EINVAL, "misaligned device pointer");
    if (n == 0)
        return PDFX_OK;
    a.scale = scale;
    const size_t nv = (size_t)g->nf * a.nx * a.nq;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t o_i1 = 0, o_i2 = o_i1 + al(4 * n), o_t1 = o_i2 + al(4 * n), o_t2 = o_t1 + al(8 * n),
                 o_tq = o_t2 + al(8 * n), o_as = o_tq + al(8 * n), o_g = o_as + al(8 * n),
                 total = o_g + al(8 * nv);
    hipError_t e;
    if (g->bwd_ws.bytes < total && (e = g->bwd_ws.upload(nullptr, total)) != hipSuccess)
        return fail_hip(e, "allocate integrand workspace");
    char *ws = (char *)g->bwd_ws.ptr;
    a.st_i1 = (int32_t *)(ws + o_i1);
    a.st_i2 = (int32_t *)(ws + o_i2);
    a.st_t1 = (double *)(ws + o_t1);
    a.st_t2 = (double *)(ws + o_t2);
    a.st_tq = (double *)(ws + o_tq);
    a.st_as = (double *)(ws + o_as);
    a.gacc = (double *)(ws + o_g);
    const bool pairs = dy_dma_ok(g);
    if (pairs) {
        // knot-gradient pass by quark-antiquark pairs, from the borderless groups
        a.gvals = g->dvals[prec].ptr;
        a.gstride = a.nx * a.nq;
        if (xf_dev) {
            if ((e = launch_grp_repack(xf_dev, g->scratch_dvals[prec].ptr, g->nf, a.nx, a.nq,
                                       g->n_groups[prec], a.gstride, false, prec == PDFX_F32S,
                                       (hipStream_t)stream)) != hipSuccess)
                return fail_hip(e, "repack launch");
            a.gvals = g->scratch_dvals[prec].ptr;
        }
    }
    e = launch_dy_backward_ex(a, prec == PDFX_F32S, grad_xf, g->cus, (hipStream_t)stream, pairs);
    if (e != hipSuccess)
        return fail_hip(e, "integrand backward launch");
    return PDFX_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Flavour-pair luminosity
// ---------------------------------------------------------------------------

extern "C" {

int pdfx_eval_lumi(const pdfx_grid *g, const void *xf_dev, int prec, int32_t n_pair,
                   const int32_t *pid_a, const int32_t *pid_b, const double *coef,
                   const double *x1, const double *x2, const double *q2, double q2_fixed,
                   int64_t n, void *out_pair, void *out_sum, int domain_mode, void *stream)
{
    using namespace pdfx;
    clear_error();
    if (!g)
        return fail(PDFX_EINVAL, "grid is NULL");
    if (prec != PDFX_F64 && prec != PDFX_F32S)
        return fail(PDFX_EINVAL, "unknown precision %d", prec);
    if (!xf_dev && !g->has_values)
        return fail(PDFX_ENOVALUES, "grid has no owned values and xf_dev is NULL");
    if (n_pair < 1 || n_pair > kLumiMaxPairs)
        return fail(PDFX_EINVAL, "n_pair = %d outside [1, %d]", n_pair, kLumiMaxPairs);
    if (!pid_a || !pid_b)
        return fail(PDFX_EINVAL, "pid_a or pid_b is NULL");
    if (domain_mode != PDFX_DOMAIN_NAN && domain_mode != PDFX_DOMAIN_CLAMP &&
        domain_mode != PDFX_DOMAIN_ERROR)
        return fail(PDFX_EINVAL, "unknown domain mode %d", domain_mode);
    const bool err = domain_mode == PDFX_DOMAIN_ERROR;
    if (err)
        domain_mode = PDFX_DOMAIN_NAN;
    if (n < 0)
        return fail(PDFX_EINVAL, "n < 0");
    if (n > 0 && !out_pair && !out_sum)
        return fail(PDFX_EINVAL, "out_pair and out_sum are both NULL");
    if (!q2 && !(q2_fixed > 0.0 && std::isfinite(q2_fixed)))
        return fail(PDFX_EINVAL, "q2 is NULL and q2_fixed is not positive and finite");
    if (coef)
        for (int k = 0; k < n_pair; ++k)
            if (!std::isfinite(coef[k]))
                return fail(PDFX_EINVAL, "coef[%d] is not finite", k);
    const bool f32 = prec == PDFX_F32S;
    const size_t vs = f32 ? 4 : 8;
    if (((uintptr_t)x1 & 7) || ((uintptr_t)x2 & 7) || ((uintptr_t)q2 & 7) ||
        ((uintptr_t)out_pair & (vs - 1)) || ((uintptr_t)out_sum & (vs - 1)))
        return fail(PDFX_EINVAL, "misaligned device pointer");
    if (!g->dma_grid || !lumi_supported(g->ax.n, g->aq.n, g->ax.nbuckets, g->aq.nbuckets))
        return fail(PDFX_EINVAL, "grid %dx%d does not fit the luminosity kernel's LDS slabs",
                    g->ax.n, g->aq.n);
    if (n == 0)
        return PDFX_OK;
    if (!x1 || !x2)
        return fail(PDFX_EINVAL, "x1 or x2 is NULL");

    // Stage plan: the flavour groups holding a parton of some pair, in grid
    // order, each with the side(s) it is evaluated at; slot s*G+g of a row.
    const int G = f32 ? 4 : 2;
    const int ng = g->n_groups[prec];
    std::vector<int> side_of_group(ng, 0), stage_of_group(ng, -1);
    std::vector<int> ra(n_pair), rb(n_pair);
    for (int k = 0; k < n_pair; ++k) {
        ra[k] = g->row_of(pid_a[k]);
        rb[k] = g->row_of(pid_b[k]);
        if (ra[k] < 0 || rb[k] < 0)
            continue;   // a pair with an absent parton is 0
        side_of_group[ra[k] / G] |= 1;
        side_of_group[rb[k] / G] |= 2;
    }
    LumiArgs a{};
    for (int gi = 0; gi < ng; ++gi) {
        if (side_of_group[gi]) {
            if (a.n_stage == kGrpMaxSlots / G)
                return fail(PDFX_EINVAL, "the pairs touch more than %d flavour groups of %d",
                            kGrpMaxSlots / G, G);
            stage_of_group[gi] = a.n_stage;
            a.sgrp[a.n_stage] = gi;
            a.side[a.n_stage] = side_of_group[gi];
            ++a.n_stage;
        }
    }
    a.n_pair = n_pair;
    for (int k = 0; k < n_pair; ++k) {
        const bool live = ra[k] >= 0 && rb[k] >= 0;
        a.ia[k] = live ? stage_of_group[ra[k] / G] * G + ra[k] % G : -1;
        a.ib[k] = live ? stage_of_group[rb[k] / G] * G + rb[k] % G : -1;
        a.coef[k] = coef ? coef[k] : 1.0;
    }
    a.ax = g->ax.dev();
    a.aq = g->aq.dev();
    a.nx = g->ax.n;
    a.nq = g->aq.n;
    a.gstride = a.nx * a.nq;
    a.gvals = g->dvals[prec].ptr;
    hipError_t e;
    if (xf_dev) {
        if ((e = launch_grp_repack(xf_dev, g->scratch_dvals[prec].ptr, g->nf, a.nx, a.nq,
                                   g->n_groups[prec], a.gstride, false, f32,
                                   (hipStream_t)stream)) != hipSuccess)
            return fail_hip(e, "repack launch");
        a.gvals = g->scratch_dvals[prec].ptr;
    }
    a.x1 = x1;
    a.x2 = x2;
    a.q2 = q2;
    a.q2_fixed = q2_fixed;
    a.n = n;
    a.out_pair = out_pair;
    a.out_sum = out_sum;
    a.domain_mode = domain_mode;
    a.dom_count = (unsigned long long *)(err ? g->call_count.ptr : g->dom_count.ptr);
    LaunchShape ls = g->lumi_shape[prec];
    if (!g->lumi_pinned[prec] && ls.ppt > 1) {
        // a small call: (512, 1) gives twice or more the workgroups
        const int64_t tile = (int64_t)ls.block * ls.ppt;
        if ((n + tile - 1) / tile < g->cus / 2)
            ls = LaunchShape{512, 1};
    }
    if (err) {
        const int rc = error_mode_begin(g->call_count.ptr, (hipStream_t)stream);
        if (rc != PDFX_OK)
            return rc;
    }
    if ((e = launch_lumi(a, f32, ls, g->cus, (hipStream_t)stream)) != hipSuccess)
        return fail_hip(e, "luminosity launch");
    if (err)
        return error_mode_end(g->call_count.ptr, (hipStream_t)stream, &g->host_count);
    return PDFX_OK;
}

}  // extern "C"
