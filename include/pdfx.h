/*
 * pdfx: batched parton-density and alpha_s interpolation on AMD MI355X (gfx950).
 *
 * The problem statement follows PDFFlow (arXiv:2012.08221), Sec. 2.1: a query
 * is a set of flavours {a} plus two arrays of equal length, momentum fractions
 * x_i and scales Q_i, and the answer is the array of interpolated values; the
 * interpolation is the LHAPDF one, i.e. log-bicubic (cubic Hermite in ln x and
 * in ln Q^2, finite-difference slopes) inside the Q^2 subgrid that holds the
 * point, subgrids meeting at the flavour thresholds.  alpha_s(Q^2) is the same
 * 1-D cubic Hermite in ln Q^2 (Sec. 2.1, last paragraph before Fig. 1).  The
 * returned PDF quantity is x f(x, Q^2) (Sec. 3.2 divides the luminosity by x1 x2).
 *
 * Conventions for every call:
 *  - All functions return PDFX_OK (0) or a negative pdfx_status.  Only errors
 *    the host can see are returned; pdfx_last_error() gives a thread-local
 *    message for the last failure on the calling thread.
 *  - Device pointers are plain HIP device addresses on the current device
 *    (e.g. torch tensor data pointers), contiguous, at least 8-byte aligned.
 *    The caller owns them and the stream; the library never frees them.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every eval call
 *    only enqueues work on it and returns; nothing is copied to or from the
 *    host on the eval path (except in domain mode PDFX_DOMAIN_ERROR, below).
 *  - A failed call leaves every handle valid and enqueues nothing.
 *  - A grid (or set) owns scratch memory that its calls share: repacked
 *    caller values, the adjoint and integrand-gradient workspaces and the
 *    domain counter.  Calls on one handle are ordered by being on one stream;
 *    calls that may run at the same time on different streams need different
 *    handles.  A handle also caches launch data on the host (occupancy, the
 *    workspace size): use each handle from one host thread at a time.
 *  - Eval calls allocate nothing, except that pdfx_eval_xfx_backward and
 *    pdfx_eval_dy_backward grow their handle's workspace (a synchronous device
 *    allocation) the first time they see a larger n; a call sequence meant
 *    for HIP graph capture is run once at full size before capturing it.
 *    No call records a memset: scratch that must start at zero is cleared by
 *    kernels on the call's stream.
 *  - PDG ids: 21 and 0 both mean the gluon; a pid absent from the grid
 *    evaluates to 0; output columns follow the request order.
 *  - Points outside the grid: PDFX_DOMAIN_NAN writes NaN for every column of
 *    that point and counts the point (pdfx_domain_errors); PDFX_DOMAIN_CLAMP
 *    evaluates at the point clamped to the grid edge (and counts nothing,
 *    except NaN inputs, which give NaN and are counted in every mode).
 *    PDFX_DOMAIN_EXTRAPOLATE (pdfx_eval_xfx and pdfx_eval_xfxQ only)
 *    continues beyond an edge from the edge knot e through the next knot n
 *    inward, with F_e, F_n the interpolation at those knot coordinates and
 *    u = ln(z/z_e) / ln(z_n/z_e): xf = F_e (F_n/F_e)^u if F_n/F_e > 0, else
 *    F_e + u (F_n - F_e); outside in x and Q^2 alike, x first, then Q^2.
 *    It counts only NaN inputs.  The other calls reject it.
 *    PDFX_DOMAIN_ERROR (every forward call: x f, alpha_s, both in one pass,
 *    sets, luminosity) evaluates as PDFX_DOMAIN_NAN, then waits for the
 *    stream and returns PDFX_EDOMAIN if any point of this call was outside
 *    the grid or NaN (its outputs are written as in NAN mode and the points
 *    are added to the pdfx_domain_errors / pdfx_set_domain_errors count).
 *    It is the one synchronous evaluation mode: do not use it under HIP
 *    graph capture.  pdfx_check_points applies the same rule to host arrays
 *    before anything is uploaded.
 *  - Ties: a Q^2 equal to a subgrid threshold uses the upper subgrid; a
 *    query on the last knot of an axis uses the last interval.
 */
#ifndef PDFX_H
#define PDFX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdfx_grid pdfx_grid; /* one PDF member, geometry + alpha_s on the device */
typedef struct pdfx_set pdfx_set;   /* many members with uneven grids */

/* Host description of one member.  Read only during pdfx_load_grid /
 * pdfx_load_set; the caller may free it afterwards. */
typedef struct pdfx_grid_desc {
    int32_t n_flav;        /* number of parton rows, 1..64 */
    const int32_t *pids;   /* [n_flav] PDG ids of the rows, distinct (0 and 21 count as equal) */
    int32_t n_x;           /* number of x knots, 2..4096 */
    const double *x;       /* [n_x] strictly increasing, x[0] > 0 */
    int32_t n_sub;         /* number of Q^2 subgrids, 1..16 */
    const int32_t *q_off;  /* [n_sub+1] offsets into q2; q_off[0] = 0, >= 2 knots per subgrid */
    const double *q2;      /* [q_off[n_sub]] GeV^2, > 0; strictly increasing inside each
                              subgrid; the last knot of subgrid s equals the first of s+1 */
    const double *xf;      /* [n_flav][n_x][n_q] host values of x f, finite; NULL = none
                              (then values must be passed to each eval call) */
    int32_t n_as;          /* alpha_s knots (0 = none) */
    const double *as_q2;   /* [n_as] non-decreasing; a repeated knot splits subgrids */
    const double *as_val;  /* [n_as] alpha_s at the knots, finite */
} pdfx_grid_desc;

enum pdfx_status {
    PDFX_OK = 0,
    PDFX_EINVAL = -1,     /* invalid argument or descriptor */
    PDFX_ENOMEM = -2,     /* device allocation failed */
    PDFX_EHIP = -3,       /* a HIP runtime call failed */
    PDFX_EDOMAIN = -4,    /* a point outside the grid: returned only by PDFX_DOMAIN_ERROR
                             calls (outputs written, NaN at those points) and by
                             pdfx_check_points */
    PDFX_ENOALPHAS = -5,  /* the grid has no alpha_s knots */
    PDFX_ENOVALUES = -6   /* no owned values and none passed */
};

/* Arithmetic of an evaluation.
 * PDFX_F64:  everything in FP64; values, outputs FP64.
 * PDFX_F32S: logs, knot search, subgrid choice and the local coordinate t in
 *            FP64; t rounded to FP32; basis, slope folding, weights, stencil
 *            FMAs, values and outputs FP32. */
enum pdfx_prec { PDFX_F64 = 0, PDFX_F32S = 1 };

enum pdfx_domain {
    PDFX_DOMAIN_NAN = 0,
    PDFX_DOMAIN_CLAMP = 1,
    PDFX_DOMAIN_EXTRAPOLATE = 2,
    PDFX_DOMAIN_ERROR = 3
};

/* Maximum number of requested pids in one call. */
#define PDFX_MAX_REQ 64

/* ---- grid lifetime (Sec. 2.1: mkPDF builds a PDF object for one member) ---- */

/* Validates d, derives per-interval tables on the host in FP64 and copies
 * geometry, alpha_s knots and (if d->xf) FP64 and FP32 copies of the values to
 * the current device.  Synchronous.  *out receives the handle. */
int pdfx_load_grid(const pdfx_grid_desc *d, pdfx_grid **out);
void pdfx_free_grid(pdfx_grid *g);

/* Shape of a loaded grid (any pointer may be NULL). */
int pdfx_grid_shape(const pdfx_grid *g, int32_t *n_flav, int32_t *n_x, int32_t *n_q,
                    int32_t *n_sub, int32_t *n_as);

/* ---- PDF evaluation (Sec. 2.1: py_xfxQ / xfxQ2 over arrays of points) ---- */

/* out[p][r] = x f_{pids[r]}(x[p], q2[p]) for p < n_pts, r < n_req.
 *  xf_dev   device values [n_flav][n_x][n_q] of the precision's type (FP64 for
 *           PDFX_F64, FP32 for PDFX_F32S), or NULL to use the owned values.
 *  pids     host array [n_req], 1 <= n_req <= PDFX_MAX_REQ.
 *  x, q2    device FP64 [n_pts]; Q^2 in GeV^2.
 *  out      device [n_pts][n_req], FP64 or FP32 by precision.
 * n_pts = 0 is a no-op. */
int pdfx_eval_xfx(const pdfx_grid *g, const void *xf_dev, int prec,
                  const int32_t *pids, int32_t n_req,
                  const double *x, const double *q2, int64_t n_pts,
                  void *out, int domain_mode, void *stream);

/* Same with Q instead of Q^2: Q^2 = Q*Q is formed in FP64 on the device. */
int pdfx_eval_xfxQ(const pdfx_grid *g, const void *xf_dev, int prec,
                   const int32_t *pids, int32_t n_req,
                   const double *x, const double *q, int64_t n_pts,
                   void *out, int domain_mode, void *stream);

/* ---- alpha_s (Sec. 2.1, alpha_s paragraph; Fig. 1 py_alphasQ) ---- */

/* out[p] = alpha_s(q2[p]) by 1-D cubic Hermite in ln Q^2 over the alpha_s
 * knots, subgrids split at repeated knots.  q2 device FP64 [n]; out device
 * FP64 (PDFX_F64) or FP32 (PDFX_F32S).  PDFX_ENOALPHAS if the grid has none. */
int pdfx_eval_alphas(const pdfx_grid *g, const double *q2, int64_t n, void *out,
                     int prec, int domain_mode, void *stream);

/* Same with Q instead of Q^2 (Fig. 1 py_alphasQ): Q^2 = Q*Q is formed in FP64
 * on the device, so the result is bit for bit that of pdfx_eval_alphas at the
 * FP64 product Q*Q.  q device FP64 [n], GeV. */
int pdfx_eval_alphasQ(const pdfx_grid *g, const double *q, int64_t n, void *out,
                      int prec, int domain_mode, void *stream);

/* x f and alpha_s at the same points in one call, as an integrand needs both
 * (Sec. 3.1; the examples of Sec. 3.2 and 3.3): the results of pdfx_eval_xfx(g, xf_dev, prec, pids,
 * n_req, x, q2, n_pts, out, domain_mode, stream) and of pdfx_eval_alphas(g,
 * q2, n_pts, as_out, prec, domain_mode, stream): x f bit for bit, alpha_s to
 * rounding (a few ulp), the same NaNs and the same domain counting (a point
 * with Q^2 outside counts once for each).  as_out:
 * device [n_pts], FP64 or FP32 per prec.  domain_mode PDFX_DOMAIN_NAN,
 * PDFX_DOMAIN_CLAMP or PDFX_DOMAIN_ERROR.  When the alpha_s knots are the grid's Q^2 knots (same
 * values, same subgrids), alpha_s is formed in the x f pass from the point's
 * Q^2 weights, one pass over the points instead of two; otherwise the two
 * passes run one after the other.  PDFX_ENOALPHAS if the grid has no alpha_s
 * knots; other errors as pdfx_eval_xfx and as_out NULL or misaligned.
 * Asynchronous on stream. */
int pdfx_eval_xfx_alphas(const pdfx_grid *g, const void *xf_dev, int prec,
                         const int32_t *pids, int32_t n_req,
                         const double *x, const double *q2, int64_t n_pts,
                         void *out, void *as_out, int domain_mode, void *stream);

/* ---- adjoint (derivative of the Sec. 2.1 map; used for differentiable fits) ----
 * For a scalar L with dL/dout = grad_out ([n_pts][n_req], precision's type):
 *  grad_xf  device [n_flav][n_x][n_q] of the precision's type, ACCUMULATED:
 *           grad_xf[f][i][k] += sum_{p,r: row(r)=f} grad_out[p][r] * dout[p][r]/dv[f][i][k];
 *           summed in FP64 on the device, then added; NULL = skip.
 *  grad_x, grad_q2  device FP64 [n_pts], OVERWRITTEN with
 *           sum_r grad_out[p][r] * dout[p][r]/dx (resp. /dQ^2); NULL = skip.
 * Points outside the grid (NaN mode) contribute nothing and get NaN in
 * grad_x/grad_q2; in CLAMP mode the derivative along a clamped axis is 0.
 * On grids of up to 5000 knots the knot gradient is summed per workgroup in
 * 64-bit fixed point (exact, with a power-of-two scale from a bound on the
 * terms that uses max |grad_out| over the workgroup's points: resolution
 * about 2^-43 of that bound at 1e7 points), then added across workgroups
 * with FP64 device atomics, so results are reproducible up to the FP64 order
 * of those sums.  Larger grids sum with FP64 atomics.  Either way a
 * non-finite grad_out value reaches only the knots of its point's stencil
 * (knots i-1 .. i+2 along each axis, cut at the axis ends). */
int pdfx_eval_xfx_backward(const pdfx_grid *g, const void *xf_dev, int prec,
                           const int32_t *pids, int32_t n_req,
                           const double *x, const double *q2, int64_t n_pts,
                           const void *grad_out, void *grad_xf,
                           double *grad_x, double *grad_q2,
                           int domain_mode, void *stream);

/* Bytes of device scratch that pdfx_eval_xfx_backward_noalloc works in. */
#define PDFX_NOALLOC_SCRATCH_BYTES (48u * 1024u * 1024u)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same adjoint
 * as pdfx_eval_xfx_backward, same arguments and results, but its workspace is
 * a fixed device array of PDFX_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends, so the call allocates nothing.  It needs
 * 256-byte-rounded n_pts * (4 + 1 + 4 * 8) bytes plus 8 * n_flav * n_x * n_q
 * plus 8 * 1024 per distinct requested flavour (about 1.3e6 points on an
 * 11 x 100 x 50 grid); a larger call returns
 * PDFX_EINVAL before enqueuing anything.  All calls on one GPU share that
 * array: calls that may overlap on one GPU (other streams or host threads)
 * race, so order them on one stream. */
int pdfx_eval_xfx_backward_noalloc(const pdfx_grid *g, const void *xf_dev, int prec,
                                   const int32_t *pids, int32_t n_req,
                                   const double *x, const double *q2, int64_t n_pts,
                                   const void *grad_out, void *grad_xf,
                                   double *grad_x, double *grad_q2,
                                   int domain_mode, void *stream);

/* ---- many members in one launch (PDF sets are collections of members, Sec. 1) ---- */

/* Loads n_mem members (each desc must carry values; grids may differ). */
int pdfx_load_set(const pdfx_grid_desc *members, int32_t n_mem, pdfx_set **out);
void pdfx_free_set(pdfx_set *s);

/* out[m][p][r] = x f^{(m)}_{pids[r]}(x[p], q2[p]) for every member m.  x, q2
 * device FP64 [n_pts] shared by all members; out device [n_mem][n_pts][n_req]
 * FP64 or FP32 by precision.  Every member evaluates in one persistent launch
 * (after a one-thread kernel that resets its work-list cursor) that walks a
 * single list of (member, run of point tiles) items, the members of the
 * dearest node-width classes first; each item runs its member's class.  A
 * member too large for every class (beyond about 19k knots in FP64) is
 * evaluated by a second, single-slab launch, and so is every member when
 * `out` or the member blocks are not 16-byte aligned or the request touches
 * more flavour groups than a class holds results for. */
int pdfx_eval_set_xfx(const pdfx_set *s, int prec, const int32_t *pids, int32_t n_req,
                      const double *x, const double *q2, int64_t n_pts,
                      void *out, int domain_mode, void *stream);

/* ---- Monte Carlo luminosity integrand (Sec. 3.1, Eq. 1 with a unit matrix element) ----
 * Per point p: x_j = exp(ln xmin + u_j[p] ln(1/xmin)) for j = 1,2;
 * Q^2 = x1 x2 s clipped to the grid's Q^2 range;
 * I[p] = (ln(1/xmin))^2 alpha_s(Q^2) sum_{q=1..5} xf_q(x1) xf_{-q}(x2),
 * the log-map Jacobian x1 x2 (ln(1/xmin))^2 cancelling the 1/(x1 x2) of f = xf/x.
 *  u1, u2   device FP64 [n] in [0,1).
 *  out      device [n] FP64 or FP32 by precision (NULL = skip).
 *  block_sums device FP64 [*n_blocks] partial sums of I (NULL = skip); the
 *           call writes the number of partial sums it produces to *n_blocks
 *           if n_blocks is non-NULL (query with n = 0 first to size it:
 *           it is at most pdfx_dy_max_blocks()).
 * Requires the grid's alpha_s knots and owned values (or xf_dev). */
int pdfx_eval_dy(const pdfx_grid *g, const void *xf_dev, int prec,
                 const double *u1, const double *u2, int64_t n,
                 double xmin, double s, void *out, double *block_sums,
                 int32_t *n_blocks, void *stream);
int32_t pdfx_dy_max_blocks(void);

/* Backward of sum_p I[p] with respect to the PDF knot values:
 * grad_xf (device [n_flav][n_x][n_q], precision's type) += d(sum_p I[p]) / dv,
 * scaled by `scale` (e.g. 1/n for a mean).  alpha_s knots are not differentiated.
 * With the 11 partons in the standard order the knot sums are kept in 64-bit
 * fixed point per workgroup (as for pdfx_eval_xfx_backward), and a non-finite
 * scale or value makes the quark and antiquark rows NaN; otherwise they are
 * FP64 atomics. */
int pdfx_eval_dy_backward(const pdfx_grid *g, const void *xf_dev, int prec,
                          const double *u1, const double *u2, int64_t n,
                          double xmin, double s, double scale, void *grad_xf,
                          void *stream);

/* ---- launch tuning ---- */

/* Times the compiled launch shapes of pdfx_eval_xfx (prec, n_req, n_pts) on
 * scratch buffers and keeps the fastest for this grid; with a non-NULL path
 * the choice is also stored in / read from a JSON cache keyed by device,
 * compute-unit count, grid signature, precision and size class.  Synchronous. */
int pdfx_autotune(pdfx_grid *g, int prec, int32_t n_req, int64_t n_pts, const char *cache_path);
int pdfx_autotune_set(pdfx_set *s, int prec, int32_t n_req, int64_t n_pts, const char *cache_path);

/* Current launch shape of a grid: workgroup size and points per thread.
 * A default or tuned shape with ppt > 1 gives way to (512, 1) in a forward
 * call whose points fill fewer workgroups than half the compute units (e.g.
 * 1e5 points): smaller tiles keep more compute units busy.  A shape set by
 * pdfx_set_launch is used at every size. */
int pdfx_get_launch(const pdfx_grid *g, int prec, int32_t *block, int32_t *ppt);
/* Forces a launch shape (must be one of the compiled ones): ppt > 0 holds
 * results in registers ((256, 2), (256, 4), (512, 1), (512, 2), (1024, 1),
 * and for PDFX_F32S also (512, 4), which only the double-buffered kernel has:
 * other FP32 kernels run it as (512, 2)); ppt < 0 stores results as they are
 * produced ((256, -2), (256, -4), (256, -8), (512, -1), (512, -2), (512, -4),
 * (1024, -1), (1024, -2)). */
int pdfx_set_launch(pdfx_grid *g, int prec, int32_t block, int32_t ppt);

/* Launch shape of the double-buffered integrand kernel (pdfx_eval_dy on
 * grids with the 11 partons in the standard order that fit its LDS):
 * workgroup size and points per thread; compiled: (512, 1), (512, 2),
 * (256, 2), and (512, 4) for PDFX_F32S.  Other grids use a fixed single-slab
 * kernel. */
int pdfx_get_dy_launch(const pdfx_grid *g, int prec, int32_t *block, int32_t *ppt);
int pdfx_set_dy_launch(pdfx_grid *g, int prec, int32_t block, int32_t ppt);

/* ---- flavour-pair luminosity (Eq. 1; the single-top example of Fig. 4) ---- */

/* For pairs k = 0 .. n_pair-1 of partons (pid_a[k] at x1, pid_b[k] at x2):
 *   L_k(p) = f_{pid_a[k]}(x1[p], Q2_p) * f_{pid_b[k]}(x2[p], Q2_p),  f = xf / x,
 *   S(p)   = sum_k coef[k] * L_k(p)        (coef NULL: every c_k = 1),
 * with Q2_p = q2[p], or q2_fixed for every point when q2 is NULL.  This is
 * the luminosity an integrand multiplies by its matrix elements; per-pair L
 * lets the caller weight each pair per point.
 * g: a grid that fits the double-buffered kernel (n_x, n_q >= 4, at most 5000
 * knots); xf_dev: caller values [n_flav][n_x][n_q] of the precision, or NULL
 * for the owned ones.  pid_a, pid_b, coef: host arrays of n_pair (1 .. 128).
 * x1, x2, q2: device FP64 [n]; out_pair: device [n][n_pair] or NULL; out_sum:
 * device [n] or NULL (not both NULL when n > 0); outputs FP64 or FP32 by
 * precision.
 * A pair with a parton absent from the grid gives 0.  A point with x1, x2 or
 * Q2 outside the grid gives NaN in NAN mode (and is counted), or is evaluated
 * at the clamped point in CLAMP mode (f = xf / x at the clamped x).  The pairs
 * may touch at most 6 flavour groups in FP64 (2 partons each in grid order)
 * and 3 in FP32 (4 each): every pair of an 11-parton grid qualifies.
 * Asynchronous on stream. */
int pdfx_eval_lumi(const pdfx_grid *g, const void *xf_dev, int prec, int32_t n_pair,
                   const int32_t *pid_a, const int32_t *pid_b, const double *coef,
                   const double *x1, const double *x2, const double *q2, double q2_fixed,
                   int64_t n, void *out_pair, void *out_sum, int domain_mode, void *stream);

/* Launch shape of the luminosity kernel per precision (default (512, 2));
 * compiled: (512, 1), (512, 2), (256, 2), and (512, 4) for PDFX_F32S.  As for
 * pdfx_get_launch, the default gives way to (512, 1) in a call too small to
 * give half the compute units a tile; a shape set here is used at every size. */
int pdfx_get_lumi_launch(const pdfx_grid *g, int prec, int32_t *block, int32_t *ppt);
int pdfx_set_lumi_launch(pdfx_grid *g, int prec, int32_t block, int32_t ppt);

/* ---- diagnostics ---- */

/* Number of out-of-grid points counted since the last call, over all eval
 * calls on g; synchronises the device, then resets the counter. */
int pdfx_domain_errors(const pdfx_grid *g, int64_t *count);

/* The same for the evaluations of a set (pdfx_eval_set_xfx counts a point
 * once per member whose grid it is outside). */
int pdfx_set_domain_errors(const pdfx_set *s, int64_t *count);

/* Host-side domain check with the rule of the eval calls (Sec. 2.1 queries
 * live inside the grid): counts the points of host arrays x[n], q2[n] (FP64,
 * Q^2 in GeV^2) outside [x_0, x_last] x [q2_0, q2_last] of the grid that d
 * describes, NaN included, into *n_outside (may be NULL).  Returns
 * PDFX_EDOMAIN if there is one, PDFX_OK if there is none, PDFX_EINVAL for an
 * invalid descriptor (the pdfx_load_grid rules; values may be absent) or
 * NULL arrays with n > 0.  Touches no device: callers use it to vet inputs
 * before uploading them. */
int pdfx_check_points(const pdfx_grid_desc *d, const double *x, const double *q2, int64_t n,
                      int64_t *n_outside);

/* Measurement helper, not part of the method: the device's rate of aligned
 * 16-byte LDS reads, the ceiling of the stencil kernels (their stencils are
 * such reads at data-dependent addresses), and of 64-bit LDS atomic adds, the
 * ceiling of the gradient scatters.  Enqueues `blocks` workgroups of 256
 * threads; each thread makes `iters` operations on a 64 KB LDS array:
 * 16-byte reads, lane-consecutive (mode 0: each wave reads 1 KB in one
 * piece) or at independent random 16-byte-aligned addresses (mode 1); FP64
 * atomic adds, lane-consecutive (mode 2) or at random 8-byte-aligned
 * addresses (mode 3); 64-bit integer atomic adds, the same two ways (modes 4,
 * 5).  Operations per call = blocks * 256 * iters; the caller
 * times the call on `stream`.  `sink`: device, blocks * 256 doubles, receives
 * per-thread values so that the work is kept.  PDFX_EINVAL for another mode,
 * blocks or iters <= 0, or a NULL sink.  Asynchronous on stream. */
int pdfx_bench_lds(int mode, int blocks, int iters, double *sink, void *stream);

/* Message for the last failed call on this thread ("" if none). */
const char *pdfx_last_error(void);

/* Library version string. */
const char *pdfx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PDFX_H */
