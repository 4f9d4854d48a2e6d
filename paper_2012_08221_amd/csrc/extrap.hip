// Continuation of x f outside the grid (domain mode EXTRAPOLATE of
// pdfx_eval_xfx).  The interpolation itself only covers the grid (Sec. 2.1
// follows LHAPDF's interpolation); beyond an edge the value continues from the
// edge knot e through the next knot n inward:
//   u = ln(z / z_e) / ln(z_n / z_e)            (u < 0 outside)
//   xf = F_e (F_n / F_e)^u   if F_n / F_e > 0,  else  F_e + u (F_n - F_e),
// where F_e, F_n are the interpolation at the knot coordinates (the other
// coordinate as queried).  Outside in both x and Q^2 the x continuation is
// taken at the two Q^2 edge knots, then continued in Q^2.
//
// The forward kernels run in clamp mode first; this pass then rewrites only
// the rows of points outside the grid.  Such points are expected to be few,
// so each is evaluated straight from the bordered per-parton slabs in global
// memory, one thread per point, with a plain binary search for its bins.
#include "extrap_internal.h"
#include "xfx_fwd_impl.h"

namespace pdfx {

namespace {

constexpr int kExtrapBlock = 256;

// Largest i in [0, n-2] with k[i] <= v (v inside [k[0], k[n-1]]); a value on a
// repeated knot takes the upper copy, as in the forward kernels.
__device__ __forceinline__ int find_bin(const double *k, int n, double v)
{
    int lo = 0, hi = n - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (k[mid] <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Weights of the window of bin i at v.  On a knot they are exactly one-hot:
// the edge values the continuation starts from are then the data along that
// knot line, and an edge value that the data make 0 (x f at x = 1) is 0, not
// a rounding residue that would pick the other branch of the continuation.
__device__ __forceinline__ void weights64(const AxisDev &ax, int i, double v, double w[4])
{
    if (ax.knots[i] == v || ax.knots[i + 1] == v) {
        const int hot = ax.knots[i] == v ? 1 : 2;
        for (int j = 0; j < 4; ++j)
            w[j] = j == hot ? 1.0 : 0.0;
        return;
    }
    const IntervalRec<double> r = ax.rec64[i];
    const double t = (log(v) - r.z) * r.inv_d;
    fwd::fold<double>(t, r.pl, r.plql, r.ql, r.qr, r.qrpr, r.pr, w);
}

// Interpolated x f of grid row `row` at a point inside the grid, from the
// bordered slab (zero border one knot wide), in FP64.
template <typename V>
__device__ double eval_inside(const ExtrapArgs &a, int row, double xv, double qv)
{
    const int ix = find_bin(a.ax.knots, a.nx, xv);
    const int kq = find_bin(a.aq.knots, a.nq, qv);
    double wx[4], wq[4];
    weights64(a.ax, ix, xv, wx);
    weights64(a.aq, kq, qv, wq);
    const V *s = reinterpret_cast<const V *>(a.vals) + (size_t)row * a.slab_elems;
    const int ld = a.nq + 2;
    double acc = 0.0;
    for (int j = 0; j < 4; ++j) {
        const V *r = s + (size_t)(ix + j) * ld + kq;   // bordered row ix-1+j+1, column kq-1+1
        double rr = 0.0;
        for (int k = 0; k < 4; ++k)
            rr = fma(wq[k], (double)r[k], rr);
        acc = fma(wx[j], rr, acc);
    }
    return acc;
}

__device__ __forceinline__ double cont(double fe, double fn, double u)
{
    const double r = fn / fe;
    if (fe != 0.0 && r > 0.0)
        return fe * exp(u * log(r));
    return fe + u * (fn - fe);
}

template <typename V>
__global__ __launch_bounds__(kExtrapBlock) void extrap_kernel(const ExtrapArgs a)
{
    V *out = reinterpret_cast<V *>(a.out);
    const double *kx = a.ax.knots, *kq = a.aq.knots;
    for (int64_t p = (int64_t)blockIdx.x * kExtrapBlock + threadIdx.x; p < a.n;
         p += (int64_t)gridDim.x * kExtrapBlock) {
        const double xv = a.x[p];
        double qv = a.q[p];
        if (a.q_is_q)
            qv = qv * qv;
        if (xv != xv || qv != qv)
            continue;   // NaN input: NaN from the forward pass
        const bool xo = xv < a.ax.lo || xv > a.ax.hi;
        const bool qo = qv < a.aq.lo || qv > a.aq.hi;
        if (!xo && !qo)
            continue;
        const bool xl = xv < a.ax.lo, ql = qv < a.aq.lo;
        const double xe = xl ? kx[0] : kx[a.nx - 1], xn = xl ? kx[1] : kx[a.nx - 2];
        const double qe = ql ? kq[0] : kq[a.nq - 1], qn = ql ? kq[1] : kq[a.nq - 2];
        const double ux = xo ? log(xv / xe) / log(xn / xe) : 0.0;
        const double uq = qo ? log(qv / qe) / log(qn / qe) : 0.0;
        V *o = out + p * a.n_req;
        for (int r = 0; r < a.n_req; ++r) {
            const int row = a.row[r];
            double v = 0.0;
            if (row >= 0) {
                if (xo && !qo) {
                    v = cont(eval_inside<V>(a, row, xe, qv), eval_inside<V>(a, row, xn, qv), ux);
                } else if (qo && !xo) {
                    v = cont(eval_inside<V>(a, row, xv, qe), eval_inside<V>(a, row, xv, qn), uq);
                } else {
                    const double ce = cont(eval_inside<V>(a, row, xe, qe),
                                           eval_inside<V>(a, row, xn, qe), ux);
                    const double cn = cont(eval_inside<V>(a, row, xe, qn),
                                           eval_inside<V>(a, row, xn, qn), ux);
                    v = cont(ce, cn, uq);
                }
            }
            o[r] = (V)v;
        }
    }
}

}  // namespace

hipError_t launch_extrap(const ExtrapArgs &a, bool f32, int cus, hipStream_t s)
{
    int64_t grid = (a.n + kExtrapBlock - 1) / kExtrapBlock;
    if (grid > (int64_t)cus * 8)
        grid = (int64_t)cus * 8;
    if (grid < 1)
        return hipSuccess;
    if (f32)
        hipLaunchKernelGGL(extrap_kernel<float>, dim3((unsigned)grid), dim3(kExtrapBlock), 0, s, a);
    else
        hipLaunchKernelGGL(extrap_kernel<double>, dim3((unsigned)grid), dim3(kExtrapBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace pdfx
