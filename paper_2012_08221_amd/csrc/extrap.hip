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
// memory, one thread per point: the edge knots' indices come from the host,
// the inside coordinate's bin and weights are found once per point, and each
// column then needs 4-tap sums along knot lines (or knot values at corners).
#include "extrap_internal.h"
#include "xfx_fwd_impl.h"

namespace pdfx {

namespace {

constexpr int kExtrapBlock = 256;

// Bin of v inside the axis: largest i in [0, n-2] with k[i] <= v (a value on
// a repeated knot takes the upper copy), by the forward kernels' seeded search
// over the axis' tables in global memory.
__device__ __forceinline__ int seeded_bin(const AxisDev &ax, double v, double lnv)
{
    fwd::LAxis l;
    l.k = ax.knots;
    l.seed = ax.seed;
    l.r64 = ax.rec64;
    l.r32 = ax.rec32;
    l.n = ax.n;
    l.nb = ax.nbuckets;
    l.ln_lo = ax.ln_lo;
    l.inv_hb = ax.inv_hb;
    return fwd::lbin(l, v, lnv);
}

// Weights of the window of bin i at v.  On a knot they are exactly one-hot,
// as everywhere in this pass: the edge values the continuation starts from
// are the data along a knot line, and an edge value that the data make 0
// (x f at x = 1) is 0, not a rounding residue that would pick the other
// branch of the continuation.
__device__ __forceinline__ void weights64(const AxisDev &ax, int i, double v, double lnv,
                                          double w[4])
{
    if (ax.knots[i] == v || ax.knots[i + 1] == v) {
        const int hot = ax.knots[i] == v ? 1 : 2;
        for (int j = 0; j < 4; ++j)
            w[j] = j == hot ? 1.0 : 0.0;
        return;
    }
    const IntervalRec<double> r = ax.rec64[i];
    const double t = (lnv - r.z) * r.inv_d;
    fwd::fold<double>(t, r.pl, r.plql, r.ql, r.qr, r.qrpr, r.pr, w);
}

__device__ __forceinline__ double cont(double fe, double fn, double u)
{
    const double r = fn / fe;
    if (fe != 0.0 && r > 0.0)
        return fe * exp(u * log(r));
    return fe + u * (fn - fe);
}

// True if a point with coordinates (xv, qv) is outside the grid (and no
// coordinate is NaN: such a point keeps the forward pass's NaN).
__device__ __forceinline__ bool outside(const ExtrapArgs &a, double xv, double qv)
{
    if (a.q_is_q)
        qv = qv * qv;
    if (xv != xv || qv != qv)
        return false;
    return xv < a.ax.lo || xv > a.ax.hi || qv < a.aq.lo || qv > a.aq.hi;
}

// The continuation of one point outside the grid, output column r.
template <typename V>
__device__ void continue_column(const ExtrapArgs &a, int64_t p, int r)
{
    V *out = reinterpret_cast<V *>(a.out);
    const int ld = a.nq + 2;   // bordered slab: knot (i, k) at (i + 1) * ld + k + 1
    {
        const double xv = a.x[p];
        double qv = a.q[p];
        if (a.q_is_q)
            qv = qv * qv;
        const bool xo = xv < a.ax.lo || xv > a.ax.hi;
        const bool qo = qv < a.aq.lo || qv > a.aq.hi;
        const bool xl = xv < a.ax.lo, ql = qv < a.aq.lo;
        // edge knot e and next knot n of each outside axis (knot indices, the
        // tie rule applied), the continuation coordinate u
        const int ie = xl ? a.kx[0] : a.kx[2], in = xl ? a.kx[1] : a.kx[3];
        const int ce = ql ? a.kq[0] : a.kq[2], cn = ql ? a.kq[1] : a.kq[3];
        const double ux = xo ? log(xv / a.ax.knots[ie]) / log(a.ax.knots[in] / a.ax.knots[ie]) : 0.0;
        const double uq = qo ? log(qv / a.aq.knots[ce]) / log(a.aq.knots[cn] / a.aq.knots[ce]) : 0.0;
        // the coordinate inside, if any: its bin and weights, once per point
        double w[4] = {0.0, 0.0, 0.0, 0.0};
        int bin = 0;
        if (!qo) {
            const double lq = log(qv);
            bin = seeded_bin(a.aq, qv, lq);
            weights64(a.aq, bin, qv, lq, w);
        } else if (!xo) {
            const double lx = log(xv);
            bin = seeded_bin(a.ax, xv, lx);
            weights64(a.ax, bin, xv, lx, w);
        }
        V *o = out + p * a.n_req;
        {
            const int row = a.row[r];
            double v = 0.0;
            if (row >= 0) {
                const V *s = reinterpret_cast<const V *>(a.vals) + (size_t)row * a.slab_elems;
                if (xo && !qo) {
                    // along Q^2 on the x knot lines ie and in (window columns bin .. bin+3)
                    const V *re = s + (size_t)(ie + 1) * ld + bin;
                    const V *rn = s + (size_t)(in + 1) * ld + bin;
                    double fe = 0.0, fn = 0.0;
                    for (int k = 0; k < 4; ++k) {
                        fe = fma(w[k], (double)re[k], fe);
                        fn = fma(w[k], (double)rn[k], fn);
                    }
                    v = cont(fe, fn, ux);
                } else if (qo && !xo) {
                    // along x on the Q^2 knot lines ce and cn (window rows bin .. bin+3)
                    double fe = 0.0, fn = 0.0;
                    for (int j = 0; j < 4; ++j) {
                        const V *rj = s + (size_t)(bin + j) * ld;
                        fe = fma(w[j], (double)rj[ce + 1], fe);
                        fn = fma(w[j], (double)rj[cn + 1], fn);
                    }
                    v = cont(fe, fn, uq);
                } else {
                    // corners: knot values; x first, then Q^2
                    const double a_e = cont((double)s[(size_t)(ie + 1) * ld + ce + 1],
                                            (double)s[(size_t)(in + 1) * ld + ce + 1], ux);
                    const double a_n = cont((double)s[(size_t)(ie + 1) * ld + cn + 1],
                                            (double)s[(size_t)(in + 1) * ld + cn + 1], ux);
                    v = cont(a_e, a_n, uq);
                }
            }
            o[r] = (V)v;
        }
    }
}

// Each workgroup takes chunks of kExtrapChunk points: it lists the chunk's
// outside points in LDS, then continues them one (point, column) per lane,
// with every lane busy (outside points are few and scattered, so most waves
// would otherwise run the long path for one lane; each column costs a log
// and an exp, so columns in parallel shorten it further).
constexpr int kExtrapChunk = 4096;
static_assert(kExtrapChunk % kExtrapBlock == 0, "a chunk is whole rounds of the workgroup");

template <typename V>
__global__ __launch_bounds__(kExtrapBlock) void extrap_kernel(const ExtrapArgs a)
{
    __shared__ int list[kExtrapChunk];
    __shared__ int count;
    for (int64_t c0 = (int64_t)blockIdx.x * kExtrapChunk; c0 < a.n;
         c0 += (int64_t)gridDim.x * kExtrapChunk) {
        if (threadIdx.x == 0)
            count = 0;
        __syncthreads();
        // all of the thread's coordinates first, so that their loads overlap
        // (clamped indices keep them global loads)
        constexpr int kPer = kExtrapChunk / kExtrapBlock;
        double xs[kPer], qs[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t p = c0 + threadIdx.x + u * kExtrapBlock;
            xs[u] = load_point(a.x, p, a.n);
            qs[u] = load_point(a.q, p, a.n);
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int i = threadIdx.x + u * kExtrapBlock;
            if (c0 + i < a.n && outside(a, xs[u], qs[u]))
                list[atomicAdd(&count, 1)] = i;
        }
        __syncthreads();
        const int n_out = count;
        for (int k = threadIdx.x; k < n_out * a.n_req; k += kExtrapBlock)
            continue_column<V>(a, c0 + list[k / a.n_req], k % a.n_req);
        __syncthreads();   // the list is read before the next chunk refills it
    }
}

}  // namespace

hipError_t launch_extrap(const ExtrapArgs &a, bool f32, int cus, hipStream_t s)
{
    int64_t grid = (a.n + kExtrapChunk - 1) / kExtrapChunk;   // one chunk per workgroup
    if (grid > (int64_t)cus * 64)
        grid = (int64_t)cus * 64;
    if (grid < 1)
        return hipSuccess;
    if (f32)
        hipLaunchKernelGGL(extrap_kernel<float>, dim3((unsigned)grid), dim3(kExtrapBlock), 0, s, a);
    else
        hipLaunchKernelGGL(extrap_kernel<double>, dim3((unsigned)grid), dim3(kExtrapBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace pdfx
