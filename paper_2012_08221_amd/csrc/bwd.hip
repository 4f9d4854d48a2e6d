// Adjoint of the batched PDF evaluation.
//
// For a scalar L with g[p][r] = dL/dout[p][r]:
//   dL/dv[f][i][k] = sum_{p, r: row(r)=f} g[p][r] * wx_{i}(p) * wq_{k}(p)
//   dL/dx[p]   = (1/x)   sum_r g[p][r] * dxf/dln x,  dL/dQ2[p] = (1/Q2) sum_r g[p][r] * dxf/dln Q2
// where the derivative along an axis uses the derivatives of the Hermite basis,
// folded with the same slope constants as the values (t-derivatives scaled by
// 1/d_i).  The knot gradient does not depend on the values (the map is linear
// in them).
//
// Grids that fit the double-buffered layout take the coordinate pass and the
// knot pass of bwd_coord.hip; the coordinate pass then leaves the per-point
// state itself, and only the finish below runs after them.  The passes here:
//   state:  per point, bins (ix, kq), FP64 local coordinates (tx, tq) and
//           flags; the logs and searches run once per point.  It also zeroes
//           the FP64 knot accumulator.
//   adjoint (larger grids): grid = (point chunk, distinct flavour).  The workgroup rebuilds
//           the FP64 weights and derivative weights from the state, scatters
//           g * wx_j * wq_k into an FP64 gradient slab in LDS (ds_add_f64) and,
//           with the value slab staged in LDS, accumulates g * dxf/dln x and
//           g * dxf/dln Q2 per point (global FP64 atomics, one point per
//           address).  At the end the LDS gradient slab is added to an FP64
//           accumulator in HBM.
//   finish: grad_xf += accumulator (in the caller's precision); grad_x,
//           grad_q2 from the per-point accumulators with the chain rule and
//           the domain rules.
#include "bwd_internal.h"
#include "xfx_fwd_impl.h"

namespace pdfx {

namespace {

constexpr int kStateBlock = 256;
constexpr int kBwdBlock = 256;

__global__ __launch_bounds__(kStateBlock) void state_kernel(const BwdArgs a)
{
    extern __shared__ uint4 smem4[];
    char *sm = reinterpret_cast<char *>(smem4);
    fwd::load_axis<kStateBlock>(sm, a.ax, a.lx, false);
    fwd::load_axis<kStateBlock>(sm, a.aq, a.lq, false);
    __syncthreads();
    const fwd::LAxis lx = fwd::lds_axis(sm, a.ax, a.lx);
    const fwd::LAxis lq = fwd::lds_axis(sm, a.aq, a.lq);
    if (a.gacc) {
        const int64_t nv = (int64_t)a.nf * a.nx * a.nq;
        for (int64_t e = (int64_t)blockIdx.x * kStateBlock + threadIdx.x; e < nv;
             e += (int64_t)gridDim.x * kStateBlock)
            a.gacc[e] = 0.0;
    }
    // each thread's next point is loaded one iteration ahead (clamped to the
    // last point), so that no iteration waits for its own
    const int64_t stride = (int64_t)gridDim.x * kStateBlock;
    int64_t p = (int64_t)blockIdx.x * kStateBlock + threadIdx.x;
    double xn = a.n > 0 ? a.x[p < a.n ? p : a.n - 1] : 0.0;
    double qn = a.n > 0 ? a.q[p < a.n ? p : a.n - 1] : 0.0;
    for (; p < a.n; p += stride) {
        double xv = xn, qv = qn;
        const int64_t pn = p + stride < a.n ? p + stride : a.n - 1;
        xn = a.x[pn];
        qn = a.q[pn];
        uint8_t flag = 0;
        const bool nan_in = (xv != xv) || (qv != qv);
        if (nan_in) {
            flag = kBwdOut;
        } else {
            const bool xin = xv >= a.ax.lo && xv <= a.ax.hi;
            const bool qin = qv >= a.aq.lo && qv <= a.aq.hi;
            if (!(xin && qin)) {
                if (a.domain_mode == 1) {
                    if (!xin)
                        flag |= kBwdXClamp;
                    if (!qin)
                        flag |= kBwdQClamp;
                    xv = fmin(fmax(xv, a.ax.lo), a.ax.hi);
                    qv = fmin(fmax(qv, a.aq.lo), a.aq.hi);
                } else {
                    flag = kBwdOut;
                }
            }
        }
        if (flag & kBwdOut) {
            xv = a.ax.lo;
            qv = a.aq.lo;
        }
        const double lnx = log(xv), lnq = log(qv);
        const int ix = fwd::lbin(lx, xv, lnx);
        const int kq = fwd::lbin(lq, qv, lnq);
        a.st_idx[p] = ix | (kq << 16);
        a.st_flag[p] = flag;
        a.st_tx[p] = (lnx - lx.r64[ix].z) * lx.r64[ix].inv_d;
        a.st_tq[p] = (lnq - lq.r64[kq].z) * lq.r64[kq].inv_d;
    }
}

// Weights and their t-derivatives for one interval record.
__device__ __forceinline__ void fold_both(double t, const IntervalRec<double> &r, double w[4],
                                          double dw[4])
{
    const double t2 = t * t, t3 = t2 * t;
    const double h00 = 2.0 * t3 - 3.0 * t2 + 1.0, h10 = t3 - 2.0 * t2 + t;
    const double h01 = -2.0 * t3 + 3.0 * t2, h11 = t3 - t2;
    const double d00 = 6.0 * t2 - 6.0 * t, d10 = 3.0 * t2 - 4.0 * t + 1.0;
    const double d01 = -6.0 * t2 + 6.0 * t, d11 = 3.0 * t2 - 2.0 * t;
    w[0] = -h10 * r.pl;
    w[1] = h00 + h10 * r.plql - h11 * r.qr;
    w[2] = h01 + h10 * r.ql + h11 * r.qrpr;
    w[3] = h11 * r.pr;
    dw[0] = -d10 * r.pl;
    dw[1] = d00 + d10 * r.plql - d11 * r.qr;
    dw[2] = d01 + d10 * r.ql + d11 * r.qrpr;
    dw[3] = d11 * r.pr;
}

template <typename V>
__global__ __launch_bounds__(kBwdBlock) void adjoint_kernel(const BwdArgs a)
{
    extern __shared__ uint4 smem4[];
    char *sm = reinterpret_cast<char *>(smem4);
    const int u = blockIdx.y;
    const int row = a.urow[u];
    const int nqp = a.nq + 2;
    const int nxp = a.nx + 2;
    const int slab_n = nxp * nqp;
    const IntervalRec<double> *rx = reinterpret_cast<const IntervalRec<double> *>(sm + a.lds_recx);
    const IntervalRec<double> *rq = reinterpret_cast<const IntervalRec<double> *>(sm + a.lds_recq);
    double *lgrad = reinterpret_cast<double *>(sm + a.lds_grad);
    V *lval = reinterpret_cast<V *>(sm + a.lds_slab);
    const bool want_knots = a.gacc != nullptr;
    const bool want_coord = a.accx != nullptr;

    fwd::copy_words<kBwdBlock>(sm + a.lds_recx, a.ax.rec64, (a.ax.n - 1) * 64);
    fwd::copy_words<kBwdBlock>(sm + a.lds_recq, a.aq.rec64, (a.aq.n - 1) * 64);
    if (want_knots)
        for (int e = threadIdx.x; e < slab_n; e += kBwdBlock)
            lgrad[e] = 0.0;
    if (want_coord) {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.vals) +
                           (size_t)row * (a.slab_elems * sizeof(V) / 16);
        fwd::stage_sync<kBwdBlock>(reinterpret_cast<uint4 *>(lval), src,
                                   a.slab_elems * (int)sizeof(V) / 16);
    }
    __syncthreads();

    const int c0 = a.ucol_off[u], c1 = a.ucol_off[u + 1];
    const V *gout = reinterpret_cast<const V *>(a.gout);
    const int64_t p_begin = (int64_t)blockIdx.x * a.chunk;
    const int64_t p_end = p_begin + a.chunk < a.n ? p_begin + a.chunk : a.n;
    for (int64_t p = p_begin + threadIdx.x; p < p_end; p += kBwdBlock) {
        const uint8_t flag = a.st_flag[p];
        if (flag & kBwdOut)
            continue;
        double g = 0.0;
        for (int c = c0; c < c1; ++c)
            g += (double)gout[p * a.n_req + a.ucols[c]];
        const int idx = a.st_idx[p];
        const int ix = idx & 0xffff, kq = idx >> 16;
        double wx[4], dwx[4], wq[4], dwq[4];
        fold_both(a.st_tx[p], rx[ix], wx, dwx);
        fold_both(a.st_tq[p], rq[kq], wq, dwq);
        const int base = ix * nqp + kq;
        if (want_knots) {
#pragma unroll
            for (int jx = 0; jx < 4; ++jx) {
                const double gx = g * wx[jx];
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    atomicAdd(&lgrad[base + jx * nqp + k], gx * wq[k]);
            }
        }
        if (want_coord) {
            double du = 0.0, dw = 0.0;
#pragma unroll
            for (int jx = 0; jx < 4; ++jx) {
                const V *s = lval + base + jx * nqp;
                double r = 0.0, dr = 0.0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const double v = (double)s[k];
                    r = fma(wq[k], v, r);
                    dr = fma(dwq[k], v, dr);
                }
                du = fma(dwx[jx], r, du);
                dw = fma(wx[jx], dr, dw);
            }
            if (!(flag & kBwdXClamp))
                unsafeAtomicAdd(&a.accx[p], g * du * rx[ix].inv_d);
            if (!(flag & kBwdQClamp))
                unsafeAtomicAdd(&a.accw[p], g * dw * rq[kq].inv_d);
        }
    }

    if (want_knots) {
        __syncthreads();
        double *dst = a.gacc + (size_t)row * a.nx * a.nq;
        for (int e = threadIdx.x; e < a.nx * a.nq; e += kBwdBlock) {
            const int i = e / a.nq, k = e - i * a.nq;
            const double v = lgrad[(i + 1) * nqp + (k + 1)];
            if (v != 0.0)
                unsafeAtomicAdd(&dst[e], v);
        }
    }
}

__global__ __launch_bounds__(256) void zero_kernel(double *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = 0.0;
}

template <typename V>
__global__ __launch_bounds__(256) void finish_kernel(const BwdArgs a, void *grad_xf, double *grad_x,
                                                     double *grad_q2)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    const int64_t t0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (grad_xf) {
        V *g = reinterpret_cast<V *>(grad_xf);
        const int64_t nv = (int64_t)a.nf * a.nx * a.nq;
        for (int64_t e = t0; e < nv; e += stride)
            g[e] = (V)((double)g[e] + a.gacc[e]);
    }
    if (grad_x || grad_q2) {
        for (int64_t p = t0; p < a.n; p += stride) {
            const uint8_t flag = a.st_flag[p];
            const bool out = flag & kBwdOut;
            if (grad_x)
                grad_x[p] = out ? __builtin_nan("") : ((flag & kBwdXClamp) ? 0.0 : a.accx[p] / a.x[p]);
            if (grad_q2)
                grad_q2[p] = out ? __builtin_nan("") : ((flag & kBwdQClamp) ? 0.0 : a.accw[p] / a.q[p]);
        }
    }
}

int grid_blocks(int64_t n, int block, int cap)
{
    int64_t b = (n + block - 1) / block;
    if (b > cap)
        b = cap;
    return b < 1 ? 1 : (int)b;
}

}  // namespace

hipError_t launch_backward_ex(const BwdArgs &a0, bool f32, void *grad_xf, double *grad_x,
                              double *grad_q2, int cus, hipStream_t s, bool coords_done)
{
    BwdArgs a = a0;
    hipError_t e;
    // state pass (x and Q^2 tables in LDS); it also zeroes the knot-gradient
    // accumulator
    size_t off = 0;
    auto take = [&](size_t bytes, size_t align) {
        off = (off + align - 1) / align * align;
        const size_t r = off;
        off += bytes;
        return (int)r;
    };
    a.lx.knots = take((size_t)a.ax.n * 8, 16);
    a.lx.seed = take((size_t)a.ax.nbuckets * 2, 16);
    a.lx.rec64 = take((size_t)(a.ax.n - 1) * 64, 64);
    a.lx.rec32 = a.lx.rec64;
    a.lq.knots = take((size_t)a.aq.n * 8, 16);
    a.lq.seed = take((size_t)a.aq.nbuckets * 2, 16);
    a.lq.rec64 = take((size_t)(a.aq.n - 1) * 64, 64);
    a.lq.rec32 = a.lq.rec64;
    const size_t lds_state = off;
    const bool knot_pass = a.n > 0 && a.n_u > 0 && a.gacc && (coords_done || !a.accx) &&
                           knot_grad_supported(a.nx, a.nq);
    if (!coords_done && (a.n > 0 || a.gacc)) {
        // without the coordinate pass the knot pass finds the maxima of
        // |dL/dout| itself
        a.gmax = nullptr;
        hipLaunchKernelGGL(state_kernel, dim3(grid_blocks(a.n, kStateBlock, 8 * cus)),
                           dim3(kStateBlock), lds_state, s, a);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    if (a.accx && a.n > 0 && !coords_done) {
        hipLaunchKernelGGL(zero_kernel, dim3(grid_blocks(a.n, 256, 4 * cus)), dim3(256), 0, s, a.accx, a.n);
        hipLaunchKernelGGL(zero_kernel, dim3(grid_blocks(a.n, 256, 4 * cus)), dim3(256), 0, s, a.accw, a.n);
    }
    // the flavour workgroups skip the coordinate sums when they are done
    BwdArgs ka = a;
    if (coords_done)
        ka.accx = ka.accw = nullptr;
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    // adjoint pass
    if (knot_pass) {
        if ((e = launch_knot_grad(ka, f32, cus, s)) != hipSuccess)
            return e;
    } else if (ka.n > 0 && ka.n_u > 0 && (ka.gacc || ka.accx)) {
        off = 0;
        ka.lds_recx = take((size_t)(ka.ax.n - 1) * 64, 64);
        ka.lds_recq = take((size_t)(ka.aq.n - 1) * 64, 64);
        const size_t slab_n = (size_t)(ka.nx + 2) * (ka.nq + 2);
        ka.lds_grad = take(ka.gacc ? slab_n * 8 : 0, 16);
        ka.lds_slab = take(ka.accx ? (size_t)ka.slab_elems * (f32 ? 4 : 8) : 0, 16);
        const size_t lds = off;
        if (lds > kLdsLimit)
            return hipErrorInvalidValue;
        // about 4 workgroups per compute unit over all (chunk, flavour) pairs
        int64_t nchunk = (4LL * cus + ka.n_u - 1) / ka.n_u;
        int64_t chunk = (ka.n + nchunk - 1) / nchunk;
        if (chunk < 1024)
            chunk = 1024;
        nchunk = (ka.n + chunk - 1) / chunk;
        ka.chunk = (int)chunk;
        auto fn = f32 ? adjoint_kernel<float> : adjoint_kernel<double>;
        if (lds > 64 * 1024) {
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL(fn, dim3((unsigned)nchunk, (unsigned)ka.n_u), dim3(kBwdBlock), lds, s, ka);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    // finish
    if (coords_done) {
        grad_x = grad_q2 = nullptr;
        if (!grad_xf)
            return hipGetLastError();
    }
    const int64_t nv = (int64_t)a.nf * a.nx * a.nq;
    const int64_t work = (grad_x || grad_q2) && a.n > nv ? a.n : nv;
    if (f32)
        hipLaunchKernelGGL(finish_kernel<float>, dim3(grid_blocks(work, 256, 4 * cus)), dim3(256), 0, s,
                           a, grad_xf, grad_x, grad_q2);
    else
        hipLaunchKernelGGL(finish_kernel<double>, dim3(grid_blocks(work, 256, 4 * cus)), dim3(256), 0,
                           s, a, grad_xf, grad_x, grad_q2);
    return hipGetLastError();
}

}  // namespace pdfx
