// Fused LO Drell-Yan-like Monte Carlo integrand (the luminosity part of the
// cross-section integral, Sec. 3.1 Eq. 1, with a unit matrix element) and its
// gradient with respect to the PDF knot values.
//
// Per point p, from two uniforms u1, u2 in [0, 1):
//   x_j = exp(ln xmin + u_j ln(1/xmin)),  Q^2 = clip(x1 x2 s, Q^2_min, Q^2_max),
//   I_p = (ln(1/xmin))^2 alpha_s(Q^2) sum_{q=1..5} xf_q(x1, Q^2) xf_{-q}(x2, Q^2),
// the log-map Jacobian x1 x2 (ln(1/xmin))^2 cancelling the 1/(x1 x2) that turns
// x f into f.
//
// Forward: one persistent kernel.  The per-point state covers both momentum
// fractions (two x bins and weight sets) and the shared Q^2 (one bin, one
// weight set) plus alpha_s (1-D Hermite from LDS tables).  The ten flavour
// slabs are walked in the order q, -q for q = 1..5 with the forward kernel's
// double-buffered staging; the quark value is held in a register until its
// antiquark partner is evaluated.  Each workgroup keeps an FP64 partial sum of
// its I_p and writes it once.
//
// Backward: a state pass (bins, FP64 local coordinates, alpha_s per point),
// then one workgroup per (point chunk, flavour) stages the partner flavour's
// value slab, forms scale * L^2 alpha_s * partner value, and scatters it times
// the flavour's own stencil weights into an FP64 gradient slab in LDS, which
// is added to an FP64 accumulator at the end.
#include "xfx_fwd_impl.h"

namespace pdfx {

namespace {

template <typename V, int BLOCK, int PPT, int PF, bool DB>
__global__ __launch_bounds__(BLOCK) void dy_kernel(const DyArgs a)
{
    extern __shared__ uint4 smem4[];
    char *sm = reinterpret_cast<char *>(smem4);
    const int tid = threadIdx.x;
    constexpr bool F32 = sizeof(V) == 4;

    fwd::load_axis<BLOCK>(sm, a.ax, a.lx, F32);
    fwd::load_axis<BLOCK>(sm, a.aq, a.lq, F32);
    fwd::load_axis<BLOCK>(sm, a.aa, a.la, F32);
    fwd::copy_words<BLOCK>(sm + a.lds_asv, a.as_vals, ((a.aa.n + 2) * (int)sizeof(V) + 7) / 8 * 8);
    const fwd::LAxis lx = fwd::lds_axis(sm, a.ax, a.lx);
    const fwd::LAxis lq = fwd::lds_axis(sm, a.aq, a.lq);
    const fwd::LAxis la = fwd::lds_axis(sm, a.aa, a.la);
    const V *asv = reinterpret_cast<const V *>(sm + a.lds_asv);

    const int nqp = a.nq + 2;
    const int schunks = a.slab_elems * (int)sizeof(V) / 16;
    const uint4 *gv = reinterpret_cast<const uint4 *>(a.vals);
    uint4 *const buf0 = reinterpret_cast<uint4 *>(sm + a.lds_slab0);
    uint4 *const buf1 = reinterpret_cast<uint4 *>(sm + a.lds_slab1);
    V *out = reinterpret_cast<V *>(a.out);
    const int n_seq = a.n_seq;
    const int64_t tile_pts = (int64_t)BLOCK * PPT;
    const int64_t ntiles = (a.n + tile_pts - 1) / tile_pts;

    uint4 pf[DB ? PF : 1];
#pragma unroll
    for (int i = 0; i < (DB ? PF : 1); ++i)
        pf[i] = make_uint4(0u, 0u, 0u, 0u);

    int cur = 0, staged = -1;
    if (n_seq > 0 && (DB || n_seq == 1)) {
        fwd::stage_sync<BLOCK>(buf0, gv + (size_t)a.seq_row[0] * schunks, schunks);
        staged = a.seq_row[0];
    }
    __syncthreads();

    double part = 0.0;   // this thread's FP64 partial sum of I
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t p0 = tile * tile_pts + tid;
        V w1[PPT][4], w2[PPT][4], wq[PPT][4];
        int b1[PPT], b2[PPT];
        bool ok[PPT], live[PPT];
        V as[PPT], lum[PPT], held[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int64_t p = p0 + (int64_t)j * BLOCK;
            live[j] = p < a.n;
            const double ua = live[j] ? a.u1[p] : 0.5;
            const double ub = live[j] ? a.u2[p] : 0.5;
            const double l1 = a.lnxmin + ua * a.lnrange;
            const double l2 = a.lnxmin + ub * a.lnrange;
            double x1 = exp(l1), x2 = exp(l2);
            double q2 = x1 * x2 * a.s;
            q2 = q2 < a.aq.lo ? a.aq.lo : (q2 > a.aq.hi ? a.aq.hi : q2);
            ok[j] = x1 >= a.ax.lo && x1 <= a.ax.hi && x2 >= a.ax.lo && x2 <= a.ax.hi &&
                    q2 >= a.aa.lo && q2 <= a.aa.hi;
            fwd::count_flagged(live[j] && !ok[j], a.dom_count);
            // ln x is the exponent itself (the bins compare raw x, so a last-bit
            // difference from log(x) cannot change them)
            double lnx1 = l1, lnx2 = l2;
            if (!ok[j]) {
                x1 = x2 = a.ax.lo;
                lnx1 = lnx2 = a.ax.ln_lo;
                q2 = a.aq.lo > a.aa.lo ? a.aq.lo : a.aa.lo;
            }
            const double lnq = log(q2);
            const int i1 = fwd::lbin(lx, x1, lnx1);
            const int i2 = fwd::lbin(lx, x2, lnx2);
            const int kq = fwd::lbin(lq, q2, lnq);
            fwd::weights<V>(lx, i1, lnx1, w1[j]);
            fwd::weights<V>(lx, i2, lnx2, w2[j]);
            fwd::weights<V>(lq, kq, lnq, wq[j]);
            b1[j] = i1 * nqp + kq;
            b2[j] = i2 * nqp + kq;
            const int ka = fwd::lbin(la, q2, lnq);
            V wa[4];
            fwd::weights<V>(la, ka, lnq, wa);
            V av = wa[0] * asv[ka];
            av = fma(wa[1], asv[ka + 1], av);
            av = fma(wa[2], asv[ka + 2], av);
            av = fma(wa[3], asv[ka + 3], av);
            as[j] = av;
            lum[j] = V(0);
            held[j] = V(0);
        }

        for (int f = 0; f < n_seq; ++f) {
            const int row = a.seq_row[f];
            const bool quark = (f & 1) == 0;   // sequence is q, -q, q', -q', ...
            bool pre = false;
            if (DB) {
                pre = n_seq > 1 && (f + 1 < n_seq || tile + gridDim.x < ntiles);
                if (pre) {
                    const uint4 *src = gv + (size_t)a.seq_row[f + 1 < n_seq ? f + 1 : 0] * schunks;
#pragma unroll
                    for (int i = 0; i < PF; ++i) {
                        const int c = tid + i * BLOCK;
                        pf[i] = src[c < schunks ? c : schunks - 1];
                    }
                }
            } else if (row != staged) {
                __syncthreads();
                fwd::stage_sync<BLOCK>(buf0, gv + (size_t)row * schunks, schunks);
                __syncthreads();
                staged = row;
            }
            const V *slab = reinterpret_cast<const V *>(cur ? buf1 : buf0);
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const V *s0 = slab + (quark ? b1[j] : b2[j]);
                const V *wx = quark ? w1[j] : w2[j];
                V acc;
#pragma unroll
                for (int jx = 0; jx < 4; ++jx) {
                    const V *s = s0 + jx * nqp;
                    V r = wq[j][0] * s[0];
                    r = fma(wq[j][1], s[1], r);
                    r = fma(wq[j][2], s[2], r);
                    r = fma(wq[j][3], s[3], r);
                    acc = (jx == 0) ? wx[0] * r : fma(wx[jx], r, acc);
                }
                if (quark)
                    held[j] = acc;
                else
                    lum[j] = fma(held[j], acc, lum[j]);
            }
            if (DB && pre) {
                uint4 *dst = cur ? buf0 : buf1;
#pragma unroll
                for (int i = 0; i < PF; ++i) {
                    const int c = tid + i * BLOCK;
                    if (c < schunks)
                        dst[c] = pf[i];
                }
                __syncthreads();
                cur ^= 1;
            }
        }
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            if (!live[j])
                continue;
            const V I = (V)a.L2 * as[j] * lum[j];
            const int64_t p = p0 + (int64_t)j * BLOCK;
            if (out)
                out[p] = ok[j] ? I : fwd::quiet_nan<V>();
            part += ok[j] ? (double)I : __builtin_nan("");
        }
    }

    // workgroup sum of the partial sums (fixed order: deterministic)
    __syncthreads();
    double *red = reinterpret_cast<double *>(sm + a.lds_slab0);
    red[tid] = part;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (tid < w)
            red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0 && a.block_sums)
        a.block_sums[blockIdx.x] = red[0];
}

// ---- backward ----

__global__ __launch_bounds__(256) void dy_state_kernel(const DyArgs a)
{
    extern __shared__ uint4 smem4[];
    char *sm = reinterpret_cast<char *>(smem4);
    fwd::load_axis<256>(sm, a.ax, a.lx, false);
    fwd::load_axis<256>(sm, a.aq, a.lq, false);
    fwd::load_axis<256>(sm, a.aa, a.la, false);
    fwd::copy_words<256>(sm + a.lds_asv, a.as_vals64, (a.aa.n + 2) * 8);
    __syncthreads();
    const fwd::LAxis lx = fwd::lds_axis(sm, a.ax, a.lx);
    const fwd::LAxis lq = fwd::lds_axis(sm, a.aq, a.lq);
    const fwd::LAxis la = fwd::lds_axis(sm, a.aa, a.la);
    const double *asv = reinterpret_cast<const double *>(sm + a.lds_asv);
    // each thread's next point's uniforms are loaded one iteration ahead
    // (clamped to the last point), so that no iteration waits for its own
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t p0 = p < a.n ? p : a.n - 1;   // launched with n > 0 only
    double u1n = a.u1[p0], u2n = a.u2[p0];
    for (; p < a.n; p += stride) {
        const double u1 = u1n, u2 = u2n;
        const int64_t pn = p + stride < a.n ? p + stride : a.n - 1;
        u1n = a.u1[pn];
        u2n = a.u2[pn];
        // ln x is the exponent itself (the bins compare raw x, so a last-bit
        // difference from log(x) cannot change them)
        double lnx1 = a.lnxmin + u1 * a.lnrange;
        double lnx2 = a.lnxmin + u2 * a.lnrange;
        double x1 = exp(lnx1);
        double x2 = exp(lnx2);
        double q2 = x1 * x2 * a.s;
        q2 = q2 < a.aq.lo ? a.aq.lo : (q2 > a.aq.hi ? a.aq.hi : q2);
        const bool ok = x1 >= a.ax.lo && x1 <= a.ax.hi && x2 >= a.ax.lo && x2 <= a.ax.hi &&
                        q2 >= a.aa.lo && q2 <= a.aa.hi;
        if (!ok) {
            x1 = x2 = a.ax.lo;
            lnx1 = lnx2 = a.ax.ln_lo;
            q2 = a.aq.lo > a.aa.lo ? a.aq.lo : a.aa.lo;
        }
        const double lnq = log(q2);
        const int i1 = fwd::lbin(lx, x1, lnx1);
        const int i2 = fwd::lbin(lx, x2, lnx2);
        const int kq = fwd::lbin(lq, q2, lnq);
        const int ka = fwd::lbin(la, q2, lnq);
        double wa[4];
        fwd::weights<double>(la, ka, lnq, wa);
        double av = wa[0] * asv[ka];
        av = fma(wa[1], asv[ka + 1], av);
        av = fma(wa[2], asv[ka + 2], av);
        av = fma(wa[3], asv[ka + 3], av);
        a.st_i1[p] = ok ? (i1 | (kq << 16)) : -1;
        a.st_i2[p] = i2;
        a.st_t1[p] = (lnx1 - lx.r64[i1].z) * lx.r64[i1].inv_d;
        a.st_t2[p] = (lnx2 - lx.r64[i2].z) * lx.r64[i2].inv_d;
        a.st_tq[p] = (lnq - lq.r64[kq].z) * lq.r64[kq].inv_d;
        a.st_as[p] = av;
    }
}

__device__ __forceinline__ void fold64(double t, const IntervalRec<double> &r, double w[4])
{
    fwd::fold<double>(t, r.pl, r.plql, r.ql, r.qr, r.qrpr, r.pr, w);
}

template <typename V>
__global__ __launch_bounds__(256) void dy_adjoint_kernel(const DyArgs a)
{
    extern __shared__ uint4 smem4[];
    char *sm = reinterpret_cast<char *>(smem4);
    const int f = blockIdx.y;                 // position in the q, -q sequence
    const int own = a.seq_row[f];
    const int partner = a.seq_row[f ^ 1];
    const bool quark = (f & 1) == 0;          // own flavour sits at x1 if a quark
    const int nqp = a.nq + 2;
    const int slab_n = (a.nx + 2) * nqp;
    const IntervalRec<double> *rx = reinterpret_cast<const IntervalRec<double> *>(sm + a.lds_recx);
    const IntervalRec<double> *rq = reinterpret_cast<const IntervalRec<double> *>(sm + a.lds_recq);
    double *lgrad = reinterpret_cast<double *>(sm + a.lds_grad);
    V *lval = reinterpret_cast<V *>(sm + a.lds_slab0);
    fwd::copy_words<256>(sm + a.lds_recx, a.ax.rec64, (a.ax.n - 1) * 64);
    fwd::copy_words<256>(sm + a.lds_recq, a.aq.rec64, (a.aq.n - 1) * 64);
    for (int e = threadIdx.x; e < slab_n; e += 256)
        lgrad[e] = 0.0;
    fwd::stage_sync<256>(reinterpret_cast<uint4 *>(lval),
                         reinterpret_cast<const uint4 *>(a.vals) +
                             (size_t)partner * (a.slab_elems * sizeof(V) / 16),
                         a.slab_elems * (int)sizeof(V) / 16);
    __syncthreads();
    const int64_t p_begin = (int64_t)blockIdx.x * a.chunk;
    const int64_t p_end = p_begin + a.chunk < a.n ? p_begin + a.chunk : a.n;
    for (int64_t p = p_begin + threadIdx.x; p < p_end; p += 256) {
        const int idx1 = a.st_i1[p];
        if (idx1 < 0)
            continue;
        const int i1 = idx1 & 0xffff, kq = idx1 >> 16, i2 = a.st_i2[p];
        double w1[4], w2[4], wq[4];
        fold64(a.st_t1[p], rx[i1], w1);
        fold64(a.st_t2[p], rx[i2], w2);
        fold64(a.st_tq[p], rq[kq], wq);
        const double *wp = quark ? w2 : w1;   // partner's x weights
        const double *wo = quark ? w1 : w2;   // own x weights
        const int bp = (quark ? i2 : i1) * nqp + kq;
        const int bo = (quark ? i1 : i2) * nqp + kq;
        double pv = 0.0;
#pragma unroll
        for (int jx = 0; jx < 4; ++jx) {
            const V *s = lval + bp + jx * nqp;
            double r = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                r = fma(wq[k], (double)s[k], r);
            pv = fma(wp[jx], r, pv);
        }
        const double mult = a.scale * a.L2 * a.st_as[p] * pv;
#pragma unroll
        for (int jx = 0; jx < 4; ++jx) {
            const double m = mult * wo[jx];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                atomicAdd(&lgrad[bo + jx * nqp + k], m * wq[k]);
        }
    }
    __syncthreads();
    double *dst = a.gacc + (size_t)own * a.nx * a.nq;
    for (int e = threadIdx.x; e < a.nx * a.nq; e += 256) {
        const int i = e / a.nq, k = e - i * a.nq;
        const double v = lgrad[(i + 1) * nqp + (k + 1)];
        if (v != 0.0)
            unsafeAtomicAdd(&dst[e], v);
    }
}

__global__ __launch_bounds__(256) void dy_zero(double *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = 0.0;
}

template <typename V>
__global__ __launch_bounds__(256) void dy_finish(const double *gacc, V *grad, int64_t nv)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nv; e += (int64_t)gridDim.x * 256)
        grad[e] = (V)((double)grad[e] + gacc[e]);
}

template <typename V>
hipError_t dy_forward_typed(const DyArgs &a, bool db, size_t lds, int cus, hipStream_t s,
                            int *grid_out)
{
    constexpr int BLOCK = 512, PPT = 1;
    const int schunks = a.slab_elems * (int)sizeof(V) / 16;
    auto go = [&](auto fn) -> hipError_t {
        if (lds > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
            if (e != hipSuccess)
                return e;
        }
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(fn), BLOCK, lds);
        if (e != hipSuccess || per_cu < 1)
            per_cu = 1;
        const int64_t ntiles = (a.n + BLOCK * PPT - 1) / (BLOCK * PPT);
        int64_t grid = (int64_t)per_cu * cus;
        if (grid > kDyMaxBlocks)
            grid = kDyMaxBlocks;
        if (grid > ntiles)
            grid = ntiles;
        if (grid < 1)
            grid = 1;
        *grid_out = (int)grid;
        hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(BLOCK), lds, s, a);
        return hipGetLastError();
    };
    if (!db)
        return go(dy_kernel<V, BLOCK, PPT, 1, false>);
    switch (fwd::pick_pf(BLOCK, schunks)) {
    case 4: return go(dy_kernel<V, BLOCK, PPT, 4, true>);
    case 8: return go(dy_kernel<V, BLOCK, PPT, 8, true>);
    case 12: return go(dy_kernel<V, BLOCK, PPT, 12, true>);
    default: return go(dy_kernel<V, BLOCK, PPT, 1, false>);
    }
}

int blocks_for(int64_t n, int cap)
{
    int64_t b = (n + 255) / 256;
    if (b > cap)
        b = cap;
    return b < 1 ? 1 : (int)b;
}

}  // namespace

// LDS layout shared by the forward kernel: tables of x, Q^2, alpha_s axes, the
// alpha_s values, then one or two slabs.  Returns 0 if one slab does not fit.
size_t dy_lds_layout(DyArgs &a, bool f32, bool *db)
{
    size_t off = 0;
    auto take = [&](size_t bytes, size_t align) {
        off = (off + align - 1) / align * align;
        const size_t r = off;
        off += bytes;
        return (int)r;
    };
    const AxisDev *axes[3] = {&a.ax, &a.aq, &a.aa};
    AxisLds *lds[3] = {&a.lx, &a.lq, &a.la};
    for (int i = 0; i < 3; ++i) {
        lds[i]->knots = take((size_t)axes[i]->n * 8, 16);
        lds[i]->seed = take((size_t)axes[i]->nbuckets * 2, 16);
        lds[i]->rec64 = take((size_t)(axes[i]->n - 1) * 64, 64);
        lds[i]->rec32 = take(f32 ? (size_t)(axes[i]->n - 1) * 32 : 0, 64);
    }
    a.lds_asv = take((size_t)(a.aa.n + 2) * 8 + 8, 16);
    const size_t slab = (size_t)a.slab_elems * (f32 ? 4 : 8);
    const size_t red = 512 * 8;   // the final reduction reuses slab 0
    a.lds_slab0 = take(slab > red ? slab : red, 16);
    if (off > kLdsLimit)
        return 0;
    if (off + slab <= kLdsLimit) {
        a.lds_slab1 = take(slab, 16);
        *db = true;
    } else {
        a.lds_slab1 = a.lds_slab0;
        *db = false;
    }
    return off;
}

hipError_t launch_dy_forward(const DyArgs &a0, bool f32, int cus, hipStream_t s, int *n_blocks)
{
    DyArgs a = a0;
    bool db = false;
    const size_t lds = dy_lds_layout(a, f32, &db);
    if (lds == 0)
        return hipErrorInvalidValue;
    return f32 ? dy_forward_typed<float>(a, db, lds, cus, s, n_blocks)
               : dy_forward_typed<double>(a, db, lds, cus, s, n_blocks);
}

hipError_t launch_dy_backward(const DyArgs &a0, bool f32, void *grad_xf, int cus, hipStream_t s)
{
    return launch_dy_backward_ex(a0, f32, grad_xf, cus, s, false);
}

// pairs: the knot-gradient pass by quark-antiquark pairs (dy_dma.hip)
hipError_t launch_dy_backward_ex(const DyArgs &a0, bool f32, void *grad_xf, int cus,
                                 hipStream_t s, bool pairs)
{
    DyArgs a = a0;
    hipError_t e;
    size_t off = 0;
    auto take = [&](size_t bytes, size_t align) {
        off = (off + align - 1) / align * align;
        const size_t r = off;
        off += bytes;
        return (int)r;
    };
    // state pass (FP64 tables)
    const AxisDev *axes[3] = {&a.ax, &a.aq, &a.aa};
    AxisLds *lds[3] = {&a.lx, &a.lq, &a.la};
    for (int i = 0; i < 3; ++i) {
        lds[i]->knots = take((size_t)axes[i]->n * 8, 16);
        lds[i]->seed = take((size_t)axes[i]->nbuckets * 2, 16);
        lds[i]->rec64 = take((size_t)(axes[i]->n - 1) * 64, 64);
        lds[i]->rec32 = lds[i]->rec64;
    }
    a.lds_asv = take((size_t)(a.aa.n + 2) * 8, 16);
    if (a.n > 0) {
        hipLaunchKernelGGL(dy_state_kernel, dim3(blocks_for(a.n, 8 * cus)), dim3(256), off, s, a);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    const int64_t nv = (int64_t)a.nf * a.nx * a.nq;
    hipLaunchKernelGGL(dy_zero, dim3(blocks_for(nv, 1024)), dim3(256), 0, s, a.gacc, nv);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if (a.n > 0 && a.n_seq > 0 && pairs) {
        if ((e = launch_dy_pair_adjoint(a, f32, cus, s)) != hipSuccess)
            return e;
    } else if (a.n > 0 && a.n_seq > 0) {
        off = 0;
        a.lds_recx = take((size_t)(a.ax.n - 1) * 64, 64);
        a.lds_recq = take((size_t)(a.aq.n - 1) * 64, 64);
        a.lds_grad = take((size_t)(a.nx + 2) * (a.nq + 2) * 8, 16);
        a.lds_slab0 = take((size_t)a.slab_elems * (f32 ? 4 : 8), 16);
        if (off > kLdsLimit)
            return hipErrorInvalidValue;
        int64_t nchunk = (4LL * cus + a.n_seq - 1) / a.n_seq;
        int64_t chunk = (a.n + nchunk - 1) / nchunk;
        if (chunk < 2048)
            chunk = 2048;
        nchunk = (a.n + chunk - 1) / chunk;
        a.chunk = (int)chunk;
        auto fn = f32 ? dy_adjoint_kernel<float> : dy_adjoint_kernel<double>;
        if (off > 64 * 1024) {
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)off);
            if (e != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL(fn, dim3((unsigned)nchunk, (unsigned)a.n_seq), dim3(256), off, s, a);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    if (f32)
        hipLaunchKernelGGL(dy_finish<float>, dim3(blocks_for(nv, 1024)), dim3(256), 0, s, a.gacc,
                           (float *)grad_xf, nv);
    else
        hipLaunchKernelGGL(dy_finish<double>, dim3(blocks_for(nv, 1024)), dim3(256), 0, s, a.gacc,
                           (double *)grad_xf, nv);
    return hipGetLastError();
}

}  // namespace pdfx
