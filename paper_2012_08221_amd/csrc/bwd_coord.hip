// Coordinate part of the adjoint of the batched evaluation: for every point,
//   dL/dln x   = sum_r g[p][r] * sum_{i,k} dwx_i wq_k v_r[i][k] / d_x,
//   dL/dln Q^2 = sum_r g[p][r] * sum_{i,k} wx_i dwq_k v_r[i][k] / d_q,
// with dw the t-derivatives of the folded Hermite weights and d the interval
// widths in ln x, ln Q^2 (Sec. 2.1's interpolant differentiated along each
// axis).  Structured like the double-buffered forward kernel: the request's
// flavour groups are staged two slabs deep by global-to-LDS copies, each
// thread holds its point's weights, derivative weights and dL/dout values,
// and the two sums are accumulated in registers and written once per point,
// instead of one global atomic per point and flavour, already divided by x
// and Q^2 with the domain rules applied.  The pass also leaves the per-point
// state (bins, local coordinates, flags) for the knot pass below, so that the
// points are located once.  Arithmetic in FP64 whatever the values' precision.
#include "bwd_internal.h"
#include "xfx_dma_impl.h"
#include "fixed_point.h"

namespace pdfx {

namespace {

using fwd::kDmaKnots;
using fwd::kDmaNodes;
using fwd::kDmaSeeds;

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

// Window of interval i on an axis of n >= 4 knots (fwd::window), moving both
// the weights and their derivatives.
__device__ __forceinline__ int window2(int i, int n, double w[4], double dw[4])
{
    double tmp[4] = {dw[0], dw[1], dw[2], dw[3]};
    const int st = fwd::window(i, n, w);
    fwd::window(i, n, tmp);
    for (int m = 0; m < 4; ++m)
        dw[m] = tmp[m];
    return st;
}

template <typename V, int BLOCK>
__global__ __launch_bounds__(BLOCK) void coord_grad_kernel(const CoordArgs c)
{
    constexpr int G = 16 / (int)sizeof(V);
    constexpr int NS = kGrpMaxSlots / G;
    constexpr int NSG = NS * G;
    __shared__ uint4 slab0[kDmaNodes];
    __shared__ uint4 slab1[kDmaNodes];
    __shared__ double knots[kDmaKnots];
    __shared__ uint16_t seeds[kDmaSeeds];
    const XfxArgs &a = c.x;
    const int tid = threadIdx.x;
    const int nx = a.nx, nq = a.nq;
    const int nodes = nx * nq;
    const uint4 *gsrc = reinterpret_cast<const uint4 *>(a.gvals);
    const V *gout = reinterpret_cast<const V *>(c.gout);
    const int n_req = a.n_req;
    const int n_stage = a.n_stage;
    const int64_t ntiles = (a.n + BLOCK - 1) / BLOCK;
    if (c.gacc)
        for (int64_t e = (int64_t)blockIdx.x * BLOCK + tid; e < c.n_gacc;
             e += (int64_t)gridDim.x * BLOCK)
            c.gacc[e] = 0.0;
    if ((int64_t)blockIdx.x >= ntiles) {
        if (c.gmax)
            for (int u = tid; u < a.n_u; u += BLOCK)
                c.gmax[(size_t)blockIdx.x * a.n_u + u] = 0.0;
        return;
    }
    // max of finite |dL/d(slot)| over the workgroup's points, per slot
    double gm[NSG];
#pragma unroll
    for (int k = 0; k < NSG; ++k)
        gm[k] = 0.0;

    if (n_stage > 0)
        fwd::dma_slab<BLOCK>(slab0, gsrc + (size_t)a.sgrp[0] * a.gstride, nodes);
    fwd::copy_words<BLOCK>(reinterpret_cast<char *>(knots), a.ax.knots, nx * 8);
    fwd::copy_words<BLOCK>(reinterpret_cast<char *>(knots + nx), a.aq.knots, nq * 8);
    fwd::copy_words<BLOCK>(reinterpret_cast<char *>(seeds), a.ax.seed, a.ax.nbuckets * 2);
    fwd::copy_words<BLOCK>(reinterpret_cast<char *>(seeds + a.ax.nbuckets), a.aq.seed,
                           a.aq.nbuckets * 2);
    __syncthreads();
    fwd::LAxis lx, lq;
    lx.k = knots;
    lx.seed = seeds;
    lx.n = nx;
    lx.nb = a.ax.nbuckets;
    lx.ln_lo = a.ax.ln_lo;
    lx.inv_hb = a.ax.inv_hb;
    lq.k = knots + nx;
    lq.seed = seeds + a.ax.nbuckets;
    lq.n = nq;
    lq.nb = a.aq.nbuckets;
    lq.ln_lo = a.aq.ln_lo;
    lq.inv_hb = a.aq.inv_hb;

    // A point's coordinates and the first dL/dout column of each slot's
    // flavour are loaded a tile ahead (clamped to the last point), during the
    // first stage of the tile before, so that the location of a tile does not
    // wait for them; further columns of a repeated pid are read when the tile
    // starts.
    const int n_slot = n_stage * G;
    bool dup_cols = false;
    for (int k = 0; k < n_slot; ++k)
        dup_cols = dup_cols || (a.slot_u[k] >= 0 &&
                                a.ucol_off[a.slot_u[k] + 1] - a.ucol_off[a.slot_u[k]] > 1);
    auto load_pt = [&](int64_t p, double &xv, double &qv, V (&g1)[NSG]) {
        xv = load_point(a.x, p, a.n);
        qv = load_point(a.q, p, a.n);
        const int64_t pc = p < a.n ? p : a.n - 1;
#pragma unroll
        for (int k = 0; k < NSG; ++k)
            if (k < n_slot && a.slot_col[k] >= 0)
                g1[k] = gout[pc * n_req + a.slot_col[k]];
    };
    double x_pt, q_pt;
    V g_pt[NSG];
#pragma unroll
    for (int k = 0; k < NSG; ++k)
        g_pt[k] = V(0);   // slots never loaded stay 0
    load_pt((int64_t)blockIdx.x * BLOCK + tid, x_pt, q_pt, g_pt);

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t p = tile * BLOCK + tid;
        const bool more = tile + gridDim.x < ntiles;
        double xv = x_pt, qv = q_pt;
        const double x_in = xv, q_in = qv;   // for the chain rule
        // flags of the domain rule, then the point clamped (CLAMP) or replaced
        // by the lower corner (outside in NaN mode, NaN input)
        uint8_t flag = 0;
        {
            const bool xin = xv >= a.ax.lo && xv <= a.ax.hi;
            const bool qin = qv >= a.aq.lo && qv <= a.aq.hi;
            if ((xv != xv) || (qv != qv))
                flag = kBwdOut;
            else if (!(xin && qin))
                flag = a.domain_mode == 1 ? (uint8_t)((xin ? 0 : kBwdXClamp) | (qin ? 0 : kBwdQClamp))
                                          : kBwdOut;
        }
        fwd::domain(a, xv, qv);
        const double lnx = log(xv), lnq = log(qv);
        const int ix = fwd::lbin(lx, xv, lnx);
        const int kq = fwd::lbin(lq, qv, lnq);
        const IntervalRec<double> rx = a.ax.rec64[ix];
        const IntervalRec<double> rq = a.aq.rec64[kq];
        const double tx = (lnx - rx.z) * rx.inv_d, tq = (lnq - rq.z) * rq.inv_d;
        if (c.st_idx && p < a.n) {
            c.st_idx[p] = ix | (kq << 16);
            c.st_flag[p] = flag;
            c.st_tx[p] = tx;
            c.st_tq[p] = tq;
        }
        double wx[4], dwx[4], wq[4], dwq[4];
        fold_both(tx, rx, wx, dwx);
        fold_both(tq, rq, wq, dwq);
        const int base = window2(ix, nx, wx, dwx) * nq + window2(kq, nq, wq, dwq);
        // dL/d(slot) summed over the slot's output columns (0 for slots that
        // hold no requested flavour)
        double gs[NSG];
#pragma unroll
        for (int k = 0; k < NSG; ++k)
            gs[k] = (double)g_pt[k];
        if (dup_cols) {
            const int64_t pc = p < a.n ? p : a.n - 1;
#pragma unroll
            for (int k = 0; k < NSG; ++k) {
                const int u = a.slot_u[k];
                if (k < n_slot && u >= 0)
                    for (int cc = a.ucol_off[u] + 1; cc < a.ucol_off[u + 1]; ++cc)
                        gs[k] += (double)gout[pc * n_req + a.ucols[cc]];
            }
        }
#pragma unroll
        for (int k = 0; k < NSG; ++k) {
            const double ag = fabs(gs[k]);
            if (ag < 1.0 / 0.0 && !(flag & kBwdOut))   // finite (false for NaN), inside
                gm[k] = fmax(gm[k], ag);
        }

        if (n_stage == 0)   // no stage to load the next point in (no pid of the grid requested)
            load_pt(p + (int64_t)gridDim.x * BLOCK, x_pt, q_pt, g_pt);
        fwd::wait_vm();
        __syncthreads();   // the tile's first group has landed
        double sx = 0.0, sw = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (s < n_stage) {
                const bool last = s + 1 == n_stage;
                uint4 *const cur = (s & 1) ? slab1 : slab0;
                uint4 *const nxt = (s & 1) ? slab0 : slab1;
                if (!last)
                    fwd::dma_slab<BLOCK>(nxt, gsrc + (size_t)a.sgrp[s + 1] * a.gstride, nodes);
                // the next tile's point: its loads land while this stage's
                // gathers run (every later wait for a slab copy covers them)
                if (s == 0)
                    load_pt(p + (int64_t)gridDim.x * BLOCK, x_pt, q_pt, g_pt);
                // each node's flavours are contracted with dL/d(slot) first, so
                // the two derivative stencils run once per group, not per flavour
#pragma unroll
                for (int jx = 0; jx < 4; ++jx) {
                    const uint4 *rowp = cur + base + jx * nq;
                    double r = 0.0, dr = 0.0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        V v[G];
                        fwd::Node<V>::get(rowp + k, v);
                        double vg = gs[s * G] * (double)v[0];
#pragma unroll
                        for (int g = 1; g < G; ++g)
                            vg = fma(gs[s * G + g], (double)v[g], vg);
                        r = fma(wq[k], vg, r);
                        dr = fma(dwq[k], vg, dr);
                    }
                    sx = fma(dwx[jx], r, sx);
                    sw = fma(wx[jx], dr, sw);
                }
                if (!last) {
                    fwd::wait_vm();
                    __syncthreads();
                }
            }
        }
        if (p < a.n) {
            const double nan = __builtin_nan("");
            if (c.grad_x)
                c.grad_x[p] = (flag & kBwdOut) ? nan
                              : (flag & kBwdXClamp) ? 0.0 : sx * rx.inv_d / x_in;
            if (c.grad_q2)
                c.grad_q2[p] = (flag & kBwdOut) ? nan
                               : (flag & kBwdQClamp) ? 0.0 : sw * rq.inv_d / q_in;
        }
        // next tile's first group into slab0 once every wave is done with it
        __syncthreads();
        if (n_stage > 1 && more)
            fwd::dma_slab<BLOCK>(slab0, gsrc + (size_t)a.sgrp[0] * a.gstride, nodes);
    }
    fwd::wait_vm();
    if (c.gmax) {
        // the slabs are free now: slab0 holds the waves' maxima
        double *red = reinterpret_cast<double *>(slab0);
        const int wave = tid >> 6;
#pragma unroll
        for (int k = 0; k < NSG; ++k) {
            double v = gm[k];
#pragma unroll
            for (int d = 1; d < 64; d <<= 1)
                v = fmax(v, __shfl_xor(v, d));
            if ((tid & 63) == 0)
                red[wave * NSG + k] = v;
        }
        __syncthreads();
        for (int u = tid; u < a.n_u; u += BLOCK) {
            double v = 0.0;
            for (int k = 0; k < NSG; ++k)
                if (a.slot_u[k] == u)
                    for (int w = 0; w < BLOCK / 64; ++w)
                        v = fmax(v, red[w * NSG + k]);
            c.gmax[(size_t)blockIdx.x * a.n_u + u] = v;
        }
    }
}

// Knot gradient, dL/dv[f][i][k] = sum_p g[p][f] wx_i(p) wq_k(p), for up to
// kKnotGroup flavours per workgroup: their gradient slabs (borderless) sit in
// LDS together, so each point's state (bins, local coordinates, flags from the
// pass that located the points) is read and its weights folded once per group
// rather than once per flavour.  The LDS sums are added to the FP64
// accumulator at the end.
//
// Each wave takes 64 consecutive points per step.  A point's 16 adds go to
// its stencil base plus offsets common to all lanes, so the wave first deals
// its points out to lanes by the base's bank (wave_deal); the keys for that
// are loaded a step ahead, so that only the dealt point's own values are
// waited for.  The interval records are read from global memory (they stay
// in the L1 cache): the LDS is the pass's bottleneck, and records staged
// there made it slower.  The sums are kept in 64-bit fixed point
// (fixed_point.h), with the scale of each flavour taken from the max of
// finite |dL/dout| (left per workgroup by the coordinate pass, else found by
// a sweep over the chunk) and from the axes' weight-sum bounds.  A non-finite
// dL/dout skips the fixed-point sums: its 16 products go to the FP64
// accumulator by global atomics on the knots of the point's stencil (the
// window of knots i-1 .. i+2 cut at the axis ends), so it poisons those knots
// only, as the FP64-atomic adjoint does.
constexpr int kKnotGroup = 3;
constexpr int kKnotBlock = 1024;

template <typename GT>
__global__ __launch_bounds__(kKnotBlock) void knot_grad_kernel(const BwdArgs a)
{
    __shared__ unsigned long long gsl[kKnotGroup][kDmaNodes];
    __shared__ int khist[kKnotBlock / 64][kDealKeys];
    __shared__ double wmax[kKnotGroup + 2][kKnotBlock / 64];
    const GT *gout = reinterpret_cast<const GT *>(a.gout);
    const int grp = blockIdx.y;
    const int u0 = grp * kKnotGroup;
    const int nu = a.n_u - u0 < kKnotGroup ? a.n_u - u0 : kKnotGroup;
    const int nx = a.nx, nq = a.nq, nodes = nx * nq;
    for (int e = threadIdx.x; e < nodes; e += kKnotBlock)
        for (int j = 0; j < kKnotGroup; ++j)
            gsl[j][e] = 0ull;
    const int64_t p_begin = (int64_t)blockIdx.x * a.chunk;
    const int64_t p_end = p_begin + a.chunk < a.n ? p_begin + a.chunk : a.n;
    int col[kKnotGroup];     // first output column of flavour j (clamped to a valid one)
    bool more[kKnotGroup];   // flavour j has further columns (duplicate pids)
#pragma unroll
    for (int j = 0; j < kKnotGroup; ++j) {
        const int u = u0 + (j < nu ? j : nu - 1);
        col[j] = a.ucols[a.ucol_off[u]];
        more[j] = j < nu && a.ucol_off[u + 1] - a.ucol_off[u] > 1;
    }
    // dL/dout of the group's flavours at point p, each summed over its columns
    // (the first columns loaded together, so that their latencies overlap)
    auto gsum = [&](int64_t p, double (&g)[kKnotGroup]) {
#pragma unroll
        for (int j = 0; j < kKnotGroup; ++j)
            g[j] = (double)gout[p * a.n_req + col[j]];
#pragma unroll
        for (int j = 0; j < kKnotGroup; ++j)
            if (more[j])
                for (int c = a.ucol_off[u0 + j] + 1; c < a.ucol_off[u0 + j + 1]; ++c)
                    g[j] += (double)gout[p * a.n_req + a.ucols[c]];
    };
    // m[j]: max of finite |dL/dout| of flavour j over all points;
    // m[kKnotGroup], m[kKnotGroup + 1]: weight-sum bounds of the x and Q^2 axes
    double m[kKnotGroup + 2];
#pragma unroll
    for (int j = 0; j < kKnotGroup + 2; ++j)
        m[j] = 0.0;
    if (a.gmax) {
        for (int i = threadIdx.x; i < a.n_part; i += kKnotBlock)
#pragma unroll
            for (int j = 0; j < kKnotGroup; ++j)
                if (j < nu)
                    m[j] = fmax(m[j], a.gmax[(size_t)i * a.n_u + u0 + j]);
    } else {
        // over the chunk's points inside the grid
        for (int64_t p = p_begin + threadIdx.x; p < p_end; p += kKnotBlock) {
            const bool in = !(a.st_flag[p] & kBwdOut);
            double g[kKnotGroup];
            gsum(p, g);
#pragma unroll
            for (int j = 0; j < kKnotGroup; ++j) {
                const double ag = fabs(g[j]);
                if (in && j < nu && ag < 1.0 / 0.0)   // finite (false for NaN)
                    m[j] = fmax(m[j], ag);
            }
        }
    }
    for (int i = threadIdx.x; i < nx - 1; i += kKnotBlock)
        m[kKnotGroup] = fmax(m[kKnotGroup], weight_sum_bound(a.ax.rec64[i]));
    for (int i = threadIdx.x; i < nq - 1; i += kKnotBlock)
        m[kKnotGroup + 1] = fmax(m[kKnotGroup + 1], weight_sum_bound(a.aq.rec64[i]));
#pragma unroll
    for (int j = 0; j < kKnotGroup + 2; ++j) {
        double v = m[j];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1)
            v = nan_max(v, __shfl_xor(v, d));
        if ((threadIdx.x & 63) == 0)
            wmax[j][threadIdx.x >> 6] = v;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kKnotGroup + 2; ++j) {
        double v = wmax[j][0];
        for (int w = 1; w < kKnotBlock / 64; ++w)
            v = nan_max(v, wmax[j][w]);
        m[j] = v;
    }
    // the scales are the same in every lane: held in scalar registers
    auto uniform = [](double v) {
        const long long b = __double_as_longlong(v);
        const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
        const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(b >> 32));
        return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    };
    double fs[kKnotGroup];
    bool fin[kKnotGroup];
    bool any = false;
#pragma unroll
    for (int j = 0; j < kKnotGroup; ++j) {
        const double bnd = uniform(m[j] * m[kKnotGroup] * m[kKnotGroup + 1]);   // |g wx wq|
        fin[j] = bnd < 1.0 / 0.0;                                               // false for NaN
        any = any || (j < nu && fin[j]);
        fs[j] = uniform(ldexp(1.0, fin[j] ? fixed_exponent(bnd, p_end - p_begin) : 0));
    }
    const int lane = threadIdx.x & 63;
    int *hist = khist[threadIdx.x >> 6];
    // The keys (state of the lane's point) are loaded a step ahead; the dealt
    // point's local coordinates and dL/dout are then read at its own index.
    int kidx, kflag;
    auto load_key = [&](int64_t p0, int &ki, int &kf) {
        const int64_t pn = p0 + lane;
        const int64_t pc = pn < p_end ? (pn > p_begin ? pn : p_begin) : p_end - 1;
        ki = a.st_idx[pc];
        kf = a.st_flag[pc];
    };
    // wave-uniform loop: every lane takes part in the dealing
    const int64_t pw = p_begin + (threadIdx.x & ~63);
    load_key(pw, kidx, kflag);
    for (int64_t p0 = pw; any && p0 < p_end; p0 += kKnotBlock) {
        int nidx, nflag;
        load_key(p0 + kKnotBlock, nidx, nflag);   // unconditional (clamped): no wait covers it
        const bool valid = p0 + lane < p_end && !(kflag & kBwdOut);
        int key = kDealKeys - 1;
        if (valid) {
            int sx = (kidx & 0xffff) - 1, sq = (kidx >> 16) - 1;
            sx = sx < 0 ? 0 : (sx > nx - 4 ? nx - 4 : sx);
            sq = sq < 0 ? 0 : (sq > nq - 4 ? nq - 4 : sq);
            key = (sx * nq + sq) & 31;
        }
        const int src = wave_deal(key, hist);
        const bool ok = __shfl((int)valid, src) != 0;
        const int idx = __shfl(kidx, src);
        kidx = nidx;
        kflag = nflag;
        if (!ok)   // outside the grid (NaN mode), NaN input, past the chunk
            continue;
        const int64_t p = p0 + src;
        const double tx = a.st_tx[p], tq = a.st_tq[p];
        double gv[kKnotGroup];
        gsum(p, gv);
        const int ix = idx & 0xffff, kq = idx >> 16;
        const IntervalRec<double> rx = a.ax.rec64[ix];
        const IntervalRec<double> rq = a.aq.rec64[kq];
        double wx[4], wq[4];
        fwd::fold<double>(tx, rx.pl, rx.plql, rx.ql, rx.qr, rx.qrpr, rx.pr, wx);
        fwd::fold<double>(tq, rq.pl, rq.plql, rq.ql, rq.qr, rq.qrpr, rq.pr, wq);
        const int base = fwd::window(ix, nx, wx) * nq + fwd::window(kq, nq, wq);
#pragma unroll
        for (int j = 0; j < kKnotGroup; ++j) {
            if (j < nu && fin[j]) {
                const double g = gv[j];
                if (fabs(g) < 1.0 / 0.0) {
#pragma unroll
                    for (int jx = 0; jx < 4; ++jx) {
                        const double gx = g * wx[jx];
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk)
                            atomicAdd(&gsl[j][base + jx * nq + kk], to_fixed(gx * wq[kk], fs[j]));
                    }
                } else {
                    // weights of knots ix-1 .. ix+2, kq-1 .. kq+2 (not shifted
                    // into the window), folded again on this rare path
                    double vx[4], vq[4];
                    const IntervalRec<double> sx = a.ax.rec64[ix];
                    const IntervalRec<double> sq = a.aq.rec64[kq];
                    fwd::fold<double>(tx, sx.pl, sx.plql, sx.ql, sx.qr, sx.qrpr, sx.pr, vx);
                    fwd::fold<double>(tq, sq.pl, sq.plql, sq.ql, sq.qr, sq.qrpr, sq.pr, vq);
                    double *dst = a.gacc + (size_t)a.urow[u0 + j] * nodes;
                    for (int jx = 0; jx < 4; ++jx) {
                        const int i = ix - 1 + jx;
                        if (i < 0 || i >= nx)
                            continue;
                        const double gx = g * vx[jx];
                        for (int kk = 0; kk < 4; ++kk) {
                            const int kk2 = kq - 1 + kk;
                            if (kk2 >= 0 && kk2 < nq)
                                unsafeAtomicAdd(&dst[i * nq + kk2], gx * vq[kk]);
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int j = 0; j < nu; ++j) {
        double *dst = a.gacc + (size_t)a.urow[u0 + j] * nodes;
        const double inv = 1.0 / fs[j];   // exact: a power of two
        for (int e = threadIdx.x; e < nodes; e += kKnotBlock) {
            const long long v = (long long)gsl[j][e];
            if (!fin[j])
                unsafeAtomicAdd(&dst[e], __builtin_nan(""));
            else if (v != 0)
                unsafeAtomicAdd(&dst[e], (double)v * inv);
        }
    }
}

}  // namespace

bool knot_grad_supported(int nx, int nq)
{
    return nx >= 4 && nq >= 4 && nx * nq <= kDmaNodes;
}

hipError_t launch_knot_grad(const BwdArgs &b, bool f32, int cus, hipStream_t s)
{
    BwdArgs k = b;
    const int ngroups = (b.n_u + kKnotGroup - 1) / kKnotGroup;
    int64_t nchunk = cus / ngroups > 0 ? cus / ngroups : 1;   // one workgroup per compute unit
    int64_t chunk = (b.n + nchunk - 1) / nchunk;
    if (chunk < kKnotBlock)
        chunk = kKnotBlock;
    nchunk = (b.n + chunk - 1) / chunk;
    k.chunk = (int)chunk;
    if (f32)
        hipLaunchKernelGGL(knot_grad_kernel<float>, dim3((unsigned)nchunk, (unsigned)ngroups),
                           dim3(kKnotBlock), 0, s, k);
    else
        hipLaunchKernelGGL(knot_grad_kernel<double>, dim3((unsigned)nchunk, (unsigned)ngroups),
                           dim3(kKnotBlock), 0, s, k);
    return hipGetLastError();
}

constexpr int kCoordBlock = 512;

int coord_grad_blocks(int64_t n, int cus)
{
    const int64_t ntiles = (n + kCoordBlock - 1) / kCoordBlock;
    int64_t grid = ntiles < cus ? ntiles : cus;   // one resident workgroup per compute unit
    if (grid > kMaxPart)
        grid = kMaxPart;
    return grid < 1 ? 1 : (int)grid;
}

hipError_t launch_coord_grad(const CoordArgs &c, bool f32, int cus, hipStream_t s)
{
    constexpr int kBlock = kCoordBlock;
    const int grid = coord_grad_blocks(c.x.n, cus);
    auto fn = f32 ? coord_grad_kernel<float, kBlock> : coord_grad_kernel<double, kBlock>;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(kBlock), 0, s, c);
    return hipGetLastError();
}

}  // namespace pdfx
