// Flavour-pair luminosity on gfx950: for every point, the partons a_k at
// (x1, Q^2) and b_k at (x2, Q^2), L_k = f_{a_k}(x1) f_{b_k}(x2) with f = xf / x,
// and S = sum_k c_k L_k (the luminosity of Eq. 1; Fig. 4 builds one for
// single top: b at x1 against u, c, dbar, sbar at x2, at a fixed Q^2, divided
// by x1 x2).
//
// The grid's flavour groups touched by the pairs are walked once per tile,
// double-buffered in LDS as in the forward kernel; a group is evaluated at
// x1, at x2 or at both, depending on which side of a pair its partons take.
// Both points share the Q^2 bin and weights.  The results sit in register
// slots fixed at compile time (group stage s, lane g); the pairs name slots
// at run time, so each thread copies its slots into a column area in LDS and
// forms the products from there (a thread reads back only what it wrote, so
// no barrier is needed between the two).
#include "lumi_internal.h"
#include "xfx_dma_impl.h"

namespace pdfx {

namespace {

using fwd::kDmaKnots;
using fwd::kDmaNodes;
using fwd::kDmaSeeds;

// Bins and weights of one point at (x1, Q^2) and (x2, Q^2).
template <typename V>
struct LumiPoint {
    V w1[4], w2[4], wq[4];
    int b1, b2;
    V inv;      // 1 / (x1 x2)
    bool ok;
};

// FQ: one Q^2 for every point (q2 null).  The Q^2 location (log, bin,
// weights, window) is then found once per thread and shared by the points,
// with the same arithmetic as per point, so the results are the same bits.
template <typename V, int BLOCK, int PPT, bool FQ>
__global__ __launch_bounds__(BLOCK) void lumi_kernel(const LumiArgs a)
{
    constexpr int G = 16 / (int)sizeof(V);
    constexpr int NS = kGrpMaxSlots / G;
    constexpr int NSG = NS * G;
    constexpr int COLS = BLOCK < 256 ? BLOCK : 256;   // threads per column area
    static_assert(2 * NSG * COLS * (int)sizeof(V) <= kDmaNodes * 16, "column area exceeds a slab");
    __shared__ uint4 slab0[kDmaNodes];
    __shared__ uint4 slab1[kDmaNodes];
    __shared__ double knots[kDmaKnots];
    __shared__ uint16_t seeds[kDmaSeeds];
    const int tid = threadIdx.x;

    const int nx = a.nx, nq = a.nq;
    const int nodes = nx * nq;
    const uint4 *gsrc = reinterpret_cast<const uint4 *>(a.gvals);
    const int n_stage = a.n_stage;
    const int n_pair = a.n_pair;
    V *out_pair = reinterpret_cast<V *>(a.out_pair);
    V *out_sum = reinterpret_cast<V *>(a.out_sum);
    const int64_t tile_pts = (int64_t)BLOCK * PPT;
    const int64_t ntiles = (a.n + tile_pts - 1) / tile_pts;
    if ((int64_t)blockIdx.x >= ntiles)
        return;

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

    // The fixed Q^2 is read once, as a value: choosing per point between it
    // and the Q^2 array would otherwise become a choice between two addresses
    // (a flat load, which holds up LDS waits).
    const double q2_fixed = a.q2_fixed;
    const bool q2_arr = a.q2 != nullptr;

    // The fixed Q^2's location: inside, clamped into the grid (CLAMP mode),
    // or, when every point is outside (NaN mode), the first knot.
    V wqf[4];
    int cqf = 0;
    bool q_in = true;
    if constexpr (FQ) {
        double q2 = q2_fixed;
        q_in = q2 >= a.aq.lo && q2 <= a.aq.hi;
        if (!q_in)
            q2 = a.domain_mode == 1 ? fmin(fmax(q2, a.aq.lo), a.aq.hi) : a.aq.lo;
        const double lnq = log(q2);
        const int kq = fwd::lbin(lq, q2, lnq);
        fwd::weights_gmem<V>(a.aq, kq, lnq, wqf);
        cqf = fwd::window(kq, nq, wqf);
    }

    // Domain rule of the forward evaluation applied to x1, x2 and Q^2
    // together; logs, bins, weights and windows of both points.
    auto locate = [&](int64_t p, double x1, double x2, double q2, LumiPoint<V> &st) {
        if constexpr (FQ) {
            const bool nan_in = (x1 != x1) || (x2 != x2);
            const bool inside = x1 >= a.ax.lo && x1 <= a.ax.hi && x2 >= a.ax.lo &&
                                x2 <= a.ax.hi && q_in;
            st.ok = true;
            if (!inside) {
                if (a.domain_mode == 1 && !nan_in) {
                    x1 = fmin(fmax(x1, a.ax.lo), a.ax.hi);
                    x2 = fmin(fmax(x2, a.ax.lo), a.ax.hi);
                } else {
                    st.ok = false;
                    x1 = x2 = a.ax.lo;
                }
            }
            fwd::count_flagged(p < a.n && !st.ok, a.dom_count);
            const double lnx1 = log(x1), lnx2 = log(x2);
            const int i1 = fwd::lbin(lx, x1, lnx1);
            const int i2 = fwd::lbin(lx, x2, lnx2);
            fwd::weights_gmem<V>(a.ax, i1, lnx1, st.w1);
            fwd::weights_gmem<V>(a.ax, i2, lnx2, st.w2);
            st.b1 = fwd::window(i1, nx, st.w1) * nq + cqf;
            st.b2 = fwd::window(i2, nx, st.w2) * nq + cqf;
            st.inv = (V)(1.0 / (x1 * x2));
            return;
        }
        const bool nan_in = (x1 != x1) || (x2 != x2) || (q2 != q2);
        const bool inside = x1 >= a.ax.lo && x1 <= a.ax.hi && x2 >= a.ax.lo && x2 <= a.ax.hi &&
                            q2 >= a.aq.lo && q2 <= a.aq.hi;
        st.ok = true;
        if (!inside) {
            if (a.domain_mode == 1 && !nan_in) {
                x1 = fmin(fmax(x1, a.ax.lo), a.ax.hi);
                x2 = fmin(fmax(x2, a.ax.lo), a.ax.hi);
                q2 = fmin(fmax(q2, a.aq.lo), a.aq.hi);
            } else {
                st.ok = false;
                x1 = x2 = a.ax.lo;
                q2 = a.aq.lo;
            }
        }
        fwd::count_flagged(p < a.n && !st.ok, a.dom_count);
        const double lnx1 = log(x1), lnx2 = log(x2), lnq = log(q2);
        const int i1 = fwd::lbin(lx, x1, lnx1);
        const int i2 = fwd::lbin(lx, x2, lnx2);
        const int kq = fwd::lbin(lq, q2, lnq);
        fwd::weights_gmem<V>(a.ax, i1, lnx1, st.w1);
        fwd::weights_gmem<V>(a.ax, i2, lnx2, st.w2);
        fwd::weights_gmem<V>(a.aq, kq, lnq, st.wq);
        const int cq = fwd::window(kq, nq, st.wq);
        st.b1 = fwd::window(i1, nx, st.w1) * nq + cq;
        st.b2 = fwd::window(i2, nx, st.w2) * nq + cq;
        st.inv = (V)(1.0 / (x1 * x2));
    };

    // Stencil of one group at one point (window base b, weights wx, wq).
    auto stencil = [&](const uint4 *slab, int b, const V (&wx)[4], const V (&wq)[4], V (&r)[G]) {
#pragma unroll
        for (int jx = 0; jx < 4; ++jx) {
            const uint4 *rowp = slab + b + jx * nq;
            V rr[G];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                V v[G];
                fwd::Node<V>::get(rowp + k, v);
#pragma unroll
                for (int g = 0; g < G; ++g)
                    rr[g] = (k == 0) ? wq[0] * v[g] : fma(wq[k], v[g], rr[g]);
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
                r[g] = (jx == 0) ? wx[0] * rr[g] : fma(wx[jx], rr[g], r[g]);
        }
    };

    // The coordinates of a tile are requested one tile ahead, so that their
    // memory latency passes during the previous tile's stages.
    double cx1[PPT], cx2[PPT], cq2[PPT];
    auto load_coords = [&](int64_t t) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int64_t p = t * tile_pts + tid + (int64_t)j * BLOCK;
            cx1[j] = load_point(a.x1, p, a.n);
            cx2[j] = load_point(a.x2, p, a.n);
            cq2[j] = q2_fixed;
            if (q2_arr)
                cq2[j] = load_point(a.q2, p, a.n);
        }
    };
    load_coords(blockIdx.x);

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t t0 = tile * tile_pts;
        const bool more = tile + gridDim.x < ntiles;
        LumiPoint<V> pt[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j)
            locate(t0 + tid + (int64_t)j * BLOCK, cx1[j], cx2[j], cq2[j], pt[j]);

        fwd::wait_vm();
        __syncthreads();   // the tile's first slab has landed
        if (more)
            load_coords(tile + gridDim.x);   // waited for with the first stage's copy

        V r1[PPT][NSG], r2[PPT][NSG];
#pragma unroll
        for (int j = 0; j < PPT; ++j)
#pragma unroll
            for (int c = 0; c < NSG; ++c)
                r1[j][c] = r2[j][c] = V(0);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (s < n_stage) {
                const bool last = s + 1 == n_stage;
                const uint4 *cur = (s & 1) ? slab1 : slab0;
                if (!last)
                    fwd::dma_slab<BLOCK>((s & 1) ? slab0 : slab1,
                                         gsrc + (size_t)a.sgrp[s + 1] * a.gstride, nodes);
                const int sd = a.side[s];
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    if (sd & 1) {
                        V t[G];
                        stencil(cur, pt[j].b1, pt[j].w1, FQ ? wqf : pt[j].wq, t);
#pragma unroll
                        for (int g = 0; g < G; ++g)
                            r1[j][s * G + g] = t[g];
                    }
                    if (sd & 2) {
                        V t[G];
                        stencil(cur, pt[j].b2, pt[j].w2, FQ ? wqf : pt[j].wq, t);
#pragma unroll
                        for (int g = 0; g < G; ++g)
                            r2[j][s * G + g] = t[g];
                    }
                }
                if (!last) {
                    fwd::wait_vm();
                    __syncthreads();
                }
            }
        }
        __syncthreads();   // every stencil read is done: both slabs are free

        // Thread t's slot c at x1 is area[c * COLS + t % COLS], at x2
        // area[(NSG + c) * COLS + t % COLS]; the first COLS threads use slab0,
        // the next COLS slab1.
        V *area = reinterpret_cast<V *>(tid < COLS ? slab0 : slab1);
        const int tl = tid % COLS;
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
#pragma unroll
            for (int c = 0; c < NSG; ++c) {
                if (c < n_stage * G) {
                    area[c * COLS + tl] = r1[j][c];
                    area[(NSG + c) * COLS + tl] = r2[j][c];
                }
            }
            const int64_t p = t0 + tid + (int64_t)j * BLOCK;
            if (p < a.n) {
                V sum = V(0);
                for (int k = 0; k < n_pair; ++k) {
                    const int ia = a.ia[k], ib = a.ib[k];
                    V l = V(0);
                    if (ia >= 0 && ib >= 0) {
                        l = area[ia * COLS + tl] * area[(NSG + ib) * COLS + tl] * pt[j].inv;
                        if (!pt[j].ok)
                            l = fwd::quiet_nan<V>();
                    }
                    if (out_pair)
                        out_pair[p * n_pair + k] = l;
                    sum = fma((V)a.coef[k], l, sum);
                }
                if (out_sum)
                    out_sum[p] = pt[j].ok ? sum : fwd::quiet_nan<V>();
            }
        }
        __syncthreads();   // the column areas are read before the next copy
        if (more && n_stage > 0)
            fwd::dma_slab<BLOCK>(slab0, gsrc + (size_t)a.sgrp[0] * a.gstride, nodes);
    }
    fwd::wait_vm();
}

constexpr LaunchShape kLumiShapes[] = {{512, 1}, {512, 2}, {256, 2}};

template <typename V>
hipError_t launch_typed(const LumiArgs &a, LaunchShape ls, int cus, hipStream_t s)
{
    auto go = [&](auto fn, int block, int ppt) -> hipError_t {
        const int64_t tile = (int64_t)block * ppt;
        int64_t grid = (a.n + tile - 1) / tile;
        if (grid > cus)
            grid = cus;   // one resident workgroup per compute unit (LDS)
        if (grid < 1)
            return hipSuccess;
        hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(block), 0, s, a);
        return hipGetLastError();
    };
    const bool fq = a.q2 == nullptr;
    if (ls.block == 512 && ls.ppt == 1)
        return fq ? go(lumi_kernel<V, 512, 1, true>, 512, 1) : go(lumi_kernel<V, 512, 1, false>, 512, 1);
    if (ls.block == 512 && ls.ppt == 2)
        return fq ? go(lumi_kernel<V, 512, 2, true>, 512, 2) : go(lumi_kernel<V, 512, 2, false>, 512, 2);
    if (ls.block == 256 && ls.ppt == 2)
        return fq ? go(lumi_kernel<V, 256, 2, true>, 256, 2) : go(lumi_kernel<V, 256, 2, false>, 256, 2);
    if constexpr (sizeof(V) == 4) {
        if (ls.block == 512 && ls.ppt == 4)
            return fq ? go(lumi_kernel<V, 512, 4, true>, 512, 4)
                      : go(lumi_kernel<V, 512, 4, false>, 512, 4);
    }
    return hipErrorInvalidValue;
}

}  // namespace

bool lumi_supported(int nx, int nq, int nbx, int nbq)
{
    return nx >= 4 && nq >= 4 && nx * nq <= kDmaNodes && nx + nq <= kDmaKnots &&
           nbx + nbq <= kDmaSeeds;
}

bool lumi_shape_supported(LaunchShape ls, bool f32)
{
    if (f32 && ls.block == 512 && ls.ppt == 4)
        return true;
    for (const auto &k : kLumiShapes)
        if (k.block == ls.block && k.ppt == ls.ppt)
            return true;
    return false;
}

hipError_t launch_lumi(const LumiArgs &a, bool f32, LaunchShape ls, int cus, hipStream_t s)
{
    return f32 ? launch_typed<float>(a, ls, cus, s) : launch_typed<double>(a, ls, cus, s);
}

}  // namespace pdfx
