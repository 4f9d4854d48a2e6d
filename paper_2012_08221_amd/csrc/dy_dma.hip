// Double-buffered forward kernel of the Drell-Yan-like integrand (same
// integrand as dy.hip) for grids that fit the double-buffered xf kernel and
// hold the 11 partons in the standard order (-5 .. -1, g, 1 .. 5).
//
// The flavour groups of the grid are walked once per tile: with that order,
// the groups up to the one holding -1 are evaluated at (x2, Q^2) and the ones
// from the group holding 1 on at (x1, Q^2) (FP32: the middle group {-1, g, 1,
// 2} at both), so every result lands in a register slot fixed at compile
// time and the partner products need no indexing.  The luminosity sum runs
// over q = 1 .. 5 in the same order and with the same operations as the
// single-slab kernel, so both give the same per-point values.
//
// Staging, LDS layout and the overlap of the next tile's point location with
// the stencil stages follow the double-buffered xf kernel; alpha_s is located
// by bisection over its knots in LDS, its interval records and values are
// read from global memory.
#include "xfx_dma_impl.h"

namespace pdfx {

namespace {

using fwd::kDmaKnots;
using fwd::kDmaNodes;
using fwd::kDmaSeeds;

// Largest i in [0, n-2] with k[i] <= v, for v in [k[0], k[n-1]].
__device__ __forceinline__ int bisect(const double *k, int n, double v)
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

// Per-point state: bins and weights of (x1, Q^2), (x2, Q^2), alpha_s.
template <typename V>
struct DyPoint {
    V w1[4], w2[4], wq[4];
    int b1, b2;
    V as;
    bool ok;
};

template <typename V, int BLOCK, int PPT>
__global__ __launch_bounds__(BLOCK) void dy_dma_kernel(const DyArgs a)
{
    constexpr int G = 16 / (int)sizeof(V);
    constexpr int NS = 12 / G;   // groups of the 11-parton grid
    __shared__ uint4 slab0[kDmaNodes];
    __shared__ uint4 slab1[kDmaNodes];
    __shared__ double knots[kDmaKnots];
    __shared__ uint16_t seeds[kDmaSeeds];
    const int tid = threadIdx.x;

    const int nx = a.nx, nq = a.nq, na = a.aa.n;
    const int nodes = nx * nq;
    const uint4 *gsrc = reinterpret_cast<const uint4 *>(a.gvals);
    V *out = reinterpret_cast<V *>(a.out);
    const V *asv = reinterpret_cast<const V *>(a.as_vals);
    const int64_t tile_pts = (int64_t)BLOCK * PPT;
    const int64_t ntiles = (a.n + tile_pts - 1) / tile_pts;

    if ((int64_t)blockIdx.x < ntiles)
        fwd::dma_slab<BLOCK>(slab0, gsrc, nodes);   // first group of the first tile
    fwd::copy_words<BLOCK>(reinterpret_cast<char *>(knots), a.ax.knots, nx * 8);
    fwd::copy_words<BLOCK>(reinterpret_cast<char *>(knots + nx), a.aq.knots, nq * 8);
    fwd::copy_words<BLOCK>(reinterpret_cast<char *>(knots + nx + nq), a.aa.knots, na * 8);
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
    const double *ka_knots = knots + nx + nq;

    auto locate = [&](double ua, double ub, int64_t p, DyPoint<V> &st) {
        const double l1 = a.lnxmin + ua * a.lnrange;
        const double l2 = a.lnxmin + ub * a.lnrange;
        double x1 = exp(l1), x2 = exp(l2);
        double q2 = x1 * x2 * a.s;
        q2 = q2 < a.aq.lo ? a.aq.lo : (q2 > a.aq.hi ? a.aq.hi : q2);
        st.ok = x1 >= a.ax.lo && x1 <= a.ax.hi && x2 >= a.ax.lo && x2 <= a.ax.hi &&
                q2 >= a.aa.lo && q2 <= a.aa.hi;
        fwd::count_flagged(p < a.n && !st.ok, a.dom_count);
        if (!st.ok) {
            x1 = x2 = a.ax.lo;
            q2 = a.aq.lo > a.aa.lo ? a.aq.lo : a.aa.lo;
        }
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
        const int ka = bisect(ka_knots, na, q2);
        V wa[4];
        fwd::weights_gmem<V>(a.aa, ka, lnq, wa);
        V av = wa[0] * asv[ka];
        av = fma(wa[1], asv[ka + 1], av);
        av = fma(wa[2], asv[ka + 2], av);
        av = fma(wa[3], asv[ka + 3], av);
        st.as = av;
    };

    // Stencil of one group at one point (window base b, weights wx, wq).
    auto stencil = [&](const uint4 *slab, int b, const V (&wx)[4], const V (&wq)[4], V (&r)[G]) {
        V acc[G];
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
                acc[g] = (jx == 0) ? wx[0] * rr[g] : fma(wx[jx], rr[g], acc[g]);
        }
#pragma unroll
        for (int g = 0; g < G; ++g)
            r[g] = acc[g];
    };

    // Point state of the current tile and of the next one; the next tile's
    // points are located during the current tile's stencil stages (point j
    // in stage j), whose time goes to LDS traffic.
    DyPoint<V> cur[PPT], nxt[PPT];
    double unext[PPT], vnext[PPT];
    if ((int64_t)blockIdx.x < ntiles) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int64_t p = (int64_t)blockIdx.x * tile_pts + tid + (int64_t)j * BLOCK;
            locate(load_point(a.u1, p, a.n), load_point(a.u2, p, a.n), p, cur[j]);
            const int64_t pn = p + (int64_t)gridDim.x * tile_pts;
            unext[j] = load_point(a.u1, pn, a.n);
            vnext[j] = load_point(a.u2, pn, a.n);
        }
    }

    double part = 0.0;   // this thread's FP64 partial sum of I
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t t0 = tile * tile_pts;
        const bool more = tile + gridDim.x < ntiles;
        const int64_t pnext0 = t0 + (int64_t)gridDim.x * tile_pts + tid;
        auto locate_next = [&](int j) {
            const int64_t pn = pnext0 + (int64_t)j * BLOCK;
            locate(unext[j], vnext[j], pn, nxt[j]);
            const int64_t pnn = pn + (int64_t)gridDim.x * tile_pts;
            unext[j] = load_point(a.u1, pnn, a.n);
            vnext[j] = load_point(a.u2, pnn, a.n);
        };

        fwd::wait_vm();
        __syncthreads();   // the tile's first group has landed

        // x2-side values by grid row (antiquarks -5 .. -1 are rows 0 .. 4;
        // the gluon slot is not used) and the luminosity sum.
        V at2[PPT][12], lum[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j)
            lum[j] = V(0);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            // (a.n_seq is 10 for this kernel: the test is always true; as a
            // runtime test it keeps each stage's arithmetic in the stage's
            // own block instead of letting it drift to the end of the tile,
            // where the loaded nodes would all have to stay live)
            if (a.n_seq < 2 * s)
                continue;
            const uint4 *cs = (s & 1) ? slab1 : slab0;
            uint4 *ns = (s & 1) ? slab0 : slab1;
            if (s + 1 < NS)
                fwd::dma_slab<BLOCK>(ns, gsrc + (size_t)(s + 1) * a.gstride, nodes);
            else if ((s & 1) && more)
                fwd::dma_slab<BLOCK>(slab0, gsrc, nodes);   // slab0 is free during the last stage
            if (s < PPT)
                locate_next(s);
            // rows s*G .. s*G+G-1: antiquarks are rows 0 .. 4, quarks rows 6 .. 10
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                V r[G];
                if (s * G <= 4) {
                    stencil(cs, cur[j].b2, cur[j].w2, cur[j].wq, r);
#pragma unroll
                    for (int g = 0; g < G; ++g)
                        at2[j][s * G + g] = r[g];
                }
                if (s * G + G - 1 >= 6) {
                    stencil(cs, cur[j].b1, cur[j].w1, cur[j].wq, r);
                    // quark q = row - 5 meets its antiquark (row 5 - q) at x2,
                    // in the order q = 1 .. 5
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const int q = s * G + g - 5;
                        if (q >= 1 && q <= 5)
                            lum[j] = fma(r[g], at2[j][5 - q], lum[j]);
                    }
                }
            }
            if (s + 1 < NS) {
                fwd::wait_vm();
                __syncthreads();
            }
        }
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const V I = (V)a.L2 * cur[j].as * lum[j];
            const int64_t p = t0 + tid + (int64_t)j * BLOCK;
            if (p < a.n) {
                if (out)
                    out[p] = cur[j].ok ? I : fwd::quiet_nan<V>();
                part += cur[j].ok ? (double)I : __builtin_nan("");
            }
            cur[j] = nxt[j];
        }
        if ((NS & 1) && more) {
            // the last stage read slab0: start the next tile's first group now
            __syncthreads();
            fwd::dma_slab<BLOCK>(slab0, gsrc, nodes);
        }
    }

    // workgroup sum of the partial sums (fixed order: deterministic)
    fwd::wait_vm();
    __syncthreads();
    double *red = reinterpret_cast<double *>(slab1);
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

template <typename V>
hipError_t dy_dma_typed(const DyArgs &a, LaunchShape ls, int cus, hipStream_t s, int *n_blocks)
{
    auto go = [&](auto fn, int block, int ppt) -> hipError_t {
        const int64_t tile_pts = (int64_t)block * ppt;
        const int64_t ntiles = (a.n + tile_pts - 1) / tile_pts;
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(fn), block, 0);
        if (e != hipSuccess || per_cu < 1)
            per_cu = 1;
        int64_t grid = (int64_t)per_cu * cus;
        if (grid > ntiles)
            grid = ntiles;
        if (grid > kDyMaxBlocks)
            grid = kDyMaxBlocks;
        if (grid < 1)
            grid = 1;
        hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(block), 0, s, a);
        *n_blocks = (int)grid;
        return hipGetLastError();
    };
    if (ls.block == 512 && ls.ppt == 1)
        return go(dy_dma_kernel<V, 512, 1>, 512, 1);
    if (ls.block == 512 && ls.ppt == 2)
        return go(dy_dma_kernel<V, 512, 2>, 512, 2);
    if (ls.block == 256 && ls.ppt == 2)
        return go(dy_dma_kernel<V, 256, 2>, 256, 2);
    return hipErrorInvalidValue;
}

}  // namespace

bool dy_shape_supported(LaunchShape ls)
{
    return (ls.block == 512 && (ls.ppt == 1 || ls.ppt == 2)) || (ls.block == 256 && ls.ppt == 2);
}

bool dy_dma_supported(int nx, int nq, int na, int nbx, int nbq)
{
    return nx >= 4 && nq >= 4 && na >= 2 && nx * nq <= kDmaNodes && nx + nq + na <= kDmaKnots &&
           nbx + nbq <= kDmaSeeds;
}

hipError_t launch_dy_dma_forward(const DyArgs &a, bool f32, LaunchShape ls, int cus,
                                 hipStream_t s, int *n_blocks)
{
    return f32 ? dy_dma_typed<float>(a, ls, cus, s, n_blocks)
               : dy_dma_typed<double>(a, ls, cus, s, n_blocks);
}

}  // namespace pdfx
