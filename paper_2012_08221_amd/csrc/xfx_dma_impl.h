// Double-buffered flavour-group forward kernel: batched x f(x, Q^2) on gfx950
// for grids of up to kDmaNodes knots (n_x * n_q).
//
// Same flavour groups and 16-byte nodes as the single-buffer grouped kernel,
// but the node slabs carry no border and two of them live in LDS: while the
// points run their stencils out of one slab, the next group's slab is copied
// into the other by global-to-LDS loads (global_load_lds_dwordx4), which
// need no registers and no LDS write instructions.  One barrier per stage
// publishes the new slab.  The slabs are two distinct __shared__ arrays,
// addressed with the buffer fixed at compile time for every stage, so the
// compiler can tell that a stencil read of one slab does not depend on a copy
// into the other and does not wait for it.
//
// Without a border, a 4-knot window that would hang over an axis end is
// moved inside the axis and its weights move with it: the weight that falls
// off is exactly 0 there (one-sided end slopes), so the sum is unchanged.
//
// Per tile of BLOCK*PPT points: prologue (locate, weights; the next tile's
// first slab is still landing meanwhile), one stencil stage per touched
// group, then the output rows are assembled in the spare slab and written
// as 16-byte chunks.  The interval records are read from global memory
// (L1/L2 resident); knots and bucket seeds are in LDS.
#pragma once

#include "xfx_grouped_impl.h"

namespace pdfx {
namespace fwd {

// Static LDS capacity: two slabs of kDmaNodes 16-byte nodes, knots of both
// axes and bucket seeds of both axes (160 KB in all).
constexpr int kDmaNodes = 5000;
constexpr int kDmaKnots = 240;
constexpr int kDmaSeeds = 960;

// Folded Hermite weights from the interval records in global memory.
template <typename W>
__device__ __forceinline__ void weights_gmem(const AxisDev &ax, int i, double lnv, W w[4]);

template <>
__device__ __forceinline__ void weights_gmem<double>(const AxisDev &ax, int i, double lnv, double w[4])
{
    const IntervalRec<double> r = ax.rec64[i];
    const double t = (lnv - r.z) * r.inv_d;
    fold<double>(t, r.pl, r.plql, r.ql, r.qr, r.qrpr, r.pr, w);
}

template <>
__device__ __forceinline__ void weights_gmem<float>(const AxisDev &ax, int i, double lnv, float w[4])
{
    const double z = ax.rec64[i].z;
    const double inv_d = ax.rec64[i].inv_d;
    const IntervalRec<float> r = ax.rec32[i];
    const float t = (float)((lnv - z) * inv_d);
    fold<float>(t, r.pl, r.plql, r.ql, r.qr, r.qrpr, r.pr, w);
}

// First knot of the 4-knot window of interval i on an axis of n >= 4 knots,
// kept inside the axis; w (weights of knots i-1 .. i+2) is moved to match.
template <typename W>
__device__ __forceinline__ int window(int i, int n, W w[4])
{
    int st = i - 1;
    if (st < 0) {
        st = 0;
        w[0] = w[1];
        w[1] = w[2];
        w[2] = w[3];
        w[3] = W(0);
    } else if (st > n - 4) {
        st = n - 4;
        w[3] = w[2];
        w[2] = w[1];
        w[1] = w[0];
        w[0] = W(0);
    }
    return st;
}

// Starts copying one node slab (nodes 16-byte chunks) from global memory into
// a __shared__ slab: wave w moves the 64-node blocks w, w + BLOCK/64, ...
// Each lane's 16 bytes land at the block start plus 16 * lane; lanes past the
// end are masked off.  Completion is tracked by vmcnt.
template <int BLOCK>
__device__ __forceinline__ void dma_slab(uint4 *dst, const uint4 *src, int nodes)
{
    const int lane = threadIdx.x & 63;
    for (int b = __builtin_amdgcn_readfirstlane(threadIdx.x & ~63); b < nodes; b += BLOCK)
        if (b + lane < nodes)
            __builtin_amdgcn_global_load_lds(
                (const __attribute__((address_space(1))) void *)(src + b + lane),
                (__attribute__((address_space(3))) void *)(dst + b), 16, 0, 0);
}

// Domain rule of the forward kernels with the Q^2 coordinate judged on its
// own as well, for alpha_s at the same point: returns whether x f is defined
// (as domain() does) and sets q_ok to whether alpha_s is (Q^2 inside, or
// clamped and not NaN).  Each out-of-range coordinate is replaced on its own,
// so a valid Q^2 keeps its value when only x is outside.
__device__ __forceinline__ bool domain_xq(const XfxArgs &a, double &xv, double &qv, bool &q_ok)
{
    const bool x_in = xv >= a.ax.lo && xv <= a.ax.hi;   // false for NaN
    const bool q_in = qv >= a.aq.lo && qv <= a.aq.hi;
    if (x_in && q_in) {
        q_ok = true;
        return true;
    }
    const bool x_nan = xv != xv;
    const bool q_nan = qv != qv;
    if (a.domain_mode == 1) {
        xv = x_nan ? a.ax.lo : fmin(fmax(xv, a.ax.lo), a.ax.hi);
        qv = q_nan ? a.aq.lo : fmin(fmax(qv, a.aq.lo), a.aq.hi);
        q_ok = !q_nan;
        return !x_nan && !q_nan;
    }
    if (!x_in)
        xv = a.ax.lo;
    if (!q_in)
        qv = a.aq.lo;
    q_ok = q_in;
    return false;
}

// Wait until this wave's outstanding vector-memory operations (global-to-LDS
// copies included) are complete; other waves read what it copied after the
// barrier that follows.
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// One stencil stage: results of the G flavours of the group in slab for the
// PPT points of this thread.
template <typename V, int PPT>
__device__ __forceinline__ void dma_stage(const uint4 *slab, const int base[PPT], int nq,
                                          const V wx[PPT][4], const V wq[PPT][4],
                                          const bool ok[PPT], V *res_s, int ldres)
{
    constexpr int G = 16 / (int)sizeof(V);
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        V acc[G];
#pragma unroll
        for (int jx = 0; jx < 4; ++jx) {
            const uint4 *rowp = slab + base[j] + jx * nq;
            V r[G];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                V v[G];
                Node<V>::get(rowp + k, v);
#pragma unroll
                for (int g = 0; g < G; ++g)
                    r[g] = (k == 0) ? wq[j][0] * v[g] : fma(wq[j][k], v[g], r[g]);
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
                acc[g] = (jx == 0) ? wx[j][0] * r[g] : fma(wx[j][jx], r[g], acc[g]);
        }
#pragma unroll
        for (int g = 0; g < G; ++g)
            res_s[j * ldres + g] = ok[j] ? acc[g] : quiet_nan<V>();
    }
}

// AS: alpha_s at the same points as well.  The alpha_s knots are the Q^2
// knots, so alpha_s is the Q^2 weights of the point applied to the alpha_s
// values of the same 4-knot window; the values sit in LDS after the knots
// (dma_alphas_fit), and alpha_s is written as soon as the point is located.
template <typename V, int BLOCK, int PPT, bool AS = false>
__global__ __launch_bounds__(BLOCK) void xfx_dma_kernel(const XfxArgs a)
{
    constexpr int G = 16 / (int)sizeof(V);
    constexpr int NS = kGrpMaxSlots / G;
    constexpr int NSG = NS * G;
    __shared__ uint4 slab0[kDmaNodes];
    __shared__ uint4 slab1[kDmaNodes];
    __shared__ double knots[kDmaKnots];
    __shared__ uint16_t seeds[kDmaSeeds];
    const int tid = threadIdx.x;

    const int nx = a.nx, nq = a.nq;
    const int nodes = nx * nq;
    const uint4 *gsrc = reinterpret_cast<const uint4 *>(a.gvals);
    V *out = reinterpret_cast<V *>(a.out);
    const int n_req = a.n_req;
    const int n_stage = a.n_stage;
    const int64_t tile_pts = (int64_t)BLOCK * PPT;
    const int64_t ntiles = (a.n + tile_pts - 1) / tile_pts;
    if ((int64_t)blockIdx.x >= ntiles)
        return;

    // first slab of the first tile, then the search tables
    if (n_stage > 0)
        dma_slab<BLOCK>(slab0, gsrc + (size_t)a.sgrp[0] * a.gstride, nodes);
    copy_words<BLOCK>(reinterpret_cast<char *>(knots), a.ax.knots, nx * 8);
    copy_words<BLOCK>(reinterpret_cast<char *>(knots + nx), a.aq.knots, nq * 8);
    copy_words<BLOCK>(reinterpret_cast<char *>(seeds), a.ax.seed, a.ax.nbuckets * 2);
    copy_words<BLOCK>(reinterpret_cast<char *>(seeds + a.ax.nbuckets), a.aq.seed,
                      a.aq.nbuckets * 2);
    // alpha_s values, padded (a zero before knot 0), after the knots
    const V *asv = reinterpret_cast<const V *>(knots + nx + nq) + 1;
    if constexpr (AS)
        copy_words<BLOCK>(reinterpret_cast<char *>(knots + nx + nq), a.as_vals,
                          ((nq + 2) * (int)sizeof(V) + 7) / 8 * 8);
    __syncthreads();
    LAxis lx, lq;
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

    // Locating a point (domain, logs, bins, weights, window) for point p
    // from its coordinates.
    auto locate = [&](double xv, double qv, int64_t p, V (&ox)[4], V (&oq)[4], int &ob, bool &ook) {
        if (a.q_is_q)
            qv = qv * qv;
        bool q_ok = true;
        if constexpr (AS)
            ook = domain_xq(a, xv, qv, q_ok);
        else
            ook = domain(a, xv, qv);
        count_flagged(p < a.n && !ook, a.dom_count);
        if constexpr (AS)
            count_flagged(p < a.n && !q_ok, a.dom_count);
        const double lnx = log(xv);
        const double lnq = log(qv);
        const int ix = lbin(lx, xv, lnx);
        const int kq = lbin(lq, qv, lnq);
        weights_gmem<V>(a.ax, ix, lnx, ox);
        weights_gmem<V>(a.aq, kq, lnq, oq);
        const int wq0 = window(kq, nq, oq);
        ob = window(ix, nx, ox) * nq + wq0;
        if constexpr (AS) {
            const V *av = asv + wq0;
            V s = oq[0] * av[0];
            s = fma(oq[1], av[1], s);
            s = fma(oq[2], av[2], s);
            s = fma(oq[3], av[3], s);
            if (p < a.n)
                reinterpret_cast<V *>(a.as_out)[p] = q_ok ? s : quiet_nan<V>();
        }
    };

    // Point state of the current tile, and of the next tile (located during
    // the current tile's stencil stages, whose time goes to LDS traffic, so
    // that the location work overlaps it: point j in stage j, or after the
    // stages when there are fewer).  xnext holds the coordinates of the tile
    // after that.
    V wx[PPT][4], wq[PPT][4];
    int base[PPT];
    bool ok[PPT];
    V nwx[PPT][4], nwq[PPT][4];
    int nbase[PPT];
    bool nok[PPT];
    double xnext[PPT], qnext[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int64_t p = (int64_t)blockIdx.x * tile_pts + tid + (int64_t)j * BLOCK;
        locate(load_point(a.x, p, a.n), load_point(a.q, p, a.n), p, wx[j], wq[j], base[j], ok[j]);
        const int64_t pn = p + (int64_t)gridDim.x * tile_pts;
        xnext[j] = load_point(a.x, pn, a.n);
        qnext[j] = load_point(a.q, pn, a.n);
    }

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t t0 = tile * tile_pts;
        const bool more = tile + gridDim.x < ntiles;
        const int64_t pnext0 = t0 + (int64_t)gridDim.x * tile_pts + tid;   // next tile, point 0
        auto locate_next = [&](int j) {
            const int64_t pn = pnext0 + (int64_t)j * BLOCK;
            locate(xnext[j], qnext[j], pn, nwx[j], nwq[j], nbase[j], nok[j]);
            const int64_t pnn = pn + (int64_t)gridDim.x * tile_pts;
            xnext[j] = load_point(a.x, pnn, a.n);
            qnext[j] = load_point(a.q, pnn, a.n);
        };

        // the tile's first slab has landed (copies of every wave)
        wait_vm();
        __syncthreads();

        // Stage s reads slab (s & 1).  The copy for stage s+1 goes into the
        // other slab during stage s.  The next tile's first slab goes into
        // slab0 after the last barrier of the output phase (every barrier
        // also waits for the copies in flight), so that it lands during the
        // output stores.  A lone group stays in slab0 unless output rows were
        // staged over it.
        V res[PPT][NSG];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (s < n_stage) {
                const bool last = s + 1 == n_stage;
                uint4 *const cur = (s & 1) ? slab1 : slab0;
                uint4 *const nxt = (s & 1) ? slab0 : slab1;
                if (!last)
                    dma_slab<BLOCK>(nxt, gsrc + (size_t)a.sgrp[s + 1] * a.gstride, nodes);
                if (s < PPT)
                    locate_next(s);
                V tmp[PPT * G];
                dma_stage<V, PPT>(cur, base, nq, wx, wq, ok, tmp, G);
#pragma unroll
                for (int j = 0; j < PPT; ++j)
#pragma unroll
                    for (int g = 0; g < G; ++g)
                        res[j][s * G + g] = tmp[j * G + g];
                if (!last) {
                    wait_vm();
                    __syncthreads();
                }
            }
        }
#pragma unroll
        for (int j = 0; j < PPT; ++j)
            if (j >= n_stage)
                locate_next(j);

        // Output rows, assembled in both slabs (rows [0, cap) of a pass in
        // slab1, the next cap in slab0) and written as 16-byte chunks; cap is
        // a multiple of 16 rows, so the slab0 part starts on a chunk.  The
        // slab0 part is written first: on the last pass the next tile's first
        // slab then goes into slab0 while slab1's part is written.
        __syncthreads();   // every stencil read is done
        const int valid = (int)(a.n - t0 < tile_pts ? a.n - t0 : tile_pts);
        const int cap = a.out_pass_pts;
        const int rb = n_req * (int)sizeof(V);
        auto write_rows = [&](const uint4 *src, char *dst, int bytes) {
            const int nch = bytes >> 4;
            for (int c = tid; c < nch; c += BLOCK)
                *reinterpret_cast<uint4 *>(dst + c * 16) = src[c];
            if (tid < (bytes & 15) / 4)
                reinterpret_cast<uint32_t *>(dst + nch * 16)[tid] =
                    reinterpret_cast<const uint32_t *>(src + nch)[tid];
        };
        for (int pa = 0; pa < valid; pa += 2 * cap) {
            const int pn = valid - pa < 2 * cap ? valid - pa : 2 * cap;
            if (pa > 0)
                __syncthreads();   // the previous pass has left LDS
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const int lp = tid + j * BLOCK - pa;
                if (lp >= 0 && lp < pn) {
                    V *r = reinterpret_cast<V *>(lp < cap ? slab1 : slab0) +
                           (lp < cap ? lp : lp - cap) * n_req;
#pragma unroll
                    for (int k = 0; k < NSG; ++k)
                        if (k < n_stage * G && a.slot_col[k] >= 0)
                            r[a.slot_col[k]] = res[j][k];
                    for (int z = 0; z < a.n_zero; ++z)
                        r[a.zcols[z]] = V(0);
                    for (int d = 0; d < a.n_dup; ++d)
                        r[a.dup_dst[d]] = r[a.dup_src[d]];
                }
            }
            __syncthreads();
            const int n1 = pn < cap ? pn : cap;   // rows in slab1; pn - n1 in slab0
            char *dst = reinterpret_cast<char *>(out + (t0 + pa) * n_req);   // 16-byte aligned
            if (pn > n1)
                write_rows(slab0, dst + n1 * rb, (pn - n1) * rb);
            // slab0 must be re-filled for the next tile when it held another
            // group (n_stage > 1) or output rows of this tile (valid > cap)
            if (pa + 2 * cap >= valid && more && (n_stage > 1 || (n_stage == 1 && valid > cap))) {
                if (pn > n1)
                    __syncthreads();   // slab0's rows are read
                dma_slab<BLOCK>(slab0, gsrc + (size_t)a.sgrp[0] * a.gstride, nodes);
            }
            write_rows(slab1, dst, n1 * rb);
        }
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                wx[j][k] = nwx[j][k];
                wq[j][k] = nwq[j][k];
            }
            base[j] = nbase[j];
            ok[j] = nok[j];
        }
    }
    wait_vm();
}

// Compiled launch shapes (block, points per thread) of the double-buffered kernel;
// FP32 also has (512, 4): its results take half the registers of FP64's, so
// twice the points per tile fit and the per-tile work is shared by more points.
constexpr LaunchShape kDmaShapes[] = {{256, 2}, {256, 4}, {512, 1}, {512, 2}, {1024, 1}};
constexpr LaunchShape kDmaShapeF32 = {512, 4};

template <typename V, bool AS, typename Call>
hipError_t with_dma_variant(LaunchShape ls, Call call)
{
    if (ls.block == 256 && ls.ppt == 2) return call(xfx_dma_kernel<V, 256, 2, AS>, 256, 2);
    if (ls.block == 256 && ls.ppt == 4) return call(xfx_dma_kernel<V, 256, 4, AS>, 256, 4);
    if (ls.block == 512 && ls.ppt == 1) return call(xfx_dma_kernel<V, 512, 1, AS>, 512, 1);
    if (ls.block == 512 && ls.ppt == 2) return call(xfx_dma_kernel<V, 512, 2, AS>, 512, 2);
    if (ls.block == 1024 && ls.ppt == 1) return call(xfx_dma_kernel<V, 1024, 1, AS>, 1024, 1);
    if constexpr (sizeof(V) == 4) {
        if (ls.block == kDmaShapeF32.block && ls.ppt == kDmaShapeF32.ppt)
            return call(xfx_dma_kernel<V, 512, 4, AS>, 512, 4);
    }
    return hipErrorInvalidValue;
}

template <typename V, bool AS>
hipError_t launch_dma_as(const XfxArgs &a0, LaunchShape ls, int max_blocks, hipStream_t s)
{
    XfxArgs a = a0;
    return with_dma_variant<V, AS>(ls, [&](auto fn, int block, int ppt) -> hipError_t {
        const int64_t tile_pts = (int64_t)block * ppt;
        // whole multiples of 16 output rows that fit one slab
        int64_t pass = (int64_t)kDmaNodes * 16 / ((int64_t)a.n_req * (int64_t)sizeof(V)) / 16 * 16;
        if (pass > tile_pts)
            pass = tile_pts;
        a.out_pass_pts = (int)pass;
        const int64_t ntiles = (a.n + tile_pts - 1) / tile_pts;
        int64_t grid = ntiles < max_blocks ? ntiles : max_blocks;
        if (grid < 1)
            grid = 1;
        hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(block), 0, s, a);
        return hipGetLastError();
    });
}

// a.as_out set: the variant that also writes alpha_s.
template <typename V>
hipError_t launch_dma_typed(const XfxArgs &a, LaunchShape ls, int max_blocks, hipStream_t s)
{
    return a.as_out ? launch_dma_as<V, true>(a, ls, max_blocks, s)
                    : launch_dma_as<V, false>(a, ls, max_blocks, s);
}

template <typename V>
hipError_t dma_occupancy_typed(LaunchShape ls, int *blocks_per_cu)
{
    return with_dma_variant<V, false>(ls, [&](auto fn, int block, int) -> hipError_t {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            blocks_per_cu, reinterpret_cast<const void *>(fn), block, 0);
    });
}

}  // namespace fwd
}  // namespace pdfx
