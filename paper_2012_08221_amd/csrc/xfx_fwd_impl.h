// Forward kernel template: batched x f(x, Q^2) on gfx950.
//
// One persistent workgroup per compute unit (or a few) walks point tiles of
// BLOCK*PPT points:
//   * once per workgroup: the axis tables (raw knots, bucket seeds, interval
//     records) are copied to LDS, and the first requested flavour's slab is
//     staged;
//   * per tile: each thread streams its PPT points (coalesced FP64 x and Q^2),
//     checks the domain, locates them (bucket seed + walk on raw knot values,
//     in LDS), forms ln x, ln Q^2 and the 4+4 folded Hermite weights; this
//     per-point state stays in registers for the whole tile;
//   * per requested flavour: every point does its 16-tap stencil out of the
//     LDS slab and stores x f; meanwhile the next flavour's slab is fetched
//     into registers and written to the second LDS buffer afterwards, so one
//     barrier per flavour separates the buffers' uses (double buffering).
// Slabs are stored in HBM already bordered ((n_x+2) x (n_q+2), zero border one
// knot wide), so staging is a straight copy of 16-byte chunks and a stencil
// hanging over an axis end reads 0 under a weight of exactly 0.
// This is gather-plus-stencil work with no contraction: no MFMA.
#pragma once

#include "pdfx_internal.h"

namespace pdfx {
namespace fwd {

struct LAxis {
    const double *k;
    const uint16_t *seed;
    const IntervalRec<double> *r64;
    const IntervalRec<float> *r32;
    int n, nb;
    double ln_lo, inv_hb;
};

__device__ __forceinline__ LAxis lds_axis(char *sm, const AxisDev &a, const AxisLds &o)
{
    LAxis l;
    l.k = reinterpret_cast<const double *>(sm + o.knots);
    l.seed = reinterpret_cast<const uint16_t *>(sm + o.seed);
    l.r64 = reinterpret_cast<const IntervalRec<double> *>(sm + o.rec64);
    l.r32 = reinterpret_cast<const IntervalRec<float> *>(sm + o.rec32);
    l.n = a.n;
    l.nb = a.nbuckets;
    l.ln_lo = a.ln_lo;
    l.inv_hb = a.inv_hb;
    return l;
}

template <int BLOCK>
__device__ __forceinline__ void copy_words(char *dst, const void *src, int bytes)
{
    const uint2 *s = reinterpret_cast<const uint2 *>(src);
    uint2 *d = reinterpret_cast<uint2 *>(dst);
    for (int i = threadIdx.x; i < bytes / 8; i += BLOCK)
        d[i] = s[i];
}

template <int BLOCK>
__device__ __forceinline__ void load_axis(char *sm, const AxisDev &a, const AxisLds &o, bool f32)
{
    copy_words<BLOCK>(sm + o.knots, a.knots, a.n * 8);
    copy_words<BLOCK>(sm + o.seed, a.seed, a.nbuckets * 2);
    copy_words<BLOCK>(sm + o.rec64, a.rec64, (a.n - 1) * 64);
    if (f32)
        copy_words<BLOCK>(sm + o.rec32, a.rec32, (a.n - 1) * 32);
}

// Largest i with k[i] <= v, clamped to n-2 (v inside [k[0], k[n-1]]).  The
// bucket seed only chooses where the walks start.
__device__ __forceinline__ int lbin(const LAxis &a, double v, double lnv)
{
    const double fb = (lnv - a.ln_lo) * a.inv_hb;
    const int b = fb <= 0.0 ? 0 : (fb >= (double)(a.nb - 1) ? a.nb - 1 : (int)fb);
    int i = a.seed[b];
    while (i < a.n - 2 && a.k[i + 1] <= v)
        ++i;
    while (i > 0 && a.k[i] > v)
        --i;
    return i;
}

template <typename W>
__device__ __forceinline__ void fold(W t, W pl, W plql, W ql, W qr, W qrpr, W pr, W w[4])
{
    const W t2 = t * t;
    const W t3 = t2 * t;
    const W h00 = W(2) * t3 - W(3) * t2 + W(1);
    const W h10 = t3 - W(2) * t2 + t;
    const W h01 = W(-2) * t3 + W(3) * t2;
    const W h11 = t3 - t2;
    w[0] = -h10 * pl;
    w[1] = h00 + h10 * plql - h11 * qr;
    w[2] = h01 + h10 * ql + h11 * qrpr;
    w[3] = h11 * pr;
}

template <typename W>
__device__ __forceinline__ void weights(const LAxis &a, int i, double lnv, W w[4]);

template <>
__device__ __forceinline__ void weights<double>(const LAxis &a, int i, double lnv, double w[4])
{
    const IntervalRec<double> r = a.r64[i];
    const double t = (lnv - r.z) * r.inv_d;
    fold<double>(t, r.pl, r.plql, r.ql, r.qr, r.qrpr, r.pr, w);
}

template <>
__device__ __forceinline__ void weights<float>(const LAxis &a, int i, double lnv, float w[4])
{
    const double z = a.r64[i].z;
    const double inv_d = a.r64[i].inv_d;
    const IntervalRec<float> r = a.r32[i];
    const float t = (float)((lnv - z) * inv_d);
    fold<float>(t, r.pl, r.plql, r.ql, r.qr, r.qrpr, r.pr, w);
}

template <typename V>
__device__ __forceinline__ V quiet_nan();
template <>
__device__ __forceinline__ double quiet_nan<double>() { return __builtin_nan(""); }
template <>
__device__ __forceinline__ float quiet_nan<float>() { return __builtin_nanf(""); }

// Clamp or flag a point; true if it is evaluated.
__device__ __forceinline__ bool domain(const XfxArgs &a, double &xv, double &qv)
{
    const bool nan_in = (xv != xv) || (qv != qv);
    const bool inside = xv >= a.ax.lo && xv <= a.ax.hi && qv >= a.aq.lo && qv <= a.aq.hi;
    if (inside)
        return true;
    if (a.domain_mode == 1 && !nan_in) {
        xv = fmin(fmax(xv, a.ax.lo), a.ax.hi);
        qv = fmin(fmax(qv, a.aq.lo), a.aq.hi);
        return true;
    }
    xv = a.ax.lo;
    qv = a.aq.lo;
    return false;
}

__device__ __forceinline__ void count_flagged(bool flagged, unsigned long long *counter)
{
    const unsigned long long m = __ballot(flagged);
    if (m != 0ull && (threadIdx.x & 63) == 0)
        atomicAdd(counter, (unsigned long long)__popcll(m));
}

template <int BLOCK>
__device__ __forceinline__ void stage_sync(uint4 *dst, const uint4 *src, int chunks)
{
    for (int c = threadIdx.x; c < chunks; c += BLOCK)
        dst[c] = src[c];
}

// DB: two slab buffers with register prefetch of PF 16-byte chunks per thread;
// otherwise one buffer restaged synchronously when the flavour changes.
// NU > 0: the results of up to NU distinct flavours stay in registers until
// the tile's flavour loop ends and each point's output row is then written in
// one burst (a row written piecewise across the whole tile would be evicted
// from L2 half-written and rewritten per piece); NU = 0 stores as it goes.
template <typename V, int BLOCK, int PPT, int PF, bool DB, int NU>
__global__ __launch_bounds__(BLOCK) void xfx_kernel(const XfxArgs a)
{
    extern __shared__ uint4 smem4[];
    char *sm = reinterpret_cast<char *>(smem4);
    const int tid = threadIdx.x;
    constexpr bool F32 = sizeof(V) == 4;

    load_axis<BLOCK>(sm, a.ax, a.lx, F32);
    load_axis<BLOCK>(sm, a.aq, a.lq, F32);
    const LAxis lx = lds_axis(sm, a.ax, a.lx);
    const LAxis lq = lds_axis(sm, a.aq, a.lq);

    const int nqp = a.nq + 2;
    const int schunks = a.slab_elems * (int)sizeof(V) / 16;
    const uint4 *gv = reinterpret_cast<const uint4 *>(a.vals);
    uint4 *const buf0 = reinterpret_cast<uint4 *>(sm + a.lds_slab0);
    uint4 *const buf1 = reinterpret_cast<uint4 *>(sm + a.lds_slab1);
    V *out = reinterpret_cast<V *>(a.out);
    const int n_req = a.n_req;
    const int n_u = a.n_u;

    const int64_t tile_pts = (int64_t)BLOCK * PPT;
    const int64_t ntiles = (a.n + tile_pts - 1) / tile_pts;

    int cur = 0;        // buffer holding the slab of a.urow[u] at the top of iteration u
    int staged = -1;    // single-buffer mode: grid row in buf[0]
    if (n_u > 0 && (DB || n_u == 1)) {
        stage_sync<BLOCK>(buf0, gv + (size_t)a.urow[0] * schunks, schunks);
        staged = a.urow[0];
    }
    __syncthreads();

    // prefetched next slab (register staging; kept at kernel scope so that
    // it is initialised once, not per flavour)
    uint4 pf[DB ? PF : 1];
#pragma unroll
    for (int i = 0; i < (DB ? PF : 1); ++i)
        pf[i] = make_uint4(0u, 0u, 0u, 0u);

    // x and Q of the workgroup's next tile are loaded while the current tile
    // runs its flavour loop.
    double xnext[PPT], qnext[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int64_t p = (int64_t)blockIdx.x * tile_pts + tid + (int64_t)j * BLOCK;
        xnext[j] = a.n > 0 ? load_point(a.x, p, a.n) : a.ax.lo;
        qnext[j] = a.n > 0 ? load_point(a.q, p, a.n) : a.aq.lo;
    }

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t p0 = tile * tile_pts + tid;
        V wx[PPT][4], wq[PPT][4];
        int base[PPT];
        bool ok[PPT], live[PPT];
        double xcur[PPT], qcur[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            xcur[j] = xnext[j];
            qcur[j] = qnext[j];
            const int64_t pn = p0 + (int64_t)gridDim.x * tile_pts + (int64_t)j * BLOCK;
            xnext[j] = load_point(a.x, pn, a.n);
            qnext[j] = load_point(a.q, pn, a.n);
        }
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int64_t p = p0 + (int64_t)j * BLOCK;
            live[j] = p < a.n;
            double xv = xcur[j];
            double qv = qcur[j];
            if (a.q_is_q)
                qv = qv * qv;
            ok[j] = domain(a, xv, qv);
            count_flagged(live[j] && !ok[j], a.dom_count);
            const double lnx = log(xv);
            const double lnq = log(qv);
            const int ix = lbin(lx, xv, lnx);
            const int kq = lbin(lq, qv, lnq);
            weights<V>(lx, ix, lnx, wx[j]);
            weights<V>(lq, kq, lnq, wq[j]);
            base[j] = ix * nqp + kq;   // bordered index of knot (ix-1, kq-1)
            for (int z = 0; z < a.n_zero; ++z)
                if (live[j])
                    out[p * n_req + a.zcols[z]] = V(0);
        }

        V res[PPT][NU > 0 ? NU : 1];
#pragma unroll
        for (int u = 0; u < (NU > 0 ? NU : kMaxReq); ++u) {
            if (u < n_u) {
            const int row = a.urow[u];
            bool pre = false;
            if (DB) {
                // fetch the slab needed next (next flavour, or the first
                // flavour of this workgroup's next tile)
                pre = n_u > 1 && (u + 1 < n_u || tile + gridDim.x < ntiles);
                if (pre) {
                    const uint4 *src = gv + (size_t)a.urow[u + 1 < n_u ? u + 1 : 0] * schunks;
#pragma unroll
                    for (int i = 0; i < PF; ++i) {
                        const int c = tid + i * BLOCK;
                        pf[i] = src[c < schunks ? c : schunks - 1];   // in bounds; extra lanes unused
                    }
                }
            } else if (row != staged) {
                __syncthreads();
                stage_sync<BLOCK>(buf0, gv + (size_t)row * schunks, schunks);
                __syncthreads();
                staged = row;
            }
            const V *slab = reinterpret_cast<const V *>(cur ? buf1 : buf0);
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const V *s0 = slab + base[j];
                V acc;
#pragma unroll
                for (int jx = 0; jx < 4; ++jx) {
                    const V *s = s0 + jx * nqp;
                    V r = wq[j][0] * s[0];
                    r = fma(wq[j][1], s[1], r);
                    r = fma(wq[j][2], s[2], r);
                    r = fma(wq[j][3], s[3], r);
                    acc = (jx == 0) ? wx[j][0] * r : fma(wx[j][jx], r, acc);
                }
                const V v = ok[j] ? acc : quiet_nan<V>();
                if (NU > 0) {
                    res[j][NU > 0 ? u : 0] = v;
                } else if (live[j]) {
                    const int64_t p = p0 + (int64_t)j * BLOCK;
                    for (int c = a.ucol_off[u]; c < a.ucol_off[u + 1]; ++c)
                        out[p * n_req + a.ucols[c]] = v;
                }
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
        }
        if (NU > 0) {
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                V *orow = out + (p0 + (int64_t)j * BLOCK) * n_req;
#pragma unroll
                for (int u = 0; u < (NU > 0 ? NU : 1); ++u) {
                    if (live[j] && u < n_u) {
                        for (int c = a.ucol_off[u]; c < a.ucol_off[u + 1]; ++c)
                            orow[a.ucols[c]] = res[j][u];
                    }
                }
            }
        }
    }
}

// Compiled launch shapes (block, points per thread).
// ppt < 0 selects the store-as-you-go kernels (see with_variant).
// Every register-result shape has a store-as-you-go twin (requests with more
// than kRegCols distinct flavours switch to it).
constexpr LaunchShape kShapes[] = {{256, 2}, {256, 4}, {512, 1}, {512, 2}, {1024, 1},
                                   {256, -2}, {256, -4}, {256, -8}, {512, -1}, {512, -2},
                                   {512, -4}, {1024, -1}, {1024, -2}};
// Distinct flavours whose results a thread holds in registers.
constexpr int kRegCols = 12;

// Prefetch depth: smallest of {4, 8, 12} chunks per thread that covers a slab.
inline int pick_pf(int block, int schunks)
{
    for (int pf : {4, 8, 12})
        if (pf * block >= schunks)
            return pf;
    return 0;
}

#define PDFX_FWD_PF(V, B, P, NU)                                                   \
    do {                                                                           \
        if (!db)                                                                   \
            return call(xfx_kernel<V, B, P, 1, false, NU>, B, P);                  \
        switch (pick_pf(B, schunks)) {                                             \
        case 4: return call(xfx_kernel<V, B, P, 4, true, NU>, B, P);               \
        case 8: return call(xfx_kernel<V, B, P, 8, true, NU>, B, P);               \
        case 12: return call(xfx_kernel<V, B, P, 12, true, NU>, B, P);             \
        default: return call(xfx_kernel<V, B, P, 1, false, NU>, B, P);             \
        }                                                                          \
    } while (0)

// Applies `call(kernel, block, ppt)` to the kernel instance for shape ls.
// ls.ppt > 0: results of up to kRegCols distinct flavours held in registers
// and written per point at the end of the tile; ls.ppt < 0: |ppt| points per
// thread, results stored as each flavour completes.  Requests with more than
// kRegCols distinct flavours always store as they go.
template <typename V, typename Call>
hipError_t with_variant(const XfxArgs &a, LaunchShape ls, bool db, Call call)
{
    const int schunks = a.slab_elems * (int)sizeof(V) / 16;
    if (a.n_u > kRegCols && ls.ppt > 0)
        ls.ppt = -ls.ppt;
    if (ls.block == 256 && ls.ppt == 2) PDFX_FWD_PF(V, 256, 2, kRegCols);
    if (ls.block == 256 && ls.ppt == 4) PDFX_FWD_PF(V, 256, 4, kRegCols);
    if (ls.block == 512 && ls.ppt == 1) PDFX_FWD_PF(V, 512, 1, kRegCols);
    if (ls.block == 512 && ls.ppt == 2) PDFX_FWD_PF(V, 512, 2, kRegCols);
    if (ls.block == 1024 && ls.ppt == 1) PDFX_FWD_PF(V, 1024, 1, kRegCols);
    if (ls.block == 256 && ls.ppt == -2) PDFX_FWD_PF(V, 256, 2, 0);
    if (ls.block == 256 && ls.ppt == -4) PDFX_FWD_PF(V, 256, 4, 0);
    if (ls.block == 256 && ls.ppt == -8) PDFX_FWD_PF(V, 256, 8, 0);
    if (ls.block == 512 && ls.ppt == -1) PDFX_FWD_PF(V, 512, 1, 0);
    if (ls.block == 512 && ls.ppt == -2) PDFX_FWD_PF(V, 512, 2, 0);
    if (ls.block == 512 && ls.ppt == -4) PDFX_FWD_PF(V, 512, 4, 0);
    if (ls.block == 1024 && ls.ppt == -1) PDFX_FWD_PF(V, 1024, 1, 0);
    if (ls.block == 1024 && ls.ppt == -2) PDFX_FWD_PF(V, 1024, 2, 0);
    return hipErrorInvalidValue;
}

#undef PDFX_FWD_PF

template <typename V>
hipError_t launch_typed(const XfxArgs &a0, LaunchShape ls, int max_blocks, hipStream_t s)
{
    XfxArgs a = a0;
    bool db = false;
    const size_t lds = xfx_lds_layout(a, sizeof(V) == 4, &db);
    if (lds == 0)
        return hipErrorInvalidValue;
    return with_variant<V>(a, ls, db, [&](auto fn, int block, int ppt) -> hipError_t {
        const int64_t tile_pts = (int64_t)block * (ppt < 0 ? -ppt : ppt);
        const int64_t ntiles = (a.n + tile_pts - 1) / tile_pts;
        int64_t grid = ntiles < max_blocks ? ntiles : max_blocks;
        if (grid < 1)
            grid = 1;
        if (lds > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
            if (e != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(block), lds, s, a);
        return hipGetLastError();
    });
}

template <typename V>
hipError_t occupancy_typed(const XfxArgs &a0, LaunchShape ls, int *blocks_per_cu)
{
    XfxArgs a = a0;
    bool db = false;
    const size_t lds = xfx_lds_layout(a, sizeof(V) == 4, &db);
    if (lds == 0)
        return hipErrorInvalidValue;
    return with_variant<V>(a, ls, db, [&](auto fn, int block, int) -> hipError_t {
        if (lds > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
            if (e != hipSuccess)
                return e;
        }
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu,
                                                            reinterpret_cast<const void *>(fn),
                                                            block, lds);
    });
}

}  // namespace fwd
}  // namespace pdfx
