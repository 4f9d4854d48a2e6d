// Double-buffered evaluation of a PDF set: many members with uneven grids
// (PDF sets are collections of members, Sec. 1), all at the same points.
//
// Each member's grid is stored as borderless flavour-group node slabs whose
// node width NB (16, 8 or 4 bytes: G = NB / sizeof(value) flavours per node)
// is the widest for which two slabs of the member fit the static LDS; the
// members of one node width (or split layout) form a class.  One persistent
// launch walks a single work list of (member, run of point tiles) items,
// dearest classes first, taken from an atomic cursor; each item runs its
// class's body.  Per item the workgroup loads the member's knots and bucket seeds
// into LDS; per tile it locates its points in the member's grid, walks the
// request's flavour groups with the next group's slab copied into the spare
// LDS slab by global-to-LDS loads (one barrier per stage), keeps the results
// in registers and writes the tile's output rows, assembled in LDS, as
// 16-byte chunks.  Members too large for any width keep the single-slab set
// kernel (members.hip).
#include "set_internal.h"
#include "xfx_dma_impl.h"

namespace pdfx {

namespace {

// G = NB / sizeof(V) values of one node from LDS.
template <typename V, int NB>
__device__ __forceinline__ void node_get(const char *p, V *v);
template <>
__device__ __forceinline__ void node_get<double, 16>(const char *p, double *v)
{
    const double2 d = *reinterpret_cast<const double2 *>(p);
    v[0] = d.x;
    v[1] = d.y;
}
template <>
__device__ __forceinline__ void node_get<double, 8>(const char *p, double *v)
{
    v[0] = *reinterpret_cast<const double *>(p);
}
template <>
__device__ __forceinline__ void node_get<float, 16>(const char *p, float *v)
{
    const float4 d = *reinterpret_cast<const float4 *>(p);
    v[0] = d.x;
    v[1] = d.y;
    v[2] = d.z;
    v[3] = d.w;
}
template <>
__device__ __forceinline__ void node_get<float, 8>(const char *p, float *v)
{
    const float2 d = *reinterpret_cast<const float2 *>(p);
    v[0] = d.x;
    v[1] = d.y;
}
template <>
__device__ __forceinline__ void node_get<float, 4>(const char *p, float *v)
{
    v[0] = *reinterpret_cast<const float *>(p);
}

__global__ void reset_cursor(unsigned int *c) { *c = 0u; }

template <typename W>
__device__ __forceinline__ void weights_g(const AxisDev &ax, int i, double lnv, W w[4]);

template <>
__device__ __forceinline__ void weights_g<double>(const AxisDev &ax, int i, double lnv, double w[4])
{
    gptr<double> r = (gptr<double>)(ax.rec64 + i);   // z, 1/d, pl, pl-ql, ql, qr, qr-pr, pr
    const double t = (lnv - r[0]) * r[1];
    fwd::fold<double>(t, r[2], r[3], r[4], r[5], r[6], r[7], w);
}

template <>
__device__ __forceinline__ void weights_g<float>(const AxisDev &ax, int i, double lnv, float w[4])
{
    gptr<double> r64 = (gptr<double>)(ax.rec64 + i);
    gptr<float> r = (gptr<float>)(ax.rec32 + i);
    const float t = (float)((lnv - r64[0]) * r64[1]);
    fwd::fold<float>(t, r[2], r[3], r[4], r[5], r[6], r[7], w);
}

// LDS of the set kernel, shared by every class body.
struct SetLds {
    uint4 *slab0, *slab1;
    double *knots;
    uint16_t *seeds;
};

// One work item of class (NB, SPLIT): a run of point tiles of member m.
// SPLIT: the member's group slab (8- or 16-byte nodes) is too large for one
// LDS slab; its rows [0, split_rows) go to slab0 and the rest to slab1, so a
// stage holds one group in both slabs, copied while no stencil runs.
// `loaded` is the member whose knots and seeds are in LDS (kept across items).
template <typename V, int NB, bool SPLIT, int BLOCK, int PPT>
__device__ __forceinline__ void set_item(const SetDmaArgs &a, const SetPlan &pl, const SetLds sh,
                                         int m, int item, int mi, int &loaded, fwd::LAxis &lx,
                                         fwd::LAxis &lq)
{
    constexpr int G = NB / (int)sizeof(V);
    constexpr int NS = kGrpMaxSlots / G;
    constexpr int NSG = NS * G;
    constexpr bool F32 = sizeof(V) == 4;
    uint4 *const slab0 = sh.slab0;
    uint4 *const slab1 = sh.slab1;
    const int tid = threadIdx.x;
    const int prec = F32 ? 1 : 0;
    const int n_req = a.n_req;
    const int n_stage = pl.n_stage;
    const int64_t tile_pts = (int64_t)BLOCK * PPT;
    const int64_t ntiles = (a.n + tile_pts - 1) / tile_pts;
    const int64_t t_first = (int64_t)(item - mi * a.items_per_member) * a.tiles_per_item;
    const int64_t t_end = t_first + a.tiles_per_item < ntiles ? t_first + a.tiles_per_item : ntiles;
    const SetMemberDev &md = a.mem[m];
    const int nx = md.nx, nq = md.nq;
    const int chunks = (nx * nq * NB + 15) / 16;   // 16-byte chunks per slab
    const uint4 *gsrc = reinterpret_cast<const uint4 *>(md.gvals[prec]);
    const size_t gstride = (size_t)md.gstride[prec] * NB / 16;   // chunks per group
    // split layout: rows below r_split in slab0, the others in slab1
    const int r_split = SPLIT ? md.split_rows[prec] : nx;
    const int chunks0 = SPLIT ? r_split * nq * NB / 16 : chunks;   // r_split * nq is even
    const int chunks1 = SPLIT ? chunks - chunks0 : 0;
    auto load_group = [&](int grp) {
        const uint4 *src = gsrc + (size_t)grp * gstride;
        fwd::dma_slab<BLOCK>(slab0, src, chunks0);
        if (SPLIT)
            fwd::dma_slab<BLOCK>(slab1, src + chunks0, chunks1);
    };
    if (n_stage > 0)
        load_group(pl.sgrp[0]);
    if (m != loaded) {
        copy_words_g(reinterpret_cast<char *>(sh.knots), md.ax.knots, nx * 8, BLOCK);
        copy_words_g(reinterpret_cast<char *>(sh.knots + nx), md.aq.knots, nq * 8, BLOCK);
        copy_words_g(reinterpret_cast<char *>(sh.seeds), md.ax.seed, md.ax.nbuckets * 2, BLOCK);
        copy_words_g(reinterpret_cast<char *>(sh.seeds + md.ax.nbuckets), md.aq.seed,
                     md.aq.nbuckets * 2, BLOCK);
        lx.k = sh.knots;
        lx.seed = sh.seeds;
        lx.n = nx;
        lx.nb = md.ax.nbuckets;
        lx.ln_lo = md.ax.ln_lo;
        lx.inv_hb = md.ax.inv_hb;
        lq.k = sh.knots + nx;
        lq.seed = sh.seeds + md.ax.nbuckets;
        lq.n = nq;
        lq.nb = md.aq.nbuckets;
        lq.ln_lo = md.aq.ln_lo;
        lq.inv_hb = md.aq.inv_hb;
        loaded = m;
        __syncthreads();
    }
    V *out = reinterpret_cast<V *>(a.out) + (int64_t)m * a.n * n_req;

    // each tile's coordinates are loaded during the first stage of the tile
    // before (clamped to the last point), so that its location does not wait
    // for them
    double x_pf[PPT], q_pf[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int64_t p = t_first * tile_pts + tid + (int64_t)j * BLOCK;
        x_pf[j] = load_point(a.x, p, a.n);
        q_pf[j] = load_point(a.q, p, a.n);
    }

    for (int64_t tile = t_first; tile < t_end; ++tile) {
        const int64_t t0 = tile * tile_pts;
        const bool more = tile + 1 < t_end;
        if (SPLIT && tile > t_first && n_stage > 0) {
            __syncthreads();   // the previous tile's output rows have left both slabs
            load_group(pl.sgrp[0]);
        }
        V wx[PPT][4], wq[PPT][4];
        int base[PPT], brow[PPT];
        bool ok[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int64_t p = t0 + tid + (int64_t)j * BLOCK;
            double xv = x_pf[j];
            double qv = q_pf[j];
            const bool nan_in = (xv != xv) || (qv != qv);
            const bool inside = xv >= md.ax.lo && xv <= md.ax.hi && qv >= md.aq.lo &&
                                qv <= md.aq.hi;
            ok[j] = true;
            if (!inside) {
                if (a.domain_mode == 1 && !nan_in) {
                    xv = fmin(fmax(xv, md.ax.lo), md.ax.hi);
                    qv = fmin(fmax(qv, md.aq.lo), md.aq.hi);
                } else {
                    ok[j] = false;
                    xv = md.ax.lo;
                    qv = md.aq.lo;
                }
            }
            fwd::count_flagged(p < a.n && !ok[j], a.dom_count);
            const double lnx = log(xv), lnq = log(qv);
            const int ix = fwd::lbin(lx, xv, lnx);
            const int kq = fwd::lbin(lq, qv, lnq);
            weights_g<V>(md.ax, ix, lnx, wx[j]);
            weights_g<V>(md.aq, kq, lnq, wq[j]);
            brow[j] = fwd::window(ix, nx, wx[j]);
            base[j] = fwd::window(kq, nq, wq[j]);   // column; the row is brow
            if (!SPLIT)
                base[j] += brow[j] * nq;
        }
        if (n_stage == 0 && more)   // no stage to load the next tile's points in
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const int64_t pn = t0 + tile_pts + tid + (int64_t)j * BLOCK;
                x_pf[j] = load_point(a.x, pn, a.n);
                q_pf[j] = load_point(a.q, pn, a.n);
            }

        fwd::wait_vm();
        __syncthreads();   // the tile's first group has landed

        V res[PPT][NSG];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (s < n_stage) {
                const bool last = s + 1 == n_stage;
                const char *cur = reinterpret_cast<const char *>((s & 1) && !SPLIT ? slab1 : slab0);
                if (SPLIT && s > 0) {
                    __syncthreads();   // the previous group's stencils are done
                    load_group(pl.sgrp[s]);
                    fwd::wait_vm();
                    __syncthreads();
                }
                if (!SPLIT && !last)
                    fwd::dma_slab<BLOCK>((s & 1) ? slab0 : slab1,
                                         gsrc + (size_t)pl.sgrp[s + 1] * gstride, chunks);
                if (s == 0 && more)
#pragma unroll
                    for (int j = 0; j < PPT; ++j) {
                        const int64_t pn = t0 + tile_pts + tid + (int64_t)j * BLOCK;
                        x_pf[j] = load_point(a.x, pn, a.n);
                        q_pf[j] = load_point(a.q, pn, a.n);
                    }
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    V acc[G];
#pragma unroll
                    for (int jx = 0; jx < 4; ++jx) {
                        const char *rowp;
                        if (SPLIT) {
                            const int r = brow[j] + jx;
                            const bool hi = r >= r_split;
                            rowp = reinterpret_cast<const char *>(hi ? slab1 : slab0) +
                                   (size_t)((hi ? r - r_split : r) * nq + base[j]) * NB;
                        } else {
                            rowp = cur + (size_t)(base[j] + jx * nq) * NB;
                        }
                        V r[G];
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            V v[G];
                            node_get<V, NB>(rowp + k * NB, v);
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
                        res[j][s * G + g] = ok[j] ? acc[g] : fwd::quiet_nan<V>();
                }
                if (!SPLIT && !last) {
                    fwd::wait_vm();
                    __syncthreads();
                }
            }
        }

        // Output rows, assembled in both slabs (rows [0, cap) of a pass in
        // slab1, the next cap in slab0; cap is a multiple of 16 rows) and
        // written as 16-byte chunks, slab0's part first: on the last pass
        // the next tile's first group then goes into slab0 while slab1's
        // part is written.
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
                        if (k < n_stage * G && pl.slot_col[k] >= 0)
                            r[pl.slot_col[k]] = res[j][k];
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
            // slab0 is re-filled when it held another group or output rows
            if (!SPLIT && pa + 2 * cap >= valid && more &&
                (n_stage > 1 || (n_stage == 1 && valid > cap))) {
                if (pn > n1)
                    __syncthreads();   // slab0's rows are read
                fwd::dma_slab<BLOCK>(slab0, gsrc + (size_t)pl.sgrp[0] * gstride, chunks);
            }
            write_rows(slab1, dst, n1 * rb);
        }
    }
}

// The set kernel: one persistent launch over the work list of every class.
// Each item names its member's class, and the workgroup runs that class's
// body (node width NB, split or not); all bodies share the LDS arrays.
template <typename V, int BLOCK, int PPT>
__global__ __launch_bounds__(BLOCK) void set_dma_kernel(const SetDmaArgs a)
{
    constexpr bool F32 = sizeof(V) == 4;
    __shared__ uint4 slab0[kSetSlabBytes / 16];
    __shared__ uint4 slab1[kSetSlabBytes / 16];
    __shared__ double knots[kSetKnots];
    __shared__ uint16_t seeds[kSetSeeds];
    __shared__ int s_item;
    const SetLds sh{slab0, slab1, knots, seeds};
    int loaded = -1;
    fwd::LAxis lx, lq;
    for (;;) {
        if (threadIdx.x == 0)
            s_item = (int)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= a.n_items)
            break;
        const int mi = item / a.items_per_member;
        const int2 mc = a.ids[mi];
        const int m = mc.x;
        switch (mc.y) {
        case 0:   // 16-byte nodes, G = 2 (FP64) or 4 (FP32)
            set_item<V, 16, false, BLOCK, PPT>(a, a.plan[F32 ? 2 : 1], sh, m, item, mi, loaded,
                                               lx, lq);
            break;
        case 1:   // 8-byte nodes, G = 1 or 2
            set_item<V, 8, false, BLOCK, PPT>(a, a.plan[F32 ? 1 : 0], sh, m, item, mi, loaded,
                                              lx, lq);
            break;
        case 2:   // 4-byte nodes (FP32 only), G = 1
            if constexpr (F32)
                set_item<V, 4, false, BLOCK, PPT>(a, a.plan[0], sh, m, item, mi, loaded, lx, lq);
            break;
        case 3:   // 8-byte nodes split over both slabs
            set_item<V, 8, true, BLOCK, PPT>(a, a.plan[F32 ? 1 : 0], sh, m, item, mi, loaded,
                                             lx, lq);
            break;
        default:  // 16-byte nodes split over both slabs
            set_item<V, 16, true, BLOCK, PPT>(a, a.plan[F32 ? 2 : 1], sh, m, item, mi, loaded,
                                              lx, lq);
            break;
        }
    }
}

constexpr LaunchShape kSetDmaShapes[] = {{512, 1}, {512, 2}, {256, 2}};

template <typename V>
hipError_t launch_typed(const SetDmaArgs &a, LaunchShape ls, int cus, hipStream_t s)
{
    auto go = [&](auto fn, int block) -> hipError_t {
        int64_t grid = cus;   // one resident workgroup per compute unit (LDS)
        if (grid > a.n_items)
            grid = a.n_items;
        if (grid < 1)
            grid = 1;
        hipLaunchKernelGGL(reset_cursor, dim3(1), dim3(1), 0, s, a.counter);
        hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(block), 0, s, a);
        return hipGetLastError();
    };
    if (ls.block == 512 && ls.ppt == 1)
        return go(set_dma_kernel<V, 512, 1>, 512);
    if (ls.block == 512 && ls.ppt == 2)
        return go(set_dma_kernel<V, 512, 2>, 512);
    if (ls.block == 256 && ls.ppt == 2)
        return go(set_dma_kernel<V, 256, 2>, 256);
    if constexpr (sizeof(V) == 4) {
        if (ls.block == 512 && ls.ppt == 4)
            return go(set_dma_kernel<V, 512, 4>, 512);
    }
    return hipErrorInvalidValue;
}

}  // namespace

int set_split_rows(int nx, int nq, int nbx, int nbq, int nb)
{
    if (nx < 4 || nq < 4 || nx + nq > kSetKnots || nbx + nbq > kSetSeeds)
        return 0;
    int r = kSetSlabBytes / (nq * nb);
    if ((r * nq * nb) % 16)
        --r;   // slab0 ends on a 16-byte chunk
    if (r < 1 || r >= nx || (nx - r) * nq * nb > kSetSlabBytes)
        return 0;
    return r;
}

int set_node_bytes(int nx, int nq, int nbx, int nbq, bool f32)
{
    if (nx < 4 || nq < 4 || nx + nq > kSetKnots || nbx + nbq > kSetSeeds)
        return 0;
    const int widths64[] = {16, 8};
    const int widths32[] = {16, 8, 4};
    const int *w = f32 ? widths32 : widths64;
    const int nw = f32 ? 3 : 2;
    for (int i = 0; i < nw; ++i) {
        const int bytes = (nx * nq * w[i] + 15) / 16 * 16;
        if (bytes <= kSetSlabBytes)
            return w[i];
    }
    return 0;
}

bool set_dma_shape_supported(LaunchShape ls, bool f32)
{
    if (f32 && ls.block == 512 && ls.ppt == 4)
        return true;
    for (const auto &k : kSetDmaShapes)
        if (k.block == ls.block && k.ppt == ls.ppt)
            return true;
    return false;
}

hipError_t launch_set_dma(const SetDmaArgs &a, bool f32, LaunchShape ls, int cus, hipStream_t s)
{
    return f32 ? launch_typed<float>(a, ls, cus, s) : launch_typed<double>(a, ls, cus, s);
}

}  // namespace pdfx
