// Flavour-group forward kernel: batched x f(x, Q^2) on gfx950.
//
// The grid's rows are taken G = 16 / sizeof(V) at a time (2 in FP64, 4 in
// FP32) and interleaved per knot into 16-byte "nodes", one bordered node slab
// of (n_x+2) x (n_q+2) nodes per group, built once when the grid is loaded.
// Every knot of the 4 x 4 stencil is then one aligned 16-byte LDS read
// (ds_read_b128) serving G flavours at once, instead of G pairs of 8-byte
// reads at arbitrary alignment; a request walks only the groups holding its
// flavours ("stages"), ceil(11 / G) of them for the full 11-flavour set.
//
// One persistent workgroup per compute unit walks tiles of BLOCK*PPT points:
//   * per tile: each thread locates its PPT points (as in the per-flavour
//     kernel) and keeps bins and weights in registers;
//   * per stage: while the points run their stencils out of the LDS slab,
//     the next stage's slab is fetched into registers; after a barrier it is
//     written into the (single) LDS slab and a second barrier publishes it;
//   * all stages' results stay in registers and each point's output row is
//     written in one burst at the end of the tile.
// x and Q^2 of the next tile are loaded after the first stage's prefetch, so
// the in-order wait on that prefetch does not also wait on them.
#pragma once

#include "xfx_fwd_impl.h"

namespace pdfx {
namespace fwd {

template <typename V>
struct Node;
template <>
struct Node<double> {
    static __device__ __forceinline__ void get(const uint4 *p, double v[2])
    {
        const double2 d = *reinterpret_cast<const double2 *>(p);
        v[0] = d.x;
        v[1] = d.y;
    }
};
template <>
struct Node<float> {
    static __device__ __forceinline__ void get(const uint4 *p, float v[4])
    {
        const float4 d = *reinterpret_cast<const float4 *>(p);
        v[0] = d.x;
        v[1] = d.y;
        v[2] = d.z;
        v[3] = d.w;
    }
};

template <typename V, int BLOCK, int PPT, int PF>
__global__ __launch_bounds__(BLOCK) void xfx_grp_kernel(const XfxArgs a)
{
    constexpr int G = 16 / (int)sizeof(V);
    constexpr int NS = kGrpMaxSlots / G;          // stages whose results fit in registers
    constexpr bool F32 = sizeof(V) == 4;
    extern __shared__ uint4 smem4[];
    char *sm = reinterpret_cast<char *>(smem4);
    const int tid = threadIdx.x;

    load_axis<BLOCK>(sm, a.ax, a.lx, F32);
    load_axis<BLOCK>(sm, a.aq, a.lq, F32);
    const LAxis lx = lds_axis(sm, a.ax, a.lx);
    const LAxis lq = lds_axis(sm, a.aq, a.lq);

    const int nqp = a.nq + 2;
    const int nodes = (a.nx + 2) * nqp;               // 16-byte chunks per stage
    const uint4 *gsrc = reinterpret_cast<const uint4 *>(a.gvals);
    uint4 *const slab = reinterpret_cast<uint4 *>(sm + a.lds_slab0);
    V *out = reinterpret_cast<V *>(a.out);
    const int n_req = a.n_req;
    const int n_stage = a.n_stage;
    const bool stage_out = a.out_pass_pts > 0;
    const int64_t tile_pts = (int64_t)BLOCK * PPT;
    const int64_t ntiles = (a.n + tile_pts - 1) / tile_pts;

    uint4 pf[PF];
#pragma unroll
    for (int i = 0; i < PF; ++i)
        pf[i] = make_uint4(0u, 0u, 0u, 0u);

    const uint32_t toff = (uint32_t)tid * 16u;   // this thread's byte offset in a prefetch row
    if (n_stage > 0)
        stage_sync<BLOCK>(slab, gsrc + (size_t)a.sgrp[0] * a.gstride, nodes);
    __syncthreads();

    double xnext[PPT], qnext[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int64_t p = (int64_t)blockIdx.x * tile_pts + tid + (int64_t)j * BLOCK;
        xnext[j] = a.n > 0 ? load_point(a.x, p, a.n) : a.ax.lo;
        qnext[j] = a.n > 0 ? load_point(a.q, p, a.n) : a.aq.lo;
    }

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t t0 = tile * tile_pts;
        const int64_t p0 = t0 + tid;
        const bool more = tile + gridDim.x < ntiles;
        V wx[PPT][4], wq[PPT][4];
        int base[PPT];
        bool ok[PPT], live[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int64_t p = p0 + (int64_t)j * BLOCK;
            live[j] = p < a.n;
            double xv = xnext[j];
            double qv = qnext[j];
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
            base[j] = ix * nqp + kq;   // node of knot (ix-1, kq-1) in the bordered layout
            if (!stage_out)
                for (int z = 0; z < a.n_zero; ++z)
                    if (live[j])
                        out[p * n_req + a.zcols[z]] = V(0);
        }

        // The slab prefetched during the tile's last stage (the next tile's
        // first) is written after the output rows have left LDS when they
        // are staged there; a lone stage is then restaged every tile too.
        bool pre_last = false;
        V res[PPT][NS * G];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (s < n_stage) {
                const bool last = s + 1 == n_stage;
                const bool pre = last ? more && (n_stage > 1 || stage_out) : true;
                if (pre) {
                    // group slabs are padded in HBM to PF*BLOCK nodes or more
                    const char *src = reinterpret_cast<const char *>(
                        gsrc + (size_t)a.sgrp[last ? 0 : s + 1] * a.gstride);
#pragma unroll
                    for (int i = 0; i < PF; ++i)
                        pf[i] = *reinterpret_cast<const uint4 *>(src + toff + i * BLOCK * 16);
                }
                if (s == 0) {
                    // next tile's points, issued after the stage prefetch
#pragma unroll
                    for (int j = 0; j < PPT; ++j) {
                        const int64_t pn = p0 + (int64_t)gridDim.x * tile_pts + (int64_t)j * BLOCK;
                        xnext[j] = load_point(a.x, pn, a.n);
                        qnext[j] = load_point(a.q, pn, a.n);
                    }
                }
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    V acc[G];
#pragma unroll
                    for (int jx = 0; jx < 4; ++jx) {
                        const uint4 *rowp = slab + base[j] + jx * nqp;
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
                        res[j][s * G + g] = ok[j] ? acc[g] : quiet_nan<V>();
                }
                if (last) {
                    pre_last = pre;
                } else {
                    __syncthreads();
#pragma unroll
                    for (int i = 0; i < PF; ++i)
                        slab[tid + i * BLOCK] = pf[i];   // slab padded to PF*BLOCK nodes
                    __syncthreads();
                }
            }
        }

        if (n_stage == 0) {
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const int64_t pn = p0 + (int64_t)gridDim.x * tile_pts + (int64_t)j * BLOCK;
                xnext[j] = load_point(a.x, pn, a.n);
                qnext[j] = load_point(a.q, pn, a.n);
            }
        }

        if (stage_out) {
            // Output rows of the tile are contiguous in HBM: assemble them
            // in LDS (over the slab, out_pass_pts points at a time) and write
            // them as 16-byte chunks, instead of each lane writing its row's
            // elements at a row-sized stride.
            __syncthreads();   // the stencils are done with the slab
            const int valid = (int)(a.n - t0 < tile_pts ? a.n - t0 : tile_pts);
            V *lrow = reinterpret_cast<V *>(slab);
            for (int pa = 0; pa < valid; pa += a.out_pass_pts) {
                const int pn = valid - pa < a.out_pass_pts ? valid - pa : a.out_pass_pts;
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    const int lp = tid + j * BLOCK - pa;
                    if (lp >= 0 && lp < pn) {
                        V *r = lrow + lp * n_req;
#pragma unroll
                        for (int k = 0; k < NS * G; ++k)
                            if (k < n_stage * G && a.slot_col[k] >= 0)
                                r[a.slot_col[k]] = res[j][k];
                        for (int z = 0; z < a.n_zero; ++z)
                            r[a.zcols[z]] = V(0);
                        for (int d = 0; d < a.n_dup; ++d)
                            r[a.dup_dst[d]] = r[a.dup_src[d]];
                    }
                }
                __syncthreads();
                const int bytes = pn * n_req * (int)sizeof(V);
                char *dst = reinterpret_cast<char *>(out + (t0 + pa) * n_req);   // 16-byte aligned
                const int nch = bytes >> 4;
                for (int c = tid; c < nch; c += BLOCK)
                    *reinterpret_cast<uint4 *>(dst + c * 16) = slab[c];
                if (tid < (bytes & 15) / 4)
                    reinterpret_cast<uint32_t *>(dst + nch * 16)[tid] =
                        reinterpret_cast<const uint32_t *>(slab + nch)[tid];
                __syncthreads();
            }
            if (pre_last) {
#pragma unroll
                for (int i = 0; i < PF; ++i)
                    slab[tid + i * BLOCK] = pf[i];
                __syncthreads();
            }
        } else {
            if (pre_last) {
                __syncthreads();
#pragma unroll
                for (int i = 0; i < PF; ++i)
                    slab[tid + i * BLOCK] = pf[i];
                __syncthreads();
            }
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                V *orow = out + (p0 + (int64_t)j * BLOCK) * n_req;
#pragma unroll
                for (int k = 0; k < NS * G; ++k) {
                    const int u = a.slot_u[k];
                    if (live[j] && k < n_stage * G && u >= 0) {
                        for (int c = a.ucol_off[u]; c < a.ucol_off[u + 1]; ++c)
                            orow[a.ucols[c]] = res[j][k];
                    }
                }
            }
        }
    }
}

// Compiled launch shapes (block, points per thread) of the grouped kernel.
constexpr LaunchShape kGrpShapes[] = {{256, 2}, {256, 4}, {512, 1}, {512, 2}, {1024, 1}};

// Prefetch depth for the grouped kernel: smallest of {2, 4, 6, 8, 12} chunks
// per thread covering one stage slab; 0 if none does.
inline int pick_pf_grp(int block, int nodes)
{
    for (int pf : {2, 4, 6, 8, 12})
        if (pf * block >= nodes)
            return pf;
    return 0;
}

template <typename V, typename Call>
hipError_t with_grp_variant(const XfxArgs &a, LaunchShape ls, Call call)
{
    const int nodes = (a.nx + 2) * (a.nq + 2);
#define PDFX_GRP(B, P)                                                                             \
    do {                                                                                           \
        switch (pick_pf_grp(B, nodes)) {                                                           \
        case 2: return call(xfx_grp_kernel<V, B, P, 2>, B, P);                                     \
        case 4: return call(xfx_grp_kernel<V, B, P, 4>, B, P);                                     \
        case 6: return call(xfx_grp_kernel<V, B, P, 6>, B, P);                                     \
        case 8: return call(xfx_grp_kernel<V, B, P, 8>, B, P);                                     \
        case 12: return call(xfx_grp_kernel<V, B, P, 12>, B, P);                                   \
        default: return hipErrorInvalidValue;                                                      \
        }                                                                                          \
    } while (0)
    if (ls.block == 256 && ls.ppt == 2) PDFX_GRP(256, 2);
    if (ls.block == 256 && ls.ppt == 4) PDFX_GRP(256, 4);
    if (ls.block == 512 && ls.ppt == 1) PDFX_GRP(512, 1);
    if (ls.block == 512 && ls.ppt == 2) PDFX_GRP(512, 2);
    if (ls.block == 1024 && ls.ppt == 1) PDFX_GRP(1024, 1);
#undef PDFX_GRP
    return hipErrorInvalidValue;
}

template <typename V>
hipError_t launch_grp_typed(const XfxArgs &a0, LaunchShape ls, int max_blocks, hipStream_t s)
{
    XfxArgs a = a0;
    const size_t lds = grp_lds_layout(a, sizeof(V) == 4, ls.block);
    if (lds == 0)
        return hipErrorInvalidValue;
    return with_grp_variant<V>(a, ls, [&](auto fn, int block, int ppt) -> hipError_t {
        const int64_t tile_pts = (int64_t)block * ppt;
        // rows staged through the LDS slab for 16-byte stores when `out` is
        // 16-byte aligned: whole multiples of 16 points that fit the slab
        const int64_t slab_bytes = (int64_t)pick_pf_grp(block, (a.nx + 2) * (a.nq + 2)) * block * 16;
        int64_t pass = slab_bytes / ((int64_t)a.n_req * (int64_t)sizeof(V)) / 16 * 16;
        if (pass > tile_pts)
            pass = tile_pts;
        a.out_pass_pts = ((uintptr_t)a.out % 16 == 0 && pass >= 16) ? (int)pass : 0;
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
hipError_t grp_occupancy_typed(const XfxArgs &a0, LaunchShape ls, int *blocks_per_cu)
{
    XfxArgs a = a0;
    const size_t lds = grp_lds_layout(a, sizeof(V) == 4, ls.block);
    if (lds == 0)
        return hipErrorInvalidValue;
    return with_grp_variant<V>(a, ls, [&](auto fn, int block, int) -> hipError_t {
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
