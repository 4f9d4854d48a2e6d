// Many PDF members in one persistent launch.
//
// A PDF set is a collection of members whose grids may differ (knot counts,
// number of Q^2 subgrids).  The launch walks a work list of items
// (member m, run of `tiles_per_item` point tiles), taken by each workgroup
// from an atomic counter until the list is exhausted (every wave reaches the
// exit test, so the grid drains).  For each item the workgroup loads member
// m's axis tables into LDS, then for each of its tiles locates the points in
// m's grid (bins, ln x, ln Q^2, folded weights in registers) and runs the
// flavour loop: stage m's slab for the flavour into LDS, 16-tap stencil,
// store x f into out[m][p][r].  LDS is sized for the largest member; the
// slab is single-buffered (a 200 x 80 FP64 slab alone takes 132 KB).
#include "set_internal.h"
#include "xfx_fwd_impl.h"

namespace pdfx {

namespace {

__global__ void reset_counter(unsigned int *c) { *c = 0u; }

template <typename V, int BLOCK, int PPT>
__global__ __launch_bounds__(BLOCK) void set_kernel(const SetArgs a)
{
    extern __shared__ uint4 smem4[];
    __shared__ int s_item;
    char *sm = reinterpret_cast<char *>(smem4);
    const int tid = threadIdx.x;
    constexpr bool F32 = sizeof(V) == 4;
    uint4 *slab4 = reinterpret_cast<uint4 *>(sm + a.lds_slab);
    const V *slab = reinterpret_cast<const V *>(slab4);
    V *out_all = reinterpret_cast<V *>(a.out);
    const int n_req = a.n_req;
    const int64_t tile_pts = (int64_t)BLOCK * PPT;
    const int64_t ntiles = (a.n + tile_pts - 1) / tile_pts;
    int loaded = -1, staged = -1;

    for (;;) {
        if (tid == 0)
            s_item = (int)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= a.n_items)
            break;
        const int mi = item / a.items_per_member;
        const int m = a.mem_ids ? a.mem_ids[mi] : mi;
        const int64_t t_first = (int64_t)(item - mi * a.items_per_member) * a.tiles_per_item;
        const MemberDev md = a.mem[m];
        if (m != loaded) {
            // member tables through global-address-space loads (the member's
            // pointers come from device memory)
            const AxisDev *axes[2] = {&md.ax, &md.aq};
            const AxisLds *lds[2] = {&a.lx, &a.lq};
            for (int i = 0; i < 2; ++i) {
                copy_words_g(sm + lds[i]->knots, axes[i]->knots, axes[i]->n * 8, BLOCK);
                copy_words_g(sm + lds[i]->seed, axes[i]->seed, axes[i]->nbuckets * 2, BLOCK);
                copy_words_g(sm + lds[i]->rec64, axes[i]->rec64, (axes[i]->n - 1) * 64, BLOCK);
                if (F32)
                    copy_words_g(sm + lds[i]->rec32, axes[i]->rec32, (axes[i]->n - 1) * 32, BLOCK);
            }
            loaded = m;
            staged = -1;
            __syncthreads();
        }
        const fwd::LAxis lx = fwd::lds_axis(sm, md.ax, a.lx);
        const fwd::LAxis lq = fwd::lds_axis(sm, md.aq, a.lq);
        const int nqp = md.nq + 2;
        const int slab_elems = F32 ? md.slab32 : md.slab64;
        const int schunks = slab_elems * (int)sizeof(V) / 16;
        const uint4 *gv = reinterpret_cast<const uint4 *>(F32 ? md.vals32 : md.vals64);
        V *out = out_all + (int64_t)m * a.n * n_req;

        for (int64_t tile = t_first; tile < t_first + a.tiles_per_item && tile < ntiles; ++tile) {
            const int64_t p0 = tile * tile_pts + tid;
            V wx[PPT][4], wq[PPT][4];
            int base[PPT];
            bool ok[PPT], live[PPT];
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const int64_t p = p0 + (int64_t)j * BLOCK;
                live[j] = p < a.n;
                double xv = load_point(a.x, p, a.n);
                double qv = load_point(a.q, p, a.n);
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
                fwd::count_flagged(live[j] && !ok[j], a.dom_count);
                const double lnx = log(xv), lnq = log(qv);
                const int ix = fwd::lbin(lx, xv, lnx);
                const int kq = fwd::lbin(lq, qv, lnq);
                fwd::weights<V>(lx, ix, lnx, wx[j]);
                fwd::weights<V>(lq, kq, lnq, wq[j]);
                base[j] = ix * nqp + kq;
                for (int z = 0; z < a.n_zero; ++z)
                    if (live[j])
                        out[p * n_req + a.zcols[z]] = V(0);
            }
            for (int u = 0; u < a.n_u; ++u) {
                const int row = a.urow[u];
                if (row != staged) {
                    __syncthreads();
                    stage_sync_g(slab4, gv + (size_t)row * schunks, schunks, BLOCK);
                    __syncthreads();
                    staged = row;
                }
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
                    if (live[j]) {
                        const V v = ok[j] ? acc : fwd::quiet_nan<V>();
                        const int64_t p = p0 + (int64_t)j * BLOCK;
                        for (int c = a.ucol_off[u]; c < a.ucol_off[u + 1]; ++c)
                            out[p * n_req + a.ucols[c]] = v;
                    }
                }
            }
        }
    }
}

template <typename V>
hipError_t launch_set_typed(const SetArgs &a, LaunchShape ls, size_t lds, int cus, hipStream_t s)
{
    auto go = [&](auto fn, int block) -> hipError_t {
        if (lds > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
            if (e != hipSuccess)
                return e;
        }
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(fn), block, lds);
        if (e != hipSuccess || per_cu < 1)
            per_cu = 1;
        int64_t grid = (int64_t)per_cu * cus;
        if (grid > a.n_items)
            grid = a.n_items;
        if (grid < 1)
            grid = 1;
        hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, s, a.counter);
        hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(block), lds, s, a);
        return hipGetLastError();
    };
    if (ls.block == 256 && ls.ppt == 2)
        return go(set_kernel<V, 256, 2>, 256);
    if (ls.block == 256 && ls.ppt == 4)
        return go(set_kernel<V, 256, 4>, 256);
    if (ls.block == 512 && ls.ppt == 1)
        return go(set_kernel<V, 512, 1>, 512);
    if (ls.block == 512 && ls.ppt == 2)
        return go(set_kernel<V, 512, 2>, 512);
    if (ls.block == 1024 && ls.ppt == 1)
        return go(set_kernel<V, 1024, 1>, 1024);
    return hipErrorInvalidValue;
}

}  // namespace

// (512, 1), (512, 2), (256, 2) also have double-buffered instances (set_dma.hip).
constexpr LaunchShape kSetShapes[] = {{256, 2}, {256, 4}, {512, 1}, {512, 2}, {1024, 1}};

bool set_shape_supported(LaunchShape ls)
{
    for (const auto &k : kSetShapes)
        if (k.block == ls.block && k.ppt == ls.ppt)
            return true;
    return false;
}

int n_set_shapes() { return (int)(sizeof(kSetShapes) / sizeof(kSetShapes[0])); }
LaunchShape set_shape_at(int i) { return kSetShapes[i]; }

hipError_t launch_set(const SetArgs &a, bool f32, LaunchShape ls, size_t lds, int cus, hipStream_t s)
{
    return f32 ? launch_set_typed<float>(a, ls, lds, cus, s)
               : launch_set_typed<double>(a, ls, lds, cus, s);
}

}  // namespace pdfx
