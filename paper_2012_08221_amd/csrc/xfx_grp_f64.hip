// FP64 instances of the flavour-group forward kernel, and its LDS layout.
#include "xfx_grouped_impl.h"

namespace pdfx {

hipError_t launch_xfx_grp_f64(const XfxArgs &a, LaunchShape ls, int max_blocks, hipStream_t s)
{
    return fwd::launch_grp_typed<double>(a, ls, max_blocks, s);
}

hipError_t xfx_grp_occupancy_f64(const XfxArgs &a, LaunchShape ls, int *blocks_per_cu)
{
    return fwd::grp_occupancy_typed<double>(a, ls, blocks_per_cu);
}

bool grp_shape_supported(LaunchShape ls, int nx, int nq)
{
    if (fwd::pick_pf_grp(ls.block, (nx + 2) * (nq + 2)) == 0)
        return false;
    for (const auto &k : fwd::kGrpShapes)
        if (k.block == ls.block && k.ppt == ls.ppt)
            return true;
    return false;
}

int grp_slab_stride(int nx, int nq)
{
    const int nodes = (nx + 2) * (nq + 2);
    int stride = nodes;
    for (const auto &k : fwd::kGrpShapes) {
        const int w = fwd::pick_pf_grp(k.block, nodes) * k.block;
        if (w > stride)
            stride = w;
    }
    return stride;
}

size_t grp_lds_layout(XfxArgs &a, bool f32, int block)
{
    size_t off = 0;
    auto take = [&](size_t bytes, size_t align) {
        off = (off + align - 1) / align * align;
        const size_t r = off;
        off += bytes;
        return (int)r;
    };
    const AxisDev *axes[2] = {&a.ax, &a.aq};
    AxisLds *lds[2] = {&a.lx, &a.lq};
    for (int i = 0; i < 2; ++i) {
        lds[i]->knots = take((size_t)axes[i]->n * 8, 16);
        lds[i]->seed = take((size_t)axes[i]->nbuckets * 2, 16);
        lds[i]->rec64 = take((size_t)(axes[i]->n - 1) * 64, 64);
        lds[i]->rec32 = take(f32 ? (size_t)(axes[i]->n - 1) * 32 : 0, 64);
    }
    // the slab is padded to the prefetch's PF * block nodes, so that every
    // thread writes all its prefetched chunks without a bounds test
    const int nodes = (a.nx + 2) * (a.nq + 2);
    const int pf = fwd::pick_pf_grp(block, nodes);
    if (pf == 0)
        return 0;
    a.lds_slab0 = take((size_t)pf * block * 16, 16);
    a.lds_slab1 = a.lds_slab0;
    return off <= kLdsLimit ? off : 0;
}

}  // namespace pdfx
