// FP64 instances of the double-buffered flavour-group forward kernel.
#include "xfx_dma_impl.h"

namespace pdfx {

hipError_t launch_xfx_dma_f64(const XfxArgs &a, LaunchShape ls, int max_blocks, hipStream_t s)
{
    return fwd::launch_dma_typed<double>(a, ls, max_blocks, s);
}

hipError_t xfx_dma_occupancy_f64(LaunchShape ls, int *blocks_per_cu)
{
    return fwd::dma_occupancy_typed<double>(ls, blocks_per_cu);
}

bool dma_alphas_fit(int nx, int nq, bool f32)
{
    const int vb = f32 ? 4 : 8;
    return (nx + nq) * 8 + ((nq + 2) * vb + 7) / 8 * 8 <= fwd::kDmaKnots * 8;
}

bool dma_supported(LaunchShape ls, int nx, int nq, int nbx, int nbq, bool f32)
{
    if (nx < 4 || nq < 4 || nx * nq > fwd::kDmaNodes || nx + nq > fwd::kDmaKnots ||
        nbx + nbq > fwd::kDmaSeeds)
        return false;
    if (f32 && ls.block == fwd::kDmaShapeF32.block && ls.ppt == fwd::kDmaShapeF32.ppt)
        return true;
    for (const auto &k : fwd::kDmaShapes)
        if (k.block == ls.block && k.ppt == ls.ppt)
            return true;
    return false;
}

}  // namespace pdfx
