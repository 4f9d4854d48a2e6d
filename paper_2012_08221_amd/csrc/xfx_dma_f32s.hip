// FP32-stencil instances of the double-buffered flavour-group forward kernel
// (logs, search and t in FP64; basis, weights, values and FMAs in FP32).
#include "xfx_dma_impl.h"

namespace pdfx {

hipError_t launch_xfx_dma_f32s(const XfxArgs &a, LaunchShape ls, int max_blocks, hipStream_t s)
{
    return fwd::launch_dma_typed<float>(a, ls, max_blocks, s);
}

hipError_t xfx_dma_occupancy_f32s(LaunchShape ls, int *blocks_per_cu)
{
    return fwd::dma_occupancy_typed<float>(ls, blocks_per_cu);
}

}  // namespace pdfx
