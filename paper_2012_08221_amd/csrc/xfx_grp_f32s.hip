// FP32-stencil instances of the flavour-group forward kernel (logs, search
// and t in FP64; basis, weights, values and FMAs in FP32).
#include "xfx_grouped_impl.h"

namespace pdfx {

hipError_t launch_xfx_grp_f32s(const XfxArgs &a, LaunchShape ls, int max_blocks, hipStream_t s)
{
    return fwd::launch_grp_typed<float>(a, ls, max_blocks, s);
}

hipError_t xfx_grp_occupancy_f32s(const XfxArgs &a, LaunchShape ls, int *blocks_per_cu)
{
    return fwd::grp_occupancy_typed<float>(a, ls, blocks_per_cu);
}

}  // namespace pdfx
