// FP32-stencil instances of the forward kernel: logs, search and the local
// coordinate t in FP64; t rounded to FP32; basis, weights, values and FMAs FP32.
#include "xfx_fwd_impl.h"

namespace pdfx {

hipError_t launch_xfx_f32s(const XfxArgs &a, LaunchShape ls, int max_blocks, hipStream_t s)
{
    return fwd::launch_typed<float>(a, ls, max_blocks, s);
}

hipError_t xfx_occupancy_f32s(const XfxArgs &a, LaunchShape ls, int *blocks_per_cu)
{
    return fwd::occupancy_typed<float>(a, ls, blocks_per_cu);
}

}  // namespace pdfx
