// FP64 instances of the forward kernel (all arithmetic in FP64).
#include "xfx_fwd_impl.h"

namespace pdfx {

hipError_t launch_xfx_f64(const XfxArgs &a, LaunchShape ls, int max_blocks, hipStream_t s)
{
    return fwd::launch_typed<double>(a, ls, max_blocks, s);
}

hipError_t xfx_occupancy_f64(const XfxArgs &a, LaunchShape ls, int *blocks_per_cu)
{
    return fwd::occupancy_typed<double>(a, ls, blocks_per_cu);
}

bool launch_shape_supported(LaunchShape ls)
{
    for (const auto &k : fwd::kShapes)
        if (k.block == ls.block && k.ppt == ls.ppt)
            return true;
    return false;
}

bool launch_shape_f32_only(LaunchShape ls) { return ls.block == 512 && ls.ppt == 4; }

int n_launch_shapes() { return (int)(sizeof(fwd::kShapes) / sizeof(fwd::kShapes[0])); }
LaunchShape launch_shape_at(int i) { return fwd::kShapes[i]; }

}  // namespace pdfx
