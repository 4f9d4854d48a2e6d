// Continuation outside the grid: arguments shared by the host runtime and extrap.hip.
#pragma once

#include "pdfx_internal.h"

namespace pdfx {

struct ExtrapArgs {
    AxisDev ax, aq;
    const void *vals;          // bordered per-row slabs (as XfxArgs::vals), precision's type
    int nx, nq, slab_elems;
    int n_req;
    int row[kMaxReq];          // grid row of output column r, or -1 (absent parton: 0)
    int kx[4];                 // x knot indices: low edge, next inward, high edge, next inward
    int kq[4];                 // Q^2 knot indices, the same (a repeated knot: its upper copy)
    const double *x, *q;       // [n]; q is Q^2, or Q if q_is_q
    int q_is_q;
    void *out;                 // [n][n_req]; only rows of points outside the grid are written
    int64_t n;
};

// Rewrites the output rows of the points outside the grid with the
// continuation (one thread per point).
hipError_t launch_extrap(const ExtrapArgs &a, bool f32, int cus, hipStream_t s);

}  // namespace pdfx
