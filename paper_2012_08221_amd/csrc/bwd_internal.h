// Adjoint launch pieces shared by the host runtime and bwd*.hip.
#pragma once

#include "pdfx_internal.h"

namespace pdfx {

// Coordinate gradients by a forward-style pass over flavour groups:
//   accx[p] = sum_r g[p][r] dxf_r/dln x,  accw[p] = sum_r g[p][r] dxf_r/dln Q^2
// (FP64), written once per point, no atomics.
struct CoordArgs {
    XfxArgs x;             // grid, points, stage plan (slots, columns), borderless group slabs
    const void *gout;      // [n][n_req] dL/dout, precision's type
    double *accx, *accw;   // [n]
};

hipError_t launch_coord_grad(const CoordArgs &c, bool f32, int cus, hipStream_t s);

// Knot gradient by groups of flavours per workgroup (grids of up to 5000
// knots, n_x, n_q >= 4): gacc[urow[u]] += sum_p g[p][u] wx wq from the state
// arrays of b; gacc must be zeroed.
struct KnotArgs {
    BwdArgs b;
    int f32;               // dL/dout is FP32 (else FP64)
};
bool knot_grad_supported(int nx, int nq);
hipError_t launch_knot_grad(const BwdArgs &b, bool f32, int cus, hipStream_t s);

// The adjoint as launch_backward, except that with coords_ready the per-point
// accumulators accx, accw already hold the coordinate sums (launch_coord_grad)
// and the flavour workgroups only scatter the knot gradient.
hipError_t launch_backward_ex(const BwdArgs &a, bool f32, void *grad_xf, double *grad_x,
                              double *grad_q2, int cus, hipStream_t s, bool coords_ready);

}  // namespace pdfx
