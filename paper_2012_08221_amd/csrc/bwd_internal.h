// Adjoint launch pieces shared by the host runtime and bwd*.hip.
#pragma once

#include "pdfx_internal.h"

namespace pdfx {

// Flag bits of the per-point state of the adjoint.
constexpr uint8_t kBwdOut = 1;      // outside the grid in NaN mode, or NaN input
constexpr uint8_t kBwdXClamp = 2;   // x clamped to the grid edge
constexpr uint8_t kBwdQClamp = 4;   // Q^2 clamped

// Coordinate gradients by a forward-style pass over flavour groups, with the
// chain rule and the domain rules applied:
//   grad_x[p]  = (1/x)   sum_r g[p][r] dxf_r/dln x,
//   grad_q2[p] = (1/Q^2) sum_r g[p][r] dxf_r/dln Q^2
// (FP64), written once per point, no atomics; NaN outside the grid in NaN
// mode or for NaN input, 0 along a clamped axis.  When st_idx is set the pass
// also writes the per-point state that the knot pass reads (as the state
// pass of BwdArgs would), and zeroes gacc.
struct CoordArgs {
    XfxArgs x;                 // grid, points, stage plan (slots, columns), borderless group slabs
    const void *gout;          // [n][n_req] dL/dout, precision's type
    double *grad_x, *grad_q2;  // [n] each, or null
    int32_t *st_idx;           // [n] ix | kq << 16, or null: no state written
    uint8_t *st_flag;          // [n] kBwd* bits
    double *st_tx, *st_tq;     // [n] FP64 local coordinates
    double *gacc;              // [n_gacc] zeroed, or null
    int64_t n_gacc;
    double *gmax;              // [workgroups][n_u] max of finite |dL/dout| per distinct
                               // flavour over each workgroup's points, or null
};

// Most workgroups of a pass that writes per-workgroup maxima (gmax).
constexpr int kMaxPart = 1024;

// Workgroups of launch_coord_grad for n points.
int coord_grad_blocks(int64_t n, int cus);
hipError_t launch_coord_grad(const CoordArgs &c, bool f32, int cus, hipStream_t s);

// Knot gradient by groups of flavours per workgroup (grids of up to 5000
// knots, n_x, n_q >= 4): gacc[urow[u]] +=
// sum_p g[p][u] wx wq from the state arrays of b and the maxima b.gmax if
// set (dL/dout FP32 if f32, else FP64); gacc must be zeroed.
bool knot_grad_supported(int nx, int nq);
hipError_t launch_knot_grad(const BwdArgs &b, bool f32, int cus, hipStream_t s);

// The adjoint after the argument checks: state pass, knot pass (or the
// per-flavour scatter for grids beyond it) and finish.  With coords_done the
// coordinate gradients are already written (launch_coord_grad), and, when a
// knot gradient is wanted, so are the per-point state and the zeroed gacc:
// only the knot pass and the finish of grad_xf remain.
hipError_t launch_backward_ex(const BwdArgs &a, bool f32, void *grad_xf, double *grad_x,
                              double *grad_q2, int cus, hipStream_t s, bool coords_done);

}  // namespace pdfx
