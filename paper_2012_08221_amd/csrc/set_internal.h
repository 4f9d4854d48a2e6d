// Double-buffered evaluation of PDF sets (many members, uneven grids).
#pragma once

#include "pdfx_internal.h"

namespace pdfx {

// Static LDS of the set kernel: two slabs of kSetSlabBytes, the knots of
// both axes (up to kSetKnots) and their bucket seeds (up to kSetSeeds).
constexpr int kSetSlabBytes = 78016;
constexpr int kSetKnots = 320;
constexpr int kSetSeeds = 1280;

// One member as the double-buffered set kernel sees it.
struct SetMemberDev {
    AxisDev ax, aq;
    const void *gvals[2];   // per precision: borderless group slabs [n_groups][gstride nodes]
    int gstride[2];         // nodes per group, per precision (node bytes * gstride % 16 == 0)
    int nb[2];              // node bytes per precision (16, 8 or 4); 0: not in a class
    int nx, nq;
};

struct SetDmaArgs {
    const SetMemberDev *mem;   // [n_mem]
    const int *ids;            // members of this launch's class
    int n_ids;
    int items_per_member, tiles_per_item, n_items;
    unsigned int *counter;     // work-list cursor (reset before the launch)
    // request plan for this class's group width (as XfxArgs)
    int n_req, n_stage, n_zero, n_dup;
    int sgrp[kGrpMaxSlots];
    int slot_col[kGrpMaxSlots];
    int zcols[kMaxReq];
    int dup_src[kMaxReq], dup_dst[kMaxReq];
    const double *x, *q;       // shared points, q = Q^2
    int64_t n;
    void *out;                 // [n_mem][n][n_req], 16-byte aligned
    int domain_mode;
    unsigned long long *dom_count;
    int out_pass_pts;          // output rows staged per pass
};

// Node bytes the set kernel uses for a member of nx x nq knots with nbx, nbq
// bucket seeds in a precision (16, 8 or 4), or 0 if it does not fit.
int set_node_bytes(int nx, int nq, int nbx, int nby, bool f32);

// Launches the class kernel of node width nb over args' work list.
hipError_t launch_set_dma(const SetDmaArgs &a, bool f32, int nb, LaunchShape ls, int cus,
                          hipStream_t s);
bool set_dma_shape_supported(LaunchShape ls);

}  // namespace pdfx
