// Double-buffered evaluation of PDF sets (many members, uneven grids).
#pragma once

#include "pdfx_internal.h"

namespace pdfx {

// Static LDS of the set kernel: two slabs of kSetSlabBytes, the knots of
// both axes (up to kSetKnots) and their bucket seeds (up to kSetSeeds).
constexpr int kSetSlabBytes = 78016;
constexpr int kSetKnots = 320;
constexpr int kSetSeeds = 1280;

// Classes of the double-buffered set kernel by node bytes; the last two are
// the classes whose slab is split over both LDS slabs (8- and 16-byte nodes).
constexpr int kSetClasses = 5;
constexpr int kSetClassWidth[kSetClasses] = {16, 8, 4, 8, 16};
constexpr bool kSetClassSplit[kSetClasses] = {false, false, false, true, true};
// Order in which the classes enter the work list: dearest per tile first
// (split 8-byte, split 16-byte, 8-byte, 16-byte, 4-byte), so that the cheap
// items are left for the end of the launch and fill its tail.
constexpr int kSetClassOrder[kSetClasses] = {3, 4, 1, 0, 2};

// One member as the double-buffered set kernel sees it.
struct SetMemberDev {
    AxisDev ax, aq;
    const void *gvals[2];   // per precision: borderless group slabs [n_groups][gstride nodes]
    int gstride[2];         // nodes per group, per precision (node bytes * gstride % 16 == 0)
    int nb[2];              // node bytes per precision (16, 8 or 4); 0: not in a class
    int nx, nq;
    int split_rows[2];      // per precision, split classes: rows held in the first slab
};

// Stage plan of a request for one group width G (as XfxArgs): the groups
// touched, in order, and the output column of each result slot.
struct SetPlan {
    int n_stage;
    int sgrp[kGrpMaxSlots];
    int slot_col[kGrpMaxSlots];
};

// The work list of one launch: every member that a class takes, in class
// order (kSetClassOrder), each split into items_per_member runs of
// tiles_per_item point tiles; workgroups take items from an atomic cursor.
struct SetDmaArgs {
    const SetMemberDev *mem;   // [n_mem]
    const int2 *ids;           // work order: (member, class)
    int n_ids;
    int items_per_member, tiles_per_item, n_items;
    unsigned int *counter;     // work-list cursor (reset before the launch)
    int n_req, n_zero, n_dup;
    SetPlan plan[3];           // for G = 1, 2, 4
    int zcols[kMaxReq];
    int dup_src[kMaxReq], dup_dst[kMaxReq];
    const double *x, *q;       // shared points, q = Q^2
    int64_t n;
    void *out;                 // [n_mem][n][n_req], 16-byte aligned
    int domain_mode;
    unsigned long long *dom_count;
    int out_pass_pts;          // output rows staged per pass
};

// The members' table pointers are read from device memory, so the compiler
// cannot tell that they address global memory and would load through them
// with flat loads (which also hold up LDS waits); these helpers read through
// global-address-space pointers instead.
template <typename T>
using gptr = const __attribute__((address_space(1))) T *;

__device__ __forceinline__ void copy_words_g(char *dst, const void *src, int bytes, int block)
{
    gptr<unsigned long long> s = (gptr<unsigned long long>)src;
    unsigned long long *d = reinterpret_cast<unsigned long long *>(dst);
    for (int i = threadIdx.x; i < bytes / 8; i += block)
        d[i] = s[i];
}

// A 16-byte-chunk copy of n chunks from global memory (through a
// global-address-space pointer) into LDS, all threads of the block.
__device__ __forceinline__ void stage_sync_g(uint4 *dst, const void *src, int n, int block)
{
    gptr<unsigned long long> s = (gptr<unsigned long long>)src;
    unsigned long long *d = reinterpret_cast<unsigned long long *>(dst);
    for (int c = threadIdx.x; c < n; c += block) {
        d[2 * c] = s[2 * c];
        d[2 * c + 1] = s[2 * c + 1];
    }
}

// Node bytes the set kernel uses for a member of nx x nq knots with nbx, nbq
// bucket seeds in a precision (16, 8 or 4), or 0 if it does not fit.
int set_node_bytes(int nx, int nq, int nbx, int nby, bool f32);

// The rows of a member's group slab of nb-byte nodes held in the first
// LDS slab when the slab is split over both (the rest fitting the second), or
// 0 if it does not fit that way.
int set_split_rows(int nx, int nq, int nbx, int nbq, int nb);

// Launches the set kernel over args' work list (one launch for every class).
hipError_t launch_set_dma(const SetDmaArgs &a, bool f32, LaunchShape ls, int cus, hipStream_t s);
// (512, 4) is compiled for FP32 only.
bool set_dma_shape_supported(LaunchShape ls, bool f32);

}  // namespace pdfx
