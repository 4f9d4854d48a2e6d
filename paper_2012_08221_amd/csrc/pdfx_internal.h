// Internal types shared by the pdfx host runtime and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdfx {

// Per-interval record of one interpolation axis (x, or the concatenated Q^2
// subgrids, or the alpha_s knots).  For the interval [z_i, z_{i+1}] in ln
// space, with t = (ln v - z_i) * inv_d and the cubic Hermite basis h.., the
// four knot weights of knots (i-1, i, i+1, i+2) are
//   w_-1 = -h10 pl
//   w_0  =  h00 + h10 (pl - ql) - h11 qr
//   w_1  =  h01 + h10 ql + h11 (qr - pr)
//   w_2  =  h11 pr
// where, for the finite-difference slopes of the method (one-sided at an end
// of the axis or subgrid, mean of the neighbouring divided differences
// inside), cl = 1/2 inside and 0 at the left end, cr likewise at the right end,
// pl = cl * d_i / d_{i-1}, ql = 1 - cl, pr = cr * d_i / d_{i+1}, qr = 1 - cr.
// A weight on a knot outside the axis/subgrid is exactly 0.
template <typename T>
struct alignas(8 * sizeof(T)) IntervalRec {
    T z;      // ln z_i   (only the FP64 table's z and inv_d are used: t is formed in FP64)
    T inv_d;  // 1 / (ln z_{i+1} - ln z_i)
    T pl, plql, ql, qr, qrpr, pr;  // pl, pl-ql, ql, qr, qr-pr, pr
};

// Coordinate of point p read with p clamped to the last point (n >= 1): a
// lane past the end reads a real point whose result is never stored.  The
// load stays a global load; choosing between the array and a default value's
// address would make it a flat load, and a pending flat load holds up every
// LDS wait issued after it.
__device__ __forceinline__ double load_point(const double *v, int64_t p, int64_t n)
{
    return v[p < n ? p : n - 1];
}

// Keys of the in-wave dealing below: 32 LDS bank keys of an 8-byte word
// (its index mod 32) and one for lanes that do no work.
constexpr int kDealKeys = 33;

// In-wave dealing for LDS atomic scatters, which run ~2.7x faster when the
// lanes of one instruction hit different banks: the 64 lanes' keys (in
// [0, kDealKeys), the last for idle lanes) are counting-sorted and sorted rank
// r goes to lane (r mod 4) * 16 + r / 4, so that every 16 lanes hold keys
// spread over the sorted order.  Returns the lane whose item this lane takes.
// hist: this wave's kDealKeys ints of LDS.  Every lane of the wave must call
// it together.
__device__ __forceinline__ int wave_deal(int key, int *hist)
{
    const int lane = threadIdx.x & 63;
    if (lane < kDealKeys)
        hist[lane] = 0;
    __builtin_amdgcn_wave_barrier();
    const int lrank = atomicAdd(&hist[key], 1);   // rank among the wave's equal keys
    __builtin_amdgcn_wave_barrier();
    const int cnt = lane < kDealKeys ? hist[lane] : 0;
    // inclusive scan over the 64 lanes by DPP (VALU only, leaving the LDS pipe
    // to the scatter): shifts within each 16-lane row, then the last lane of
    // row 0 (of row 2) added to row 1 (row 3), then lane 31 to rows 2 and 3
    int incl = cnt;
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x111, 0xf, 0xf, true);   // row_shr:1
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x112, 0xf, 0xf, true);   // row_shr:2
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x114, 0xf, 0xf, true);   // row_shr:4
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x118, 0xf, 0xf, true);   // row_shr:8
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x142, 0xa, 0xf, false);  // row_bcast:15
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x143, 0xc, 0xf, false);  // row_bcast:31
    const int rank = __shfl(incl - cnt, key) + lrank;
    const int dest = (rank & 3) * 16 + (rank >> 2);
    return __builtin_amdgcn_ds_permute(dest * 4, lane);
}

// Device view of one axis (global-memory tables).
struct AxisDev {
    const double *knots;          // raw knots, non-decreasing (search on raw values)
    const IntervalRec<double> *rec64;
    const IntervalRec<float> *rec32;
    const uint16_t *seed;         // bucket -> starting interval for the search
    int n;                        // knots
    int nbuckets;                 // multiple of 4
    double lo;                    // raw knots[0]
    double hi;                    // raw knots[n-1]
    double ln_lo;                 // ln knots[0]
    double inv_hb;                // nbuckets / (ln knots[n-1] - ln knots[0])
};

constexpr int kMaxReq = 64;
// Result slots a thread of the flavour-group kernel holds in registers.
constexpr int kGrpMaxSlots = 12;

// Byte offsets of one axis' tables inside the workgroup's LDS.
struct AxisLds {
    int knots, seed, rec64, rec32;
};

struct XfxArgs {
    AxisDev ax, aq;
    // Values: one bordered slab per grid row, (nx+2) x (nq+2) with a zero
    // border one knot wide, row-major (Q fastest), slab stride slab_elems
    // elements (a multiple of 16 bytes).
    const void *vals;
    int nf, nx, nq;
    int slab_elems;
    int n_req;                    // output columns
    int n_u;                      // distinct grid rows among the requested pids
    int urow[kMaxReq];            // grid row of distinct u
    int ucol_off[kMaxReq + 1];    // its output columns: ucols[ucol_off[u] .. ucol_off[u+1])
    int ucols[kMaxReq];
    int n_zero;                   // columns of pids absent from the grid (always 0)
    int zcols[kMaxReq];
    const double *x;
    const double *q;              // Q^2, or Q if q_is_q
    int q_is_q;
    void *out;                    // [n][n_req]
    int64_t n;
    int domain_mode;
    unsigned long long *dom_count;
    AxisLds lx, lq;               // table offsets in LDS
    int lds_slab0, lds_slab1;     // slab buffer offsets in LDS
    // Flavour-group staging: grid rows gi*G .. gi*G+G-1 (G = 16 / value
    // size, rows >= nf zero) interleaved per knot into 16-byte nodes, one
    // bordered node slab of (nx+2) x (nq+2) nodes per group.
    const void *gvals;            // [n_groups][gstride] nodes, node slab first, then zeros
    int gstride;                  // nodes per group in HBM
    int n_stage;                  // groups touched by the request
    int sgrp[kGrpMaxSlots];       // group of stage s
    int slot_u[kGrpMaxSlots];     // slot s*G+g -> distinct request row u, or -1
    int slot_col[kGrpMaxSlots];   // slot -> first output column of its row, or -1
    int n_dup;                    // further columns of a row requested more than once:
    int dup_src[kMaxReq];         //   column dup_dst[d] repeats column dup_src[d]
    int dup_dst[kMaxReq];
    int out_pass_pts;             // > 0: output rows staged in LDS this many points at a time
    // alpha_s at the same points (double-buffered kernel only, when the
    // alpha_s knots are the Q^2 knots): knot values padded with a zero at
    // each end, and the output [n]; as_out NULL = no alpha_s
    const void *as_vals;
    void *as_out;
};

struct BwdArgs {
    AxisDev ax, aq;
    AxisLds lx, lq;               // LDS layout of the state pass
    const void *vals;             // bordered slabs (as XfxArgs::vals)
    int nf, nx, nq, slab_elems;
    int n_req, n_u;
    int urow[kMaxReq];
    int ucol_off[kMaxReq + 1];
    int ucols[kMaxReq];
    const double *x, *q;          // q is Q^2
    int64_t n;
    int domain_mode;
    const void *gout;             // [n][n_req] dL/dout, precision's type
    int gout_f32;                 // dL/dout is FP32 (else FP64)
    int32_t *st_idx;              // per point: ix | kq << 16
    uint8_t *st_flag;             // per point: outside / x clamped / Q^2 clamped
    double *st_tx, *st_tq;        // per point: FP64 local coordinates
    double *gacc;                 // [nf][nx][nq] FP64 knot-gradient accumulator, or null
    double *accx, *accw;          // [n] FP64 sum_r g dxf/dln x, sum_r g dxf/dln Q^2, or null
    double *gmax;                 // [n_part][n_u] per-workgroup max of finite |dL/dout| per
                                  // distinct flavour (written by the coordinate pass), or
                                  // null: the knot pass finds it
    int n_part;
    int lds_recx, lds_recq, lds_grad, lds_slab;
    int chunk;                    // points per workgroup of the adjoint pass
};

// One member of a set on the device.
struct MemberDev {
    AxisDev ax, aq;
    const void *vals64, *vals32;  // bordered slabs per precision
    int nx, nq, slab64, slab32;   // slab elements per precision
};

struct SetArgs {
    const MemberDev *mem;         // [n_mem] on the device
    const int *mem_ids;           // members to evaluate (work-list order), or null: all
    int n_mem;
    int n_req, n_u;
    int urow[kMaxReq];
    int ucol_off[kMaxReq + 1];
    int ucols[kMaxReq];
    int n_zero;
    int zcols[kMaxReq];
    const double *x, *q;          // shared points, q = Q^2
    int64_t n;
    void *out;                    // [n_mem][n][n_req]
    int domain_mode;
    unsigned long long *dom_count;
    unsigned int *counter;        // work-list cursor (reset before each launch)
    int n_items, items_per_member, tiles_per_item;
    AxisLds lx, lq;               // LDS offsets, sized for the largest member
    int lds_slab;
};

// Drell-Yan-like integrand (forward and backward).
constexpr int kDyMaxBlocks = 4096;
struct DyArgs {
    AxisDev ax, aq, aa;           // x, Q^2 and alpha_s axes
    AxisLds lx, lq, la;
    int lds_asv;                  // padded alpha_s values in LDS
    const void *as_vals;          // padded alpha_s values, precision's type
    const double *as_vals64;      // padded alpha_s values, FP64 (backward state pass)
    const void *vals;             // bordered slabs
    int nf, nx, nq, slab_elems;
    int n_seq;                    // flavours in the sequence q, -q, q', -q', ...
    int seq_row[10];              // their grid rows
    const double *u1, *u2;
    int64_t n;
    double lnxmin, lnrange, s, L2, scale;
    void *out;                    // [n] or null
    double *block_sums;           // [grid] or null
    unsigned long long *dom_count;
    int lds_slab0, lds_slab1;
    int32_t *st_i1, *st_i2;       // backward state: x1 bin | Q^2 bin << 16 (-1: skip), x2 bin
    double *st_t1, *st_t2, *st_tq, *st_as;
    double *gacc;                 // [nf][nx][nq] FP64
    int lds_recx, lds_recq, lds_grad;
    int chunk;
    const void *gvals;            // borderless flavour-group node slabs (double-buffered kernel)
    int gstride;                  // nodes per group
};

struct AlphasArgs {
    AxisDev a;
    const void *vals;             // padded [n+2] FP64 or FP32: vals[k+1] = alpha_s knot k
    const double *q2;             // Q^2, or Q when q_is_q (squared in FP64 first)
    void *out;
    int64_t n;
    int domain_mode;
    int q_is_q;
    unsigned long long *dom_count;
};

struct RepackArgs {
    const void *src;              // [nf][nx][nq]
    void *dst;                    // [nf][slab_elems] bordered
    int nf, nx, nq, slab_elems;
};

// Launch shape of the forward kernel.
struct LaunchShape {
    int block;
    int ppt;
};

// Kernel launchers.  Return a hipError_t.
hipError_t launch_xfx_f64(const XfxArgs &a, LaunchShape ls, int max_blocks, hipStream_t s);
hipError_t launch_xfx_f32s(const XfxArgs &a, LaunchShape ls, int max_blocks, hipStream_t s);
hipError_t xfx_occupancy_f64(const XfxArgs &a, LaunchShape ls, int *blocks_per_cu);
hipError_t xfx_occupancy_f32s(const XfxArgs &a, LaunchShape ls, int *blocks_per_cu);
hipError_t launch_xfx_grp_f64(const XfxArgs &a, LaunchShape ls, int max_blocks, hipStream_t s);
hipError_t launch_xfx_grp_f32s(const XfxArgs &a, LaunchShape ls, int max_blocks, hipStream_t s);
hipError_t xfx_grp_occupancy_f64(const XfxArgs &a, LaunchShape ls, int *blocks_per_cu);
hipError_t xfx_grp_occupancy_f32s(const XfxArgs &a, LaunchShape ls, int *blocks_per_cu);
// True if the grouped kernel is compiled for ls and its prefetch covers a
// node slab of an nx x nq grid.
bool grp_shape_supported(LaunchShape ls, int nx, int nq);
// Nodes per flavour group in HBM: the node slab padded with zeros up to the
// widest prefetch of the compiled grouped shapes, so prefetches need no
// bounds test.
int grp_slab_stride(int nx, int nq);
// Raw caller values [nf][nx][nq] -> flavour-group node slabs [n_groups][gstride]
// ((nx+2) x (nq+2) nodes with a zero border, or nx x nq without; zero padding
// rows and nodes).
hipError_t launch_grp_repack(const void *src, void *dst, int nf, int nx, int nq, int n_groups,
                             int gstride, bool border, bool f32, hipStream_t s);
hipError_t launch_xfx_dma_f64(const XfxArgs &a, LaunchShape ls, int max_blocks, hipStream_t s);
hipError_t launch_xfx_dma_f32s(const XfxArgs &a, LaunchShape ls, int max_blocks, hipStream_t s);
hipError_t xfx_dma_occupancy_f64(LaunchShape ls, int *blocks_per_cu);
hipError_t xfx_dma_occupancy_f32s(LaunchShape ls, int *blocks_per_cu);
// True if the double-buffered kernel is compiled for ls and its static LDS
// holds two node slabs and the search tables of an nx x nq grid with nbx and
// nbq bucket seeds.
bool dma_supported(LaunchShape ls, int nx, int nq, int nbx, int nbq, bool f32 = false);
// The alpha_s values of a Q^2 axis of nq knots fit the kernel's LDS after the knots.
bool dma_alphas_fit(int nx, int nq, bool f32);
hipError_t launch_alphas(const AlphasArgs &a, bool f32, hipStream_t s);
hipError_t launch_repack(const RepackArgs &a, bool f32, hipStream_t s);
hipError_t launch_set(const SetArgs &a, bool f32, LaunchShape ls, size_t lds, int cus, hipStream_t s);
hipError_t launch_dy_forward(const DyArgs &a, bool f32, int cus, hipStream_t s, int *n_blocks);
hipError_t launch_dy_backward(const DyArgs &a, bool f32, void *grad_xf, int cus, hipStream_t s);
size_t dy_lds_layout(DyArgs &a, bool f32, bool *db);
// Double-buffered integrand kernel: fits an nx x nq grid with na alpha_s
// knots and nbx, nbq bucket seeds (the standard 11-parton order is checked
// by the caller).
bool dy_dma_supported(int nx, int nq, int na, int nbx, int nbq);
bool dy_shape_supported(LaunchShape ls, bool f32);
// Knot-gradient pass of the integrand backward by quark-antiquark pairs
// (standard parton order; a.gvals/gstride: borderless group slabs; the state
// arrays and the zeroed FP64 accumulator as for launch_dy_backward).
hipError_t launch_dy_pair_adjoint(const DyArgs &a, bool f32, int cus, hipStream_t s);
hipError_t launch_dy_backward_ex(const DyArgs &a, bool f32, void *grad_xf, int cus,
                                 hipStream_t s, bool pairs);
hipError_t launch_dy_dma_forward(const DyArgs &a, bool f32, LaunchShape ls, int cus,
                                 hipStream_t s, int *n_blocks);
bool set_shape_supported(LaunchShape ls);
int n_set_shapes();
LaunchShape set_shape_at(int i);
bool launch_shape_supported(LaunchShape ls);
// Shapes only the FP32 double-buffered kernel has (other FP32 kernels run
// them as (512, 2)).
bool launch_shape_f32_only(LaunchShape ls);
int n_launch_shapes();
LaunchShape launch_shape_at(int i);

// LDS layout of the forward kernel for a grid: fills the offsets in a and
// returns the total bytes (0 if even one slab does not fit).  double_buffer
// receives whether two slabs fit.
size_t xfx_lds_layout(XfxArgs &a, bool f32, bool *double_buffer);
// Elements per bordered slab, rounded up to 16 bytes.
int slab_elems_for(int nx, int nq, bool f32);

constexpr size_t kLdsLimit = 160 * 1024;

// LDS bytes of the flavour-group kernel with workgroup size block (axis
// tables + one node slab padded to the prefetch width), 0 if that exceeds the
// LDS of a compute unit or no prefetch width covers the slab.
size_t grp_lds_layout(XfxArgs &a, bool f32, int block);

}  // namespace pdfx
