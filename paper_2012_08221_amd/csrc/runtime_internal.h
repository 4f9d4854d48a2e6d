// Host-side objects of the pdfx runtime (not part of the C-ABI).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pdfx.h"
#include "pdfx_internal.h"
#include "set_internal.h"

namespace pdfx {

// Owning device allocation.
struct DeviceBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DeviceBuf() = default;
    DeviceBuf(const DeviceBuf &) = delete;
    DeviceBuf &operator=(const DeviceBuf &) = delete;
    ~DeviceBuf();
    // Allocates n bytes and copies src (or zero-fills if src is NULL).
    hipError_t upload(const void *src, size_t n);
};

// One interpolation axis: host tables derived in FP64, plus their device copies.
struct AxisHost {
    int n = 0;
    int nbuckets = 0;
    double ln_lo = 0.0;
    double inv_hb = 0.0;
    std::vector<double> knots;
    std::vector<IntervalRec<double>> rec64;
    std::vector<IntervalRec<float>> rec32;
    std::vector<uint16_t> seed;
    DeviceBuf d_knots, d_rec64, d_rec32, d_seed;
    int build(const double *z, const int32_t *off, int n_sub);
    AxisDev dev() const;
};

int fail(int code, const char *fmt, ...);
int fail_hip(hipError_t e, const char *what);
void clear_error();
int validate_desc(const pdfx_grid_desc *d, bool need_values);
int device_cu_count();
LaunchShape default_shape(bool f32);
bool grid_fits_lds(int nx, int nq, int n_as, bool f32);

}  // namespace pdfx

struct pdfx_grid {
    int nf = 0;
    int n_sub = 0;
    int cus = 256;
    bool has_values = false;
    bool has_alphas = false;
    // alpha_s axis identical to the Q^2 axis (knots, subgrid split, tables):
    // alpha_s can then use the Q^2 weights of the forward kernel
    bool alphas_on_q = false;
    std::vector<int32_t> pids;
    std::vector<int32_t> q_off;
    pdfx::AxisHost ax, aq, aa;
    int slab_elems[2] = {0, 0};              // per precision
    pdfx::DeviceBuf vals[2];                 // owned values, bordered slabs, per precision
    pdfx::DeviceBuf scratch_vals[2];         // bordered copy of caller values, per precision
    int n_groups[2] = {0, 0};                // flavour groups per precision (G = 2 / 4 rows)
    int gstride = 0;                         // nodes per group slab in HBM (padded)
    bool dma_grid = false;                   // fits the double-buffered kernel's LDS
    pdfx::DeviceBuf dvals[2];                // owned values as borderless group slabs
    pdfx::DeviceBuf scratch_dvals[2];        // caller values as borderless group slabs
    pdfx::DeviceBuf gvals[2];                // owned values as flavour-group node slabs
    pdfx::DeviceBuf scratch_gvals[2];        // caller values as flavour-group node slabs
    pdfx::DeviceBuf as_vals64, as_vals32;    // padded [n_as + 2]
    pdfx::DeviceBuf dom_count;               // unsigned long long
    // PDFX_DOMAIN_ERROR calls: their own counter (cleared per call) and the
    // total of the points they found, added to the pdfx_domain_errors count
    pdfx::DeviceBuf call_count;              // unsigned long long
    mutable int64_t host_count = 0;
    pdfx::LaunchShape shape[2];              // per precision
    // shape[prec] set by pdfx_set_launch: used as it is at every size (a tuned
    // or default shape gives way to (512, 1) when a call has too few points
    // to give every other compute unit a tile)
    bool shape_pinned[2] = {false, false};
    pdfx::LaunchShape dy_shape[2] = {{512, 1}, {512, 2}};   // double-buffered integrand kernel
    pdfx::LaunchShape lumi_shape[2] = {{512, 2}, {512, 2}};  // flavour-pair luminosity kernel
    bool lumi_pinned[2] = {false, false};    // lumi_shape set by pdfx_set_lumi_launch
    mutable pdfx::DeviceBuf bwd_ws;          // adjoint workspace (grows on demand)
    // resident-workgroup cache per [precision][kernel: per-flavour, grouped,
    // double-buffered], two shapes each (a grid's own shape and the one small
    // calls take), the older entry replaced on a miss
    mutable pdfx::LaunchShape occ_shape[2][3][2] = {};
    mutable int occ_blocks[2][3][2] = {};
    mutable int occ_next[2][3] = {};
    int row_of(int pid) const;
    int max_blocks(int prec, const pdfx::XfxArgs &a, int kernel, pdfx::LaunchShape ls) const;
    void reset_occupancy(int prec) const
    {
        for (int k = 0; k < 3; ++k)
            occ_blocks[prec][k][0] = occ_blocks[prec][k][1] = 0;
    }
};

namespace pdfx {

int grid_init(pdfx_grid *g, const pdfx_grid_desc *d);
int prepare_xfx_args(const pdfx_grid *g, const void *xf_dev, int prec, const int32_t *pids,
                     int32_t n_req, const double *x, const double *q, int64_t n_pts, void *out,
                     int domain_mode, XfxArgs *a);
// Runs the forward pass.  With a.as_out set, the double-buffered kernel also
// writes alpha_s; *as_done tells whether it did (the other kernels do not).
int run_xfx(const pdfx_grid *g, XfxArgs &a, const void *xf_dev, int prec, hipStream_t s,
            bool *as_done = nullptr);

// Domain mode PDFX_DOMAIN_ERROR: the evaluation runs in NAN mode with its
// outside points counted in a per-call counter that error_mode_begin clears
// by a kernel on the stream; error_mode_end waits for the stream, adds the
// count to *total and returns PDFX_EDOMAIN if it is not 0.
int error_mode_begin(void *counter, hipStream_t s);
int error_mode_end(void *counter, hipStream_t s, int64_t *total);

// The adjoint (pdfx_eval_xfx_backward) with its workspace grown in the grid
// (fixed_ws NULL) or taken from fixed_ws of fixed_cap bytes; a call that
// needs more than fixed_cap is rejected before anything is enqueued.
int eval_xfx_backward(const pdfx_grid *g, const void *xf_dev, int prec, const int32_t *pids,
                      int32_t n_req, const double *x, const double *q2, int64_t n_pts,
                      const void *grad_out, void *grad_xf, double *grad_x, double *grad_q2,
                      int domain_mode, void *stream, void *fixed_ws, size_t fixed_cap);

}  // namespace pdfx

struct pdfx_set {
    std::vector<pdfx_grid *> members;
    std::vector<int32_t> pids;               // shared by every member
    pdfx::DeviceBuf mem_desc;                // MemberDev[n_mem]
    pdfx::DeviceBuf counter;                 // work-list cursor
    pdfx::DeviceBuf dom_count;
    pdfx::DeviceBuf call_count;              // PDFX_DOMAIN_ERROR calls, as for a grid
    mutable int64_t host_count = 0;
    pdfx::LaunchShape shape[2] = {{512, 2}, {512, 2}};
    int tiles_per_item[2] = {4, 4};
    int cus = 256;
    // double-buffered classes (set_dma.hip): members by node width, per precision
    pdfx::DeviceBuf dma_mem;                 // SetMemberDev[n_mem]
    std::vector<pdfx::DeviceBuf *> dma_vals; // group slabs of every member and precision
    int max_nx = 0, max_nq = 0;              // largest member grid (tuning key)
    std::vector<int> cls_ids[2][pdfx::kSetClasses];   // members per class (kSetClassWidth, kSetClassSplit)
    std::vector<int> rest_ids[2];            // members left to the single-slab kernel
    pdfx::DeviceBuf order_dev[2];            // the classes' work list: (member, class) pairs
    int n_order[2] = {0, 0};
    pdfx::DeviceBuf rest_dev[2];             // rest_ids on the device
    ~pdfx_set();
};
