// Flavour-pair luminosity: arguments shared by the host runtime and lumi_dma.hip.
#pragma once

#include "pdfx_internal.h"

namespace pdfx {

// Pairs per call (an 11 x 11 luminosity matrix fits).
constexpr int kLumiMaxPairs = 128;

// L_k(p) = f_{a_k}(x1_p, Q^2_p) f_{b_k}(x2_p, Q^2_p) with f = xf / x, and
// S(p) = sum_k c_k L_k(p), for the pairs (a_k, b_k) of a user integrand
// (Eq. 1's luminosity; the single-top example of Fig. 4).
struct LumiArgs {
    AxisDev ax, aq;
    int nx, nq;
    const void *gvals;            // borderless flavour-group node slabs
    int gstride;                  // nodes per group
    int n_stage;                  // flavour groups touched, grid order
    int sgrp[kGrpMaxSlots];       // group of stage s
    int side[kGrpMaxSlots];       // bit 0: stencil at (x1, Q^2), bit 1: at (x2, Q^2)
    int n_pair;
    int ia[kLumiMaxPairs];        // result slot s*G+g of a_k at x1, or -1 (absent: L_k = 0)
    int ib[kLumiMaxPairs];        // result slot of b_k at x2, or -1
    double coef[kLumiMaxPairs];   // c_k
    const double *x1, *x2;        // [n]
    const double *q2;             // [n], or null: q2_fixed for every point
    double q2_fixed;
    int64_t n;
    void *out_pair;               // [n][n_pair] or null
    void *out_sum;                // [n] or null
    int domain_mode;
    unsigned long long *dom_count;
};

bool lumi_supported(int nx, int nq, int nbx, int nbq);
bool lumi_shape_supported(LaunchShape ls, bool f32);
hipError_t launch_lumi(const LumiArgs &a, bool f32, LaunchShape ls, int cus, hipStream_t s);

}  // namespace pdfx
