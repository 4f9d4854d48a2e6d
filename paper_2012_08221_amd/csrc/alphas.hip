// alpha_s(Q^2): 1-D cubic Hermite in ln Q^2 over the alpha_s knots, subgrids
// split at repeated knots (same search, tie and weight rules as the PDF axis).
// Persistent workgroups; the axis tables live in LDS.
#include "xfx_fwd_impl.h"

namespace pdfx {

namespace {

constexpr int kAsBlock = 256;
constexpr int kAsPpt = 4;

template <typename V>
__global__ __launch_bounds__(kAsBlock) void alphas_kernel(const AlphasArgs a, AxisLds lo)
{
    extern __shared__ uint4 smem4[];
    char *sm = reinterpret_cast<char *>(smem4);
    fwd::load_axis<kAsBlock>(sm, a.a, lo, sizeof(V) == 4);
    fwd::copy_words<kAsBlock>(sm + lo.rec32 + (sizeof(V) == 4 ? (a.a.n - 1) * 32 : 0),
                              a.vals, ((a.a.n + 2) * (int)sizeof(V) + 7) / 8 * 8);
    __syncthreads();
    const fwd::LAxis la = fwd::lds_axis(sm, a.a, lo);
    const V *vals = reinterpret_cast<const V *>(sm + lo.rec32 + (sizeof(V) == 4 ? (a.a.n - 1) * 32 : 0));
    V *out = reinterpret_cast<V *>(a.out);
    const int64_t tile = (int64_t)kAsBlock * kAsPpt;
    for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < a.n; t0 += (int64_t)gridDim.x * tile) {
        // all of the thread's points first (clamped indices keep these global
        // loads; a select with a default value would make them flat loads)
        double qs[kAsPpt];
#pragma unroll
        for (int j = 0; j < kAsPpt; ++j)
            qs[j] = load_point(a.q2, t0 + (int64_t)j * kAsBlock + threadIdx.x, a.n);
#pragma unroll
        for (int j = 0; j < kAsPpt; ++j) {
            const int64_t p = t0 + (int64_t)j * kAsBlock + threadIdx.x;
            const bool live = p < a.n;
            double qv = qs[j];
            if (a.q_is_q)
                qv = qv * qv;
            const bool nan_in = qv != qv;
            bool ok = true;
            if (!(qv >= a.a.lo && qv <= a.a.hi)) {
                if (a.domain_mode == 1 && !nan_in) {
                    qv = fmin(fmax(qv, a.a.lo), a.a.hi);
                } else {
                    ok = false;
                    qv = a.a.lo;
                }
            }
            fwd::count_flagged(live && !ok, a.dom_count);
            const double lq = log(qv);
            const int k = fwd::lbin(la, qv, lq);
            V w[4];
            fwd::weights<V>(la, k, lq, w);
            // padded values: vals[k'] holds knot k'-1, so knot k-1 is vals[k]
            V acc = w[0] * vals[k];
            acc = fma(w[1], vals[k + 1], acc);
            acc = fma(w[2], vals[k + 2], acc);
            acc = fma(w[3], vals[k + 3], acc);
            if (live)
                out[p] = ok ? acc : fwd::quiet_nan<V>();
        }
    }
}

}  // namespace

hipError_t launch_alphas(const AlphasArgs &a, bool f32, hipStream_t s)
{
    AxisLds lo;
    size_t off = 0;
    auto take = [&](size_t bytes, size_t align) {
        off = (off + align - 1) / align * align;
        size_t r = off;
        off += bytes;
        return (int)r;
    };
    lo.knots = take((size_t)a.a.n * 8, 16);
    lo.seed = take((size_t)a.a.nbuckets * 2, 16);
    lo.rec64 = take((size_t)(a.a.n - 1) * 64, 64);
    lo.rec32 = take((size_t)(a.a.n - 1) * 32 + (size_t)(a.a.n + 2) * 8 + 8, 64);
    const size_t lds = off;
    if (lds > kLdsLimit)
        return hipErrorInvalidValue;
    const int64_t tile = (int64_t)kAsBlock * kAsPpt;
    int64_t blocks = (a.n + tile - 1) / tile;
    if (blocks > 2048)
        blocks = 2048;
    if (blocks < 1)
        blocks = 1;
    if (f32)
        hipLaunchKernelGGL(alphas_kernel<float>, dim3((unsigned)blocks), dim3(kAsBlock), lds, s, a, lo);
    else
        hipLaunchKernelGGL(alphas_kernel<double>, dim3((unsigned)blocks), dim3(kAsBlock), lds, s, a, lo);
    return hipGetLastError();
}

}  // namespace pdfx
