// LDS read and atomic rates of the device, measured: the ceilings the
// stencil and gradient kernels are held to.  The stencils are aligned
// 16-byte LDS reads at data-dependent addresses, the gradient scatters 64-bit
// LDS atomic adds (FP64, or integer for fixed-point sums); for each, two
// patterns bracket the kernels' own:
// lane-consecutive addresses (no bank conflicts) and independent random
// ones (the pattern for points in random order).
#include "runtime_internal.h"

namespace pdfx {
namespace {

constexpr int kMbBlock = 256;
constexpr int kMbLdsBytes = 64 * 1024;
constexpr int kMbChunks = kMbLdsBytes / 16;   // power of two

template <bool RANDOM>
__global__ __launch_bounds__(kMbBlock) void lds_read_kernel(int iters, unsigned seed, double *sink)
{
    __shared__ __align__(16) double s[kMbLdsBytes / 8];
    for (int i = threadIdx.x; i < kMbLdsBytes / 8; i += kMbBlock)
        s[i] = (double)i;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    unsigned r = seed ^ (threadIdx.x * 2654435761u) ^ (blockIdx.x * 40503u);
    double acc = 0.0;
#pragma unroll 8
    for (int it = 0; it < iters; ++it) {
        int c;
        if (RANDOM) {
            r = r * 1664525u + 1013904223u;   // Numerical Recipes LCG
            c = (int)(r >> 12) & (kMbChunks - 1);
        } else {
            c = ((it * (kMbBlock / 64) + wave) * 64 + lane) & (kMbChunks - 1);
        }
        const double2 v = *reinterpret_cast<const double2 *>(&s[2 * c]);
        acc += v.x + v.y;
    }
    sink[(size_t)blockIdx.x * kMbBlock + threadIdx.x] = acc;
}

// 64-bit LDS atomic adds (no return), FP64 or integer (T), as the gradient
// scatters make them: at lane-consecutive 8-byte addresses, or at
// independent random ones.
template <typename T, bool RANDOM>
__global__ __launch_bounds__(kMbBlock) void lds_atomic_kernel(int iters, unsigned seed, double *sink)
{
    __shared__ T s[kMbLdsBytes / 8];
    for (int i = threadIdx.x; i < kMbLdsBytes / 8; i += kMbBlock)
        s[i] = T(0);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    unsigned r = seed ^ (threadIdx.x * 2654435761u) ^ (blockIdx.x * 40503u);
    const T v = T(1 + threadIdx.x);
#pragma unroll 8
    for (int it = 0; it < iters; ++it) {
        int c;
        if (RANDOM) {
            r = r * 1664525u + 1013904223u;
            c = (int)(r >> 12) & (kMbLdsBytes / 8 - 1);
        } else {
            c = ((it * (kMbBlock / 64) + wave) * 64 + lane) & (kMbLdsBytes / 8 - 1);
        }
        atomicAdd(&s[c], v);
    }
    __syncthreads();
    sink[(size_t)blockIdx.x * kMbBlock + threadIdx.x] = (double)s[threadIdx.x];
}

}  // namespace
}  // namespace pdfx

using namespace pdfx;

extern "C" int pdfx_bench_lds(int mode, int blocks, int iters, double *sink, void *stream)
{
    clear_error();
    if (mode < 0 || mode > 5)
        return fail(PDFX_EINVAL, "unknown mode %d", mode);
    if (blocks <= 0 || iters <= 0)
        return fail(PDFX_EINVAL, "blocks and iters must be positive");
    if (!sink)
        return fail(PDFX_EINVAL, "sink is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (mode == 0)
        hipLaunchKernelGGL(lds_read_kernel<false>, dim3(blocks), dim3(kMbBlock), 0, s, iters, 1u, sink);
    else if (mode == 1)
        hipLaunchKernelGGL(lds_read_kernel<true>, dim3(blocks), dim3(kMbBlock), 0, s, iters, 1u, sink);
    else if (mode == 2)
        hipLaunchKernelGGL((lds_atomic_kernel<double, false>), dim3(blocks), dim3(kMbBlock), 0, s,
                           iters, 1u, sink);
    else if (mode == 3)
        hipLaunchKernelGGL((lds_atomic_kernel<double, true>), dim3(blocks), dim3(kMbBlock), 0, s,
                           iters, 1u, sink);
    else if (mode == 4)
        hipLaunchKernelGGL((lds_atomic_kernel<unsigned long long, false>), dim3(blocks),
                           dim3(kMbBlock), 0, s, iters, 1u, sink);
    else
        hipLaunchKernelGGL((lds_atomic_kernel<unsigned long long, true>), dim3(blocks),
                           dim3(kMbBlock), 0, s, iters, 1u, sink);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail_hip(e, "LDS micro-benchmark launch");
    return PDFX_OK;
}
