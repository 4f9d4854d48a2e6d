// Copies caller-provided values [nf][nx][nq] into the bordered slab layout the
// forward kernels stage from: [nf][slab_elems], slab (nx+2) x (nq+2) with a
// zero border one knot wide, zero-filled up to slab_elems.
#include "pdfx_internal.h"

namespace pdfx {

namespace {

template <typename V>
__global__ __launch_bounds__(256) void repack_kernel(const RepackArgs a)
{
    const V *src = reinterpret_cast<const V *>(a.src);
    V *dst = reinterpret_cast<V *>(a.dst);
    const int nqp = a.nq + 2;
    const int64_t total = (int64_t)a.nf * a.slab_elems;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int f = (int)(e / a.slab_elems);
        const int r = (int)(e - (int64_t)f * a.slab_elems);
        const int i = r / nqp, k = r - i * nqp;
        V v = V(0);
        if (i >= 1 && i <= a.nx && k >= 1 && k <= a.nq)
            v = src[((int64_t)f * a.nx + (i - 1)) * a.nq + (k - 1)];
        dst[e] = v;
    }
}

}  // namespace

hipError_t launch_repack(const RepackArgs &a, bool f32, hipStream_t s)
{
    const int64_t total = (int64_t)a.nf * a.slab_elems;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 2048)
        blocks = 2048;
    if (f32)
        hipLaunchKernelGGL(repack_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(repack_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace pdfx
