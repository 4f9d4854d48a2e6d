// Copies caller-provided values [nf][nx][nq] into the layouts the forward
// kernels stage from: bordered slabs [nf][slab_elems], slab (nx+2) x (nq+2)
// with a zero border one knot wide, zero-filled up to slab_elems; or
// flavour-group node slabs (rows G at a time interleaved per knot).
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

// One thread per node component: dst[gi][node][g] = row gi*G+g of src at the
// node's knot; 0 past the last row, past the node slab and, with a border, on
// the border.
template <typename V>
__global__ __launch_bounds__(256) void grp_repack_kernel(const V *src, V *dst, int nf, int nx,
                                                         int nq, int gstride, int border,
                                                         int64_t total)
{
    constexpr int G = 16 / (int)sizeof(V);
    const int w = nq + 2 * border;   // nodes per slab row
    const int64_t per_group = (int64_t)gstride * G;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int gi = (int)(e / per_group);
        const int r = (int)(e - (int64_t)gi * per_group);
        const int node = r / G, g = r - node * G;
        const int i = node / w - border, k = node % w - border;
        const int row = gi * G + g;
        V v = V(0);
        if (row < nf && i >= 0 && i < nx && k >= 0 && k < nq)
            v = src[((int64_t)row * nx + i) * nq + k];
        dst[e] = v;
    }
}

}  // namespace

hipError_t launch_grp_repack(const void *src, void *dst, int nf, int nx, int nq, int n_groups,
                             int gstride, bool border, bool f32, hipStream_t s)
{
    const int64_t total = (int64_t)n_groups * gstride * (f32 ? 4 : 2);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 2048)
        blocks = 2048;
    if (blocks < 1)
        return hipSuccess;
    if (f32)
        hipLaunchKernelGGL(grp_repack_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const float *)src, (float *)dst, nf, nx, nq, gstride, border ? 1 : 0, total);
    else
        hipLaunchKernelGGL(grp_repack_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const double *)src, (double *)dst, nf, nx, nq, gstride, border ? 1 : 0, total);
    return hipGetLastError();
}

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
