// Forward kernels: batched x f(x, Q^2) and alpha_s(Q^2) for gfx950.
//
// Work decomposition (one workgroup = BLOCK threads, PPT points per thread):
//   1. each thread streams its PPT points (coalesced FP64 loads of x and Q^2),
//      locates them (bucket seed + walk on raw knot values), forms ln x, ln Q^2
//      and the 4+4 folded Hermite weights, all kept in registers;
//   2. for every requested flavour the workgroup stages that flavour's slab
//      [n_x][n_q] into LDS (with a zero border one knot wide, so a stencil that
//      hangs over an axis end reads 0 under a weight of exactly 0) and every
//      point does its 16-tap stencil out of LDS;
//   3. results go straight to out[p][r].
// Flavours are walked forwards on even tiles and backwards on odd tiles, so
// the slab left in LDS by one tile is the first one the next tile needs.
// This is gather-plus-stencil work with no contraction: no MFMA.
#include "pdfx_internal.h"

namespace pdfx {

namespace {

__device__ __forceinline__ int axis_bin(const AxisDev &a, double v, double lnv)
{
    double fb = (lnv - a.ln_lo) * a.inv_hb;
    int b = fb <= 0.0 ? 0 : (fb >= (double)(a.nbuckets - 1) ? a.nbuckets - 1 : (int)fb);
    int i = a.seed[b];
    // The seed is only a starting point: the two walks below make i the
    // largest index with knots[i] <= v, clamped to n-2, whatever the seed.
    while (i < a.n - 2 && a.knots[i + 1] <= v)
        ++i;
    while (i > 0 && a.knots[i] > v)
        --i;
    return i;
}

template <typename W>
__device__ __forceinline__ void fold_weights(W t, W pl, W plql, W ql, W qr, W qrpr, W pr, W w[4])
{
    W t2 = t * t;
    W t3 = t2 * t;
    W h00 = W(2) * t3 - W(3) * t2 + W(1);
    W h10 = t3 - W(2) * t2 + t;
    W h01 = W(-2) * t3 + W(3) * t2;
    W h11 = t3 - t2;
    w[0] = -h10 * pl;
    w[1] = h00 + h10 * plql - h11 * qr;
    w[2] = h01 + h10 * ql + h11 * qrpr;
    w[3] = h11 * pr;
}

template <typename W>
__device__ __forceinline__ void axis_weights(const AxisDev &a, int i, double lnv, W w[4]);

template <>
__device__ __forceinline__ void axis_weights<double>(const AxisDev &a, int i, double lnv, double w[4])
{
    const IntervalRec<double> r = a.rec64[i];
    double t = (lnv - r.z) * r.inv_d;
    fold_weights<double>(t, r.pl, r.plql, r.ql, r.qr, r.qrpr, r.pr, w);
}

template <>
__device__ __forceinline__ void axis_weights<float>(const AxisDev &a, int i, double lnv, float w[4])
{
    const double z = a.rec64[i].z;
    const double inv_d = a.rec64[i].inv_d;
    const IntervalRec<float> r = a.rec32[i];
    float t = (float)((lnv - z) * inv_d);
    fold_weights<float>(t, r.pl, r.plql, r.ql, r.qr, r.qrpr, r.pr, w);
}

template <typename V>
__device__ __forceinline__ V quiet_nan();
template <>
__device__ __forceinline__ double quiet_nan<double>() { return __builtin_nan(""); }
template <>
__device__ __forceinline__ float quiet_nan<float>() { return __builtin_nanf(""); }

// Clamp or flag a point; returns true if the point is evaluated.
__device__ __forceinline__ bool domain(const XfxArgs &a, double &xv, double &qv)
{
    bool nan_in = (xv != xv) || (qv != qv);
    bool inside = xv >= a.ax.lo && xv <= a.ax.hi && qv >= a.aq.lo && qv <= a.aq.hi;
    if (inside)
        return true;
    if (a.domain_mode == 1 && !nan_in) {
        xv = fmin(fmax(xv, a.ax.lo), a.ax.hi);
        qv = fmin(fmax(qv, a.aq.lo), a.aq.hi);
        return true;
    }
    xv = a.ax.lo;
    qv = a.aq.lo;
    return false;
}

__device__ __forceinline__ void count_flagged(bool flagged, unsigned long long *counter)
{
    unsigned long long m = __ballot(flagged);
    if (m != 0ull && (threadIdx.x & 63) == 0)
        atomicAdd(counter, (unsigned long long)__popcll(m));
}

template <typename V, int BLOCK>
__device__ __forceinline__ void stage_slab(V *slab, const V *src, int nx, int nq, int nqp)
{
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    for (int i = wave; i < nx; i += BLOCK / 64) {
        const V *srow = src + (size_t)i * nq;
        V *drow = slab + (i + 1) * nqp + 1;
        for (int k = lane; k < nq; k += 64)
            drow[k] = srow[k];
    }
}

template <typename V, int BLOCK, int PPT>
__global__ __launch_bounds__(BLOCK) void xfx_kernel(const XfxArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    V *slab = reinterpret_cast<V *>(smem);
    const int nqp = a.nq + 2;
    const int nxp = a.nx + 2;
    const int tid = threadIdx.x;

    // Zero border of the slab (staging never writes it).
    for (int e = tid; e < nqp; e += BLOCK) {
        slab[e] = V(0);
        slab[(nxp - 1) * nqp + e] = V(0);
    }
    for (int i = tid; i < a.nx; i += BLOCK) {
        slab[(i + 1) * nqp] = V(0);
        slab[(i + 1) * nqp + nqp - 1] = V(0);
    }

    const int64_t tile_pts = (int64_t)BLOCK * PPT;
    const int64_t ntiles = (a.n + tile_pts - 1) / tile_pts;
    const V *vals = reinterpret_cast<const V *>(a.vals);
    V *out = reinterpret_cast<V *>(a.out);
    const int n_req = a.n_req;
    int staged = -1;
    int dir = 0;

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x, dir ^= 1) {
        V wx[PPT][4], wq[PPT][4];
        int base[PPT];
        bool ok[PPT];
        bool live[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int64_t p = tile * tile_pts + (int64_t)j * BLOCK + tid;
            live[j] = p < a.n;
            double xv = live[j] ? a.x[p] : a.ax.lo;
            double qv = live[j] ? a.q[p] : a.aq.lo;
            if (a.q_is_q)
                qv = qv * qv;
            ok[j] = domain(a, xv, qv);
            count_flagged(live[j] && !ok[j], a.dom_count);
            const double lx = log(xv);
            const double lq = log(qv);
            const int ix = axis_bin(a.ax, xv, lx);
            const int kq = axis_bin(a.aq, qv, lq);
            axis_weights<V>(a.ax, ix, lx, wx[j]);
            axis_weights<V>(a.aq, kq, lq, wq[j]);
            // slab index of knot (ix-1, kq-1) in the bordered layout
            base[j] = ix * nqp + kq;
        }

        for (int c = 0; c < n_req; ++c) {
            const int r = dir ? (n_req - 1 - c) : c;
            const int row = a.rows[r];
            if (row < 0) {
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    const int64_t p = tile * tile_pts + (int64_t)j * BLOCK + tid;
                    if (live[j])
                        out[p * n_req + r] = V(0);
                }
                continue;
            }
            if (row != staged) {
                __syncthreads();
                stage_slab<V, BLOCK>(slab, vals + (size_t)row * a.nx * a.nq, a.nx, a.nq, nqp);
                __syncthreads();
                staged = row;
            }
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const V *s0 = slab + base[j];
                V acc = V(0);
#pragma unroll
                for (int jx = 0; jx < 4; ++jx) {
                    const V *s = s0 + jx * nqp;
                    V rowsum = wq[j][0] * s[0];
                    rowsum = fma(wq[j][1], s[1], rowsum);
                    rowsum = fma(wq[j][2], s[2], rowsum);
                    rowsum = fma(wq[j][3], s[3], rowsum);
                    acc = (jx == 0) ? wx[j][0] * rowsum : fma(wx[j][jx], rowsum, acc);
                }
                const int64_t p = tile * tile_pts + (int64_t)j * BLOCK + tid;
                if (live[j])
                    out[p * n_req + r] = ok[j] ? acc : quiet_nan<V>();
            }
        }
    }
}

template <typename V>
__global__ __launch_bounds__(256) void alphas_kernel(const AlphasArgs a)
{
    const V *vals = reinterpret_cast<const V *>(a.vals);
    V *out = reinterpret_cast<V *>(a.out);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.n;
         p += (int64_t)gridDim.x * blockDim.x) {
        double qv = a.q2[p];
        bool nan_in = qv != qv;
        bool inside = qv >= a.a.lo && qv <= a.a.hi;
        bool ok = true;
        if (!inside) {
            if (a.domain_mode == 1 && !nan_in) {
                qv = fmin(fmax(qv, a.a.lo), a.a.hi);
            } else {
                ok = false;
                qv = a.a.lo;
            }
        }
        count_flagged(!ok, a.dom_count);
        const double lq = log(qv);
        const int k = axis_bin(a.a, qv, lq);
        V w[4];
        axis_weights<V>(a.a, k, lq, w);
        // padded values: vals[k'] holds knot k'-1, so knot k-1 is vals[k]
        V acc = w[0] * vals[k];
        acc = fma(w[1], vals[k + 1], acc);
        acc = fma(w[2], vals[k + 2], acc);
        acc = fma(w[3], vals[k + 3], acc);
        out[p] = ok ? acc : quiet_nan<V>();
    }
}

template <typename V, int BLOCK, int PPT>
hipError_t launch_one(const XfxArgs &a, int max_blocks, hipStream_t s)
{
    const int64_t tile_pts = (int64_t)BLOCK * PPT;
    const int64_t ntiles = (a.n + tile_pts - 1) / tile_pts;
    const int64_t grid = ntiles < max_blocks ? ntiles : max_blocks;
    const size_t lds = xfx_lds_bytes(a.nx, a.nq, sizeof(V) == 4);
    auto fn = xfx_kernel<V, BLOCK, PPT>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(BLOCK), lds, s, a);
    return hipGetLastError();
}

// Compiled launch shapes: (block, points per thread).
constexpr LaunchShape kShapes[] = {{256, 1}, {256, 2}, {256, 4}, {512, 2}, {512, 4}, {1024, 2}};

template <typename V>
hipError_t dispatch(const XfxArgs &a, LaunchShape ls, int max_blocks, hipStream_t s)
{
    if (ls.block == 256 && ls.ppt == 1) return launch_one<V, 256, 1>(a, max_blocks, s);
    if (ls.block == 256 && ls.ppt == 2) return launch_one<V, 256, 2>(a, max_blocks, s);
    if (ls.block == 256 && ls.ppt == 4) return launch_one<V, 256, 4>(a, max_blocks, s);
    if (ls.block == 512 && ls.ppt == 2) return launch_one<V, 512, 2>(a, max_blocks, s);
    if (ls.block == 512 && ls.ppt == 4) return launch_one<V, 512, 4>(a, max_blocks, s);
    if (ls.block == 1024 && ls.ppt == 2) return launch_one<V, 1024, 2>(a, max_blocks, s);
    return hipErrorInvalidValue;
}

}  // namespace

size_t xfx_lds_bytes(int nx, int nq, bool f32)
{
    return (size_t)(nx + 2) * (nq + 2) * (f32 ? 4 : 8);
}

bool launch_shape_supported(LaunchShape ls)
{
    for (const auto &k : kShapes)
        if (k.block == ls.block && k.ppt == ls.ppt)
            return true;
    return false;
}

int n_launch_shapes() { return (int)(sizeof(kShapes) / sizeof(kShapes[0])); }
LaunchShape launch_shape_at(int i) { return kShapes[i]; }

hipError_t launch_xfx_f64(const XfxArgs &a, LaunchShape ls, int max_blocks, hipStream_t s)
{
    return dispatch<double>(a, ls, max_blocks, s);
}

hipError_t launch_xfx_f32s(const XfxArgs &a, LaunchShape ls, int max_blocks, hipStream_t s)
{
    return dispatch<float>(a, ls, max_blocks, s);
}

hipError_t launch_alphas(const AlphasArgs &a, bool f32, hipStream_t s)
{
    int64_t blocks = (a.n + 255) / 256;
    if (blocks > 8192)
        blocks = 8192;
    if (blocks < 1)
        blocks = 1;
    if (f32)
        hipLaunchKernelGGL(alphas_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(alphas_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace pdfx
