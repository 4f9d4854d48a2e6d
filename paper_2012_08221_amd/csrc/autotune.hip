// Launch-shape tuner for the forward and set kernels.
//
// Times every compiled launch shape on scratch buffers of the real shape
// (points drawn log-uniformly inside the grid by a counter-based hash on the
// device), keeps the fastest, and optionally records the choice in a
// JSON-lines cache: one object per line,
//   {"key": "<arch>|cu<N>|<kind>|<signature>|p<prec>|r<n_req>|n2^<k>", "block": B, "ppt": P, "tpi": T}
// so a later process with the same device and workload skips the timing.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/pdfx.h"
#include "pdfx_internal.h"
#include "runtime_internal.h"

namespace pdfx {

namespace {

// splitmix64 finaliser: a counter-based generator of uniform 64-bit words.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void synth_points(double *x, double *q2, int64_t n, double lx0,
                                                    double lx1, double lq0, double lq1)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double u = (double)(mix64(2 * i) >> 11) * 0x1.0p-53;
        const double v = (double)(mix64(2 * i + 1) >> 11) * 0x1.0p-53;
        x[i] = exp(lx0 + u * (lx1 - lx0));
        q2[i] = exp(lq0 + v * (lq1 - lq0));
    }
}

std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess)
        return "unknown";
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

struct CacheEntry {
    int block = 0, ppt = 0, tpi = 0;
    bool found = false;
};

CacheEntry cache_lookup(const char *path, const std::string &key)
{
    CacheEntry ce;
    if (!path)
        return ce;
    std::ifstream in(path);
    std::string line;
    const std::string needle = "\"key\": \"" + key + "\"";
    while (std::getline(in, line)) {
        if (line.find(needle) == std::string::npos)
            continue;
        int b = 0, p = 0, t = 0;
        const char *s = std::strstr(line.c_str(), "\"block\":");
        const char *q = std::strstr(line.c_str(), "\"ppt\":");
        const char *r = std::strstr(line.c_str(), "\"tpi\":");
        if (s && q && r && std::sscanf(s, "\"block\": %d", &b) == 1 &&
            std::sscanf(q, "\"ppt\": %d", &p) == 1 && std::sscanf(r, "\"tpi\": %d", &t) == 1) {
            ce.block = b;
            ce.ppt = p;
            ce.tpi = t;
            ce.found = true;   // the last matching line wins
        }
    }
    return ce;
}

void cache_store(const char *path, const std::string &key, int block, int ppt, int tpi, double ms)
{
    if (!path)
        return;
    std::ofstream out(path, std::ios::app);
    out << "{\"key\": \"" << key << "\", \"block\": " << block << ", \"ppt\": " << ppt
        << ", \"tpi\": " << tpi << ", \"ms\": " << ms << "}\n";
}

// Minimum over `reps` timed calls of fn(stream).
template <typename F>
double time_min(F fn, hipStream_t s, int reps)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return 1e30;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return 1e30;
    }
    double best = 1e30;
    if (fn(s) != PDFX_OK) {   // warm-up; also rejects shapes that cannot launch
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return 1e30;
    }
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(e0, s);
        const int rc = fn(s);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        if (rc == PDFX_OK && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < best)
            best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

struct Scratch {
    DeviceBuf x, q2, out;
    int64_t n = 0;
    int make(const AxisHost &ax, const AxisHost &aq, int64_t n_pts, size_t out_bytes)
    {
        n = n_pts;
        hipError_t e;
        if ((e = x.upload(nullptr, n * 8)) != hipSuccess || (e = q2.upload(nullptr, n * 8)) != hipSuccess ||
            (e = out.upload(nullptr, out_bytes)) != hipSuccess)
            return fail_hip(e, "allocate tuning buffers");
        int64_t blocks = (n + 255) / 256;
        if (blocks > 4096)
            blocks = 4096;
        hipLaunchKernelGGL(synth_points, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)0,
                           (double *)x.ptr, (double *)q2.ptr, n, std::log(ax.knots.front()),
                           std::log(ax.knots.back()), std::log(aq.knots.front()),
                           std::log(aq.knots.back()));
        if ((e = hipGetLastError()) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess)
            return fail_hip(e, "generate tuning points");
        return PDFX_OK;
    }
};

int size_class(int64_t n)
{
    int k = 0;
    while ((1LL << (k + 1)) <= n)
        ++k;
    return k;
}

}  // namespace

}  // namespace pdfx

using namespace pdfx;

extern "C" int pdfx_autotune(pdfx_grid *g, int prec, int32_t n_req, int64_t n_pts,
                             const char *cache_path)
{
    clear_error();
    if (!g)
        return fail(PDFX_EINVAL, "grid is NULL");
    if (prec != PDFX_F64 && prec != PDFX_F32S)
        return fail(PDFX_EINVAL, "unknown precision %d", prec);
    if (n_req < 1 || n_req > PDFX_MAX_REQ || n_pts < 1)
        return fail(PDFX_EINVAL, "need 1 <= n_req <= %d and n_pts >= 1", PDFX_MAX_REQ);
    if (!g->has_values)
        return fail(PDFX_ENOVALUES, "tuning needs owned values");
    std::ostringstream key;
    key << arch_name() << "|cu" << g->cus << "|xfx|" << g->nf << "x" << g->ax.n << "x" << g->aq.n
        << "s" << g->n_sub << "|p" << prec << "|r" << n_req << "|n2^" << size_class(n_pts);
    CacheEntry ce = cache_lookup(cache_path, key.str());
    const LaunchShape cached{ce.block, ce.ppt};
    if (ce.found && (launch_shape_supported(cached) ||
                     (prec == PDFX_F32S && launch_shape_f32_only(cached)))) {
        g->shape[prec] = cached;
        g->shape_pinned[prec] = false;
        return PDFX_OK;
    }
    const int64_t n = n_pts < (1LL << 23) ? n_pts : (1LL << 23);
    std::vector<int32_t> pids(n_req);
    for (int r = 0; r < n_req; ++r)
        pids[r] = g->pids[r % g->nf];
    Scratch sc;
    int rc = sc.make(g->ax, g->aq, n, (size_t)n * n_req * (prec == PDFX_F64 ? 8 : 4));
    if (rc != PDFX_OK)
        return rc;
    const LaunchShape keep = g->shape[prec];
    double best = 1e30;
    LaunchShape best_ls = keep;
    std::vector<LaunchShape> cand;
    for (int i = 0; i < n_launch_shapes(); ++i)
        cand.push_back(launch_shape_at(i));
    if (prec == PDFX_F32S)
        cand.push_back(LaunchShape{512, 4});
    g->shape_pinned[prec] = true;   // each candidate runs as it is
    for (const LaunchShape ls : cand) {
        g->shape[prec] = ls;
        g->reset_occupancy(prec);
        const double ms = time_min(
            [&](hipStream_t s) {
                return pdfx_eval_xfx(g, nullptr, prec, pids.data(), n_req, (const double *)sc.x.ptr,
                                     (const double *)sc.q2.ptr, n, sc.out.ptr, PDFX_DOMAIN_NAN, s);
            },
            (hipStream_t)0, 3);
        if (ms < best) {
            best = ms;
            best_ls = ls;
        }
    }
    g->shape[prec] = best_ls;
    g->shape_pinned[prec] = false;
    g->reset_occupancy(prec);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess)
        return fail_hip(e, "tuning");
    if (best >= 1e30)
        return fail(PDFX_EHIP, "no launch shape ran");
    cache_store(cache_path, key.str(), best_ls.block, best_ls.ppt, 0, best);
    return PDFX_OK;
}

extern "C" int pdfx_autotune_set(pdfx_set *s, int prec, int32_t n_req, int64_t n_pts,
                                 const char *cache_path)
{
    clear_error();
    if (!s)
        return fail(PDFX_EINVAL, "set is NULL");
    if (prec != PDFX_F64 && prec != PDFX_F32S)
        return fail(PDFX_EINVAL, "unknown precision %d", prec);
    if (n_req < 1 || n_req > PDFX_MAX_REQ || n_pts < 1)
        return fail(PDFX_EINVAL, "need 1 <= n_req <= %d and n_pts >= 1", PDFX_MAX_REQ);
    const pdfx_grid *g0 = s->members[0];
    std::ostringstream key;
    key << arch_name() << "|cu" << s->cus << "|set|" << s->members.size() << "m" << g0->nf << "f"
        << s->max_nx << "x" << s->max_nq << "|p" << prec << "|r" << n_req << "|n2^"
        << size_class(n_pts);
    CacheEntry ce = cache_lookup(cache_path, key.str());
    const LaunchShape cached_set{ce.block, ce.ppt};
    if (ce.found && ce.tpi >= 1 &&
        (set_shape_supported(cached_set) ||
         (prec == PDFX_F32S && launch_shape_f32_only(cached_set)))) {
        s->shape[prec] = LaunchShape{ce.block, ce.ppt};
        s->tiles_per_item[prec] = ce.tpi;
        return PDFX_OK;
    }
    // tune on a subset of the points (all members, up to 2^18 points)
    const int64_t n = n_pts < (1LL << 18) ? n_pts : (1LL << 18);
    std::vector<int32_t> pids(n_req);
    for (int r = 0; r < n_req; ++r)
        pids[r] = s->pids[r % s->pids.size()];
    Scratch sc;
    int rc = sc.make(g0->ax, g0->aq, n,
                     (size_t)n * n_req * s->members.size() * (prec == PDFX_F64 ? 8 : 4));
    if (rc != PDFX_OK)
        return rc;
    double best = 1e30;
    LaunchShape best_ls = s->shape[prec];
    int best_tpi = s->tiles_per_item[prec];
    std::vector<LaunchShape> cand;
    for (int i = 0; i < n_set_shapes(); ++i)
        cand.push_back(set_shape_at(i));
    if (prec == PDFX_F32S)
        cand.push_back(LaunchShape{512, 4});
    for (const LaunchShape ls : cand) {
        for (int tpi : {1, 2, 4, 8}) {
            s->shape[prec] = ls;
            s->tiles_per_item[prec] = tpi;
            const double ms = time_min(
                [&](hipStream_t st) {
                    return pdfx_eval_set_xfx(s, prec, pids.data(), n_req, (const double *)sc.x.ptr,
                                             (const double *)sc.q2.ptr, n, sc.out.ptr,
                                             PDFX_DOMAIN_CLAMP, st);
                },
                (hipStream_t)0, 2);
            if (ms < best) {
                best = ms;
                best_ls = ls;
                best_tpi = tpi;
            }
        }
    }
    s->shape[prec] = best_ls;
    s->tiles_per_item[prec] = best_tpi;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess)
        return fail_hip(e, "tuning");
    if (best >= 1e30)
        return fail(PDFX_EHIP, "no launch shape ran");
    cache_store(cache_path, key.str(), best_ls.block, best_ls.ppt, best_tpi, best);
    return PDFX_OK;
}
