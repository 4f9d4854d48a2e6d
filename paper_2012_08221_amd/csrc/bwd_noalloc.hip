// Allocation-free form of the adjoint, for callers that cannot allocate
// device memory: code under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc.  pdfx_eval_xfx_backward grows a per-grid workspace on
// demand; this call takes its workspace from `scratch`, a file-scope device
// array of fixed size that each GPU the library runs on holds until the
// process ends.
//
// The array's name in host code is a host-side stand-in, not a device
// address: its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// ever handed to kernels.  Every call on one GPU shares that GPU's array and
// finds the previous call's contents there; the adjoint clears what must
// start at zero with kernels on the call's stream, and calls that may overlap
// on one GPU (different streams, different host threads) race.
#include <mutex>

#include "runtime_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)PDFX_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
int scratch_address(void **ptr)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return pdfx::fail_hip(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return pdfx::fail(PDFX_EINVAL, "device %d beyond the %d the scratch table holds", dev,
                          kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return pdfx::fail_hip(e, "hipGetSymbolAddress(scratch)");
        if (!p)
            return pdfx::fail(PDFX_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return PDFX_OK;
}

}  // namespace

extern "C" int pdfx_eval_xfx_backward_noalloc(const pdfx_grid *g, const void *xf_dev, int prec,
                                              const int32_t *pids, int32_t n_req,
                                              const double *x, const double *q2, int64_t n_pts,
                                              const void *grad_out, void *grad_xf,
                                              double *grad_x, double *grad_q2, int domain_mode,
                                              void *stream)
{
    pdfx::clear_error();
    if (!g)
        return pdfx::fail(PDFX_EINVAL, "grid is NULL");
    void *ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc != PDFX_OK)
        return rc;
    return pdfx::eval_xfx_backward(g, xf_dev, prec, pids, n_req, x, q2, n_pts, grad_out, grad_xf,
                                   grad_x, grad_q2, domain_mode, stream, ws, kScratchBytes);
}
