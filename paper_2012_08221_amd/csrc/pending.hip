// Entry points whose kernels are not built yet: they fail cleanly.
#include "../../include/pdfx.h"
#include "runtime_internal.h"

using namespace pdfx;

extern "C" {

int pdfx_eval_dy(const pdfx_grid *, const void *, int, const double *, const double *, int64_t,
                 double, double, void *, double *, int32_t *, void *)
{
    return fail(PDFX_EINVAL, "pdfx_eval_dy: not available in this build");
}

int32_t pdfx_dy_max_blocks(void) { return 0; }

int pdfx_eval_dy_backward(const pdfx_grid *, const void *, int, const double *, const double *,
                          int64_t, double, double, double, void *, void *)
{
    return fail(PDFX_EINVAL, "pdfx_eval_dy_backward: not available in this build");
}

}  // extern "C"
