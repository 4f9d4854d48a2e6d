// Entry points whose kernels are not built yet: they fail cleanly.
#include "../../include/pdfx.h"
#include "runtime_internal.h"

using namespace pdfx;

extern "C" {

int pdfx_load_set(const pdfx_grid_desc *, int32_t, pdfx_set **out)
{
    if (out)
        *out = nullptr;
    return fail(PDFX_EINVAL, "pdfx_load_set: not available in this build");
}

void pdfx_free_set(pdfx_set *) {}

int pdfx_eval_set_xfx(const pdfx_set *, int, const int32_t *, int32_t, const double *,
                      const double *, int64_t, void *, int, void *)
{
    return fail(PDFX_EINVAL, "pdfx_eval_set_xfx: not available in this build");
}

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

int pdfx_autotune(pdfx_grid *, int, int32_t, int64_t, const char *)
{
    return fail(PDFX_EINVAL, "pdfx_autotune: not available in this build");
}

int pdfx_autotune_set(pdfx_set *, int, int32_t, int64_t, const char *)
{
    return fail(PDFX_EINVAL, "pdfx_autotune_set: not available in this build");
}

}  // extern "C"
