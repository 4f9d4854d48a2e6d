"""The allocation-free adjoint, pdfx_eval_xfx_backward_noalloc, against the
allocating pdfx_eval_xfx_backward, through the C ABI: two calls in a row on
the same grid, the second with fewer points (so the shared scratch array
holds the first call's contents), in both precisions, with owned and with
caller-provided grid values.  Knot gradients are summed across workgroups
with FP64 atomics, so they agree to the rounding of that order; coordinate
gradients are written without atomics and agree bit for bit.  A call too
large for the scratch array is rejected and writes nothing."""
import numpy as np
import pytest

from helpers import cfg0_grid
from paper_2012_08221_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _grads(torch, B, fn, pdf, prec, pids, x, q2, gout, values):
    dt = torch.float64 if prec == B.PDFX_F64 else torch.float32
    gv = torch.zeros(pdf.shape, dtype=dt, device="cuda")
    gx = torch.full_like(x, -1.0)
    gq = torch.full_like(q2, -1.0)
    fn(pdf.handle, None if values is None else values.data_ptr(), prec, pids, x.data_ptr(),
       q2.data_ptr(), x.numel(), gout.data_ptr(), gv.data_ptr(), gx.data_ptr(), gq.data_ptr(),
       B.PDFX_DOMAIN_NAN, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return gv.double().cpu().numpy(), gx.cpu().numpy(), gq.cpu().numpy()


@pytest.mark.parametrize("prec_name", ["f64", "f32s"])
def test_noalloc_matches_allocating_adjoint(torch, prec_name):
    from paper_2012_08221_amd import api
    from paper_2012_08221_amd import binding as B
    g = cfg0_grid()
    pdf = api.mkPDF(g)
    prec = B.PDFX_F64 if prec_name == "f64" else B.PDFX_F32S
    dt = torch.float64 if prec == B.PDFX_F64 else torch.float32
    tol = 1e-12 if prec == B.PDFX_F64 else 2e-7
    pids = [int(p) for p in g.pids]
    for k, (n, values) in enumerate([(1_000_000, None), (300_001, None),
                                     (1_000_000, "caller"), (65_537, "caller")]):
        x_np, q2_np = wl.queries(60 + k, n)
        x_np[::1000] = 1e-12                      # a few points outside: NaN coordinate grads
        x = torch.as_tensor(x_np, device="cuda")
        q2 = torch.as_tensor(q2_np, device="cuda")
        gout = torch.as_tensor(wl.loss_weights(60 + k, n), device="cuda").to(dt)
        vals = None if values is None else torch.as_tensor(g.xf, device="cuda").to(dt)
        a = _grads(torch, B, B.pdfx_eval_xfx_backward, pdf, prec, pids, x, q2, gout, vals)
        b = _grads(torch, B, B.pdfx_eval_xfx_backward_noalloc, pdf, prec, pids, x, q2, gout, vals)
        scale = np.abs(a[0]).max(axis=(1, 2), keepdims=True)
        assert np.all(np.abs(b[0] - a[0]) <= tol * scale), (n, values)
        assert np.abs(a[0]).max() > 0
        np.testing.assert_array_equal(b[1], a[1])
        np.testing.assert_array_equal(b[2], a[2])
        assert np.isnan(b[1][::1000]).all() and np.isfinite(b[1][1::1000]).all()


def test_noalloc_rejects_calls_beyond_its_scratch(torch):
    from paper_2012_08221_amd import api
    from paper_2012_08221_amd import binding as B
    g = cfg0_grid()
    pdf = api.mkPDF(g)
    per_point = 4 + 1 + 4 * 8
    n = B.PDFX_NOALLOC_SCRATCH_BYTES // per_point + 1000
    x = torch.full((n,), 0.1, dtype=torch.float64, device="cuda")
    q2 = torch.full((n,), 100.0, dtype=torch.float64, device="cuda")
    gout = torch.ones((n, 11), dtype=torch.float64, device="cuda")
    gx = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    gv = torch.zeros(pdf.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(B.PdfxError) as e:
        B.pdfx_eval_xfx_backward_noalloc(pdf.handle, None, B.PDFX_F64, [int(p) for p in g.pids],
                                         x.data_ptr(), q2.data_ptr(), n, gout.data_ptr(),
                                         gv.data_ptr(), gx.data_ptr(), None, B.PDFX_DOMAIN_NAN,
                                         torch.cuda.current_stream().cuda_stream)
    assert e.value.code == B.PDFX_EINVAL and "allocation-free" in str(e.value)
    torch.cuda.synchronize()
    assert bool((gx == -1.0).all()) and bool((gv == 0.0).all())
