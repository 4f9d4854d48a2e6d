"""Boundary behaviour of the C ABI and the torch API on the GPU:

* domain mode PDFX_DOMAIN_ERROR (every forward call): the NAN-mode outputs
  bit for bit, PDFX_EDOMAIN exactly when some point is outside the grid or
  NaN, and the points added to the domain count;
* pdfx_eval_alphasQ: Q^2 = Q*Q formed on the device, bit for bit the
  alpha_s of the FP64 product (the paper's py_alphasQ, Fig. 1);
* the torch API rejects mismatched lengths, output and value tensors of the
  wrong shape, dtype or layout before anything is launched;
* a request served by one flavour group whose output rows are staged in the
  LDS slab that holds that group (more than one tile per workgroup): the
  next tile must see the group again, not the rows.
"""
import numpy as np
import pytest

import oracle
from helpers import capped_rel_err, cfg0_grid, cfg0_queries
from paper_2012_08221_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def api(torch):
    from paper_2012_08221_amd import api as a
    return a


@pytest.fixture(scope="module")
def B():
    from paper_2012_08221_amd import binding as b
    return b


@pytest.fixture(scope="module")
def pdf0(api):
    return api.mkPDF(cfg0_grid())


def _pts(n=20_003):
    return cfg0_queries(n)


def _with_outside(x, q2):
    x, q2 = x.copy(), q2.copy()
    x[[10, 500]] = [1e-12, np.nan]
    q2[[20, 700, 9000]] = [0.5, 2e10, np.nan]
    return x, q2, 5


# ---------------------------------------------------------------------------
# PDFX_DOMAIN_ERROR
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f64", "f32s"])
def test_error_mode_xfx(pdf0, torch, api, B, prec):
    g = cfg0_grid()
    x, q2 = _pts()
    pdf0.domain_errors()
    ok = pdf0.xfxQ2(g.pids, x, q2, prec=prec, domain="error").cpu().numpy()
    np.testing.assert_array_equal(ok, pdf0.xfxQ2(g.pids, x, q2, prec=prec).cpu().numpy())
    assert pdf0.domain_errors() == 0
    xb, qb, nbad = _with_outside(x, q2)
    out = torch.empty((x.size, 11), dtype=api.prec_dtype(prec), device="cuda")
    with pytest.raises(B.PdfxDomainError) as e:
        pdf0.xfxQ2(g.pids, xb, qb, prec=prec, domain="error", out=out)
    assert e.value.code == B.PDFX_EDOMAIN
    ref = pdf0.xfxQ2(g.pids, xb, qb, prec=prec, domain="nan").cpu().numpy()
    np.testing.assert_array_equal(out.cpu().numpy(), ref)
    assert pdf0.domain_errors() == 2 * nbad          # the ERROR call and the NAN call
    with pytest.raises(B.PdfxDomainError):
        pdf0.xfxQ(g.pids, xb, np.sqrt(qb), prec=prec, domain="error")
    assert pdf0.domain_errors() == nbad


@pytest.mark.parametrize("prec", ["f64", "f32s"])
def test_error_mode_alphas_and_one_pass(pdf0, torch, api, B, prec):
    g = cfg0_grid()
    x, q2 = _pts()
    pdf0.domain_errors()
    a = pdf0.alphasQ2(q2, prec=prec, domain="error").cpu().numpy()
    np.testing.assert_array_equal(a, pdf0.alphasQ2(q2, prec=prec).cpu().numpy())
    f, fa = pdf0.xfx_alphasQ2(g.pids, x, q2, prec=prec, domain="error")
    assert pdf0.domain_errors() == 0
    xb, qb, _ = _with_outside(x, q2)
    with pytest.raises(B.PdfxDomainError):
        pdf0.alphasQ2(qb, prec=prec, domain="error")
    with pytest.raises(B.PdfxDomainError):
        pdf0.alphasQ(np.sqrt(qb), prec=prec, domain="error")
    out = torch.empty((x.size, 11), dtype=api.prec_dtype(prec), device="cuda")
    aso = torch.empty(x.size, dtype=api.prec_dtype(prec), device="cuda")
    with pytest.raises(B.PdfxDomainError):
        pdf0.xfx_alphasQ2(g.pids, xb, qb, prec=prec, domain="error", out=out, as_out=aso)
    rf, ra = pdf0.xfx_alphasQ2(g.pids, xb, qb, prec=prec, domain="nan")
    np.testing.assert_array_equal(out.cpu().numpy(), rf.cpu().numpy())
    np.testing.assert_array_equal(aso.cpu().numpy(), ra.cpu().numpy())
    # x outside alone leaves alpha_s defined but is still an error for x f
    xo = x.copy()
    xo[3] = 2.0
    with pytest.raises(B.PdfxDomainError):
        pdf0.xfx_alphasQ2(g.pids, xo, q2, prec=prec, domain="error")
    pdf0.domain_errors()


@pytest.mark.parametrize("prec", ["f64", "f32s"])
def test_error_mode_set_and_lumi(api, torch, B, prec):
    members = wl.member_grids(5)
    pset = api.PDFSet(members)
    x, q2 = wl.queries(2, 4096)
    pset.domain_errors()
    a = pset.xfxQ2([21, 1], x, q2, prec=prec, domain="error").cpu().numpy()
    np.testing.assert_array_equal(a, pset.xfxQ2([21, 1], x, q2, prec=prec).cpu().numpy())
    assert pset.domain_errors() == 0
    xb = x.copy()
    xb[7] = 3.0
    with pytest.raises(B.PdfxDomainError):
        pset.xfxQ2([21, 1], xb, q2, prec=prec, domain="error")
    assert pset.domain_errors() == len(members)       # once per member
    pdf = api.mkPDF(cfg0_grid())
    x1, x2 = x, x[::-1].copy()
    L, S = pdf.lumi([5, 1], [2, -1], x1, x2, q2_fixed=172.5 ** 2, prec=prec, domain="error")
    L0, S0 = pdf.lumi([5, 1], [2, -1], x1, x2, q2_fixed=172.5 ** 2, prec=prec)
    np.testing.assert_array_equal(S.cpu().numpy(), S0.cpu().numpy())
    with pytest.raises(B.PdfxDomainError):
        pdf.lumi([5, 1], [2, -1], x1, x2, q2_fixed=1e12, prec=prec, domain="error")
    assert pdf.domain_errors() == x.size


def test_error_mode_rejected_by_backward(pdf0, torch, B):
    g = cfg0_grid()
    x = torch.full((8,), 0.1, dtype=torch.float64, device="cuda")
    q = torch.full((8,), 100.0, dtype=torch.float64, device="cuda")
    go = torch.ones((8, 11), dtype=torch.float64, device="cuda")
    gx = torch.empty(8, dtype=torch.float64, device="cuda")
    with pytest.raises(B.PdfxError) as e:
        B.pdfx_eval_xfx_backward(pdf0.handle, None, B.PDFX_F64, g.pids, x.data_ptr(),
                                 q.data_ptr(), 8, go.data_ptr(), None, gx.data_ptr(), None,
                                 B.PDFX_DOMAIN_ERROR, 0)
    assert e.value.code == B.PDFX_EINVAL


# ---------------------------------------------------------------------------
# alpha_s at Q
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f64", "f32s"])
@pytest.mark.parametrize("domain", ["nan", "clamp"])
def test_alphasQ_bitwise_equals_alphasQ2_of_product(pdf0, torch, prec, domain):
    g = cfg0_grid()
    _, q2 = _pts(50_001)
    q = np.sqrt(q2)
    q = np.r_[q, np.sqrt(g.as_q2), [0.1, 1e6, np.nan, 1.0, 1e5]]
    qd = torch.as_tensor(q, device="cuda")
    pdf0.domain_errors()
    a = pdf0.alphasQ(qd, prec=prec, domain=domain).cpu().numpy()
    n_q = pdf0.domain_errors()
    b = pdf0.alphasQ2(qd * qd, prec=prec, domain=domain).cpu().numpy()
    n_q2 = pdf0.domain_errors()
    np.testing.assert_array_equal(a, b)
    assert n_q == n_q2
    ora = oracle.alphas(g.as_q2, g.as_val, q * q, mode=0 if domain == "nan" else 1)
    np.testing.assert_array_equal(np.isnan(a), np.isnan(ora))
    ok = ~np.isnan(ora)
    assert np.max(np.abs(a[ok] - ora[ok]) / ora[ok]) <= (1e-12 if prec == "f64" else 1e-5)


# ---------------------------------------------------------------------------
# torch API argument checks
# ---------------------------------------------------------------------------

def test_api_rejects_bad_tensors_before_launch(pdf0, torch, api):
    g = cfg0_grid()
    x, q2 = _pts(1000)
    xd = torch.as_tensor(x, device="cuda")
    qd = torch.as_tensor(q2, device="cuda")
    sentinel = torch.full((1000, 11), -3.0, dtype=torch.float64, device="cuda")
    pdf0.domain_errors()
    with pytest.raises(ValueError):
        pdf0.xfxQ2(g.pids, xd, qd[:999], out=sentinel)
    with pytest.raises(ValueError):
        pdf0.xfxQ2(g.pids, xd[:999], qd, out=sentinel)
    with pytest.raises(ValueError):
        pdf0.xfxQ2(g.pids, xd, qd, out=torch.empty((999, 11), dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        pdf0.xfxQ2(g.pids, xd, qd, out=torch.empty((1000, 11), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        pdf0.xfxQ2(g.pids, xd, qd, out=torch.empty((11, 1000), dtype=torch.float64,
                                                  device="cuda").t())
    with pytest.raises(ValueError):
        pdf0.xfxQ2(g.pids, xd, qd, out=torch.empty((1000, 11), dtype=torch.float64))
    with pytest.raises(ValueError):
        pdf0.xfxQ2(g.pids, xd, qd, values=torch.zeros((11, 100, 49), dtype=torch.float64,
                                                      device="cuda"))
    with pytest.raises(TypeError):
        pdf0.xfxQ2(g.pids, xd, qd, prec="f32s",
                   values=torch.zeros((11, 100, 50), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        pdf0.xfx_alphasQ2(g.pids, xd, qd, as_out=torch.empty(999, dtype=torch.float64,
                                                             device="cuda"))
    with pytest.raises(ValueError):
        pdf0.alphasQ2(qd, out=torch.empty(1001, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        pdf0.lumi([1], [-1], xd, xd[:500], q2_fixed=100.0)
    with pytest.raises(ValueError):
        pdf0.lumi([1], [-1], xd, xd, q2=qd[:10])
    with pytest.raises(ValueError):
        pdf0.xfxQ2(g.pids, xd, qd, domain="wrap")
    torch.cuda.synchronize()
    assert bool((sentinel == -3.0).all())
    assert pdf0.domain_errors() == 0


# ---------------------------------------------------------------------------
# one flavour group, output rows staged over it, several tiles per workgroup
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec,shape,pids", [
    ("f64", (512, 2), [21] * 12),
    ("f64", (512, 2), [21] + [7] * 10),
    ("f64", (512, 1), [-5] * 24),
    ("f32s", (512, 4), [2] * 12),
    ("f32s", (512, 4), [1] + [8] * 11),
    ("f32s", (512, 2), [-1] * 24),
])
def test_lone_group_with_staged_rows(api, torch, prec, shape, pids):
    g = cfg0_grid()
    pdf = api.mkPDF(g)
    pdf.set_launch(prec, *shape)
    n = 1_500_003
    x, q2 = wl.queries(12, n)
    xd, qd = torch.as_tensor(x, device="cuda"), torch.as_tensor(q2, device="cuda")
    out = pdf.xfxQ2(pids, xd, qd, prec=prec)
    idx = np.r_[np.random.default_rng(4).choice(n, 20_000, replace=False), [0, n - 1]]
    got = out[torch.as_tensor(idx, device="cuda")].double().cpu().numpy()
    ora = oracle.xfx(g, pids, x[idx], q2[idx])
    M = oracle.stencil_absmax(g, pids, x[idx], q2[idx])
    e = capped_rel_err(got, ora, M)
    assert e.max() <= (1e-12 if prec == "f64" else 1e-5), e.max()
    # columns of one parton are equal bit for bit; absent ones are 0
    col = pids.index(pids[0])
    for c, p in enumerate(pids):
        if p == pids[0]:
            np.testing.assert_array_equal(got[:, c], got[:, col])
        else:
            assert np.all(got[:, c] == 0)


@pytest.mark.parametrize("prec", ["f64", "f32s"])
def test_set_lone_group_several_tiles_per_item(api, torch, prec, tmp_path):
    from paper_2012_08221_amd import binding as B
    members = wl.member_grids(3)
    pset = api.PDFSet(members)
    n = 200_000
    x, q2 = wl.queries(13, n)
    pids = [21] * 12
    cache = tmp_path / "tune.jsonl"
    pset.autotune(prec, n_req=12, n_pts=n, cache_path=str(cache))
    key = cache.read_text().strip().splitlines()[-1].split('"key": "')[1].split('"')[0]
    with open(cache, "a") as fh:
        fh.write('{"key": "%s", "block": 512, "ppt": %d, "tpi": 4, "ms": 0}\n'
                 % (key, 2 if prec == "f64" else 4))
    B.pdfx_autotune_set(pset.handle, B.PDFX_F64 if prec == "f64" else B.PDFX_F32S, 12, n,
                        str(cache))
    out = pset.xfxQ2(pids, x, q2, prec=prec).double().cpu().numpy()
    for k, m in enumerate(members):
        ora = oracle.xfx(m, [21], x, q2)[:, 0]
        M = oracle.stencil_absmax(m, [21], x, q2)[:, 0]
        for c in range(12):
            e = capped_rel_err(out[k][:, c], ora, M)
            assert e.max() <= (1e-12 if prec == "f64" else 1e-5), (k, c, e.max())
