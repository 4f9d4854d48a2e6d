"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects invalid descriptors on the host (before any HIP
call).  Also checks the seeded generators are deterministic and shaped as the
workloads state."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2012_08221_amd import binding as B
from paper_2012_08221_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdfx.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdfx_[A-Za-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libpdfx.so is not built; run __graft_entry__.build()")
    return B.lib()


def test_exports_every_declared_symbol(L):
    declared = header_functions()
    assert len(declared) >= 15
    assert sorted(B.EXPORTS) == declared
    for name in declared:
        assert hasattr(L, name), name


def test_version_and_error_string(L):
    assert "gfx950" in B.pdfx_version()
    assert isinstance(B.last_error(), str)


def _desc(**over):
    g = wl.config0_grid()
    d = dict(pids=g.pids, x=g.x, q2=g.q2, q_off=g.q_off, xf=g.xf, as_q2=g.as_q2, as_val=g.as_val)
    d.update(over)
    return B.HostDesc(**d)


@pytest.mark.parametrize("case,over", [
    ("dup pid", lambda g: dict(pids=np.where(g.pids == 21, 0, g.pids) * 0 + np.r_[g.pids[:5], [21, 0], g.pids[7:]])),
    ("x not increasing", lambda g: dict(x=np.r_[g.x[:10], g.x[9:10], g.x[11:]])),
    ("x nonpositive", lambda g: dict(x=np.r_[[0.0], g.x[1:]])),
    ("x nan", lambda g: dict(x=np.r_[g.x[:3], [np.nan], g.x[4:]])),
    ("one x knot", lambda g: dict(x=g.x[:1], xf=g.xf[:, :1, :])),
    ("boundary not repeated", lambda g: dict(q2=np.r_[g.q2[:3], [g.q2[3] * 1.0001], g.q2[4:]])),
    ("q_off start", lambda g: dict(q_off=g.q_off + 1)),
    ("subgrid of one knot", lambda g: dict(q_off=np.array([0, 1, 10, 50], np.int32))),
    ("nonfinite value", lambda g: dict(xf=np.where(np.arange(g.xf.size).reshape(g.xf.shape) == 7, np.inf, g.xf))),
    ("alpha_s nonfinite", lambda g: dict(as_val=np.r_[[np.nan], g.as_val[1:]])),
    ("alpha_s triple knot", lambda g: dict(as_q2=np.r_[g.as_q2[:4], g.as_q2[3:4], g.as_q2[4:]],
                                           as_val=np.r_[g.as_val[:4], g.as_val[3:4], g.as_val[4:]])),
])
def test_invalid_descriptors_rejected_on_host(L, case, over):
    g = wl.config0_grid()
    d = _desc(**over(g))
    h = ctypes.c_void_p()
    rc = L.pdfx_load_grid(ctypes.byref(d.desc), ctypes.byref(h))
    assert rc == B.PDFX_EINVAL, case
    assert h.value is None
    assert B.last_error() != ""


def test_null_arguments_rejected(L):
    h = ctypes.c_void_p()
    assert L.pdfx_load_grid(None, ctypes.byref(h)) == B.PDFX_EINVAL
    assert L.pdfx_eval_xfx(None, None, 0, None, 1, None, None, 10, None, 0, None) == B.PDFX_EINVAL
    assert L.pdfx_eval_alphas(None, None, 10, None, 0, 0, None) == B.PDFX_EINVAL
    assert L.pdfx_domain_errors(None, None) == B.PDFX_EINVAL
    assert L.pdfx_grid_shape(None, None, None, None, None, None) == B.PDFX_EINVAL
    assert L.pdfx_eval_xfx_alphas(None, None, 0, None, 1, None, None, 10, None, None, 0,
                                  None) == B.PDFX_EINVAL
    assert L.pdfx_bench_lds(6, 8, 8, 1024, None) == B.PDFX_EINVAL
    assert L.pdfx_bench_lds(-1, 8, 8, 1024, None) == B.PDFX_EINVAL
    assert L.pdfx_bench_lds(0, 0, 8, 1024, None) == B.PDFX_EINVAL
    assert L.pdfx_bench_lds(1, 8, 8, None, None) == B.PDFX_EINVAL


def test_generators_deterministic_and_shaped():
    a, b = wl.config0_grid(), wl.config0_grid()
    for f in ("x", "q2", "q_off", "xf", "as_q2", "as_val"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    assert a.xf.shape == (11, 100, 50)
    assert list(np.diff(a.q_off)) == [4, 6, 40]
    assert list(np.diff(wl.config0_grid("alternate").q_off)) == [6, 44]
    assert wl.allocate_knots(20, wl.MEMBER_EDGES[4]) == [4, 4, 6, 6]
    # boundary knots bitwise repeated; top knot is exactly (1e5)^2
    for s in range(1, a.n_sub):
        assert a.q2[a.q_off[s] - 1] == a.q2[a.q_off[s]]
    assert a.q2[-1] == 1e10 and a.x[-1] == 1.0 and a.x[0] == 1e-9
    x, q2 = wl.queries(0, 1000)
    assert x.min() >= 1e-6 and x.max() <= 0.99 and q2.min() >= 4.0 and q2.max() <= 1e8
    np.testing.assert_array_equal(x, wl.queries(0, 1000)[0])
    assert not np.array_equal(x, wl.queries(1, 1000)[0])
    assert abs(wl.alphas_values(np.array([1.0]))[0] - 0.363) < 2e-3
    assert abs(wl.alphas_values(np.array([91.1876 ** 2]))[0] - 0.118) < 1e-12


def test_member_grids_uneven():
    ms = wl.member_grids(6)
    assert len({m.n_x for m in ms}) > 1
    for m in ms:
        assert 50 <= m.n_x <= 200 and 20 <= m.n_q <= 80 and 2 <= m.n_sub <= 4
        assert np.all(np.diff(m.q_off) >= 4)


def test_host_domain_check_returns_edomain(L):
    """pdfx_check_points applies the eval calls' domain rule to host arrays:
    PDFX_EDOMAIN with the count of outside points (NaN included), PDFX_OK
    when every point is inside, PDFX_EINVAL for a bad descriptor."""
    g = wl.config0_grid()
    d = _desc(xf=None)
    x, q2 = wl.queries(0, 1000)
    n_out = ctypes.c_int64(-1)
    xp, qp = x.ctypes.data, q2.ctypes.data
    assert L.pdfx_check_points(ctypes.byref(d.desc), xp, qp, 1000, ctypes.byref(n_out)) == B.PDFX_OK
    assert n_out.value == 0
    # the grid's own edges are inside (closed interval)
    ex = np.array([g.x[0], g.x[-1], g.x[0], g.x[-1]])
    eq = np.array([g.q2[0], g.q2[-1], g.q2[-1], g.q2[0]])
    assert B.pdfx_check_points(d, ex, eq) == 0
    bad_x = x.copy()
    bad_q = q2.copy()
    bad_x[[3, 70]] = [np.nextafter(g.x[0], 0.0), 1.5]
    bad_q[[5, 900]] = [np.nextafter(g.q2[0], 0.0), np.nan]
    bad_x[11] = np.nan
    rc = L.pdfx_check_points(ctypes.byref(d.desc), bad_x.ctypes.data, bad_q.ctypes.data, 1000,
                             ctypes.byref(n_out))
    assert rc == B.PDFX_EDOMAIN and n_out.value == 5
    assert "outside" in B.last_error()
    assert B.pdfx_check_points(d, bad_x, bad_q) == 5
    assert L.pdfx_check_points(ctypes.byref(d.desc), None, None, 0, None) == B.PDFX_OK
    assert L.pdfx_check_points(ctypes.byref(d.desc), None, None, 5, None) == B.PDFX_EINVAL
    bad_desc = _desc(x=np.r_[g.x[:10], g.x[9:10], g.x[11:]])
    assert L.pdfx_check_points(ctypes.byref(bad_desc.desc), xp, qp, 1000, None) == B.PDFX_EINVAL
    assert L.pdfx_check_points(None, xp, qp, 1000, None) == B.PDFX_EINVAL


def test_new_entry_points_reject_null_handles(L):
    assert L.pdfx_eval_alphasQ(None, None, 10, None, 0, 0, None) == B.PDFX_EINVAL
    assert L.pdfx_set_domain_errors(None, None) == B.PDFX_EINVAL


def test_api_argument_checks_on_host_tensors():
    """The torch API's checks (length, shape, dtype, device, contiguity) run
    before any launch; here on CPU tensors against a CPU 'device'."""
    import torch
    from paper_2012_08221_amd import api
    cpu = torch.device("cpu")
    a = torch.zeros(5, dtype=torch.float64)
    assert api._same_length(("x", a), ("q2", torch.zeros(5))) == 5
    with pytest.raises(ValueError):
        api._same_length(("x", a), ("q2", torch.zeros(4)))
    api._check_tensor(torch.zeros(5, 3), (5, 3), torch.float32, cpu, "out")
    with pytest.raises(ValueError):
        api._check_tensor(torch.zeros(5, 2), (5, 3), torch.float32, cpu, "out")
    with pytest.raises(TypeError):
        api._check_tensor(torch.zeros(5, 3, dtype=torch.float64), (5, 3), torch.float32, cpu,
                          "out")
    with pytest.raises(ValueError):
        api._check_tensor(torch.zeros(3, 5).t(), (5, 3), torch.float32, cpu, "out")
    with pytest.raises(TypeError):
        api._check_tensor(np.zeros((5, 3), np.float32), (5, 3), torch.float32, cpu, "out")
    with pytest.raises(ValueError):
        api._domain("wrap")
    assert api._domain("error") == B.PDFX_DOMAIN_ERROR
