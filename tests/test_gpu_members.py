"""Many members in one persistent launch (pdfx_eval_set_xfx) against the oracle:
101 replica-style members with uneven grids; every member on 1e4 points, and a
few members on 1e6 shared points (sampled)."""
import numpy as np
import pytest

import oracle
from helpers import capped_rel_err, f32_tolerance
from paper_2012_08221_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def members():
    return wl.member_grids(101)


@pytest.fixture(scope="module")
def pset(torch, members):
    from paper_2012_08221_amd import api
    return api.PDFSet(members)


def check_member(m, got, x, q2, pids, prec):
    ora = oracle.xfx(m, pids, x, q2)
    M = oracle.stencil_absmax(m, pids, x, q2)
    np.testing.assert_array_equal(np.isnan(got), np.isnan(ora))
    ok = ~np.isnan(ora)
    e = capped_rel_err(got[ok], ora[ok], M[ok])
    tol = 1e-12 if prec == "f64" else f32_tolerance(m)
    return e.max() if e.size else 0.0, tol


@pytest.mark.parametrize("prec", ["f64", "f32s"])
def test_all_members_small(pset, members, prec):
    x, q2 = wl.queries(2, 10_000)
    pids = members[0].pids
    out = pset.xfxQ2(pids, x, q2, prec=prec).double().cpu().numpy()
    assert out.shape == (101, 10_000, 11)
    worst = 0.0
    for k, m in enumerate(members):
        e, tol = check_member(m, out[k], x, q2, pids, prec)
        worst = max(worst, e)
        assert e <= tol, (k, e, tol)
    print("101 members x 1e4 points, %s: worst %.2e" % (prec, worst))


@pytest.mark.parametrize("prec", ["f64", "f32s"])
def test_few_members_full_points_sampled(pset, members, torch, prec):
    n = 1_000_000
    x, q2 = wl.queries(2, n)
    xd, qd = torch.as_tensor(x, device="cuda"), torch.as_tensor(q2, device="cuda")
    out = pset.xfxQ2(members[0].pids, xd, qd, prec=prec)
    idx = np.random.default_rng(1).choice(n, 20_000, replace=False)
    sel = out[:, torch.as_tensor(idx, device="cuda")].double().cpu().numpy()
    for k in (0, 1, 50, 99, 100):
        e, tol = check_member(members[k], sel[k], x[idx], q2[idx], members[0].pids, prec)
        assert e <= tol, (k, e)
    assert bool(torch.isfinite(out).all())


def test_shapes_and_work_split_agree(pset, members, tmp_path):
    """Every compiled set shape and several work splits give the same result,
    whichever kernel evaluates a member: each (shape, tiles per item) is forced
    through a tuning-cache entry."""
    from paper_2012_08221_amd import binding as B
    x, q2 = wl.queries(9, 30_001)
    ref = None
    cache = tmp_path / "tune.jsonl"
    pset.autotune("f64", n_req=3, n_pts=30_001, cache_path=str(cache))
    key_line = cache.read_text().strip().splitlines()[-1]
    key = key_line.split('"key": "')[1].split('"')[0]
    # (512, 1), (512, 2), (256, 2) take the double-buffered class kernels for
    # the members that fit them; the others the single-slab kernel
    for blk, ppt in ((256, 4), (512, 2), (1024, 1), (512, 1), (256, 2)):
        for tpi in (1, 3):
            with open(cache, "a") as fh:
                fh.write('{"key": "%s", "block": %d, "ppt": %d, "tpi": %d, "ms": 0}\n'
                         % (key, blk, ppt, tpi))
            B.pdfx_autotune_set(pset.handle, B.PDFX_F64, 3, 30_001, str(cache))
            out = pset.xfxQ2([21, 2, -3], x, q2).cpu().numpy()
            if ref is None:
                ref = out
            np.testing.assert_array_equal(out, ref)
    for k in (0, 7, 100):
        e, tol = check_member(members[k], ref[k], x, q2, [21, 2, -3], "f64")
        assert e <= tol


def test_f32_class_shape_and_fallback_agree(pset, members, torch, tmp_path):
    """FP32 sets: the class kernels at (512, 2) and at the FP32-only (512, 4),
    with two work splits, and an unaligned output (every member through the
    single-slab kernel, which runs (512, 4) as (512, 2) with twice the tiles
    per work item) all give the same bits."""
    from paper_2012_08221_amd import api
    from paper_2012_08221_amd import binding as B
    n = 30_000                                   # 16-byte aligned member blocks
    x, q2 = wl.queries(11, n)
    pids = [21, 2, -3]
    cache = tmp_path / "tune32.jsonl"
    pset.autotune("f32s", n_req=3, n_pts=n, cache_path=str(cache))
    key = cache.read_text().strip().splitlines()[-1].split('"key": "')[1].split('"')[0]
    ref = None
    try:
        for blk, ppt in ((512, 2), (512, 4)):
            for tpi in (1, 3):
                with open(cache, "a") as fh:
                    fh.write('{"key": "%s", "block": %d, "ppt": %d, "tpi": %d, "ms": 0}\n'
                             % (key, blk, ppt, tpi))
                B.pdfx_autotune_set(pset.handle, B.PDFX_F32S, 3, n, str(cache))
                out = pset.xfxQ2(pids, x, q2, prec="f32s").cpu().numpy()
                if ref is None:
                    ref = out
                np.testing.assert_array_equal(out, ref)
        buf = torch.empty(101 * n * 3 + 1, dtype=torch.float32, device="cuda")
        un = buf[1:].view(101, n, 3)
        pset.xfxQ2(pids, x, q2, prec="f32s", out=un)
        np.testing.assert_array_equal(un.cpu().numpy(), ref)
    finally:
        pset.autotune("f32s", n_req=3, n_pts=n)
    for k in (0, 50, 100):
        e, tol = check_member(members[k], ref[k], x, q2, pids, "f32s")
        assert e <= tol, (k, e)


def test_one_member_set_matches_single_grid(torch, members):
    from paper_2012_08221_amd import api
    m = members[3]
    s1 = api.PDFSet([m])
    g1 = api.mkPDF(m)
    x, q2 = wl.queries(4, 50_000)
    for prec in ("f64", "f32s"):
        a = s1.xfxQ2(m.pids, x, q2, prec=prec)[0].cpu().numpy()
        b = g1.xfxQ2(m.pids, x, q2, prec=prec).cpu().numpy()
        np.testing.assert_array_equal(a, b)


def test_set_domain_and_pid_requests(pset, members):
    x = np.array([0.1, 1e-12, 0.3])
    q2 = np.array([50.0, 50.0, 1e11])
    out = pset.xfxQ2([21, 7, 1], x, q2, domain="nan").cpu().numpy()
    assert np.all(np.isfinite(out[:, 0, [0, 2]])) and np.all(out[:, :, 1] == 0)
    assert np.all(np.isnan(out[:, 1:, 0]))
    outc = pset.xfxQ2([21], x, q2, domain="clamp").cpu().numpy()
    assert np.all(np.isfinite(outc))
    for k in (0, 60):
        ora = oracle.xfx(members[k], [21], x, q2, mode=1)
        np.testing.assert_allclose(outc[k], ora, rtol=1e-12)


def test_large_members_split_slab(torch):
    """Members whose FP64 group slab needs both LDS slabs (rows split between
    them; odd n_q moves the split one row down), one at the largest grid that
    split fits, and a small one, on random points and on points at every x
    knot around the split row.  A member beyond the split (230 x 90) is too
    large for any FP64 kernel and raises; in FP32 it takes the single-slab
    kernel beside the class kernels."""
    from paper_2012_08221_amd import api
    from paper_2012_08221_amd.binding import PdfxError
    p = wl.draw_params(np.random.default_rng(3))
    geo = [(200, 79), (200, 81), (240, 80), (60, 30), (230, 90)]
    mems = [wl.make_grid(p * (1 + 0.01 * k), nx, wl.MEMBER_EDGES[3], nq, with_alphas=False)
            for k, (nx, nq) in enumerate(geo)]
    x, q2 = wl.queries(5, 8_000)
    for m in mems[:4]:
        r = 78016 // (m.n_q * 8)
        kx = m.x[max(r - 6, 0):r + 6]
        mid = np.sqrt(kx[1:] * kx[:-1])
        qs = np.geomspace(m.q2[0], m.q2[-1], 7)
        xe, qe = np.meshgrid(np.concatenate([kx, mid]), qs)
        x = np.concatenate([x, xe.ravel()])
        q2 = np.concatenate([q2, qe.ravel()])
    n = x.size - x.size % 2   # 16-byte aligned FP64 output blocks
    x, q2 = x[:n], q2[:n]
    pids = mems[0].pids
    fit = api.PDFSet(mems[:4])
    for prec in ("f64", "f32s"):
        out = fit.xfxQ2(pids, x, q2, prec=prec).double().cpu().numpy()
        for k, m in enumerate(mems[:4]):
            e, tol = check_member(m, out[k], x, q2, pids, prec)
            assert e <= tol, (prec, k, e, tol)
    big = api.PDFSet(mems)
    with pytest.raises(PdfxError, match="does not fit LDS"):
        big.xfxQ2(pids, x, q2, prec="f64")
    out = big.xfxQ2(pids, x, q2, prec="f32s").double().cpu().numpy()
    for k, m in enumerate(mems):
        e, tol = check_member(m, out[k], x, q2, pids, "f32s")
        assert e <= tol, ("f32s", k, e, tol)


@pytest.mark.parametrize("n", [0, 1, 63, 1025, 4097])
def test_set_ragged_sizes(pset, members, n):
    """Empty and ragged point counts through the one-launch set call (every
    class of the bench set runs), each member against the oracle."""
    x, q2 = wl.queries(8, max(n, 1))
    x, q2 = x[:n], q2[:n]
    pids = members[0].pids
    for prec in ("f64", "f32s"):
        out = pset.xfxQ2(pids, x, q2, prec=prec).double().cpu().numpy()
        assert out.shape == (101, n, 11)
        if n == 0:
            continue
        for k in range(0, 101, 10):
            e, tol = check_member(members[k], out[k], x, q2, pids, prec)
            assert e <= tol, (n, k, prec, e, tol)


def test_set_request_the_grids_lack(torch):
    """pids no member holds: zero columns, and the outside points still counted
    once per member in every tile (the kernel has no flavour group to stage,
    so each tile must still read its own points)."""
    from paper_2012_08221_amd import api
    members = wl.member_grids(5)
    pset = api.PDFSet(members)
    n = 300_001
    x, q2 = wl.queries(9, n)
    bad = np.arange(1000, n, 20_011)                      # outside points over many tiles
    x[bad] = 3.0
    pset.domain_errors()
    for prec in ("f64", "f32s"):
        out = pset.xfxQ2([7, 8], x, q2, prec=prec).cpu().numpy()
        assert not out.any()
        assert pset.domain_errors() == bad.size * len(members), prec
