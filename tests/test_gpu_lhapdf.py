"""Grids read from the standard PDF grid folders, evaluated by the library
against the oracle on the same read-back grids: a set written from the
synthetic config grid (with alpha_s), five uneven members as one set, and the
hand-written 3 x 5 fixture (subgrids of 2 and 3 Q knots)."""
import os

import numpy as np
import pytest

import oracle
from helpers import capped_rel_err
from paper_2012_08221_amd import lhapdf
from paper_2012_08221_amd import workloads as wl

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lhagrid")


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_08221_amd import api as a
    return a


def rel(got, ora, m, pids, x, q2):
    M = oracle.stencil_absmax(m, pids, x, q2)
    return capped_rel_err(got, ora, M).max()


def test_mkpdf_by_name_matches_oracle(api, tmp_path):
    lhapdf.write_set(str(tmp_path), "cfg", [wl.config0_grid()])
    m = lhapdf.load_member("cfg/0", str(tmp_path))
    pdf = api.mkPDF("cfg/0", str(tmp_path))
    x, q2 = wl.queries(6, 20_000)
    for prec, tol in (("f64", 1e-12), ("f32s", 1e-5)):
        got = pdf.xfxQ2(m.pids, x, q2, prec=prec).double().cpu().numpy()
        assert rel(got, oracle.xfx(m, m.pids, x, q2), m, m.pids, x, q2) <= tol
    a = pdf.alphasQ2(q2).cpu().numpy()
    np.testing.assert_allclose(a, oracle.alphas(m.as_q2, m.as_val, q2), rtol=1e-12)


def test_pdfset_by_name_matches_oracle(api, tmp_path):
    mem = wl.member_grids(5)
    lhapdf.write_set(str(tmp_path), "mem", mem)
    back = lhapdf.load_set("mem", str(tmp_path))
    s = api.PDFSet("mem", str(tmp_path))
    x, q2 = wl.queries(7, 10_000)
    out = s.xfxQ2(back[0].pids, x, q2).cpu().numpy()
    for k, m in enumerate(back):
        assert rel(out[k], oracle.xfx(m, m.pids, x, q2), m, m.pids, x, q2) <= 1e-12, k


def test_hand_written_fixture(api):
    m = lhapdf.load_member("tiny/0", GOLDEN)
    pdf = api.mkPDF("tiny/0", GOLDEN)
    rng = np.random.default_rng(11)
    x = np.exp(rng.uniform(np.log(1e-3), np.log(0.1), 4000))
    q2 = np.exp(rng.uniform(0.0, np.log(64.0), 4000))
    x[:5] = m.x[[0, 1, 2, 1, 0]]      # knots and the threshold itself
    q2[:5] = [1.0, 4.0, 64.0, 16.0, 4.0]
    pids = [21, 2, -1, 3]             # 3 is absent: zeros
    got = pdf.xfxQ2(pids, x, q2).cpu().numpy()
    ora = oracle.xfx(m, pids, x, q2)
    assert np.all(got[:, 3] == 0)
    assert rel(got, ora, m, pids, x, q2) <= 1e-12
