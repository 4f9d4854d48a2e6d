"""Reader/writer of the standard PDF grid folders (host side, no GPU).

The hand-written set tests/golden/lhagrid/tiny pins the reading of the format:
value lines run over x (outer) and Q (inner) with one column per parton, and
blocks are concatenated along Q with their shared boundary knot kept twice.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2012_08221_amd import lhapdf
from paper_2012_08221_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lhagrid")


def test_tiny_fixture_layout():
    m = lhapdf.load_member("tiny/0", GOLDEN)
    assert list(m.pids) == [21, 2, -1]
    np.testing.assert_array_equal(m.x, [0.001, 0.01, 0.1])
    np.testing.assert_array_equal(m.q2, [1.0, 4.0, 4.0, 16.0, 64.0])
    np.testing.assert_array_equal(m.q_off, [0, 2, 5])
    p, i, j = np.meshgrid(np.arange(3), np.arange(3), np.arange(5), indexing="ij")
    np.testing.assert_array_equal(m.xf, 100 * p + 10 * i + j)
    np.testing.assert_array_equal(m.as_q2, [1.0, 4.0, 4.0, 16.0, 64.0])
    np.testing.assert_array_equal(m.as_val, [0.5, 0.4, 0.41, 0.3, 0.2])


def test_tiny_member_header_overrides_info():
    m = lhapdf.load_member("tiny/1", GOLDEN)
    p, i, j = np.meshgrid(np.arange(3), np.arange(3), np.arange(5), indexing="ij")
    np.testing.assert_array_equal(m.xf, 1000 + 100 * p + 10 * i + j)
    np.testing.assert_array_equal(m.as_val, [0.6, 0.5, 0.51, 0.4, 0.3])
    assert m.meta["PdfType"] == "replica" and m.meta["SetDesc"] == "format fixture"
    assert len(lhapdf.load_set("tiny", GOLDEN)) == 2


def test_name_and_search_path(monkeypatch, tmp_path):
    assert lhapdf.parse_name("NNPDF/7") == ("NNPDF", 7)
    assert lhapdf.parse_name("NNPDF") == ("NNPDF", 0)
    monkeypatch.setenv("LHAPDF_DATA_PATH", str(tmp_path) + ":" + GOLDEN)
    assert lhapdf.find_set("tiny") == os.path.join(GOLDEN, "tiny")
    monkeypatch.setenv("LHAPDF_DATA_PATH", str(tmp_path))
    with pytest.raises(FileNotFoundError):
        lhapdf.find_set("tiny")


def test_round_trip_config_grid_and_members(tmp_path):
    g = wl.config0_grid()
    mem = wl.member_grids(4)
    lhapdf.write_set(str(tmp_path), "cfg", [g])
    lhapdf.write_set(str(tmp_path), "mem", mem)
    back = lhapdf.load_member("cfg/0", str(tmp_path))
    np.testing.assert_array_equal(back.xf, g.xf)
    np.testing.assert_array_equal(back.x, g.x)
    np.testing.assert_array_equal(back.q_off, g.q_off)
    np.testing.assert_array_equal(back.pids, g.pids)
    # Q is stored, Q^2 = Q * Q is read back: within one rounding
    np.testing.assert_allclose(back.q2, g.q2, rtol=4.5e-16, atol=0)
    np.testing.assert_allclose(back.as_q2, g.as_q2, rtol=4.5e-16, atol=0)
    np.testing.assert_array_equal(back.as_val, g.as_val)
    allm = lhapdf.load_set("mem", str(tmp_path))
    assert len(allm) == 4
    for a, b in zip(allm, mem):
        np.testing.assert_array_equal(a.xf, b.xf)
        np.testing.assert_array_equal(a.q_off, b.q_off)
    # the oracle gives the same x f on the read-back grid
    x, q2 = wl.queries(3, 2000)
    np.testing.assert_allclose(oracle.xfx(back, g.pids, x, q2), oracle.xfx(g, g.pids, x, q2),
                               rtol=1e-13, atol=0)


def _write(tmp_path, body):
    d = tmp_path / "bad"
    d.mkdir(exist_ok=True)
    (d / "bad.info").write_text("Format: lhagrid1\nNumMembers: 1\n")
    (d / "bad_0000.dat").write_text("PdfType: central\n---\n" + body)
    return str(tmp_path)


@pytest.mark.parametrize("body, msg", [
    ("0.1 0.2\n1 2\n21\n1\n2\n3\n---\n", "value lines"),
    ("0.1 0.2\n1 2\n21 1\n1\n2\n3\n4\n---\n", "entries"),
    ("0.1 0.2\n1 2\n21\n1\n2\n3\n4\n---\n0.1 0.3\n2 3\n21\n1\n2\n3\n4\n---\n", "other x knots"),
    ("0.1 0.2\n1 2\n21\n1\n2\n3\n4\n---\n0.1 0.2\n2.5 3\n21\n1\n2\n3\n4\n---\n", "boundary Q"),
    ("0.1 0.2\n1 2\n21\n1\n2\n3\n4\n---\n0.1 0.2\n2 3\n1\n1\n2\n3\n4\n---\n", "parton list"),
    ("0.1 zz\n1 2\n21\n1\n2\n3\n4\n---\n", "bad x knot"),
])
def test_malformed_members_are_rejected(tmp_path, body, msg):
    d = _write(tmp_path, body)
    with pytest.raises(lhapdf.FormatError, match=msg):
        lhapdf.load_member("bad/0", d)
