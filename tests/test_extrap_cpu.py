"""Pins of the oracle's out-of-grid continuation (oracle.xfx_extrapolated)
against closed forms: a power law in x and Q^2 continues exactly; opposite
signs at the edge fall back to a straight line in the log coordinate; the
continuation meets the interpolation at the edge; inside points are xfx."""
import numpy as np
import pytest

import oracle
from paper_2012_08221_amd import workloads as wl


@pytest.fixture(scope="module")
def grid():
    return wl.config0_grid()


def power_grid(g, A=1.7, a=-0.35, b=0.12):
    c = 1.0 + np.arange(11.0)
    xf = A * g.x[None, :, None] ** a * g.q2[None, None, :] ** b * c[:, None, None]
    return wl.GridSpec(pids=g.pids, x=g.x, q2=g.q2, q_off=g.q_off, xf=xf), a, b


def test_power_law_continues_exactly(grid):
    pg, a, b = power_grid(grid)
    x = np.array([1e-12, 1e-10, 1e-3, 1e-11, 1e-3, 1e-13, 0.5, 0.7])
    q2 = np.array([100.0, 0.5, 1e12, 1e13, 0.1, 0.2, 1e11, 50.0])
    got = oracle.xfx_extrapolated(pg, [21, 1, -3], x, q2)
    xc = np.clip(x, grid.x[0], grid.x[-1])
    qc = np.clip(q2, grid.q2[0], grid.q2[-1])
    # the continuation factor is exact: (x/x_e)^a (q2/q2_e)^b times the edge value
    want = oracle.xfx(pg, [21, 1, -3], xc, qc) * ((x / xc) ** a * (q2 / qc) ** b)[:, None]
    np.testing.assert_allclose(got, want, rtol=2e-13)
    # outside in both: the edge value is a knot value, so the result is the power law
    both = (x < grid.x[0]) & ((q2 < grid.q2[0]) | (q2 > grid.q2[-1]))
    exact = 1.7 * x[both, None] ** a * q2[both, None] ** b * np.array([6.0, 7.0, 3.0])
    np.testing.assert_allclose(got[both], exact, rtol=2e-13)


def test_opposite_signs_give_a_line_in_log_x(grid):
    xf = grid.xf.copy()
    xf[5, 0, :] = 1.0     # gluon: +1 on the first x knot, -1 on the second
    xf[5, 1, :] = -1.0
    g = wl.GridSpec(pids=grid.pids, x=grid.x, q2=grid.q2, q_off=grid.q_off, xf=xf)
    x = np.array([1e-10, 1e-12])
    q2 = np.array([grid.q2[20], grid.q2[30]])   # on Q^2 knots: edge values are exact
    got = oracle.xfx_extrapolated(g, [21], x, q2)[:, 0]
    u = np.log(x / grid.x[0]) / np.log(grid.x[1] / grid.x[0])
    np.testing.assert_allclose(got, 1.0 - 2.0 * u, rtol=1e-13)


def test_continuation_meets_the_grid_and_leaves_inside_alone(grid):
    pids = list(grid.pids)
    x, q2 = wl.queries(9, 3000)
    np.testing.assert_array_equal(oracle.xfx_extrapolated(grid, pids, x, q2),
                                  oracle.xfx(grid, pids, x, q2))
    for xv, qv in ((grid.x[0] * (1 - 1e-13), 100.0), (0.01, grid.q2[0] * (1 - 1e-13)),
                   (0.01, grid.q2[-1] * (1 + 1e-13)), (grid.x[-1] * (1 + 1e-13), 1e4)):
        got = oracle.xfx_extrapolated(grid, pids, [xv], [qv])[0]
        edge = oracle.xfx(grid, pids, [np.clip(xv, grid.x[0], grid.x[-1])],
                          [np.clip(qv, grid.q2[0], grid.q2[-1])])[0]
        np.testing.assert_allclose(got, edge, rtol=1e-10, atol=1e-12)   # x f(1) = 0
    assert np.all(np.isnan(oracle.xfx_extrapolated(grid, pids, [np.nan, 0.1], [10.0, np.nan])))
