"""Pins of the luminosity oracle (oracle.lumi) against facts it does not
compute itself: the Drell-Yan integrand oracle (separate C code), a grid of
constant x f (closed form), absent partons and the clamp rule."""
import numpy as np
import pytest

import oracle
from paper_2012_08221_amd import workloads as wl


@pytest.fixture(scope="module")
def grid():
    return wl.config0_grid()


def test_quark_antiquark_pairs_reproduce_the_integrand_oracle(grid):
    """I = (ln 1/xmin)^2 alpha_s(Q^2) sum_q xf_q(x1) xf_qbar(x2) (the C oracle)
    equals (ln 1/xmin)^2 alpha_s x1 x2 S with S = sum_q f_q(x1) f_qbar(x2)."""
    u1, u2 = wl.dy_uniforms(0, 20_000)
    xmin, s = wl.DY_XMIN, wl.SQRT_S_DY ** 2
    lnr = np.log(1.0 / xmin)
    x1 = np.exp(np.log(xmin) + u1 * lnr)
    x2 = np.exp(np.log(xmin) + u2 * lnr)
    q2 = np.clip(x1 * x2 * s, grid.q2.min(), grid.q2.max())
    L, S = oracle.lumi(grid, [1, 2, 3, 4, 5], [-1, -2, -3, -4, -5], x1, x2, q2)
    np.testing.assert_allclose(S, L.sum(axis=1), rtol=4e-15)   # 5 terms, any order
    a = oracle.alphas(grid.as_q2, grid.as_val, q2)
    I = oracle.dy(grid, u1, u2, xmin, s)
    np.testing.assert_allclose(lnr ** 2 * a * S * x1 * x2, I, rtol=1e-12)


def test_constant_xf_grid_closed_form(grid):
    """xf_a = c_a on every knot is reproduced exactly, so L = c_a c_b / (x1 x2):
    catches a missing 1/x, swapped sides or a wrong parton."""
    g = wl.GridSpec(pids=grid.pids, x=grid.x, q2=grid.q2, q_off=grid.q_off,
                    xf=np.broadcast_to((1.0 + np.arange(11.0))[:, None, None],
                                       grid.xf.shape).copy())
    c = {int(p): 1.0 + i for i, p in enumerate(grid.pids)}
    x1, q2 = wl.queries(5, 5000)
    x2 = x1[::-1].copy()
    pa, pb = [5, 21, -2, 1], [2, -3, 21, 1]
    coef = [0.5, -2.0, 3.0, 1.0]
    L, S = oracle.lumi(g, pa, pb, x1, x2, q2, coef=coef)
    want = np.stack([c[a] * c[b] / (x1 * x2) for a, b in zip(pa, pb)], axis=1)
    np.testing.assert_allclose(L, want, rtol=1e-14)
    np.testing.assert_allclose(S, want @ np.array(coef), rtol=1e-13)
    # gluon id 0 and 21 are the same parton
    L0, _ = oracle.lumi(g, [0], [0], x1, x2, q2)
    np.testing.assert_allclose(L0[:, 0], c[21] ** 2 / (x1 * x2), rtol=1e-14)


def test_absent_partons_and_domain(grid):
    x1 = np.array([1e-3, 1e-3, 2.0, 1e-3, np.nan])
    x2 = np.array([0.2, 0.2, 0.2, 0.2, 0.2])
    q2 = np.array([100.0, 1e12, 100.0, 100.0, 100.0])
    L, S = oracle.lumi(grid, [1, 7, 21], [-1, 1, 6], x1, x2, q2)
    assert np.all(L[:, 1] == 0) and np.all(L[:, 2] == 0)   # pid 7 and 6 absent
    assert np.isfinite(L[0, 0]) and np.isfinite(L[3, 0])
    assert np.all(np.isnan(L[[1, 2, 4], 0])) and np.all(np.isnan(S[[1, 2, 4]]))
    Lc, Sc = oracle.lumi(grid, [1], [-1], x1, x2, q2, mode=1)
    # clamped: the value at the clamped point, with f = xf / x at the clamped x
    xe, qe = np.clip(x1[:4], grid.x[0], grid.x[-1]), np.clip(q2[:4], grid.q2[0], grid.q2[-1])
    want = (oracle.xfx(grid, [1], xe, qe)[:, 0] / xe) * (oracle.xfx(grid, [-1], x2[:4], qe)[:, 0]
                                                        / x2[:4])
    np.testing.assert_allclose(Lc[:4, 0], want, rtol=1e-15)
    assert np.isnan(Lc[4, 0])
