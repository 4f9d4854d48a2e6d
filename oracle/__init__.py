"""CPU FP64 oracle (ctypes wrapper around ``pdf_oracle.c``).

TEST INFRASTRUCTURE.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU library; it is compiled from its own C source with gcc.

Functions follow the method of PDFFlow (arXiv:2012.08221): batched PDF
evaluation over independent points (Sec. 2.1), alpha_s by the same 1-D
interpolation (Sec. 2.1), and the luminosity part of the Monte Carlo integrand
of Eq. (1) (Sec. 3.1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pdf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math: IEEE FP64)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                        "-ffp-contract=off", "-o", tmp, _SRC, "-lm", "-lpthread"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        # ORACLE_LIB_OVERRIDE: a library built from a deliberately altered copy
        # of the source, used only by the test that checks that the pins catch
        # planted mistakes
        path = os.environ.get("ORACLE_LIB_OVERRIDE")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        _lib = ctypes.CDLL(path)
        d, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_long
        _lib.ora_xfx.argtypes = [i32, d, i32, d, i32, d, d, d, i32, d, i64, d, d, d, i32, i32]
        _lib.ora_locate.argtypes = [i32, d, i32, d, d, i64, d, d, d, d, d, d]
        _lib.ora_stencil_absmax.argtypes = [i32, d, i32, d, i32, d, d, d, i32, d, i64, d, d, d]
        _lib.ora_alphas.argtypes = [i32, d, d, i64, d, d, i32, i32]
        _lib.ora_dy.argtypes = [i32, d, i32, d, i32, d, d, d, i32, d, d, i64, d, d,
                                ctypes.c_double, ctypes.c_double, d, i32]
        _lib.ora_hermite_basis.argtypes = [ctypes.c_double, d]
        _lib.ora_hermite_eval.argtypes = [ctypes.c_double] * 7
        _lib.ora_hermite_eval.restype = ctypes.c_double
        _lib.ora_hermite_1d.argtypes = [d, d, ctypes.c_long, i32, i32, ctypes.c_double]
        _lib.ora_hermite_1d.restype = ctypes.c_double
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def default_threads() -> int:
    n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def xfx(grid, pids, x, q2, mode: int = 0, nthreads: int | None = None) -> np.ndarray:
    """xf for pids (request order = column order) at points (x, q2) -> [n, len(pids)].

    ``grid`` is any object with pids, x, q2, q_off, xf arrays (FP64 values).
    mode 0: NaN outside the grid; mode 1: clamp to the grid edge.
    """
    lib = _load()
    gp, gx, gq, go, gv = _i32(grid.pids), _f64(grid.x), _f64(grid.q2), _i32(grid.q_off), _f64(grid.xf)
    rp = _i32(np.atleast_1d(pids))
    x, q2 = _f64(x), _f64(q2)
    n = x.shape[0]
    out = np.empty((n, rp.shape[0]), dtype=np.float64)
    lib.ora_xfx(gp.shape[0], _p(gp), gx.shape[0], _p(gx), go.shape[0] - 1, _p(go), _p(gq), _p(gv),
                rp.shape[0], _p(rp), n, _p(x), _p(q2), _p(out), mode,
                nthreads or default_threads())
    return out


def locate(grid, x, q2):
    """(ix, s, iq, inside) per point: x interval, subgrid, subgrid-local Q^2 interval."""
    lib = _load()
    gx, gq, go = _f64(grid.x), _f64(grid.q2), _i32(grid.q_off)
    x, q2 = _f64(x), _f64(q2)
    n = x.shape[0]
    ix, s, iq, ins = (np.empty(n, dtype=np.int32) for _ in range(4))
    lib.ora_locate(gx.shape[0], _p(gx), go.shape[0] - 1, _p(go), _p(gq), n, _p(x), _p(q2),
                   _p(ix), _p(s), _p(iq), _p(ins))
    return ix, s, iq, ins.astype(bool)


def stencil_absmax(grid, pids, x, q2) -> np.ndarray:
    """max |knot value| over each point's stencil, per requested pid -> [n, len(pids)]."""
    lib = _load()
    gp, gx, gq, go, gv = _i32(grid.pids), _f64(grid.x), _f64(grid.q2), _i32(grid.q_off), _f64(grid.xf)
    rp = _i32(np.atleast_1d(pids))
    x, q2 = _f64(x), _f64(q2)
    n = x.shape[0]
    out = np.empty((n, rp.shape[0]), dtype=np.float64)
    lib.ora_stencil_absmax(gp.shape[0], _p(gp), gx.shape[0], _p(gx), go.shape[0] - 1, _p(go),
                           _p(gq), _p(gv), rp.shape[0], _p(rp), n, _p(x), _p(q2), _p(out))
    return out


def alphas(as_q2, as_val, q2, mode: int = 0, nthreads: int | None = None) -> np.ndarray:
    lib = _load()
    aq, av, q2 = _f64(as_q2), _f64(as_val), _f64(q2)
    out = np.empty(q2.shape[0], dtype=np.float64)
    lib.ora_alphas(aq.shape[0], _p(aq), _p(av), q2.shape[0], _p(q2), _p(out), mode,
                   nthreads or default_threads())
    return out


def _continue(f0, f1, u):
    """Continuation from the edge value f0 through the next knot's f1, u in
    units of that knot step (u <= 0 outside): power law (linear in ln|f| against
    the log coordinate) when f1 / f0 > 0, else linear in the log coordinate."""
    with np.errstate(divide="ignore", invalid="ignore"):
        r = f1 / f0
        pw = f0 * np.exp(u * np.log(np.where(r > 0, r, 1.0)))
    return np.where((f0 != 0) & (r > 0), pw, f0 + u * (f1 - f0))


def xfx_extrapolated(grid, pids, x, q2, nthreads: int | None = None) -> np.ndarray:
    """x f with continuation outside the grid (the out-of-grid reading of the
    library's EXTRAPOLATE mode; inside the grid it is xfx itself).

    Along an axis the edge knot e and the next knot n inward give F_e and F_n
    (the interpolation evaluated at those knot coordinates, the other
    coordinate as queried); beyond the edge, with u = ln(z/z_e) / ln(z_n/z_e),
    xf = F_e (F_n/F_e)^u if F_n/F_e > 0, else F_e + u (F_n - F_e).  Outside in
    both x and Q^2: continue in x at the two Q^2 edge knots, then in Q^2.
    NaN inputs give NaN.
    """
    rp = np.atleast_1d(np.asarray(pids, dtype=np.int32))
    x, q2 = _f64(x), _f64(q2)
    out = xfx(grid, rp, x, q2, 0, nthreads)
    gx, gq = np.asarray(grid.x, dtype=np.float64), np.asarray(grid.q2, dtype=np.float64)
    xo = (x < gx[0]) | (x > gx[-1])
    qo = (q2 < gq[0]) | (q2 > gq[-1])
    sel = (xo | qo) & ~np.isnan(x) & ~np.isnan(q2)
    if not sel.any():
        return out
    xs, qs, xos, qos = x[sel], q2[sel], xo[sel], qo[sel]
    low_x = xs < gx[0]
    xe = np.where(low_x, gx[0], gx[-1])
    xn = np.where(low_x, gx[1], gx[-2])
    low_q = qs < gq[0]
    qe = np.where(low_q, gq[0], gq[-1])
    qn = np.where(low_q, gq[1], gq[-2])
    with np.errstate(divide="ignore", invalid="ignore"):
        ux = np.log(xs / xe) / np.log(xn / xe)
        uq = np.log(qs / qe) / np.log(qn / qe)
    ev = lambda xx, qq: xfx(grid, rp, xx, qq, 0, nthreads)  # noqa: E731
    res = np.empty((xs.shape[0], rp.shape[0]))
    m = xos & ~qos                      # x outside only
    if m.any():
        res[m] = _continue(ev(xe[m], qs[m]), ev(xn[m], qs[m]), ux[m][:, None])
    m = qos & ~xos                      # Q^2 outside only
    if m.any():
        res[m] = _continue(ev(xs[m], qe[m]), ev(xs[m], qn[m]), uq[m][:, None])
    m = xos & qos                       # both
    if m.any():
        a = _continue(ev(xe[m], qe[m]), ev(xn[m], qe[m]), ux[m][:, None])
        b = _continue(ev(xe[m], qn[m]), ev(xn[m], qn[m]), ux[m][:, None])
        res[m] = _continue(a, b, uq[m][:, None])
    out[sel] = res
    return out


def lumi(grid, pid_a, pid_b, x1, x2, q2, coef=None, mode: int = 0,
         nthreads: int | None = None):
    """Flavour-pair luminosity of the integrand of Eq. (1) (Sec. 3.1; the
    single-top example of Fig. 4 divides the PDF products by x1 x2):

        L[p, k] = f_{pid_a[k]}(x1[p], q2[p]) * f_{pid_b[k]}(x2[p], q2[p]),  f = xf / x,
        S[p]    = sum_k coef[k] * L[p, k]     (coef None: all 1).

    q2 is an array or a scalar.  mode 0: NaN where x1, x2 or q2 is outside
    the grid; mode 1: every coordinate clamped to the grid edge, x included in
    f = xf / x.  A pair with a pid absent from the grid is 0.  Returns (L, S).
    """
    pid_a = np.atleast_1d(np.asarray(pid_a, dtype=np.int32))
    pid_b = np.atleast_1d(np.asarray(pid_b, dtype=np.int32))
    x1, x2 = _f64(x1), _f64(x2)
    q2 = np.broadcast_to(np.asarray(q2, dtype=np.float64), x1.shape).copy()
    xlo, xhi = float(np.min(grid.x)), float(np.max(grid.x))
    qlo, qhi = float(np.min(grid.q2)), float(np.max(grid.q2))
    bad = ~((x1 >= xlo) & (x1 <= xhi) & (x2 >= xlo) & (x2 <= xhi) & (q2 >= qlo) & (q2 <= qhi))
    if mode == 1:
        nan_in = np.isnan(x1) | np.isnan(x2) | np.isnan(q2)
        x1 = np.where(nan_in, x1, np.clip(x1, xlo, xhi))
        x2 = np.where(nan_in, x2, np.clip(x2, xlo, xhi))
        q2 = np.where(nan_in, q2, np.clip(q2, qlo, qhi))
        bad = nan_in
    fa = xfx(grid, pid_a, x1, q2, mode, nthreads) / x1[:, None]
    fb = xfx(grid, pid_b, x2, q2, mode, nthreads) / x2[:, None]
    L = fa * fb
    L[bad, :] = np.nan
    present = set(int(p) for p in grid.pids)
    canon = lambda p: 21 if p == 0 else p  # noqa: E731  (gluon id 0 or 21)
    pset = set(canon(p) for p in present)
    for k in range(pid_a.shape[0]):
        if canon(int(pid_a[k])) not in pset or canon(int(pid_b[k])) not in pset:
            L[:, k] = 0.0
    c = np.ones(pid_a.shape[0]) if coef is None else np.asarray(coef, dtype=np.float64)
    S = L @ c
    return L, S


def dy(grid, u1, u2, xmin: float, s: float, nthreads: int | None = None) -> np.ndarray:
    """Per-point LO Drell-Yan-like integrand I(u1, u2) (see pdf_oracle.c)."""
    lib = _load()
    gp, gx, gq, go, gv = _i32(grid.pids), _f64(grid.x), _f64(grid.q2), _i32(grid.q_off), _f64(grid.xf)
    aq, av = _f64(grid.as_q2), _f64(grid.as_val)
    u1, u2 = _f64(u1), _f64(u2)
    out = np.empty(u1.shape[0], dtype=np.float64)
    lib.ora_dy(gp.shape[0], _p(gp), gx.shape[0], _p(gx), go.shape[0] - 1, _p(go), _p(gq), _p(gv),
               aq.shape[0], _p(aq), _p(av), u1.shape[0], _p(u1), _p(u2), xmin, s, _p(out),
               nthreads or default_threads())
    return out


def hermite_basis(t: float) -> np.ndarray:
    h = np.empty(4, dtype=np.float64)
    _load().ora_hermite_basis(t, _p(h))
    return h


def hermite_eval(z0, z1, y0, y1, m0, m1, z) -> float:
    return _load().ora_hermite_eval(z0, z1, y0, y1, m0, m1, z)


def hermite_1d(z, y, i: int, zq: float) -> float:
    """1-D interpolant of knots (z, y) with the method's finite-difference slopes."""
    z, y = _f64(z), _f64(y)
    return _load().ora_hermite_1d(_p(z), _p(y), 1, z.shape[0], i, zq)
