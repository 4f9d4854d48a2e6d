"""torch-facing API, named after the paper's interface (Sec. 2.1, Fig. 1):
``mkPDF`` builds a PDF object for one member; ``xfxQ2`` / ``xfxQ`` /
``py_xfxQ`` evaluate x f for a list of pids at arrays of points;
``alphasQ2`` / ``alphasQ`` / ``py_alphasQ`` evaluate alpha_s; ``trace`` warms
the kernels up and tunes the launch shape (HIP code is compiled ahead of time,
so there is nothing to trace).

torch provides device memory and the current stream; the computation itself
is done by libpdfx's HIP kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B

_PREC = {"f64": B.PDFX_F64, "fp64": B.PDFX_F64, "f32s": B.PDFX_F32S, "fp32": B.PDFX_F32S,
         "f32": B.PDFX_F32S}
_DOMAIN = {"nan": B.PDFX_DOMAIN_NAN, "clamp": B.PDFX_DOMAIN_CLAMP,
           "extrapolate": B.PDFX_DOMAIN_EXTRAPOLATE, "error": B.PDFX_DOMAIN_ERROR}


def prec_code(prec) -> int:
    return prec if isinstance(prec, int) else _PREC[prec]


def prec_dtype(prec) -> torch.dtype:
    return torch.float64 if prec_code(prec) == B.PDFX_F64 else torch.float32


def _device_f64(a, device=None) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        if a.device.type != "cuda":
            a = a.to(device or "cuda")
        if a.dtype != torch.float64:
            a = a.to(torch.float64)
        return a.contiguous()
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device=device or "cuda")


def _stream(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


# Argument checks before any launch: the C ABI takes raw device pointers and
# sizes, so a tensor of the wrong length, type or device would be read or
# written past its end.

def _same_length(*named):
    n = named[0][1].numel()
    for name, t in named[1:]:
        if t.numel() != n:
            raise ValueError("%s has %d elements, %s has %d" % (named[0][0], n, name, t.numel()))
    return n


def _on_device(t, device, name):
    if t.device != device:
        raise ValueError("%s is on %s, expected %s" % (name, t.device, device))


def _check_tensor(t, shape, dtype, device, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    if t.dtype != dtype:
        raise TypeError("%s has dtype %s, expected %s" % (name, t.dtype, dtype))
    _on_device(t, device, name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def _out(out, shape, prec, device, name="out"):
    if out is None:
        return torch.empty(shape, dtype=prec_dtype(prec), device=device)
    _check_tensor(out, shape, prec_dtype(prec), device, name)
    return out


def _domain(domain):
    if domain not in _DOMAIN:
        raise ValueError("domain must be one of %s" % sorted(_DOMAIN))
    return _DOMAIN[domain]


class PDF:
    """One PDF member resident on the current GPU."""

    def __init__(self, spec, with_values: bool = True):
        self._desc = B.HostDesc.from_spec(spec, with_values)
        self.handle = B.pdfx_load_grid(self._desc)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.pids = np.array(spec.pids, dtype=np.int32)
        self.n_flav, self.n_x, self.n_q, self.n_sub, self.n_as = B.pdfx_grid_shape(self.handle)
        self.shape = (self.n_flav, self.n_x, self.n_q)

    def close(self):
        if getattr(self, "handle", None):
            B.pdfx_free_grid(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _values(self, values, prec):
        if values is not None:
            _check_tensor(values, self.shape, prec_dtype(prec), self.device, "values")
        return _ptr(values)

    def _points(self, *arrays):
        """FP64 contiguous tensors on the grid's device, of one length."""
        ts = [_device_f64(a, self.device) for a in arrays]
        for t in ts:
            _on_device(t, self.device, "points")
        _same_length(*[("point array %d" % i, t) for i, t in enumerate(ts)])
        return ts

    # -- PDF --
    def xfxQ2(self, pids, x, q2, prec="f64", values=None, domain="nan", out=None):
        """x f for each pid (columns, request order) at each point -> [n, len(pids)]."""
        x, q2 = self._points(x, q2)
        pids = np.atleast_1d(np.asarray(pids, dtype=np.int32))
        n = x.numel()
        vp = self._values(values, prec)
        out = _out(out, (n, pids.shape[0]), prec, self.device)
        B.pdfx_eval_xfx(self.handle, vp, prec_code(prec), pids, x.data_ptr(),
                        q2.data_ptr(), n, out.data_ptr(), _domain(domain), _stream(x.device))
        return out

    def xfxQ(self, pids, x, q, prec="f64", values=None, domain="nan", out=None):
        x, q = self._points(x, q)
        pids = np.atleast_1d(np.asarray(pids, dtype=np.int32))
        n = x.numel()
        vp = self._values(values, prec)
        out = _out(out, (n, pids.shape[0]), prec, self.device)
        B.pdfx_eval_xfxQ(self.handle, vp, prec_code(prec), pids, x.data_ptr(),
                         q.data_ptr(), n, out.data_ptr(), _domain(domain), _stream(x.device))
        return out

    py_xfxQ = xfxQ
    py_xfxQ2 = xfxQ2

    def xfx_alphasQ2(self, pids, x, q2, prec="f64", values=None, domain="nan", out=None,
                     as_out=None):
        """x f for each pid and alpha_s at the same points, in one call
        -> ([n, len(pids)], [n]); x f equal to xfxQ2, alpha_s to alphasQ2 up to rounding."""
        x, q2 = self._points(x, q2)
        pids = np.atleast_1d(np.asarray(pids, dtype=np.int32))
        n = x.numel()
        vp = self._values(values, prec)
        out = _out(out, (n, pids.shape[0]), prec, self.device)
        as_out = _out(as_out, (n,), prec, self.device, "as_out")
        B.pdfx_eval_xfx_alphas(self.handle, vp, prec_code(prec), pids, x.data_ptr(),
                               q2.data_ptr(), n, out.data_ptr(), as_out.data_ptr(),
                               _domain(domain), _stream(x.device))
        return out, as_out

    # -- alpha_s --
    def alphasQ2(self, q2, prec="f64", domain="nan", out=None):
        (q2,) = self._points(q2)
        n = q2.numel()
        out = _out(out, (n,), prec, self.device)
        B.pdfx_eval_alphas(self.handle, q2.data_ptr(), n, out.data_ptr(), prec_code(prec),
                           _domain(domain), _stream(q2.device))
        return out

    def alphasQ(self, q, prec="f64", domain="nan", out=None):
        """alpha_s at scales Q (GeV): Q^2 = Q*Q is formed in FP64 by the library."""
        (q,) = self._points(q)
        n = q.numel()
        out = _out(out, (n,), prec, self.device)
        B.pdfx_eval_alphasQ(self.handle, q.data_ptr(), n, out.data_ptr(), prec_code(prec),
                            _domain(domain), _stream(q.device))
        return out

    py_alphasQ = alphasQ

    # -- misc --
    def domain_errors(self) -> int:
        return B.pdfx_domain_errors(self.handle)

    def launch(self, prec="f64"):
        return B.pdfx_get_launch(self.handle, prec_code(prec))

    def set_launch(self, prec, block, ppt):
        B.pdfx_set_launch(self.handle, prec_code(prec), block, ppt)

    def dy_launch(self, prec="f64"):
        return B.pdfx_get_dy_launch(self.handle, prec_code(prec))

    def set_dy_launch(self, prec, block, ppt):
        B.pdfx_set_dy_launch(self.handle, prec_code(prec), block, ppt)

    def lumi_launch(self, prec="f64"):
        return B.pdfx_get_lumi_launch(self.handle, prec_code(prec))

    def set_lumi_launch(self, prec, block, ppt):
        B.pdfx_set_lumi_launch(self.handle, prec_code(prec), block, ppt)

    def lumi(self, pid_a, pid_b, x1, x2, q2=None, q2_fixed=None, coef=None, prec="f64",
             pairs=True, total=True, domain="nan", values=None):
        """Flavour-pair luminosity (Eq. 1; Fig. 4's single-top example):
        L[p, k] = f_{pid_a[k]}(x1[p], Q2) f_{pid_b[k]}(x2[p], Q2) with f = xf / x
        and S[p] = sum_k coef[k] L[p, k], at Q2 = q2[p] or q2_fixed.
        Returns (L or None, S or None)."""
        if q2 is None and q2_fixed is None:
            raise ValueError("give q2 or q2_fixed")
        if q2 is None:
            x1, x2 = self._points(x1, x2)
            q2t = None
        else:
            x1, x2, q2t = self._points(x1, x2, q2)
        pid_a = np.atleast_1d(np.asarray(pid_a, dtype=np.int32))
        n = x1.numel()
        vp = self._values(values, prec)
        L = _out(None, (n, pid_a.shape[0]), prec, self.device) if pairs else None
        S = _out(None, (n,), prec, self.device) if total else None
        B.pdfx_eval_lumi(self.handle, vp, prec_code(prec), pid_a, pid_b, coef,
                         x1.data_ptr(), x2.data_ptr(), _ptr(q2t),
                         0.0 if q2_fixed is None else q2_fixed, n, _ptr(L), _ptr(S),
                         _domain(domain), _stream(x1.device))
        return L, S

    def autotune(self, prec="f64", n_req=None, n_pts=1 << 22, cache_path=None):
        B.pdfx_autotune(self.handle, prec_code(prec), n_req or self.n_flav, n_pts, cache_path)
        return self.launch(prec)

    def trace(self, n_pts=1 << 20, tune=True):
        """Warm-up: one small call per precision (and a launch-shape tune)."""
        for prec in ("f64", "f32s"):
            if tune:
                try:
                    self.autotune(prec, n_pts=n_pts)
                except B.PdfxError:
                    pass
            x = torch.full((256,), 0.1, dtype=torch.float64, device="cuda")
            self.xfxQ2(self.pids, x, torch.full_like(x, 100.0), prec=prec)
        torch.cuda.synchronize()

    alphas_trace = trace


def check_points(spec, x, q2) -> int:
    """Number of host points (x, q2) outside the grid of spec (a grid object or
    a set member 'NAME/M'), by the library's host-side check; no GPU needed."""
    if isinstance(spec, str):
        from . import lhapdf
        spec = lhapdf.load_member(spec, None)
    return B.pdfx_check_points(B.HostDesc.from_spec(spec, False), x, q2)


def mkPDF(spec, dirname: str | None = None, with_values: bool = True) -> PDF:
    """Build a PDF object for one member (the paper's mkPDF, Sec. 2.1, Fig. 1,
    Fig. 4): spec is a grid object (pids, x, q2, q_off, xf, optional alpha_s
    knots) or a set member named 'NAME/M' read from the standard grid folders
    under dirname (else LHAPDF_DATA_PATH)."""
    if isinstance(spec, str):
        from . import lhapdf
        spec = lhapdf.load_member(spec, dirname)
    return PDF(spec, with_values)


class PDFSet:
    """Many members (uneven grids, shared pid list) evaluated in one launch;
    specs is a list of grid objects or the name of a set in the standard grid
    folders (every member; dirname as for mkPDF)."""

    def __init__(self, specs, dirname: str | None = None):
        if isinstance(specs, str):
            from . import lhapdf
            specs = lhapdf.load_set(specs, dirname)
        self._descs = [B.HostDesc(s.pids, s.x, s.q2, s.q_off, s.xf) for s in specs]
        self.handle = B.pdfx_load_set(self._descs)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.n_mem = len(specs)
        self.pids = np.array(specs[0].pids, dtype=np.int32)

    def close(self):
        if getattr(self, "handle", None):
            B.pdfx_free_set(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def xfxQ2(self, pids, x, q2, prec="f64", domain="nan", out=None):
        """x f of every member -> [n_mem, n, len(pids)]."""
        x = _device_f64(x, self.device)
        q2 = _device_f64(q2, self.device)
        _on_device(x, self.device, "x")
        _on_device(q2, self.device, "q2")
        n = _same_length(("x", x), ("q2", q2))
        pids = np.atleast_1d(np.asarray(pids, dtype=np.int32))
        out = _out(out, (self.n_mem, n, pids.shape[0]), prec, self.device)
        B.pdfx_eval_set_xfx(self.handle, prec_code(prec), pids, x.data_ptr(), q2.data_ptr(), n,
                            out.data_ptr(), _domain(domain), _stream(x.device))
        return out

    def domain_errors(self) -> int:
        return B.pdfx_set_domain_errors(self.handle)

    def autotune(self, prec="f64", n_req=None, n_pts=1 << 20, cache_path=None):
        B.pdfx_autotune_set(self.handle, prec_code(prec), n_req or len(self.pids), n_pts, cache_path)


def dy_integrand(pdf, u1, u2, xmin=1e-5, s=13000.0 ** 2, prec="f64", values=None, out=True):
    """Per-point LO Drell-Yan-like integrand I(u1, u2) (pdfx_eval_dy) and the
    per-workgroup FP64 partial sums of I.  Returns (I or None, partial sums)."""
    u1, u2 = pdf._points(u1, u2)
    n = u1.numel()
    vp = pdf._values(values, prec)
    res = _out(None, (n,), prec, pdf.device) if out else None
    sums = torch.empty(B.pdfx_dy_max_blocks(), dtype=torch.float64, device=u1.device)
    nb = B.pdfx_eval_dy(pdf.handle, vp, prec_code(prec), u1.data_ptr(), u2.data_ptr(),
                        n, xmin, s, _ptr(res), sums.data_ptr(), _stream(u1.device))
    return res, sums[:nb]


def dy_backward(pdf, u1, u2, grad_xf, xmin=1e-5, s=13000.0 ** 2, scale=1.0, prec="f64",
                values=None):
    """grad_xf += scale * d(sum_p I_p)/d(knot values) (pdfx_eval_dy_backward)."""
    u1, u2 = pdf._points(u1, u2)
    vp = pdf._values(values, prec)
    _check_tensor(grad_xf, pdf.shape, prec_dtype(prec), pdf.device, "grad_xf")
    B.pdfx_eval_dy_backward(pdf.handle, vp, prec_code(prec), u1.data_ptr(),
                            u2.data_ptr(), u1.numel(), xmin, s, scale, grad_xf.data_ptr(),
                            _stream(u1.device))
    return grad_xf
