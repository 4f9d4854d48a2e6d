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
           "extrapolate": B.PDFX_DOMAIN_EXTRAPOLATE}


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


class PDF:
    """One PDF member resident on the current GPU."""

    def __init__(self, spec, with_values: bool = True):
        self._desc = B.HostDesc.from_spec(spec, with_values)
        self.handle = B.pdfx_load_grid(self._desc)
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

    # -- PDF --
    def xfxQ2(self, pids, x, q2, prec="f64", values=None, domain="nan", out=None):
        """x f for each pid (columns, request order) at each point -> [n, len(pids)]."""
        x = _device_f64(x)
        q2 = _device_f64(q2, x.device)
        pids = np.atleast_1d(np.asarray(pids, dtype=np.int32))
        n = x.numel()
        if out is None:
            out = torch.empty((n, pids.shape[0]), dtype=prec_dtype(prec), device=x.device)
        B.pdfx_eval_xfx(self.handle, _ptr(values), prec_code(prec), pids, x.data_ptr(),
                        q2.data_ptr(), n, out.data_ptr(), _DOMAIN[domain], _stream(x.device))
        return out

    def xfxQ(self, pids, x, q, prec="f64", values=None, domain="nan", out=None):
        x = _device_f64(x)
        q = _device_f64(q, x.device)
        pids = np.atleast_1d(np.asarray(pids, dtype=np.int32))
        n = x.numel()
        if out is None:
            out = torch.empty((n, pids.shape[0]), dtype=prec_dtype(prec), device=x.device)
        B.pdfx_eval_xfxQ(self.handle, _ptr(values), prec_code(prec), pids, x.data_ptr(),
                         q.data_ptr(), n, out.data_ptr(), _DOMAIN[domain], _stream(x.device))
        return out

    py_xfxQ = xfxQ
    py_xfxQ2 = xfxQ2

    def xfx_alphasQ2(self, pids, x, q2, prec="f64", values=None, domain="nan", out=None,
                     as_out=None):
        """x f for each pid and alpha_s at the same points, in one call
        -> ([n, len(pids)], [n]); x f equal to xfxQ2, alpha_s to alphasQ2 up to rounding."""
        x = _device_f64(x)
        q2 = _device_f64(q2, x.device)
        pids = np.atleast_1d(np.asarray(pids, dtype=np.int32))
        n = x.numel()
        if out is None:
            out = torch.empty((n, pids.shape[0]), dtype=prec_dtype(prec), device=x.device)
        if as_out is None:
            as_out = torch.empty(n, dtype=prec_dtype(prec), device=x.device)
        B.pdfx_eval_xfx_alphas(self.handle, _ptr(values), prec_code(prec), pids, x.data_ptr(),
                               q2.data_ptr(), n, out.data_ptr(), as_out.data_ptr(),
                               _DOMAIN[domain], _stream(x.device))
        return out, as_out

    # -- alpha_s --
    def alphasQ2(self, q2, prec="f64", domain="nan", out=None):
        q2 = _device_f64(q2)
        n = q2.numel()
        if out is None:
            out = torch.empty(n, dtype=prec_dtype(prec), device=q2.device)
        B.pdfx_eval_alphas(self.handle, q2.data_ptr(), n, out.data_ptr(), prec_code(prec),
                           _DOMAIN[domain], _stream(q2.device))
        return out

    def alphasQ(self, q, prec="f64", domain="nan", out=None):
        q = _device_f64(q)
        return self.alphasQ2(q * q, prec, domain, out)

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
        x1 = _device_f64(x1)
        x2 = _device_f64(x2, x1.device)
        q2t = None if q2 is None else _device_f64(q2, x1.device)
        if q2t is None and q2_fixed is None:
            raise ValueError("give q2 or q2_fixed")
        pid_a = np.atleast_1d(np.asarray(pid_a, dtype=np.int32))
        n = x1.numel()
        dt = prec_dtype(prec)
        L = torch.empty((n, pid_a.shape[0]), dtype=dt, device=x1.device) if pairs else None
        S = torch.empty(n, dtype=dt, device=x1.device) if total else None
        B.pdfx_eval_lumi(self.handle, _ptr(values), prec_code(prec), pid_a, pid_b, coef,
                         x1.data_ptr(), x2.data_ptr(), _ptr(q2t),
                         0.0 if q2_fixed is None else q2_fixed, n, _ptr(L), _ptr(S),
                         _DOMAIN[domain], _stream(x1.device))
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
        x = _device_f64(x)
        q2 = _device_f64(q2, x.device)
        pids = np.atleast_1d(np.asarray(pids, dtype=np.int32))
        n = x.numel()
        if out is None:
            out = torch.empty((self.n_mem, n, pids.shape[0]), dtype=prec_dtype(prec), device=x.device)
        B.pdfx_eval_set_xfx(self.handle, prec_code(prec), pids, x.data_ptr(), q2.data_ptr(), n,
                            out.data_ptr(), _DOMAIN[domain], _stream(x.device))
        return out

    def autotune(self, prec="f64", n_req=None, n_pts=1 << 20, cache_path=None):
        B.pdfx_autotune_set(self.handle, prec_code(prec), n_req or len(self.pids), n_pts, cache_path)


def dy_integrand(pdf, u1, u2, xmin=1e-5, s=13000.0 ** 2, prec="f64", values=None, out=True):
    """Per-point LO Drell-Yan-like integrand I(u1, u2) (pdfx_eval_dy) and the
    per-workgroup FP64 partial sums of I.  Returns (I or None, partial sums)."""
    u1 = _device_f64(u1)
    u2 = _device_f64(u2, u1.device)
    n = u1.numel()
    res = torch.empty(n, dtype=prec_dtype(prec), device=u1.device) if out else None
    sums = torch.empty(B.pdfx_dy_max_blocks(), dtype=torch.float64, device=u1.device)
    nb = B.pdfx_eval_dy(pdf.handle, _ptr(values), prec_code(prec), u1.data_ptr(), u2.data_ptr(),
                        n, xmin, s, _ptr(res), sums.data_ptr(), _stream(u1.device))
    return res, sums[:nb]


def dy_backward(pdf, u1, u2, grad_xf, xmin=1e-5, s=13000.0 ** 2, scale=1.0, prec="f64",
                values=None):
    """grad_xf += scale * d(sum_p I_p)/d(knot values) (pdfx_eval_dy_backward)."""
    u1 = _device_f64(u1)
    u2 = _device_f64(u2, u1.device)
    B.pdfx_eval_dy_backward(pdf.handle, _ptr(values), prec_code(prec), u1.data_ptr(),
                            u2.data_ptr(), u1.numel(), xmin, s, scale, grad_xf.data_ptr(),
                            _stream(u1.device))
    return grad_xf
