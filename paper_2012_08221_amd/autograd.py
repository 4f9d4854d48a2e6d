"""Differentiable evaluation: x f as a torch.autograd.Function.

forward runs pdfx_eval_xfx on caller-provided grid values; backward runs
pdfx_eval_xfx_backward, the hand-written adjoint, which returns the gradient
with respect to the grid knot values (summed in FP64 on the device) and with
respect to x and Q^2.  Gradients with respect to the values are exact (the
interpolation is linear in them); those with respect to x and Q^2 are the
derivatives of the piecewise cubic (one-sided at knots).
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B
from .api import _DOMAIN, _stream, prec_code, prec_dtype


class XfxFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, x, q2, pdf, pids, prec, domain):
        pids = np.atleast_1d(np.asarray(pids, dtype=np.int32))
        if values.dtype != prec_dtype(prec):
            raise TypeError("values must be %s for precision %s" % (prec_dtype(prec), prec))
        if tuple(values.shape) != tuple(pdf.shape):
            raise ValueError("values must have shape %s" % (pdf.shape,))
        values = values.contiguous()
        out = pdf.xfxQ2(pids, x, q2, prec=prec, values=values, domain=domain)
        ctx.save_for_backward(values, x, q2)
        ctx.pdf, ctx.pids, ctx.prec, ctx.domain = pdf, pids, prec, domain
        return out

    @staticmethod
    def backward(ctx, gout):
        values, x, q2 = ctx.saved_tensors
        pdf, pids, prec = ctx.pdf, ctx.pids, ctx.prec
        gout = gout.contiguous().to(prec_dtype(prec))
        gv = torch.zeros_like(values) if ctx.needs_input_grad[0] else None
        gx = torch.empty_like(x) if ctx.needs_input_grad[1] else None
        gq = torch.empty_like(q2) if ctx.needs_input_grad[2] else None
        if gv is not None or gx is not None or gq is not None:
            B.pdfx_eval_xfx_backward(
                pdf.handle, values.data_ptr(), prec_code(prec), pids, x.data_ptr(), q2.data_ptr(),
                x.numel(), gout.data_ptr(), None if gv is None else gv.data_ptr(),
                None if gx is None else gx.data_ptr(), None if gq is None else gq.data_ptr(),
                _DOMAIN[ctx.domain], _stream(x.device))
        return gv, gx, gq, None, None, None, None


def xfx(pdf, values, pids, x, q2, prec="f32s", domain="nan"):
    """x f for pids at (x, Q^2) from grid values `values` [n_flav, n_x, n_q],
    differentiable in values, x and q2 (x and q2 FP64 device tensors)."""
    x, q2 = pdf._points(x, q2)
    return XfxFunction.apply(values, x, q2, pdf, pids, prec, domain)
