"""Thin ctypes binding of libpdfx.so (the C-ABI declared in include/pdfx.h).

Argument marshalling only: every step of an evaluation runs in the library's
HIP kernels.  torch supplies device memory and the stream.  If the library is
not built this module raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdfx.so")

PDFX_OK = 0
PDFX_EINVAL = -1
PDFX_ENOMEM = -2
PDFX_EHIP = -3
PDFX_EDOMAIN = -4
PDFX_ENOALPHAS = -5
PDFX_ENOVALUES = -6
PDFX_F64 = 0
PDFX_F32S = 1
PDFX_DOMAIN_NAN = 0
PDFX_DOMAIN_CLAMP = 1
PDFX_DOMAIN_EXTRAPOLATE = 2
PDFX_DOMAIN_ERROR = 3
PDFX_MAX_REQ = 64

# Launch shapes (workgroup size, points per thread) compiled into the forward
# kernels; a negative count selects the store-as-you-go variant.  A positive
# count holds results in registers and stages flavour groups when the
# request allows it (else one flavour at a time).
LAUNCH_SHAPES = ((256, 2), (256, 4), (512, 1), (512, 2), (1024, 1),
                 (256, -2), (256, -4), (256, -8), (512, -1), (512, -2), (512, -4), (1024, -1),
                 (1024, -2))
# Shapes compiled for the FP32-stencil precision only (double-buffered kernel).
LAUNCH_SHAPES_F32 = ((512, 4),)

# Every function the header declares, in header order.
EXPORTS = (
    "pdfx_load_grid", "pdfx_free_grid", "pdfx_grid_shape", "pdfx_eval_xfx", "pdfx_eval_xfxQ",
    "pdfx_eval_alphas", "pdfx_eval_alphasQ", "pdfx_eval_xfx_alphas", "pdfx_eval_xfx_backward",
    "pdfx_eval_xfx_backward_noalloc", "pdfx_load_set", "pdfx_free_set",
    "pdfx_eval_set_xfx", "pdfx_eval_dy", "pdfx_dy_max_blocks", "pdfx_eval_dy_backward",
    "pdfx_autotune", "pdfx_autotune_set", "pdfx_get_launch", "pdfx_set_launch",
    "pdfx_get_dy_launch", "pdfx_set_dy_launch",
    "pdfx_eval_lumi", "pdfx_get_lumi_launch", "pdfx_set_lumi_launch",
    "pdfx_domain_errors", "pdfx_set_domain_errors", "pdfx_check_points", "pdfx_bench_lds", "pdfx_last_error", "pdfx_version",
)


class PdfxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("pdfx error %d: %s" % (code, msg))
        self.code = code


class PdfxDomainError(PdfxError):
    """PDFX_EDOMAIN: a PDFX_DOMAIN_ERROR call found points outside the grid
    (its outputs were written, NaN at those points)."""


class GridDesc(ctypes.Structure):
    _fields_ = [
        ("n_flav", ctypes.c_int32), ("pids", ctypes.c_void_p),
        ("n_x", ctypes.c_int32), ("x", ctypes.c_void_p),
        ("n_sub", ctypes.c_int32), ("q_off", ctypes.c_void_p),
        ("q2", ctypes.c_void_p), ("xf", ctypes.c_void_p),
        ("n_as", ctypes.c_int32), ("as_q2", ctypes.c_void_p), ("as_val", ctypes.c_void_p),
    ]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime under the same soname as ROCm's;
        # load torch first so that one runtime serves both (a second runtime
        # loaded under torch hides the GPUs from it).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpdfx.so is not built (run __graft_entry__.build() or "
                               "python paper_2012_08221_amd/build.py); no fallback exists")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "pdfx_load_grid": ([vp, vp], i32),
            "pdfx_free_grid": ([vp], None),
            "pdfx_grid_shape": ([vp, vp, vp, vp, vp, vp], i32),
            "pdfx_eval_xfx": ([vp, vp, i32, vp, i32, vp, vp, i64, vp, i32, vp], i32),
            "pdfx_eval_xfxQ": ([vp, vp, i32, vp, i32, vp, vp, i64, vp, i32, vp], i32),
            "pdfx_eval_alphas": ([vp, vp, i64, vp, i32, i32, vp], i32),
            "pdfx_eval_alphasQ": ([vp, vp, i64, vp, i32, i32, vp], i32),
            "pdfx_eval_xfx_alphas": ([vp, vp, i32, vp, i32, vp, vp, i64, vp, vp, i32, vp], i32),
            "pdfx_eval_xfx_backward": ([vp, vp, i32, vp, i32, vp, vp, i64, vp, vp, vp, vp, i32,
                                        vp], i32),
            "pdfx_eval_xfx_backward_noalloc": ([vp, vp, i32, vp, i32, vp, vp, i64, vp, vp, vp, vp,
                                                i32, vp], i32),
            "pdfx_load_set": ([vp, i32, vp], i32),
            "pdfx_free_set": ([vp], None),
            "pdfx_eval_set_xfx": ([vp, i32, vp, i32, vp, vp, i64, vp, i32, vp], i32),
            "pdfx_eval_dy": ([vp, vp, i32, vp, vp, i64, dbl, dbl, vp, vp, vp, vp], i32),
            "pdfx_dy_max_blocks": ([], i32),
            "pdfx_eval_dy_backward": ([vp, vp, i32, vp, vp, i64, dbl, dbl, dbl, vp, vp], i32),
            "pdfx_autotune": ([vp, i32, i32, i64, ctypes.c_char_p], i32),
            "pdfx_autotune_set": ([vp, i32, i32, i64, ctypes.c_char_p], i32),
            "pdfx_get_launch": ([vp, i32, vp, vp], i32),
            "pdfx_set_launch": ([vp, i32, i32, i32], i32),
            "pdfx_get_dy_launch": ([vp, i32, vp, vp], i32),
            "pdfx_set_dy_launch": ([vp, i32, i32, i32], i32),
            "pdfx_eval_lumi": ([vp, vp, i32, i32, vp, vp, vp, vp, vp, vp, dbl, i64, vp, vp, i32,
                                vp], i32),
            "pdfx_get_lumi_launch": ([vp, i32, vp, vp], i32),
            "pdfx_set_lumi_launch": ([vp, i32, i32, i32], i32),
            "pdfx_domain_errors": ([vp, vp], i32),
            "pdfx_set_domain_errors": ([vp, vp], i32),
            "pdfx_check_points": ([vp, vp, vp, i64, vp], i32),
            "pdfx_bench_lds": ([i32, i32, i32, vp, vp], i32),
            "pdfx_last_error": ([], ctypes.c_char_p),
            "pdfx_version": ([], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(rc: int):
    if rc != PDFX_OK:
        cls = PdfxDomainError if rc == PDFX_EDOMAIN else PdfxError
        raise cls(rc, lib().pdfx_last_error().decode())
    return rc


def last_error() -> str:
    return lib().pdfx_last_error().decode()


class HostDesc:
    """Keeps the numpy arrays behind a GridDesc alive while it is used."""

    def __init__(self, pids, x, q2, q_off, xf=None, as_q2=None, as_val=None):
        self.pids = np.ascontiguousarray(pids, dtype=np.int32)
        self.x = np.ascontiguousarray(x, dtype=np.float64)
        self.q2 = np.ascontiguousarray(q2, dtype=np.float64)
        self.q_off = np.ascontiguousarray(q_off, dtype=np.int32)
        self.xf = None if xf is None else np.ascontiguousarray(xf, dtype=np.float64)
        self.as_q2 = None if as_q2 is None or len(as_q2) == 0 else np.ascontiguousarray(as_q2, np.float64)
        self.as_val = None if as_val is None or len(as_val) == 0 else np.ascontiguousarray(as_val, np.float64)
        p = lambda a: None if a is None else a.ctypes.data  # noqa: E731
        self.desc = GridDesc(
            n_flav=self.pids.shape[0], pids=p(self.pids), n_x=self.x.shape[0], x=p(self.x),
            n_sub=self.q_off.shape[0] - 1, q_off=p(self.q_off), q2=p(self.q2), xf=p(self.xf),
            n_as=0 if self.as_q2 is None else self.as_q2.shape[0],
            as_q2=p(self.as_q2), as_val=p(self.as_val))

    @classmethod
    def from_spec(cls, spec, with_values=True):
        return cls(spec.pids, spec.x, spec.q2, spec.q_off, spec.xf if with_values else None,
                   getattr(spec, "as_q2", None), getattr(spec, "as_val", None))


# ---- C-named wrappers (pointers are ints; streams are hipStream_t ints) ----

def pdfx_load_grid(desc: HostDesc) -> int:
    h = ctypes.c_void_p()
    check(lib().pdfx_load_grid(ctypes.byref(desc.desc), ctypes.byref(h)))
    return h.value


def pdfx_free_grid(h: int):
    lib().pdfx_free_grid(h)


def _pids(pids):
    arr = np.ascontiguousarray(np.atleast_1d(pids), dtype=np.int32)
    return arr, arr.ctypes.data


def pdfx_eval_xfx(h, xf_dev, prec, pids, x_ptr, q2_ptr, n_pts, out_ptr, domain_mode, stream):
    arr, p = _pids(pids)
    return check(lib().pdfx_eval_xfx(h, xf_dev, prec, p, arr.shape[0], x_ptr, q2_ptr, n_pts,
                                     out_ptr, domain_mode, stream))


def pdfx_eval_xfxQ(h, xf_dev, prec, pids, x_ptr, q_ptr, n_pts, out_ptr, domain_mode, stream):
    arr, p = _pids(pids)
    return check(lib().pdfx_eval_xfxQ(h, xf_dev, prec, p, arr.shape[0], x_ptr, q_ptr, n_pts,
                                      out_ptr, domain_mode, stream))


def pdfx_eval_xfx_alphas(h, xf_dev, prec, pids, x_ptr, q2_ptr, n_pts, out_ptr, as_ptr,
                         domain_mode, stream):
    arr, p = _pids(pids)
    return check(lib().pdfx_eval_xfx_alphas(h, xf_dev, prec, p, arr.shape[0], x_ptr, q2_ptr,
                                            n_pts, out_ptr, as_ptr, domain_mode, stream))


def pdfx_eval_alphas(h, q2_ptr, n, out_ptr, prec, domain_mode, stream):
    return check(lib().pdfx_eval_alphas(h, q2_ptr, n, out_ptr, prec, domain_mode, stream))


def pdfx_eval_alphasQ(h, q_ptr, n, out_ptr, prec, domain_mode, stream):
    return check(lib().pdfx_eval_alphasQ(h, q_ptr, n, out_ptr, prec, domain_mode, stream))


def pdfx_eval_xfx_backward(h, xf_dev, prec, pids, x_ptr, q2_ptr, n_pts, gout_ptr, gxf_ptr,
                           gx_ptr, gq2_ptr, domain_mode, stream):
    arr, p = _pids(pids)
    return check(lib().pdfx_eval_xfx_backward(h, xf_dev, prec, p, arr.shape[0], x_ptr, q2_ptr,
                                              n_pts, gout_ptr, gxf_ptr, gx_ptr, gq2_ptr,
                                              domain_mode, stream))


def pdfx_eval_xfx_backward_noalloc(h, xf_dev, prec, pids, x_ptr, q2_ptr, n_pts, gout_ptr,
                                   gxf_ptr, gx_ptr, gq2_ptr, domain_mode, stream):
    arr, p = _pids(pids)
    return check(lib().pdfx_eval_xfx_backward_noalloc(h, xf_dev, prec, p, arr.shape[0], x_ptr,
                                                      q2_ptr, n_pts, gout_ptr, gxf_ptr, gx_ptr,
                                                      gq2_ptr, domain_mode, stream))


PDFX_NOALLOC_SCRATCH_BYTES = 48 * 1024 * 1024


def pdfx_load_set(descs) -> int:
    arr = (GridDesc * len(descs))(*[d.desc for d in descs])
    h = ctypes.c_void_p()
    check(lib().pdfx_load_set(arr, len(descs), ctypes.byref(h)))
    return h.value


def pdfx_free_set(h: int):
    lib().pdfx_free_set(h)


def pdfx_eval_set_xfx(h, prec, pids, x_ptr, q2_ptr, n_pts, out_ptr, domain_mode, stream):
    arr, p = _pids(pids)
    return check(lib().pdfx_eval_set_xfx(h, prec, p, arr.shape[0], x_ptr, q2_ptr, n_pts, out_ptr,
                                         domain_mode, stream))


def pdfx_dy_max_blocks() -> int:
    return lib().pdfx_dy_max_blocks()


def pdfx_eval_dy(h, xf_dev, prec, u1_ptr, u2_ptr, n, xmin, s, out_ptr, sums_ptr, stream) -> int:
    nb = ctypes.c_int32(0)
    check(lib().pdfx_eval_dy(h, xf_dev, prec, u1_ptr, u2_ptr, n, xmin, s, out_ptr, sums_ptr,
                             ctypes.byref(nb), stream))
    return nb.value


def pdfx_eval_dy_backward(h, xf_dev, prec, u1_ptr, u2_ptr, n, xmin, s, scale, gxf_ptr, stream):
    return check(lib().pdfx_eval_dy_backward(h, xf_dev, prec, u1_ptr, u2_ptr, n, xmin, s, scale,
                                             gxf_ptr, stream))


def pdfx_autotune(h, prec, n_req, n_pts, cache_path=None):
    return check(lib().pdfx_autotune(h, prec, n_req, n_pts,
                                     None if cache_path is None else cache_path.encode()))


def pdfx_autotune_set(h, prec, n_req, n_pts, cache_path=None):
    return check(lib().pdfx_autotune_set(h, prec, n_req, n_pts,
                                         None if cache_path is None else cache_path.encode()))


def pdfx_get_launch(h, prec):
    b, p = ctypes.c_int32(), ctypes.c_int32()
    check(lib().pdfx_get_launch(h, prec, ctypes.byref(b), ctypes.byref(p)))
    return b.value, p.value


def pdfx_set_launch(h, prec, block, ppt):
    return check(lib().pdfx_set_launch(h, prec, block, ppt))


def pdfx_get_dy_launch(h, prec):
    b, p = ctypes.c_int32(), ctypes.c_int32()
    check(lib().pdfx_get_dy_launch(h, prec, ctypes.byref(b), ctypes.byref(p)))
    return b.value, p.value


def pdfx_set_dy_launch(h, prec, block, ppt):
    return check(lib().pdfx_set_dy_launch(h, prec, block, ppt))


def pdfx_eval_lumi(h, xf_dev, prec, pid_a, pid_b, coef, x1, x2, q2, q2_fixed, n, out_pair,
                   out_sum, domain_mode, stream):
    """pid_a, pid_b, coef: host sequences (coef may be None); device pointers as ints."""
    a, pa = _pids(pid_a)
    b, pb = _pids(pid_b)
    if a.shape != b.shape:
        raise ValueError("pid_a and pid_b differ in length")
    c = None if coef is None else np.ascontiguousarray(coef, dtype=np.float64)
    if c is not None and c.shape != a.shape:
        raise ValueError("coef and the pid lists differ in length")
    return check(lib().pdfx_eval_lumi(h, xf_dev, prec, a.shape[0], pa, pb,
                                      None if c is None else c.ctypes.data, x1, x2, q2,
                                      float(q2_fixed), n, out_pair, out_sum, domain_mode, stream))


def pdfx_get_lumi_launch(h, prec):
    b, p = ctypes.c_int32(), ctypes.c_int32()
    check(lib().pdfx_get_lumi_launch(h, prec, ctypes.byref(b), ctypes.byref(p)))
    return b.value, p.value


def pdfx_set_lumi_launch(h, prec, block, ppt):
    return check(lib().pdfx_set_lumi_launch(h, prec, block, ppt))


def pdfx_domain_errors(h) -> int:
    c = ctypes.c_int64()
    check(lib().pdfx_domain_errors(h, ctypes.byref(c)))
    return c.value


def pdfx_set_domain_errors(h) -> int:
    c = ctypes.c_int64()
    check(lib().pdfx_set_domain_errors(h, ctypes.byref(c)))
    return c.value


def pdfx_check_points(desc: HostDesc, x, q2) -> int:
    """Host arrays x, q2 against the grid that desc describes: the number of
    points outside it (PDFX_EDOMAIN is not raised; invalid arguments are)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    q2 = np.ascontiguousarray(q2, dtype=np.float64)
    if x.shape != q2.shape:
        raise ValueError("x and q2 differ in length")
    c = ctypes.c_int64()
    rc = lib().pdfx_check_points(ctypes.byref(desc.desc), x.ctypes.data, q2.ctypes.data,
                                 x.shape[0], ctypes.byref(c))
    if rc not in (PDFX_OK, PDFX_EDOMAIN):
        check(rc)
    return c.value


def pdfx_grid_shape(h):
    v = [ctypes.c_int32() for _ in range(5)]
    check(lib().pdfx_grid_shape(h, *[ctypes.byref(a) for a in v]))
    return tuple(a.value for a in v)


def pdfx_bench_lds(mode: int, blocks: int, iters: int, sink_ptr: int, stream: int):
    """Enqueues the LDS micro-benchmark: 16-byte reads (mode 0 lane-consecutive,
    1 random), FP64 atomic adds (2 lane-consecutive, 3 random) or 64-bit
    integer atomic adds (4, 5);
    blocks * 256 * iters operations."""
    check(lib().pdfx_bench_lds(mode, blocks, iters, sink_ptr, stream))


def pdfx_version() -> str:
    return lib().pdfx_version().decode()
