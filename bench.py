#!/usr/bin/env python3
"""Benchmark of the batched PDF evaluation hot path on one MI355X.

Headline step (timed K times after W warm-ups): x f for all 11 partons at 1e7
query points (log-uniform x in [1e-6, 0.99], Q in [2, 1e4] GeV) on the
11 x 100 x 50 three-subgrid member grid, plus alpha_s at the same points, in
the precision given by --prec.  Inputs are resident in HBM before timing.

Also measured (reported under "variants"):
  * the other precision of the same step;
  * forward + backward (knot and coordinate gradients) of sum w * xf on 1e6
    points with the grid as an FP32 tensor;
  * 101 members with uneven grids at 1e6 shared points, one launch, FP64 and
    FP32 stencil;
  * the fused Drell-Yan-like integrand over 1e8 points in 10 chunks of 1e7,
    forward and knot-gradient backward, FP64 and FP32 stencil;
  * the error against the CPU oracle on the first 1e6 points, and the oracle
    itself timed on the host cores (cpu_baseline).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_VEC_TFLOPS = 78.6         # MI355X vector FP64
FP32_VEC_TFLOPS = 157.3        # MI355X vector FP32 (no packed math)
N_PTS = 10_000_000
METRIC = "PDF evals/sec (points×flavours) FP32 vs FP64 at stated rel. error; fwd+bwd/s"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--prec", default="f64", choices=["f64", "f32s"])
    ap.add_argument("--n", type=int, default=N_PTS)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="only the headline step")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--only", default=None, choices=["xfx", "members", "folder", "dy", "bwd", "lumi"],
                    help="run one workload for a few steps (profiler runs) and print its timing")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a plain copy kernel of known size (counter scaling) and exit")
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cpu_model():
    """The host CPU's model name, from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def forward_kernel_sources():
    """Sources of the forward kernels (any change voids recorded counters)."""
    import glob
    csrc = os.path.join(HERE, "paper_2012_08221_amd", "csrc")
    return sorted(glob.glob(os.path.join(csrc, "xfx_*"))) + [os.path.join(csrc, "pdfx_internal.h")]


def forward_kernel_name(prec, launch):
    """Kernel that pdfx_eval_xfx_alphas runs for the bench grid (it fits the
    double-buffered kernel, and its alpha_s knots are its Q^2 knots, so x f and
    alpha_s come from one pass) with launch shape (block, ppt)."""
    v = "double" if prec == "f64" else "float"
    block, ppt = launch
    if ppt > 0:
        return "xfx_dma_kernel<%s, %d, %d, true>" % (v, block, ppt)
    return "xfx_kernel<%s, %d, %d, PF, DB, 0>" % (v, block, -ppt)


def lds_bytes(prec, launch, n, nf, nx, nq):
    """LDS bytes one forward launch moves (double-buffered kernel, ppt > 0):
    stencil reads (16 nodes of 16 B per point and flavour group), global-to-
    LDS slab copies (one slab per group and tile), the output rows staged
    through LDS (written, then read) and the four alpha_s values per point.
    None for the per-flavour kernel."""
    block, ppt = launch
    if ppt <= 0:
        return None
    vb = 8 if prec == "f64" else 4
    g = 16 // vb
    stages = (nf + g - 1) // g
    tiles = (n + block * ppt - 1) // (block * ppt)
    return n * stages * 16 * 16 + tiles * stages * nx * nq * 16 + 2 * n * nf * vb + n * 4 * vb


def recorded_traffic(prec, launch):
    """HBM bytes per launch of the forward kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE record, if it was taken on the same kernel source,
    precision and launch shape; otherwise None."""
    import hashlib
    path = os.path.join(HERE, "profiles", "xfx_fwd_1e7x11_hbm_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for f in forward_kernel_sources():
        with open(f, "rb") as fh:
            h.update(fh.read())
    if (rec.get("kernel_source_sha256") != h.hexdigest() or rec.get("prec") != prec
            or list(rec.get("launch_shape", [])) != list(launch)):
        return None
    return float(rec["traffic_bytes"])


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2012_08221_amd import api, autograd as ag
    from paper_2012_08221_amd import binding as B
    from paper_2012_08221_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    def timed(fn, reps, warm=1):
        """Median ms per call over `reps` calls (at least 20 for calls under
        10 ms), each bracketed by HIP events on the launch stream."""
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        ev = []
        for i in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            ev.append((e0, e1))
            if i == 0 and reps < 20:
                torch.cuda.synchronize()
                if e0.elapsed_time(e1) < 10.0:
                    reps = 20
        while len(ev) < reps:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            ev.append((e0, e1))
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))

    def copy_gbs():
        """HBM bandwidth a plain copy reaches: 1 GiB of FP64 read, 1 GiB written."""
        n = 1 << 27
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        ms = timed(lambda: torch.mul(a, 1.0, out=b), 5)
        del a, b
        return n, ms, 2 * n * 8 / ms / 1e6

    def lds_read_gbs():
        """LDS read rates the device reaches (pdfx_bench_lds, 8 workgroups
        per CU): aligned 16-byte reads, lane-consecutive and at random addresses."""
        cus = torch.cuda.get_device_properties(dev).multi_processor_count
        blocks, iters = cus * 8, 4096
        sink = torch.empty(blocks * 256, dtype=torch.float64, device=dev)
        rates = {}
        for mode, name in ((0, "measured_stream_gbs"), (1, "measured_random_gbs")):
            ms = timed(lambda: B.pdfx_bench_lds(mode, blocks, iters, sink.data_ptr(),
                                                     stream.cuda_stream), 5)
            rates[name] = blocks * 256 * iters * 16 / ms / 1e6
        return rates

    def lds_atomic_rates():
        """64-bit LDS atomic adds per second (pdfx_bench_lds modes 2-5), FP64 and
        integer: the ceilings of the gradient scatters (fixed-point sums use the
        integer adds)."""
        cus = torch.cuda.get_device_properties(dev).multi_processor_count
        blocks, iters = cus * 8, 1024
        sink = torch.empty(blocks * 256, dtype=torch.float64, device=dev)
        rates = {}
        for mode, name in ((2, "f64_consecutive_per_s"), (3, "f64_random_per_s"),
                           (4, "u64_consecutive_per_s"), (5, "u64_random_per_s")):
            ms = timed(lambda: B.pdfx_bench_lds(mode, blocks, iters, sink.data_ptr(),
                                                     stream.cuda_stream), 5)
            rates[name] = blocks * 256 * iters / (ms * 1e-3)
        return rates

    lds_cache = {}
    atomic_cache = {}

    def atomics_all():
        if not atomic_cache:
            atomic_cache.update(lds_atomic_rates())
        return atomic_cache

    def lds_meas_all():
        if not lds_cache:
            lds_cache.update(lds_read_gbs())
        return lds_cache

    def dy_fractions(prec, npts, chunk, ms_f, ms_b, lds, atomics, nx, nq, shape):
        """LDS and VALU fractions of the integrand (bound by neither HBM nor
        MFMA).  Forward LDS: the method's 164 values per point (10 partons x 16
        knots + 4 alpha_s) and the kernel's own node reads and slab copies, both
        against the measured LDS read rates.  VALU: the stencil arithmetic (2
        flops per multiply-add: 16 + 4 per parton, 4 for alpha_s) in the value
        precision plus the per-point FP64 work (3 weight folds of ~30 flops, 2 exp
        and 1 log at ~40 flops each, luminosity and Jacobian ~12), against
        MI355X's vector peaks.  Backward: 10 partons x 16 knot adds per point
        against the measured 64-bit LDS atomic rate."""
        vb = 8 if prec == "f64" else 4
        g = 16 // vb
        stencils = 6 if prec == "f64" else 4          # FP32: the middle group at both sides
        slabs = 12 // g
        tile = shape[0] * shape[1]
        tiles = npts // chunk * ((chunk + tile - 1) // tile)
        alg = npts * 164 * vb
        kern = npts * stencils * 16 * 16 + tiles * slabs * nx * nq * 16
        t = ms_f * 1e-3
        f_val = 10 * 2 * 20 + 2 * 4                  # flops in the value precision
        f_64 = 3 * 30 + 3 * 40 + 12                    # FP64 flops per point
        if prec == "f64":
            f_64 += f_val
            t_peak = npts * f_64 / (FP64_VEC_TFLOPS * 1e12)
        else:
            t_peak = npts * (f_64 / (FP64_VEC_TFLOPS * 1e12) + f_val / (FP32_VEC_TFLOPS * 1e12))
        adds = npts * 10 * 16
        return {
            "forward_lds": {"algorithmic_bytes_per_point": 164 * vb,
                            "algorithmic_gbs": alg / t / 1e9,
                            "kernel_bytes": kern, "kernel_gbs": kern / t / 1e9,
                            "frac_of_stream": kern / t / 1e9 / lds["measured_stream_gbs"],
                            "frac_of_random": kern / t / 1e9 / lds["measured_random_gbs"]},
            "forward_valu": {"flops_per_point_fp64": f_64,
                             "flops_per_point_fp32": 0 if prec == "f64" else f_val,
                             "time_at_vector_peak_ms": t_peak * 1e3,
                             "frac": t_peak / t},
            "backward_lds_atomics": {"adds": adds, "adds_per_s": adds / (ms_b * 1e-3),
                                     "frac_of_u64_random": adds / (ms_b * 1e-3)
                                     / atomics["u64_random_per_s"]}}

    if args.calib_copy:
        n, ms, gbs = copy_gbs()
        print(json.dumps({"calib_copy_bytes_read": n * 8, "calib_copy_bytes_written": n * 8,
                          "ms": ms, "gbs": gbs}))
        return

    grid = wl.config0_grid()
    pdf = api.mkPDF(grid)
    pids = grid.pids
    nf = len(pids)
    n = args.n
    variants = {}

    if args.only in (None, "xfx"):
        log("generating %d query points" % n)
        x_np, q2_np = wl.queries(1, n)
        x = torch.as_tensor(x_np, device=dev)
        q2 = torch.as_tensor(q2_np, device=dev)
        torch.cuda.synchronize()
        if not args.no_tune:
            for prec in ("f64", "f32s"):
                pdf.autotune(prec, n_req=nf, n_pts=n)
        results = {}
        precs = [args.prec] + ([] if (args.no_extra or args.only)
                               else [p for p in ("f64", "f32s") if p != args.prec])
        for prec in precs:
            dt = api.prec_dtype(prec)
            out = torch.empty((n, nf), dtype=dt, device=dev)
            aout = torch.empty(n, dtype=dt, device=dev)
            ev = []

            def step(rec):
                if rec:
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                pdf.xfx_alphasQ2(pids, x, q2, prec=prec, out=out, as_out=aout)
                if rec:
                    e1.record(stream)
                    ev.append((e0, e1))

            for _ in range(args.warmup):
                step(False)
            torch.cuda.synchronize()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record(stream)
            for _ in range(args.steps):
                step(True)
            t1.record(stream)
            torch.cuda.synchronize()
            ms = t0.elapsed_time(t1) / args.steps
            per = [a.elapsed_time(b) for a, b in ev]
            k_ms = float(np.mean(per))
            results[prec] = {"ms": ms, "xfx_ms": k_ms, "median_ms": float(np.median(per)),
                             "out": out, "as": aout, "launch": list(pdf.launch(prec))}
            log("%s: %.3f ms per step, xfx kernel %.3f ms" % (prec, ms, k_ms))
        if args.only == "xfx":
            r = results[args.prec]
            print(json.dumps({"only": "xfx", "prec": args.prec, "xfx_ms": r["xfx_ms"]}))
            return

        # latency of one call at the small size (1e5 points x 11 flavours and
        # alpha_s, the parity configuration): mean over 200 back-to-back calls
        if args.only is None and not args.no_extra:
            xs_np, qs_np = wl.queries(0, 100_000)
            xs = torch.as_tensor(xs_np, device=dev)
            qs = torch.as_tensor(qs_np, device=dev)
            lat = {"n_points": 100_000}
            for prec in ("f64", "f32s"):
                dt = api.prec_dtype(prec)
                o = torch.empty((100_000, nf), dtype=dt, device=dev)
                oa = torch.empty(100_000, dtype=dt, device=dev)
                lat[prec + "_ms"] = timed(
                    lambda: pdf.xfx_alphasQ2(pids, xs, qs, prec=prec, out=o, as_out=oa), 200, 5)
            variants["latency_1e5"] = lat
            log("1e5 points: %.1f us FP64, %.1f us FP32 per call"
                % (lat["f64_ms"] * 1e3, lat["f32s_ms"] * 1e3))
            del xs, qs, o, oa

        # EXTRAPOLATE mode on the same points with 1% of them moved below the
        # grid's x range (one decade): the forward pass plus the continuation
        if args.only is None and not args.no_extra:
            xe = x.clone()
            xe[::100] = float(grid.x[0]) * 0.1
            oute = torch.empty((n, nf), dtype=torch.float64, device=dev)
            ms_e = timed(lambda: pdf.xfxQ2(pids, xe, q2, out=oute, domain="extrapolate"), 5)
            ms_c = timed(lambda: pdf.xfxQ2(pids, xe, q2, out=oute, domain="clamp"), 5)
            variants["extrapolate"] = {"n_points": n, "outside_fraction": 0.01, "f64_ms": ms_e,
                                       "f64_clamp_ms": ms_c,
                                       "continuation_ms": ms_e - ms_c}
            log("extrapolate f64: %.3f ms (clamp %.3f ms)" % (ms_e, ms_c))
            del xe, oute

    # forward + backward: loss = sum w * xf on 1e6 points, grid as an FP32 tensor
    if args.only == "bwd" or (args.only is None and not args.no_extra):
        nb = 1_000_000
        xb_np, qb_np = wl.queries(3, nb)
        xb = torch.as_tensor(xb_np, device=dev).requires_grad_(True)
        qb = torch.as_tensor(qb_np, device=dev).requires_grad_(True)
        vals = torch.as_tensor(grid.xf, device=dev).to(torch.float32).requires_grad_(True)
        w = torch.as_tensor(wl.loss_weights(3, nb), device=dev).to(torch.float32)
        pdf3 = api.mkPDF(grid, with_values=False)

        def fwd():
            return ag.xfx(pdf3, vals, pids, xb, qb, prec="f32s")

        def fwd_bwd():
            vals.grad = xb.grad = qb.grad = None
            (fwd() * w).sum().backward()

        ms_f = timed(fwd, 10, 2)
        ms_fb = timed(fwd_bwd, 10, 2)
        variants["fwd_bwd"] = {
            "value": nb * nf / (ms_fb * 1e-3), "unit": "pf/s (forward+backward)",
            "ms_per_step": ms_fb, "forward_ms": ms_f, "backward_ms": ms_fb - ms_f,
            "n_points": nb, "dtype": "f32 stencil forward, FP64 adjoint",
            "what": "sum w*xf, gradients w.r.t. the 11x100x50 knots, x and Q^2",
            "knot_scatter_atomics": nb * nf * 16,
            "lds_atomic_64bit": atomics_all()}
        log("fwd+bwd: %.3f ms (forward %.3f)" % (ms_fb, ms_f))
        if args.only == "bwd":
            print(json.dumps({"only": "bwd", **variants["fwd_bwd"]}))
            return

    # 101 members, one launch
    if args.only == "members" or (args.only is None and not args.no_extra):
        members = wl.member_grids(101)
        pset = api.PDFSet(members)
        nm = 1_000_000
        xm_np, qm_np = wl.queries(2, nm)
        xm = torch.as_tensor(xm_np, device=dev)
        qm = torch.as_tensor(qm_np, device=dev)
        mres = {}
        for prec in ("f64", "f32s"):
            if not args.no_tune:
                pset.autotune(prec, n_req=nf, n_pts=nm)
            outm = torch.empty((101, nm, nf), dtype=api.prec_dtype(prec), device=dev)
            ms = timed(lambda: pset.xfxQ2(pids, xm, qm, prec=prec, out=outm), 3 if args.only else 5)
            bpe = 8 if prec == "f64" else 4
            gbs = (101 * nm * nf * bpe + 16 * nm) / ms / 1e6
            mres[prec] = {"value": 101 * nm * nf / (ms * 1e-3), "unit": "pf/s", "ms": ms,
                          "hbm_gbs_algorithmic": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
            del outm
            log("members %s: %.3f ms" % (prec, ms))
        variants["members"] = {"n_members": 101, "n_points": nm, **mres}
        del pset
        if args.only == "members":
            print(json.dumps({"only": "members", **variants["members"]}))
            return

    # The same 101 members as a set folder in the standard grid format: written
    # out (not timed), then read back on the host and read back onto the GPU
    if args.only == "folder" or (args.only is None and not args.no_extra):
        import shutil
        import tempfile
        from paper_2012_08221_amd import lhapdf
        members = wl.member_grids(101)
        tmp = tempfile.mkdtemp()
        try:
            folder = lhapdf.write_set(tmp, "SYNTH101", members)
            text = sum(os.path.getsize(os.path.join(folder, f)) for f in os.listdir(folder))
            t0 = time.perf_counter()
            lhapdf.load_set("SYNTH101", tmp)
            t_parse = time.perf_counter() - t0
            t0 = time.perf_counter()
            pset = api.PDFSet("SYNTH101", tmp)
            torch.cuda.synchronize()
            t_set = time.perf_counter() - t0
            del pset
        finally:
            shutil.rmtree(tmp, ignore_errors=True)
        variants["grid_folder"] = {
            "n_members": 101, "text_mb": text / 1e6, "parse_s": t_parse,
            "parse_mb_per_s": text / 1e6 / t_parse, "pdfset_from_folder_s": t_set,
            "what": "host reader of the standard grid format; PDFSet(name, dir) = read + "
                    "validate + device upload of every member"}
        log("grid folder: %.0f MB parsed in %.2f s; PDFSet from the folder %.2f s"
            % (text / 1e6, t_parse, t_set))
        if args.only == "folder":
            print(json.dumps({"only": "folder", **variants["grid_folder"]}))
            return

    # Drell-Yan-like integrand, 1e8 points in 10 chunks of 1e7
    if args.only == "dy" or (args.only is None and not args.no_extra):
        nchunk, csize = (10, 10_000_000) if not args.only else (2, 10_000_000)
        us = []
        for c in range(nchunk):
            gen = torch.Generator(device=dev)
            gen.manual_seed(wl.SEED_BASE + 4 + c)
            us.append((torch.rand(csize, dtype=torch.float64, device=dev, generator=gen),
                       torch.rand(csize, dtype=torch.float64, device=dev, generator=gen)))
        dres = {}
        for prec in ("f64", "f32s"):
            outd = torch.empty(csize, dtype=api.prec_dtype(prec), device=dev)
            sums = torch.empty(4096, dtype=torch.float64, device=dev)
            gxf = torch.zeros(grid.xf.shape, dtype=api.prec_dtype(prec), device=dev)
            from paper_2012_08221_amd import binding as B

            def fwd_all():
                for u1, u2 in us:
                    B.pdfx_eval_dy(pdf.handle, None, api.prec_code(prec), u1.data_ptr(),
                                   u2.data_ptr(), csize, wl.DY_XMIN, wl.SQRT_S_DY ** 2,
                                   outd.data_ptr(), sums.data_ptr(), stream.cuda_stream)

            def bwd_all():
                for u1, u2 in us:
                    B.pdfx_eval_dy_backward(pdf.handle, None, api.prec_code(prec), u1.data_ptr(),
                                            u2.data_ptr(), csize, wl.DY_XMIN, wl.SQRT_S_DY ** 2,
                                            1.0 / (nchunk * csize), gxf.data_ptr(),
                                            stream.cuda_stream)

            # launch shape of the integrand kernel: the fastest on the first chunk
            def fwd_one():
                u1, u2 = us[0]
                B.pdfx_eval_dy(pdf.handle, None, api.prec_code(prec), u1.data_ptr(),
                               u2.data_ptr(), csize, wl.DY_XMIN, wl.SQRT_S_DY ** 2,
                               outd.data_ptr(), sums.data_ptr(), stream.cuda_stream)
            tune = {}
            for shape in ((512, 1), (512, 2), (256, 2)) + (((512, 4),) if prec == "f32s" else ()):
                pdf.set_dy_launch(prec, *shape)
                tune[shape] = timed(fwd_one, 3)
            best = min(tune, key=tune.get)
            pdf.set_dy_launch(prec, *best)
            ms_f = timed(fwd_all, 2)
            ms_b = timed(bwd_all, 2)
            npts = nchunk * csize
            fr = dy_fractions(prec, npts, csize, ms_f, ms_b, lds_meas_all(), atomics_all(),
                              grid.n_x, grid.n_q, best)
            dres[prec] = {**fr, "forward_points_per_s": npts / (ms_f * 1e-3),
                          "backward_points_per_s": npts / (ms_b * 1e-3),
                          "forward_ms_per_chunk": ms_f / nchunk,
                          "backward_ms_per_chunk": ms_b / nchunk,
                          "forward_launch_shape": list(best),
                          "forward_shape_ms_chunk0": {"%dx%d" % k: v for k, v in tune.items()}}
            log("dy %s: forward %.3f ms/chunk (shape %s), backward %.3f ms/chunk" %
                (prec, ms_f / nchunk, best, ms_b / nchunk))
        variants["drell_yan"] = {"n_points": nchunk * csize, "chunk": csize, **dres}
        if args.only == "dy":
            print(json.dumps({"only": "dy", **variants["drell_yan"]}))
            return

    # flavour-pair luminosity, the single-top pattern of Fig. 4: b at x1
    # against u, c, dbar, sbar at x2, Q^2 = m_t^2, 1e7 points
    if args.only == "lumi" or (args.only is None and not args.no_extra):
        nl = 10_000_000
        g = torch.Generator(device=dev)
        g.manual_seed(201208226)
        lo = float(np.log(1e-5))
        x1 = torch.exp(lo - lo * torch.rand(nl, generator=g, dtype=torch.float64, device=dev))
        x2 = torch.exp(lo - lo * torch.rand(nl, generator=g, dtype=torch.float64, device=dev))
        pa, pb = [5, 5, 5, 5], [2, 4, -1, -3]
        lres = {}
        for prec in ("f64", "f32s"):
            dt = api.prec_dtype(prec)
            S = torch.empty(nl, dtype=dt, device=dev)
            L = torch.empty((nl, 4), dtype=dt, device=dev)
            code = api.prec_code(prec)

            def run_sum():
                B.pdfx_eval_lumi(pdf.handle, None, code, pa, pb, None, x1.data_ptr(),
                                 x2.data_ptr(), None, 172.5 ** 2, nl, None, S.data_ptr(), 0,
                                 stream.cuda_stream)

            def run_both():
                B.pdfx_eval_lumi(pdf.handle, None, code, pa, pb, None, x1.data_ptr(),
                                 x2.data_ptr(), None, 172.5 ** 2, nl, L.data_ptr(), S.data_ptr(),
                                 0, stream.cuda_stream)
            tune = {}
            for shape in ((512, 1), (512, 2), (256, 2)) + (((512, 4),) if prec == "f32s" else ()):
                pdf.set_lumi_launch(prec, *shape)
                tune[shape] = timed(run_sum, 3)
            best = min(tune, key=tune.get)
            pdf.set_lumi_launch(prec, *best)
            ms_s = timed(run_sum, 5)
            ms_b = timed(run_both, 5)
            vb = 8 if prec == "f64" else 4
            lres[prec] = {"sum_ms": ms_s, "sum_points_per_s": nl / (ms_s * 1e-3),
                          "sum_hbm_gbs_algorithmic": nl * (16 + vb) / ms_s / 1e6,
                          "sum_hbm_frac": nl * (16 + vb) / ms_s / 1e6 / HBM_PEAK_GBS,
                          "pairs_and_sum_ms": ms_b,
                          "pairs_and_sum_hbm_gbs_algorithmic": nl * (16 + 5 * vb) / ms_b / 1e6,
                          "pairs_and_sum_hbm_frac": nl * (16 + 5 * vb) / ms_b / 1e6 / HBM_PEAK_GBS,
                          "launch_shape": list(best),
                          "shape_sum_ms": {"%dx%d" % k: v for k, v in tune.items()}}
            log("lumi %s: sum %.3f ms, pairs+sum %.3f ms" % (prec, ms_s, ms_b))
            del S, L
        variants["lumi"] = {"n_points": nl, "pairs": [list(t) for t in zip(pa, pb)],
                            "q2": 172.5 ** 2, **lres}
        if args.only == "lumi":
            print(json.dumps({"only": "lumi", **variants["lumi"]}))
            return

    head = results[args.prec]
    value = n * nf / (head["ms"] * 1e-3)
    bytes_per_pt = 16 + (nf + 1) * (8 if args.prec == "f64" else 4)   # x, Q^2 in; x f, alpha_s out
    achieved = n * bytes_per_pt / (head["xfx_ms"] * 1e-3) / 1e9

    # CPU baseline: the oracle on the host cores over the workload's points
    # (median of 3), one thread on a 1e5-point sample, and stated samples of the
    # members and integrand workloads; the GPU error on the first 1e6 points
    cpu = None
    err = {}
    if not args.no_cpu:
        import oracle
        nc = n
        threads = oracle.default_threads()
        log("oracle on %d points, %d threads" % (nc, threads))
        walls = []
        for _ in range(3):
            t0 = time.perf_counter()
            ora = oracle.xfx(grid, pids, x_np[:nc], q2_np[:nc], nthreads=threads)
            ora_as = oracle.alphas(grid.as_q2, grid.as_val, q2_np[:nc], nthreads=threads)
            walls.append(time.perf_counter() - t0)
        dt = sorted(walls)[1]
        n1 = min(nc, 100_000)
        t0 = time.perf_counter()
        oracle.xfx(grid, pids, x_np[:n1], q2_np[:n1], nthreads=1)
        dt1 = time.perf_counter() - t0
        cpu = {"value": nc * nf / dt, "unit": "pf/s", "cores": threads, "kind": "oracle",
               "sample": "all %d points x %d flavours and alpha_s of the step, FP64, median "
                         "of 3: %.2f s wall" % (nc, nf, dt),
               "cpu_model": cpu_model(),
               "one_thread": {"value": n1 * nf / dt1, "unit": "pf/s",
                              "sample": "first %d points, FP64" % n1}}
        if not args.no_extra:
            members = wl.member_grids(101)
            xs, qs = wl.queries(2, 100_000)
            t0 = time.perf_counter()
            for m in members:
                oracle.xfx(m, m.pids, xs, qs, nthreads=threads)
            dtm = time.perf_counter() - t0
            cpu["members"] = {"value": 101 * xs.size * nf / dtm, "unit": "pf/s",
                              "sample": "101 members x 1e5 points x 11 flavours, FP64"}
            u1, u2 = wl.dy_uniforms(0, 10_000_000)
            t0 = time.perf_counter()
            oracle.dy(grid, u1, u2, wl.DY_XMIN, wl.SQRT_S_DY ** 2, nthreads=threads)
            dtd = time.perf_counter() - t0
            cpu["drell_yan"] = {"value": u1.size / dtd, "unit": "points/s",
                                "sample": "one 1e7-point chunk (seed of chunk 0), FP64 forward"}
            log("oracle: members %.2f s, integrand chunk %.2f s" % (dtm, dtd))
        ns = min(nc, 1_000_000)
        M = oracle.stencil_absmax(grid, pids, x_np[:ns], q2_np[:ns])
        for prec, r in results.items():
            got = r["out"][:ns].double().cpu().numpy()
            den = np.maximum(np.abs(ora[:ns]), 0.1 * M)
            e = np.abs(got - ora[:ns]) / np.where(den == 0, 1.0, den)
            got_as = r["as"][:ns].double().cpu().numpy()
            err[prec] = {"max_rel_err_capped": float(e.max()),
                         "alphas_max_rel_err": float(np.max(np.abs(got_as - ora_as[:ns])
                                                            / np.abs(ora_as[:ns]))),
                         "per_flavour_max": [float(v) for v in e.max(axis=0)],
                         "points_checked": ns}

    lds_meas = lds_meas_all() if results else {}
    for prec, r in results.items():
        bpp = 16 + (nf + 1) * (8 if prec == "f64" else 4)
        variants[prec] = {
            "value": n * nf / (r["ms"] * 1e-3), "unit": "pf/s", "ms_per_step": r["ms"],
            "xfx_kernel_ms": r["xfx_ms"], "launch_shape": r["launch"],
            "xfx_hbm_gbs_algorithmic": n * bpp / (r["xfx_ms"] * 1e-3) / 1e9,
            "hbm_roofline_pf_s": HBM_PEAK_GBS * 1e9 / bpp * nf,
            **err.get(prec, {})}
        lb = lds_bytes(prec, r["launch"], n, nf, grid.n_x, grid.n_q)
        if lb is not None:
            # LDS ceiling: the rates the device is measured to reach in this
            # run (pdfx_bench_lds), lane-consecutive reads as the peak
            ach = lb / (r["xfx_ms"] * 1e-3) / 1e9
            peak = lds_meas["measured_stream_gbs"]
            variants[prec]["lds"] = {
                "bytes_per_launch": lb, "achieved_gbs": ach, "peak_gbs": peak,
                "peak_kind": "measured, lane-consecutive 16-byte LDS reads", "frac": ach / peak,
                "random_gbs": lds_meas["measured_random_gbs"],
                "frac_of_random": ach / lds_meas["measured_random_gbs"]}

    copy = copy_gbs()[2]
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "pf/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "f64" else "f32 stencil, f64 search",
        "data": "synthetic",
        "config": {"workload": "1e7 points x 11 flavours on an 11x100x50 grid with 3 Q^2 "
                               "subgrids, plus alpha_s at the same points",
                   "n_points": n, "n_flav": nf, "grid": [nf, grid.n_x, grid.n_q],
                   "q_subgrids": [int(v) for v in np.diff(grid.q_off)], "prec": args.prec},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": recorded_traffic(args.prec, head["launch"]),
                     "kernel": forward_kernel_name(args.prec, head["launch"]),
                     "bytes_per_point": bytes_per_pt,
                     "copy_gbs": copy, "frac_of_copy": achieved / copy,
                     "lds": variants.get(args.prec, {}).get("lds")},
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
