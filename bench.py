#!/usr/bin/env python3
"""Benchmark of the batched PDF evaluation hot path on one MI355X.

One step = one pass of the whole forward path over one batch: x f for all 11
partons at 1e7 query points (log-uniform x in [1e-6, 0.99], Q in [2, 1e4] GeV)
on the 11 x 100 x 50 three-subgrid member grid, plus alpha_s at the same
points.  Inputs are resident in HBM before the timed region.

Prints one JSON line.  `value` is points x flavours per second of the chosen
precision (--prec f64 | f32s); the other precision, the backward pass
(points x flavours per second of forward + backward on 1e6 points), the error
against the oracle and the roofline of the dominant kernel ride along.
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
    ap.add_argument("--no-extra", action="store_true", help="only the headline precision")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a plain copy kernel of known size (for counter scaling) and exit")
    ap.add_argument("--only", default=None, choices=[None, "xfx"],
                    help="time only the xfx kernel (for profiler runs)")
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def time_steps(torch, fn_step, steps, warmup, stream):
    """W untimed steps, then exactly K timed steps bracketed by synchronize."""
    for _ in range(warmup):
        fn_step(None)
    torch.cuda.synchronize()
    ev = []
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn_step(ev)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(end)
    return total_ms / steps, wall, ev


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2012_08221_amd import api
    from paper_2012_08221_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    if args.calib_copy:
        n = 1 << 27                                   # 1 GiB of FP64 in, 1 GiB out
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes_read": n * 8, "calib_copy_bytes_written": n * 8,
                          "launches": 5}))
        return

    grid = wl.config0_grid()
    pdf = api.mkPDF(grid)
    n = args.n
    log("generating %d query points" % n)
    x_np, q2_np = wl.queries(1, n)
    x = torch.as_tensor(x_np, device=dev)
    q2 = torch.as_tensor(q2_np, device=dev)
    pids = grid.pids
    nf = len(pids)
    torch.cuda.synchronize()

    def bench_prec(prec, with_alphas=True):
        dt = api.prec_dtype(prec)
        out = torch.empty((n, nf), dtype=dt, device=dev)
        aout = torch.empty(n, dtype=dt, device=dev)

        def step(ev):
            if ev is not None:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            pdf.xfxQ2(pids, x, q2, prec=prec, out=out)
            if ev is not None:
                e1.record(stream)
                ev.append((e0, e1))
            if with_alphas:
                pdf.alphasQ2(q2, prec=prec, out=aout)

        ms, wall, ev = time_steps(torch, step, args.steps, args.warmup, stream)
        k_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        return {"ms_per_step": ms, "wall_s": wall, "xfx_ms": k_ms, "out": out, "aout": aout}

    results = {}
    precs = [args.prec] + ([] if args.no_extra else [p for p in ("f64", "f32s") if p != args.prec])
    for prec in precs:
        log("timing %s" % prec)
        results[prec] = bench_prec(prec, with_alphas=args.only != "xfx")
    if args.only == "xfx":
        r = results[args.prec]
        print(json.dumps({"only": "xfx", "prec": args.prec, "xfx_ms": r["xfx_ms"]}))
        return

    # Backward (loss = sum w * xf) on 1e6 points, FP32 grid as a tensor, if built.
    fwd_bwd = None
    try:
        from paper_2012_08221_amd import autograd as ag
        nb = 1_000_000
        vals = torch.as_tensor(grid.xf, device=dev).to(torch.float32).requires_grad_(True)
        xb, qb = x[:nb].clone(), q2[:nb].clone()
        w = torch.as_tensor(wl.loss_weights(3, nb), device=dev).to(torch.float32)

        def fb(ev):
            vals.grad = None
            y = ag.xfx(pdf, vals, pids, xb, qb)
            (y * w).sum().backward()
        ms_fb, _, _ = time_steps(torch, fb, max(5, args.steps // 5), 2, stream)
        fwd_bwd = {"value": nb * nf / (ms_fb * 1e-3), "unit": "pf/s", "n_points": nb,
                   "ms_per_step": ms_fb, "dtype": "f32s",
                   "what": "forward + backward (grad wrt 11x100x50 knots) of sum w*xf"}
    except (ImportError, AttributeError) as e:
        log("backward not timed: %s" % e)
    except Exception as e:  # noqa: BLE001
        log("backward not timed: %s: %s" % (type(e).__name__, e))

    head = results[args.prec]
    value = n * nf / (head["ms_per_step"] * 1e-3)
    bytes_per_pt = 16 + nf * (8 if args.prec == "f64" else 4)
    traffic_alg = n * bytes_per_pt
    achieved = traffic_alg / (head["xfx_ms"] * 1e-3) / 1e9

    # CPU baseline: the oracle on the host cores, on a bounded prefix of the workload.
    cpu = None
    err = {}
    if not args.no_cpu:
        import oracle
        nc = min(n, 10_000_000)
        threads = oracle.default_threads()
        log("oracle on %d points, %d threads" % (nc, threads))
        t0 = time.perf_counter()
        ora = oracle.xfx(grid, pids, x_np[:nc], q2_np[:nc], nthreads=threads)
        dt = time.perf_counter() - t0
        cpu = {"value": nc * nf / dt, "unit": "pf/s", "cores": threads, "kind": "oracle",
               "sample": "first %d of the %d points x %d flavours, FP64, %.1f s wall"
                         % (nc, n, nf, dt)}
        ns = min(nc, 1_000_000)
        M = oracle.stencil_absmax(grid, pids, x_np[:ns], q2_np[:ns])
        for prec, r in results.items():
            got = r["out"][:ns].double().cpu().numpy()
            den = np.maximum(np.abs(ora[:ns]), 0.1 * M)
            e = np.abs(got - ora[:ns]) / np.where(den == 0, 1.0, den)
            err[prec] = {"max_rel_err_capped": float(e.max()),
                         "per_flavour_max": [float(v) for v in e.max(axis=0)],
                         "points_checked": ns}

    variants = {}
    for prec, r in results.items():
        bpp = 16 + nf * (8 if prec == "f64" else 4)
        variants[prec] = {
            "value": n * nf / (r["ms_per_step"] * 1e-3), "unit": "pf/s",
            "ms_per_step": r["ms_per_step"], "xfx_kernel_ms": r["xfx_ms"],
            "xfx_hbm_gbs_algorithmic": n * bpp / (r["xfx_ms"] * 1e-3) / 1e9,
            "hbm_roofline_pf_s": HBM_PEAK_GBS * 1e9 / bpp * nf,
            **err.get(prec, {})}
    if fwd_bwd:
        variants["fwd_bwd"] = fwd_bwd

    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "pf/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
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
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "xfx_kernel<%s>" % ("double" if args.prec == "f64" else "float"),
                     "bytes_per_point": bytes_per_pt},
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
