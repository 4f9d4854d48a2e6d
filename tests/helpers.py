"""Shared test utilities: device checks, the error metric, workload caches."""
from __future__ import annotations

import functools

import numpy as np

import oracle
from paper_2012_08221_amd import workloads as wl


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def capped_rel_err(got, ora, absmax, cap=0.1):
    """|got - ora| / max(|ora|, cap * M): M = largest |knot| in the point's
    stencil, so values that cross zero inside a cell (the (1 + gamma ln Q^2)
    factor, the x -> 1 fall-off) are judged against the scale of the data
    around them (condition number capped at 1/cap)."""
    got = np.asarray(got, dtype=np.float64)
    ora = np.asarray(ora, dtype=np.float64)
    den = np.maximum(np.abs(ora), cap * np.asarray(absmax, dtype=np.float64))
    den = np.where(den == 0, 1.0, den)
    return np.abs(got - ora) / den


@functools.lru_cache(maxsize=None)
def cfg0_grid(reading="primary"):
    return wl.config0_grid(reading)


@functools.lru_cache(maxsize=None)
def cfg0_queries(n=100_000):
    return wl.queries(0, n)


def oracle_ref(grid, pids, x, q2, mode=0):
    return oracle.xfx(grid, pids, x, q2, mode=mode)


def _axis_weight_sum_bound(lnz, off):
    """Upper bound of sum_j |w_j| over the 4 folded weights of any interval.

    With r- = d_i/d_{i-1}, r+ = d_i/d_{i+1} the weights are
    h00 + h01 (= 1, both >= 0 on [0,1]) plus h10 and h11 times slope terms whose
    absolute sum is at most 2 max(1, r-/2) and 2 max(1, r+/2); |h10|, |h11| <= 4/27.
    """
    worst = 1.0
    for s in range(len(off) - 1):
        a, b = off[s], off[s + 1]
        d = np.diff(lnz[a:b])
        for i in range(len(d)):
            rm = d[i] / d[i - 1] if i > 0 else 0.0
            rp = d[i] / d[i + 1] if i + 1 < len(d) else 0.0
            worst = max(worst, 1.0 + 8.0 / 27.0 * (max(1.0, rm / 2) + max(1.0, rp / 2)))
    return worst


def f32_tolerance(grid, base=1e-5):
    """FP32-stencil tolerance for a grid: the 1e-5 target scaled by how much
    larger the weight condition (product of the per-axis bounds of sum |w|)
    is than on a uniformly spaced grid, where both bounds equal 1 + 16/27."""
    ax = _axis_weight_sum_bound(np.log(grid.x), [0, len(grid.x)])
    aq = _axis_weight_sum_bound(np.log(grid.q2), list(grid.q_off))
    uniform = (1.0 + 16.0 / 27.0) ** 2
    return base * max(1.0, ax * aq / uniform)
