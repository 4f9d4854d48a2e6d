"""Seeded synthetic inputs: grids, members, query points, loss weights, MC draws.

This module only *generates inputs*.  It holds none of the interpolation
arithmetic: no search, no Hermite basis, no slopes, no stencil.  Both the HIP
path and the CPU oracle are fed from here, and neither is imported here.

What is generated, and why it has this shape:

* The paper evaluates an unnamed LHAPDF set member (Sec. 2.1, the ``mkPDF``
  example of Fig. 1).  No set ships with this project, so synthetic grids of the
  same structure stand in for it: about 100 log-spaced x knots over
  [1e-9, 1], 11 partons (d..b antiquarks, gluon, d..b quarks), Q^2 subgrids that
  break at the charm and bottom thresholds, Q up to 1e5 GeV.
* Values are xf = A x^alpha (1-x)^beta (1 + gamma ln Q^2), so the Q^2 dependence
  is linear in ln Q^2 and the x dependence has the usual small-x rise and
  large-x fall.
* alpha_s knot values come from one-loop running with continuous matching at
  the quark thresholds (a value generator only).
* Query points are log-uniform in x and in Q, as Monte Carlo integrands produce
  them (Sec. 3.1).

Seeds: numpy ``default_rng(SeedSequence(201208221 + k))`` for workload k, with
four child streams spawned in the order params, members, queries, weights.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 201208221

# PDG ids in storage order: d..b antiquarks, gluon, d..b quarks.
PIDS_11 = np.array([-5, -4, -3, -2, -1, 21, 1, 2, 3, 4, 5], dtype=np.int32)

# Subgrid edges in GeV.  The primary reading keeps the three subgrids split at
# 1.51 and 4.92 GeV by starting the Q range at 1 GeV; the alternate fixture
# keeps the stated lower edge 1.65 GeV, which leaves only the 4.92 split.
Q_EDGES_PRIMARY = (1.0, 1.51, 4.92, 1.0e5)
Q_EDGES_ALTERNATE = (1.65, 4.92, 1.0e5)
# Thresholds available to many-member grids (the fourth edge is the top mass).
MEMBER_EDGES = {2: (1.0, 4.92, 1.0e5),
                3: (1.0, 1.51, 4.92, 1.0e5),
                4: (1.0, 1.51, 4.92, 172.5, 1.0e5)}

ALPHAS_MZ = 0.118
MZ = 91.1876
M_CHARM = 1.51
M_BOTTOM = 4.92

SQRT_S_DY = 13000.0
DY_XMIN = 1.0e-5


def _streams(k: int):
    ss = np.random.SeedSequence(SEED_BASE + k)
    kids = ss.spawn(4)
    return {name: np.random.default_rng(kid)
            for name, kid in zip(("params", "members", "queries", "weights"), kids)}


def _uniform(rng, lo, hi, n):
    return lo + (hi - lo) * rng.random(n)


@dataclass
class GridSpec:
    """One PDF member: knots, subgrid offsets, values, alpha_s knots (all FP64).

    ``xf`` is [n_flav][n_x][n_q] with Q innermost; ``q2`` concatenates the
    subgrids, the boundary knot appearing once at the end of the lower subgrid
    and once at the start of the upper one.
    """
    pids: np.ndarray
    x: np.ndarray
    q2: np.ndarray
    q_off: np.ndarray
    xf: np.ndarray
    as_q2: np.ndarray = field(default_factory=lambda: np.zeros(0))
    as_val: np.ndarray = field(default_factory=lambda: np.zeros(0))

    @property
    def n_flav(self):
        return int(self.xf.shape[0])

    @property
    def n_x(self):
        return int(self.x.shape[0])

    @property
    def n_q(self):
        return int(self.q2.shape[0])

    @property
    def n_sub(self):
        return int(self.q_off.shape[0] - 1)


def allocate_knots(n_q_total: int, edges_q) -> list[int]:
    """Knots per subgrid: S subgrids share n_q_total - S intervals.

    Every subgrid but the longest (in ln Q^2) gets max(3, round(share)) intervals
    where share is proportional to its ln Q^2 length; the longest takes the
    remainder.  Knot count = intervals + 1.
    """
    edges = np.asarray(edges_q, dtype=np.float64)
    lengths = 2.0 * np.log(edges[1:] / edges[:-1])
    n_sub = len(lengths)
    intervals = n_q_total - n_sub
    longest = int(np.argmax(lengths))
    alloc = [0] * n_sub
    for s in range(n_sub):
        if s != longest:
            alloc[s] = max(3, int(round(intervals * lengths[s] / lengths.sum())))
    alloc[longest] = intervals - sum(alloc)
    if alloc[longest] < 3:
        raise ValueError("too few knots for the subgrid layout")
    return [a + 1 for a in alloc]


def x_knots(n_x: int) -> np.ndarray:
    """n_x knots log-spaced over [1e-9, 1]: x_i = 10^(-9 + 9 i/(n_x-1))."""
    i = np.arange(n_x, dtype=np.float64)
    return 10.0 ** (-9.0 + 9.0 * i / (n_x - 1))


def q2_knots(edges_q, counts) -> tuple[np.ndarray, np.ndarray]:
    """Concatenated Q^2 knots, log-spaced in Q^2 inside each subgrid.

    Subgrid ends are set to the exact edge value Q*Q so that the two copies of a
    boundary knot are bitwise equal.
    """
    parts = []
    for s, n_s in enumerate(counts):
        lo = edges_q[s] * edges_q[s]
        hi = edges_q[s + 1] * edges_q[s + 1]
        k = np.arange(n_s, dtype=np.float64)
        part = np.exp(np.log(lo) + (np.log(hi) - np.log(lo)) * k / (n_s - 1))
        part[0] = lo
        part[-1] = hi
        parts.append(part)
    q_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    return np.concatenate(parts), q_off


def draw_params(rng, n_flav: int = 11) -> np.ndarray:
    """Per-flavour (A, alpha, beta, gamma); draws in the order alpha, beta, gamma, A."""
    alpha = _uniform(rng, -0.3, 0.8, n_flav)
    beta = _uniform(rng, 2.0, 6.0, n_flav)
    gamma = _uniform(rng, -0.1, 0.1, n_flav)
    amp = _uniform(rng, 0.5, 2.0, n_flav)
    return np.stack([amp, alpha, beta, gamma], axis=1)


def grid_values(params: np.ndarray, x: np.ndarray, q2: np.ndarray) -> np.ndarray:
    """xf[f][i][k] = A_f x_i^alpha_f (1-x_i)^beta_f (1 + gamma_f ln q2_k)."""
    amp, alpha, beta, gamma = (params[:, j][:, None] for j in range(4))
    xs = amp * x[None, :] ** alpha * (1.0 - x[None, :]) ** beta        # [f][i]
    qs = 1.0 + gamma * np.log(q2)[None, :]                              # [f][k]
    return np.ascontiguousarray(xs[:, :, None] * qs[:, None, :])


def alphas_values(q2: np.ndarray) -> np.ndarray:
    """One-loop alpha_s at the knots, alpha_s(MZ) = 0.118, nf = 5/4/3 with
    continuity at the bottom and charm masses; a knot sitting exactly on a
    threshold gets the same value from both sides."""
    def b0(nf):
        return (33.0 - 2.0 * nf) / (12.0 * math.pi)
    inv_b = 1.0 / ALPHAS_MZ + b0(5) * math.log(M_BOTTOM ** 2 / MZ ** 2)
    inv_c = inv_b + b0(4) * math.log(M_CHARM ** 2 / M_BOTTOM ** 2)
    out = np.empty_like(q2)
    for j, v in enumerate(q2):
        if v >= M_BOTTOM ** 2:
            inv = 1.0 / ALPHAS_MZ + b0(5) * math.log(v / MZ ** 2)
        elif v >= M_CHARM ** 2:
            inv = inv_b + b0(4) * math.log(v / M_BOTTOM ** 2)
        else:
            inv = inv_c + b0(3) * math.log(v / M_CHARM ** 2)
        out[j] = 1.0 / inv
    return out


def make_grid(params, n_x, edges_q, n_q_total, pids=PIDS_11, with_alphas=True) -> GridSpec:
    x = x_knots(n_x)
    counts = allocate_knots(n_q_total, edges_q)
    q2, q_off = q2_knots(edges_q, counts)
    xf = grid_values(params, x, q2)
    g = GridSpec(pids=np.asarray(pids, dtype=np.int32), x=x, q2=q2, q_off=q_off, xf=xf)
    if with_alphas:
        g.as_q2 = q2.copy()
        g.as_val = alphas_values(q2)
    return g


def config0_grid(reading: str = "primary") -> GridSpec:
    """Single member: 11 flavours, 100 x knots, 50 Q^2 knots in 3 subgrids."""
    params = draw_params(_streams(0)["params"])
    edges = Q_EDGES_PRIMARY if reading == "primary" else Q_EDGES_ALTERNATE
    return make_grid(params, 100, edges, 50)


def config0_params() -> np.ndarray:
    return draw_params(_streams(0)["params"])


def queries(k: int, n: int, xlo=1e-6, xhi=0.99, qlo=2.0, qhi=1e4):
    """n points, x log-uniform in [xlo, xhi], Q log-uniform in [qlo, qhi]; returns (x, q2=Q*Q)."""
    rng = _streams(k)["queries"]
    x = np.exp(math.log(xlo) + (math.log(xhi) - math.log(xlo)) * rng.random(n))
    q = np.exp(math.log(qlo) + (math.log(qhi) - math.log(qlo)) * rng.random(n))
    return x, q * q


def member_grids(n_mem: int = 101, k: int = 2) -> list[GridSpec]:
    """Replica-style members with uneven grids.

    Member 0 has the central parameters; members 1.. multiply every (A, alpha,
    beta, gamma) by (1 + 0.05 eps), eps ~ N(0,1).  Geometry per member: n_x in
    [50, 200], 2..4 subgrids, 20..80 Q^2 knots in total.
    """
    st = _streams(k)
    central = draw_params(st["params"])
    rng = st["members"]
    grids = []
    for m in range(n_mem):
        n_x = int(rng.integers(50, 201))
        n_sub = int(rng.integers(2, 5))
        n_q = int(rng.integers(20, 81))
        if m == 0:
            params = central.copy()
        else:
            params = central * (1.0 + 0.05 * rng.standard_normal(central.shape))
        grids.append(make_grid(params, n_x, MEMBER_EDGES[n_sub], n_q, with_alphas=False))
    return grids


def loss_weights(k: int, n: int, n_flav: int = 11) -> np.ndarray:
    """w[i][a] ~ N(0,1) for the loss sum_i sum_a w[i][a] xf_a(x_i, Q_i)."""
    return _streams(k)["weights"].standard_normal((n, n_flav))


def dy_uniforms(chunk: int, n: int):
    """(u1, u2) in [0,1) for one Drell-Yan chunk, from the queries stream of
    seed 201208225 + chunk (numpy; the GPU benchmark draws its own on the device)."""
    rng = _streams(4 + chunk)["queries"]
    return rng.random(n), rng.random(n)


# DY pids: quark q at x1 paired with antiquark -q at x2, q = 1..5.
DY_QUARKS = np.array([1, 2, 3, 4, 5], dtype=np.int32)


def threshold_jump_grid(n_x: int, n_sub: int, n_q_total: int, k: int = 30,
                        jump: float = 0.25) -> GridSpec:
    """A member whose two copies of each boundary Q^2 knot hold different values,
    as when a parton switches on at its threshold: the generated values with the
    upper copy of every boundary row raised by jump * (1 + |value|), and the
    upper copy of every repeated alpha_s knot raised by 5%.  Thresholds as for
    many-member grids (MEMBER_EDGES[n_sub])."""
    params = draw_params(_streams(k)["params"])
    g = make_grid(params, n_x, MEMBER_EDGES[n_sub], n_q_total)
    for s in range(1, g.n_sub):
        kk = int(g.q_off[s])
        g.xf[:, :, kk] += jump * (1.0 + np.abs(g.xf[:, :, kk]))
        g.as_val[kk] *= 1.05
    return g


def threshold_points(g: GridSpec, k: int, n_random: int, n_x_per_threshold: int):
    """Query points for the threshold tie rule: n_random points log-uniform over
    the grid, then for every threshold Q^2 (exactly, one ulp below and one ulp
    above) the x knots and n_x_per_threshold log-uniform x.  Returns (x, q2)."""
    rng = _streams(k)["queries"]
    lx0, lx1 = math.log(g.x[0]), math.log(g.x[-1])
    lq0, lq1 = math.log(g.q2[0]), math.log(g.q2[-1])
    xs = [np.exp(lx0 + (lx1 - lx0) * rng.random(n_random))]
    qs = [np.exp(lq0 + (lq1 - lq0) * rng.random(n_random))]
    for s in range(1, g.n_sub):
        thr = g.q2[g.q_off[s]]
        xt = np.r_[g.x, np.exp(lx0 + (lx1 - lx0) * rng.random(n_x_per_threshold))]
        for qv in (thr, np.nextafter(thr, 0.0), np.nextafter(thr, np.inf)):
            xs.append(xt)
            qs.append(np.full(xt.shape, qv))
    return np.concatenate(xs), np.concatenate(qs)
