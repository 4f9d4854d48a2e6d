"""The eval calls inside a captured HIP graph (torch.cuda.CUDAGraph): forward
x f in both precisions, alpha_s, x f and alpha_s in one pass, the continuation
mode, the luminosity, a set of members and the integrand forward.  The graph is replayed several times,
with new inputs copied in and eager work and synchronisations between the
replays; every replay must give the eager result's bits."""
import numpy as np
import pytest

from paper_2012_08221_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def test_eval_calls_replay_in_a_graph(torch):
    from paper_2012_08221_amd import api
    g = wl.config0_grid()
    pdf = api.mkPDF(g)
    members = wl.member_grids(6)
    pset = api.PDFSet(members)
    pids = list(g.pids)
    n = 40_000
    dev = "cuda"
    x = torch.empty(n, dtype=torch.float64, device=dev)
    q2 = torch.empty(n, dtype=torch.float64, device=dev)
    u1 = torch.empty(n, dtype=torch.float64, device=dev)
    u2 = torch.empty(n, dtype=torch.float64, device=dev)
    o64 = torch.empty((n, 11), dtype=torch.float64, device=dev)
    o32 = torch.empty((n, 11), dtype=torch.float32, device=dev)
    oex = torch.empty((n, 11), dtype=torch.float64, device=dev)
    oas = torch.empty(n, dtype=torch.float64, device=dev)
    o1 = torch.empty((n, 11), dtype=torch.float64, device=dev)
    o1as = torch.empty(n, dtype=torch.float64, device=dev)
    oset = torch.empty((6, n, 3), dtype=torch.float64, device=dev)

    def inputs(k):
        xs, qs = wl.queries(20 + k, n)
        xs[::50] = 1e-11                       # a few points below the grid
        a, b = wl.dy_uniforms(k, n)
        x.copy_(torch.as_tensor(xs))
        q2.copy_(torch.as_tensor(qs))
        u1.copy_(torch.as_tensor(a))
        u2.copy_(torch.as_tensor(b))

    def work():
        pdf.xfxQ2(pids, x, q2, out=o64)
        pdf.xfxQ2(pids, x, q2, prec="f32s", out=o32)
        pdf.xfxQ2(pids, x, q2, out=oex, domain="extrapolate")
        pdf.alphasQ2(q2, out=oas)
        pdf.xfx_alphasQ2(pids, x, q2, out=o1, as_out=o1as)
        pset.xfxQ2([21, 1, -2], x, q2, out=oset)
        L, S = pdf.lumi([5, 5], [2, -1], x, torch.flip(x, [0]), q2=q2)
        I, _ = api.dy_integrand(pdf, u1, u2, wl.DY_XMIN, wl.SQRT_S_DY ** 2)
        return L, S, I

    def snapshot(L, S, I):
        return [t.cpu().numpy().copy() for t in (o64, o32, oex, oas, o1, o1as, oset, L, S, I)]

    inputs(0)
    work()                                     # warm-up outside the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        Lg, Sg, Ig = work()
    for k in range(1, 4):
        inputs(k)
        want = snapshot(*work())               # eager, same inputs
        torch.cuda.synchronize()
        for t in (o64, o32, oex, oas, o1, o1as, oset, Lg, Sg, Ig):
            t.fill_(np.nan)
        graph.replay()
        torch.cuda.synchronize()
        got = snapshot(Lg, Sg, Ig)
        for a, b in zip(got, want):
            np.testing.assert_array_equal(a, b)
        assert np.isfinite(got[2]).all()       # the continuation rewrote the outside rows
        np.testing.assert_array_equal(got[4], got[0])   # one-pass x f = x f alone
