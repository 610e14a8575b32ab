"""Solves reuse the host thread's capture stream and update the previous
solve's executable graph in place when the new graph has the same shape.
Problems of one shape solved alternately (so every solve after the first
updates an executable captured for another problem's buffers), with solves
of other shapes and graph lengths in between (which replace it), must give
bit for bit the results of their first solve, in every precision; the batched
solver's graphs likewise."""
import numpy as np
import pytest
import torch

from paper_2306_06581_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_06581_amd import api as A
    return A


def _solve(api, p, precision, graph_iters=0):
    prob = api.Problem(p.x, p.y, p.a, p.b, problem_index=p.problem_index)
    r = api.spar_sink_ot(prob, eps=p.eps, s=p.s, seed=p.seed, tol=1e-9, max_iter=400,
                         precision=precision, graph_iters=graph_iters, return_scalings=True)
    return r.iters, r.estimate, r.u.cpu().numpy(), r.v.cpu().numpy()


def _same(a, b):
    assert a[0] == b[0] and a[1] == b[1]
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


@pytest.mark.parametrize("precision", ["f64", "f32", "f32_log"])
def test_alternating_solves_are_bit_identical(api, precision):
    pa = W.ot_gauss2d(700, seed=1, m=650)
    pb = W.ot_gauss2d(700, seed=2, m=650)
    pc = W.ot_gauss2d(300, seed=3, m=333)
    first_a = _solve(api, pa, precision)
    first_b = _solve(api, pb, precision)
    for _ in range(2):
        _same(_solve(api, pa, precision), first_a)
        _same(_solve(api, pb, precision), first_b)
    # another shape, then another graph length, then the first shape again
    first_c = _solve(api, pc, precision)
    _same(_solve(api, pa, precision, graph_iters=6), first_a)
    _same(_solve(api, pa, precision), first_a)
    _same(_solve(api, pc, precision), first_c)


def test_batched_graphs_reused(api):
    rng = np.random.default_rng(5)
    probs = []
    for k in range(6):
        n, m = int(rng.integers(40, 300)), int(rng.integers(40, 300))
        x, y = rng.standard_normal((n, 3)), rng.standard_normal((m, 3)) + 0.5
        a, b = rng.dirichlet(np.ones(n)), rng.dirichlet(np.ones(m))
        probs.append(W.Problem(x, y, a, b, eps=0.05, s=W.s_budget(max(n, m), 8.0), seed=5,
                               problem_index=k))
    B1 = api.Batch.from_problems(probs[:3])
    B2 = api.Batch.from_problems(probs[3:])
    kw = dict(eps=0.05, tol=1e-7, max_iter=500, seed=5, precision="f64")
    r1 = api.spar_sink_batched(B1, **kw)[1]
    r2 = api.spar_sink_batched(B2, **kw)[1]
    for _ in range(2):
        for B, ref in ((B1, r1), (B2, r2)):
            out = api.spar_sink_batched(B, **kw)[1]
            for x, y in zip(out, ref):
                assert (x.iters, x.estimate, x.nnz) == (y.iters, y.estimate, y.nnz)
