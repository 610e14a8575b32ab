"""The allocation-free entry point (spar_sink_ot_noalloc, through the C ABI)
against spar_sink_ot with a caller workspace: two calls in a row on the same
GPU, the second with a smaller, ragged problem (the static scratch keeps the
first call's contents), must each give the workspace solve's result bit for
bit: same sketch size, iterations, error, estimate and scalings."""
import math

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


def _same(ref, got):
    assert got.status == ref.status
    assert (got.nnz, got.iters, got.empty_rows, got.empty_cols) == \
        (ref.nnz, ref.iters, ref.empty_rows, ref.empty_cols)
    assert got.marginal_err == ref.marginal_err
    assert got.estimate == ref.estimate and got.sparse_objective == ref.sparse_objective
    assert got.cmax == ref.cmax
    assert torch.equal(got.u, ref.u) and torch.equal(got.v, ref.v)


@pytest.mark.parametrize("precision", ["f64", "f32", "f32_log"])
def test_noalloc_matches_workspace_solve_twice(api, precision):
    # first: the 2-D Gaussian workload at n = 1024 (s = 8 n ln n); second: a
    # smaller ragged problem, so stale scratch from the first call would show
    big = W.ot_gauss2d(1024, seed=0)
    small = W.ot_gauss2d(300, seed=1, m=333)
    for p, tol in ((big, 1e-8), (small, 1e-6)):
        prob = api.Problem(p.x, p.y, p.a, p.b)
        kw = dict(eps=p.eps, s=p.s, seed=p.seed, tol=tol, max_iter=500, precision=precision,
                  return_scalings=True)
        ref = api.spar_sink_ot(prob, **kw)
        got = api.spar_sink_ot_noalloc(prob, **kw)
        print(f"{precision} n={p.n} m={p.m}: iters {got.iters}, nnz {got.nnz}, "
              f"estimate {got.estimate:.15f}")
        _same(ref, got)
        assert got.t_iter_ms == 0.0 and got.t_sample_ms == 0.0


def test_noalloc_rejects_problems_beyond_its_scratch(api):
    from paper_2306_06581_amd import native as N
    p = W.ot_gauss2d(8192, seed=2)
    prob = api.Problem(p.x, p.y, p.a, p.b)
    r = api.spar_sink_ot_noalloc(prob, eps=p.eps, s=p.s, seed=p.seed, precision="f64",
                                 raise_on_error=False)
    assert r.status == N.SS_E_WORKSPACE
    assert "spar_sink_ot_noalloc" in N.lib.ss_last_error().decode()
    # the next call on the same GPU still works
    q = W.ot_gauss2d(256, seed=3)
    pq = api.Problem(q.x, q.y, q.a, q.b)
    kw = dict(eps=q.eps, s=q.s, seed=q.seed, tol=1e-6, max_iter=500, precision="f64",
              return_scalings=True)
    _same(api.spar_sink_ot(pq, **kw), api.spar_sink_ot_noalloc(pq, **kw))
