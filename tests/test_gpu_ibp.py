"""Parity of Spar-IBP (the barycenter section's Alg. Spar-IBP) between the HIP
path, through the C ABI, and the CPU FP64 oracle.

Bars as for Spar-Sink: each measure's mask, CSR and CSC bit for bit; FP64
barycenter and scalings within 1e-10 relative after a fixed number of steps;
FP32 stored values give the barycenter within 1e-4 (L1, relative to its
mass)."""
import math

import numpy as np
import pytest
import torch

from oracle import ibp_oracle as I
from paper_2306_06581_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_06581_amd import api as A
    return A


def _mask_np(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("n,d,shrink", [(700, 5, 0.0), (333, 3, 0.5), (64, 2, 1.0), (1, 2, 0.0)])
def test_ibp_sample_bit_exact(api, n, d, shrink):
    p = W.ibp_synthetic(n, d=d, seed=11, eps=0.05)
    if n == 1:
        p.s = 1.0       # s0(1) = 0
    prob = api.IBPProblem(p.x, p.b, p.w)
    for k in range(p.count):
        sk = I.ibp_sketch(p.x, p.b[k], k, p.eps, p.s, seed=p.seed, shrink=shrink)
        g = api.ss_ibp_sample(prob, k, eps=p.eps, s=p.s, seed=p.seed, shrink=shrink)
        assert g["nnz"] == sk.nnz
        assert np.array_equal(_mask_np(g["mask"]), sk.mask)
        for key in ("row_ptr", "col_idx", "col_ptr", "row_idx"):
            assert np.array_equal(g[key].cpu().numpy(), getattr(sk, key)), (k, key)
        assert np.array_equal(g["row_fac"].cpu().numpy(), sk.prob.alpha)
        assert np.array_equal(g["col_fac"].cpu().numpy(), sk.prob.rb)
        assert g["cmax"] == sk.cmax
        assert np.array_equal(g["val"].cpu().numpy(), sk.val)
        assert np.array_equal(g["val_t"].cpu().numpy(), sk.val_t)


def _run(api, p, **kw):
    return api.spar_ibp(api.IBPProblem(p.x, p.b, p.w), eps=p.eps, s=p.s, seed=p.seed, **kw)


@pytest.mark.parametrize("n,d", [(600, 5), (257, 10)])
def test_spar_ibp_f64_fixed_steps(api, n, d):
    p = W.ibp_synthetic(n, d=d, seed=12, eps=0.05)
    T = 30
    o = I.spar_ibp(p.x, p.b, p.w, p.eps, p.s, seed=p.seed, tol=0.0, max_iter=T)
    r = _run(api, p, tol=0.0, max_iter=T, return_scalings=True, return_hist=True)
    assert r.status == 1 and r.iters == T == o.ibp.iters
    assert r.nnz == o.nnz
    np.testing.assert_allclose(r.q.cpu().numpy(), o.ibp.q, rtol=1e-10, atol=0)
    for k in range(p.count):
        np.testing.assert_allclose(r.u[k].cpu().numpy(), o.ibp.u[k], rtol=1e-10, atol=0)
        np.testing.assert_allclose(r.v[k].cpu().numpy(), o.ibp.v[k], rtol=1e-10, atol=0)
    # late errors are differences of nearly equal barycenters: absolute bar
    np.testing.assert_allclose(r.err_hist.cpu().numpy(), np.array(o.ibp.hist), rtol=1e-7,
                               atol=1e-13)
    assert r.err == pytest.approx(o.ibp.err, rel=1e-7, abs=1e-13)


def test_spar_ibp_f64_to_tolerance(api):
    p = W.ibp_synthetic(1000, d=5, seed=0, eps=0.05)
    o = I.spar_ibp(p.x, p.b, p.w, p.eps, p.s, seed=p.seed, tol=1e-9, max_iter=5000)
    r = _run(api, p, tol=1e-9, max_iter=5000)
    assert r.status == 0 and r.err <= 1e-9
    assert abs(r.iters - o.ibp.iters) <= 1
    assert np.abs(r.q.cpu().numpy() - o.ibp.q).sum() < 1e-8


def test_spar_ibp_f32_values(api):
    p = W.ibp_synthetic(800, d=5, seed=13, eps=0.05)
    o = I.spar_ibp(p.x, p.b, p.w, p.eps, p.s, seed=p.seed, tol=1e-8, max_iter=5000)
    r = _run(api, p, tol=1e-8, max_iter=5000, precision="f32")
    assert r.status == 0
    assert np.abs(r.q.cpu().numpy() - o.ibp.q).sum() < 1e-4 * o.ibp.q.sum()


@pytest.mark.parametrize("count,shrink", [(1, 0.0), (5, 0.0), (3, 1.0)])
def test_spar_ibp_measure_counts_and_rand_ibp(api, count, shrink):
    base = W.ibp_synthetic(300, d=3, seed=14, eps=0.05)
    rng = np.random.default_rng(15)
    b = np.stack([base.b[k % 3] for k in range(count)])
    if count > 3:
        b[3:] = rng.dirichlet(np.ones(base.n), size=count - 3) * 0.5 + b[3:] * 0.5
    w = rng.dirichlet(np.ones(count)) if count > 1 else np.ones(1)
    T = 25
    # one measure reaches its fixed point within two steps (the oracle's err
    # is then exactly 0, the kernel's a rounding of q = exp(log g)): a tolerance
    # far below every other case's err stops both at the same step
    tol = 1e-14
    o = I.spar_ibp(base.x, b, w, base.eps, base.s, seed=3, tol=tol, max_iter=T, shrink=shrink)
    r = api.spar_ibp(api.IBPProblem(base.x, b, w), eps=base.eps, s=base.s, seed=3, tol=tol,
                     max_iter=T, shrink=shrink)
    assert r.iters == o.ibp.iters and r.nnz == o.nnz
    assert r.iters == T or count == 1
    np.testing.assert_allclose(r.q.cpu().numpy(), o.ibp.q, rtol=1e-10, atol=0)


def test_plain_launches_match_the_graph_and_repeat(api):
    p = W.ibp_synthetic(500, d=5, seed=16, eps=0.05)
    a = _run(api, p, tol=1e-7, max_iter=400)
    b = _run(api, p, tol=1e-7, max_iter=400, graph_iters=-1)
    c = _run(api, p, tol=1e-7, max_iter=400, graph_iters=3)
    d = _run(api, p, tol=1e-7, max_iter=400)
    assert a.iters == b.iters == c.iters == d.iters
    for other in (b, c, d):
        assert torch.equal(a.q, other.q)


def test_max_iter_one(api):
    p = W.ibp_synthetic(200, d=2, seed=17, eps=0.1)
    o = I.spar_ibp(p.x, p.b, p.w, p.eps, p.s, seed=p.seed, tol=0.0, max_iter=1)
    r = _run(api, p, tol=0.0, max_iter=1)
    assert r.iters == 1 and r.status == 1
    np.testing.assert_allclose(r.q.cpu().numpy(), o.ibp.q, rtol=1e-12, atol=0)
    assert r.err == pytest.approx(o.ibp.err, rel=1e-12)


def test_bad_inputs_rejected(api):
    from paper_2306_06581_amd import native as N
    p = W.ibp_synthetic(50, d=2, seed=18, eps=0.1)
    bneg = p.b.copy()
    bneg[1, 3] = -1e-3
    with pytest.raises(N.SparSinkError) as e:
        api.spar_ibp(api.IBPProblem(p.x, bneg, p.w), eps=p.eps, s=p.s)
    assert e.value.code == -1
    xnan = p.x.copy()
    xnan[2, 0] = math.nan
    with pytest.raises(N.SparSinkError) as e:
        api.spar_ibp(api.IBPProblem(xnan, p.b, p.w), eps=p.eps, s=p.s)
    assert e.value.code == -1
