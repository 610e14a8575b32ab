"""Parity of the Sinkhorn divergence (eq. (sink-div)) and its envelope
gradients between the HIP path, through the C ABI, and the CPU FP64 oracle:
FP64 values and gradients within 1e-10 relative after a fixed number of
iterations; the log-domain FP32 path within 1e-4 (value) and 1e-3 (relative
L2 of the gradients)."""
import numpy as np
import pytest
import torch

from oracle import divergence_oracle as D
from oracle import sparsink_oracle as O
from paper_2306_06581_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_06581_amd import api as A
    return A


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("n,m,d", [(300, 257, 10), (200, 200, 3)])
def test_divergence_f64_fixed_iterations(api, n, m, d):
    p = W.latent_pair(max(n, m), d=d, seed=31, eps=2.0)
    x, y = p.x[:n], p.y[:m]
    a, b = np.full(n, 1.0 / n), np.full(m, 1.0 / m)
    T = 30
    opt = O.Options(eps=p.eps, s=p.s, seed=p.seed, cost="plain", tol=0.0, max_iter=T)
    o = D.sinkhorn_divergence(x, a, y, b, opt)
    r = api.sinkhorn_divergence(api.Problem(x, y, a, b), eps=p.eps, s=p.s, seed=p.seed, tol=0.0,
                                max_iter=T)
    assert r.iters_xy == r.iters_xx == r.iters_yy == T
    assert r.nnz == o.xy.nnz + o.xx.nnz + o.yy.nnz
    for got, ref in ((r.ot_xy, o.xy), (r.ot_xx, o.xx), (r.ot_yy, o.yy)):
        assert _rel(got, ref.estimate.estimate) < 1e-10
    assert _rel(r.value, o.value) < 1e-9
    assert _rel(r.value_sparse, o.value_sparse) < 1e-9
    np.testing.assert_allclose(r.grad_x.cpu().numpy(), o.grad_x, rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose(r.grad_y.cpu().numpy(), o.grad_y, rtol=1e-9, atol=1e-14)


def test_divergence_log_domain(api):
    # latent codes against the prior with s = 10 s0(n); the self terms'
    # sketches rarely hold the diagonal, so the sparse problems converge
    # slowly at small eps: eps = 1 keeps the oracle within seconds
    p = W.latent_pair(400, d=3, seed=32, eps=1.0)
    opt = O.Options(eps=p.eps, s=p.s, seed=p.seed, cost="plain", tol=1e-6, max_iter=5000,
                    log_domain=True)
    o = D.sinkhorn_divergence(p.x, p.a, p.y, p.b, opt)
    r = api.sinkhorn_divergence(api.Problem(p.x, p.y, p.a, p.b), eps=p.eps, s=p.s, seed=p.seed,
                                tol=1e-6, max_iter=5000, precision="f32_log")
    assert r.status == 0
    assert _rel(r.value_sparse, o.value_sparse) < 1e-4
    assert _rel(r.value, o.value) < 1e-4
    assert _l2(r.grad_x.cpu().numpy(), o.grad_x) < 1e-3
    assert _l2(r.grad_y.cpu().numpy(), o.grad_y) < 1e-3


def test_divergence_without_gradients_and_determinism(api):
    p = W.latent_pair(256, d=3, seed=33, eps=0.5)
    prob = api.Problem(p.x, p.y, p.a, p.b)
    r1 = api.sinkhorn_divergence(prob, eps=p.eps, s=p.s, tol=1e-8, max_iter=3000)
    r2 = api.sinkhorn_divergence(prob, eps=p.eps, s=p.s, tol=1e-8, max_iter=3000,
                                 return_grad=False)
    assert r1.value == r2.value and r2.grad_x is None


@pytest.mark.parametrize("n,m,d", [(300, 257, 10), (200, 200, 3)])
def test_divergence_euclidean_cost_f64(api, n, m, d):
    # C = |x - y|, the distance the generative-modelling section names
    p = W.latent_pair(max(n, m), d=d, seed=34, eps=1.0)
    x, y = p.x[:n], p.y[:m]
    a, b = np.full(n, 1.0 / n), np.full(m, 1.0 / m)
    T = 30
    opt = O.Options(eps=p.eps, s=p.s, seed=p.seed, cost="euclid", tol=0.0, max_iter=T)
    o = D.sinkhorn_divergence(x, a, y, b, opt)
    r = api.sinkhorn_divergence(api.Problem(x, y, a, b), eps=p.eps, s=p.s, seed=p.seed, tol=0.0,
                                max_iter=T, cost="euclid")
    assert r.iters_xy == r.iters_xx == r.iters_yy == T
    for got, ref in ((r.ot_xy, o.xy), (r.ot_xx, o.xx), (r.ot_yy, o.yy)):
        assert _rel(got, ref.estimate.estimate) < 1e-10
    assert _rel(r.value_sparse, o.value_sparse) < 1e-9
    np.testing.assert_allclose(r.grad_x.cpu().numpy(), o.grad_x, rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose(r.grad_y.cpu().numpy(), o.grad_y, rtol=1e-9, atol=1e-14)


def test_divergence_section_setup(api):
    # the section's set-up: batch n = 500 latent codes in R^10 against prior
    # draws, uniform weights, Euclidean distance, eps = 0.01, s = 10 s0(n).
    # C / eps reaches ~870 here, past FP64's exponent range, so both sides
    # run the log domain (the library in FP32 with FP64 potentials, the
    # oracle in FP64).  At this eps the sparse problems converge sublinearly
    # (the oracle's residual is 2e-4 after 3000 iterations), so the terms run
    # a fixed number of iterations, as an auto-encoder's inner loop does, and
    # are compared there.
    p = W.latent_pair(500, d=10, seed=0, eps=0.01)
    T = 200
    opt = O.Options(eps=p.eps, s=p.s, seed=p.seed, cost="euclid", tol=0.0, max_iter=T,
                    log_domain=True)
    o = D.sinkhorn_divergence(p.x, p.a, p.y, p.b, opt)
    r = api.sinkhorn_divergence(api.Problem(p.x, p.y, p.a, p.b), eps=p.eps, s=p.s, seed=p.seed,
                                tol=0.0, max_iter=T, cost="euclid", precision="f32_log")
    assert r.iters_xy == r.iters_xx == r.iters_yy == T
    assert r.nnz == o.xy.nnz + o.xx.nnz + o.yy.nnz
    print(f"S = {r.value_sparse:.10f} (oracle {o.value_sparse:.10f}), "
          f"grad rel L2 {_l2(r.grad_x.cpu().numpy(), o.grad_x):.2e}")
    assert _rel(r.value_sparse, o.value_sparse) < 1e-4
    assert _rel(r.value, o.value) < 1e-4
    assert _l2(r.grad_x.cpu().numpy(), o.grad_x) < 1e-3
    assert _l2(r.grad_y.cpu().numpy(), o.grad_y) < 1e-3
