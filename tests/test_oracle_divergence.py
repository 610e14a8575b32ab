"""Pins of the Sinkhorn-divergence oracle (no GPU): the properties the
divergence has by construction with a full budget (zero on equal measures,
symmetry, positivity for the Gaussian kernel, translation invariance), and
the envelope gradients against finite differences of independent solves."""
import numpy as np
import pytest

from oracle import divergence_oracle as D
from oracle import sparsink_oracle as O


def _measures(n, m, d, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, d)) * 0.5
    y = rng.standard_normal((m, d)) * 0.5 + 0.3
    a = rng.dirichlet(np.ones(n))
    b = rng.dirichlet(np.ones(m))
    return x, a, y, b


FULL = dict(eps=0.5, s=1e12, cost="plain", tol=1e-13, max_iter=20000)


def test_full_budget_divergence_vanishes_on_equal_measures():
    x, a, _, _ = _measures(30, 30, 2, 1)
    r = D.sinkhorn_divergence(x, a, x, a, O.Options(**FULL))
    assert abs(r.value) < 1e-12 and abs(r.value_sparse) < 1e-12
    assert np.abs(r.grad_x + r.grad_y).max() < 1e-12


def test_full_budget_symmetry_and_positivity():
    x, a, y, b = _measures(25, 31, 3, 2)
    r1 = D.sinkhorn_divergence(x, a, y, b, O.Options(**FULL))
    r2 = D.sinkhorn_divergence(y, b, x, a, O.Options(**FULL))
    assert r1.value == pytest.approx(r2.value, rel=1e-10)
    np.testing.assert_allclose(r1.grad_x, r2.grad_y, rtol=1e-8, atol=1e-12)
    # the Gaussian kernel exp(-|x-y|^2/eps) is positive definite: S > 0 for mu != nu
    assert r1.value_sparse > 0


def test_translation_invariance():
    x, a, y, b = _measures(40, 35, 2, 3)
    opt = O.Options(eps=0.3, s=400.0, cost="plain", tol=1e-12, max_iter=20000, seed=4)
    r = D.sinkhorn_divergence(x, a, y, b, opt)
    t = np.array([0.7, -1.3])
    r2 = D.sinkhorn_divergence(x + t, a, y + t, b, opt)
    assert r2.value == pytest.approx(r.value, rel=1e-9)
    np.testing.assert_allclose(r2.grad_x, r.grad_x, rtol=1e-6, atol=1e-10)
    # and the gradients sum to zero over all points (translation of both clouds)
    assert np.abs(r.grad_x.sum(axis=0) + r.grad_y.sum(axis=0)).max() < 1e-8


def _fd_check(opt, x, a, y, b, which, value_attr, rel):
    r = D.sinkhorn_divergence(x, a, y, b, opt)
    g = r.grad_x if which == "x" else r.grad_y
    rng = np.random.default_rng(5)
    h = 1e-5
    for _ in range(4):
        i = int(rng.integers(0, (x if which == "x" else y).shape[0]))
        k = int(rng.integers(0, x.shape[1]))
        vals = []
        for sgn in (1.0, -1.0):
            xp, yp = x.copy(), y.copy()
            (xp if which == "x" else yp)[i, k] += sgn * h
            vals.append(getattr(D.sinkhorn_divergence(xp, a, yp, b, opt), value_attr))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert fd == pytest.approx(g[i, k], rel=rel, abs=1e-7), (which, i, k)


@pytest.mark.parametrize("which", ["x", "y"])
def test_envelope_gradient_of_the_dense_divergence(which):
    # every p* = 1: the sparse value is OT_eps itself and the envelope
    # theorem applies to the exact optimum
    x, a, y, b = _measures(20, 18, 2, 6)
    _fd_check(O.Options(**FULL), x, a, y, b, which, "value", 1e-6)


@pytest.mark.parametrize("seed", [0, 3, 8])
@pytest.mark.parametrize("which", ["x", "y"])
def test_envelope_gradient_of_the_sketched_divergence(which, seed):
    # OT sampling depends on the masses only: moving a point keeps the mask and
    # changes the sketch's values, so the sparse value's derivative is the
    # envelope sum over the kept entries.  The finite differences need the
    # sparse optimum to 1e-13, so every sketch must admit the marginals with a
    # well-conditioned loop: shrinkage toward uniform sampling (Sec. 4, its
    # lower bound on p) with g = 1/2 and s = nm/2 keeps every p* >= 1/4, so
    # each line keeps about a quarter of its entries or more, for any hash key.
    x, a, y, b = _measures(40, 36, 2, 7)
    opt = O.Options(eps=0.4, s=0.5 * 40 * 36, shrink=0.5, cost="plain", tol=1e-13,
                    max_iter=50000, seed=seed)
    r = D.sinkhorn_divergence(x, a, y, b, opt)
    assert all(t.sinkhorn.converged for t in (r.xy, r.xx, r.yy))
    assert r.xy.nnz < 40 * 36
    _fd_check(opt, x, a, y, b, which, "value_sparse", 1e-5)


@pytest.mark.parametrize("which", ["x", "y"])
def test_envelope_gradient_with_the_euclidean_cost(which):
    # the section's distance between samples, C = |x - y|: the gradient term
    # of an entry is T~ (x_i - y_j) / |x_i - y_j|; checked against finite
    # differences of independent solves, dense (every p* = 1) and sketched
    x, a, y, b = _measures(20, 18, 3, 9)
    full = dict(FULL, cost="euclid")
    _fd_check(O.Options(**full), x, a, y, b, which, "value", 1e-6)
    opt = O.Options(eps=0.4, s=0.5 * 20 * 18, shrink=0.5, cost="euclid", tol=1e-13,
                    max_iter=50000, seed=2)
    r = D.sinkhorn_divergence(x, a, y, b, opt)
    assert all(t.sinkhorn.converged for t in (r.xy, r.xx, r.yy)) and r.xy.nnz < 20 * 18
    _fd_check(opt, x, a, y, b, which, "value_sparse", 1e-5)


def test_euclidean_cost_is_the_distance():
    # C = sqrt of the squared distance, with the self term's zero on the diagonal
    rng = np.random.default_rng(11)
    x = rng.standard_normal((7, 4))
    c = O.cost_from_sq(O.sq_dist(x, x), "euclid", 1.0, 1.0)
    ref = np.linalg.norm(x[:, None, :] - x[None, :, :], axis=-1)
    np.testing.assert_allclose(c, ref, rtol=4e-16, atol=0)
    assert np.all(np.diag(c) == 0.0)
