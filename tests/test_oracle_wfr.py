"""Pins of the oracle's Wasserstein-Fisher-Rao cost (no GPU): its small-angle
limit, its structural zeros, the workload's sparsity levels, the single-point
UOT closed form under it, and the full-budget sketch equal to the dense
kernel with its zeros."""
import math

import numpy as np
import pytest

from oracle import sparsink_oracle as O
from paper_2306_06581_amd import workloads as W


def test_small_angle_limit_is_the_scaled_squared_distance():
    # -log cos^2 z = z^2 + z^4/6 + O(z^6): for d << eta the cost is d^2/(4 eta^2)
    rng = np.random.default_rng(1)
    c = rng.uniform(0.0, 1.0, 200)
    for eta in (10.0, 100.0):
        C = O.cost_from_sq(c, "wfr", 1.0, eta)
        z2 = c / (4 * eta * eta)
        # cos z rounds to within 2^-53 of 1, so -2 log cos z carries an absolute
        # error of about 2^-52 on top of the z^6 term of the series
        np.testing.assert_allclose(C, z2 + z2 * z2 / 6, rtol=z2.max() ** 2 / 20, atol=5e-16)


def test_cost_values_against_the_definition_by_another_route():
    # cos_+ written as a clipped angle and the square taken before the log
    rng = np.random.default_rng(2)
    eta = 0.3
    d = rng.uniform(0.0, 1.5, 500)
    C = O.cost_from_sq(d * d, "wfr", 1.0, eta)
    z = np.minimum(np.hypot(d, 0.0) / (2 * eta), math.pi / 2)
    with np.errstate(divide="ignore"):
        ref = -np.log(np.cos(z) ** 2)
    inside = d * (0.5 / eta) < math.pi / 2
    np.testing.assert_allclose(C[inside], ref[inside], rtol=1e-12, atol=1e-15)
    # blocked transport: K = 0 exactly from d = pi eta on
    assert np.all(np.isinf(C[~inside]))
    assert np.all(np.exp(-C[~inside] / 0.1) == 0.0)
    assert np.all(d[~inside] >= math.pi * eta * (1 - 1e-15))


@pytest.mark.parametrize("ratio", [0.7, 0.5, 0.3])
def test_workload_sparsity_levels(ratio):
    p = W.wfr_synthetic(500, d=5, seed=3, nnz_ratio=ratio)
    C = O.cost_from_sq(O.sq_dist(p.x, p.y), "wfr", 1.0, p.meta["eta"])
    assert abs(np.isfinite(C).mean() - ratio) < 0.03
    assert np.all(np.isfinite(np.diag(C))) and np.all(np.diag(C) == 0.0)


def test_single_point_uot_closed_form_under_wfr():
    # n = m = 1: T* = (a b)^(lam/(2 lam + eps)) exp(-C/(2 lam + eps)), with C
    # the WFR cost of the single pair (optimality of eq. (ruot) in one variable)
    x = np.array([[0.0, 0.0]])
    y = np.array([[0.3, 0.4]])           # d = 0.5
    a, b = np.array([2.0]), np.array([0.7])
    eps, lam, eta = 0.1, 0.5, 0.4
    C = -math.log(math.cos(0.5 / (2 * eta)) ** 2)
    t_star = (a[0] * b[0]) ** (lam / (2 * lam + eps)) * math.exp(-C / (2 * lam + eps))
    opt = O.Options(eps=eps, s=1.0, lam=lam, tol=1e-15, max_iter=10000, cost="wfr", eta=eta)
    r = O.dense_sinkhorn(x, y, a, b, opt)
    t = r.sinkhorn.u[0] * math.exp(-C / eps) * r.sinkhorn.v[0]
    assert t == pytest.approx(t_star, rel=1e-12)


def test_full_budget_sketch_is_the_dense_kernel_with_its_zeros():
    p = W.wfr_synthetic(80, d=3, seed=4, nnz_ratio=0.5)
    eta = p.meta["eta"]
    # p* = min(1, s q / Z) reaches 1 on every entry with K > 0 only for a budget
    # beyond the smallest q near the blocking distance (q ~ 1e-100 there)
    opt = O.Options(eps=p.eps, s=1e300, lam=p.lam, seed=5, tol=1e-10, max_iter=3000,
                    cost="wfr", eta=eta)
    sk = O.build_sketch(p.x, p.y, p.a, p.b, opt)
    C = O.cost_from_sq(O.sq_dist(p.x, p.y), "wfr", 1.0, eta)
    keep = np.unpackbits(sk.mask.view(np.uint8), axis=1, bitorder="little")[:, :80].astype(bool)
    # every entry with K > 0 is kept with p* = 1, and no structural zero is kept
    assert np.array_equal(keep, np.isfinite(C))
    assert np.all(sk.pstar == 1.0)
    s = O.spar_sink(p.x, p.y, p.a, p.b, opt)
    d = O.dense_sinkhorn(p.x, p.y, p.a, p.b, opt)
    assert s.sinkhorn.iters == d.sinkhorn.iters
    np.testing.assert_allclose(s.sinkhorn.u, d.sinkhorn.u, rtol=1e-12)
    np.testing.assert_allclose(s.estimate.estimate, d.estimate.estimate, rtol=1e-12)


def test_large_eta_matches_the_scaled_squared_euclidean_problem():
    # WFR with d << eta is the squared Euclidean UOT of the points scaled by
    # 1/(2 eta), up to the z^4/6 term of the cost
    p = W.wfr_synthetic(60, d=2, seed=6)
    eta = 50.0
    base = dict(eps=0.1, s=1.0, lam=0.1, tol=1e-12, max_iter=20000)
    wfr = O.dense_sinkhorn(p.x, p.y, p.a, p.b, O.Options(cost="wfr", eta=eta, **base))
    sq = O.dense_sinkhorn(p.x / (2 * eta), p.y / (2 * eta), p.a, p.b,
                          O.Options(cost="plain", **base))
    assert wfr.estimate.estimate == pytest.approx(sq.estimate.estimate, rel=1e-6)


def test_sparse_sampling_never_keeps_a_structural_zero():
    p = W.wfr_synthetic(400, d=5, seed=7, nnz_ratio=0.3)
    eta = p.meta["eta"]
    opt = O.Options(eps=p.eps, s=p.s, lam=p.lam, seed=8, cost="wfr", eta=eta)
    sk = O.build_sketch(p.x, p.y, p.a, p.b, opt)
    assert sk.nnz > 0 and np.all(np.isfinite(sk.cost)) and np.all(sk.val > 0)
    rows = np.repeat(np.arange(sk.n), np.diff(sk.row_ptr))
    d = np.sqrt(((p.x[rows] - p.y[sk.col_idx]) ** 2).sum(axis=1))
    assert np.all(d < math.pi * eta)
