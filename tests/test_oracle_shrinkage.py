"""Pins of the oracle's shrinkage probabilities (no GPU).

Sec. 4 mixes the proposed sampling probability with the uniform one
linearly, p = (1 - g) p_ij + g / (nm); Sec. 5's Rand-Sink is the
equal-probability case g = 1.  The oracle is checked against the mixture
written out from the definitions (eq. (pij-ot), eq. (pij-uot)), against the
closed form of the uniform case, and against sampling statistics."""
import math

import numpy as np
import pytest
import scipy.spatial

from oracle import sparsink_oracle as O
from paper_2306_06581_amd import workloads as W


@pytest.mark.parametrize("g", [0.0, 0.25, 0.5, 1.0])
def test_ot_shrinkage_is_the_linear_mixture(g):
    p = W.ot_gauss2d(200, seed=11, m=150)
    n, m = 200, 150
    pr = O.ot_probabilities(p.a, p.b, p.s, shrink=g)
    full = pr.pstar(np.arange(n), np.arange(m))
    assert full.max() < 1.0
    direct = np.sqrt(np.outer(p.a, p.b))
    mix = (1 - g) * direct / direct.sum() + g / (n * m)
    np.testing.assert_allclose(full, p.s * mix, rtol=1e-12)
    assert full.sum() == pytest.approx(p.s, rel=1e-12)


def test_rand_sink_is_uniform_and_spar_sink_is_unchanged():
    p = W.ot_gauss2d(64, seed=12)
    rs = O.ot_probabilities(p.a, p.b, p.s, shrink=1.0)
    full = rs.pstar(np.arange(64), np.arange(64))
    assert np.all(full == p.s / (64.0 * 64.0))
    # g = 0 reproduces the unmixed probabilities bit for bit
    a0 = O.ot_probabilities(p.a, p.b, p.s)
    b0 = O.ot_probabilities(p.a, p.b, p.s, shrink=0.0)
    assert np.array_equal(a0.pstar(np.arange(64), np.arange(64)),
                          b0.pstar(np.arange(64), np.arange(64)))
    opt = O.Options(eps=p.eps, s=p.s, seed=3)
    s0 = O.build_sketch(p.x, p.y, p.a, p.b, opt)
    s1 = O.build_sketch(p.x, p.y, p.a, p.b, O.Options(eps=p.eps, s=p.s, seed=3, shrink=0.0))
    assert np.array_equal(s0.mask, s1.mask) and np.array_equal(s0.val, s1.val)


@pytest.mark.parametrize("g", [0.3, 1.0])
def test_uot_shrinkage_is_the_linear_mixture(g):
    p = W.uot_mix3(150, seed=13, eps=0.05)
    cmax, inv_cmax = O.cost_scale(p.x, p.y, O.Options(eps=p.eps, s=p.s))
    pr = O.uot_probabilities(p.a, p.b, p.x, p.y, p.s, 1.0, p.eps, inv_cmax, shrink=g)
    rows, cols = np.arange(150), np.arange(150)
    C = scipy.spatial.distance.cdist(p.x, p.y, "sqeuclidean") / cmax
    K = np.exp(-C / p.eps)
    raw = np.outer(p.a, p.b) ** (1.0 / (2 + p.eps)) * K ** (p.eps / (2 + p.eps))
    mix = (1 - g) * raw / raw.sum() + g / (150 * 150)
    np.testing.assert_allclose(pr.pstar(rows, cols), np.minimum(1, p.s * mix), rtol=1e-11)


def test_rand_sink_nnz_and_inclusion_frequencies():
    # uniform p* = s / (nm): E[nnz] = s exactly, and inclusion frequencies
    # over many keys match p* (chi-square over a 5 x 5 problem)
    p = W.ot_gauss2d(512, seed=14)
    opt = O.Options(eps=p.eps, s=p.s, seed=1, shrink=1.0)
    sk = O.build_sketch(p.x, p.y, p.a, p.b, opt)
    e, var = O.expected_nnz_ot(sk.prob)
    assert e == pytest.approx(p.s, rel=1e-12)
    assert abs(sk.nnz - e) <= 6 * math.sqrt(var)
    rng = np.random.default_rng(15)
    a, b = rng.dirichlet(np.ones(5)), rng.dirichlet(np.ones(5))
    pr = O.ot_probabilities(a, b, 8.0, shrink=0.5)
    P = pr.pstar(np.arange(5), np.arange(5))
    R = 3000
    counts = np.zeros((5, 5))
    i, j = np.meshgrid(np.arange(5), np.arange(5), indexing="ij")
    for key in range(R):
        counts += O.uniform01(i, j, 0, key * 104729 + 7) < P
    chi2 = float((((counts - R * P) ** 2) / (R * P * (1 - P))).sum())
    assert chi2 < 70.0          # chi^2_25: P(X > 70) ~ 5e-6
