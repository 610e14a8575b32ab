"""Seeded synthetic inputs shaped like the workloads of the Spar-Sink paper.

This module only draws point clouds and marginal weights with NumPy's
``default_rng``; it holds none of the method's arithmetic (no costs, no
probabilities, no hashing, no scaling).  It is the single input source shared
by the tests, the benchmark and the oracle-vs-device parity checks.

Draw order per problem is fixed: x, y, a, b (then per-problem parameters).
The subsample budget ``s`` is returned as a plain number derived from n.

Workload families (the sizes named here are the default ones; every generator
takes an explicit ``n`` so tests can use small or ragged shapes):

* ``ot_gauss2d``  -- OT, d=2, x~N(0,I), y~N((1,1),I), a,b ~ U(0,1) normalised,
  eps=0.1, s = 8 n ln n, squared Euclidean cost divided by its maximum.
  Paper context: the simulations of Section 5.1 use n=1000 synthetic supports.
* ``ot_t5_d10``   -- OT, d=10, x~N(0,I), y = t_5 per coordinate + 0.5,
  a,b ~ Dirichlet(1), eps=0.05, s in {4,8,16} n ln n, normalised cost.
* ``uot_mix3``    -- UOT (lambda=1), d=3, x ~ equal mixture of 3 isotropic
  Gaussians (means U[-1,1]^3, sigma 0.25), y = x + N(0, 0.1^2 I) (paired),
  a,b ~ U(0,1) scaled to total masses 1.0 and 1.3, eps in {0.01, 0.05},
  s = 8 n ln n, normalised cost.
* ``batch_ot``    -- many independent OT problems, n_k ~ U{256..4096}, d=3,
  x ~ N(mu_x, I), y ~ N(mu_y, I), mu ~ U[-1,1]^3, a,b ~ Dirichlet(1),
  eps=0.05, s_k = 8 n_k ln n_k.
* ``ibp_synthetic`` -- fixed-support barycenter of three measures on n points
  x ~ U(0,1)^d (the paper's barycenter simulation): b_1 a Gaussian
  N(1/5, 1/50), b_2 the mixture N(1/2, 1/60)/2 + N(4/5, 1/80)/2, b_3 a t_5
  with location 3/5 and scale^2 1/100, each a density evaluated on the index
  grid i/n, raised by 1e-2 of its maximum and normalised; equal weights;
  s = factor * s0(n), s0(n) = 1e-3 n ln^4 n.
* ``wfr_synthetic`` -- UOT with the Wasserstein-Fisher-Rao cost (the paper's
  UOT simulation): one support of n points shared by a and b (C1: x ~
  U(0,1)^d; C2: x ~ N(0, Sigma), Sigma_jk = 0.5^|j-k|; C3: as C1), a and b
  densities on the index grid i/n (C1, C2: Gaussians N(1/3, 1/20) and
  N(1/2, 1/20); C3: t_5 with the same locations and scales^2) scaled to total
  masses 5 and 3; eps = 0.1, lambda = 0.1; eta set so that a given share of
  the pairs has d_ij < pi eta (K > 0): 0.7, 0.5, 0.3 for R1, R2, R3, taken
  as a quantile of the distances of 20000 random pairs (a workload parameter,
  not part of the method).
* ``latent_pair``  -- the Sinkhorn-divergence regulariser of the generative-
  modelling section: a batch of n latent codes in R^d (a fixed non-Gaussian
  warp of Gaussian draws, standing in for encoder outputs) against n draws of
  the standard Gaussian prior, uniform weights, eps = 0.01 (the section's
  value; the default, which callers may override), s = 10 s0(n).  The cost
  (the section's Euclidean distance, or its square) is the solver's option.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = ["Problem", "ot_gauss2d", "ot_t5_d10", "uot_mix3", "batch_ot", "s_budget",
           "IBPProblem", "ibp_synthetic", "s0_budget", "wfr_synthetic", "latent_pair"]


@dataclass
class Problem:
    """One transport problem: supports, weights and the method's parameters."""

    x: np.ndarray            # (n, d) float64, row-major
    y: np.ndarray            # (m, d) float64, row-major
    a: np.ndarray            # (n,) float64, non-negative
    b: np.ndarray            # (m,) float64, non-negative
    eps: float
    s: float
    lam: float = math.inf    # inf => balanced OT
    seed: int = 0            # hash key for the Poisson mask
    problem_index: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def m(self) -> int:
        return int(self.y.shape[0])

    @property
    def d(self) -> int:
        return int(self.x.shape[1])


def s_budget(n: int, factor: float) -> float:
    """Subsample budget factor * n * ln(n) (natural log)."""
    return float(factor * n * math.log(n))


def _uniform_weights(rng: np.random.Generator, n: int, total: float) -> np.ndarray:
    w = rng.uniform(0.0, 1.0, size=n)
    return w * (total / w.sum())


def ot_gauss2d(n: int = 1024, seed: int = 0, m: int | None = None,
               s_factor: float = 8.0, eps: float = 0.1) -> Problem:
    m = n if m is None else m
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 2))
    y = rng.standard_normal((m, 2)) + 1.0
    a = _uniform_weights(rng, n, 1.0)
    b = _uniform_weights(rng, m, 1.0)
    return Problem(x, y, a, b, eps=eps, s=s_budget(max(n, 2), s_factor), seed=seed,
                   name=f"ot_gauss2d_n{n}")


def ot_t5_d10(n: int = 16384, seed: int = 0, m: int | None = None,
              s_factor: float = 8.0, eps: float = 0.05, d: int = 10) -> Problem:
    m = n if m is None else m
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, d))
    y = rng.standard_t(5.0, size=(m, d)) + 0.5
    a = rng.dirichlet(np.ones(n))
    b = rng.dirichlet(np.ones(m))
    return Problem(x, y, a, b, eps=eps, s=s_budget(max(n, 2), s_factor), seed=seed,
                   name=f"ot_t5_d{d}_n{n}_s{s_factor:g}")


def uot_mix3(n: int = 65536, seed: int = 0, eps: float = 0.05, lam: float = 1.0,
             s_factor: float = 8.0, mass_a: float = 1.0, mass_b: float = 1.3) -> Problem:
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, size=(3, 3))
    comp = rng.integers(0, 3, size=n)
    x = means[comp] + 0.25 * rng.standard_normal((n, 3))
    y = x + 0.1 * rng.standard_normal((n, 3))
    a = _uniform_weights(rng, n, mass_a)
    b = _uniform_weights(rng, n, mass_b)
    return Problem(x, y, a, b, eps=eps, s=s_budget(max(n, 2), s_factor), lam=lam,
                   seed=seed, name=f"uot_mix3_n{n}_eps{eps:g}")


def batch_ot(count: int = 512, seed: int = 0, n_lo: int = 256, n_hi: int = 4096,
             eps: float = 0.05, s_factor: float = 8.0) -> list[Problem]:
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_lo, n_hi + 1, size=count)
    out = []
    for k, nk in enumerate(sizes):
        nk = int(nk)
        mu_x = rng.uniform(-1.0, 1.0, size=3)
        mu_y = rng.uniform(-1.0, 1.0, size=3)
        x = mu_x + rng.standard_normal((nk, 3))
        y = mu_y + rng.standard_normal((nk, 3))
        a = rng.dirichlet(np.ones(nk))
        b = rng.dirichlet(np.ones(nk))
        out.append(Problem(x, y, a, b, eps=eps, s=s_budget(nk, s_factor), seed=seed,
                           problem_index=k, name=f"batch_ot_{k}_n{nk}"))
    return out


@dataclass
class IBPProblem:
    """A fixed-support barycenter problem: support x, measures b[k], weights w."""

    x: np.ndarray            # (n, d) float64
    b: np.ndarray            # (m, n) float64, each row sums to 1
    w: np.ndarray            # (m,) float64, sums to 1
    eps: float
    s: float
    seed: int = 0
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def count(self) -> int:
        return int(self.b.shape[0])


def s0_budget(n: int) -> float:
    """The barycenter experiments' unit budget 1e-3 n ln^4 n (natural log)."""
    return 1e-3 * n * math.log(n) ** 4


def ibp_synthetic(n: int = 1000, d: int = 5, seed: int = 0, eps: float = 0.01,
                  s_factor: float = 20.0) -> IBPProblem:
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(n, d))
    t = np.arange(n) / n

    def gauss(mu, var):
        return np.exp(-0.5 * (t - mu) ** 2 / var)

    def student5(mu, scale2):
        return (1.0 + (t - mu) ** 2 / scale2 / 5.0) ** -3.0

    dens = [gauss(0.2, 1 / 50), 0.5 * gauss(0.5, 1 / 60) + 0.5 * gauss(0.8, 1 / 80),
            student5(0.6, 1 / 100)]
    b = []
    for g in dens:
        g = g / g.sum()
        g = g + 1e-2 * g.max()
        b.append(g / g.sum())
    return IBPProblem(x=x, b=np.array(b), w=np.full(3, 1.0 / 3.0), eps=eps,
                      s=s_factor * s0_budget(n), seed=seed, name=f"ibp_synthetic_n{n}_d{d}")


def wfr_synthetic(n: int = 1000, d: int = 5, seed: int = 0, pattern: str = "C1",
                  nnz_ratio: float = 0.5, eps: float = 0.1, lam: float = 0.1,
                  s_factor: float = 8.0) -> Problem:
    rng = np.random.default_rng(seed)
    if pattern == "C2":
        idx = np.arange(d)
        cov = 0.5 ** np.abs(idx[:, None] - idx[None, :])
        x = rng.multivariate_normal(np.zeros(d), cov, size=n)
    else:
        x = rng.uniform(0.0, 1.0, size=(n, d))
    t = np.arange(n) / n
    if pattern == "C3":
        a = (1.0 + (t - 1 / 3) ** 2 / (1 / 20) / 5.0) ** -3.0
        b = (1.0 + (t - 1 / 2) ** 2 / (1 / 20) / 5.0) ** -3.0
    else:
        a = np.exp(-0.5 * (t - 1 / 3) ** 2 / (1 / 20))
        b = np.exp(-0.5 * (t - 1 / 2) ** 2 / (1 / 20))
    a = a * (5.0 / a.sum())
    b = b * (3.0 / b.sum())
    i = rng.integers(0, n, size=20000)
    j = rng.integers(0, n, size=20000)
    dist = np.sqrt(((x[i] - x[j]) ** 2).sum(axis=1))
    eta = float(np.quantile(dist, nnz_ratio)) / math.pi
    return Problem(x, x.copy(), a, b, eps=eps, s=s_factor * s0_budget(max(n, 2)), lam=lam,
                   seed=seed, name=f"wfr_{pattern}_n{n}_d{d}_r{nnz_ratio:g}",
                   meta={"eta": eta, "pattern": pattern, "nnz_ratio": nnz_ratio})


def latent_pair(n: int = 500, d: int = 10, seed: int = 0, eps: float = 0.01,
                s_factor: float = 10.0) -> Problem:
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, d))
    x = 0.8 * z + 0.4 * np.sin(3.0 * z) + 0.3
    y = rng.standard_normal((n, d))
    a = np.full(n, 1.0 / n)
    b = np.full(n, 1.0 / n)
    return Problem(x, y, a, b, eps=eps, s=s_factor * s0_budget(max(n, 2)), seed=seed,
                   name=f"latent_pair_n{n}_d{d}")
