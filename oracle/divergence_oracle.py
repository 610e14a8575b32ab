"""CPU FP64 oracle for the Sinkhorn divergence built from Spar-Sink estimates
(the generative-modelling section, eq. (sink-div)).  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or call this module; the HIP library shares no code
with it.  Plain NumPy in float64:

* eq. (sink-div): S(mu, nu) = OT_eps(mu, nu) - (OT_eps(mu, mu) + OT_eps(nu, nu)) / 2,
  each term replaced by its Spar-Sink estimate (Alg. 3).

Readings (restated in the design notes):

* The three terms are three Spar-Sink OT solves on hash streams
  problem_index, problem_index + 1 and problem_index + 2.
* The cost is unnormalised (the three terms must share one cost function,
  which a per-problem maximum would break): the Euclidean distance the
  section names between samples ("euclid"), or the squared Euclidean
  distance ("plain") as an option.  The section's ground cost reads as the
  Euclidean distance itself.
* Gradients with respect to the points are those of the sparse problems'
  values at their optima (envelope theorem): for OT the sampling probability
  depends on the masses only, so with the mask fixed the sparse value
  <T~, C~> - eps H(T~), C~ = C + eps log p*, has d/dx_i = sum_j T~_ij dC_ij/dx_i
  with dC_ij/dx_i = 2 (x_i - y_j) (squared) or (x_i - y_j) / |x_i - y_j|
  (Euclidean; 0 where the points coincide).  In a self term both arguments
  move.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np

from . import sparsink_oracle as O


def plan_entries(res: O.SolveResult, log_domain: bool):
    """(rows, cols, T~ entries) of a solve, in CSR order."""
    sk = res.sketch
    rows = np.repeat(np.arange(sk.n), np.diff(sk.row_ptr))
    cols = sk.col_idx.astype(np.int64)
    u, v = res.sinkhorn.u, res.sinkhorn.v
    if log_domain:
        lu, lv = res.sinkhorn.logs()
        t = np.exp(lu[rows] + sk.logval + lv[cols])
    else:
        t = u[rows] * sk.val * v[cols]
    return rows, cols, t


def envelope_grad(x, y, rows, cols, t, cost: str = "plain"):
    """(d/dx, d/dy) of the sparse value: sum over kept entries of t_ij dC_ij."""
    diff = x[rows] - y[cols]
    if cost == "euclid":
        dist = np.sqrt((diff * diff).sum(axis=1))
        with np.errstate(invalid="ignore", divide="ignore"):
            w = np.where(dist > 0.0, t / dist, 0.0)
    else:
        w = 2.0 * t
    gx = np.zeros_like(x)
    gy = np.zeros_like(y)
    np.add.at(gx, rows, w[:, None] * diff)
    np.add.at(gy, cols, -w[:, None] * diff)
    return gx, gy


@dataclass
class DivergenceResult:
    value: float            # from the Alg. 3 estimates
    value_sparse: float     # from the sparse problems' values
    xy: O.SolveResult
    xx: O.SolveResult
    yy: O.SolveResult
    grad_x: np.ndarray
    grad_y: np.ndarray


def sinkhorn_divergence(x, a, y, b, opt: O.Options) -> DivergenceResult:
    if opt.cost not in ("plain", "euclid") or O.is_uot(opt):
        raise ValueError("the divergence uses an unnormalised (squared) Euclidean OT cost")
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    pi = opt.problem_index
    o_xy = O.spar_sink(x, y, a, b, replace(opt, problem_index=pi))
    o_xx = O.spar_sink(x, x, a, a, replace(opt, problem_index=pi + 1))
    o_yy = O.spar_sink(y, y, b, b, replace(opt, problem_index=pi + 2))
    value = o_xy.estimate.estimate - 0.5 * (o_xx.estimate.estimate + o_yy.estimate.estimate)
    value_sp = o_xy.estimate.sparse_objective - 0.5 * (o_xx.estimate.sparse_objective
                                                        + o_yy.estimate.sparse_objective)
    gx_xy, gy_xy = envelope_grad(x, y, *plan_entries(o_xy, opt.log_domain), cost=opt.cost)
    g1, g2 = envelope_grad(x, x, *plan_entries(o_xx, opt.log_domain), cost=opt.cost)
    h1, h2 = envelope_grad(y, y, *plan_entries(o_yy, opt.log_domain), cost=opt.cost)
    grad_x = gx_xy - 0.5 * (g1 + g2)
    grad_y = gy_xy - 0.5 * (h1 + h2)
    return DivergenceResult(value, value_sp, o_xy, o_xx, o_yy, grad_x, grad_y)
