"""CPU FP64 oracle for Spar-IBP (fixed-support Wasserstein barycenters).
TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or call this module; the HIP library shares no code
with it.  Plain NumPy/SciPy in float64, written from the barycenter section of
the paper (Li, Yu, Li & Meng, "Importance Sparsification for Sinkhorn
Algorithm", JMLR 2023):

* eq. (wb), eq. (rwb) -- q* minimises sum_k w_k OT_eps(q, b_k) over the simplex,
  with the measures b_k on one support {x_i} and K_k = exp(-C_k / eps).
* Alg. IBP            -- the iterative Bregman projections: v_k = b_k / K_k^T u_k,
  then the barycenter as the weighted geometric mean of the K_k v_k, then
  u_k = q / K_k v_k; stop when |q^t - q^(t-1)|_1 <= delta.
* eq. (pois-k), Alg. Spar-IBP -- the same loop on sketches K~_k sampled with
  p_{k,ij} = sqrt(b_kj) / (n sum_j sqrt(b_kj)) (the OT probability with the
  unknown barycenter replaced by its uniform start), p* = min(1, s p).

Readings (restated in the design notes):

* Order of the updates.  The printed loop forms u_k from the barycenter of the
  previous iteration and the barycenter afterwards.  With that order the
  weighted sum of log u_k is no longer zero and the iteration stalls away from
  the optimum (|q^t - q^(t-1)|_1 stays near 1e-3 on the paper's own set-up);
  the Bregman projections the section cites form the barycenter first and
  then u_k = q^t / K_k v_k.  We take the projection order.
* A line of a sketch with no entry gives a zero product; the quotients are
  then 0 (as in the Spar-Sink oracle) and a zero factor with positive weight
  makes that barycenter entry 0.  At budgets of a few entries per line the
  sketch's bipartite graph can fall apart and the linear-domain iteration can
  overflow; the paper's budgets at its sizes keep clear of that.
* The sampling probability is evaluated as c_k sqrt(b_kj) with
  c_k = s / (n * tree_sum(sqrt(b_k))), and shrinkage (Sec. 4) mixes in the
  uniform probability 1/n^2 exactly as for Spar-Sink.
* The hash stream of measure k is the Spar-Sink stream with problem index k.
* Cost: as in the Spar-Sink oracle (squared Euclidean, divided by its maximum
  unless ``cost="plain"``); one cost for all measures (the support is shared).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import sparsink_oracle as O


@dataclass
class IBPResult:
    q: np.ndarray
    u: list
    v: list
    iters: int
    err: float
    hist: list
    converged: bool


def _quotient(num, den):
    """num / den where den > 0, 0 elsewhere."""
    out = np.zeros_like(num)
    pos = den > 0
    out[pos] = num[pos] / den[pos]
    return out


def geometric_mean(gs, w):
    """prod_k g_k^(w_k) (0^w = 0 for w > 0, g^0 = 1)."""
    out = np.ones_like(gs[0])
    for g, wk in zip(gs, w):
        out = out * (g ** wk)
    return out


def ibp(Ks, bs, w, tol: float, max_iter: int, u0=None) -> IBPResult:
    """Alg. IBP on the kernels Ks (dense or sparse, n x n) in the projection
    order: for every k, v_k = b_k / K_k^T u_k; q = prod_k (K_k v_k)^(w_k);
    for every k, u_k = q / K_k v_k.  q^0 = 1/n, u_k^0 = 1."""
    m = len(Ks)
    n = Ks[0].shape[0]
    KT = [K.T.tocsr() if sp.issparse(K) else K.T for K in Ks]
    q = np.full(n, 1.0 / n)
    u = [np.ones(n) if u0 is None else np.array(u0[k], np.float64) for k in range(m)]
    v = [np.zeros(n) for _ in range(m)]
    hist = []
    err = math.inf
    t = 0
    for t in range(1, max_iter + 1):
        gs = []
        for k in range(m):
            v[k] = _quotient(np.asarray(bs[k], np.float64), KT[k] @ u[k])
            gs.append(Ks[k] @ v[k])
        q_new = geometric_mean(gs, w)
        for k in range(m):
            u[k] = _quotient(q_new, gs[k])
        err = float(np.abs(q_new - q).sum())
        q = q_new
        hist.append(err)
        if err <= tol:
            break
    return IBPResult(q=q, u=u, v=v, iters=t, err=err, hist=hist, converged=err <= tol)


def ibp_probabilities(b, s, shrink: float = 0.0) -> O.ProbOT:
    """Alg. Spar-IBP: p_ij = sqrt(b_j) / (n sum_j sqrt(b_j)) for every row i,
    mixed with the uniform 1/n^2 with weight `shrink` (Sec. 4)."""
    rb = np.sqrt(np.asarray(b, dtype=np.float64))
    n = rb.size
    s_b = O.tree_sum(rb)
    c = s / (float(n) * s_b)
    w, c0 = O.shrink_terms(s, shrink, n, n)
    return O.ProbOT(alpha=np.full(n, c * w), rb=rb, s_a=float(n), s_b=s_b, c0=c0)


def ibp_options(eps, s, seed=0, tol=1e-6, max_iter=1000, cost="maxnorm", shrink=0.0,
                k=0) -> O.Options:
    return O.Options(eps=eps, s=s, seed=seed, tol=tol, max_iter=max_iter, problem_index=k,
                     cost=cost, shrink=shrink)


def ibp_sketch(x, b_k, k: int, eps, s, seed=0, cost="maxnorm", shrink=0.0) -> O.Sketch:
    """eq. (pois-k): the sketch of measure k (hash stream k)."""
    opt = ibp_options(eps, s, seed=seed, cost=cost, shrink=shrink, k=k)
    prob = ibp_probabilities(b_k, s, shrink)
    return O.build_sketch(x, x, None, b_k, opt, prob=prob)


@dataclass
class SparIBPResult:
    ibp: IBPResult
    sketches: list
    nnz: int
    cmax: float


def spar_ibp(x, bs, w, eps, s, seed=0, tol=1e-6, max_iter=1000, cost="maxnorm",
             shrink=0.0) -> SparIBPResult:
    """Alg. Spar-IBP: IBP on the sketches of all measures."""
    sks = [ibp_sketch(x, bs[k], k, eps, s, seed, cost, shrink) for k in range(len(bs))]
    res = ibp([sk.csr() for sk in sks], bs, w, tol, max_iter)
    return SparIBPResult(ibp=res, sketches=sks, nnz=sum(sk.nnz for sk in sks),
                         cmax=sks[0].cmax)


def dense_kernel(x, eps, cost="maxnorm"):
    """K = exp(-C / eps) on the shared support."""
    x = np.asarray(x, np.float64)
    cmax, inv_cmax = O.cost_scale(x, x, O.Options(eps=eps, s=1.0, cost=cost))
    return np.exp(-((O.sq_dist(x, x) * inv_cmax) / eps)), cmax


def dense_ibp(x, bs, w, eps, tol=1e-6, max_iter=1000, cost="maxnorm") -> IBPResult:
    """Alg. IBP with the full kernel (the same K for every measure)."""
    K, _ = dense_kernel(x, eps, cost)
    return ibp([K] * len(bs), bs, w, tol, max_iter)
