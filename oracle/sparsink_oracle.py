"""CPU FP64 oracle for the Spar-Sink hot path.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or call this module.  The product (the HIP library and
its Python binding) never does: it shares no code, headers, tables or constants
with this file.

Everything here is plain NumPy/SciPy in float64, written from the paper
(Li, Yu, Li & Meng, "Importance Sparsification for Sinkhorn Algorithm",
JMLR 2023):

* Sec. 2.1, eq. (rot)/(rot-solu)  -- K = exp(-C/eps), T = diag(u) K diag(v).
* Alg. 1 (SinkhornOT), Alg. 2 (SinkhornUOT) -- the scaling iterations.
* Sec. 3.1, eq. (pois)            -- Poisson sparsification, p* = min(1, s p).
* Sec. 3.1, eq. (pij-ot)          -- p_ij proportional to sqrt(a_i b_j).
* Sec. 3.2, eq. (pij-uot)         -- p_ij proportional to
                                     (a_i b_j)^(lam/(2lam+eps)) K_ij^(eps/(2lam+eps)).
* Alg. 3 / Alg. 4                 -- the Spar-Sink estimates.
* Sec. 2 notation                 -- KL(x||y) = sum x log(x/y) - x + y, 0 log 0 = 0;
                                     H(T) = -sum T (log T - 1).
* Appendix, proof of Thm. 3       -- log-domain form with C~ = C + eps log p*.

Choices where the paper is silent (all restated in the design notes):

* Randomness: the Bernoulli draw for entry (i, j) of problem k is a
  counter-based hash, Philox4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw,
  "Parallel random numbers: as easy as 1, 2, 3", SC 2011), with counters
  (q, i, k, w) and key (seed lo32, seed hi32).  Column j maps to counter word
  q = (j >> 9) * 64 + (j & 63) and slot s = (j >> 6) & 7.  The high 16 bits
  of a 48-bit word are 16-bit half s & 1 (low half first) of output word
  s >> 1 of the w = 0 call; the low 32 bits are output word s & 3 of the
  w = 1 + (s >> 2) call.  U = bits * 2^-48 and the entry is kept iff U < p*.
* Sums that decide sampled entries (sum sqrt(a), sum sqrt(b)) are the perfect
  binary-tree sum over the zero-padded power-of-two vector (adjacent pairs,
  level by level), so the OT mask is reproducible bit for bit.
* Cost: c_ij = sum_k (x_ik - y_jk)^2 accumulated in k order, each product
  and sum separately rounded; with max-normalisation C = c * (1 / max c).
* UOT sampling weight: q_ij = exp(th*(log a_i + log b_j) - C_ij/(2lam+eps)),
  th = lam/(2lam+eps) (the identity K^(eps/(2lam+eps)) = exp(-C/(2lam+eps)));
  Z = sum q; p* = min(1, (s/Z) q).
* Every exponential, logarithm and cosine that decides a sampled entry or
  forms a stored value (q, log a, log b, the WFR cost, K = exp(-C/eps),
  log p*) is the fixed operation sequence of ``elementary.py`` (Cody-Waite
  reduction and Taylor polynomials), so that an independent implementation
  of the same sequence reproduces the mask and the values bit for bit; given
  the same Z this holds for UOT as well.  The iterations and the estimate
  use the platform's exp and log.
* Empty rows/columns (no sampled entry): OT renormalises a and b over the
  non-empty support ("renormalize"); UOT sets u_i = 0 there ("zero"), the
  exact optimum of the sparse UOT problem for that row.
* Stopping: the L1 marginal error of the iterate (u^t, v^t) on the matrix that
  is iterated; for UOT the fixed-point residual
  sum |u^(1/th) (K~ v) - a| + sum |v^(1/th) (K~^T u) - b|, th = lam/(lam+eps),
  summed over rows/columns with at least one entry.  The paper's own rule
  (change of the scalings) is available as ``stop_rule="delta"``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .elementary import cos_spec, exp_spec, log_spec

# --------------------------------------------------------------------------
# Philox4x32-10 (Salmon et al., SC 2011), vectorised over counters.
# --------------------------------------------------------------------------
_PHILOX_M0 = np.uint64(0xD2511F53)
_PHILOX_M1 = np.uint64(0xCD9E8D57)
_PHILOX_W0 = 0x9E3779B9
_PHILOX_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)
_SH32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds.

    ctr: sequence of four uint32 arrays (broadcastable); key: (k0, k1) ints.
    Returns four uint32 arrays (as uint64 dtype holding 32-bit values).
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK32 for c in ctr)
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for _ in range(10):
        p0 = _PHILOX_M0 * c0
        p1 = _PHILOX_M1 * c2
        hi0, lo0 = p0 >> _SH32, p0 & _MASK32
        hi1, lo1 = p1 >> _SH32, p1 & _MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0
        k0 = (k0 + _PHILOX_W0) & 0xFFFFFFFF
        k1 = (k1 + _PHILOX_W1) & 0xFFFFFFFF
    return c0, c1, c2, c3


def uniform_bits(i, j, problem_index: int, seed: int):
    """48-bit hash word for entries (i, j) (broadcast arrays) of one problem."""
    i = np.asarray(i, dtype=np.uint64)
    j = np.asarray(j, dtype=np.uint64)
    q = (j >> np.uint64(9)) * np.uint64(64) + (j & np.uint64(63))
    slot = ((j >> np.uint64(6)) & np.uint64(7)).astype(np.int64)
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    k = np.uint64(problem_index)
    coarse = philox4x32_10((q, i, k, np.uint64(0)), key)
    word = np.choose(slot >> 1, coarse)
    hi = (word >> (np.uint64(16) * (slot & 1).astype(np.uint64))) & np.uint64(0xFFFF)
    fine_a = philox4x32_10((q, i, k, np.uint64(1)), key)
    fine_b = philox4x32_10((q, i, k, np.uint64(2)), key)
    lo = np.where(slot < 4, np.choose(slot & 3, fine_a), np.choose(slot & 3, fine_b))
    return (hi << _SH32) | lo


def uniform01(i, j, problem_index: int, seed: int):
    """U_ij = bits * 2^-48, exactly representable in float64."""
    return uniform_bits(i, j, problem_index, seed).astype(np.float64) * 2.0 ** -48


# --------------------------------------------------------------------------
# Small helpers with a plain definition.
# --------------------------------------------------------------------------
def tree_sum(v) -> float:
    """Perfect binary-tree sum of v zero-padded to a power of two."""
    v = np.asarray(v, dtype=np.float64).ravel()
    if v.size == 0:
        return 0.0
    size = 1 << (v.size - 1).bit_length()
    w = np.zeros(size)
    w[: v.size] = v
    while w.size > 1:
        w = w[0::2] + w[1::2]
    return float(w[0])


def sq_dist(x, y):
    """c_ij = sum_k (x_ik - y_jk)^2, accumulated in k order (x: (r,d), y: (c,d))."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    diff = x[:, None, 0] - y[None, :, 0]
    acc = diff * diff
    for k in range(1, x.shape[1]):
        diff = x[:, None, k] - y[None, :, k]
        acc = acc + diff * diff
    return acc


def _map_chunks(fn, starts, workers: int) -> list:
    """[fn(r0) for r0 in starts], optionally on a thread pool (numpy releases
    the interpreter lock in its array loops); the results keep the order of
    `starts`, so every caller's arithmetic is the same for any `workers`."""
    starts = list(starts)
    if workers <= 1:
        return [fn(r0) for r0 in starts]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, starts))


def max_sq_dist(x, y, chunk: int = 512, workers: int = 1) -> float:
    """max_ij c_ij (the maximum does not depend on the order of the scan)."""
    maxima = _map_chunks(lambda r0: float(sq_dist(x[r0:r0 + chunk], y).max()),
                         range(0, x.shape[0], chunk), workers)
    return max([0.0] + maxima)


def kl_div(x, y) -> float:
    """KL(x||y) = sum x log(x/y) - x + y with 0 log 0 = 0 (Sec. 2 notation)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    pos = x > 0
    out = np.zeros_like(x)
    out[pos] = x[pos] * np.log(x[pos] / y[pos])
    return float(np.sum(out - x + y))


# --------------------------------------------------------------------------
# Options and the problem's derived scalars.
# --------------------------------------------------------------------------
@dataclass
class Options:
    eps: float
    s: float
    lam: float = math.inf          # inf => balanced OT
    tol: float = 1e-6
    max_iter: int = 1000
    seed: int = 0
    problem_index: int = 0
    cost: str = "maxnorm"          # "maxnorm" (C = c / max c), "plain" (C = c),
                                   # "euclid" (C = sqrt c), "wfr"
    empty_policy: str = "auto"     # auto | renormalize | zero | fail
    stop_rule: str = "marginal"    # marginal | delta
    log_domain: bool = False
    # weight g of the uniform probability 1/(nm) mixed into the sampling
    # probability (Sec. 4, shrinkage: p = (1 - g) p + g / (nm)); g = 1 is the
    # equal-probability subsampling of Sec. 5 (Rand-Sink)
    shrink: float = 0.0
    # eta of the Wasserstein-Fisher-Rao cost (cost="wfr")
    eta: float = 1.0


class EmptySupportError(RuntimeError):
    pass


class NonFiniteError(RuntimeError):
    """A scaling became NaN or +inf (the library reports SS_E_NONFINITE)."""


def is_uot(opt: Options) -> bool:
    return math.isfinite(opt.lam)


def cost_scale(x, y, opt: Options, workers: int = 1) -> tuple[float, float]:
    """(cmax, inv_cmax) -- C_ij = c_ij * inv_cmax for the squared Euclidean
    costs (cmax is reported for every cost)."""
    cmax = max_sq_dist(x, y, workers=workers)
    if opt.cost == "maxnorm":
        return cmax, (1.0 / cmax if cmax > 0 else 1.0)
    return cmax, 1.0


HALF_PI = math.pi / 2


def cost_from_sq(c, kind: str, inv_cmax: float, eta: float):
    """C from squared Euclidean distances c.  "maxnorm" / "plain": c * inv_cmax.
    "euclid": the Euclidean distance sqrt(c) (the distance the generative-
    modelling section names; correctly rounded square root).
    "wfr": the Wasserstein-Fisher-Rao cost of the UOT background section,
    C = -log cos_+^2(d / (2 eta)) with the Euclidean distance d = sqrt(c) and
    cos_+(z) = cos(min(z, pi/2)); written -2 log cos(z) with
    z = sqrt(c) * (0.5 / eta), and +inf (K = 0) where z >= pi/2, which the
    section states for d >= pi eta."""
    if kind == "euclid":
        return np.sqrt(c)
    if kind != "wfr":
        return c * inv_cmax
    z = np.sqrt(c) * (0.5 / eta)
    inside = z < HALF_PI
    out = np.full(np.shape(z), np.inf)
    out[inside] = -2.0 * log_spec(cos_spec(z[inside]))
    return out


# --------------------------------------------------------------------------
# Sampling probabilities: eq. (pij-ot) and eq. (pij-uot), then eq. (pois).
# --------------------------------------------------------------------------
@dataclass
class ProbOT:
    alpha: np.ndarray   # (1 - g) s sqrt(a_i) / (S_a S_b)
    rb: np.ndarray      # sqrt(b_j)
    s_a: float
    s_b: float
    c0: float = 0.0     # s g / (nm): the uniform part of s p

    def pstar(self, rows, cols):
        return np.minimum(1.0, self.alpha[rows][:, None] * self.rb[cols][None, :] + self.c0)


def shrink_terms(s, shrink, n, m) -> tuple[float, float]:
    """(1 - g, s g / (nm)): s p = (1 - g) s p_ij + s g / (nm) (Sec. 4, shrinkage)."""
    return 1.0 - shrink, s * shrink / (float(n) * float(m))


def ot_probabilities(a, b, s, shrink: float = 0.0) -> ProbOT:
    """eq. (pij-ot): p_ij = sqrt(a_i) sqrt(b_j) / (sum_i sqrt(a_i) sum_j sqrt(b_j)),
    mixed with the uniform probability with weight `shrink`."""
    ra = np.sqrt(np.asarray(a, dtype=np.float64))
    rb = np.sqrt(np.asarray(b, dtype=np.float64))
    s_a, s_b = tree_sum(ra), tree_sum(rb)
    kappa = s / (s_a * s_b)
    w, c0 = shrink_terms(s, shrink, ra.size, rb.size)
    return ProbOT(alpha=(kappa * ra) * w, rb=rb, s_a=s_a, s_b=s_b, c0=c0)


@dataclass
class ProbUOT:
    la: np.ndarray      # th_u * log a_i
    lb: np.ndarray      # th_u * log b_j
    inv_tau: float      # 1 / (2 lam + eps)
    inv_cmax: float
    z: float            # sum_ij q_ij
    kappa: float        # (1 - g) s / z
    x: np.ndarray
    y: np.ndarray
    c0: float = 0.0     # s g / (nm)
    cost: str = "maxnorm"
    eta: float = 1.0

    def exponent(self, rows, cols):
        """(la_i + lb_j) - C_ij / (2 lam + eps), the log of q_ij."""
        cij = cost_from_sq(sq_dist(self.x[rows], self.y[cols]), self.cost, self.inv_cmax,
                           self.eta)
        with np.errstate(invalid="ignore"):
            return (self.la[rows][:, None] + self.lb[cols][None, :]) - cij * self.inv_tau

    def q(self, rows, cols):
        return exp_spec(self.exponent(rows, cols))

    def pstar(self, rows, cols):
        return np.minimum(1.0, self.kappa * self.q(rows, cols) + self.c0)


def uot_probabilities(a, b, x, y, s, lam, eps, inv_cmax, chunk: int = 256,
                      shrink: float = 0.0, workers: int = 1, cost: str = "maxnorm",
                      eta: float = 1.0) -> ProbUOT:
    """eq. (pij-uot) with K^(eps/(2lam+eps)) written as exp(-C/(2lam+eps)),
    mixed with the uniform probability with weight `shrink`.

    Z = sum_ij q_ij is a sum of nm terms whose rounding order neither side
    fixes, so its last bits are not part of the specification; it is formed
    here with the platform exponential of the same exponents (each term
    within an ulp or two of exp_spec's, Z within ~1e-15 relative) because the
    nm specified exponentials cost too much at n = 65536.  Every keep
    decision and stored value takes Z as given: the library's ss_sample
    accepts the oracle's Z (z_in) and then matches bit for bit."""
    tau = 2.0 * lam + eps
    th = lam / tau
    la = th * log_spec(np.asarray(a, dtype=np.float64))
    lb = th * log_spec(np.asarray(b, dtype=np.float64))
    pr = ProbUOT(la=la, lb=lb, inv_tau=1.0 / tau, inv_cmax=inv_cmax, z=0.0, kappa=0.0,
                 x=np.asarray(x, np.float64), y=np.asarray(y, np.float64), cost=cost, eta=eta)
    cols = np.arange(len(b))
    rowsums = _map_chunks(
        lambda r0: np.exp(pr.exponent(np.arange(r0, min(len(a), r0 + chunk)), cols)).sum(axis=1),
        range(0, len(a), chunk), workers)
    pr.z = float(np.sum(np.concatenate(rowsums)))
    w, pr.c0 = shrink_terms(s, shrink, len(a), len(b))
    pr.kappa = w * (s / pr.z)
    return pr


# --------------------------------------------------------------------------
# eq. (pois): the Poisson mask and the sparse sketch K~ = K / p* (CSR, CSC).
# --------------------------------------------------------------------------
@dataclass
class Sketch:
    n: int
    m: int
    mask: np.ndarray        # (n, ceil(m/64)) uint64, bit j&63 of word j>>6
    row_ptr: np.ndarray     # (n+1,) int64
    col_idx: np.ndarray     # (nnz,) int32, ascending within a row
    val: np.ndarray         # (nnz,) float64, K~_ij = K_ij / p*_ij
    logval: np.ndarray      # (nnz,) float64, -C_ij/eps - log p*_ij
    cost: np.ndarray        # (nnz,) float64, C_ij of each kept entry
    pstar: np.ndarray       # (nnz,) float64
    col_ptr: np.ndarray     # (m+1,) int64
    row_idx: np.ndarray     # (nnz,) int32, ascending within a column
    val_t: np.ndarray       # (nnz,) float64 (CSC order)
    logval_t: np.ndarray
    cmax: float
    inv_cmax: float
    prob: object

    @property
    def nnz(self) -> int:
        return int(self.col_idx.size)

    def csr(self):
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.m))


def _pack_mask(keep: np.ndarray) -> np.ndarray:
    n, m = keep.shape
    words = (m + 63) // 64
    padded = np.zeros((n, words * 64), dtype=bool)
    padded[:, :m] = keep
    packed = np.packbits(padded, axis=1, bitorder="little")
    return packed.view("<u8").reshape(n, words).astype(np.uint64)


def sample_rows(x, y, a, b, opt: Options, rows, prob=None, inv_cmax=None):
    """Keep-decisions, p* and U for the given rows over all columns."""
    m = len(b)
    cols = np.arange(m)
    rows = np.asarray(rows)
    pst = prob.pstar(rows, cols)
    u01 = uniform01(rows[:, None], cols[None, :], opt.problem_index, opt.seed)
    keep = u01 < pst
    return keep, pst, u01


def build_sketch(x, y, a, b, opt: Options, chunk: int = 256, prob=None,
                 workers: int = 1) -> Sketch:
    """Alg. 3/4 step 1: construct K~ by eq. (pois) with eq. (pij-ot)/(pij-uot),
    or with the given probabilities `prob` (an object with pstar(rows, cols)).
    `workers` > 1 scans row chunks on a thread pool; every decision and value
    is the same."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    n, m = x.shape[0], y.shape[0]
    cmax, inv_cmax = cost_scale(x, y, opt, workers=workers)
    if prob is not None:
        pass
    elif is_uot(opt):
        prob = uot_probabilities(a, b, x, y, opt.s, opt.lam, opt.eps, inv_cmax,
                                 shrink=opt.shrink, cost=opt.cost, eta=opt.eta, workers=workers)
    else:
        prob = ot_probabilities(a, b, opt.s, shrink=opt.shrink)

    def one_chunk(r0):
        rows = np.arange(r0, min(n, r0 + chunk))
        keep, pst, _ = sample_rows(x, y, a, b, opt, rows, prob)
        rr, cc = np.nonzero(keep)
        return _pack_mask(keep), rows[rr], cc, pst[rr, cc]

    parts = _map_chunks(one_chunk, range(0, n, chunk), workers)
    masks = [q[0] for q in parts]
    ri = [q[1] for q in parts]
    ci = [q[2] for q in parts]
    pvals = [q[3] for q in parts]
    mask = np.concatenate(masks, axis=0) if masks else np.zeros((0, (m + 63) // 64), np.uint64)
    ri = np.concatenate(ri).astype(np.int64) if ri else np.zeros(0, np.int64)
    ci = np.concatenate(ci).astype(np.int64) if ci else np.zeros(0, np.int64)
    ps = np.concatenate(pvals) if pvals else np.zeros(0)
    # Entry values: C recomputed from the coordinates, K = exp(-C/eps).
    cvals = np.array([sq_dist(x[i:i + 1], y[j:j + 1])[0, 0] for i, j in zip(ri, ci)]) \
        if ri.size < 4096 else _pair_sq_dist(x, y, ri, ci)
    cost = cost_from_sq(cvals, opt.cost, inv_cmax, opt.eta)
    kval = exp_spec(-(cost / opt.eps))
    val = kval / ps
    logval = -(cost / opt.eps) - log_spec(ps)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(ri, minlength=n), out=row_ptr[1:])
    # CSC: stable order by (column, row).
    order = np.lexsort((ri, ci))
    col_ptr = np.zeros(m + 1, np.int64)
    np.cumsum(np.bincount(ci, minlength=m), out=col_ptr[1:])
    return Sketch(n=n, m=m, mask=mask, row_ptr=row_ptr, col_idx=ci.astype(np.int32),
                  val=val, logval=logval, cost=cost, pstar=ps, col_ptr=col_ptr,
                  row_idx=ri[order].astype(np.int32), val_t=val[order],
                  logval_t=logval[order], cmax=cmax, inv_cmax=inv_cmax, prob=prob)


def _pair_sq_dist(x, y, ri, ci):
    diff = x[ri, 0] - y[ci, 0]
    acc = diff * diff
    for k in range(1, x.shape[1]):
        diff = x[ri, k] - y[ci, k]
        acc = acc + diff * diff
    return acc


def expected_nnz_ot(prob: ProbOT) -> tuple[float, float]:
    """E[nnz] = sum p*, Var[nnz] = sum p*(1-p*) (eq. (pois) and its remark)."""
    e, v = 0.0, 0.0
    for i in range(prob.alpha.size):
        p = np.minimum(1.0, prob.alpha[i] * prob.rb + prob.c0)
        e += p.sum()
        v += (p * (1 - p)).sum()
    return e, v


# --------------------------------------------------------------------------
# Empty rows / columns.
# --------------------------------------------------------------------------
def apply_empty_policy(a, b, row_cnt, col_cnt, opt: Options):
    """Returns (a_eff, b_eff, row_active, col_active, dropped_a, dropped_b)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    ra = row_cnt > 0
    ca = col_cnt > 0
    dropped_a = float(a[~ra].sum())
    dropped_b = float(b[~ca].sum())
    policy = opt.empty_policy
    if policy == "auto":
        policy = "zero" if is_uot(opt) else "renormalize"
    if policy == "fail" and (np.any(~ra & (a > 0)) or np.any(~ca & (b > 0))):
        raise EmptySupportError("empty row or column in the sparse sketch")
    a_eff = np.where(ra, a, 0.0)
    b_eff = np.where(ca, b, 0.0)
    if policy == "renormalize":
        a_eff = a_eff / a_eff.sum()
        b_eff = b_eff / b_eff.sum()
    return a_eff, b_eff, ra, ca, dropped_a, dropped_b


# --------------------------------------------------------------------------
# Alg. 1 / Alg. 2 on a given (sparse or dense) kernel.
# --------------------------------------------------------------------------
@dataclass
class SinkhornResult:
    u: np.ndarray
    v: np.ndarray
    iters: int
    err: float
    hist: list
    converged: bool
    # log-domain runs: the potentials f = log u, g = log v themselves (exp(f)
    # may overflow where f is finite)
    log_u: np.ndarray | None = None
    log_v: np.ndarray | None = None

    def logs(self):
        """(log u, log v), from the potentials where the run kept them."""
        if self.log_u is not None:
            return self.log_u, self.log_v
        with np.errstate(divide="ignore"):
            return np.log(self.u), np.log(self.v)


def _quotient(num, den, th):
    """(num / den)^th on positions with den > 0; 0 elsewhere."""
    out = np.zeros_like(num)
    pos = den > 0
    q = num[pos] / den[pos]
    out[pos] = q if th == 1.0 else q ** th
    return out


def marginal_error(K, KT, u, v, a, b, th, row_active, col_active) -> float:
    """Sum |u^(1/th) (K v) - a| + sum |v^(1/th) (K^T u) - b| over active rows/cols."""
    kv = K @ v
    ktu = KT @ u
    up = u if th == 1.0 else u ** (1.0 / th)
    vp = v if th == 1.0 else v ** (1.0 / th)
    # only active lines enter (an empty line's scaling may be infinite)
    ra, ca = row_active, col_active
    err = float(np.abs(up[ra] * kv[ra] - a[ra]).sum() + np.abs(vp[ca] * ktu[ca] - b[ca]).sum())
    if math.isnan(err):
        raise NonFiniteError("the marginal error is NaN")
    return err


def _check_finite(u, v):
    """Linear domain: every scaling finite (empty lines hold 0)."""
    if not (np.all(np.isfinite(u)) and np.all(np.isfinite(v))):
        raise NonFiniteError("a scaling is not finite")


def _check_finite_log(f, g):
    """Log domain: no potential NaN or +inf (-inf is a zero scaling)."""
    for p in (f, g):
        if np.any(np.isnan(p)) or np.any(p == np.inf):
            raise NonFiniteError("a potential is NaN or +inf")


def sinkhorn(K, a, b, opt: Options, row_active=None, col_active=None, u0=None, v0=None):
    """Alg. 1 (th = 1) / Alg. 2 (th = lam/(lam+eps)), linear domain.

    The loop stops at the first t with err(u^t, v^t) <= tol, or at max_iter.
    """
    n, m = K.shape
    th = opt.lam / (opt.lam + opt.eps) if is_uot(opt) else 1.0
    row_active = np.ones(n, bool) if row_active is None else row_active
    col_active = np.ones(m, bool) if col_active is None else col_active
    KT = K.T.tocsr() if sp.issparse(K) else K.T
    u = np.where(row_active, 1.0, 0.0) if u0 is None else np.array(u0, np.float64)
    v = np.where(col_active, 1.0, 0.0) if v0 is None else np.array(v0, np.float64)
    hist = []
    err = math.inf
    t = 0
    for t in range(1, opt.max_iter + 1):
        u_prev, v_prev = u, v
        with np.errstate(over="ignore"):
            u = _quotient(a, K @ v, th)
            v = _quotient(b, KT @ u, th)
        _check_finite(u, v)
        if opt.stop_rule == "delta":
            err = float(np.abs(u - u_prev).sum() + np.abs(v - v_prev).sum())
        else:
            err = marginal_error(K, KT, u, v, a, b, th, row_active, col_active)
        hist.append(err)
        if err <= opt.tol:
            break
    return SinkhornResult(u=u, v=v, iters=t, err=err, hist=hist, converged=err <= opt.tol)


def _segment_logsumexp(z, seg_ptr):
    """log sum exp over CSR segments; -inf for empty segments."""
    n = seg_ptr.size - 1
    out = np.full(n, -np.inf)
    for i in range(n):
        lo, hi = seg_ptr[i], seg_ptr[i + 1]
        if hi > lo:
            zz = z[lo:hi]
            mx = zz.max()
            out[i] = mx + math.log(np.exp(zz - mx).sum())
    return out


def sinkhorn_log(sk: Sketch, a, b, opt: Options, row_active, col_active, f0=None, g0=None):
    """Log-domain Alg. 1/2 on K~: f = log u, g = log v, with
    f_i = th (log a_i - log sum_j exp(l_ij + g_j)),  l_ij = log K~_ij
    (appendix, proof of Thm. 3: the same update with C~ = C + eps log p*)."""
    th = opt.lam / (opt.lam + opt.eps) if is_uot(opt) else 1.0
    order_rows = sk.row_idx.astype(np.int64)
    l_r, c_r = sk.logval, sk.col_idx.astype(np.int64)
    l_c = sk.logval_t
    with np.errstate(divide="ignore"):
        la, lb = np.log(a), np.log(b)
    f = np.zeros(sk.n) if f0 is None else np.array(f0, np.float64)
    g = np.zeros(sk.m) if g0 is None else np.array(g0, np.float64)
    f[~row_active] = -np.inf
    g[~col_active] = -np.inf
    hist = []
    err = math.inf
    t = 0
    for t in range(1, opt.max_iter + 1):
        f_prev, g_prev = f, g
        lse_r = _segment_logsumexp(l_r + g[c_r], sk.row_ptr)
        with np.errstate(invalid="ignore"):
            f = np.where(row_active, th * (la - lse_r), -np.inf)
        lse_c = _segment_logsumexp(l_c + f[order_rows], sk.col_ptr)
        with np.errstate(invalid="ignore"):
            g = np.where(col_active, th * (lb - lse_c), -np.inf)
        _check_finite_log(f, g)
        if opt.stop_rule == "delta":
            err = float(np.abs(np.exp(f) - np.exp(f_prev)).sum()
                        + np.abs(np.exp(g) - np.exp(g_prev)).sum())
        else:
            lse_r2 = _segment_logsumexp(l_r + g[c_r], sk.row_ptr)
            lse_c2 = _segment_logsumexp(l_c + f[order_rows], sk.col_ptr)
            r_row = np.abs(np.exp(f / th + lse_r2) - a)[row_active].sum()
            r_col = np.abs(np.exp(g / th + lse_c2) - b)[col_active].sum()
            err = float(r_row + r_col)
        hist.append(err)
        if err <= opt.tol:
            break
    with np.errstate(over="ignore"):
        u, v = np.exp(f), np.exp(g)
    return SinkhornResult(u=u, v=v, iters=t, err=err, hist=hist, log_u=f, log_v=g,
                          converged=err <= opt.tol)


# --------------------------------------------------------------------------
# Alg. 3 / Alg. 4 output: <T~, C> - eps H(T~) (+ lam KL terms for UOT).
# --------------------------------------------------------------------------
@dataclass
class Estimate:
    estimate: float
    transport: float
    neg_entropy: float       # sum T (log T - 1) = -H(T)
    kl_a: float
    kl_b: float
    sparse_objective: float  # <T~, C~> - eps H(T~) (+ lam KLs), C~ = -eps log K~


def estimate_from_entries(rows, cols, t, cost, u, v, a, b, opt: Options,
                          logs=None) -> Estimate:
    """`logs` = (log u, log v) where the run kept its potentials."""
    pos = t > 0
    # entries with t = 0 carry no transport, also where C = +inf (WFR)
    transport = float(np.sum(t[pos] * cost[pos]))
    neg_ent = float(np.sum(t[pos] * (np.log(t[pos]) - 1.0)))
    row_sum = np.bincount(rows, weights=t, minlength=len(a))
    col_sum = np.bincount(cols, weights=t, minlength=len(b))
    if logs is not None:
        lu, lv = logs
    else:
        with np.errstate(divide="ignore"):
            lu, lv = np.log(u), np.log(v)
    sparse_obj = opt.eps * float(np.sum(t[pos] * (lu[rows[pos]] + lv[cols[pos]] - 1.0)))
    est = transport + opt.eps * neg_ent
    kl_a = kl_b = 0.0
    if is_uot(opt):
        kl_a = kl_div(row_sum, a)
        kl_b = kl_div(col_sum, b)
        est += opt.lam * (kl_a + kl_b)
        sparse_obj += opt.lam * (kl_a + kl_b)
    return Estimate(est, transport, neg_ent, kl_a, kl_b, sparse_obj)


# --------------------------------------------------------------------------
# Entry points mirroring the library's calls.
# --------------------------------------------------------------------------
@dataclass
class SolveResult:
    estimate: Estimate
    sinkhorn: SinkhornResult
    sketch: Sketch | None
    nnz: int
    empty_rows: int
    empty_cols: int
    dropped_a: float
    dropped_b: float
    cmax: float


def spar_sink(x, y, a, b, opt: Options, workers: int = 1) -> SolveResult:
    """Alg. 3 (OT, lam = inf) and Alg. 4 (UOT).  `workers`: threads of the
    sketch's full scans (the result does not depend on it)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    sk = build_sketch(x, y, a, b, opt, workers=workers)
    row_cnt = np.diff(sk.row_ptr)
    col_cnt = np.diff(sk.col_ptr)
    a_eff, b_eff, ra, ca, da, db = apply_empty_policy(a, b, row_cnt, col_cnt, opt)
    rows = np.repeat(np.arange(sk.n), row_cnt)
    cols = sk.col_idx.astype(np.int64)
    if opt.log_domain:
        res = sinkhorn_log(sk, a_eff, b_eff, opt, ra, ca)
        lu, lv = res.logs()
        t = np.exp(lu[rows] + sk.logval + lv[cols])
    else:
        res = sinkhorn(sk.csr(), a_eff, b_eff, opt, ra, ca)
        t = res.u[rows] * sk.val * res.v[cols]
    est = estimate_from_entries(rows, cols, t, sk.cost, res.u, res.v, a, b, opt, res.logs())
    return SolveResult(est, res, sk, sk.nnz, int(np.sum(~ra & (a > 0))),
                       int(np.sum(~ca & (b > 0))), da, db, sk.cmax)


def dense_sinkhorn(x, y, a, b, opt: Options) -> SolveResult:
    """Alg. 1 / Alg. 2 on the full kernel K = exp(-C/eps)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    cmax, inv_cmax = cost_scale(x, y, opt)
    cost = cost_from_sq(sq_dist(x, y), opt.cost, inv_cmax, opt.eta)
    K = exp_spec(-(cost / opt.eps))
    n, m = K.shape
    if opt.log_domain:
        sk = _dense_as_sketch(cost, opt, cmax, inv_cmax)
        res = sinkhorn_log(sk, a, b, opt, np.ones(n, bool), np.ones(m, bool))
        lu, lv = res.logs()
        t = np.exp(lu[:, None] - cost / opt.eps + lv[None, :])
    else:
        res = sinkhorn(K, a, b, opt)
        t = res.u[:, None] * K * res.v[None, :]
    rows = np.repeat(np.arange(n), m)
    cols = np.tile(np.arange(m), n)
    est = estimate_from_entries(rows, cols, t.ravel(), cost.ravel(), res.u, res.v, a, b, opt,
                                res.logs())
    return SolveResult(est, res, None, n * m, 0, 0, 0.0, 0.0, cmax)


def _dense_as_sketch(cost, opt, cmax, inv_cmax) -> Sketch:
    n, m = cost.shape
    logval = -(cost / opt.eps)
    row_ptr = np.arange(0, n * m + 1, m, dtype=np.int64)
    col_ptr = np.arange(0, n * m + 1, n, dtype=np.int64)
    return Sketch(n=n, m=m, mask=np.zeros((n, 0), np.uint64), row_ptr=row_ptr,
                  col_idx=np.tile(np.arange(m), n).astype(np.int32), val=exp_spec(logval).ravel(),
                  logval=logval.ravel(), cost=cost.ravel(), pstar=np.ones(n * m),
                  col_ptr=col_ptr, row_idx=np.tile(np.arange(n), m).astype(np.int32),
                  val_t=exp_spec(logval.T).ravel(), logval_t=logval.T.ravel(), cmax=cmax,
                  inv_cmax=inv_cmax, prob=None)
