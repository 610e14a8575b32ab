"""FP64 CPU reference of the learned warm start.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline
may import this module; the library never does, and it shares no code with
the HIP kernels.

A DeepSets-style network predicts initial scalings for Alg. 1.  Sinkhorn's
first update u^1 = a / (K v^0) reads only v^0, and (u, v) -> (c u, v / c)
leaves the plan unchanged (Sec. 2.1, eq. (rot-solu)), so only log v^0 up to
an additive constant matters: the loss is a centred (shift-invariant) squared
error of the predicted log-correction.  The same network is applied with the
roles of the two measures swapped to predict log u^0.

Inputs are the points of a problem centred on the mean of all its points
(both measures, unweighted) and divided by the kernel length sqrt(eps C_s)
with C_s = max_ij |x_i - y_j|^2 for the max-normalised cost (eq. (rot):
K = exp(-|x - y|^2 / (eps C_s)) becomes exp(-|x' - y'|^2)), C_s = 1 for the
plain cost.  For the side that predicts the scalings of points z_i (weights
w_i, count n) given the opposite measure (points o_j, weights q_j, count m),
all in these units:

    phi_j  = ReLU(P [o_j, m q_j] + p)            (4 -> H)
    e      = mean_j phi_j                        (H)
    g      = U e + c1                            (H)
    h1_i   = ReLU(W1 z_i + g)                    (3 -> H)
    h2_i   = ReLU(W2 h1_i + c2)                  (H -> H)
    psi_i  = w3 . h2_i + c3
    log y0_i = log w_i + psi_i

Loss of one side with target t_i = log y*_i - log w_i on the points with a
finite target (mask M): d = psi - t, L = mean_M (d - mean_M d)^2.  A batch
loss is the mean over problems and both sides.  The backward pass below is
written out by hand and checked against finite differences and against an
independent automatic differentiation in the tests.
"""
from __future__ import annotations

from dataclasses import dataclass, fields

import numpy as np

PARAM_NAMES = ("P", "p", "W1", "U", "c1", "W2", "c2", "w3", "c3")


@dataclass
class Params:
    P: np.ndarray    # (H, 4)
    p: np.ndarray    # (H,)
    W1: np.ndarray   # (H, 3)
    U: np.ndarray    # (H, H)
    c1: np.ndarray   # (H,)
    W2: np.ndarray   # (H, H)
    c2: np.ndarray   # (H,)
    w3: np.ndarray   # (H,)
    c3: np.ndarray   # (1,)

    @property
    def H(self) -> int:
        return int(self.p.shape[0])

    def copy(self) -> "Params":
        return Params(**{f.name: np.array(getattr(self, f.name), np.float64) for f in fields(self)})

    def flat(self) -> np.ndarray:
        return np.concatenate([np.ravel(getattr(self, n)) for n in PARAM_NAMES])

    @staticmethod
    def zeros(H: int) -> "Params":
        return Params(np.zeros((H, 4)), np.zeros(H), np.zeros((H, 3)), np.zeros((H, H)),
                      np.zeros(H), np.zeros((H, H)), np.zeros(H), np.zeros(H), np.zeros(1))


def init_params(H: int = 256, seed: int = 0) -> Params:
    """He-style initialisation (ReLU layers), zero biases except a small c1."""
    rng = np.random.default_rng(seed)
    return Params(P=rng.standard_normal((H, 4)) * np.sqrt(2.0 / 4),
                  p=np.zeros(H),
                  W1=rng.standard_normal((H, 3)) * np.sqrt(2.0 / 3),
                  U=rng.standard_normal((H, H)) * np.sqrt(1.0 / H),
                  c1=np.full(H, 0.01),
                  W2=rng.standard_normal((H, H)) * np.sqrt(2.0 / H),
                  c2=np.zeros(H),
                  w3=rng.standard_normal(H) * np.sqrt(1.0 / H),
                  c3=np.zeros(1))


def _relu(z):
    return np.maximum(z, 0.0)


def normalise(x, y, eps: float, cost: str = "maxnorm"):
    """x, y in kernel units: centred on the mean of all points, divided by
    sqrt(eps C_s)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    center = np.concatenate([x, y]).mean(axis=0)
    cs = 1.0
    if cost == "maxnorm":
        d2 = ((x[:, None, :] - y[None, :, :]) ** 2).sum(-1)
        cs = float(d2.max()) if d2.max() > 0 else 1.0
    scale = 1.0 / np.sqrt(eps * cs)
    return (x - center) * scale, (y - center) * scale


def side_forward(par: Params, z, o, q):
    """psi for points z (n, 3) given the opposite measure (o (m, 3), q (m,))."""
    z = np.asarray(z, np.float64)
    o = np.asarray(o, np.float64)
    q = np.asarray(q, np.float64)
    m = o.shape[0]
    f = np.concatenate([o, (m * q)[:, None]], axis=1)
    zphi = f @ par.P.T + par.p
    phi = _relu(zphi)
    e = phi.mean(axis=0)
    g = par.U @ e + par.c1
    z1 = z @ par.W1.T + g
    h1 = _relu(z1)
    z2 = h1 @ par.W2.T + par.c2
    h2 = _relu(z2)
    psi = h2 @ par.w3 + par.c3[0]
    cache = dict(z=z, f=f, zphi=zphi, e=e, z1=z1, h1=h1, z2=z2, h2=h2, m=m)
    return psi, cache


def side_loss(psi, target, mask):
    """Centred squared error over the masked points, and dL/dpsi."""
    mask = np.asarray(mask, bool)
    cnt = int(mask.sum())
    dpsi = np.zeros_like(psi)
    if cnt == 0:
        return 0.0, dpsi
    d = np.where(mask, psi - np.where(mask, target, 0.0), 0.0)
    dbar = d[mask].mean()
    r = np.where(mask, d - dbar, 0.0)
    loss = float((r[mask] ** 2).mean())
    dpsi = 2.0 * r / cnt   # the mean's own gradient sums to zero
    return loss, dpsi


def side_backward(par: Params, cache, dpsi) -> Params:
    """Gradients of sum_i dpsi_i psi_i with respect to every parameter."""
    gr = Params.zeros(par.H)
    h2, h1, z2, z1 = cache["h2"], cache["h1"], cache["z2"], cache["z1"]
    gr.w3 = h2.T @ dpsi
    gr.c3 = np.array([dpsi.sum()])
    dz2 = np.outer(dpsi, par.w3) * (z2 > 0)
    gr.W2 = dz2.T @ h1
    gr.c2 = dz2.sum(axis=0)
    dz1 = (dz2 @ par.W2) * (z1 > 0)
    gr.W1 = dz1.T @ cache["z"]
    dg = dz1.sum(axis=0)
    gr.c1 = dg
    gr.U = np.outer(dg, cache["e"])
    de = par.U.T @ dg
    dzphi = np.broadcast_to(de / cache["m"], cache["zphi"].shape) * (cache["zphi"] > 0)
    gr.P = dzphi.T @ cache["f"]
    gr.p = dzphi.sum(axis=0)
    return gr


def _add(acc: Params, g: Params, s: float):
    for n in PARAM_NAMES:
        setattr(acc, n, getattr(acc, n) + s * getattr(g, n))


def problem_sides(x, a, y, b, log_u, log_v):
    """The two sides of one problem: (points, weights, opposite points,
    opposite weights, target, mask) for the u-side and for the v-side."""
    out = []
    for z, w, o, q, ly in ((x, a, y, b, log_u), (y, b, x, a, log_v)):
        w = np.asarray(w, np.float64)
        ly = np.asarray(ly, np.float64)
        with np.errstate(divide="ignore", invalid="ignore"):
            t = ly - np.log(w)
        mask = np.isfinite(t)
        out.append((z, w, o, q, np.where(mask, t, 0.0), mask))
    return out


def batch_loss_and_grad(par: Params, problems, eps: float | None = None, cost="maxnorm"):
    """problems: list of (x, a, y, b, log_u*, log_v*).  Mean loss over
    problems and sides, and its gradient.  With eps the points are first put
    in kernel units (normalise); without, they are used as given."""
    total = 0.0
    grad = Params.zeros(par.H)
    nside = 2 * len(problems)
    for x, a, y, b, lu, lv in problems:
        if eps is not None:
            x, y = normalise(x, y, eps, cost)
        for z, w, o, q, t, mask in problem_sides(x, a, y, b, lu, lv):
            psi, cache = side_forward(par, z, o, q)
            loss, dpsi = side_loss(psi, t, mask)
            total += loss / nside
            _add(grad, side_backward(par, cache, dpsi), 1.0 / nside)
    return total, grad


def predict(par: Params, x, a, y, b, eps: float | None = None, cost="maxnorm"):
    """Initial log u^0, log v^0 (log w + psi on each side); with eps the
    points are first put in kernel units."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if eps is not None:
        x, y = normalise(x, y, eps, cost)
    psi_u, _ = side_forward(par, x, y, b)
    psi_v, _ = side_forward(par, y, x, a)
    with np.errstate(divide="ignore"):
        return np.log(a) + psi_u, np.log(b) + psi_v


def adam_step(par: Params, grad: Params, m1: Params, m2: Params, t: int, lr: float,
              beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma & Ba, ICLR 2015) with bias correction, in place."""
    for n in PARAM_NAMES:
        g = getattr(grad, n)
        a = beta1 * getattr(m1, n) + (1 - beta1) * g
        b = beta2 * getattr(m2, n) + (1 - beta2) * g * g
        setattr(m1, n, a)
        setattr(m2, n, b)
        ah = a / (1 - beta1 ** t)
        bh = b / (1 - beta2 ** t)
        setattr(par, n, getattr(par, n) - lr * ah / (np.sqrt(bh) + eps))
