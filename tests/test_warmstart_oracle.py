"""Pins of the FP64 warm-start oracle (no GPU).

The hand-written backward pass is checked against central finite differences
and against torch.autograd (FP64, CPU) applied to an independent expression
of the same network; the forward pass against invariances it must have and a
closed form."""
import numpy as np
import pytest
import torch

from oracle import warmstart_oracle as WO


def _problem(rng, n=7, m=5):
    x, y = rng.standard_normal((n, 3)), rng.standard_normal((m, 3)) + 0.5
    a, b = rng.dirichlet(np.ones(n)), rng.dirichlet(np.ones(m))
    lu, lv = rng.standard_normal(n) + np.log(a), rng.standard_normal(m) + np.log(b)
    return x, a, y, b, lu, lv


def _small_params(H=6, seed=1):
    par = WO.init_params(H, seed)
    rng = np.random.default_rng(seed + 10)
    par.p = rng.standard_normal(H) * 0.3
    par.c2 = rng.standard_normal(H) * 0.3
    par.c3 = np.array([0.2])
    return par


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    probs = [_problem(rng, 7, 5), _problem(rng, 4, 9)]
    par = _small_params()
    _, g = WO.batch_loss_and_grad(par, probs)
    h = 1e-6
    for name in WO.PARAM_NAMES:
        arr = getattr(par, name)
        ga = np.ravel(getattr(g, name))
        for idx in range(min(arr.size, 12)):
            p1, p2 = par.copy(), par.copy()
            np.ravel(getattr(p1, name))[idx] += h
            np.ravel(getattr(p2, name))[idx] -= h
            fd = (WO.batch_loss_and_grad(p1, probs)[0] - WO.batch_loss_and_grad(p2, probs)[0]) / (2 * h)
            assert ga[idx] == pytest.approx(fd, rel=1e-5, abs=1e-8), (name, idx)


def test_gradient_matches_autograd():
    rng = np.random.default_rng(1)
    probs = [_problem(rng, 6, 8), _problem(rng, 9, 3)]
    par = _small_params(H=8, seed=3)
    loss, g = WO.batch_loss_and_grad(par, probs)
    T = {n: torch.tensor(np.array(getattr(par, n)), dtype=torch.float64, requires_grad=True)
         for n in WO.PARAM_NAMES}

    def side(z, o, q, t, mask):
        z, o, q = (torch.tensor(v, dtype=torch.float64) for v in (z, o, q))
        f = torch.cat([o, (o.shape[0] * q)[:, None]], 1)
        e = torch.relu(f @ T["P"].T + T["p"]).mean(0)
        h1 = torch.relu(z @ T["W1"].T + (T["U"] @ e + T["c1"]))
        psi = torch.relu(h1 @ T["W2"].T + T["c2"]) @ T["w3"] + T["c3"][0]
        mk = torch.tensor(mask)
        d = (psi - torch.tensor(t))[mk]
        return ((d - d.mean()) ** 2).mean()

    total = 0
    for x, a, y, b, lu, lv in probs:
        for z, w, o, q, t, mask in WO.problem_sides(x, a, y, b, lu, lv):
            total = total + side(z, o, q, t, mask) / (2 * len(probs))
    total.backward()
    assert total.item() == pytest.approx(loss, rel=1e-12)
    for n in WO.PARAM_NAMES:
        np.testing.assert_allclose(np.ravel(getattr(g, n)), T[n].grad.numpy().ravel(),
                                   rtol=1e-10, atol=1e-14)


def test_embedding_is_permutation_invariant_and_loss_shift_invariant():
    rng = np.random.default_rng(2)
    x, a, y, b, lu, lv = _problem(rng, 8, 11)
    par = _small_params(H=10, seed=4)
    perm = rng.permutation(len(y))
    psi1, _ = WO.side_forward(par, x, y, b)
    psi2, _ = WO.side_forward(par, x, y[perm], b[perm])
    np.testing.assert_allclose(psi1, psi2, rtol=1e-13, atol=1e-13)
    l1, g1 = WO.batch_loss_and_grad(par, [(x, a, y, b, lu, lv)])
    l2, g2 = WO.batch_loss_and_grad(par, [(x, a, y, b, lu + 3.7, lv - 1.1)])
    assert l1 == pytest.approx(l2, rel=1e-12)
    np.testing.assert_allclose(g1.flat(), g2.flat(), rtol=1e-9, atol=1e-12)


def test_constant_network_closed_form():
    # W2 = 0 and w3 = 0: psi is the constant c3, the loss is the variance of
    # the targets over the masked points and the bias gets no gradient
    rng = np.random.default_rng(3)
    x, a, y, b, lu, lv = _problem(rng, 6, 6)
    lv[2] = -np.inf  # an empty column: excluded from the mask
    par = _small_params(H=5, seed=5)
    par.W2[:] = 0.0
    par.w3[:] = 0.0
    loss, g = WO.batch_loss_and_grad(par, [(x, a, y, b, lu, lv)])
    tu = lu - np.log(a)
    tv = (lv - np.log(b))[np.isfinite(lv)]
    assert loss == pytest.approx(0.5 * (tu.var() + tv.var()), rel=1e-12)
    assert abs(g.c3[0]) < 1e-14
    pu, pv = WO.predict(par, x, a, y, b)
    np.testing.assert_allclose(pu, np.log(a) + par.c3[0], rtol=1e-14)


def test_adam_first_step_moves_by_lr():
    par = _small_params(H=4, seed=6)
    g = WO.Params.zeros(4)
    g.W2[:] = 3.0
    g.c3[:] = -0.5
    m1, m2 = WO.Params.zeros(4), WO.Params.zeros(4)
    before = par.copy()
    WO.adam_step(par, g, m1, m2, t=1, lr=1e-3)
    np.testing.assert_allclose(par.W2, before.W2 - 1e-3, rtol=0, atol=1e-10)
    np.testing.assert_allclose(par.c3, before.c3 + 1e-3, rtol=0, atol=1e-10)
    np.testing.assert_allclose(par.U, before.U)  # zero gradient, zero step


def test_normalisation_makes_the_kernel_unit_free():
    # kernel units: exp(-|x' - y'|^2) is the Gibbs kernel of eq. (rot) with the
    # max-normalised cost, and a common shift of both clouds changes nothing
    rng = np.random.default_rng(7)
    x, y = rng.standard_normal((9, 3)), rng.standard_normal((6, 3)) + 2.0
    eps = 0.05
    xs, ys = WO.normalise(x, y, eps)
    d2 = ((x[:, None] - y[None]) ** 2).sum(-1)
    K = np.exp(-d2 / d2.max() / eps)
    Ks = np.exp(-((xs[:, None] - ys[None]) ** 2).sum(-1))
    np.testing.assert_allclose(Ks, K, rtol=1e-12)
    xs2, ys2 = WO.normalise(x + 5.0, y + 5.0, eps)
    np.testing.assert_allclose(xs2, xs, atol=1e-12)
    np.testing.assert_allclose(ys2, ys, atol=1e-12)
    np.testing.assert_allclose(xs2.mean(0) * 9 + ys2.mean(0) * 6, 0.0, atol=1e-10)
