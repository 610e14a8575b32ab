"""The learned warm start on the GPU against the FP64 oracle, and its gain.

The oracle runs with the BF16-rounded weights the kernels use, so the
remaining differences are BF16 activations into the matrix cores and FP32
accumulation: outputs within 2e-2, gradients within 5e-2 (relative L2 per
parameter block).  The gain test trains the network on problems of the
batched workload's law with the project's own kernels and checks that fresh
problems need fewer Sinkhorn iterations than from the plain start."""
import numpy as np
import pytest
import torch

from oracle import warmstart_oracle as WO
from paper_2306_06581_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_06581_amd import api as A
    return A


def _params(flat):
    out, off = {}, 0
    for name, shape in (("P", (256, 4)), ("p", (256,)), ("W1", (256, 3)), ("U", (256, 256)),
                        ("c1", (256,)), ("W2", (256, 256)), ("c2", (256,)), ("w3", (256,)),
                        ("c3", (1,))):
        k = int(np.prod(shape))
        out[name] = np.asarray(flat[off:off + k], np.float64).reshape(shape)
        off += k
    return WO.Params(**out)


def _problems(seed, sizes):
    rng = np.random.default_rng(seed)
    probs = []
    for k, (n, m) in enumerate(sizes):
        mu_x, mu_y = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
        x = mu_x + rng.standard_normal((n, 3))
        y = mu_y + rng.standard_normal((m, 3))
        a, b = rng.dirichlet(np.ones(n)), rng.dirichlet(np.ones(m))
        probs.append(W.Problem(x, y, a, b, eps=0.05, s=W.s_budget(max(n, 2), 8.0), seed=seed,
                               problem_index=k))
    return probs


SIZES = [(37, 50), (200, 180), (33, 17), (1, 5), (130, 129)]


def _targets(probs, seed):
    rng = np.random.default_rng(seed)
    tu, tv = [], []
    for p in probs:
        lu = np.log(p.a) + 0.7 * p.x[:, 0] - 0.3 * p.x[:, 2] + 0.1 * rng.standard_normal(p.n)
        lv = np.log(p.b) - 0.5 * p.y[:, 1] + 0.1 * rng.standard_normal(p.m)
        lv[0] = -np.inf  # an empty column: no target
        tu.append(lu)
        tv.append(lv)
    return tu, tv


def test_forward_matches_oracle(api):
    probs = _problems(1, SIZES)
    B = api.Batch.from_problems(probs)
    net = api.WarmStartNet(seed=3)
    par = _params(net.bf16_weights())
    lu, lv = net.predict(B, eps=0.05)
    lu, lv = lu.cpu().numpy(), lv.cpu().numpy()
    for k, p in enumerate(probs):
        ou, ov = WO.predict(par, p.x, p.a, p.y, p.b, eps=0.05)
        gu = lu[B.row_off[k]:B.row_off[k + 1]] - np.log(p.a)
        gv = lv[B.col_off[k]:B.col_off[k + 1]] - np.log(p.b)
        for g, o, w in ((gu, ou, p.a), (gv, ov, p.b)):
            ref = o - np.log(w)
            np.testing.assert_allclose(g, ref, rtol=2e-2, atol=2e-2 * max(1.0, np.abs(ref).max()))


def test_forward_matches_oracle_many_tiles(api):
    """Enough points that every head block works through several groups of
    tiles, with groups spanning sides and ragged ends of blocks' ranges."""
    rng = np.random.default_rng(7)
    sizes = [(int(rng.integers(300, 2000)), int(rng.integers(300, 2000))) for _ in range(24)]
    probs = _problems(8, sizes)
    B = api.Batch.from_problems(probs)
    net = api.WarmStartNet(seed=5)
    par = _params(net.bf16_weights())
    lu, lv = net.predict(B, eps=0.05)
    lu, lv = lu.cpu().numpy(), lv.cpu().numpy()
    for k, p in enumerate(probs):
        ou, ov = WO.predict(par, p.x, p.a, p.y, p.b, eps=0.05)
        gu = lu[B.row_off[k]:B.row_off[k + 1]] - np.log(p.a)
        gv = lv[B.col_off[k]:B.col_off[k + 1]] - np.log(p.b)
        for g, o, w in ((gu, ou, p.a), (gv, ov, p.b)):
            ref = o - np.log(w)
            np.testing.assert_allclose(g, ref, rtol=2e-2, atol=2e-2 * max(1.0, np.abs(ref).max()))


def test_gradient_matches_oracle(api):
    probs = _problems(2, SIZES)
    B = api.Batch.from_problems(probs)
    tu, tv = _targets(probs, 5)
    net = api.WarmStartNet(seed=4)
    par = _params(net.bf16_weights())
    before = net.weights().copy()
    loss, grad = net.train_step(B, np.concatenate(tu), np.concatenate(tv), lr=0.0, eps=0.05,
                                want_grad=True)
    assert net.step == 0 and np.array_equal(net.weights(), before)
    oloss, og = WO.batch_loss_and_grad(
        par, [(p.x, p.a, p.y, p.b, u, v) for p, u, v in zip(probs, tu, tv)], eps=0.05)
    assert loss == pytest.approx(oloss, rel=2e-2)
    g = _params(grad.cpu().numpy())
    scale = np.linalg.norm(og.flat())
    for name in WO.PARAM_NAMES:
        a, b = np.ravel(getattr(g, name)), np.ravel(getattr(og, name))
        if name == "c3":
            # the centred loss does not depend on the output bias: its gradient
            # is zero, on the GPU up to rounding
            assert abs(b[0]) < 1e-12 * scale and abs(a[0]) < 1e-5 * scale
            continue
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert err < 5e-2, (name, err)


def test_adam_step_updates_weights(api):
    probs = _problems(3, SIZES[:3])
    B = api.Batch.from_problems(probs)
    tu, tv = _targets(probs, 6)
    net = api.WarmStartNet(seed=5)
    w0 = net.weights().astype(np.float64)
    _, grad = net.train_step(B, np.concatenate(tu), np.concatenate(tv), lr=0.0, eps=0.05,
                             want_grad=True)
    net.train_step(B, np.concatenate(tu), np.concatenate(tv), lr=1e-3, eps=0.05)
    assert net.step == 1
    g = grad.cpu().numpy().astype(np.float64)
    # first Adam step: m_hat = g, v_hat = g^2
    expect = w0 - 1e-3 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(net.weights(), expect, rtol=0, atol=2e-6)
    # the BF16 copy follows the master weights
    np.testing.assert_allclose(net.bf16_weights(), net.weights(), rtol=1e-2, atol=1e-6)


def _solve(api, B, **kw):
    rc, res = api.spar_sink_batched(B, eps=0.05, seed=0, schedule=(8, 256), **kw)
    assert rc >= 0
    return res


def test_trained_network_saves_iterations(api):
    # training set: problems of the batched workload's law (smaller sizes so
    # the test stays short), solved to 1e-9 in FP64 by the batched solver
    train = W.batch_ot(256, seed=1000, n_lo=256, n_hi=1024)
    fresh = W.batch_ot(64, seed=2000, n_lo=256, n_hi=1024)
    batches, targets = [], []
    for i in range(0, len(train), 32):
        chunk = train[i:i + 32]
        B = api.Batch.from_problems(chunk)
        res = _solve(api, B, tol=1e-9, max_iter=3000, precision="f64", return_scalings=True)
        batches.append(B)
        targets.append((torch.cat([torch.log(r.u) for r in res]),
                        torch.cat([torch.log(r.v) for r in res])))
    net = api.WarmStartNet(seed=7)
    losses = []
    for epoch in range(30):
        for B, (tu, tv) in zip(batches, targets):
            losses.append(net.train_step(B, tu, tv, lr=1e-3, eps=0.05))
    assert np.mean(losses[-8:]) < 0.5 * np.mean(losses[:8])

    Bf = api.Batch.from_problems(fresh)
    lu, lv = net.predict(Bf, eps=0.05)
    cold = _solve(api, Bf, tol=1e-6, max_iter=1000, precision="f32")
    warm = _solve(api, Bf, tol=1e-6, max_iter=1000, precision="f32", init_log_u=lu, init_log_v=lv)
    ok = [i for i in range(len(fresh)) if cold[i].status == 0]
    assert len(ok) >= 60
    # every problem the plain start solves is solved from the learned start
    assert all(warm[i].status == 0 for i in ok), [warm[i].status for i in ok]
    kept = sum(warm[i].warm_start == 1 for i in ok)
    it_cold = np.mean([cold[i].iters for i in ok])
    it_warm = np.mean([warm[i].iters for i in ok])
    print(f"mean iterations to 1e-6: plain start {it_cold:.2f}, learned start {it_warm:.2f} "
          f"(prediction kept for {kept} of {len(ok)})")
    assert it_warm < 0.9 * it_cold
    # the warm start changes where the loop starts, not what it converges to
    for i in ok:
        assert abs(warm[i].estimate - cold[i].estimate) <= 1e-4 * abs(cold[i].estimate)


def _same_as_plain(cold, warm):
    """A start replaced by the plain one gives the plain solve bit for bit."""
    for k, (c, w) in enumerate(zip(cold, warm)):
        assert c.warm_start == -1 and w.warm_start == 0, k
        assert (w.status, w.iters, w.nnz) == (c.status, c.iters, c.nnz), k
        assert w.estimate == c.estimate and w.marginal_err == c.marginal_err, k
        assert w.sparse_objective == c.sparse_objective, k


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_corrupted_network_falls_back_to_plain_start(api, precision):
    # zero-init Sinkhorn is the warm start's fallback: a network whose weights
    # are corrupted (a NaN output bias makes every prediction NaN) must leave
    # every problem exactly where the plain start takes it
    probs = W.batch_ot(12, seed=2100, n_lo=200, n_hi=900)
    B = api.Batch.from_problems(probs)
    flat = api.WarmStartNet(seed=7).weights().copy()
    flat[-1] = np.nan
    lu, lv = api.WarmStartNet(flat).predict(B, eps=0.05)
    assert torch.isnan(lu).all() and torch.isnan(lv).all()
    kw = dict(tol=1e-6, max_iter=1000, precision=precision)
    cold = _solve(api, B, **kw)
    warm = _solve(api, B, **kw, init_log_u=lu, init_log_v=lv)
    _same_as_plain(cold, warm)
    # overflowing starts (exp(+800) is +inf in FP64 and FP32) likewise
    big = torch.full_like(lu, 800.0)
    _same_as_plain(cold, _solve(api, B, **kw, init_log_u=big, init_log_v=lv.nan_to_num(0.0)))


def test_poor_finite_start_is_judged_worse_than_plain(api):
    # a finite start far from the solution (log-scalings with unit-scale noise
    # times 30) has a larger first row marginal error than u = v = 1 and is
    # replaced; a start at the solution is kept and stops at once
    probs = W.batch_ot(8, seed=2200, n_lo=200, n_hi=900)
    B = api.Batch.from_problems(probs)
    g = torch.Generator(device="cpu").manual_seed(0)
    rows, cols = int(B.row_off[-1]), int(B.col_off[-1])
    lu = (30.0 * torch.randn(rows, generator=g, dtype=torch.float64)).cuda()
    lv = (30.0 * torch.randn(cols, generator=g, dtype=torch.float64)).cuda()
    kw = dict(tol=1e-8, max_iter=2000, precision="f64")
    cold = _solve(api, B, **kw, return_scalings=True)
    _same_as_plain(cold, _solve(api, B, **kw, init_log_u=lu, init_log_v=lv))
    su = torch.cat([torch.log(r.u) for r in cold])
    sv = torch.cat([torch.log(r.v) for r in cold])
    warm = _solve(api, B, **kw, init_log_u=su, init_log_v=sv)
    for c, w in zip(cold, warm):
        assert w.warm_start == 1 and w.status == 0 and w.iters <= 1
        assert abs(w.estimate - c.estimate) <= 1e-9 * abs(c.estimate)


def _same_solve(a, b):
    for k, (x, y) in enumerate(zip(a, b)):
        assert (x.status, x.iters, x.nnz, x.warm_start) == (y.status, y.iters, y.nnz,
                                                            y.warm_start), k
        assert x.estimate == y.estimate and x.marginal_err == y.marginal_err, k
        assert torch.equal(x.u, y.u) and torch.equal(x.v, y.v), k


@pytest.mark.parametrize("corrupt", [False, True])
def test_overlapped_learned_solve_equals_two_calls(api, corrupt):
    # spar_sink_batched_learned predicts on a second stream beside the
    # sampling stage; the loop must read the finished prediction, so the
    # result is the one of predict followed by spar_sink_batched, bit for bit:
    # on the current stream, then on another one with a smaller batch
    flat = api.WarmStartNet(seed=7).weights().copy()
    if corrupt:
        flat[-1] = np.nan  # every prediction NaN: each problem falls back
    net = api.WarmStartNet(flat)
    other = torch.cuda.Stream()
    kw = dict(eps=0.05, seed=0, schedule=(8, 256), tol=1e-6, max_iter=1000, precision="f32",
              return_scalings=True)
    for count, seed, stream in ((24, 2300, None), (9, 2301, other)):
        B = api.Batch.from_problems(W.batch_ot(count, seed=seed, n_lo=200, n_hi=1200))
        lu, lv = net.predict(B, eps=0.05)
        rc2, two = api.spar_sink_batched(B, init_log_u=lu, init_log_v=lv, **kw)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
            rc1, one = api.spar_sink_batched_learned(B, net, stream=stream, **kw)
        torch.cuda.synchronize()
        assert rc1 == rc2 and rc1 >= 0
        _same_solve(one, two)
        if corrupt:
            assert all(r.warm_start == 0 for r in one)
        print(f"{count} problems: prediction kept for "
              f"{sum(r.warm_start == 1 for r in one)}")
