"""Parity of the batched solver (spar_sink_batched, through the C ABI).

Every problem of a batch must reproduce the single-problem solve: the same
mask (entry counts, empty lines) as the FP64 oracle run with that problem's
hash counter word, FP64 iterates and estimates within 1e-10 relative, FP32
estimates within 1e-4 of the FP64 reference.  Sizes are ragged (1 x 1 up to
the 4096-point limit) so that tiles, queue order and LDS sizing are all
exercised."""
import numpy as np
import pytest
import torch

from oracle import sparsink_oracle as O
from paper_2306_06581_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_06581_amd import api as A
    return A


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _ragged_batch(seed=0):
    rng = np.random.default_rng(seed)
    sizes = [(1, 1), (5, 7), (37, 64), (130, 65), (300, 333), (64, 200), (513, 257), (1000, 999)]
    probs = []
    for k, (n, m) in enumerate(sizes):
        mu_x, mu_y = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
        x = mu_x + rng.standard_normal((n, 3))
        y = mu_y + rng.standard_normal((m, 3))
        a, b = rng.dirichlet(np.ones(n)), rng.dirichlet(np.ones(m))
        probs.append(W.Problem(x, y, a, b, eps=0.05, s=W.s_budget(max(n, 2), 8.0), seed=seed,
                               problem_index=k, name=f"ragged_{k}"))
    return probs


def _oracle(p, **kw):
    opt = O.Options(eps=p.eps, s=p.s, seed=p.seed, problem_index=p.problem_index, **kw)
    return O.spar_sink(p.x, p.y, p.a, p.b, opt)


def test_batched_f64_fixed_iterations_match_oracle(api):
    probs = _ragged_batch(0)
    B = api.Batch.from_problems(probs)
    T = 30
    rc, res = api.spar_sink_batched(B, eps=0.05, tol=0.0, max_iter=T, seed=0, precision="f64",
                                    schedule=(8, 256), return_scalings=True)
    assert rc == 1  # problems stop at max_iter unless their error is exactly 0 (1 x 1)
    for p, g in zip(probs, res):
        o = _oracle(p, tol=0.0, max_iter=T)
        assert g.iters == o.sinkhorn.iters, p.name
        assert g.status == (0 if o.sinkhorn.converged else 1), p.name
        assert g.nnz == o.nnz and g.empty_rows == o.empty_rows and g.empty_cols == o.empty_cols
        np.testing.assert_allclose(g.u.cpu().numpy(), o.sinkhorn.u, rtol=1e-10, atol=0)
        np.testing.assert_allclose(g.v.cpu().numpy(), o.sinkhorn.v, rtol=1e-10, atol=0)
        assert _rel(g.estimate, o.estimate.estimate) < 1e-10, p.name
        assert _rel(g.sparse_objective, o.estimate.sparse_objective) < 1e-10, p.name
        assert g.cmax == o.cmax
        assert g.dropped_mass_a == pytest.approx(o.dropped_a, rel=1e-12, abs=1e-300)


def test_batched_f64_to_tolerance_matches_oracle(api):
    probs = _ragged_batch(1)
    B = api.Batch.from_problems(probs)
    rc, res = api.spar_sink_batched(B, eps=0.05, tol=1e-8, max_iter=3000, seed=1,
                                    precision="f64", schedule=(16, 512))
    assert rc == 0
    for p, g in zip(probs, res):
        o = _oracle(p, tol=1e-8, max_iter=3000)
        assert g.status == 0 and g.marginal_err <= 1e-8
        assert abs(g.iters - o.sinkhorn.iters) <= 1, p.name
        assert _rel(g.estimate, o.estimate.estimate) < 1e-9, p.name


def test_batched_matches_single_problem_solver(api):
    # problems of the config-4 generator, FP32, against the single-problem FP64
    # GPU solver (itself at parity with the oracle) and its FP32 twin
    probs = W.batch_ot(24, seed=5)
    B = api.Batch.from_problems(probs)
    rc, res = api.spar_sink_batched(B, eps=0.05, tol=1e-6, max_iter=3000, seed=5,
                                    precision="f32")
    assert rc == 0
    for p, g in zip(probs, res):
        prob = api.Problem(p.x, p.y, p.a, p.b, problem_index=p.problem_index)
        r64 = api.spar_sink_ot(prob, eps=0.05, s=p.s, seed=5, tol=1e-6, max_iter=3000,
                               precision="f64")
        r32 = api.spar_sink_ot(prob, eps=0.05, s=p.s, seed=5, tol=1e-6, max_iter=3000,
                               precision="f32")
        assert g.nnz == r64.nnz and g.empty_rows == r64.empty_rows
        assert g.status == 0 and g.marginal_err <= 1e-6
        assert _rel(g.estimate, r64.estimate) < 1e-4, p.name
        assert _rel(g.sparse_objective, r64.sparse_objective) < 1e-4, p.name
        assert abs(g.iters - r32.iters) <= max(2, 0.02 * r32.iters), p.name


def test_batched_straggler_hand_off(api):
    # A batch in which one problem needs many more iterations than the rest:
    # every problem but the slowest starts from its own solution (it stops
    # within an iteration or two), the slowest from zero.  Past the batch
    # loop's first 64 iterations the slowest is the only one left and
    # continues on the single-problem solver from its iterate; it must end
    # where a single-problem FP64 solve of the same problem (same sketch) ends.
    probs = W.batch_ot(6, seed=3)
    B = api.Batch.from_problems(probs)
    kw = dict(eps=0.01, tol=1e-9, max_iter=3000, seed=3, precision="f64")
    rc, first = api.spar_sink_batched(B, **kw, return_scalings=True)
    assert rc == 0
    slow = int(np.argmax([r.iters for r in first]))
    assert first[slow].iters > 64  # the precondition of the hand-off
    lu = torch.cat([torch.zeros_like(r.u) if k == slow else torch.log(r.u)
                    for k, r in enumerate(first)])
    lv = torch.cat([torch.zeros_like(r.v) if k == slow else torch.log(r.v)
                    for k, r in enumerate(first)])
    rc, res = api.spar_sink_batched(B, **kw, init_log_u=lu, init_log_v=lv)
    assert rc == 0
    for k, r in enumerate(res):
        if k != slow:
            assert r.iters <= 2, k
    p = probs[slow]
    prob = api.Problem(p.x, p.y, p.a, p.b, problem_index=p.problem_index)
    ref = api.spar_sink_ot(prob, eps=0.01, s=p.s, seed=3, tol=1e-9, max_iter=3000,
                           precision="f64")
    g = res[slow]
    assert g.nnz == ref.nnz and g.empty_rows == ref.empty_rows and g.empty_cols == ref.empty_cols
    assert g.status == 0 and g.marginal_err <= 1e-9
    assert abs(g.iters - ref.iters) <= 1
    assert g.iters == first[slow].iters or abs(g.iters - first[slow].iters) <= 1
    assert _rel(g.estimate, ref.estimate) < 1e-9
    assert _rel(g.sparse_objective, ref.sparse_objective) < 1e-9


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_every_schedule_gives_the_same_answer(api, precision):
    probs = _ragged_batch(2)[3:]
    B = api.Batch.from_problems(probs)
    ref = None
    for lanes in (4, 8, 16, 32):
        for block in (256, 512, 1024):
            rc, res = api.spar_sink_batched(B, eps=0.05, tol=0.0, max_iter=25, seed=2,
                                            precision=precision, schedule=(lanes, block))
            est = np.array([r.estimate for r in res])
            nnz = [r.nnz for r in res]
            if ref is None:
                ref = (est, nnz)
                continue
            assert nnz == ref[1]
            tol = 1e-12 if precision == "f64" else 1e-5
            np.testing.assert_allclose(est, ref[0], rtol=tol, atol=0)


def test_batched_largest_problems_and_autotuner(api):
    probs = W.batch_ot(6, seed=7, n_lo=4000, n_hi=4096)
    B = api.Batch.from_problems(probs)
    best, times = api.ss_autotune_batched(B, eps=0.05, seed=7, precision="f32")
    assert best in times and len(times) == 12
    assert times[best] == min(times.values()) and all(t > 0 for t in times.values())
    rc, res = api.spar_sink_batched(B, eps=0.05, tol=1e-6, max_iter=3000, seed=7,
                                    precision="f32")
    assert rc == 0 and all(r.status == 0 and r.marginal_err <= 1e-6 for r in res)
    for p, g in zip(probs[:2], res[:2]):
        prob = api.Problem(p.x, p.y, p.a, p.b, problem_index=p.problem_index)
        r64 = api.spar_sink_ot(prob, eps=0.05, s=p.s, seed=7, tol=1e-6, max_iter=3000,
                               precision="f64")
        assert g.nnz == r64.nnz
        assert _rel(g.estimate, r64.estimate) < 1e-4


@pytest.mark.skip(reason="went silent for more than 180 s on the GPU (no fault reported) and "
                         "no cause was found by reading the code; the FAIL policy is rejected "
                         "for batches until one is")
def test_batched_empty_fail_is_per_problem(api):
    probs = _ragged_batch(3)[2:5]
    # a tiny budget leaves lines without entries in every problem but the last
    probs[0].s = probs[1].s = 3.0
    B = api.Batch.from_problems(probs)
    rc, res = api.spar_sink_batched(B, eps=0.05, tol=1e-6, max_iter=2000, seed=3,
                                    precision="f64", empty_policy="fail")
    assert rc == -5
    assert res[0].status == -5 and res[1].status == -5
    assert res[2].status in (0, -5)
    if res[2].empty_rows == 0 and res[2].empty_cols == 0:
        assert res[2].status == 0


def test_batched_warm_start_from_solution(api):
    probs = _ragged_batch(4)[4:]
    B = api.Batch.from_problems(probs)
    rc, res = api.spar_sink_batched(B, eps=0.05, tol=1e-9, max_iter=3000, seed=4,
                                    precision="f64", return_scalings=True)
    assert rc == 0
    lu = torch.cat([torch.log(r.u) for r in res])
    lv = torch.cat([torch.log(r.v) for r in res])
    rc2, res2 = api.spar_sink_batched(B, eps=0.05, tol=1e-8, max_iter=3000, seed=4,
                                      precision="f64", init_log_u=lu, init_log_v=lv)
    assert rc2 == 0 and all(r.iters <= 1 for r in res2)
    for r, r2 in zip(res, res2):
        assert _rel(r2.estimate, r.estimate) < 1e-8
