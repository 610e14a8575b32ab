"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Bars: integer/index/bit outputs bit-exact; FP64 scalings and estimates within
1e-10 relative; FP32 and log-FP32 estimates within 1e-4 relative of the FP64
oracle.  The UOT keep decision takes its exponentials and logarithms from the
specified functions both sides implement, so given the oracle's normaliser
(z_in) the UOT mask, offsets, indices and stored values are compared bit for
bit as well; a failure reports the differing positions and their distance to
the boundary.  The library's own normaliser is compared separately."""
import math

import numpy as np
import pytest
import torch

from oracle import sparsink_oracle as O
from paper_2306_06581_amd import workloads as W
from maskcheck import assert_mask_equal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_06581_amd import api as A
    return A


def _oopt(p, **kw):
    base = dict(eps=p.eps, s=p.s, lam=p.lam, seed=p.seed, problem_index=p.problem_index)
    base.update(kw)
    return O.Options(**base)


def _prob(api, p):
    return api.Problem(p.x, p.y, p.a, p.b, problem_index=p.problem_index)


def _kw(p, **kw):
    base = dict(eps=p.eps, s=p.s, lam=p.lam, seed=p.seed)
    base.update(kw)
    return base


def _mask_np(t):
    return t.cpu().numpy().view(np.uint64)


def _check_sketch_structure(g, sk):
    assert g["nnz"] == sk.nnz
    assert np.array_equal(_mask_np(g["mask"]), sk.mask)
    assert np.array_equal(g["row_ptr"].cpu().numpy(), sk.row_ptr)
    assert np.array_equal(g["col_idx"].cpu().numpy(), sk.col_idx)
    assert np.array_equal(g["col_ptr"].cpu().numpy(), sk.col_ptr)
    assert np.array_equal(g["row_idx"].cpu().numpy(), sk.row_idx)


OT_CASES = [
    ("ot_gauss2d_n1024", lambda: W.ot_gauss2d(1024, seed=0)),
    ("ragged_300x333_d2", lambda: W.ot_gauss2d(300, seed=3, m=333)),
    ("ot_t5_d10_n700", lambda: W.ot_t5_d10(700, seed=1, s_factor=4.0)),
    ("tiny_5x7", lambda: W.ot_gauss2d(5, seed=2, m=7)),
    ("single_1x1", lambda: W.ot_gauss2d(1, seed=4)),
]


@pytest.mark.parametrize("name,make", OT_CASES)
def test_sample_ot_bit_exact(api, name, make):
    p = make()
    if p.n == 1:
        p.s = 1.0
    sk = O.build_sketch(p.x, p.y, p.a, p.b, _oopt(p))
    g = api.ss_sample(_prob(api, p), **_kw(p), precision="f64")
    _check_sketch_structure(g, sk)
    # sqrt and the tree sums are exact operations: the p* factors match bitwise
    assert np.array_equal(g["row_fac"].cpu().numpy(), sk.prob.alpha)
    assert np.array_equal(g["col_fac"].cpu().numpy(), sk.prob.rb)
    assert g["cmax"] == sk.cmax
    # values: K / p* with K = exp(-C/eps) by the specified exponential on both
    # sides, so the CSR and CSC values are bit-exact as well
    assert np.array_equal(g["val"].cpu().numpy(), sk.val)
    assert np.array_equal(g["val_t"].cpu().numpy(), sk.val_t)


def test_sample_ot_weights_over_300_decades(api):
    """Four in five weights of each marginal are 10^-U(0,300): about 400 row
    and column factors lie below the FP32 range, where the hash filter's FP32
    bounds are clamped up to 2^-126.  The filter only ever admits a superset
    of the kept entries, so the mask and CSR/CSC still match bit for bit."""
    p = W.ot_gauss2d(700, seed=6, m=650)
    rng = np.random.default_rng(6)
    a = 10.0 ** -rng.uniform(0, 300, p.n)
    a[::5] = rng.uniform(0.5, 1.0, a[::5].shape)
    b = 10.0 ** -rng.uniform(0, 300, p.m)
    b[::5] = rng.uniform(0.5, 1.0, b[::5].shape)
    p.a, p.b = a / a.sum(), b / b.sum()
    sk = O.build_sketch(p.x, p.y, p.a, p.b, _oopt(p))
    assert (sk.prob.alpha * 65536 < 2.0 ** -126).sum() > 100
    assert (sk.prob.rb < 2.0 ** -126).sum() > 100
    g = api.ss_sample(_prob(api, p), **_kw(p), precision="f64")
    _check_sketch_structure(g, sk)
    assert np.array_equal(g["val"].cpu().numpy(), sk.val)


def test_sample_uot_weights_over_300_decades(api):
    """The UOT bound factors of weights 10^-U(0,300) (one in five of order
    one) fall below the FP32 range too; given the oracle's normaliser the
    mask, CSR/CSC and values stay bit-exact."""
    p = W.uot_mix3(500, seed=8, eps=0.05, lam=1.0)
    rng = np.random.default_rng(8)
    p.a = p.a * 10.0 ** -rng.uniform(0, 300, p.n)
    p.b = p.b * 10.0 ** -rng.uniform(0, 300, p.m)
    p.a[::5] = 1.0 / p.n
    p.b[::5] = 1.0 / p.m
    sk = O.build_sketch(p.x, p.y, p.a, p.b, _oopt(p))
    assert sk.nnz > 1000
    _uot_bit_exact(api, p, sk, precision="f64")


def test_sample_precisions_share_the_mask(api):
    p = W.ot_gauss2d(512, seed=5)
    sk = O.build_sketch(p.x, p.y, p.a, p.b, _oopt(p))
    g32 = api.ss_sample(_prob(api, p), **_kw(p), precision="f32")
    glog = api.ss_sample(_prob(api, p), **_kw(p), precision="f32_log")
    for g in (g32, glog):
        _check_sketch_structure(g, sk)
    # FP32 value = round-to-nearest of the (bit-exact) FP64 value; the log
    # value likewise
    assert np.array_equal(g32["val"].cpu().numpy(), sk.val.astype(np.float32))
    assert np.array_equal(glog["val"].cpu().numpy(), sk.logval.astype(np.float32))
    assert np.array_equal(glog["val_t"].cpu().numpy(), sk.logval_t.astype(np.float32))


def _uot_mask_compare(g_mask, sk, p, rows):
    assert_mask_equal(g_mask[rows], sk.mask[rows], p, sk.prob, rows)


def _uot_bit_exact(api, p, sk, **kw):
    """ss_sample given the oracle's normaliser Z: every keep decision and
    value is then the same IEEE operation sequence on both sides, so the
    mask, CSR, CSC, values and p* factors must match bit for bit."""
    g = api.ss_sample(_prob(api, p), **_kw(p), z_in=sk.prob.z, **kw)
    assert g["z_norm"] == sk.prob.z
    assert np.array_equal(_mask_np(g["mask"]), sk.mask)
    _check_sketch_structure(g, sk)
    assert np.array_equal(g["row_fac"].cpu().numpy(), sk.prob.la)
    assert np.array_equal(g["col_fac"].cpu().numpy(), sk.prob.lb)
    prec = kw.get("precision", "f64")
    if prec == "f64":
        ref, ref_t = sk.val, sk.val_t
    elif prec == "f32":
        ref, ref_t = sk.val.astype(np.float32), sk.val_t.astype(np.float32)
    else:
        ref, ref_t = sk.logval.astype(np.float32), sk.logval_t.astype(np.float32)
    assert np.array_equal(g["val"].cpu().numpy(), ref)
    assert np.array_equal(g["val_t"].cpu().numpy(), ref_t)
    return g


# lam = 1: the normaliser's short-range exponential (1/(2 lam + eps) <= 1/2);
# lam = 0.3: the general exponential
@pytest.mark.parametrize("n,eps,lam", [(600, 0.05, 1.0), (513, 0.01, 1.0), (400, 0.05, 0.3)])
def test_sample_uot(api, n, eps, lam):
    p = W.uot_mix3(n, seed=7, eps=eps, lam=lam)
    sk = O.build_sketch(p.x, p.y, p.a, p.b, _oopt(p))
    # the library's own normaliser: Z within 1e-13, every mask bit equal
    g = api.ss_sample(_prob(api, p), **_kw(p), precision="f64")
    assert g["z_norm"] == pytest.approx(sk.prob.z, rel=1e-13)
    _uot_mask_compare(_mask_np(g["mask"]), sk, p, np.arange(p.n))
    _check_sketch_structure(g, sk)
    np.testing.assert_allclose(g["val"].cpu().numpy(), sk.val, rtol=1e-14)
    # given the oracle's Z: bit-exact in every precision
    for prec in ("f64", "f32", "f32_log"):
        _uot_bit_exact(api, p, sk, precision=prec)


# Budgets at which most or all entries are kept: the mask kernel's per-wave
# candidate list then fills within every few rows of a tile, so its exact
# decision phase runs many times per tile; with p* = 1 everywhere every entry
# is kept.  m = 333 leaves a partial hash group and a partial mask word.
@pytest.mark.parametrize("frac", [0.5, 1e6])
def test_sample_ot_dense_budgets(api, frac):
    p = W.ot_gauss2d(300, seed=9, m=333)
    p.s = frac * p.n * p.m
    sk = O.build_sketch(p.x, p.y, p.a, p.b, _oopt(p))
    g = api.ss_sample(_prob(api, p), **_kw(p), precision="f64")
    _check_sketch_structure(g, sk)
    if frac > 1:
        assert sk.nnz == p.n * p.m
    assert np.array_equal(g["val"].cpu().numpy(), sk.val)


def test_sample_ot_columns_of_every_length(api):
    """Columns of very different lengths in one sketch: n = 5000 rows; heavy
    columns hold more than 4096 entries (one has half the column mass: about
    every row), most hold a few thousand, ten light ones a few hundred, one
    none.  The CSC must still list every column's rows in order."""
    rng = np.random.default_rng(21)
    n, m = 5000, 130
    x = rng.standard_normal((n, 2))
    y = rng.standard_normal((m, 2)) + 0.5
    a = rng.dirichlet(np.ones(n))
    b = rng.dirichlet(np.ones(m)) * 0.4
    b[7] = 0.5
    b[50] = 0.003
    b[100:110] = 1e-5
    b[-1] = 0.0
    b /= b.sum()
    p = W.Problem(x, y, a, b, eps=0.1, s=W.s_budget(n, 8.0), seed=21)
    sk = O.build_sketch(p.x, p.y, p.a, p.b, _oopt(p))
    counts = np.diff(sk.col_ptr)
    assert (counts > 4096).any() and ((counts > 256) & (counts <= 4096)).any()
    assert ((counts > 1) & (counts <= 256)).any() and counts[-1] == 0
    g = api.ss_sample(_prob(api, p), **_kw(p), precision="f64")
    _check_sketch_structure(g, sk)
    assert np.array_equal(g["val_t"].cpu().numpy(), sk.val_t)


def test_sample_uot_dense_budget(api):
    p = W.uot_mix3(300, seed=10, eps=0.05)
    p.s = 0.5 * p.n * p.m
    sk = O.build_sketch(p.x, p.y, p.a, p.b, _oopt(p))
    g = api.ss_sample(_prob(api, p), **_kw(p), precision="f64")
    _uot_mask_compare(_mask_np(g["mask"]), sk, p, np.arange(p.n))
    _check_sketch_structure(g, sk)
    _uot_bit_exact(api, p, sk, precision="f64")


def test_sample_uot_plain_cost(api):
    # unnormalised squared Euclidean cost (C up to ~10): the mask's FP32 bound of
    # the cost factor decides most candidates
    p = W.uot_mix3(500, seed=8, eps=0.5)
    sk = O.build_sketch(p.x, p.y, p.a, p.b, _oopt(p, cost="plain"))
    g = api.ss_sample(_prob(api, p), **_kw(p), cost="plain", precision="f64")
    assert g["z_norm"] == pytest.approx(sk.prob.z, rel=1e-13)
    _uot_mask_compare(_mask_np(g["mask"]), sk, p, np.arange(p.n))
    _check_sketch_structure(g, sk)
    np.testing.assert_allclose(g["val"].cpu().numpy(), sk.val, rtol=1e-13)
    _uot_bit_exact(api, p, sk, cost="plain", precision="f64")


# ---------------------------------------------------------------- Sinkhorn loop
def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.mark.parametrize("name,make", OT_CASES[:3])
def test_spar_sink_ot_f64_fixed_iterations(api, name, make):
    p = make()
    T = 40
    o = O.spar_sink(p.x, p.y, p.a, p.b, _oopt(p, tol=0.0, max_iter=T))
    g = api.spar_sink_ot(_prob(api, p), **_kw(p, tol=0.0, max_iter=T), precision="f64",
                         return_scalings=True, return_hist=True)
    assert g.status == 1 and g.iters == T == o.sinkhorn.iters
    assert g.nnz == o.nnz and g.empty_rows == o.empty_rows and g.empty_cols == o.empty_cols
    np.testing.assert_allclose(g.u.cpu().numpy(), o.sinkhorn.u, rtol=1e-10, atol=0)
    np.testing.assert_allclose(g.v.cpu().numpy(), o.sinkhorn.v, rtol=1e-10, atol=0)
    np.testing.assert_allclose(g.err_hist.cpu().numpy(), np.array(o.sinkhorn.hist), rtol=1e-6,
                               atol=1e-15)
    assert _rel(g.estimate, o.estimate.estimate) < 1e-10
    assert _rel(g.sparse_objective, o.estimate.sparse_objective) < 1e-10
    assert _rel(g.transport, o.estimate.transport) < 1e-10
    assert g.dropped_mass_a == pytest.approx(o.dropped_a, rel=1e-12, abs=1e-300)


def test_spar_sink_ot_f64_to_tolerance(api):
    p = W.ot_gauss2d(1024, seed=0)
    o = O.spar_sink(p.x, p.y, p.a, p.b, _oopt(p, tol=1e-8, max_iter=500))
    g = api.spar_sink_ot(_prob(api, p), **_kw(p, tol=1e-8, max_iter=500), precision="f64")
    assert g.status == 0 and abs(g.iters - o.sinkhorn.iters) <= 1
    assert g.marginal_err <= 1e-8
    assert _rel(g.estimate, o.estimate.estimate) < 1e-9


@pytest.mark.parametrize("stop_rule", ["marginal", "delta"])
def test_spar_sink_uot_f64(api, stop_rule):
    p = W.uot_mix3(700, seed=9, eps=0.05)
    T = 60
    o = O.spar_sink(p.x, p.y, p.a, p.b, _oopt(p, tol=0.0, max_iter=T, stop_rule=stop_rule))
    g = api.spar_sink_uot(_prob(api, p), **_kw(p, tol=0.0, max_iter=T, stop_rule=stop_rule),
                          precision="f64", return_scalings=True)
    assert g.iters == T
    np.testing.assert_allclose(g.u.cpu().numpy(), o.sinkhorn.u, rtol=1e-10, atol=0)
    np.testing.assert_allclose(g.v.cpu().numpy(), o.sinkhorn.v, rtol=1e-10, atol=0)
    assert _rel(g.estimate, o.estimate.estimate) < 1e-10
    assert _rel(g.kl_a, o.estimate.kl_a) < 1e-10 and _rel(g.kl_b, o.estimate.kl_b) < 1e-10
    assert _rel(g.marginal_err, o.sinkhorn.err) < 1e-6


@pytest.mark.parametrize("precision", ["f32", "f32_log"])
def test_spar_sink_ot_reduced_precision(api, precision):
    p = W.ot_t5_d10(2048, seed=2)
    o = O.spar_sink(p.x, p.y, p.a, p.b, _oopt(p, tol=1e-6, max_iter=2000))
    g = api.spar_sink_ot(_prob(api, p), **_kw(p, tol=1e-6, max_iter=2000), precision=precision)
    assert g.status == 0 and g.marginal_err <= 1e-6
    assert _rel(g.estimate, o.estimate.estimate) < 1e-4
    assert _rel(g.sparse_objective, o.estimate.sparse_objective) < 1e-4


@pytest.mark.parametrize("eps", [0.05, 0.01])
def test_spar_sink_uot_log_domain(api, eps):
    p = W.uot_mix3(1500, seed=11, eps=eps)
    o = O.spar_sink(p.x, p.y, p.a, p.b, _oopt(p, tol=1e-6, max_iter=3000, log_domain=True))
    g = api.spar_sink_uot(_prob(api, p), **_kw(p, tol=1e-6, max_iter=3000), precision="f32_log")
    assert g.status == 0 and g.marginal_err <= 1e-6
    assert abs(g.iters - o.sinkhorn.iters) <= max(2, 0.02 * o.sinkhorn.iters)
    assert _rel(g.estimate, o.estimate.estimate) < 1e-4


# ---------------------------------------------------------------- dense baseline
@pytest.mark.parametrize("lam", [math.inf, 1.0])
def test_dense_f64(api, lam):
    p = W.uot_mix3(400, seed=12, eps=0.05) if math.isfinite(lam) else W.ot_gauss2d(500, seed=12)
    T = 30
    o = O.dense_sinkhorn(p.x, p.y, p.a, p.b, _oopt(p, tol=0.0, max_iter=T, lam=lam))
    g = api.dense_sinkhorn(_prob(api, p), **_kw(p, tol=0.0, max_iter=T, lam=lam), precision="f64",
                           return_scalings=True)
    assert g.iters == T and g.nnz == p.n * p.m
    np.testing.assert_allclose(g.u.cpu().numpy(), o.sinkhorn.u, rtol=1e-10)
    np.testing.assert_allclose(g.v.cpu().numpy(), o.sinkhorn.v, rtol=1e-10)
    assert _rel(g.estimate, o.estimate.estimate) < 1e-10


@pytest.mark.parametrize("precision", ["f32", "f32_log"])
def test_dense_reduced_precision(api, precision):
    p = W.ot_gauss2d(1024, seed=13)
    o = O.dense_sinkhorn(p.x, p.y, p.a, p.b, _oopt(p, tol=1e-6, max_iter=1000))
    g = api.dense_sinkhorn(_prob(api, p), **_kw(p, tol=1e-6, max_iter=1000), precision=precision)
    assert g.status == 0 and g.marginal_err <= 1e-6
    assert _rel(g.estimate, o.estimate.estimate) < 1e-4


# ---------------------------------------------------------------- edge cases
def test_empty_rows_renormalised(api):
    p = W.ot_gauss2d(400, seed=14)
    p.s = 2.0 * 400   # ~2 entries per row: many empty lines
    o = O.spar_sink(p.x, p.y, p.a, p.b, _oopt(p, tol=0.0, max_iter=20))
    g = api.spar_sink_ot(_prob(api, p), **_kw(p, tol=0.0, max_iter=20), precision="f64",
                         return_scalings=True)
    assert o.empty_rows > 0 and g.empty_rows == o.empty_rows and g.empty_cols == o.empty_cols
    assert g.dropped_mass_a == pytest.approx(o.dropped_a, rel=1e-12)
    np.testing.assert_allclose(g.u.cpu().numpy(), o.sinkhorn.u, rtol=1e-10, atol=0)


def test_fail_policy_and_bad_inputs(api):
    from paper_2306_06581_amd import native as N
    p = W.ot_gauss2d(400, seed=15)
    p.s = 400.0
    with pytest.raises(N.SparSinkError) as ei:
        api.spar_sink_ot(_prob(api, p), **_kw(p), empty_policy="fail")
    assert ei.value.code == N.SS_E_EMPTY
    q = W.ot_gauss2d(64, seed=16)
    q.a[3] = -1.0
    with pytest.raises(N.SparSinkError) as ei:
        api.spar_sink_ot(_prob(api, q), **_kw(q))
    assert ei.value.code == N.SS_E_INVALID_ARG
    q = W.ot_gauss2d(64, seed=16)
    q.x[5, 1] = math.nan
    with pytest.raises(N.SparSinkError) as ei:
        api.spar_sink_ot(_prob(api, q), **_kw(q))
    assert ei.value.code == N.SS_E_INVALID_ARG


def test_max_iter_one_and_determinism(api):
    p = W.ot_gauss2d(1024, seed=17)
    g = api.spar_sink_ot(_prob(api, p), **_kw(p, tol=1e-12, max_iter=1))
    assert g.status == 1 and g.iters == 1
    r1 = api.spar_sink_ot(_prob(api, p), **_kw(p, tol=1e-9), precision="f32", return_scalings=True)
    r2 = api.spar_sink_ot(_prob(api, p), **_kw(p, tol=1e-9), precision="f32", return_scalings=True,
                          graph_iters=-1)
    assert r1.iters == r2.iters and r1.estimate == r2.estimate
    assert torch.equal(r1.u, r2.u) and torch.equal(r1.v, r2.v)


@pytest.mark.parametrize("threads", [256, 1024])
@pytest.mark.parametrize("precision", ["f64", "f32", "f32_log"])
def test_block_schedules_agree(api, threads, precision):
    # 40000 columns: several LDS slices per sweep in every precision
    p = W.ot_gauss2d(777, seed=18, m=40000)
    o = O.spar_sink(p.x, p.y, p.a, p.b, _oopt(p, tol=0.0, max_iter=15))
    g = api.spar_sink_ot(_prob(api, p), **_kw(p, tol=0.0, max_iter=15), precision=precision,
                         block_threads=threads, return_scalings=True)
    rtol = 1e-11 if precision == "f64" else 2e-4
    np.testing.assert_allclose(g.u.cpu().numpy(), o.sinkhorn.u, rtol=rtol)
    np.testing.assert_allclose(g.v.cpu().numpy(), o.sinkhorn.v, rtol=rtol, atol=1e-300)


def test_long_lines_take_several_chunks(api):
    # s large enough that rows hold ~1500 entries (> one register chunk)
    p = W.ot_gauss2d(300, seed=21, m=2000)
    p.s = 0.75 * 300 * 2000
    o = O.spar_sink(p.x, p.y, p.a, p.b, _oopt(p, tol=0.0, max_iter=10))
    g = api.spar_sink_ot(_prob(api, p), **_kw(p, tol=0.0, max_iter=10), precision="f64",
                         return_scalings=True)
    assert g.nnz == o.nnz
    np.testing.assert_allclose(g.u.cpu().numpy(), o.sinkhorn.u, rtol=1e-11)


@pytest.mark.parametrize("precision", ["f64", "f32", "f32_log"])
def test_multi_pass_steps(api, precision):
    # ~6.3e6 entries over 3000 lines: the single-pass step plan would need
    # more steps than there are resident blocks, so the planner switches to
    # steps of several passes each (one step per block); iterates and
    # estimates must not change
    p = W.ot_gauss2d(3000, seed=23)
    p.s = 0.7 * 3000 * 3000
    T = 12
    o = O.spar_sink(p.x, p.y, p.a, p.b, _oopt(p, tol=0.0, max_iter=T), workers=8)
    assert o.nnz > 5_500_000
    g = api.spar_sink_ot(_prob(api, p), **_kw(p, tol=0.0, max_iter=T), precision=precision,
                         return_scalings=True)
    assert g.nnz == o.nnz and g.iters == T
    if precision == "f64":
        np.testing.assert_allclose(g.u.cpu().numpy(), o.sinkhorn.u, rtol=1e-10, atol=0)
        np.testing.assert_allclose(g.v.cpu().numpy(), o.sinkhorn.v, rtol=1e-10, atol=0)
        assert _rel(g.estimate, o.estimate.estimate) < 1e-10
    else:
        assert _rel(g.estimate, o.estimate.estimate) < 1e-4


def test_warm_start_from_solution_converges_immediately(api):
    p = W.ot_gauss2d(1024, seed=19)
    g = api.spar_sink_ot(_prob(api, p), **_kw(p, tol=1e-10, max_iter=500), return_scalings=True)
    w = api.spar_sink_ot(_prob(api, p), **_kw(p, tol=1e-10, max_iter=500),
                         init_log_u=torch.log(g.u), init_log_v=torch.log(g.v))
    assert w.iters <= 2 and w.status == 0
