"""Parity of the Wasserstein-Fisher-Rao cost (UOT background section; the
paper's UOT simulation) between the HIP path, through the C ABI, and the CPU
FP64 oracle: sampling (mask and CSR bit for bit, values within 1e-13, no
structural zero ever kept), the sparse and dense FP64 iterates within 1e-10,
and the reduced-precision estimates within 1e-4."""
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
    base = dict(eps=p.eps, s=p.s, lam=p.lam, seed=p.seed, problem_index=p.problem_index,
                cost="wfr", eta=p.meta["eta"])
    base.update(kw)
    return O.Options(**base)


def _kw(p, **kw):
    base = dict(eps=p.eps, s=p.s, lam=p.lam, seed=p.seed, cost="wfr", eta=p.meta["eta"])
    base.update(kw)
    return base


def _prob(api, p):
    return api.Problem(p.x, p.y, p.a, p.b, problem_index=p.problem_index)


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.mark.parametrize("pattern,ratio", [("C1", 0.7), ("C2", 0.5), ("C3", 0.3)])
def test_sample_wfr(api, pattern, ratio):
    p = W.wfr_synthetic(450, d=5, seed=21, pattern=pattern, nnz_ratio=ratio)
    eta = p.meta["eta"]
    sk = O.build_sketch(p.x, p.y, p.a, p.b, _oopt(p))
    g = api.ss_sample(_prob(api, p), **_kw(p), precision="f64")
    assert g["z_norm"] == pytest.approx(sk.prob.z, rel=1e-13)
    assert_mask_equal(g["mask"].cpu().numpy().view(np.uint64), sk.mask, p, sk.prob)
    assert g["nnz"] == sk.nnz
    for k in ("row_ptr", "col_idx", "col_ptr", "row_idx"):
        assert np.array_equal(g[k].cpu().numpy(), getattr(sk, k)), k
    np.testing.assert_allclose(g["val"].cpu().numpy(), sk.val, rtol=1e-13)
    np.testing.assert_allclose(g["val_t"].cpu().numpy(), sk.val_t, rtol=1e-13)
    # given the oracle's normaliser, the specified logarithm, cosine and
    # exponential make mask, CSR, CSC, values and factors bit-exact
    ge = api.ss_sample(_prob(api, p), **_kw(p), z_in=sk.prob.z, precision="f64")
    assert np.array_equal(ge["mask"].cpu().numpy().view(np.uint64), sk.mask)
    for k in ("row_ptr", "col_idx", "col_ptr", "row_idx", "val", "val_t"):
        assert np.array_equal(ge[k].cpu().numpy(), getattr(sk, k)), k
    assert np.array_equal(ge["row_fac"].cpu().numpy(), sk.prob.la)
    assert np.array_equal(ge["col_fac"].cpu().numpy(), sk.prob.lb)
    # no kept entry lies at or beyond the blocking distance pi eta
    rows = np.repeat(np.arange(p.n), np.diff(g["row_ptr"].cpu().numpy()))
    cols = g["col_idx"].cpu().numpy()
    d = np.sqrt(((p.x[rows] - p.y[cols]) ** 2).sum(axis=1))
    assert np.all(d < math.pi * eta)
    assert np.all(np.isfinite(g["val"].cpu().numpy())) and np.all(g["val"].cpu().numpy() > 0)


@pytest.mark.parametrize("n,m,d,s_factor", [(2100, 1337, 5, 8.0), (700, 4500, 5, 40.0),
                                             (900, 611, 3, 8.0)])
def test_sample_wfr_filter(api, n, m, d, s_factor):
    # The mask kernel's filter bounds the WFR cost factor in FP32 before the
    # exact decision; the mask must still be the pair-by-pair one: bit for
    # bit with the oracle's, over many row tiles, two column tiles and ragged
    # edges, and at a budget where a third of the pairs are kept.
    p = W.wfr_synthetic(max(n, m), d=d, seed=23, pattern="C1", nnz_ratio=0.5,
                        s_factor=s_factor)
    p = W.Problem(p.x[:n], p.y[:m], p.a[:n] * (5.0 / p.a[:n].sum()),
                  p.b[:m] * (3.0 / p.b[:m].sum()), eps=p.eps, s=p.s, lam=p.lam, seed=p.seed,
                  name=p.name, meta=p.meta)
    sk = O.build_sketch(p.x, p.y, p.a, p.b, _oopt(p))
    assert sk.nnz > 1000
    g = api.ss_sample(_prob(api, p), **_kw(p), precision="f64")
    assert g["z_norm"] == pytest.approx(sk.prob.z, rel=1e-13)
    ge = api.ss_sample(_prob(api, p), **_kw(p), z_in=sk.prob.z, precision="f64")
    assert np.array_equal(ge["mask"].cpu().numpy().view(np.uint64), sk.mask)
    for k in ("row_ptr", "col_idx", "col_ptr", "row_idx", "val", "val_t"):
        assert np.array_equal(ge[k].cpu().numpy(), getattr(sk, k)), k


def test_sample_wfr_filter_far_points(api):
    # One point in 25 of each side moved out by 1e25: its FP32 squared norm
    # overflows, so the filter makes every pair of it a candidate and leaves
    # the exact decision to block it (d >= pi eta); the mask, CSR, CSC and
    # values stay bit-exact with the oracle's.
    p = W.wfr_synthetic(800, d=5, seed=31, pattern="C1", nnz_ratio=0.5)
    x, y = p.x.copy(), p.y.copy()
    x[::25] *= 1e25
    y[3::25] *= 1e25
    p = W.Problem(x, y, p.a, p.b, eps=p.eps, s=p.s, lam=p.lam, seed=p.seed, name=p.name,
                  meta=p.meta)
    sk = O.build_sketch(p.x, p.y, p.a, p.b, _oopt(p))
    assert sk.nnz > 1000
    ge = api.ss_sample(_prob(api, p), **_kw(p), z_in=sk.prob.z, precision="f64")
    assert np.array_equal(ge["mask"].cpu().numpy().view(np.uint64), sk.mask)
    for k in ("row_ptr", "col_idx", "col_ptr", "row_idx", "val", "val_t"):
        assert np.array_equal(ge[k].cpu().numpy(), getattr(sk, k)), k


@pytest.mark.parametrize("perturb", [False, True])
def test_wfr_normaliser_same_support(api, perturb):
    # With y equal to x bit for bit the normaliser sums each unordered pair
    # once with both weights; one coordinate of y moved by one ulp takes the
    # general path.  Both agree with the oracle's plain sum over all pairs.
    p = W.wfr_synthetic(1500, d=5, seed=29, pattern="C3", nnz_ratio=0.6)
    y = p.y.copy()
    if perturb:
        y[777, 3] = np.nextafter(y[777, 3], 2.0)
    p = W.Problem(p.x, y, p.a, p.b, eps=p.eps, s=p.s, lam=p.lam, seed=p.seed, name=p.name,
                  meta=p.meta)
    pr = O.uot_probabilities(p.a, p.b, p.x, p.y, p.s, p.lam, p.eps, 1.0, cost="wfr",
                             eta=p.meta["eta"])
    g = api.ss_sample(_prob(api, p), **_kw(p), precision="f64")
    assert g["z_norm"] == pytest.approx(pr.z, rel=1e-13)


@pytest.mark.parametrize("lam,eps", [(5.0, 0.1), (0.02, 0.05), (0.1, 0.1)])
def test_wfr_normaliser_exponents(api, lam, eps):
    # the device evaluates cos(z)^(2/(2 lam + eps)) from a series in z^2; the
    # exponent runs from about 0.2 (pairs near the blocking distance weigh in)
    # to 22 (only close pairs count)
    p = W.wfr_synthetic(700, d=5, seed=23, pattern="C2", nnz_ratio=0.6)
    sk = O.build_sketch(p.x, p.y, p.a, p.b, _oopt(p, lam=lam, eps=eps))
    g = api.ss_sample(_prob(api, p), **_kw(p, lam=lam, eps=eps), precision="f64")
    assert g["z_norm"] == pytest.approx(sk.prob.z, rel=1e-13)


def test_spar_sink_uot_wfr_f64_fixed_iterations(api):
    p = W.wfr_synthetic(500, d=5, seed=22, nnz_ratio=0.5)
    T = 40
    o = O.spar_sink(p.x, p.y, p.a, p.b, _oopt(p, tol=0.0, max_iter=T))
    r = api.spar_sink_uot(_prob(api, p), **_kw(p, tol=0.0, max_iter=T), precision="f64",
                          return_scalings=True)
    assert r.iters == T and r.nnz == o.nnz and r.empty_rows == o.empty_rows
    np.testing.assert_allclose(r.u.cpu().numpy(), o.sinkhorn.u, rtol=1e-10, atol=0)
    np.testing.assert_allclose(r.v.cpu().numpy(), o.sinkhorn.v, rtol=1e-10, atol=0)
    assert _rel(r.estimate, o.estimate.estimate) < 1e-10
    assert _rel(r.transport, o.estimate.transport) < 1e-10


def test_dense_wfr_f64(api):
    p = W.wfr_synthetic(300, d=5, seed=23, nnz_ratio=0.5)
    T = 30
    o = O.dense_sinkhorn(p.x, p.y, p.a, p.b, _oopt(p, tol=0.0, max_iter=T))
    r = api.dense_sinkhorn(_prob(api, p), **_kw(p, tol=0.0, max_iter=T), precision="f64",
                           return_scalings=True)
    assert r.iters == T
    np.testing.assert_allclose(r.u.cpu().numpy(), o.sinkhorn.u, rtol=1e-10, atol=0)
    np.testing.assert_allclose(r.v.cpu().numpy(), o.sinkhorn.v, rtol=1e-10, atol=0)
    assert _rel(r.estimate, o.estimate.estimate) < 1e-10


@pytest.mark.parametrize("precision", ["f32", "f32_log"])
def test_dense_wfr_reduced_precision(api, precision):
    p = W.wfr_synthetic(700, d=5, seed=24, nnz_ratio=0.3)
    o = O.dense_sinkhorn(p.x, p.y, p.a, p.b, _oopt(p, tol=1e-6, max_iter=3000))
    r = api.dense_sinkhorn(_prob(api, p), **_kw(p, tol=1e-6, max_iter=3000), precision=precision)
    assert r.status == 0 and r.marginal_err <= 1e-6
    assert _rel(r.estimate, o.estimate.estimate) < 1e-4


def test_spar_sink_uot_wfr_log_domain(api):
    p = W.wfr_synthetic(1500, d=5, seed=25, nnz_ratio=0.5, s_factor=16.0)
    o = O.spar_sink(p.x, p.y, p.a, p.b, _oopt(p, tol=1e-6, max_iter=3000, log_domain=True))
    r = api.spar_sink_uot(_prob(api, p), **_kw(p, tol=1e-6, max_iter=3000), precision="f32_log")
    assert r.status == 0 and r.marginal_err <= 1e-6 and r.nnz == o.nnz
    assert _rel(r.estimate, o.estimate.estimate) < 1e-4
