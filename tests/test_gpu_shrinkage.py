"""Parity of the shrunk sampling probabilities (Sec. 4) and of Rand-Sink
(Sec. 5, g = 1) between the HIP path and the CPU FP64 oracle.

Only the probability stage changes, so the bars are the sampling ones: for OT
the mask, CSR and CSC bit for bit and the row factors exactly; for UOT the
mask and CSR/CSC bit for bit as well (a failure names the differing positions
and their distance to the keep boundary) and the values within 1e-14; the
Sinkhorn iterates on the same sketch within 1e-10 relative (FP64)."""
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


def _kw(p, **kw):
    base = dict(eps=p.eps, s=p.s, lam=p.lam, seed=p.seed)
    base.update(kw)
    return base


def _prob(api, p):
    return api.Problem(p.x, p.y, p.a, p.b, problem_index=p.problem_index)


def _mask_np(t):
    return t.cpu().numpy().view(np.uint64)


def _structure_equal(g, sk):
    assert g["nnz"] == sk.nnz
    assert np.array_equal(_mask_np(g["mask"]), sk.mask)
    for k in ("row_ptr", "col_idx", "col_ptr", "row_idx"):
        assert np.array_equal(g[k].cpu().numpy(), getattr(sk, k)), k


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.mark.parametrize("g", [0.5, 1.0])
def test_sample_ot_shrink_bit_exact(api, g):
    # ragged 700 x 513: several mask tiles and a partial last word
    p = W.ot_gauss2d(700, seed=21, m=513)
    sk = O.build_sketch(p.x, p.y, p.a, p.b, _oopt(p, shrink=g))
    out = api.ss_sample(_prob(api, p), **_kw(p), shrink=g, precision="f64")
    _structure_equal(out, sk)
    assert np.array_equal(out["row_fac"].cpu().numpy(), sk.prob.alpha)
    assert np.array_equal(out["col_fac"].cpu().numpy(), sk.prob.rb)
    assert np.array_equal(out["val"].cpu().numpy(), sk.val)
    assert np.array_equal(out["val_t"].cpu().numpy(), sk.val_t)
    if g == 1.0:
        # Rand-Sink: every kept value is K_ij nm / s
        assert np.all(sk.pstar == p.s / (700.0 * 513.0))


def test_sample_ot_shrink_zero_is_spar_sink(api):
    p = W.ot_gauss2d(300, seed=22, m=333)
    a = api.ss_sample(_prob(api, p), **_kw(p), precision="f64")
    b = api.ss_sample(_prob(api, p), **_kw(p), shrink=0.0, precision="f64")
    for k in ("mask", "row_ptr", "col_idx", "val", "row_fac"):
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("lam,g", [(1.0, 0.3), (0.3, 0.3), (1.0, 1.0)])
def test_sample_uot_shrink(api, lam, g):
    p = W.uot_mix3(450, seed=23, eps=0.05, lam=lam)
    sk = O.build_sketch(p.x, p.y, p.a, p.b, _oopt(p, shrink=g))
    out = api.ss_sample(_prob(api, p), **_kw(p), shrink=g, precision="f64")
    assert out["z_norm"] == pytest.approx(sk.prob.z, rel=1e-13)
    assert_mask_equal(_mask_np(out["mask"]), sk.mask, p, sk.prob)
    _structure_equal(out, sk)
    np.testing.assert_allclose(out["val"].cpu().numpy(), sk.val, rtol=1e-14)
    np.testing.assert_allclose(out["val_t"].cpu().numpy(), sk.val_t, rtol=1e-14)
    # given the oracle's normaliser: bit-exact
    ex = api.ss_sample(_prob(api, p), **_kw(p), shrink=g, z_in=sk.prob.z, precision="f64")
    assert np.array_equal(_mask_np(ex["mask"]), sk.mask)
    _structure_equal(ex, sk)
    for k in ("val", "val_t"):
        assert np.array_equal(ex[k].cpu().numpy(), getattr(sk, k)), k


@pytest.mark.parametrize("g", [0.5, 1.0])
def test_spar_sink_ot_shrink_fixed_iterations(api, g):
    p = W.ot_gauss2d(600, seed=24, m=520)
    T = 40
    o = O.spar_sink(p.x, p.y, p.a, p.b, _oopt(p, tol=0.0, max_iter=T, shrink=g))
    r = api.spar_sink_ot(_prob(api, p), **_kw(p, tol=0.0, max_iter=T), shrink=g,
                         precision="f64", return_scalings=True)
    assert r.iters == T and r.nnz == o.nnz
    assert r.empty_rows == o.empty_rows and r.empty_cols == o.empty_cols
    np.testing.assert_allclose(r.u.cpu().numpy(), o.sinkhorn.u, rtol=1e-10, atol=0)
    np.testing.assert_allclose(r.v.cpu().numpy(), o.sinkhorn.v, rtol=1e-10, atol=0)
    assert _rel(r.estimate, o.estimate.estimate) < 1e-10
    assert _rel(r.sparse_objective, o.estimate.sparse_objective) < 1e-10


def test_spar_sink_uot_shrink_fixed_iterations(api):
    p = W.uot_mix3(500, seed=25, eps=0.05)
    T = 50
    o = O.spar_sink(p.x, p.y, p.a, p.b, _oopt(p, tol=0.0, max_iter=T, shrink=0.4))
    r = api.spar_sink_uot(_prob(api, p), **_kw(p, tol=0.0, max_iter=T), shrink=0.4,
                          precision="f64", return_scalings=True)
    assert r.iters == T and r.nnz == o.nnz
    np.testing.assert_allclose(r.u.cpu().numpy(), o.sinkhorn.u, rtol=1e-10, atol=0)
    np.testing.assert_allclose(r.v.cpu().numpy(), o.sinkhorn.v, rtol=1e-10, atol=0)
    assert _rel(r.estimate, o.estimate.estimate) < 1e-10


def test_rand_sink_log_domain_to_tolerance(api):
    # Rand-Sink through the FP32 log-domain kernel against the FP64 oracle
    p = W.ot_t5_d10(1024, seed=26, s_factor=8.0)
    o = O.spar_sink(p.x, p.y, p.a, p.b, _oopt(p, tol=1e-6, max_iter=3000, shrink=1.0,
                                              log_domain=True))
    r = api.spar_sink_ot(_prob(api, p), **_kw(p, tol=1e-6, max_iter=3000), shrink=1.0,
                         precision="f32_log")
    assert r.status == 0 and r.marginal_err <= 1e-6 and r.nnz == o.nnz
    assert _rel(r.estimate, o.estimate.estimate) < 1e-4


@pytest.mark.parametrize("bad", [-0.1, 1.5, math.nan])
def test_bad_shrink_is_rejected(api, bad):
    from paper_2306_06581_amd import native as N
    p = W.ot_gauss2d(64, seed=27)
    with pytest.raises(N.SparSinkError) as e:
        api.spar_sink_ot(_prob(api, p), **_kw(p), shrink=bad)
    assert e.value.code == -1 and "shrink" in str(e.value)
