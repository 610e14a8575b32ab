"""Host-only checks of the C ABI: the library loads, exports every function the
header declares, its structs have the header's layout (checked against a C
program compiled from the header), and argument errors are reported before
any device work.  No GPU needed."""
import ctypes
import math
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sparsink.h")
LIB = os.path.join(ROOT, "paper_2306_06581_amd", "libsparsink.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsparsink.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (\w+)$", out, flags=re.M))
    names = declared_functions()
    assert len(names) >= 8
    missing = [nme for nme in names if nme not in exported]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2306_06581_amd import native as N
    assert sorted(N.SIGNATURES) == declared_functions()
    assert N.lib.ss_version() == 100


def _c_layout():
    src = r"""
#include <stddef.h>
#include <stdio.h>
#include "sparsink.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("ss_problem %zu\nss_options %zu\nss_result %zu\nss_sparse %zu\n",
         sizeof(ss_problem), sizeof(ss_options), sizeof(ss_result), sizeof(ss_sparse));
  printf("ss_batch %zu\nss_schedule %zu\n", sizeof(ss_batch), sizeof(ss_schedule));
  P(ss_batch, s) P(ss_batch, x) P(ss_batch, b) P(ss_schedule, block_threads)
  P(ss_problem, x) P(ss_options, seed) P(ss_options, init_log_u) P(ss_options, err_hist) P(ss_options, shrink) P(ss_options, eta)
  P(ss_result, nnz) P(ss_result, iters) P(ss_result, t_obj_ms) P(ss_result, warm_start)
  P(ss_sparse, capacity)
  P(ss_sparse, z_norm) P(ss_ibp_problem, x) P(ss_ibp_problem, w) P(ss_ibp_result, nnz)
  P(ss_ibp_result, t_iter_ms) P(ss_divergence, nnz) P(ss_divergence, status)
  printf("ss_divergence %zu\n", sizeof(ss_divergence));
  printf("ss_ibp_problem %zu\nss_ibp_result %zu\n", sizeof(ss_ibp_problem), sizeof(ss_ibp_result));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "layout.c")
        exe = os.path.join(td, "layout")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    return {k: int(v) for k, v in (line.split() for line in out.strip().splitlines())}


def test_struct_layout_matches_header():
    from paper_2306_06581_amd import native as N
    lay = _c_layout()
    assert ctypes.sizeof(N.SsProblem) == lay["ss_problem"]
    assert ctypes.sizeof(N.SsOptions) == lay["ss_options"]
    assert ctypes.sizeof(N.SsResult) == lay["ss_result"]
    assert ctypes.sizeof(N.SsSparse) == lay["ss_sparse"]
    assert N.SsProblem.x.offset == lay["ss_problem.x"]
    assert N.SsOptions.seed.offset == lay["ss_options.seed"]
    assert N.SsOptions.init_log_u.offset == lay["ss_options.init_log_u"]
    assert N.SsOptions.err_hist.offset == lay["ss_options.err_hist"]
    assert N.SsOptions.shrink.offset == lay["ss_options.shrink"]
    assert N.SsOptions.eta.offset == lay["ss_options.eta"]
    assert N.SsResult.nnz.offset == lay["ss_result.nnz"]
    assert N.SsResult.iters.offset == lay["ss_result.iters"]
    assert N.SsResult.t_obj_ms.offset == lay["ss_result.t_obj_ms"]
    assert N.SsResult.warm_start.offset == lay["ss_result.warm_start"]
    assert N.SsSparse.capacity.offset == lay["ss_sparse.capacity"]
    assert N.SsSparse.z_norm.offset == lay["ss_sparse.z_norm"]
    assert ctypes.sizeof(N.SsBatch) == lay["ss_batch"]
    assert ctypes.sizeof(N.SsSchedule) == lay["ss_schedule"]
    assert N.SsBatch.s.offset == lay["ss_batch.s"]
    assert N.SsBatch.x.offset == lay["ss_batch.x"]
    assert N.SsBatch.b.offset == lay["ss_batch.b"]
    assert N.SsSchedule.block_threads.offset == lay["ss_schedule.block_threads"]
    assert ctypes.sizeof(N.SsIbpProblem) == lay["ss_ibp_problem"]
    assert ctypes.sizeof(N.SsIbpResult) == lay["ss_ibp_result"]
    assert N.SsIbpProblem.x.offset == lay["ss_ibp_problem.x"]
    assert N.SsIbpProblem.w.offset == lay["ss_ibp_problem.w"]
    assert N.SsIbpResult.nnz.offset == lay["ss_ibp_result.nnz"]
    assert N.SsIbpResult.t_iter_ms.offset == lay["ss_ibp_result.t_iter_ms"]
    assert ctypes.sizeof(N.SsDivergence) == lay["ss_divergence"]
    assert N.SsDivergence.nnz.offset == lay["ss_divergence.nnz"]
    assert N.SsDivergence.status.offset == lay["ss_divergence.status"]


def _fake_problem(N, n=8, m=8, d=2):
    # non-null dummy device pointers: argument checks never dereference them
    return N.SsProblem(n, m, d, 0, 256, 512, 768, 1024)


@pytest.mark.parametrize("field,value", [("n", 0), ("m", -3), ("d", 0), ("d", 65)])
def test_bad_sizes_rejected(field, value):
    from paper_2306_06581_amd import native as N
    from paper_2306_06581_amd.api import make_options
    p = _fake_problem(N)
    setattr(p, field, value)
    out = ctypes.c_size_t(0)
    rc = N.lib.ss_workspace_size(ctypes.byref(p), ctypes.byref(make_options(0.1, 10.0)),
                                 ctypes.byref(out))
    assert rc == N.SS_E_INVALID_ARG
    assert N.lib.ss_last_error().decode()


@pytest.mark.parametrize("kw", [dict(eps=0.0), dict(eps=-1.0), dict(eps=math.nan),
                                dict(s=0.0), dict(tol=-1.0), dict(max_iter=0),
                                dict(block_threads=512), dict(lam=0.0)])
def test_bad_options_rejected(kw):
    from paper_2306_06581_amd import native as N
    from paper_2306_06581_amd.api import make_options
    base = dict(eps=0.1, s=10.0)
    base.update(kw)
    out = ctypes.c_size_t(0)
    rc = N.lib.ss_workspace_size(ctypes.byref(_fake_problem(N)), ctypes.byref(make_options(**base)),
                                 ctypes.byref(out))
    assert rc == N.SS_E_INVALID_ARG


def test_null_pointers_and_workspace_errors():
    from paper_2306_06581_amd import native as N
    from paper_2306_06581_amd.api import make_options
    res = N.SsResult()
    opts = make_options(0.1, 10.0)
    p = _fake_problem(N)
    p.a = None
    assert N.lib.spar_sink_ot(ctypes.byref(p), ctypes.byref(opts), None, 0, None,
                              ctypes.byref(res)) == N.SS_E_INVALID_ARG
    p = _fake_problem(N)
    assert N.lib.spar_sink_ot(ctypes.byref(p), ctypes.byref(opts), None, 0, None,
                              ctypes.byref(res)) == N.SS_E_WORKSPACE
    assert N.lib.spar_sink_ot(ctypes.byref(p), ctypes.byref(opts), ctypes.c_void_p(4096 + 8), 1 << 30,
                              None, ctypes.byref(res)) == N.SS_E_WORKSPACE    # misaligned
    assert N.lib.spar_sink_ot(ctypes.byref(p), ctypes.byref(opts), ctypes.c_void_p(4096), 16,
                              None, ctypes.byref(res)) == N.SS_E_WORKSPACE    # too small
    # OT entry point refuses a finite lambda, UOT refuses an infinite one
    uot = make_options(0.1, 10.0, lam=1.0)
    assert N.lib.spar_sink_ot(ctypes.byref(p), ctypes.byref(uot), ctypes.c_void_p(4096), 1 << 40,
                              None, ctypes.byref(res)) == N.SS_E_INVALID_ARG
    assert N.lib.spar_sink_uot(ctypes.byref(p), ctypes.byref(opts), ctypes.c_void_p(4096), 1 << 40,
                               None, ctypes.byref(res)) == N.SS_E_INVALID_ARG
    # dense is limited to d <= 16
    p = _fake_problem(N, d=17)
    assert N.lib.dense_sinkhorn(ctypes.byref(p), ctypes.byref(opts), ctypes.c_void_p(4096), 1 << 40,
                                None, ctypes.byref(res)) == N.SS_E_INVALID_ARG


def test_workspace_grows_with_problem():
    from paper_2306_06581_amd import native as N
    from paper_2306_06581_amd.api import make_options
    sizes = []
    for n in (64, 1024, 4096):
        out = ctypes.c_size_t(0)
        rc = N.lib.ss_workspace_size(ctypes.byref(_fake_problem(N, n, n)),
                                     ctypes.byref(make_options(0.1, 8 * n * math.log(n))),
                                     ctypes.byref(out))
        assert rc == 0
        sizes.append(out.value)
    assert sizes[0] < sizes[1] < sizes[2]
    # the mask dominates: at least n*m/8 bytes twice (mask and its transpose)
    assert sizes[2] >= 2 * 4096 * 4096 // 8


def test_status_strings():
    from paper_2306_06581_amd import native as N
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert N.lib.ss_status_string(code).decode() != "unknown status"
    assert N.lib.ss_status_string(99).decode() == "unknown status"


def _fake_batch(N, ns=(3, 5), ms=(4, 6), ss=(10.0, 20.0), d=3):
    import numpy as np
    keep = dict(n=np.array(ns, dtype=np.int64), m=np.array(ms, dtype=np.int64),
                s=np.array(ss, dtype=np.float64))
    b = N.SsBatch(len(ns), d, keep["n"].ctypes.data, keep["m"].ctypes.data, keep["s"].ctypes.data,
                  None, 256, 512, 768, 1024)
    return b, keep


@pytest.mark.parametrize("change", ["count0", "n_big", "m0", "s_neg", "d0", "lam", "log",
                                    "delta", "hist", "fail_policy"])
def test_batch_arguments_rejected(change):
    import numpy as np
    from paper_2306_06581_amd import native as N
    from paper_2306_06581_amd.api import make_options
    b, keep = _fake_batch(N)
    opts = make_options(0.05, precision="f32")
    if change == "count0":
        b.count = 0
    elif change == "n_big":
        keep["n"][1] = N.BATCH_MAX_SIDE + 1
    elif change == "m0":
        keep["m"][0] = 0
    elif change == "s_neg":
        keep["s"][0] = -1.0
    elif change == "d0":
        b.d = 0
    elif change == "lam":
        opts = make_options(0.05, lam=1.0, precision="f32")
    elif change == "log":
        opts = make_options(0.05, precision="f32_log")
    elif change == "delta":
        opts = make_options(0.05, precision="f32", stop_rule="delta")
    elif change == "hist":
        opts = make_options(0.05, precision="f32", err_hist=None)
        opts.err_hist = 4096
    elif change == "fail_policy":
        opts = make_options(0.05, precision="f32", empty_policy="fail")
    out = ctypes.c_size_t(0)
    assert N.lib.ss_batch_workspace_size(ctypes.byref(b), ctypes.byref(opts),
                                         ctypes.byref(out)) == N.SS_E_INVALID_ARG
    res = (N.SsResult * 2)()
    assert N.lib.spar_sink_batched(ctypes.byref(b), ctypes.byref(opts), None, ctypes.c_void_p(4096),
                                   1 << 40, None, res) == N.SS_E_INVALID_ARG


def test_batch_workspace_and_schedule_checks():
    from paper_2306_06581_amd import native as N
    from paper_2306_06581_amd.api import make_options
    b, keep = _fake_batch(N, ns=(4096, 300), ms=(4096, 17), ss=(8 * 4096 * 8.3, 500.0))
    opts = make_options(0.05, precision="f32")
    out = ctypes.c_size_t(0)
    assert N.lib.ss_batch_workspace_size(ctypes.byref(b), ctypes.byref(opts), ctypes.byref(out)) == 0
    # masks of both problems and their transposes at least
    assert out.value >= 2 * (4096 * 64 + 300 * 1) * 8
    res = (N.SsResult * 2)()
    assert N.lib.spar_sink_batched(ctypes.byref(b), ctypes.byref(opts), None, ctypes.c_void_p(4096),
                                   16, None, res) == N.SS_E_WORKSPACE
    bad = N.SsSchedule(12, 256)
    assert N.lib.spar_sink_batched(ctypes.byref(b), ctypes.byref(opts), ctypes.byref(bad),
                                   ctypes.c_void_p(4096), 1 << 40, None, res) == N.SS_E_INVALID_ARG
    bad = N.SsSchedule(8, 128)
    assert N.lib.spar_sink_batched(ctypes.byref(b), ctypes.byref(opts), ctypes.byref(bad),
                                   ctypes.c_void_p(4096), 1 << 40, None, res) == N.SS_E_INVALID_ARG


@pytest.mark.parametrize("change", ["none", "init", "mlp", "d2", "small_ws", "schedule",
                                    "cost"])
def test_batch_learned_checks(change):
    # every argument of the overlapped learned solve is checked on the host,
    # before the library takes a stream or launches anything
    from paper_2306_06581_amd import native as N
    from paper_2306_06581_amd.api import make_options
    b, keep = _fake_batch(N, ns=(300, 70), ms=(200, 90), ss=(3000.0, 700.0))
    opts = make_options(0.05, precision="f32")
    mlp = N.SsMlp(4096, 8192, 12288, 0, 0, 0, 0)
    sched = None
    plain, learned = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert N.lib.ss_batch_workspace_size(ctypes.byref(b), ctypes.byref(opts),
                                         ctypes.byref(plain)) == 0
    assert N.lib.ss_batch_learned_workspace_size(ctypes.byref(b), ctypes.byref(opts),
                                                 ctypes.byref(learned)) == 0
    # the batch's workspace, the network's and both start vectors (FP64)
    assert learned.value >= plain.value + 8 * (300 + 70 + 200 + 90)
    ws_bytes, want = learned.value, N.SS_E_INVALID_ARG
    if change == "none":
        return
    if change == "init":
        opts.init_log_u = 4096
    elif change == "mlp":
        mlp.bf16 = None
    elif change == "d2":
        b.d = 2
    elif change == "small_ws":
        ws_bytes, want = learned.value - 256, N.SS_E_WORKSPACE
    elif change == "schedule":
        sched = N.SsSchedule(8, 128)
    elif change == "cost":
        opts.cost = 7
    res = (N.SsResult * 2)()
    assert N.lib.spar_sink_batched_learned(ctypes.byref(b), ctypes.byref(opts),
                                           ctypes.byref(sched) if sched is not None else None,
                                           ctypes.byref(mlp), ctypes.c_void_p(4096), ws_bytes,
                                           None, res) == want


def _ibp_problem(N, n=8, d=2, count=2, w=(0.5, 0.5)):
    warr = (ctypes.c_double * len(w))(*w)
    prob = N.SsIbpProblem(n, d, count, ctypes.c_void_p(16), ctypes.c_void_p(16),
                          ctypes.cast(warr, ctypes.c_void_p))
    return prob, warr


@pytest.mark.parametrize("change", ["count0", "count65", "wsum", "wneg", "lam", "log", "shrink",
                                    "n0", "d0", "warm"])
def test_ibp_arguments_rejected(change):
    from paper_2306_06581_amd import native as N
    from paper_2306_06581_amd import api as A
    kw = dict(n=8, d=2, count=2, w=(0.5, 0.5))
    opt = dict(eps=0.1, s=10.0)
    if change == "count0":
        kw.update(count=0, w=(1.0,))
    elif change == "count65":
        kw.update(count=65, w=(1.0 / 65,) * 65)
    elif change == "wsum":
        kw.update(w=(0.5, 0.6))
    elif change == "wneg":
        kw.update(w=(1.5, -0.5))
    elif change == "n0":
        kw.update(n=0)
    elif change == "d0":
        kw.update(d=0)
    prob, keep = _ibp_problem(N, **kw)
    o = A.make_options(lam=1.0 if change == "lam" else math.inf,
                       precision="f32_log" if change == "log" else "f64",
                       shrink=1.5 if change == "shrink" else 0.0, **opt)
    if change == "warm":
        o.init_log_u = ctypes.c_void_p(16)
    out = ctypes.c_size_t(0)
    rc = N.lib.ss_ibp_workspace_size(ctypes.byref(prob), ctypes.byref(o), ctypes.byref(out))
    assert rc == -1, change


def test_ibp_workspace_grows_with_measures():
    from paper_2306_06581_amd import native as N
    from paper_2306_06581_amd import api as A
    sizes = []
    for count in (1, 2, 4):
        prob, keep = _ibp_problem(N, n=1000, count=count, w=(1.0 / count,) * count)
        out = ctypes.c_size_t(0)
        rc = N.lib.ss_ibp_workspace_size(ctypes.byref(prob), ctypes.byref(A.make_options(eps=0.1, s=5e4)),
                                         ctypes.byref(out))
        assert rc == 0
        sizes.append(out.value)
    assert sizes[0] < sizes[1] < sizes[2]


@pytest.mark.parametrize("case", ["ot_sparse", "shrink", "eta0", "etainf"])
def test_wfr_arguments_rejected(case):
    from paper_2306_06581_amd import native as N
    from paper_2306_06581_amd import api as A
    prob = N.SsProblem(8, 8, 2, 0, ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16),
                       ctypes.c_void_p(16))
    o = A.make_options(eps=0.1, s=10.0, lam=math.inf if case == "ot_sparse" else 0.1, cost="wfr",
                       shrink=0.5 if case == "shrink" else 0.0,
                       eta={"eta0": 0.0, "etainf": math.inf}.get(case, 0.3))
    out = ctypes.c_size_t(0)
    assert N.lib.ss_workspace_size(ctypes.byref(prob), ctypes.byref(o), ctypes.byref(out)) == -1


@pytest.mark.parametrize("case", ["uot", "maxnorm", "wfr"])
def test_divergence_arguments_rejected(case):
    from paper_2306_06581_amd import native as N
    from paper_2306_06581_amd import api as A
    prob = N.SsProblem(8, 6, 2, 0, ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16),
                       ctypes.c_void_p(16))
    o = A.make_options(eps=0.1, s=10.0, lam=0.5 if case == "uot" else math.inf,
                       cost={"uot": "plain", "maxnorm": "maxnorm", "wfr": "wfr"}[case], eta=0.3)
    out = ctypes.c_size_t(0)
    assert N.lib.ss_divergence_workspace_size(ctypes.byref(prob), ctypes.byref(o),
                                              ctypes.byref(out)) == -1
    o2 = A.make_options(eps=0.1, s=10.0, cost="plain")
    assert N.lib.ss_divergence_workspace_size(ctypes.byref(prob), ctypes.byref(o2),
                                              ctypes.byref(out)) == 0
    assert out.value > 0


def test_batch_results_sequence():
    # the batched call returns its results as a lazy sequence over one copy
    # of the ss_result array: every Result equals a field-by-field read, in
    # batch order, with list-like indexing, slicing and iteration
    import numpy as np
    import torch
    from paper_2306_06581_amd import native as N
    from paper_2306_06581_amd.api import BatchResults, Result
    count = 37
    outs = (N.SsResult * count)()
    for k in range(count):
        outs[k].estimate = 0.25 * k - 3.0
        outs[k].iters = 3 * k
        outs[k].status = -3 if k % 5 == 0 else 0
        outs[k].nnz = 2 ** 40 + k
        outs[k].t_iter_ms = 0.5 + k
        outs[k].warm_start = k % 3 - 1
    res = BatchResults(outs, count)
    outs[0].iters = 999  # the sequence holds its own copy
    assert len(res) == count
    for k in range(count):
        r = res[k]
        assert isinstance(r, Result) and r is res[k]
        assert (r.estimate, r.iters, r.status, r.nnz, r.warm_start) == \
            (0.25 * k - 3.0, 3 * k, -3 if k % 5 == 0 else 0, 2 ** 40 + k, k % 3 - 1)
        assert r.t_iter_ms == np.float32(0.5 + k)
        assert r.u is None and r.v is None and r.extra == {}
    assert res[-1] is res[count - 1] and [r.iters for r in res[2:5]] == [6, 9, 12]
    assert [r.iters for r in res] == list(range(0, 3 * count, 3))
    assert (res.column("iters") == np.arange(0, 3 * count, 3)).all()
    with pytest.raises(IndexError):
        res[count]
    # per-problem views of the concatenated scalings
    u = torch.arange(10.0, dtype=torch.float64)
    off = np.array([0, 4, 4, 10] + [10] * (count - 3))
    sc = BatchResults(outs, count)
    sc._scalings(u, u, off, off)
    assert sc[0].u.tolist() == [0.0, 1.0, 2.0, 3.0] and sc[1].u.numel() == 0
    assert sc[2].v.tolist() == [4.0, 5.0, 6.0, 7.0, 8.0, 9.0]
