"""Python binding of libsparsink: argument marshalling only.

Every step of the solve runs in the HIP library; this module moves inputs to
the device as torch tensors, sizes and caches the workspace, passes raw
pointers and the current torch stream through the C ABI, and returns the host
result.  Names follow the C calls: ``spar_sink_ot``, ``spar_sink_uot``,
``dense_sinkhorn``, ``ss_sample``.
"""
from __future__ import annotations

import ctypes
import math
from collections.abc import Sequence
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import native as N

_WS: dict = {}


def _dev(t, dtype=torch.float64) -> torch.Tensor:
    if isinstance(t, torch.Tensor):
        if t.device.type != "cuda":
            t = t.to("cuda")
        return t.to(dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(t), dtype=dtype, device="cuda")


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def workspace(nbytes: int, device=None) -> torch.Tensor:
    """A cached, 256-byte aligned uint8 device buffer of at least nbytes."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    buf = _WS.get(dev)
    if buf is None or buf.numel() < nbytes:
        _WS.pop(dev, None)
        buf = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, device=dev)
        assert buf.data_ptr() % 256 == 0
        _WS[dev] = buf
    return buf


@dataclass
class Result:
    status: int
    estimate: float
    transport: float
    neg_entropy: float
    kl_a: float
    kl_b: float
    sparse_objective: float
    marginal_err: float
    cmax: float
    z_norm: float
    dropped_mass_a: float
    dropped_mass_b: float
    nnz: int
    empty_rows: int
    empty_cols: int
    iters: int
    t_prep_ms: float
    t_sample_ms: float
    t_iter_ms: float
    t_obj_ms: float
    warm_start: int = -1
    reserved: int = 0
    u: Optional[torch.Tensor] = None
    v: Optional[torch.Tensor] = None
    err_hist: Optional[torch.Tensor] = None
    extra: dict = field(default_factory=dict)


class Problem:
    """Device-resident inputs of one problem (FP64, contiguous)."""

    def __init__(self, x, y, a, b, problem_index: int = 0):
        self.x, self.y, self.a, self.b = _dev(x), _dev(y), _dev(a), _dev(b)
        if self.x.dim() != 2 or self.y.dim() != 2 or self.x.shape[1] != self.y.shape[1]:
            raise ValueError("x and y must be (n, d) and (m, d)")
        if self.a.numel() != self.x.shape[0] or self.b.numel() != self.y.shape[0]:
            raise ValueError("a must have n entries and b m entries")
        self.problem_index = int(problem_index)
        self.c = N.SsProblem(self.x.shape[0], self.y.shape[0], self.x.shape[1],
                             self.problem_index, _ptr(self.x), _ptr(self.y), _ptr(self.a),
                             _ptr(self.b))

    @property
    def n(self):
        return int(self.x.shape[0])

    @property
    def m(self):
        return int(self.y.shape[0])


def make_options(eps, s=1.0, lam=math.inf, tol=1e-6, max_iter=1000, seed=0, precision="f64",
                 cost="maxnorm", stop_rule="marginal", empty_policy="auto", block_threads=0,
                 graph_iters=0, init_log_u=None, init_log_v=None, u_out=None, v_out=None,
                 err_hist=None, shrink=0.0, eta=1.0) -> N.SsOptions:
    return N.SsOptions(float(eps), float(lam), float(s), float(tol), int(seed) & (2 ** 64 - 1),
                       int(max_iter), N.PRECISION[precision], N.COST[cost], N.STOP[stop_rule],
                       N.EMPTY[empty_policy], int(block_threads), int(graph_iters), 0,
                       _ptr(init_log_u), _ptr(init_log_v), _ptr(u_out), _ptr(v_out),
                       _ptr(err_hist), float(shrink), float(eta))


def workspace_size(prob: Problem, opts: N.SsOptions) -> int:
    out = ctypes.c_size_t(0)
    rc = N.lib.ss_workspace_size(ctypes.byref(prob.c), ctypes.byref(opts), ctypes.byref(out))
    if rc < 0:
        raise N.SparSinkError(rc, "ss_workspace_size")
    return int(out.value)


def _solve(fn_name: str, prob: Problem, *, eps, s=1.0, lam=math.inf, tol=1e-6, max_iter=1000,
           seed=0, precision="f64", cost="maxnorm", stop_rule="marginal", empty_policy="auto",
           block_threads=0, graph_iters=0, init_log_u=None, init_log_v=None, shrink=0.0,
           eta=1.0, return_scalings=False, return_hist=False, stream=None,
           raise_on_error=True) -> Result:
    u_out = torch.empty(prob.n, dtype=torch.float64, device="cuda") if return_scalings else None
    v_out = torch.empty(prob.m, dtype=torch.float64, device="cuda") if return_scalings else None
    hist = torch.full((max_iter,), float("nan"), dtype=torch.float64, device="cuda") \
        if return_hist else None
    ilu = _dev(init_log_u) if init_log_u is not None else None
    ilv = _dev(init_log_v) if init_log_v is not None else None
    opts = make_options(eps, s, lam, tol, max_iter, seed, precision, cost, stop_rule,
                        empty_policy, block_threads, graph_iters, ilu, ilv, u_out, v_out, hist,
                        shrink, eta)
    nbytes = workspace_size(prob, opts)
    ws = workspace(nbytes)
    res = N.SsResult()
    rc = getattr(N.lib, fn_name)(ctypes.byref(prob.c), ctypes.byref(opts),
                                 ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                 _stream(stream), ctypes.byref(res))
    if rc < 0 and raise_on_error:
        raise N.SparSinkError(rc, fn_name)
    out = Result(status=rc, **{k: getattr(res, k) for k, _ in N.SsResult._fields_
                               if k != "status"})
    out.u, out.v = u_out, v_out
    if hist is not None:
        out.err_hist = hist[: max(res.iters, 0)]
    return out


def spar_sink_ot(prob: Problem, **kw) -> Result:
    """Alg. 3: Spar-Sink for entropic OT (lam must stay +inf)."""
    return _solve("spar_sink_ot", prob, **kw)


def spar_sink_uot(prob: Problem, **kw) -> Result:
    """Alg. 4: Spar-Sink for entropic UOT (finite lam > 0)."""
    return _solve("spar_sink_uot", prob, **kw)


def spar_sink_ot_noalloc(prob: Problem, *, eps, s=1.0, tol=1e-6, max_iter=1000, seed=0,
                         precision="f64", cost="maxnorm", stop_rule="marginal",
                         empty_policy="auto", block_threads=0, shrink=0.0,
                         return_scalings=False, raise_on_error=True, stream=None) -> Result:
    """Alg. 3 through the allocation-free entry point: the library's static
    per-GPU scratch replaces the workspace."""
    u_out = v_out = None
    if return_scalings:
        u_out = torch.empty(prob.n, dtype=torch.float64, device="cuda")
        v_out = torch.empty(prob.m, dtype=torch.float64, device="cuda")
    opts = make_options(eps, s, math.inf, tol, max_iter, seed, precision, cost, stop_rule,
                        empty_policy, block_threads, 0, None, None, u_out, v_out, None, shrink)
    res = N.SsResult()
    rc = N.lib.spar_sink_ot_noalloc(ctypes.byref(prob.c), ctypes.byref(opts), _stream(stream),
                                    ctypes.byref(res))
    if rc < 0 and raise_on_error:
        raise N.SparSinkError(rc, "spar_sink_ot_noalloc")
    out = Result(status=rc, **{k: getattr(res, k) for k, _ in N.SsResult._fields_
                               if k != "status"})
    out.u, out.v = u_out, v_out
    return out


def dense_sinkhorn(prob: Problem, **kw) -> Result:
    """Alg. 1 / Alg. 2 with the full kernel recomputed on the fly."""
    return _solve("dense_sinkhorn", prob, **kw)


def ss_time_iterations(prob: Problem, iters: int = 64, *, eps, s=1.0, lam=math.inf, seed=0,
                       precision="f64", cost="maxnorm", block_threads=0, shrink=0.0,
                       eta=1.0, stream=None) -> float:
    """Mean duration (ms) of one iteration-kernel launch over `iters` iterations."""
    opts = make_options(eps, s, lam, seed=seed, precision=precision, cost=cost,
                        block_threads=block_threads, shrink=shrink, eta=eta)
    ws = workspace(workspace_size(prob, opts))
    ms = ctypes.c_double(0.0)
    rc = N.lib.ss_time_iterations(ctypes.byref(prob.c), ctypes.byref(opts),
                                  ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                  _stream(stream), int(iters), ctypes.byref(ms))
    if rc < 0:
        raise N.SparSinkError(rc, "ss_time_iterations")
    return float(ms.value)


def ss_sample(prob: Problem, *, eps, s, lam=math.inf, seed=0, precision="f64", cost="maxnorm",
              shrink=0.0, eta=1.0, capacity: Optional[int] = None, want_mask=True,
              z_in: float = 0.0, stream=None) -> dict:
    """Step 1 of Alg. 3/4: returns the mask words, CSR, CSC and p* factors.
    z_in > 0 (UOT): use it as the normaliser Z of eq. (pij-uot)."""
    opts = make_options(eps, s, lam, seed=seed, precision=precision, cost=cost, shrink=shrink,
                        eta=eta)
    nbytes = workspace_size(prob, opts)
    ws = workspace(nbytes)
    n, m = prob.n, prob.m
    cap = capacity if capacity is not None else int(min(n * m, math.floor(s + 8 * math.sqrt(s) + 64)))
    vdt = torch.float64 if precision == "f64" else torch.float32
    out = {
        "mask": torch.empty((n, (m + 63) // 64), dtype=torch.int64, device="cuda") if want_mask else None,
        "row_ptr": torch.empty(n + 1, dtype=torch.int64, device="cuda"),
        "col_idx": torch.empty(cap, dtype=torch.int32, device="cuda"),
        "val": torch.empty(cap, dtype=vdt, device="cuda"),
        "col_ptr": torch.empty(m + 1, dtype=torch.int64, device="cuda"),
        "row_idx": torch.empty(cap, dtype=torch.int32, device="cuda"),
        "val_t": torch.empty(cap, dtype=vdt, device="cuda"),
        "row_fac": torch.empty(n, dtype=torch.float64, device="cuda"),
        "col_fac": torch.empty(m, dtype=torch.float64, device="cuda"),
    }
    sp = N.SsSparse(*[_ptr(out[k]) for k in ("mask", "row_ptr", "col_idx", "val", "col_ptr",
                                             "row_idx", "val_t", "row_fac", "col_fac")],
                    cap, 0, 0.0, 0.0, float(z_in))
    rc = N.lib.ss_sample(ctypes.byref(prob.c), ctypes.byref(opts), ctypes.byref(sp),
                         ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                         _stream(stream))
    if rc < 0:
        raise N.SparSinkError(rc, "ss_sample")
    nnz = int(sp.nnz)
    for k in ("col_idx", "val", "row_idx", "val_t"):
        out[k] = out[k][:nnz]
    out["nnz"], out["cmax"], out["z_norm"] = nnz, sp.cmax, sp.z_norm
    return out


class Batch:
    """Device-resident inputs of a batch of OT problems (concatenated FP64)."""

    def __init__(self, xs, ys, as_, bs, s, problem_index=None):
        if not (len(xs) == len(ys) == len(as_) == len(bs) == len(s)) or len(xs) == 0:
            raise ValueError("a batch needs the same number (>= 1) of x, y, a, b and s")
        self.count = len(xs)
        self.n = np.array([len(x) for x in xs], dtype=np.int64)
        self.m = np.array([len(y) for y in ys], dtype=np.int64)
        self.d = int(np.asarray(xs[0]).shape[1])
        self.s = np.ascontiguousarray(s, dtype=np.float64)
        self.pidx = (np.arange(self.count, dtype=np.uint32) if problem_index is None
                     else np.ascontiguousarray(problem_index, dtype=np.uint32))
        self.x = _dev(np.concatenate([np.asarray(x, np.float64) for x in xs]))
        self.y = _dev(np.concatenate([np.asarray(y, np.float64) for y in ys]))
        self.a = _dev(np.concatenate([np.asarray(a, np.float64) for a in as_]))
        self.b = _dev(np.concatenate([np.asarray(b, np.float64) for b in bs]))
        self.row_off = np.concatenate([[0], np.cumsum(self.n)])
        self.col_off = np.concatenate([[0], np.cumsum(self.m)])
        self.c = N.SsBatch(self.count, self.d, self.n.ctypes.data, self.m.ctypes.data,
                           self.s.ctypes.data, self.pidx.ctypes.data, _ptr(self.x), _ptr(self.y),
                           _ptr(self.a), _ptr(self.b))

    def subset(self, k0: int, k1: int) -> "Batch":
        """Problems k0 .. k1 - 1 as a batch whose device arrays are views of
        this one's (no copy)."""
        sub = Batch.__new__(Batch)
        sub.count = k1 - k0
        sub.d = self.d
        sub.n = np.ascontiguousarray(self.n[k0:k1])
        sub.m = np.ascontiguousarray(self.m[k0:k1])
        sub.s = np.ascontiguousarray(self.s[k0:k1])
        sub.pidx = np.ascontiguousarray(self.pidx[k0:k1])
        r0, r1 = int(self.row_off[k0]), int(self.row_off[k1])
        c0, c1 = int(self.col_off[k0]), int(self.col_off[k1])
        sub.x, sub.a = self.x[r0:r1], self.a[r0:r1]
        sub.y, sub.b = self.y[c0:c1], self.b[c0:c1]
        sub.row_off = self.row_off[k0:k1 + 1] - r0
        sub.col_off = self.col_off[k0:k1 + 1] - c0
        sub.c = N.SsBatch(sub.count, sub.d, sub.n.ctypes.data, sub.m.ctypes.data,
                          sub.s.ctypes.data, sub.pidx.ctypes.data, _ptr(sub.x), _ptr(sub.y),
                          _ptr(sub.a), _ptr(sub.b))
        return sub

    @classmethod
    def from_problems(cls, probs):
        """From workload Problems (x, y, a, b, s, problem_index attributes)."""
        return cls([p.x for p in probs], [p.y for p in probs], [p.a for p in probs],
                   [p.b for p in probs], [p.s for p in probs],
                   [p.problem_index for p in probs])


def batch_workspace_size(batch: Batch, opts: N.SsOptions) -> int:
    out = ctypes.c_size_t(0)
    rc = N.lib.ss_batch_workspace_size(ctypes.byref(batch.c), ctypes.byref(opts), ctypes.byref(out))
    if rc < 0:
        raise N.SparSinkError(rc, "ss_batch_workspace_size")
    return int(out.value)


def _batched(name, batch, net, eps, tol, max_iter, seed, precision, cost, empty_policy, schedule,
             init_log_u, init_log_v, return_scalings, stream, raise_on_error):
    rows, cols = int(batch.row_off[-1]), int(batch.col_off[-1])
    u_out = torch.empty(rows, dtype=torch.float64, device="cuda") if return_scalings else None
    v_out = torch.empty(cols, dtype=torch.float64, device="cuda") if return_scalings else None
    ilu = _dev(init_log_u) if init_log_u is not None else None
    ilv = _dev(init_log_v) if init_log_v is not None else None
    if (ilu is not None and ilu.numel() != rows) or (ilv is not None and ilv.numel() != cols):
        raise ValueError("init_log_u / init_log_v need sum(n) / sum(m) entries")
    opts = make_options(eps, 1.0, math.inf, tol, max_iter, seed, precision, cost, "marginal",
                        empty_policy, 0, 0, ilu, ilv, u_out, v_out, None)
    nb = ctypes.c_size_t(0)
    size_fn = N.lib.ss_batch_learned_workspace_size if net is not None else \
        N.lib.ss_batch_workspace_size
    rc = size_fn(ctypes.byref(batch.c), ctypes.byref(opts), ctypes.byref(nb))
    if rc < 0:
        raise N.SparSinkError(rc, size_fn.__name__)
    ws = workspace(nb.value)
    outs = (N.SsResult * batch.count)()
    sched = N.SsSchedule(*schedule) if schedule is not None else None
    args = [ctypes.byref(batch.c), ctypes.byref(opts),
            ctypes.byref(sched) if sched is not None else None]
    if net is not None:
        args.append(ctypes.byref(net.c))
    rc = getattr(N.lib, name)(*args, ctypes.c_void_p(ws.data_ptr()),
                              ctypes.c_size_t(ws.numel()), _stream(stream), outs)
    if rc < 0 and raise_on_error and rc not in (N.SS_E_NONFINITE, N.SS_E_EMPTY):
        raise N.SparSinkError(rc, name)
    res = BatchResults(outs, batch.count)
    if return_scalings:
        res._scalings(u_out, v_out, batch.row_off, batch.col_off)
    return rc, res


_RESULT_NAMES = tuple(f for f, _ in N.SsResult._fields_)
_RESULT_DTYPE = np.dtype(N.SsResult)


class BatchResults(Sequence):
    """The Result of every problem of a batched solve, in batch order.

    Each Result (and its u / v views) is built on first access from a copy of
    the library's ss_result array, so returning a batch of thousands costs no
    Python work per problem; column(name) gives one field of every problem as
    a NumPy array."""

    def __init__(self, outs, count: int):
        self._rows = np.frombuffer(outs, dtype=_RESULT_DTYPE, count=count).copy()
        self._cache = [None] * count
        self._uv = None

    def _scalings(self, u_out, v_out, row_off, col_off):
        self._uv = (u_out, v_out, row_off, col_off)

    def __len__(self) -> int:
        return len(self._cache)

    def __getitem__(self, k):
        if isinstance(k, slice):
            return [self[i] for i in range(*k.indices(len(self)))]
        r = self._cache[k]  # IndexError past the end, as a list
        if r is None:
            k = k % len(self)
            r = object.__new__(Result)
            r.__dict__.update(zip(_RESULT_NAMES, self._rows[k].tolist()))
            r.__dict__.update(u=None, v=None, err_hist=None, extra={})
            if self._uv is not None:
                u, v, ro, co = self._uv
                r.u, r.v = u[ro[k]:ro[k + 1]], v[co[k]:co[k + 1]]
            self._cache[k] = r
        return r

    def column(self, name: str) -> np.ndarray:
        return self._rows[name].copy()


def spar_sink_batched(batch: Batch, *, eps, tol=1e-6, max_iter=1000, seed=0, precision="f32",
                      cost="maxnorm", empty_policy="auto", schedule=None, init_log_u=None,
                      init_log_v=None, return_scalings=False, stream=None,
                      raise_on_error=True):
    """Alg. 3 for every problem of the batch; returns (status, BatchResults),
    one Result per problem in batch order.

    schedule: (lanes_per_line, block_threads), or None for the library's default
    (8, 1024); ss_autotune_batched picks one for a given batch.
    With return_scalings, each Result carries its u and v (FP64 device views)."""
    return _batched("spar_sink_batched", batch, None, eps, tol, max_iter, seed, precision, cost,
                    empty_policy, schedule, init_log_u, init_log_v, return_scalings, stream,
                    raise_on_error)


def spar_sink_batched_learned(batch: Batch, net: "WarmStartNet", *, eps, tol=1e-6,
                              max_iter=1000, seed=0, precision="f32", cost="maxnorm",
                              empty_policy="auto", schedule=None, return_scalings=False,
                              stream=None, raise_on_error=True):
    """spar_sink_batched started from net's prediction, which the library
    computes on a second stream beside the sampling stage (d = 3)."""
    return _batched("spar_sink_batched_learned", batch, net, eps, tol, max_iter, seed, precision,
                    cost, empty_policy, schedule, None, None, return_scalings, stream,
                    raise_on_error)


def ss_autotune_batched(batch: Batch, *, eps, seed=0, precision="f32", cost="maxnorm",
                        stream=None):
    """Times every candidate schedule; returns ((lanes_per_line, block_threads), {schedule: ms})."""
    opts = make_options(eps, 1.0, math.inf, 1e-6, 16, seed, precision, cost, "marginal")
    ws = workspace(batch_workspace_size(batch, opts))
    best = N.SsSchedule()
    ms = (ctypes.c_float * 16)()
    nc = ctypes.c_int32(16)
    rc = N.lib.ss_autotune_batched(ctypes.byref(batch.c), ctypes.byref(opts),
                                   ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                   _stream(stream), ctypes.byref(best), ms, ctypes.byref(nc))
    if rc < 0:
        raise N.SparSinkError(rc, "ss_autotune_batched")
    cands = [(l, b) for l in (4, 8, 16, 32) for b in (256, 512, 1024)]
    return (best.lanes_per_line, best.block_threads), {c: float(ms[i]) for i, c in
                                                          enumerate(cands[: nc.value])}


# ---------------------------------------------------------------- warm start
_MLP_SHAPES = (("P", (256, 4)), ("p", (256,)), ("W1", (256, 3)), ("U", (256, 256)),
               ("c1", (256,)), ("W2", (256, 256)), ("c2", (256,)), ("w3", (256,)), ("c3", (1,)))


class WarmStartNet:
    """Device weights and Adam state of the DeepSets warm-start network."""

    def __init__(self, flat=None, seed: int = 0):
        if flat is None:
            flat = self.initial_weights(seed)
        flat = np.asarray(flat, dtype=np.float32)
        if flat.size != N.MLP_PARAMS:
            raise ValueError(f"expected {N.MLP_PARAMS} weights")
        self.params = torch.tensor(flat, device="cuda")
        self.bf16 = torch.empty(N.MLP_PARAMS, dtype=torch.bfloat16, device="cuda")
        self.w2t = torch.empty(256 * 256, dtype=torch.bfloat16, device="cuda")
        self.adam_m = torch.zeros(N.MLP_PARAMS, dtype=torch.float32, device="cuda")
        self.adam_v = torch.zeros(N.MLP_PARAMS, dtype=torch.float32, device="cuda")
        self.c = N.SsMlp(_ptr(self.params), _ptr(self.bf16), _ptr(self.w2t), _ptr(self.adam_m),
                         _ptr(self.adam_v), 0, 0)
        rc = N.lib.ss_mlp_sync(ctypes.byref(self.c), _stream())
        if rc < 0:
            raise N.SparSinkError(rc, "ss_mlp_sync")

    @staticmethod
    def initial_weights(seed: int = 0) -> np.ndarray:
        """He-scaled Gaussian matrices for the ReLU layers, small first bias."""
        rng = np.random.default_rng(seed)
        scale = {"P": np.sqrt(2 / 4), "W1": np.sqrt(2 / 3), "U": np.sqrt(1 / 256),
                 "W2": np.sqrt(2 / 256), "w3": np.sqrt(1 / 256)}
        parts = []
        for name, shape in _MLP_SHAPES:
            if name in scale:
                parts.append(rng.standard_normal(shape).ravel() * scale[name])
            else:
                parts.append(np.full(int(np.prod(shape)), 0.01 if name == "c1" else 0.0))
        return np.concatenate(parts).astype(np.float32)

    @property
    def step(self) -> int:
        return int(self.c.step)

    def weights(self) -> np.ndarray:
        return self.params.cpu().numpy()

    def bf16_weights(self) -> np.ndarray:
        return self.bf16.float().cpu().numpy()

    def predict(self, batch: "Batch", eps: float, cost="maxnorm", stream=None):
        """(log u^0, log v^0) as FP64 device tensors of sum(n), sum(m) entries
        for a solve with this eps and cost."""
        out_u = torch.empty(int(batch.row_off[-1]), dtype=torch.float64, device="cuda")
        out_v = torch.empty(int(batch.col_off[-1]), dtype=torch.float64, device="cuda")
        nb = ctypes.c_size_t(0)
        rc = N.lib.ss_warmstart_workspace_size(ctypes.byref(batch.c), ctypes.byref(nb))
        if rc < 0:
            raise N.SparSinkError(rc, "ss_warmstart_workspace_size")
        ws = workspace(nb.value)
        rc = N.lib.ss_warmstart_predict(ctypes.byref(self.c), ctypes.byref(batch.c), float(eps),
                                        N.COST[cost], _ptr(out_u), _ptr(out_v),
                                        ctypes.c_void_p(ws.data_ptr()),
                                        ctypes.c_size_t(ws.numel()), _stream(stream))
        if rc < 0:
            raise N.SparSinkError(rc, "ss_warmstart_predict")
        return out_u, out_v

    def train_step(self, batch: "Batch", tgt_log_u, tgt_log_v, lr: float, eps: float,
                   cost="maxnorm", want_grad=False, stream=None):
        """One Adam step; returns the loss before it (and the gradient)."""
        tu, tv = _dev(tgt_log_u), _dev(tgt_log_v)
        if tu.numel() != int(batch.row_off[-1]) or tv.numel() != int(batch.col_off[-1]):
            raise ValueError("targets need sum(n) and sum(m) entries")
        grad = torch.empty(N.MLP_PARAMS, dtype=torch.float32, device="cuda") if want_grad else None
        nb = ctypes.c_size_t(0)
        rc = N.lib.ss_warmstart_workspace_size(ctypes.byref(batch.c), ctypes.byref(nb))
        if rc < 0:
            raise N.SparSinkError(rc, "ss_warmstart_workspace_size")
        ws = workspace(nb.value)
        loss = ctypes.c_float(0.0)
        rc = N.lib.ss_warmstart_train_step(ctypes.byref(self.c), ctypes.byref(batch.c), float(eps),
                                           N.COST[cost], _ptr(tu), _ptr(tv), float(lr),
                                           ctypes.c_void_p(ws.data_ptr()),
                                           ctypes.c_size_t(ws.numel()), _stream(stream),
                                           ctypes.byref(loss), _ptr(grad))
        if rc < 0:
            raise N.SparSinkError(rc, "ss_warmstart_train_step")
        return (float(loss.value), grad) if want_grad else float(loss.value)


# ---------------------------------------------------------------- Spar-IBP
class IBPProblem:
    """Device-resident inputs of one barycenter problem: support x (n, d),
    measures b (count, n) and host weights w (count)."""

    def __init__(self, x, b, w):
        self.x = _dev(x)
        self.b = _dev(b)
        if self.x.dim() != 2:
            raise ValueError("x must be (n, d)")
        if self.b.dim() == 1:
            self.b = self.b.reshape(1, -1)
        if self.b.dim() != 2 or self.b.shape[1] != self.x.shape[0]:
            raise ValueError("b must be (count, n)")
        self.b = self.b.contiguous()
        self.w = np.ascontiguousarray(w, dtype=np.float64)
        if self.w.size != self.b.shape[0]:
            raise ValueError("w must have one entry per measure")
        self.c = N.SsIbpProblem(self.x.shape[0], self.x.shape[1], self.b.shape[0], _ptr(self.x),
                                _ptr(self.b), self.w.ctypes.data)

    @property
    def n(self):
        return int(self.x.shape[0])

    @property
    def count(self):
        return int(self.b.shape[0])


@dataclass
class IBPResult:
    status: int
    q: torch.Tensor
    err: float
    cmax: float
    nnz: int
    empty_rows: int
    empty_cols: int
    iters: int
    t_sample_ms: float
    t_iter_ms: float
    u: Optional[torch.Tensor] = None
    v: Optional[torch.Tensor] = None
    err_hist: Optional[torch.Tensor] = None


def _ibp_options(eps, s, tol, max_iter, seed, precision, cost, shrink, graph_iters,
                 u_out=None, v_out=None, err_hist=None) -> N.SsOptions:
    return make_options(eps, s, math.inf, tol, max_iter, seed, precision, cost, "marginal",
                        "auto", 0, graph_iters, None, None, u_out, v_out, err_hist, shrink)


def ibp_workspace_size(prob: IBPProblem, opts: N.SsOptions) -> int:
    out = ctypes.c_size_t(0)
    rc = N.lib.ss_ibp_workspace_size(ctypes.byref(prob.c), ctypes.byref(opts), ctypes.byref(out))
    if rc < 0:
        raise N.SparSinkError(rc, "ss_ibp_workspace_size")
    return int(out.value)


def spar_ibp(prob: IBPProblem, *, eps, s, tol=1e-6, max_iter=1000, seed=0, precision="f64",
             cost="maxnorm", shrink=0.0, graph_iters=0, return_scalings=False, return_hist=False,
             stream=None, raise_on_error=True) -> IBPResult:
    """Alg. Spar-IBP: the barycenter q of the measures on the shared support."""
    n, K = prob.n, prob.count
    q = torch.empty(n, dtype=torch.float64, device="cuda")
    u_out = torch.empty((K, n), dtype=torch.float64, device="cuda") if return_scalings else None
    v_out = torch.empty((K, n), dtype=torch.float64, device="cuda") if return_scalings else None
    hist = torch.full((max_iter,), float("nan"), dtype=torch.float64, device="cuda") \
        if return_hist else None
    opts = _ibp_options(eps, s, tol, max_iter, seed, precision, cost, shrink, graph_iters, u_out,
                        v_out, hist)
    ws = workspace(ibp_workspace_size(prob, opts))
    res = N.SsIbpResult()
    rc = N.lib.spar_ibp(ctypes.byref(prob.c), ctypes.byref(opts), _ptr(q),
                        ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                        _stream(stream), ctypes.byref(res))
    if rc < 0 and raise_on_error:
        raise N.SparSinkError(rc, "spar_ibp")
    out = IBPResult(status=rc, q=q, **{k: getattr(res, k) for k, _ in N.SsIbpResult._fields_
                                       if k != "status"})
    out.u, out.v = u_out, v_out
    if hist is not None:
        out.err_hist = hist[: max(res.iters, 0)]
    return out


def ss_ibp_sample(prob: IBPProblem, k: int, *, eps, s, seed=0, precision="f64", cost="maxnorm",
                  shrink=0.0, capacity: Optional[int] = None, stream=None) -> dict:
    """eq. (pois-k): the sketch of measure k (mask, CSR, CSC, factors)."""
    opts = _ibp_options(eps, s, 1e-6, 1, seed, precision, cost, shrink, 0)
    ws = workspace(ibp_workspace_size(prob, opts))
    n = prob.n
    cap = capacity if capacity is not None else int(min(n * n, math.floor(s + 8 * math.sqrt(s) + 64)))
    vdt = torch.float64 if precision == "f64" else torch.float32
    out = {
        "mask": torch.empty((n, (n + 63) // 64), dtype=torch.int64, device="cuda"),
        "row_ptr": torch.empty(n + 1, dtype=torch.int64, device="cuda"),
        "col_idx": torch.empty(cap, dtype=torch.int32, device="cuda"),
        "val": torch.empty(cap, dtype=vdt, device="cuda"),
        "col_ptr": torch.empty(n + 1, dtype=torch.int64, device="cuda"),
        "row_idx": torch.empty(cap, dtype=torch.int32, device="cuda"),
        "val_t": torch.empty(cap, dtype=vdt, device="cuda"),
        "row_fac": torch.empty(n, dtype=torch.float64, device="cuda"),
        "col_fac": torch.empty(n, dtype=torch.float64, device="cuda"),
    }
    sp = N.SsSparse(*[_ptr(out[key]) for key in ("mask", "row_ptr", "col_idx", "val", "col_ptr",
                                                 "row_idx", "val_t", "row_fac", "col_fac")],
                    cap, 0, 0.0, 0.0)
    rc = N.lib.ss_ibp_sample(ctypes.byref(prob.c), ctypes.byref(opts), int(k), ctypes.byref(sp),
                             ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                             _stream(stream))
    if rc < 0:
        raise N.SparSinkError(rc, "ss_ibp_sample")
    nnz = int(sp.nnz)
    for key in ("col_idx", "val", "row_idx", "val_t"):
        out[key] = out[key][:nnz]
    out["nnz"], out["cmax"] = nnz, sp.cmax
    return out


def ss_ibp_time_iterations(prob: IBPProblem, iters: int = 64, *, eps, s, seed=0, precision="f64",
                           cost="maxnorm", shrink=0.0, stream=None) -> tuple:
    """(mean ms of one Spar-IBP step over `iters` graph-replayed steps, nnz)."""
    opts = _ibp_options(eps, s, 0.0, iters, seed, precision, cost, shrink, 0)
    ws = workspace(ibp_workspace_size(prob, opts))
    ms = ctypes.c_double(0.0)
    nnz = ctypes.c_int64(0)
    rc = N.lib.ss_ibp_time_iterations(ctypes.byref(prob.c), ctypes.byref(opts),
                                      ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                      _stream(stream), int(iters), ctypes.byref(ms),
                                      ctypes.byref(nnz))
    if rc < 0:
        raise N.SparSinkError(rc, "ss_ibp_time_iterations")
    return float(ms.value), int(nnz.value)


# ---------------------------------------------------------------- divergence
@dataclass
class DivergenceResult:
    status: int
    value: float
    value_sparse: float
    ot_xy: float
    ot_xx: float
    ot_yy: float
    sparse_xy: float
    sparse_xx: float
    sparse_yy: float
    nnz: int
    iters_xy: int
    iters_xx: int
    iters_yy: int
    grad_x: Optional[torch.Tensor] = None
    grad_y: Optional[torch.Tensor] = None


def sinkhorn_divergence(prob: Problem, *, eps, s, tol=1e-6, max_iter=1000, seed=0,
                        precision="f64", shrink=0.0, graph_iters=0, cost="plain",
                        return_grad=True, stream=None, raise_on_error=True) -> DivergenceResult:
    """eq. (sink-div) from three Spar-Sink OT solves, with the envelope
    gradients in x and y; cost "plain" (|x - y|^2) or "euclid" (|x - y|),
    both unnormalised."""
    opts = make_options(eps, s, math.inf, tol, max_iter, seed, precision, cost, "marginal",
                        "auto", 0, graph_iters, shrink=shrink)
    out = ctypes.c_size_t(0)
    rc = N.lib.ss_divergence_workspace_size(ctypes.byref(prob.c), ctypes.byref(opts),
                                            ctypes.byref(out))
    if rc < 0:
        raise N.SparSinkError(rc, "ss_divergence_workspace_size")
    ws = workspace(int(out.value))
    gx = torch.empty_like(prob.x) if return_grad else None
    gy = torch.empty_like(prob.y) if return_grad else None
    res = N.SsDivergence()
    rc = N.lib.ss_sinkhorn_divergence(ctypes.byref(prob.c), ctypes.byref(opts), _ptr(gx), _ptr(gy),
                                      ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                      _stream(stream), ctypes.byref(res))
    if rc < 0 and raise_on_error:
        raise N.SparSinkError(rc, "ss_sinkhorn_divergence")
    return DivergenceResult(status=rc, grad_x=gx, grad_y=gy,
                            **{k: getattr(res, k) for k, _ in N.SsDivergence._fields_
                               if k != "status"})
