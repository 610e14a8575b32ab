"""Learned warm start: training data from the method's own solutions, training
with the library's GPU step, and evaluation against the plain start.

The network and its step live in the HIP library (``ss_warmstart_*``); this
module only schedules them: it solves batches with ``spar_sink_batched`` to
get log u*, log v*, cuts them into minibatches, calls the training step, and
compares iteration counts and times to a tolerance with and without the
predicted start.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import api as A


@dataclass
class Minibatch:
    batch: A.Batch
    tgt_u: torch.Tensor
    tgt_v: torch.Tensor


def solution_minibatches(problems, *, eps, seed, minibatch=64, precision="f32", tol=1e-6,
                         max_iter=1000):
    """Solves the problems as one batch and returns minibatches of
    (problems, log u*, log v*); lines without entries have -inf targets, which
    the loss leaves out."""
    B = A.Batch.from_problems(problems)
    rc, res = A.spar_sink_batched(B, eps=eps, tol=tol, max_iter=max_iter, seed=seed,
                                  precision=precision, return_scalings=True)
    if rc < 0:
        raise RuntimeError(f"spar_sink_batched failed: {rc}")
    out = []
    for i in range(0, len(problems), minibatch):
        j = min(i + minibatch, len(problems))
        lu = torch.cat([torch.log(r.u) for r in res[i:j]])
        lv = torch.cat([torch.log(r.v) for r in res[i:j]])
        out.append(Minibatch(B.subset(i, j), lu, lv))
    return out


def train(net: A.WarmStartNet, minibatches, *, eps, lr=1e-3, epochs=1):
    """Adam steps over the minibatches; returns the losses."""
    losses = []
    for _ in range(epochs):
        for mb in minibatches:
            losses.append(net.train_step(mb.batch, mb.tgt_u, mb.tgt_v, lr=lr, eps=eps))
    return losses


def evaluate(net: A.WarmStartNet, problems, *, eps, seed, tol=1e-6, max_iter=1000,
             precision="f32", schedule=None, repeats=3):
    """Iterations and wall time to tol from the plain start and from the
    predicted one, on the same batch; the prediction time is reported apart,
    and the solve that predicts on a second stream beside its sampling
    (spar_sink_batched_learned) is timed whole."""
    B = A.Batch.from_problems(problems)
    kw = dict(eps=eps, tol=tol, max_iter=max_iter, seed=seed, precision=precision,
              schedule=schedule)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(repeats):
            out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) * 1e3 / repeats

    (lu, lv), t_pred = timed(lambda: net.predict(B, eps=eps))
    (rc0, cold), t_cold = timed(lambda: A.spar_sink_batched(B, **kw))
    (rc1, warm), t_warm = timed(lambda: A.spar_sink_batched(B, init_log_u=lu, init_log_v=lv, **kw))
    (rc2, fused), t_fused = timed(lambda: A.spar_sink_batched_learned(B, net, **kw))
    same = all(f.iters == w.iters and f.estimate == w.estimate and f.status == w.status
               for f, w in zip(fused, warm))
    both = [i for i in range(len(problems)) if cold[i].status == 0 and warm[i].status == 0]
    ic = np.array([cold[i].iters for i in both], dtype=np.float64)
    iw = np.array([warm[i].iters for i in both], dtype=np.float64)
    dev = max((abs(warm[i].estimate - cold[i].estimate) / max(abs(cold[i].estimate), 1e-300)
               for i in both), default=0.0)
    return {"problems": len(problems), "converged_both": len(both),
            "iters_plain_mean": float(ic.mean()), "iters_learned_mean": float(iw.mean()),
            "iters_saved_frac": float(1.0 - iw.mean() / ic.mean()),
            "batch_ms_plain": t_cold, "batch_ms_learned": t_warm, "predict_ms": t_pred,
            "batch_ms_learned_overlapped": t_fused, "overlapped_matches_two_calls": same,
            "loop_ms_plain": cold[0].t_iter_ms, "loop_ms_learned": warm[0].t_iter_ms,
            "max_rel_estimate_change": dev}
