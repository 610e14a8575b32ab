"""Benchmark: seconds to a 1e-6 marginal error, Spar-Sink vs dense Sinkhorn, and
the HBM bandwidth of the sparse iteration kernel, on one MI355X.

Workload (default): UOT between n = m = 65536 points in R^3, x from an equal
mixture of three isotropic Gaussians, y = x + N(0, 0.1^2 I), masses U(0,1)
scaled to totals 1.0 and 1.3, lambda = 1, eps = 0.05, normalised squared
Euclidean cost, s = 8 n ln n, log-domain FP32 iteration with FP64 potentials,
stop at L1 fixed-point residual <= 1e-6.

A step is one whole Spar-Sink solve (probabilities, hash mask, CSR/CSC,
Sinkhorn loop to tolerance, estimate) with the inputs already in HBM.  The
dense baseline (same stop rule and tolerance, K recomputed on the fly) is
timed on the same GPU.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "s to 1e-6 marginal err, Spar-Sink vs dense Sinkhorn; SpMV HBM GB/s"
HBM_PEAK_GBPS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--eps", type=float, default=0.05)
    ap.add_argument("--s-factor", type=float, default=8.0,
                    help="budget s = factor * n ln n of the headline workload")
    ap.add_argument("--precision", default="f32_log")
    ap.add_argument("--dense-precision", default="auto")
    ap.add_argument("--dense-runs", type=int, default=1)
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--timing-iters", type=int, default=64)
    ap.add_argument("--kernel-only", action="store_true",
                    help="only sample once and time the iteration kernel (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="copy 1 GiB device to device three times (PMC byte-counter scale)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched workload (profiling runs)")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched workload on the library's default schedule (counter runs)")
    ap.add_argument("--warmstart-train", type=int, default=100_000,
                    help="training problems for the learned warm start (0: skip)")
    ap.add_argument("--warmstart-only", action="store_true")
    ap.add_argument("--predict-only", action="store_true",
                    help="only the warm-start prediction for the batched workload (untrained "
                         "weights; profiling runs)")
    ap.add_argument("--no-ibp", action="store_true")
    ap.add_argument("--ibp-only", action="store_true", help="only the Spar-IBP workload")
    ap.add_argument("--ibp-n", type=int, default=16384)
    ap.add_argument("--no-wfr", action="store_true")
    ap.add_argument("--wfr-only", action="store_true", help="only the WFR workload")
    ap.add_argument("--wfr-n", type=int, default=65536)
    ap.add_argument("--no-divergence", action="store_true")
    ap.add_argument("--no-eps-small", action="store_true")
    ap.add_argument("--no-hbm", action="store_true")
    ap.add_argument("--no-ot-scale", action="store_true")
    ap.add_argument("--sections-only", action="store_true",
                    help="only the eps 0.01, HBM-resident and OT-scale sections")
    ap.add_argument("--divergence-only", action="store_true")
    ap.add_argument("--divergence-n", type=int, default=4096)
    return ap.parse_args()


PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "k_iterate_uot_mix3_n65536_f32_log_traffic.txt")
PROFILE_TRAFFIC_S32 = os.path.join(ROOT, "profiles",
                                   "k_iterate_uot_mix3_n65536_s32_f32_log_traffic.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2306_06581_amd", "csrc", "iterate.hip")


def iteration_bytes_per_launch(precision: str, nnz: int, n: int, m: int) -> float:
    """Algorithmic HBM bytes of one iteration-kernel launch, averaged over the
    u-launch (CSR, n lines) and the v-launch (CSC, m lines).

    Per stored entry: its value and a 4-byte column index.  Per line: its
    int64 offset, FP64 mass, the previous and the new scaling (FP64 potential
    plus its FP32 gathered copy in the log domain).  The gathered vector of
    the other side is counted once (it stays in cache)."""
    ev = 8 if precision == "f64" else 4                  # stored value
    ys = {"f64": 8, "f32": 4, "f32_log": 8}[precision]   # stored scaling / potential
    gs = 8 if precision == "f64" else 4                  # gathered copy
    per_line = 8 + 8 + 2 * ys + (4 if precision == "f32_log" else 0)
    u = nnz * (ev + 4) + n * per_line + m * gs
    v = nnz * (ev + 4) + m * per_line + n * gs
    return (u + v) / 2.0


def measured_traffic(bytes_launch: float, path: str = PROFILE_TRAFFIC):
    """HBM bytes per iteration launch from the committed PMC summary, scaled
    by the copy calibration; None when the summary is missing or the kernel
    source changed since the counters were taken."""
    import hashlib
    try:
        kv = {}
        for line in open(path):
            parts = line.split()
            if len(parts) == 2 and not line.startswith("#"):
                kv[parts[0]] = parts[1]
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
        if kv.get("kernel_source_sha256") != src:
            return None
        fetch = float(kv["fetch_kib_per_dispatch"]) * 1024 * float(kv["copy_fetch_scale"])
        write = float(kv["write_kib_per_dispatch"]) * 1024 * float(kv["copy_write_scale"])
        return {"bytes": fetch + write, "fetch_bytes": fetch, "write_bytes": write,
                "ratio_to_algorithmic": (fetch + write) / bytes_launch}
    except (OSError, KeyError, ValueError):
        return None


def copy_calibration():
    """1 GiB device-to-device copies: each reads and writes exactly 2^30 bytes."""
    import torch
    torch.cuda.set_device(0)
    n = 2 ** 30 // 4
    a = torch.ones(n, device="cuda")
    b = torch.empty(n, device="cuda")
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 2 ** 30, "copy_bytes_written": 2 ** 30, "copies": 3}))


def batched_bench(count: int, steps: int, autotune: bool = True) -> dict:
    """512 OT problems, n_k = m_k ~ U{256..4096}, d = 3, Dirichlet weights,
    eps = 0.05, s_k = 8 n_k ln n_k, FP32, tol 1e-6 with at most 1000 iterations
    (the paper's cap): one batched solve per step.  A sampled support can
    admit no exact fit of the marginals (the error then stalls above tol); such
    problems stop at the cap and are reported as not converged."""
    import torch

    from paper_2306_06581_amd import api as A
    from paper_2306_06581_amd import workloads as W

    probs = W.batch_ot(count, seed=0)
    B = A.Batch.from_problems(probs)
    t0 = time.perf_counter()
    if autotune:
        sched, cand = A.ss_autotune_batched(B, eps=0.05, seed=0, precision="f32")
    else:
        sched, cand = (8, 1024), {}
    t_tune = time.perf_counter() - t0
    kw = dict(eps=0.05, tol=1e-6, max_iter=1000, seed=0, precision="f32", schedule=sched)
    A.spar_sink_batched(B, **kw)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rc, res = A.spar_sink_batched(B, **kw)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    if rc < 0:
        raise SystemExit(f"batched solve failed with status {rc}")
    iters = res.column("iters")
    nnz = res.column("nnz").astype(np.float64)
    n = np.array([p.n for p in probs], dtype=np.float64)
    m = np.array([p.m for p in probs], dtype=np.float64)
    # per iteration of a problem: value (4 B) + 16-bit index per entry in both
    # directions, int64 line pointer and FP64 marginal per line; the scalings
    # stay in LDS
    bytes_iter = nnz * 2 * (4 + 2) + (n + m) * (8 + 8)
    moved = float(np.sum(bytes_iter * (iters + 1)))
    t_iter = res[0].t_iter_ms
    gbps = moved / (t_iter * 1e-3) / 1e9
    return {"workload": f"batch_ot {count} problems n_k=m_k~U{{256..4096}} d=3 eps=0.05 "
                        f"s_k=8 n_k ln n_k f32 tol=1e-6 max_iter=1000",
            "ms_per_batch": ms, "problems_per_s": count / (ms * 1e-3),
            "iters_mean": float(iters.mean()), "iters_max": int(iters.max()),
            "nnz_total": int(nnz.sum()), "schedule": {"lanes_per_line": sched[0],
                                                      "block_threads": sched[1]},
            "autotune_s": t_tune, "candidates_ms": {f"{l}x{b}": v for (l, b), v in cand.items()},
            "stage_ms": {"sample": res[0].t_sample_ms, "iterate": t_iter,
                         "objective": res[0].t_obj_ms},
            "loop_bytes": moved, "loop_GBps": gbps, "loop_frac_of_8TBps": gbps / HBM_PEAK_GBPS,
            "converged": int(np.sum(res.column("status") == 0)),
            "max_marginal_err": float(res.column("marginal_err").max())}


def warmstart_bench(ntrain: int, count: int) -> dict:
    """The DeepSets warm start trained on the GPU with the library's own step:
    ntrain problems of the batched workload's generator (seeds 1000 + k, one
    chunk of 512 per seed), targets from spar_sink_batched (FP32, tol 1e-6),
    one pass in minibatches of 64 with Adam (lr 1e-3); evaluated on the
    batched workload itself (seed 0) against the plain start."""
    import torch

    from paper_2306_06581_amd import api as A
    from paper_2306_06581_amd import warmstart as WS
    from paper_2306_06581_amd import workloads as W

    net = A.WarmStartNet(seed=0)
    chunk = 512
    t_gen = t_train = 0.0
    losses = []
    for c in range((ntrain + chunk - 1) // chunk):
        probs = W.batch_ot(min(chunk, ntrain - c * chunk), seed=1000 + c)
        t0 = time.perf_counter()
        mbs = WS.solution_minibatches(probs, eps=0.05, seed=1000 + c)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        losses += WS.train(net, mbs, eps=0.05, lr=1e-3)
        torch.cuda.synchronize()
        t_gen += t1 - t0
        t_train += time.perf_counter() - t1
    ev = WS.evaluate(net, W.batch_ot(count, seed=0), eps=0.05, seed=0)
    ev.update({"train_problems": ntrain, "train_steps": len(losses),
               "loss_first": float(np.mean(losses[:20])), "loss_last": float(np.mean(losses[-20:])),
               "data_s": t_gen, "train_s": t_train,
               "train_ms_per_step": t_train * 1e3 / max(len(losses), 1)})
    return ev


def ibp_step_bytes(nnz: int, n: int, count: int, precision: str) -> float:
    """Algorithmic HBM bytes of one Spar-IBP step (column launch + row launch).

    Per stored entry, in both directions: its value and a 4-byte index.  Per
    measure and line: the two int64 offsets (CSR and CSC), b_k read, v_k and u_k
    written, and the gathered u_k and v_k counted once (they stay in cache).
    Per step: the barycenter read and written."""
    ev = 8 if precision == "f64" else 4
    return 2.0 * nnz * (ev + 4) + count * (2 * 8 * (n + 1) + 3 * 8 * n + 2 * 8 * n) + 2 * 8 * n


def ibp_bench(n: int, steps: int, cpu: bool) -> dict:
    """Spar-IBP (barycenter of three measures, the paper's barycenter
    simulation scaled up): n support points in (0,1)^5, eps = 0.05 on the
    normalised cost, s = 20 s0(n) per measure, FP32 stored values, stop at
    |q^t - q^(t-1)|_1 <= 1e-8.  Also the paper's own size n = 1000."""
    import torch

    from paper_2306_06581_amd import api as A
    from paper_2306_06581_amd import workloads as W

    out = {}
    for nn in (n, 1000):
        p = W.ibp_synthetic(nn, d=5, seed=0, eps=0.05, s_factor=20.0)
        prob = A.IBPProblem(p.x, p.b, p.w)
        kw = dict(eps=p.eps, s=p.s, seed=p.seed, tol=1e-8, max_iter=5000, precision="f32")
        A.spar_ibp(prob, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [A.spar_ibp(prob, **kw) for _ in range(steps)]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        r = res[-1]
        ms_it, nnz = A.ss_ibp_time_iterations(prob, 64, eps=p.eps, s=p.s, seed=p.seed,
                                              precision="f32")
        by = ibp_step_bytes(nnz, nn, p.count, "f32")
        gbps = by / (ms_it * 1e-3) / 1e9
        out[f"n{nn}"] = {
            "workload": f"ibp_synthetic n={nn} d=5 3 measures eps=0.05 s=20 s0(n) f32 tol=1e-8",
            "ms_per_solve": ms, "iters": r.iters, "status": r.status, "err": r.err,
            "nnz": r.nnz, "stage_ms": {"sample": r.t_sample_ms, "iterate": r.t_iter_ms},
            "ms_per_step": ms_it, "bytes_per_step": by, "step_GBps": gbps,
            "step_frac_of_8TBps": gbps / HBM_PEAK_GBPS}
        if cpu and nn == 1000:
            from oracle import ibp_oracle as I
            t0 = time.perf_counter()
            o = I.spar_ibp(p.x, p.b, p.w, p.eps, p.s, seed=p.seed, tol=1e-8, max_iter=5000)
            out[f"n{nn}"]["cpu_oracle"] = {"s": time.perf_counter() - t0, "iters": o.ibp.iters,
                                           "cores": 1, "kind": "oracle",
                                           "l1_vs_gpu": float(np.abs(o.ibp.q -
                                                                     r.q.cpu().numpy()).sum())}
    return out


def wfr_bench(n: int, steps: int, dense: bool) -> dict:
    """UOT with the Wasserstein-Fisher-Rao cost (the paper's UOT simulation,
    pattern C1, d = 5, eps = 0.1, lambda = 0.1, masses 5 and 3) at n points,
    half of the pairs within the blocking distance (R2), s = 8 s0(n),
    log-domain FP32, stop at residual <= 1e-6; the dense baseline (FP32, K
    recomputed with its zeros) beside it."""
    import torch

    from paper_2306_06581_amd import api as A
    from paper_2306_06581_amd import workloads as W

    p = W.wfr_synthetic(n, d=5, seed=0, pattern="C1", nnz_ratio=0.5, s_factor=8.0)
    prob = A.Problem(p.x, p.y, p.a, p.b)
    kw = dict(eps=p.eps, s=p.s, lam=p.lam, seed=p.seed, tol=1e-6, max_iter=5000,
              precision="f32_log", cost="wfr", eta=p.meta["eta"])
    A.spar_sink_uot(prob, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [A.spar_sink_uot(prob, **kw) for _ in range(steps)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    r = res[-1]
    ms_launch = A.ss_time_iterations(prob, 64, eps=p.eps, s=p.s, lam=p.lam, seed=p.seed,
                                     precision="f32_log", cost="wfr", eta=p.meta["eta"])
    by = iteration_bytes_per_launch("f32_log", r.nnz, p.n, p.m)
    out = {"workload": f"wfr_C1 n=m={n} d=5 R2 eta={p.meta['eta']:.4f} eps=0.1 lambda=0.1 "
                       f"s=8 s0(n) f32_log tol=1e-6",
           "ms_per_solve": ms, "iters": r.iters, "status": r.status, "nnz": r.nnz,
           "estimate": r.estimate, "sparse_objective": r.sparse_objective,
           "stage_ms": {"prep": r.t_prep_ms, "sample": r.t_sample_ms, "iterate": r.t_iter_ms,
                        "objective": r.t_obj_ms},
           "ms_per_launch": ms_launch, "launch_GBps": by / (ms_launch * 1e-3) / 1e9}
    if dense:
        dkw = dict(kw, precision="f32")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d = A.dense_sinkhorn(prob, **dkw)
        torch.cuda.synchronize()
        dms = (time.perf_counter() - t0) * 1e3
        out.update({"dense_ms": dms, "dense_iters": d.iters, "dense_status": d.status,
                    "dense_estimate": d.estimate, "speedup_vs_dense": dms / ms,
                    "rel_err_vs_dense": abs(r.estimate - d.estimate) / abs(d.estimate),
                    "sparse_objective_rel_err_vs_dense":
                        abs(r.sparse_objective - d.estimate) / abs(d.estimate)})
    return out


def divergence_bench(n: int, steps: int, cpu: bool) -> dict:
    """Sinkhorn divergence with gradients (the generative-modelling section's
    regulariser) at the section's set-up: latent codes in R^10 against prior
    draws, uniform weights, the Euclidean distance, eps = 0.01, s = 10 s0(n)
    per term, log-domain FP32.  At this eps the sparse problems converge
    sublinearly, so each term runs a fixed 200 iterations (an auto-encoder's
    inner loop); three Spar-Sink solves plus the envelope gradients per
    evaluation, at the section's batch n = 500 and at n; the CPU oracle
    beside the n = 500 row."""
    from paper_2306_06581_amd import api as A
    from paper_2306_06581_amd import workloads as W

    out = {}
    T = 200
    for nn in (500, n):
        p = W.latent_pair(nn, d=10, seed=0, eps=0.01)
        prob = A.Problem(p.x, p.y, p.a, p.b)
        kw = dict(eps=p.eps, s=p.s, seed=p.seed, tol=0.0, max_iter=T, precision="f32_log",
                  cost="euclid")
        r, ms = timed_solves(lambda: A.sinkhorn_divergence(prob, **kw), steps)
        row = {"workload": f"latent_pair n=m={nn} d=10 euclidean eps=0.01 s=10 s0(n) f32_log, "
                           f"{T} iterations per term, with gradients",
               "ms_per_evaluation": ms, "status": r.status, "value": r.value,
               "value_sparse": r.value_sparse, "iters": [r.iters_xy, r.iters_xx, r.iters_yy],
               "nnz": r.nnz}
        if cpu and nn == 500:
            from oracle import divergence_oracle as D
            from oracle import sparsink_oracle as O
            t0 = time.perf_counter()
            o = D.sinkhorn_divergence(p.x, p.a, p.y, p.b,
                                      O.Options(eps=p.eps, s=p.s, seed=p.seed, cost="euclid",
                                                tol=0.0, max_iter=T, log_domain=True))
            row["cpu_oracle"] = {"s": time.perf_counter() - t0, "cores": 1, "kind": "oracle",
                                 "value_sparse": o.value_sparse,
                                 "value_sparse_rel_err": _rel(r.value_sparse, o.value_sparse),
                                 "grad_rel_l2_vs_gpu": float(
                                     np.linalg.norm(o.grad_x - r.grad_x.cpu().numpy())
                                     / np.linalg.norm(o.grad_x))}
        out[f"n{nn}"] = row
    return out


GOLDEN = os.path.join(ROOT, "tests", "golden", "bench_oracle.json")


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def timed_solves(fn, steps):
    """fn() once as a warm-up, then `steps` timed calls; (last result, ms per call)."""
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t0) * 1e3 / steps


def eps_small_bench(n: int, steps: int, dense: bool) -> dict:
    """The headline UOT workload at the configuration's smaller eps = 0.01
    (log-domain FP32, tol 1e-6), with the dense baseline (log-domain FP32,
    the linear FP32 kernel underflows at this eps) beside it."""
    from paper_2306_06581_amd import api as A
    from paper_2306_06581_amd import workloads as W

    p = W.uot_mix3(n, seed=0, eps=0.01)
    prob = A.Problem(p.x, p.y, p.a, p.b)
    kw = dict(eps=p.eps, s=p.s, lam=p.lam, seed=p.seed, tol=1e-6, max_iter=5000,
              precision="f32_log")
    r, ms = timed_solves(lambda: A.spar_sink_uot(prob, **kw), steps)
    out = {"workload": f"uot_mix3 n=m={n} d=3 lambda=1 eps=0.01 s=8nlnn tol=1e-6 f32_log",
           "ms_per_solve": ms, "iters": r.iters, "status": r.status, "nnz": r.nnz,
           "estimate": r.estimate, "sparse_objective": r.sparse_objective,
           "stage_ms": {"prep": r.t_prep_ms, "sample": r.t_sample_ms, "iterate": r.t_iter_ms,
                        "objective": r.t_obj_ms}}
    r64 = A.spar_sink_uot(prob, **dict(kw, precision="f64"), raise_on_error=False)
    out["f64_gpu"] = {"iters": r64.iters, "status": r64.status, "estimate": r64.estimate,
                      "f32_log_rel_err": _rel(r.estimate, r64.estimate)}
    if dense:
        import torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d = A.dense_sinkhorn(prob, **dict(kw, precision="f32_log"))
        torch.cuda.synchronize()
        dms = (time.perf_counter() - t0) * 1e3
        out.update({"dense_ms": dms, "dense_iters": d.iters, "dense_status": d.status,
                    "dense_precision": "f32_log", "dense_estimate": d.estimate,
                    "speedup_vs_dense": dms / ms})
    return out


def hbm_bench(steps: int) -> dict:
    """Iteration-kernel bandwidth where the per-iteration data cannot stay in
    the 256 MB Infinity Cache: the headline generator at s = 32 n ln n
    (2 x 140 MB of entries per iteration) and at n = 131072 (s = 8 n ln n),
    plus the whole solve at s = 32 n ln n."""
    from paper_2306_06581_amd import api as A
    from paper_2306_06581_amd import workloads as W

    out = {}
    for n, f in ((65536, 32.0), (131072, 8.0)):
        p = W.uot_mix3(n, seed=0, eps=0.05, s_factor=f)
        prob = A.Problem(p.x, p.y, p.a, p.b)
        kw = dict(eps=p.eps, s=p.s, lam=p.lam, seed=p.seed, precision="f32_log")
        ms_launch = A.ss_time_iterations(prob, 64, **kw)
        r1 = A.spar_sink_uot(prob, **kw, tol=1e-6, max_iter=1, raise_on_error=False)
        by = iteration_bytes_per_launch("f32_log", r1.nnz, p.n, p.m)
        gbps = by / (ms_launch * 1e-3) / 1e9
        key = f"uot_mix3_n{n}_s{f:g}"
        out[key] = {"workload": f"uot_mix3 n=m={n} d=3 lambda=1 eps=0.05 s={f:g}nlnn f32_log",
                    "nnz": r1.nnz, "ms_per_launch": ms_launch, "bytes_per_launch": by,
                    "GBps": gbps, "frac_of_8TBps": gbps / HBM_PEAK_GBPS}
        if n == 65536 and f == 32.0:
            tr = measured_traffic(by, PROFILE_TRAFFIC_S32)
            out[key]["roofline"] = {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS,
                                    "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS,
                                    "traffic": tr["bytes"] if tr else None,
                                    "kernel": "k_iterate (sparse iteration)"}
            if tr:
                out[key]["roofline"]["traffic_detail"] = tr
        if n == 65536:
            r, ms = timed_solves(lambda: A.spar_sink_uot(prob, **kw, tol=1e-6, max_iter=5000),
                                 steps)
            out[key].update({"ms_per_solve": ms, "iters": r.iters, "status": r.status,
                             "stage_ms": {"sample": r.t_sample_ms, "iterate": r.t_iter_ms}})
    return out


def ot_scale_bench(steps: int, dense: bool) -> dict:
    """OT at scale: n = m = 16384, d = 10, x ~ N(0, I), y ~ t5 + 0.5,
    Dirichlet(1) weights, eps = 0.05 on the max-normalised cost, FP32,
    tol 1e-6, s in {4, 8, 16} n ln n, against dense Sinkhorn (FP32, K
    recomputed) on the same GPU; each FP32 estimate's relative error against
    the FP64 oracle (tests/golden/bench_oracle.json, written by the oracle)
    and against the library's FP64 solve.  Also the OT row at n = 65536."""
    from paper_2306_06581_amd import api as A
    from paper_2306_06581_amd import workloads as W

    gold = {}
    if os.path.exists(GOLDEN):
        gold = json.load(open(GOLDEN))
    out = {}
    for n, factors in ((16384, (4.0, 8.0, 16.0)), (65536, (8.0,))):
        dense_ms = dense_iters = dense_est = None
        for f in factors:
            p = W.ot_t5_d10(n, seed=0, s_factor=f)
            prob = A.Problem(p.x, p.y, p.a, p.b)
            kw = dict(eps=p.eps, s=p.s, seed=p.seed, tol=1e-6, max_iter=5000, precision="f32")
            r, ms = timed_solves(lambda: A.spar_sink_ot(prob, **kw), steps)
            r64 = A.spar_sink_ot(prob, **dict(kw, precision="f64"))
            ms_launch = A.ss_time_iterations(prob, 64, eps=p.eps, s=p.s, seed=p.seed,
                                             precision="f32")
            by = iteration_bytes_per_launch("f32", r.nnz, p.n, p.m)
            key = f"ot_t5_d10_n{n}_s{f:g}"
            row = {"workload": f"ot_t5_d10 n=m={n} d=10 eps=0.05 s={f:g}nlnn f32 tol=1e-6",
                   "ms_per_solve": ms, "iters": r.iters, "status": r.status, "nnz": r.nnz,
                   "estimate": r.estimate, "sparse_objective": r.sparse_objective,
                   "stage_ms": {"sample": r.t_sample_ms, "iterate": r.t_iter_ms},
                   "ms_per_launch": ms_launch, "GBps": by / (ms_launch * 1e-3) / 1e9,
                   "f64_gpu_estimate": r64.estimate,
                   "rel_err_vs_f64_gpu": _rel(r.estimate, r64.estimate)}
            g = gold.get(key)
            if g is not None:
                row["oracle_f64"] = {"estimate": g["estimate"], "iters": g["iters"],
                                     "nnz": g["nnz"]}
                row["rel_err_vs_oracle_f64"] = _rel(r.estimate, g["estimate"])
                row["sparse_objective_rel_err_vs_oracle_f64"] = _rel(r.sparse_objective,
                                                                     g["sparse_objective"])
            if dense and dense_ms is None:
                import torch
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                d = A.dense_sinkhorn(prob, **kw)
                torch.cuda.synchronize()
                dense_ms = (time.perf_counter() - t0) * 1e3
                dense_iters, dense_est = d.iters, d.estimate
            if dense_ms is not None:
                row.update({"dense_ms": dense_ms, "dense_iters": dense_iters,
                            "dense_estimate": dense_est, "speedup_vs_dense": dense_ms / ms,
                            "rel_err_vs_dense": _rel(r.estimate, dense_est),
                            "sparse_objective_rel_err_vs_dense": _rel(r.sparse_objective,
                                                                      dense_est)})
            out[key] = row
    return out


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, gpu_iters: int, precision_log: bool, z_gpu: float, cmax_gpu: float,
                 dense_iters: int | None) -> dict:
    """The FP64 oracle on the host's cores, on a bounded sample of the same
    workload; every part is extrapolated to the full size and labelled so.

    * cost scan, UOT normaliser and hash mask: R rows against all m columns
      (the normaliser's row sums timed on those rows; the p* of the timed
      mask uses the full normaliser, taken from the GPU solve, which matches
      the oracle's to 1e-12), scaled by n / R;
    * Sinkhorn iterations: the oracle's loop on the same generator at
      n = 4096 (its own sketch), per iteration scaled by (nnz + n + m) to
      the full size, times the GPU's iteration count;
    * dense FP64 Sinkhorn (K recomputed): one product K v on R rows timed,
      scaled by n / R, two per iteration, times the dense GPU run's count."""
    import numpy as np

    from oracle import elementary as EL
    from oracle import sparsink_oracle as O
    from paper_2306_06581_amd import workloads as W

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    workers = max(1, cores or 1)
    t_all = time.perf_counter()
    R = 1024
    uot = math.isfinite(p.lam)
    opt = O.Options(eps=p.eps, s=p.s, lam=p.lam, seed=p.seed, log_domain=precision_log)
    rows = np.arange(R)
    chunk = max(1, R // workers)
    t0 = time.perf_counter()
    O.max_sq_dist(p.x[:R], p.y, chunk=chunk, workers=workers)
    t_cmax = time.perf_counter() - t0
    inv_cmax = 1.0 / cmax_gpu  # the full maximum (the oracle's equals it bit for bit)
    t0 = time.perf_counter()
    if uot:
        O.uot_probabilities(p.a[:R], p.b, p.x[:R], p.y, p.s, p.lam, p.eps, inv_cmax,
                            chunk=chunk, workers=workers)
        t_z = time.perf_counter() - t0
        # the mask's p* with the full normaliser
        full = O.uot_probabilities(p.a[:1], p.b, p.x[:1], p.y, p.s, p.lam, p.eps, inv_cmax)
        prob = O.ProbUOT(la=p.lam / (2 * p.lam + p.eps) * EL.log_spec(p.a), lb=full.lb,
                         inv_tau=full.inv_tau, inv_cmax=inv_cmax, z=z_gpu, kappa=p.s / z_gpu,
                         x=np.asarray(p.x, np.float64), y=full.y)
    else:
        prob = O.ot_probabilities(p.a, p.b, p.s)
        t_z = time.perf_counter() - t0
    t0 = time.perf_counter()
    O._map_chunks(lambda r0: O.sample_rows(p.x, p.y, p.a, p.b, opt,
                                           rows[r0:r0 + chunk], prob)[0].sum(),
                  range(0, R, chunk), workers)
    t_mask = time.perf_counter() - t0
    scale = p.n / R
    t_sample = (t_cmax + t_z + t_mask) * scale
    # iterations at n = 4096 of the same generator
    ns = 4096
    q = W.uot_mix3(ns, seed=p.seed, eps=p.eps) if uot else W.ot_t5_d10(ns, seed=p.seed)
    it = 20
    optq = O.Options(eps=q.eps, s=q.s, lam=q.lam, seed=q.seed, tol=0.0, max_iter=it,
                     log_domain=precision_log)
    sk = O.build_sketch(q.x, q.y, q.a, q.b, optq, workers=workers)
    a_eff, b_eff, ra, ca, _, _ = O.apply_empty_policy(q.a, q.b, np.diff(sk.row_ptr),
                                                      np.diff(sk.col_ptr), optq)
    t0 = time.perf_counter()
    if precision_log:
        O.sinkhorn_log(sk, a_eff, b_eff, optq, ra, ca)
    else:
        O.sinkhorn(sk.csr(), a_eff, b_eff, optq, ra, ca)
    t_it_small = (time.perf_counter() - t0) / it
    t_iter = t_it_small * (p.s + p.n + p.m) / (sk.nnz + q.n + q.m) * gpu_iters
    out = {"value": t_sample + t_iter, "unit": "s", "cores": workers, "kind": "oracle",
           "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "extrapolated": True,
           "sample": (f"oracle on {workers} threads: cost scan, normaliser row sums and hash "
                      f"mask on {R} of {p.n} rows (x{scale:g}); {it} oracle iterations at "
                      f"n={ns} scaled by (nnz+n+m) to the full size x {gpu_iters} GPU "
                      f"iterations; measured {time.perf_counter() - t_all:.1f} s"),
           "parts_s": {"sample": t_sample, "iterations": t_iter}}
    if dense_iters:
        # one dense half-step on R rows: K recomputed (cost, specified exp) and K v
        v = np.ones(p.m)
        t0 = time.perf_counter()

        def krows(r0):
            rr = np.arange(r0, min(R, r0 + chunk))
            c = O.cost_from_sq(O.sq_dist(p.x[rr], p.y), "maxnorm", inv_cmax, 1.0)
            return EL.exp_spec(-(c / p.eps)) @ v

        O._map_chunks(krows, range(0, R, chunk), workers)
        t_half = (time.perf_counter() - t0) * scale
        out["dense_fp64"] = {"value": t_half * 2 * dense_iters, "unit": "s",
                             "extrapolated": True, "iters": dense_iters,
                             "sample": f"one K v over {R} of {p.n} rows (K recomputed), x{scale:g} "
                                       f"rows, x2 half-steps, x{dense_iters} iterations"}
    return out


def progress(msg: str) -> None:
    """A line on stderr as each section ends (the JSON line stays alone on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs a problem (or a batch) on a "
              "single device and has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.batched_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"batched": batched_bench(args.batch_count, args.steps, not args.no_autotune)}))
        return
    if args.divergence_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"divergence": divergence_bench(args.divergence_n, args.steps,
                                                         not args.no_cpu)}))
        return
    if args.wfr_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"wfr": wfr_bench(args.wfr_n, args.steps, not args.no_dense)}))
        return
    if args.ibp_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"ibp": ibp_bench(args.ibp_n, args.steps, not args.no_cpu)}))
        return
    if args.sections_only:
        import torch
        torch.cuda.set_device(0)
        out = {}
        if not args.no_eps_small:
            out["eps_small"] = eps_small_bench(args.n, args.steps, not args.no_dense)
        if not args.no_hbm:
            out["hbm_resident"] = hbm_bench(args.steps)
        if not args.no_ot_scale:
            out["ot_scale"] = ot_scale_bench(args.steps, not args.no_dense)
        print(json.dumps(out))
        return
    if args.predict_only:
        import torch

        from paper_2306_06581_amd import api as A
        from paper_2306_06581_amd import workloads as W
        torch.cuda.set_device(0)
        B = A.Batch.from_problems(W.batch_ot(args.batch_count, seed=0))
        net = A.WarmStartNet(seed=0)
        _, ms = timed_solves(lambda: net.predict(B, eps=0.05), args.steps)
        print(json.dumps({"predict_ms": ms, "problems": args.batch_count,
                          "points": int(B.row_off[-1] + B.col_off[-1])}))
        return
    if args.warmstart_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"warmstart": warmstart_bench(args.warmstart_train, args.batch_count)}))
        return
    import torch

    from paper_2306_06581_amd import api as A
    from paper_2306_06581_amd import workloads as W

    torch.cuda.set_device(0)
    p = W.uot_mix3(args.n, seed=0, eps=args.eps, s_factor=args.s_factor)
    prob = A.Problem(p.x, p.y, p.a, p.b)
    kw = dict(eps=p.eps, s=p.s, lam=p.lam, seed=p.seed, tol=1e-6, max_iter=5000,
              precision=args.precision)
    if args.kernel_only:
        ms_launch = A.ss_time_iterations(prob, args.timing_iters, eps=p.eps, s=p.s, lam=p.lam,
                                         seed=p.seed, precision=args.precision)
        r = A.spar_sink_uot(prob, **dict(kw, max_iter=1), raise_on_error=False)
        by = iteration_bytes_per_launch(args.precision, r.nnz, p.n, p.m)
        print(json.dumps({"kernel": "k_iterate", "n": p.n, "s_factor": args.s_factor,
                          "nnz": r.nnz, "ms_per_launch": ms_launch,
                          "launches": 4 * args.timing_iters, "bytes_per_launch": by,
                          "GBps": by / (ms_launch * 1e-3) / 1e9}))
        return

    for _ in range(args.warmup):
        A.spar_sink_uot(prob, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [A.spar_sink_uot(prob, **kw) for _ in range(args.steps)]
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    r = results[-1]
    for rr in results:
        if rr.status != 0:
            raise SystemExit(f"Spar-Sink did not converge: status {rr.status}")

    # dominant kernel: the sparse iteration kernel, timed with HIP events
    ms_launch = A.ss_time_iterations(prob, args.timing_iters, eps=p.eps, s=p.s, lam=p.lam,
                                     seed=p.seed, precision=args.precision)
    bytes_launch = iteration_bytes_per_launch(args.precision, r.nnz, p.n, p.m)
    gbps = bytes_launch / (ms_launch * 1e-3) / 1e9

    out = {
        "metric": METRIC, "value": ms_step / 1e3, "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"uot_mix3 n=m={p.n} d=3 lambda=1 eps={p.eps:g} s=8nlnn "
                               f"tol=1e-6 {args.precision}",
                   "n": p.n, "m": p.m, "d": 3, "eps": p.eps, "lambda": p.lam, "s": p.s,
                   "tol": 1e-6},
        "iters": r.iters, "nnz": r.nnz, "estimate": r.estimate, "marginal_err": r.marginal_err,
        "stage_ms": {"prep": r.t_prep_ms, "sample": r.t_sample_ms, "iterate": r.t_iter_ms,
                     "objective": r.t_obj_ms},
        "spmv_GBps": gbps,
        "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": gbps / HBM_PEAK_GBPS, "traffic": None,
                     "kernel": "k_iterate (sparse iteration)",
                     "ms_per_launch": ms_launch, "bytes_per_launch": bytes_launch},
    }
    tr = measured_traffic(bytes_launch)
    if tr is not None:
        out["roofline"]["traffic"] = tr["bytes"]
        out["roofline"]["traffic_detail"] = tr
    if not args.no_dense:
        dp = args.dense_precision
        if dp == "auto":
            dp = "f32" if p.eps >= 0.03 else "f32_log"
        dkw = dict(kw, precision=dp)
        dres = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.dense_runs):
            dres.append(A.dense_sinkhorn(prob, **dkw))
        torch.cuda.synchronize()
        dms = (time.perf_counter() - t0) * 1e3 / args.dense_runs
        d = dres[-1]
        out["dense_s"] = dms / 1e3
        out["dense_iters"] = d.iters
        out["dense_status"] = d.status
        out["dense_precision"] = dp
        out["dense_estimate"] = d.estimate
        out["speedup_vs_dense"] = dms / ms_step
        # Sec. 5's comparison at the same budget s: the relative error of the
        # estimate against the dense one, for Spar-Sink and for Rand-Sink
        # (uniform probabilities, shrink = 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = A.spar_sink_uot(prob, **kw, shrink=1.0, raise_on_error=False)
        torch.cuda.synchronize()
        rel = lambda e: abs(e - d.estimate) / abs(d.estimate)
        out["rand_sink"] = {"s": (time.perf_counter() - t0), "iters": rs.iters,
                            "status": rs.status, "nnz": rs.nnz, "estimate": rs.estimate,
                            "rel_err_vs_dense": rel(rs.estimate),
                            "sparse_objective_rel_err_vs_dense": rel(rs.sparse_objective),
                            "spar_sink_rel_err_vs_dense": rel(r.estimate),
                            "spar_sink_sparse_objective_rel_err_vs_dense":
                                rel(r.sparse_objective)}
    progress(f"headline {ms_step:.3f} ms per solve")
    if not args.no_batched:
        out["batched"] = batched_bench(args.batch_count, args.steps)
        progress("batched")
    if args.warmstart_train > 0:
        out["warmstart"] = warmstart_bench(args.warmstart_train, args.batch_count)
        progress("warmstart")
    if not args.no_ibp:
        out["ibp"] = ibp_bench(args.ibp_n, args.steps, not args.no_cpu)
        progress("ibp")
    if not args.no_wfr:
        out["wfr"] = wfr_bench(args.wfr_n, args.steps, not args.no_dense)
        progress("wfr")
    if not args.no_divergence:
        out["divergence"] = divergence_bench(args.divergence_n, args.steps, not args.no_cpu)
        progress("divergence")
    if not args.no_eps_small:
        out["eps_small"] = eps_small_bench(args.n, args.steps, not args.no_dense)
        progress("eps_small")
    if not args.no_hbm:
        out["hbm_resident"] = hbm_bench(args.steps)
        progress("hbm_resident")
        # the same kernel where its data cannot stay in the Infinity Cache
        out["roofline_hbm_resident"] = dict(
            out["hbm_resident"]["uot_mix3_n65536_s32"].get("roofline", {}),
            workload=out["hbm_resident"]["uot_mix3_n65536_s32"]["workload"])
    if not args.no_ot_scale:
        out["ot_scale"] = ot_scale_bench(args.steps, not args.no_dense)
        progress("ot_scale")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p, r.iters, args.precision == "f32_log", r.z_norm,
                                           r.cmax, out.get("dense_iters"))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
